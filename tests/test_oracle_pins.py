"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formulas: each compares it with an
independent formulation (exact rationals, brute force over voxels without any
mesh logic, scipy's interpolation and k-d tree, closed forms, invariants).
"""
import json
import os

import numpy as np
import pytest
from scipy import ndimage
from scipy.spatial import cKDTree

import exact_raster
import oracle
import synth
from conftest import rel_err

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def box_mesh(dims, shape, lo, hi):
    """Kuhn grid on the box [lo, hi]^3 (per axis), with pinned-axis mask."""
    pts, tets, fixed = synth.kuhn_grid((1, 1, 1), shape)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    steps = np.asarray(shape, dtype=np.float64) - 1
    idx = np.rint((pts + 0.5) * steps)
    pts = lo + idx * ((hi - lo) / steps)
    return pts.astype(np.float32), tets, fixed


def candidates(S, T):
    return np.stack([np.asarray(S, np.float32).T, np.asarray(T, np.float32).T])[None]


def make_oracle(dims, img_s, img_t, pts, tets, sets_s=(), sets_t=(), radius=4.0, elast=None):
    elast = np.ones(len(tets), np.float32) if elast is None else elast
    return oracle.Problem(dims, img_s, img_t, tets, pts, elast, list(sets_s), list(sets_t), radius)


# ------------------------------------------------------------------ rasterization
def _kuhn_cases():
    rs = np.random.default_rng(7)
    cases = []
    for shape in [(2, 2, 2), (3, 3, 3)]:
        pts, tets, fixed = synth.kuhn_grid((8, 8, 8), shape)
        cases.append((pts, tets))
        # interior moves in multiples of 1/8 voxel: many centres land on faces
        for _ in range(2):
            p2 = pts.copy()
            mv = rs.integers(-6, 7, size=p2.shape) / 8.0
            mv[fixed] = 0
            cases.append((p2 + mv, tets))
    return cases


@pytest.mark.parametrize("case", range(6))
def test_raster_matches_exact_rationals(case):
    pts, tets = _kuhn_cases()[case]
    dims = (8, 8, 8)
    seen = np.zeros(512, np.int32)
    for t in tets:
        v = pts[t]
        got = oracle.tet_voxels(v, dims)
        want = exact_raster.tet_voxels(v, dims)
        assert sorted(got.tolist()) == want
        seen[got] += 1
    # the box [-0.5, 7.5]^3 is tiled without folds: every centre exactly once
    assert np.all(seen == 1)


def test_raster_random_tets_exact():
    rs = np.random.default_rng(3)
    dims = (6, 5, 7)
    for _ in range(20):
        v = rs.integers(-4, 60, size=(4, 3)) / 8.0
        got = oracle.tet_voxels(v, dims)
        assert sorted(got.tolist()) == exact_raster.tet_voxels(v, dims)


def test_coverage_population(c1, c1_oracle):
    pop = synth.make_population(c1)
    out = c1_oracle.evaluate(pop)
    V = int(np.prod(c1.dims))
    assert np.all(out["flags"] == 0)
    assert np.all(out["counts"] == V)


# -------------------------------------------------------------- volumes and folds
def test_signed_volumes_sum_to_box_volume(c1):
    rs = np.random.default_rng(11)
    pts = c1.ref_points.astype(np.float64)
    interior = ~c1.fixed_axes.any(axis=1)
    moved = pts.copy()
    moved[interior] += rs.normal(0, 4.0, size=(interior.sum(), 3))   # large: folds likely
    moved = moved.astype(np.float32)
    ref = np.array([np.sign(oracle.orient(c1.ref_points[t])) for t in c1.tets])
    vols = np.array([oracle.orient(moved[t]) for t in c1.tets])
    box = 6 * (32 ** 3) * 2 ** 30
    assert np.sum(ref * vols) == box
    assert np.sum(np.abs(vols)) > box          # the large motion folded the mesh
    vols0 = np.array([oracle.orient(c1.ref_points[t]) for t in c1.tets])
    assert np.sum(np.abs(vols0)) == box


def test_one_cube_tets_are_one_sixth():
    pts, tets, _ = synth.kuhn_grid((8, 8, 8), (2, 2, 2))
    for t in tets:
        assert abs(oracle.orient(pts[t])) == 8 ** 3 * 2 ** 30


def test_fold_flag_and_severity(c1, c1_oracle):
    S = c1.ref_points.astype(np.float64)
    # rigid translation of both meshes: no fold
    out = c1_oracle.evaluate(candidates(S + [1.25, -0.5, 2.0], S + [0.75, 0.5, 0.0]))
    assert out["flags"][0] == 0 and out["severity"][0] == 0
    # push an interior point through the face opposite to it in one tet
    v = int(np.flatnonzero(~c1.fixed_axes.any(axis=1))[0])
    tet = c1.tets[np.flatnonzero((c1.tets == v).any(axis=1))[0]]
    face = [w for w in tet if w != v]
    T = S.copy()
    cf = T[face].mean(axis=0)
    T[v] = cf + 0.5 * (cf - T[v])
    T = T.astype(np.float32)
    out = c1_oracle.evaluate(candidates(S, T))
    assert out["flags"][0] == 2
    ref = np.array([np.sign(oracle.orient(c1.ref_points[t])) for t in c1.tets])
    vols = np.array([oracle.orient(T[t]) for t in c1.tets])
    viol = np.sign(vols) != ref
    assert viol.any()
    want = np.sum(np.abs(vols[viol])) / 6 / 2 ** 30
    assert out["severity"][0] == pytest.approx(want, rel=1e-14)


def test_invalid_candidate(c1, c1_oracle):
    S = c1.ref_points.astype(np.float32).copy()
    T = S.copy()
    T[5, 0] = 600.0
    out = c1_oracle.evaluate(candidates(S, T))
    assert out["flags"][0] == 4 and np.all(np.isnan(out["obj"][0]))


# --------------------------------------------------------------------- intensity
def test_identity_gives_zero_intensity(c1):
    img = c1.image_src
    op = make_oracle(c1.dims, img, img, c1.ref_points, c1.tets)
    S = c1.ref_points
    out = op.evaluate(candidates(S, S))
    assert out["obj"][0, 0] == 0.0


def test_constant_images_identity():
    dims = (12, 10, 9)
    pts, tets, _ = synth.kuhn_grid(dims, (3, 3, 3))
    a, b = 0.75, 0.25
    op = make_oracle(dims, np.full(dims[::-1], a), np.full(dims[::-1], b), pts, tets)
    out = op.evaluate(candidates(pts, pts))
    assert out["obj"][0, 0] == pytest.approx((a - b) ** 2, rel=1e-14)


def test_foreground_background_mismatch_is_one():
    dims = (12, 10, 9)
    pts, tets, fixed = synth.kuhn_grid(dims, (3, 3, 3))
    rs = np.random.default_rng(1)
    T = pts + np.where(fixed, 0, rs.normal(0, 0.4, pts.shape))
    op = make_oracle(dims, np.full(dims[::-1], 0.6), np.zeros(dims[::-1]), pts, tets)
    out = op.evaluate(candidates(pts, T.astype(np.float32)))
    assert out["obj"][0, 0] == 1.0


def test_linear_ramp_translation():
    dims = (24, 20, 18)
    pts, tets, _ = box_mesh(dims, (4, 3, 3), (3.5, 3.5, 3.5), (19.5, 15.5, 13.5))
    alpha, beta = 0.03125, 0.125   # exact in FP32
    z, y, x = np.meshgrid(*[np.arange(n) for n in dims[::-1]], indexing="ij")
    ramp = (alpha * x + beta).astype(np.float32)
    t = np.array([307, -211, 97]) / 1024.0
    op = make_oracle(dims, ramp, ramp, pts, tets)
    out = op.evaluate(candidates(pts, pts + t))
    assert out["obj"][0, 0] == pytest.approx((alpha * t[0]) ** 2, rel=1e-9)


def _h(a, b):
    fa, fb = a > 0, b > 0
    return np.where(fa & fb, (a - b) ** 2, np.where(~fa & ~fb, 0.0, 1.0))


def test_affine_brute_force(c1):
    """T = A S + t on an inset mesh: the piecewise-affine map is the affine map,
    so both sums can be computed voxel by voxel with scipy, without tets."""
    dims = c1.dims
    lo, hi = np.array([5.5, 6.5, 4.5]), np.array([25.5, 24.5, 26.5])
    pts, tets, _ = box_mesh(dims, (5, 4, 5), lo, hi)
    A = np.array([[1.0 + 27 / 512, 13 / 512, -9 / 512],
                  [-21 / 512, 1.0 - 31 / 512, 17 / 512],
                  [11 / 512, 5 / 512, 1.0 + 19 / 512]])
    t = np.array([389, -613, 251]) / 1024.0
    T = pts.astype(np.float64) @ A.T + t
    assert np.array_equal(T, T.astype(np.float32))   # exactly representable
    op = make_oracle(dims, c1.image_src, c1.image_tgt, pts, tets)
    out = op.evaluate(candidates(pts, T.astype(np.float32)))

    zz, yy, xx = np.meshgrid(*[np.arange(n) for n in dims[::-1]], indexing="ij")
    P = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], -1).astype(np.float64)
    # source side: centres strictly inside the box (faces at half-integers)
    ins = np.all((P > lo) & (P < hi), axis=1)
    q = P[ins] @ A.T + t
    b = ndimage.map_coordinates(c1.image_tgt.astype(np.float64), q[:, ::-1].T, order=1,
                                mode="grid-constant", cval=0.0)
    a = c1.image_src.ravel()[ins].astype(np.float64)
    hs = _h(a, b).sum()
    # target side: centres strictly inside A(box) + t
    pre = (P - t) @ np.linalg.inv(A).T
    dist = np.minimum(np.abs(pre - lo), np.abs(pre - hi)).min(axis=1)
    assert dist.min() > 1e-9                           # no centre on a face
    ins_t = np.all((pre > lo) & (pre < hi), axis=1)
    b2 = ndimage.map_coordinates(c1.image_src.astype(np.float64), pre[ins_t][:, ::-1].T, order=1,
                                 mode="grid-constant", cval=0.0)
    a2 = c1.image_tgt.ravel()[ins_t].astype(np.float64)
    ht = _h(a2, b2).sum()
    assert out["counts"][0].tolist() == [int(ins.sum()), int(ins_t.sum())]
    want = (hs + ht) / (ins.sum() + ins_t.sum())
    assert rel_err(out["obj"][0, 0], want) < 1e-12


def test_trilinear_matches_scipy(c1):
    rs = np.random.default_rng(5)
    img = c1.image_src
    for _ in range(200):
        q = rs.uniform(-1.5, 32.5, size=3)
        want = ndimage.map_coordinates(img.astype(np.float64), q[::-1].reshape(3, 1), order=1,
                                       mode="grid-constant", cval=0.0)[0]
        assert oracle.trilinear(img, q) == pytest.approx(want, abs=1e-15)
        want_c = ndimage.map_coordinates(img.astype(np.float64), q[::-1].reshape(3, 1), order=1,
                                         mode="nearest")[0]
        assert oracle.trilinear(img, q, clamp=True) == pytest.approx(want_c, abs=1e-15)


# --------------------------------------------------------------------- magnitude
def test_magnitude_translation_is_zero_bitwise(c1, c1_oracle):
    S = c1.ref_points.astype(np.float64)
    rs = np.random.default_rng(2)
    S = np.rint((S + rs.normal(0, 0.3, S.shape)) * 1024) / 1024
    out = c1_oracle.evaluate(candidates(S, S + np.array([3379, -1741, 922]) / 1024))
    assert out["obj"][0, 1] == 0.0


def test_magnitude_uniform_scale_closed_form(c1):
    S = c1.ref_points.astype(np.float64)
    s = 1.25
    T = S * s
    elast = np.random.default_rng(4).uniform(0.5, 10, len(c1.tets)).astype(np.float32)
    op = make_oracle(c1.dims, c1.image_src, c1.image_tgt, c1.ref_points, c1.tets, elast=elast)
    out = op.evaluate(candidates(S, T))
    v = S[c1.tets]                                  # [T][4][3]
    cen = v.mean(axis=1, keepdims=True)
    # sum over 6 edges of |e|^2 = 4 sum |v - c|^2; 4 spokes add sum |v - c|^2
    sum_e2 = 5.0 * np.sum((v - cen) ** 2, axis=(1, 2))
    want = (1 - s) ** 2 * np.sum(elast * sum_e2) / (10 * len(c1.tets))
    assert out["obj"][0, 1] == pytest.approx(want, rel=1e-12)


def test_magnitude_unit_tet_golden():
    g = json.load(open(os.path.join(GOLDEN, "unit_tet_magnitude.json")))
    S = np.array(g["source"], np.float32)
    T = np.array(g["target"], np.float32)
    dims = (4, 4, 4)
    op = make_oracle(dims, np.zeros((4, 4, 4)), np.zeros((4, 4, 4)), S, np.array([[0, 1, 2, 3]]),
                     elast=np.array([g["elasticity"]], np.float32))
    out = op.evaluate(candidates(S, T))
    assert out["obj"][0, 1] == pytest.approx(g["f_magnitude"], rel=1e-14)


# ---------------------------------------------------------------------- guidance
def test_distance_map_matches_kdtree(c1):
    pts = c1.sets_src[0]
    dm = oracle.distance_map(c1.dims, pts)
    zz, yy, xx = np.meshgrid(*[np.arange(n) for n in c1.dims[::-1]], indexing="ij")
    P = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], -1)
    snapped = np.rint(pts.astype(np.float64) * 1024) / 1024
    d, _ = cKDTree(snapped).query(P)
    assert np.max(np.abs(dm.ravel() - d) / np.maximum(d, 1e-30)) < 1.2e-7


def test_guidance_identity_is_zero(c1):
    op = make_oracle(c1.dims, c1.image_src, c1.image_tgt, c1.ref_points, c1.tets,
                     c1.sets_src, c1.sets_src, radius=4.0)
    out = op.evaluate(candidates(c1.ref_points, c1.ref_points))
    assert out["obj"][0, 2] == 0.0


def test_guidance_integer_translation_is_zero(c1):
    dims = c1.dims
    pts, tets, _ = box_mesh(dims, (4, 4, 4), (4.5, 4.5, 4.5), (25.5, 25.5, 25.5))
    t = np.array([2.0, -1.0, 3.0])
    cs = c1.sets_src[0]
    op = make_oracle(dims, c1.image_src, c1.image_tgt, pts, tets, [cs], [cs + t], radius=4.0)
    out = op.evaluate(candidates(pts, pts + t))
    assert out["obj"][0, 2] == 0.0


def test_guidance_translation_brute_force(c1):
    dims = c1.dims
    lo, hi = np.array([4.5, 4.5, 4.5]), np.array([25.5, 25.5, 25.5])
    pts, tets, _ = box_mesh(dims, (4, 4, 4), lo, hi)
    t = np.array([523, -301, 177]) / 1024.0
    cs = c1.sets_src[0]
    ct = c1.sets_tgt[0]
    r = 4.0
    op = make_oracle(dims, c1.image_src, c1.image_tgt, pts, tets, [cs], [ct], radius=r)
    out = op.evaluate(candidates(pts, pts + t))
    zz, yy, xx = np.meshgrid(*[np.arange(n) for n in dims[::-1]], indexing="ij")
    P = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], -1).astype(np.float64)
    snap = lambda a: np.rint(a.astype(np.float64) * 1024) / 1024
    Ds = cKDTree(snap(cs)).query(P)[0].astype(np.float32).astype(np.float64)
    Dt = cKDTree(snap(ct)).query(P)[0].astype(np.float32).astype(np.float64)
    Ds_img, Dt_img = Ds.reshape(dims[::-1]), Dt.reshape(dims[::-1])

    def g(Pin, d_own, map_oth, shift):
        q = Pin + shift
        d2 = ndimage.map_coordinates(map_oth, q[:, ::-1].T, order=1, mode="nearest")
        band = d_own < r
        return np.sum(((r - d_own) / r * (d_own - d2) ** 2)[band])

    ins_s = np.all((P > lo) & (P < hi), axis=1)
    ins_t = np.all((P > lo + t) & (P < hi + t), axis=1)
    gs = g(P[ins_s], Ds[ins_s], Dt_img, t)
    gt = g(P[ins_t], Dt[ins_t], Ds_img, -t)
    want = (gs + gt) / (ins_s.sum() + ins_t.sum())     # one set: weights are 1
    assert out["counts"][0].tolist() == [int(ins_s.sum()), int(ins_t.sum())]
    assert want > 0
    assert rel_err(out["obj"][0, 2], want) < 1e-10


def test_guidance_set_weights_are_linear():
    """f(A, B) = (|A| f(A) + |B| f(B)) / (|A| + |B|) when each set has the
    same size in both images: pins the |C| / |G| weights."""
    p = synth.make_problem(1)
    rs = np.random.default_rng(9)
    A_s = p.sets_src[0]
    A_t = p.sets_tgt[0]
    B_s = rs.uniform(8, 24, size=(7, 3)).astype(np.float32)
    B_t = (B_s + rs.normal(0, 1.0, B_s.shape)).astype(np.float32)
    pop = synth.make_population(p, pop=2)
    f = {}
    for name, ss, tt in [("A", [A_s], [A_t]), ("B", [B_s], [B_t]), ("AB", [A_s, B_s], [A_t, B_t])]:
        op = make_oracle(p.dims, p.image_src, p.image_tgt, p.ref_points, p.tets, ss, tt, radius=4.0)
        f[name] = op.evaluate(pop)["obj"][:, 2]
    nA, nB = len(A_s), len(B_s)
    want = (nA * f["A"] + nB * f["B"]) / (nA + nB)
    assert np.all(rel_err(f["AB"], want) < 1e-12)


# ----------------------------------------------------------------- barycentric map
def test_map_vertices_and_centroid():
    own = np.array([[1, 1, 1], [9, 2, 1], [2, 10, 3], [3, 2, 12]], np.float64)
    oth = own + np.array([[0.5, 0.25, 0], [1, -1, 0.5], [-0.75, 0.5, 1], [0.25, 0.25, -0.5]])
    # the centroid of own is (15, 15, 17) / 4: use a tet whose centroid is integer
    own[3] = [4, 3, 11]
    cen = own.mean(axis=0)
    assert np.all(cen == np.round(cen))
    for i in range(4):
        q, ex = oracle.map_point(own, oth, own[i].astype(int))
        assert np.array_equal(q, oth[i]) and ex.tolist() == [oth[i][a] == round(oth[i][a])
                                                            for a in range(3)]
    q, _ = oracle.map_point(own, oth, cen.astype(int))
    assert np.allclose(q, oth.mean(axis=0), rtol=0, atol=1e-15)


def test_flat_tet_is_a_fold():
    """A candidate tet of exactly zero volume violates the constraint (a zero
    signed volume cannot have the reference sign); its severity adds 0."""
    ref = np.array([[1, 1, 1], [9, 2, 1], [2, 10, 3], [3, 2, 12]], np.float32)
    flat = ref.copy()
    flat[3] = (ref[0] + ref[1]) / 2                    # on the edge v0-v1: exactly coplanar
    assert oracle.orient(flat) == 0.0
    dims = (16, 16, 16)
    img = np.full(dims[::-1], 0.5, np.float32)
    op = make_oracle(dims, img, img, ref, np.array([[0, 1, 2, 3]], np.int32))
    out = op.evaluate(candidates(flat, ref))
    assert out["flags"][0] == 1 and out["severity"][0] == 0.0
    out = op.evaluate(candidates(ref, ref))
    assert out["flags"][0] == 0


def test_full_box_translation_brute_force(c1):
    """Mesh over the whole image translated by t: mapped points leave the
    grid, so zero padding (intensity) and edge clamping (distance maps) both
    matter; both sums equal a brute-force voxel evaluation."""
    dims = c1.dims
    S = c1.ref_points.astype(np.float64)
    t = np.array([615, -307, 461]) / 1024.0
    r = 3.0
    cs, ct = c1.sets_src[0], c1.sets_tgt[0]
    # foreground up to the border, so that padding and clamping differ
    img_s = (c1.image_src + 0.25).astype(np.float32)
    img_t = (c1.image_tgt + 0.125).astype(np.float32)
    op = make_oracle(dims, img_s, img_t, c1.ref_points, c1.tets, [cs], [ct], radius=r)
    out = op.evaluate(candidates(S, S + t))
    zz, yy, xx = np.meshgrid(*[np.arange(n) for n in dims[::-1]], indexing="ij")
    P = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], -1).astype(np.float64)
    lo, hi = -0.5, np.array(dims) - 0.5
    ins_t = np.all((P - t > lo) & (P - t < hi), axis=1)
    assert out["counts"][0].tolist() == [len(P), int(ins_t.sum())]

    def samp(img, q, mode):
        return ndimage.map_coordinates(img.astype(np.float64), q[:, ::-1].T, order=1, mode=mode,
                                       cval=0.0)

    hs = _h(img_s.ravel().astype(np.float64), samp(img_t, P + t, "grid-constant")).sum()
    ht = _h(img_t.ravel()[ins_t].astype(np.float64), samp(img_s, P[ins_t] - t, "grid-constant")).sum()
    N = len(P) + ins_t.sum()
    assert rel_err(out["obj"][0, 0], (hs + ht) / N) < 1e-12
    snap = lambda a: np.rint(a.astype(np.float64) * 1024) / 1024
    Ds = cKDTree(snap(cs)).query(P)[0].astype(np.float32).astype(np.float64)
    Dt = cKDTree(snap(ct)).query(P)[0].astype(np.float32).astype(np.float64)
    Ds_img, Dt_img = Ds.reshape(dims[::-1]), Dt.reshape(dims[::-1])

    def g(d_own, q, map_oth):
        d2 = samp(map_oth, q, "nearest")
        band = d_own < r
        return np.sum(((r - d_own) / r * (d_own - d2) ** 2)[band])

    gs = g(Ds, P + t, Dt_img)
    gt = g(Dt[ins_t], P[ins_t] - t, Ds_img)
    assert rel_err(out["obj"][0, 2], (gs + gt) / N) < 1e-10
