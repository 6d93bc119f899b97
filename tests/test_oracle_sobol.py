"""Pins of the oracle's Sobol-sampled estimator (App. A.2) against what the
mathematics fixes: the Sobol sequence against SciPy's, -log against NumPy
within a stated bound, the barycentric points against the moments of the
uniform distribution on a tetrahedron, the sample count against the exact
volume, the intensity term against closed forms on affine images, and the
per-tet sums against SciPy's trilinear interpolation at the same points."""
import numpy as np
import pytest
from scipy import ndimage
from scipy.stats import qmc

import oracle
import synth

TET = np.array([[3.25, 4.0, 5.5], [17.0, 6.125, 4.75], [6.5, 19.5, 7.0], [8.0, 7.25, 18.375]], np.float32)


def bary(tet, pts):
    """Barycentric coordinates of pts [n][3] in tet [4][3] (FP64 solve)."""
    t = tet.astype(np.float64)
    E = (t[1:] - t[0]).T
    lam = np.linalg.solve(E, (pts.astype(np.float64) - t[0]).T).T
    return np.column_stack([1.0 - lam.sum(axis=1), lam])


def six_volume(tet):
    """|6 V| of the snapped tet in 2^-30 voxel^3 units, as a Python integer."""
    v = [[int(np.rint(np.float64(x) * 1024.0)) for x in row] for row in tet]
    a = [v[1][k] - v[0][k] for k in range(3)]
    b = [v[2][k] - v[0][k] for k in range(3)]
    c = [v[3][k] - v[0][k] for k in range(3)]
    d = a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) + a[2] * (b[0] * c[1] - b[1] * c[0])
    return abs(d)


def test_sobol_sequence_matches_scipy():
    # SciPy enumerates the same sequence in Gray-code order: its point i is
    # point i ^ (i >> 1) of the natural order
    ref = qmc.Sobol(d=4, scramble=False, bits=32).random(4096)
    got = np.array([[oracle.sobol_coord(j, i ^ (i >> 1)) for j in range(4)] for i in range(4096)],
                   np.float64) / 2.0 ** 32
    np.testing.assert_array_equal(got, ref)


def test_neg_ln_within_bound():
    rs = np.random.default_rng(0)
    k = np.concatenate([np.arange(64), (1 << 23) - 1 - np.arange(64), rs.integers(0, 1 << 23, 20000)])
    r = ((2 * k + 1) * 2.0 ** -24).astype(np.float32)
    got = np.array([oracle.neg_ln_f32(x) for x in r], np.float64)
    want = -np.log(r.astype(np.float64))
    assert np.all(np.abs(got - want) <= 3e-7 * want + 1e-12)


def test_points_uniform_in_the_tet():
    other = TET * np.float32(0.5) + np.float32(2.0)
    p, q, n = oracle.sobol_points(TET, other, seed=7, rate=4.0)
    assert n == len(p) > 1000
    lam = bary(TET, p)
    assert lam.min() > -1e-5 and lam.max() < 1 + 1e-5
    # moments of the uniform distribution on a tetrahedron (Dirichlet(1,1,1,1)):
    # E[l_i] = 1/4, E[l_i^2] = 1/10, E[l_i l_j] = 1/20
    second = lam.T @ lam / n
    np.testing.assert_allclose(lam.mean(axis=0), 0.25, atol=3e-3)
    np.testing.assert_allclose(np.diag(second), 0.1, atol=3e-3)
    np.testing.assert_allclose(second[~np.eye(4, dtype=bool)], 0.05, atol=3e-3)
    # q has the same barycentric coordinates in the other tet
    np.testing.assert_allclose(bary(other, q), lam, atol=2e-5)


def test_sample_count_is_rounded_volume():
    for rate in (1.0, 0.5, 3.7):
        p, q, n = oracle.sobol_points(TET, TET, rate=rate, cap=0)
        assert n == int(np.floor(rate * six_volume(TET) / 6.0 / 2.0 ** 30 + 0.5))
    flat = TET.copy()
    flat[3] = flat[1] + flat[2] - flat[0]          # in the plane of the other three (exact)
    assert oracle.sobol_points(flat, flat, cap=0)[2] == 0
    huge = np.array([[0, 0, 0], [400, 0, 0], [0, 400, 0], [0, 0, 400]], np.float32)
    assert oracle.sobol_points(huge, huge, cap=0)[2] == 1 << 20
    with pytest.raises(ValueError):
        oracle.sobol_points(TET, TET, rate=0.0)


def test_points_depend_on_own_tet_seed_and_direction_only():
    p0, _, _ = oracle.sobol_points(TET, TET, seed=1)
    p1, q1, _ = oracle.sobol_points(TET, TET + np.float32(1.5), seed=1)
    np.testing.assert_array_equal(p0, p1)
    assert not np.array_equal(oracle.sobol_points(TET, TET, seed=2)[0], p0)
    assert not np.array_equal(oracle.sobol_points(TET, TET, direction=1, seed=1)[0], p0)
    moved = TET.copy()
    moved[0, 0] += np.float32(2 ** -10)
    assert not np.array_equal(oracle.sobol_points(moved, moved, seed=1)[0][:10], p0[:10])


def affine_problem(grad, c0, shift_img=(0.0, 0.0, 0.0), n=32):
    """Config-1 topology squeezed into [4, 27]^3 on n^3 affine images
    I(x) = c0 + grad . (x - shift_img) (I_s unshifted, I_t shifted), so that
    every trilinear stencil stays inside the grid and reproduces the affine
    function exactly; no guidance sets."""
    p = synth.make_problem(1)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    img_s = (c0 + grad[0] * x + grad[1] * y + grad[2] * z).astype(np.float32)
    img_t = (c0 + grad[0] * (x - shift_img[0]) + grad[1] * (y - shift_img[1]) +
             grad[2] * (z - shift_img[2])).astype(np.float32)
    ref = (np.float32(4.0) + (p.ref_points + np.float32(0.5)) * np.float32(23.0 / 32.0)).astype(np.float32)
    ref = np.rint(ref * 1024) / 1024
    prob = oracle.Problem((n, n, n), img_s, img_t, p.tets, ref, p.elasticity, [], [], 1.0)
    return prob, ref.astype(np.float32)


def test_translated_mesh_on_affine_images_closed_form():
    grad = np.array([0.013, -0.021, 0.017])
    t = np.array([0.375, -0.5, 0.8125], np.float32)
    prob, ref = affine_problem(grad, 2.0)
    pts = np.stack([ref.T, (ref + t).T])[None].astype(np.float32)
    out = prob.evaluate_sobol(pts, seed=3)
    # every sample is in the foreground of both images; b - a = grad . t
    assert out["flags"][0] == 0
    np.testing.assert_allclose(out["obj"][0, 0], float(grad @ t) ** 2, rtol=1e-4)
    assert out["counts"][0, 0] == out["counts"][0, 1]
    assert abs(out["counts"][0, 0] - 23.0 ** 3) <= prob.n_tets / 2
    # I_t shifted by the same t: the deformation is matched exactly, h = 0
    prob2, _ = affine_problem(grad, 2.0, shift_img=t)
    assert prob2.evaluate_sobol(pts, seed=3)["obj"][0, 0] < 1e-10


def test_scaled_mesh_on_affine_image_matches_uniform_moments():
    """T = s S about the centre: b - a = grad . (q - p) is affine in p, so the
    mean of h over uniform samples of a tet is (grad . (q(c) - c))^2 +
    beta^T Cov beta with Cov = sum_i (v_i - c)(v_i - c)^T / 20; the total is
    checked against the volume-weighted sum of those exact tet means."""
    grad = np.array([0.02, 0.011, -0.015])
    prob, ref = affine_problem(grad, 3.0)
    centre = np.float32(15.5)
    tgt = (centre + (ref - centre) * np.float32(0.92)).astype(np.float32)
    tgt = np.rint(tgt * 1024) / 1024
    pts = np.stack([ref.T, tgt.T])[None].astype(np.float32)
    out = prob.evaluate_sobol(pts, seed=5, rate=4.0)
    want_h, want_n = 0.0, 0.0
    for own, oth in ((ref, tgt), (tgt, ref)):
        for tet in prob.tets:
            v, w = own[tet].astype(np.float64), oth[tet].astype(np.float64)
            vol = abs(np.linalg.det(v[1:] - v[0])) / 6.0
            E = v[1:] - v[0]
            L = (w[1:] - w[0]).T @ np.linalg.inv(E.T)          # q = w0 + L (p - v0)
            c = v.mean(axis=0)
            beta = (L - np.eye(3)).T @ grad
            alpha = grad @ (w[0] + L @ (c - v[0]) - c)
            cov = sum(np.outer(x - c, x - c) for x in v) / 20.0
            want_h += vol * (alpha ** 2 + beta @ cov @ beta)
            want_n += vol
    got = out["obj"][0, 0]
    np.testing.assert_allclose(got, want_h / want_n, rtol=2e-2)


def scipy_tet_terms(prob, p, q, own_img, oth_img, own_maps, oth_maps, set_w):
    """h and guidance sums at given points, interpolated by SciPy."""
    def interp(vol, x, mode):
        return ndimage.map_coordinates(vol.astype(np.float64), [x[:, 2], x[:, 1], x[:, 0]], order=1, mode=mode)

    def support_fg(vol, x):
        x = x.astype(np.float64)
        k = np.floor(x).astype(np.int64)
        f = x - k
        nz, ny, nx = vol.shape
        fg = np.zeros(len(x), bool)
        for cz in (0, 1):
            for cy in (0, 1):
                for cx in (0, 1):
                    w = (f[:, 0] > 0) | (cx == 0)
                    w &= (f[:, 1] > 0) | (cy == 0)
                    w &= (f[:, 2] > 0) | (cz == 0)
                    ix, iy, iz = k[:, 0] + cx, k[:, 1] + cy, k[:, 2] + cz
                    inb = (ix >= 0) & (ix < nx) & (iy >= 0) & (iy < ny) & (iz >= 0) & (iz < nz)
                    val = np.zeros(len(x))
                    val[inb] = vol[iz[inb], iy[inb], ix[inb]]
                    fg |= w & (val > 0)
        return fg

    fa, fb = support_fg(own_img, p), support_fg(oth_img, q)
    a = np.where(fa, interp(own_img, p, "grid-constant"), 0.0)
    b = np.where(fb, interp(oth_img, q, "grid-constant"), 0.0)
    h = np.where(fa & fb, (a - b) ** 2, np.where(fa == fb, 0.0, 1.0)).sum()
    g = 0.0
    r = prob.radius
    for s in range(len(set_w)):
        d = interp(own_maps[s], p, "nearest")
        d2 = interp(oth_maps[s], q, "nearest")
        m = d < r
        g += set_w[s] * np.sum((r - d[m]) / r * (d[m] - d2[m]) ** 2)
    return h, g


def test_tet_sums_match_scipy_interpolation():
    p = synth.make_problem(1)
    prob = oracle.Problem.from_synth(p)
    pop = synth.make_population(p, pop=2, seed=11)
    out = prob.evaluate_sobol(pop, seed=9, records=True)
    rec = out["records"]
    ws = np.array([len(s) for s in prob.sets_src], np.float64)
    wt = np.array([len(s) for s in prob.sets_tgt], np.float64)
    ws, wt = ws / ws.sum(), wt / wt.sum()
    rs = np.random.default_rng(1)
    checked = 0
    for c in range(2):
        S = pop[c, 0].T
        T = pop[c, 1].T
        for t in rs.choice(prob.n_tets, 40, replace=False):
            tet = prob.tets[t]
            for d, (own, oth, oi, xi, om, xm, w) in enumerate((
                    (S, T, prob.image_src, prob.image_tgt, prob.dmap_s, prob.dmap_t, ws),
                    (T, S, prob.image_tgt, prob.image_src, prob.dmap_t, prob.dmap_s, wt))):
                pp, qq, n = oracle.sobol_points(own[tet], oth[tet], direction=d, seed=9)
                assert n == rec[c, t, d, 2]
                if n == 0:
                    continue
                h, g = scipy_tet_terms(prob, pp, qq, oi, xi, om, xm, w)
                np.testing.assert_allclose(rec[c, t, d, 0], h, rtol=1e-9, atol=1e-12)
                np.testing.assert_allclose(rec[c, t, d, 1], g, rtol=1e-9, atol=1e-12)
                checked += 1
    assert checked > 100
    # the objectives are these sums over all tets
    H = rec[..., 0].sum(axis=(1, 2))
    N = rec[..., 2].sum(axis=(1, 2))
    np.testing.assert_allclose(out["obj"][:, 0], H / N, rtol=1e-12)
    np.testing.assert_array_equal(out["counts"].sum(axis=1), N)


def test_sobol_shares_magnitude_folds_and_volume_with_rasterized():
    """The magnitude and the folds do not depend on the samples; the point
    counts are the rounded volumes, so each direction's total is within half a
    point per tet of the voxel count of a mesh tiling the grid."""
    p = synth.make_problem(1)
    prob = oracle.Problem.from_synth(p)
    pop = synth.make_population(p, pop=3, seed=4)
    a = prob.evaluate(pop)
    b = prob.evaluate_sobol(pop, seed=1)
    np.testing.assert_array_equal(b["obj"][:, 1], a["obj"][:, 1])
    np.testing.assert_array_equal(b["flags"], a["flags"])
    np.testing.assert_array_equal(b["severity"], a["severity"])
    ident = np.stack([p.ref_points.T, p.ref_points.T])[None].astype(np.float32)
    c = prob.evaluate_sobol(ident, seed=1)["counts"][0]
    assert np.all(np.abs(c - 32 ** 3) <= prob.n_tets / 2)
