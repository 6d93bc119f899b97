"""Pins of the FP64 reference of the surrogate's inputs and targets.

Region statistics: against SciPy's labelled-region statistics
(scipy.ndimage.mean / variance / sum over a label volume built from the
oracle's voxel lists), closed forms on constant images, and the reference
mesh's exact tiling of the grid.  Targets: the count-weighted sum of a
candidate's per-tet targets is its intensity objective times its sample
count (Sec. 4.1.2's objective is the mean of h over all samples); an offspring
equal to its parent has zero targets.  Input rows: vertex moves of known
offsets, and on an affine image (which trilinear interpolation reproduces
exactly) the image samples in closed form, points outside the box clamped."""
import numpy as np
import pytest
from scipy import ndimage

import oracle
import synth
from conftest import oracle_problem, synth_problem
from oracle import surrogate_inputs as si


def label_volume(op):
    lab = np.zeros(int(np.prod(op.dims)), np.int64)
    for t, tet in enumerate(op.tets):
        vox = oracle.tet_voxels(op.ref_points[tet], op.dims)
        assert np.all(lab[vox] == 0)                      # no voxel in two tets
        lab[vox] = t + 1
    return lab


def test_region_stats_match_scipy_labelled_statistics():
    op = oracle_problem(1)
    st, cnt = si.region_stats(op)
    lab = label_volume(op)
    assert np.all(lab > 0)                                # every voxel in one tet
    idx = np.arange(1, op.n_tets + 1)
    Is = op.image_src.reshape(-1).astype(np.float64)
    It = op.image_tgt.reshape(-1).astype(np.float64)
    np.testing.assert_array_equal(cnt, ndimage.sum(np.ones_like(Is), lab, idx))
    for k, (img, fn) in enumerate([(Is, ndimage.mean), (Is, ndimage.variance), (Is > 0, ndimage.mean),
                                   (It, ndimage.mean), (It, ndimage.variance), (It > 0, ndimage.mean),
                                   ((Is - It) ** 2, ndimage.mean)]):
        with np.errstate(invalid="ignore"):       # SciPy's unused label 0 has no voxels
            want = fn(img.astype(np.float64), lab, idx)
        got = st[:, k] ** 2 if fn is ndimage.variance else st[:, k]
        np.testing.assert_allclose(got, want, rtol=1e-9, atol=1e-14, err_msg=f"stat {k}")
    np.testing.assert_allclose(st[:, 7], cnt * op.n_tets / np.prod(op.dims), rtol=1e-15)


def test_region_stats_constant_images():
    p = synth_problem(1)
    a = np.full(p.image_src.shape, 0.25, np.float32)
    b = np.full(p.image_src.shape, 0.75, np.float32)
    b[:, :, :16] = 0.0                                    # half the grid is background in I_t
    op = oracle.Problem.from_synth(p, image_src=a, image_tgt=b)
    st, cnt = si.region_stats(op)
    assert cnt.sum() == np.prod(p.dims)
    np.testing.assert_allclose(st[:, 0], 0.25, rtol=1e-15)
    np.testing.assert_allclose(st[:, 1], 0.0, atol=1e-15)
    np.testing.assert_allclose(st[:, 2], 1.0, rtol=0)
    # per tet: the fraction f of its voxels with x >= 16 sees 0.75, the rest 0
    lab = label_volume(op)
    x = np.arange(np.prod(p.dims)) % p.dims[0]
    f = ndimage.mean((x >= 16).astype(np.float64), lab, np.arange(1, op.n_tets + 1))
    np.testing.assert_allclose(st[:, 3], 0.75 * f, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(st[:, 4], 0.75 * np.sqrt(f * (1 - f)), rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(st[:, 5], f, rtol=1e-15)
    np.testing.assert_allclose(st[:, 6], f * 0.25 + (1 - f) * 0.0625, rtol=1e-12)


def test_targets_weighted_sum_is_the_intensity_objective():
    p = synth_problem(1)
    op = oracle_problem(1)
    pop = synth.make_population(p, pop=4, seed=17, perturb_source=True, fold_fraction=0.5)
    out = op.evaluate(pop, records=True)
    t = si.mean_terms(out["records"])
    rec = out["records"]
    n = rec[..., 0, 2] + rec[..., 1, 2]
    np.testing.assert_allclose((t * n).sum(axis=1), out["obj"][:, 0] * out["counts"].sum(axis=1),
                               rtol=1e-12)
    assert np.all(t[n == 0] == 0)


def test_records_fields_consistent_with_outputs():
    """The records' sums reproduce every output of the evaluation: counts,
    flags (any violation per direction), severity, magnitude and guidance."""
    p = synth_problem(1)
    op = oracle_problem(1)
    pop = synth.make_population(p, pop=4, seed=19, perturb_source=True, fold_fraction=0.5)
    out = op.evaluate(pop, records=True)
    rec = out["records"]
    assert (out["flags"] & 3).any()
    np.testing.assert_array_equal(rec[..., 2].sum(axis=1).astype(np.int64), out["counts"])
    fl = (rec[..., 0, 5].max(axis=1) > 0).astype(int) | (rec[..., 1, 5].max(axis=1) > 0).astype(int) << 1
    np.testing.assert_array_equal(fl, out["flags"])
    np.testing.assert_allclose(rec[..., 4].sum(axis=(1, 2)), out["severity"], rtol=1e-12)
    assert np.all(rec[..., 4][rec[..., 5] == 0] == 0)
    N = out["counts"].sum(axis=1)
    np.testing.assert_allclose(rec[..., 1].sum(axis=(1, 2)) / N, out["obj"][:, 2], rtol=1e-12)
    np.testing.assert_allclose(rec[..., 0, 3].sum(axis=1) / (10 * op.n_tets), out["obj"][:, 1], rtol=1e-12)
    assert np.all(rec[..., 1, 3] == 0)


def test_targets_are_changes_from_the_parent():
    p = synth_problem(1)
    op = oracle_problem(1)
    parents = synth.make_population(p, pop=2, seed=23, perturb_source=False, fold_fraction=0.0)
    kids = parents[[0, 1, 1, 0]].copy()
    kids[2, 1] += np.float32(0.25)                        # a shift of the whole target mesh
    kids[3, 1, :, 5] += np.float32(0.5)
    po = op.evaluate(parents, records=True)
    ko = op.evaluate(kids, records=True)
    of = np.array([0, 1, 1, 7])
    t = si.targets(ko["records"], po["records"], of, 0.5)
    assert np.all(t[0] == 0) and np.all(t[1] == 0)
    assert np.any(t[2] != 0)
    assert np.all(np.isnan(t[3]))
    # the mean terms come back as parent term + scale x target
    np.testing.assert_allclose(0.5 * t[2] + si.mean_terms(po["records"])[1], si.mean_terms(ko["records"])[2],
                               rtol=1e-12, atol=1e-15)


def test_point_sets_by_hand():
    L = si.point_sets()
    assert L.shape == (26, 4)
    np.testing.assert_array_equal(L[:4], np.eye(4))
    np.testing.assert_array_equal(L[4], [0.5, 0.5, 0, 0])
    np.testing.assert_array_equal(L[9], [0, 0, 0.5, 0.5])
    # Halton j = 1: (1/2, 1/3, 1/5); j = 2: (1/4, 2/3, 2/5); j = 3: (3/4, 1/9, 3/5)
    np.testing.assert_allclose(L[10], [1 / 5, 1 / 3 - 1 / 5, 1 / 2 - 1 / 3, 1 / 2], rtol=1e-15)
    np.testing.assert_allclose(L[11], [1 / 4, 2 / 5 - 1 / 4, 2 / 3 - 2 / 5, 1 / 3], rtol=1e-15)
    np.testing.assert_allclose(L[12], [1 / 9, 3 / 5 - 1 / 9, 3 / 4 - 3 / 5, 1 / 4], rtol=1e-15)
    assert np.all(L >= 0) and np.allclose(L.sum(axis=1), 1.0, rtol=0, atol=1e-15)
    assert len({tuple(r) for r in L[10:]}) == 16 and np.all(L[10:] > 0)


def test_weights_tile_the_box_and_score_forms():
    p = synth_problem(1)
    op = oracle_problem(1)
    ident = np.stack([p.ref_points.T, p.ref_points.T]).astype(np.float32)
    w = si.weights(op, ident)
    nx, ny, nz = p.dims
    lo, hi = p.ref_points.min(axis=0), p.ref_points.max(axis=0)        # the mesh's box
    np.testing.assert_allclose(w.sum(), 2.0 * np.prod(hi.astype(np.float64) - lo), rtol=1e-12)
    parents = synth.make_population(p, pop=2, seed=37, perturb_source=False, fold_fraction=0.0)
    po = op.evaluate(parents, records=True)
    tp = si.mean_terms(po["records"])
    kids = parents[[1, 0]]
    zero = np.zeros((2, op.n_tets))
    sc = si.score(op, kids, po["records"], np.array([1, 0]), zero)
    for k, q in enumerate([1, 0]):
        wk = si.weights(op, kids[k])
        np.testing.assert_allclose(sc[k], (wk * tp[q]).sum() / wk.sum(), rtol=1e-12)
    # the parent itself with zero change: close to its exact f_int (the
    # volumes stand in for the sample counts)
    np.testing.assert_allclose(sc, po["obj"][[1, 0], 0], rtol=0.02)
    hs = si.h_scale(op)
    sc2 = si.score(op, kids, po["records"], np.array([1, 0]), zero + 3.0)
    np.testing.assert_allclose(sc2 - sc, 3.0 * hs, rtol=1e-9)
    assert np.all(np.isinf(si.score(op, kids, po["records"], np.array([-1, 2]), zero)))


def test_features_closed_forms_on_an_affine_image():
    """I_s constant c0 and I_t affine: every h value has a closed form at
    the point clamped into the box."""
    p = synth_problem(1)
    nx, ny, nz = p.dims
    a = np.array([0.011, -0.007, 0.013])
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    img = (a[0] * i + a[1] * j + a[2] * k + 0.4).astype(np.float32)
    c0 = np.float32(0.3)
    op = oracle.Problem.from_synth(p, image_src=np.full(img.shape, c0, np.float32), image_tgt=img)
    st, _ = si.region_stats(op)
    hs = si.h_scale(op)
    np.testing.assert_allclose(hs, np.mean((np.float64(c0) - img.astype(np.float64)) ** 2), rtol=1e-12)
    parents = synth.make_population(p, pop=2, seed=29, perturb_source=False, fold_fraction=0.0)
    rs = np.random.default_rng(3)
    kids = parents[[1, 0, 1]].copy()
    kids[:, 1] += rs.normal(0, 0.5, kids[:, 1].shape).astype(np.float32)
    kids[2, 1, :, 0] += np.float32(4.0 * max(p.dims))     # one vertex far outside the box
    po = op.evaluate(parents, records=True)
    of = np.array([1, 0, 1])
    F = si.features(op, st, kids, parents, po["records"], of)
    hi = np.array([nx - 1, ny - 1, nz - 1], np.float64)
    L = si.point_sets()

    def means(cand):
        T = cand[1].astype(np.float64).T[p.tets]                          # [n_tets][4][3]
        y = np.einsum("jv,tva->tja", L, T)
        h = (np.float64(c0) - (np.clip(y, 0.0, hi) @ a + 0.4)) ** 2       # [n_tets][26]
        return np.stack([h[:, :4].mean(1), h[:, 4:10].mean(1), h[:, 10:].mean(1)], axis=1)

    tp = si.mean_terms(po["records"])
    for e, q in enumerate(of):
        moved = (kids[e, 1].astype(np.float64) - parents[q, 1].astype(np.float64)).T[p.tets]
        np.testing.assert_allclose(F[e, :, :12], 2.0 * moved.reshape(-1, 12), rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(F[e, :, 12:15], (means(kids[e]) - means(parents[q])) / hs, rtol=1e-5,
                                   atol=1e-6)
        np.testing.assert_array_equal(F[e, :, 15:21], st[:, :6])
        np.testing.assert_allclose(F[e, :, 21], st[:, 6] / hs, rtol=1e-15)
        np.testing.assert_allclose(F[e, :, 22], tp[q] / hs, rtol=1e-15)
    # no parent: a row of NaN
    F2 = si.features(op, st, kids[:1], parents, po["records"], np.array([-1]))
    assert np.all(np.isnan(F2))
