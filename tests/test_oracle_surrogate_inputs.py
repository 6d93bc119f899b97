"""Pins of the FP64 reference of the surrogate's inputs and targets.

Region statistics: against SciPy's labelled-region statistics
(scipy.ndimage.mean / variance / sum over a label volume built from the
oracle's voxel lists), closed forms on constant images, and the reference
mesh's exact tiling of the grid.  Targets: the count-weighted sum of a
candidate's per-tet targets is its intensity objective times its sample
count (Sec. 4.1.2's objective is the mean of h over all samples)."""
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
    t = si.targets(out["records"])
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
