"""Pins of the oracle's deformation vector fields (Sec. 5.4: forward DVF on
the source grid, inverse DVF on the target grid, rasterized from the two
meshes): identity, translations and global affine maps in closed form, the
coverage of fold-free and folded meshes, and displacements of doubly covered
voxels against a floating-point barycentric solve in the smallest-index tet."""
import numpy as np

import oracle
import synth


def cand(S, T):
    return np.ascontiguousarray(np.stack([np.asarray(S, np.float32).T, np.asarray(T, np.float32).T]))


def grid_points(dims):
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([x, y, z], axis=-1).astype(np.float64)


def test_identity_and_translation():
    p = synth.make_problem(1)
    op = oracle.Problem.from_synth(p)
    fwd, inv, cover = op.dvf(cand(p.ref_points, p.ref_points))
    assert np.all(fwd == 0) and np.all(inv == 0) and np.all(cover == 1)
    t = np.array([1.25, -2.375, 0.6875], np.float32)
    fwd, inv, cover = op.dvf(cand(p.ref_points, p.ref_points + t))
    assert np.all(cover[0] == 1)
    np.testing.assert_array_equal(fwd, np.broadcast_to(t.astype(np.float64), fwd.shape))
    # the target mesh covers the shifted box (-0.5, 31.5) + t
    g = grid_points(p.dims)
    inside = np.all((g > -0.5 + t) & (g < 31.5 + t), axis=-1)
    np.testing.assert_array_equal(cover[1], inside.astype(np.int32))
    np.testing.assert_array_equal(inv[inside], np.broadcast_to(-t.astype(np.float64), inv[inside].shape))
    assert np.all(inv[~inside] == 0)


def test_global_affine_closed_form():
    p = synth.make_problem(1)
    op = oracle.Problem.from_synth(p)
    A = np.array([[1.0625, 0.125, 0.0], [-0.0625, 0.9375, 0.0625], [0.0, 0.03125, 1.0]])
    b = np.array([-0.75, 1.25, 0.5])
    c = np.array([15.5, 15.5, 15.5])
    T = ((p.ref_points.astype(np.float64) - c) @ A.T + c + b).astype(np.float32)
    assert np.array_equal(T.astype(np.float64), (p.ref_points.astype(np.float64) - c) @ A.T + c + b)
    fwd, inv, cover = op.dvf(cand(p.ref_points, T))
    g = grid_points(p.dims)
    np.testing.assert_allclose(fwd, (g - c) @ A.T + c + b - g, rtol=0, atol=1e-9)
    covered = cover[1] == 1
    want_inv = (g - c - b) @ np.linalg.inv(A).T + c - g
    np.testing.assert_allclose(inv[covered], want_inv[covered], rtol=0, atol=1e-9)
    assert np.all(cover[1] <= 1) and covered.mean() > 0.8


def test_folded_mesh_coverage_and_smallest_tet():
    p = synth.make_problem(1)
    op = oracle.Problem.from_synth(p)
    pop = synth.make_population(p, pop=8, seed=31, perturb_source=True, fold_fraction=1.0)
    checked = 0
    for c in range(8):
        fwd, inv, cover = op.dvf(pop[c])
        for d, out in ((0, fwd), (1, inv)):
            if not np.any(cover[d] >= 2):
                continue
            # the meshes on the 2^-10 voxel grid of the rasterization
            own = np.rint(pop[c, d].T.astype(np.float64) * 1024) / 1024
            oth = np.rint(pop[c, 1 - d].T.astype(np.float64) * 1024) / 1024
            zz, yy, xx = np.argwhere(cover[d] >= 2)[0]
            pt = np.array([xx, yy, zz], np.float64)
            # the smallest-index tet whose exact voxel set holds the centre
            v = (zz * p.dims[1] + yy) * p.dims[0] + xx
            for t, tv in enumerate(p.tets):
                if v in oracle.tet_voxels(own[tv], p.dims):
                    break
            E = (own[tv[1:]] - own[tv[0]]).T
            lam = np.linalg.solve(E, pt - own[tv[0]])
            q = oth[tv[0]] + (oth[tv[1:]] - oth[tv[0]]).T @ lam
            np.testing.assert_allclose(out[zz, yy, xx], q - pt, rtol=0, atol=1e-8)
            checked += 1
        # coverage counts sum to the tets' voxel counts
        assert cover[0].sum() == sum(len(oracle.tet_voxels(pop[c, 0].T[tv], p.dims)) for tv in p.tets)
    assert checked >= 3


def test_invalid_vertex_skips_its_tets():
    p = synth.make_problem(1)
    op = oracle.Problem.from_synth(p)
    T = p.ref_points.copy()
    T[62] = np.float32(600.0)                      # the centre point of the 5x5x5 grid
    fwd, inv, cover = op.dvf(cand(p.ref_points, T))
    hole = cover[0] == 0
    assert hole.sum() > 100 and np.all(fwd[hole] == 0) and np.all(cover[0] <= 1)
