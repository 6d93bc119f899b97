"""GPU parity of DVF rasterization and of the point-based guidance error (HIP
path via the C-ABI) against the oracle: coverage counts and unmapped counts
bit-exact, displacements within FP32 rounding of the oracle's exact
barycentric images (2e-6 voxel + 1e-6 relative), guidance errors within 1e-6
relative (FP64 sums rounded to FP32)."""
import numpy as np
import pytest

import oracle
import synth
from conftest import oracle_problem, synth_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2303_04873_amd as morea  # noqa: E402


def run(prob, cand):
    out = prob.rasterize_dvf(torch.from_numpy(np.ascontiguousarray(cand, dtype=np.float32)).cuda())
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def check(prob, op, cand):
    g = run(prob, cand)
    fwd, inv, cover = op.dvf(cand)
    np.testing.assert_array_equal(g["cover"], cover)
    np.testing.assert_allclose(g["fwd"], fwd, rtol=1e-6, atol=2e-6)
    np.testing.assert_allclose(g["inv"], inv, rtol=1e-6, atol=2e-6)
    return g, cover


def test_c1_identity_translation_perturbed_and_folded():
    p = synth_problem(1)
    prob = morea.Problem.from_synth(p, max_population=1)
    op = oracle_problem(1)
    S = p.ref_points
    check(prob, op, np.stack([S.T, S.T]))
    check(prob, op, np.stack([S.T, (S + np.float32(1.25)).T]))
    pop = synth.make_population(p, pop=6, seed=31, perturb_source=True, fold_fraction=0.5)
    folded = 0
    for c in range(6):
        _, cover = check(prob, op, pop[c])
        folded += int((cover != 1).any())
    assert folded >= 2


def test_invalid_vertex_and_mesh_outside():
    p = synth_problem(1)
    prob = morea.Problem.from_synth(p, max_population=1)
    op = oracle_problem(1)
    T = p.ref_points.copy()
    T[62] = np.float32(np.inf)
    _, cover = check(prob, op, np.stack([p.ref_points.T, T.T]))
    assert (cover[0] == 0).sum() > 100
    far = p.ref_points + np.float32(40.0)          # the target mesh entirely outside the grid
    g, cover = check(prob, op, np.stack([p.ref_points.T, far.T]))
    assert np.all(cover[1] == 0) and np.all(g["inv"] == 0)


def test_c2_candidate_full_size():
    p = synth_problem(2)
    prob = morea.Problem.from_synth(p, max_population=1)
    pop = synth.make_population(p, pop=2)
    for c in range(2):                                # candidate 0 carries a fold
        check(prob, oracle_problem(2), pop[c])


def guidance(prob, pts):
    f, un = prob.point_guidance(torch.from_numpy(np.ascontiguousarray(pts, dtype=np.float32)).cuda())
    torch.cuda.synchronize()
    return f.cpu().numpy().astype(np.float64), un.cpu().numpy()


def test_point_guidance_c1_population_and_edges():
    p = synth_problem(1)
    pop = synth.make_population(p, pop=16, seed=51, perturb_source=True, fold_fraction=0.25)
    pop[15, 0, 1, 3] = np.nan                           # invalid
    prob = morea.Problem.from_synth(p, max_population=16)
    f, un = guidance(prob, pop)
    fo, uno = oracle_problem(1).point_guidance(pop)
    np.testing.assert_array_equal(un, uno)
    assert np.isnan(f[15]) and np.isnan(fo[15])
    np.testing.assert_allclose(f[:15], fo[:15], rtol=1e-6)
    # points outside the mesh, and a problem without guidance sets
    pts = (np.rint(np.array([[4.25, 5.5, 6.0], [-3.0, 5.0, 5.0], [20.0, 8.25, 12.5]]) * 1024) / 1024).astype(np.float32)
    prob2 = morea.Problem(p.dims, p.image_src, p.image_tgt, p.tets, p.ref_points, p.elasticity, [pts],
                          [pts + np.float32(0.5)], radius=2.0, max_population=16)
    op2 = oracle.Problem(p.dims, p.image_src, p.image_tgt, p.tets, p.ref_points, p.elasticity, [pts],
                         [pts + np.float32(0.5)], 2.0)
    f, un = guidance(prob2, pop[:4])
    fo, uno = op2.point_guidance(pop[:4])
    np.testing.assert_array_equal(un, uno)
    assert np.all(un >= 1)
    np.testing.assert_allclose(f, fo, rtol=1e-6)
    prob3 = morea.Problem(p.dims, p.image_src, p.image_tgt, p.tets, p.ref_points, p.elasticity, [], [],
                          radius=2.0, max_population=16)
    f, un = guidance(prob3, pop[:2])
    assert np.all(np.isnan(f)) and np.all(un == 0)


def test_point_guidance_c2_population():
    p = synth_problem(2)
    pop = synth.make_population(p)
    prob = morea.Problem.from_synth(p, max_population=512)
    f, un = guidance(prob, pop)
    idx = [0, 1, 300, 511]
    fo, uno = oracle_problem(2).point_guidance(pop[idx])
    np.testing.assert_array_equal(un[idx], uno)
    np.testing.assert_allclose(f[idx], fo, rtol=1e-6)
    assert np.all(np.isfinite(f)) and np.all(un == 0)
