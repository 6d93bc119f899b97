"""GPU parity of full evaluation (HIP path via the C-ABI) against the oracle.

Sizes: the 32^3 phantom with 384 tets (the oracle finishes the whole
population in well under a second; tets span several rows and sample
batches, with ragged tails) and the 128x128x96 phantom with 3,402 tets and
population 512 in the launch configuration of the benchmark, compared on a
sample of candidates that the oracle evaluates one by one, plus properties
that hold for every candidate at full size."""
import numpy as np
import pytest

import oracle
import synth
from conftest import oracle_problem, synth_problem
from parity import assert_parity, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2303_04873_amd as morea  # noqa: E402


def gpu_problem(p, storage="f32", max_pop=16, **kw):
    return morea.Problem.from_synth(p, storage=storage, max_population=max_pop, **kw)


def run(prob, pts):
    t = torch.from_numpy(np.ascontiguousarray(pts)).cuda()
    out = prob.eval_full(t)
    torch.cuda.synchronize()
    return to_host(out)


def cand(S, T):
    return np.stack([np.asarray(S, np.float32).T, np.asarray(T, np.float32).T])[None]


def test_c1_population():
    p = synth_problem(1)
    pop = synth.make_population(p)
    g = run(gpu_problem(p), pop)
    assert_parity(g, oracle_problem(1).evaluate(pop), what="c1")
    assert np.all(g["counts"] == np.prod(p.dims))


def test_c1_dual_with_folds_and_invalid():
    p = synth_problem(1)
    pop = synth.make_population(p, pop=16, seed=101, perturb_source=True, fold_fraction=0.25)
    pop[15, 1, 0, 7] = 700.0        # invalid coordinate
    pop[14, 0, 2, 3] = np.nan       # invalid coordinate
    g = run(gpu_problem(p), pop)
    o = oracle_problem(1).evaluate(pop)
    assert (o["flags"] & 3).any() and (o["flags"][14:] == 4).all()
    assert_parity(g, o, what="c1 dual")


def test_c1_identity_and_exact_paths():
    """S = T = grid: every mapped point is a voxel centre, so every sample takes
    the exact support path; with I_t = I_s the intensity is exactly 0."""
    p = synth_problem(1)
    S = p.ref_points
    prob = gpu_problem(p, image_tgt=p.image_src)
    g = run(prob, cand(S, S))
    assert g["obj"][0, 0] == 0.0 and g["obj"][0, 1] == 0.0
    prob2 = gpu_problem(p)
    g2 = run(prob2, cand(S, S))
    assert_parity(g2, oracle_problem(1).evaluate(cand(S, S)), what="identity")
    # integer translation of the target mesh: mapped points on the grid again
    T = S + np.array([1.0, -2.0, 1.0], np.float32)
    pts = cand(S, T)
    assert_parity(run(prob2, pts), oracle_problem(1).evaluate(pts), what="integer shift")


def test_tiny_intensities_take_corner_test():
    """Positive intensities below 2^-39 (here 1e-30 and 1e-37, both normal
    FP32) switch the foreground test of ordinary samples from b > 0 to the
    corners' bits: b of a sample whose only positive corner holds 1e-37
    underflows to 0 while the exact support still says foreground."""
    p = synth_problem(1)
    img = p.image_src.copy()
    bg = np.argwhere(img == 0)
    rs = np.random.default_rng(7)
    pick = bg[rs.choice(len(bg), 400, replace=False)]
    img[tuple(pick[:200].T)] = 1e-30
    img[tuple(pick[200:].T)] = 1e-37
    pop = synth.make_population(p, pop=8, seed=17, perturb_source=True)
    g = run(gpu_problem(p, image_src=img), pop)
    o = oracle.Problem.from_synth(p, image_src=img).evaluate(pop)
    assert_parity(g, o, what="tiny intensities")


def test_large_tets_take_int64_path():
    """Tets wider than 64 voxels use the int64 plane arithmetic."""
    dims = (100, 90, 80)
    pts, tets, fixed = synth.kuhn_grid(dims, (2, 2, 2))
    rs = np.random.default_rng(3)
    img_s = (rs.uniform(0, 1, dims[::-1]) * (rs.uniform(0, 1, dims[::-1]) > 0.3)).astype(np.float32)
    img_t = (rs.uniform(0, 1, dims[::-1]) * (rs.uniform(0, 1, dims[::-1]) > 0.3)).astype(np.float32)
    el = np.ones(len(tets), np.float32)
    sets = [rs.uniform(10, 70, size=(5, 3)).astype(np.float32)]
    prob = morea.Problem(dims, img_s, img_t, tets, pts, el, sets, [sets[0] + 1.5], radius=6.0,
                         max_population=4)
    op = oracle.Problem(dims, img_s, img_t, tets, pts, el, sets, [sets[0] + 1.5], 6.0)
    cands = []
    for k in range(4):
        T = pts + np.where(fixed, 0, rs.normal(0, 3.0, pts.shape))
        S = pts + np.where(fixed, 0, rs.normal(0, 1.0, pts.shape)) if k % 2 else pts
        cands.append(cand(S, T)[0])
    cands = np.stack(cands).astype(np.float32)
    assert_parity(run(prob, cands), op.evaluate(cands), what="int64 path")


def test_mesh_partly_outside_image():
    p = synth_problem(1)
    S = p.ref_points + np.array([5.25, -3.5, 2.0], np.float32)
    rs = np.random.default_rng(5)
    T = p.target_base + rs.normal(0, 0.5, p.target_base.shape).astype(np.float32) + 7.0
    pts = cand(S, T)
    g = run(gpu_problem(p), pts)
    o = oracle_problem(1).evaluate(pts)
    assert o["counts"][0, 0] < np.prod(p.dims)
    assert_parity(g, o, what="outside")


def test_degenerate_candidate_tet():
    p = synth_problem(1)
    S = p.ref_points.copy()
    T = p.target_base.copy()
    t = p.tets[100]
    T[t[3]] = (T[t[0]] + T[t[1]] + T[t[2]]) / 3   # flatten (not exactly, snapped)
    T[t[3]] = T[t[0]]                               # exactly flat
    pts = cand(S, T)
    assert_parity(run(gpu_problem(p), pts), oracle_problem(1).evaluate(pts), what="flat")


def test_distance_maps_match_oracle():
    p = synth_problem(1)
    prob = gpu_problem(p)
    op = oracle_problem(1)
    for img in (0, 1):
        for s in range(len(p.sets_src)):
            dm, band = prob.distance_map(img, s)
            ref = (op.dmap_s if img == 0 else op.dmap_t)[s]
            ulp = np.abs(dm.view(np.int32).astype(np.int64) - ref.view(np.int32).astype(np.int64))
            assert ulp.max() <= 1
            np.testing.assert_array_equal((band >> s) & 1, (ref < np.float32(p.radius)).astype(np.uint8))


def test_determinism_and_pop_sizes():
    p = synth_problem(1)
    pop = synth.make_population(p)
    prob = gpu_problem(p)
    a = run(prob, pop)
    b = run(prob, pop)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])
    one = run(prob, pop[5:6])
    for k in a:
        np.testing.assert_array_equal(one[k][0], a[k][5])
    # empty population is a no-op
    empty = torch.empty((0, 2, 3, p.n_points), dtype=torch.float32, device="cuda")
    prob.eval_full(empty)
    with pytest.raises(morea.MoreaError):
        prob.eval_full(torch.from_numpy(np.concatenate([pop, pop[:1]])).cuda())


def test_c2_population_sampled():
    """Config 2 at full size in the benchmark's launch configuration (pop 512):
    sampled candidates against the oracle, coverage for every fold-free one."""
    p = synth_problem(2)
    pop = synth.make_population(p)
    prob = gpu_problem(p, max_pop=512)
    g = run(prob, pop)
    V = int(np.prod(p.dims))
    free = (g["flags"] == 0)
    assert free.sum() >= 400
    assert np.all(g["counts"][free] == V)
    idx = [0, 1, 17, 300, 511]          # 0 has an injected fold
    o = oracle_problem(2).evaluate(pop[idx])
    assert o["flags"][0] != 0
    assert_parity(g, o, idx=idx, what="c2")
