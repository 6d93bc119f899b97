"""GPU parity of the Sobol-sampled estimator (HIP path via the C-ABI) against
the oracle's, on the same seeded inputs: sample counts and flags bit-exact,
objectives within 1e-5 relative.  Both sides form the sample points from the
same definition in FP32, so the same points are sampled; the oracle then
interpolates in FP64.

Sizes: the 32^3 phantom (whole population, several rates and seeds,
folds, invalid and flat candidates, reduced-precision storage) and the
128x128x96 phantom with population 512 in the benchmark's launch
configuration, compared on sampled candidates."""
import numpy as np
import pytest

import oracle
import synth
from conftest import oracle_problem, synth_problem
from parity import assert_parity, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2303_04873_amd as morea  # noqa: E402


def run(prob, pts, rate=1.0, seed=0):
    t = torch.from_numpy(np.ascontiguousarray(pts)).cuda()
    out = prob.eval_sobol(t, rate=rate, seed=seed)
    torch.cuda.synchronize()
    return to_host(out)


def cand(S, T):
    return np.stack([np.asarray(S, np.float32).T, np.asarray(T, np.float32).T])[None]


@pytest.mark.parametrize("rate,seed", [(1.0, 0), (2.5, 12345), (0.3, 7)])
def test_c1_population(rate, seed):
    p = synth_problem(1)
    pop = synth.make_population(p)
    prob = morea.Problem.from_synth(p, max_population=16)
    assert_parity(run(prob, pop, rate, seed), oracle_problem(1).evaluate_sobol(pop, rate=rate, seed=seed),
                  what=f"c1 rate {rate} seed {seed}")


def test_c1_dual_with_folds_invalid_and_flat():
    p = synth_problem(1)
    pop = synth.make_population(p, pop=16, seed=101, perturb_source=True, fold_fraction=0.25)
    pop[15, 1, 0, 7] = 700.0        # invalid coordinate
    pop[14, 0, 2, 3] = np.nan       # invalid coordinate
    t = p.tets[100]
    pop[13, 1, :, t[3]] = pop[13, 1, :, t[0]]   # a flat target tet: no samples, a fold
    prob = morea.Problem.from_synth(p, max_population=16)
    o = oracle_problem(1).evaluate_sobol(pop, seed=3)
    assert (o["flags"] & 3).any() and (o["flags"][14:] == 4).all() and o["flags"][13] & 2
    assert_parity(run(prob, pop, seed=3), o, what="c1 dual")


def test_mesh_partly_outside_image():
    p = synth_problem(1)
    S = p.ref_points + np.array([5.25, -3.5, 2.0], np.float32)
    rs = np.random.default_rng(5)
    T = p.target_base + rs.normal(0, 0.5, p.target_base.shape).astype(np.float32) + 7.0
    pts = cand(S, T)
    prob = morea.Problem.from_synth(p, max_population=1)
    assert_parity(run(prob, pts, seed=4), oracle_problem(1).evaluate_sobol(pts, seed=4), what="outside")


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_reduced_precision_storage(storage):
    """Parity against the oracle on the same quantized images."""
    p = synth_problem(1)
    pop = synth.make_population(p)
    prob = morea.Problem.from_synth(p, storage=storage, max_population=16)
    op = oracle.Problem.from_synth(p, image_src=oracle.quantize(p.image_src, storage),
                                   image_tgt=oracle.quantize(p.image_tgt, storage))
    assert_parity(run(prob, pop, seed=2), op.evaluate_sobol(pop, seed=2), what=storage)


def test_no_guidance_sets_and_large_tets():
    """A problem without guidance sets, and tets wider than 64 voxels."""
    dims = (100, 90, 80)
    pts, tets, fixed = synth.kuhn_grid(dims, (2, 2, 2))
    rs = np.random.default_rng(3)
    img_s = (rs.uniform(0, 1, dims[::-1]) * (rs.uniform(0, 1, dims[::-1]) > 0.3)).astype(np.float32)
    img_t = (rs.uniform(0, 1, dims[::-1]) * (rs.uniform(0, 1, dims[::-1]) > 0.3)).astype(np.float32)
    el = np.ones(len(tets), np.float32)
    prob = morea.Problem(dims, img_s, img_t, tets, pts, el, [], [], radius=6.0, max_population=3)
    op = oracle.Problem(dims, img_s, img_t, tets, pts, el, [], [], 6.0)
    cands = []
    for k in range(3):
        T = pts + np.where(fixed, 0, rs.normal(0, 3.0, pts.shape))
        S = pts + np.where(fixed, 0, rs.normal(0, 1.0, pts.shape)) if k % 2 else pts
        cands.append(cand(S, T)[0])
    cands = np.stack(cands).astype(np.float32)
    g = run(prob, cands, rate=0.05, seed=8)
    o = op.evaluate_sobol(cands, rate=0.05, seed=8)
    assert np.all(o["obj"][:, 2] == 0)
    assert_parity(g, o, what="no sets")


def test_determinism_errors_and_empty():
    p = synth_problem(1)
    pop = synth.make_population(p)
    prob = morea.Problem.from_synth(p, max_population=16)
    a = run(prob, pop, seed=9)
    b = run(prob, pop, seed=9)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])
    one = run(prob, pop[5:6], seed=9)
    for k in a:
        np.testing.assert_array_equal(one[k][0], a[k][5])
    c = run(prob, pop, seed=10)
    assert not np.array_equal(c["obj"][:, 0], a["obj"][:, 0])
    np.testing.assert_array_equal(c["counts"], a["counts"])
    # the magnitude, flags and severity are the full evaluation's
    full = to_host(prob.eval_full(torch.from_numpy(pop).cuda()))
    np.testing.assert_array_equal(a["flags"], full["flags"])
    np.testing.assert_allclose(a["obj"][:, 1], full["obj"][:, 1], rtol=1e-6)
    empty = torch.empty((0, 2, 3, p.n_points), dtype=torch.float32, device="cuda")
    prob.eval_sobol(empty)
    t = torch.from_numpy(pop).cuda()
    for bad in (0.0, -1.0, float("inf"), float("nan")):
        with pytest.raises(morea.MoreaError):
            prob.eval_sobol(t, rate=bad)
    with pytest.raises(morea.MoreaError):
        prob.eval_sobol(torch.from_numpy(np.concatenate([pop, pop[:1]])).cuda())


def test_c2_population_sampled():
    """Config 2 at full size in the benchmark's launch configuration (pop 512):
    sampled candidates against the oracle; every candidate's counts against
    the rounded tet volumes."""
    p = synth_problem(2)
    pop = synth.make_population(p)
    prob = morea.Problem.from_synth(p, max_population=512)
    g = run(prob, pop, seed=1)
    idx = [0, 1, 300, 511]          # 0 has an injected fold
    o = oracle_problem(2).evaluate_sobol(pop[idx], seed=1)
    assert o["flags"][0] != 0
    assert_parity(g, o, idx=idx, what="c2")
    V = float(np.prod(p.dims))
    free = g["flags"] == 0
    assert free.sum() >= 400
    assert np.all(np.abs(g["counts"][free].astype(np.float64) - V) <= p.n_tets / 2)
