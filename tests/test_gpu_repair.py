"""GPU parity of fold repair (Sec. 4.3.1, HIP path via the C-ABI) against the
reference in oracle/repair.py on the same candidates and draws: repaired
coordinates, moves and outcomes bit-exact (every decision is integer
arithmetic on the fixed-point grid)."""
import numpy as np
import pytest

import oracle
import synth
from conftest import oracle_problem, synth_problem
from oracle import repair as R

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2303_04873_amd as morea  # noqa: E402


def pinned_of(p):
    return (p.fixed_axes.astype(np.uint8) * np.array([1, 2, 4], np.uint8)).sum(axis=1).astype(np.uint8)


def run(prob, pts, draws, pinned):
    t = torch.from_numpy(np.ascontiguousarray(pts)).cuda()
    d = torch.from_numpy(np.ascontiguousarray(draws)).cuda()
    pn = None if pinned is None else torch.from_numpy(pinned).cuda()
    info = prob.repair_folds(t, d, pn)
    torch.cuda.synchronize()
    return t.cpu().numpy(), info.cpu().numpy()


def check(p, prob, pts, draws, pinned):
    g, info = run(prob, pts, draws, pinned)
    o, moves, outcome, _ = R.repair(p.tets, p.ref_points, pts, draws, fixed=pinned)
    np.testing.assert_array_equal(info[:, 0], moves)
    np.testing.assert_array_equal(info[:, 1], outcome)
    np.testing.assert_array_equal(g.view(np.uint32), o.view(np.uint32))
    return g, info


def test_c1_folded_population():
    p = synth_problem(1)
    pop = synth.make_population(p, pop=16, seed=21, perturb_source=True, fold_fraction=0.5)
    draws = np.random.default_rng(3).normal(size=(16, 12, 64, 3)).astype(np.float32)
    prob = morea.Problem.from_synth(p, max_population=16)
    g, info = check(p, prob, pop, draws, pinned_of(p))
    assert info[:, 0].sum() >= 8
    # the repaired candidates evaluate fold-free (oracle) where all moves succeeded
    after = oracle_problem(1).evaluate(g)
    assert (after["flags"][::2] == 0).sum() >= 6


def test_edge_cases():
    p = synth_problem(1)
    pop = synth.make_population(p, pop=16, seed=22, perturb_source=True, fold_fraction=0.5)
    pop[3, 1, 2, 5] = 600.0                                  # invalid: untouched
    prob = morea.Problem.from_synth(p, max_population=16)
    rs = np.random.default_rng(4)
    # one draw block only; no pinned axes
    check(p, prob, pop, rs.normal(size=(16, 1, 64, 3)).astype(np.float32), None)
    # zero draws: every trial ties with the current position, nothing moves
    g, info = check(p, prob, pop, np.zeros((16, 4, 64, 3), np.float32), pinned_of(p))
    assert np.all(info[:, 0] == 0) and info[3, 1] == R.INVALID
    np.testing.assert_array_equal(g, pop)
    # large draws: every trial leaves the range or worsens -> aborted
    check(p, prob, pop, (rs.normal(size=(16, 3, 64, 3)) * 1e6).astype(np.float32), pinned_of(p))
    # empty population, bad arguments
    empty = torch.empty((0, 2, 3, p.n_points), dtype=torch.float32, device="cuda")
    prob.repair_folds(empty, torch.empty((0, 1, 64, 3), dtype=torch.float32, device="cuda"))
    t = torch.from_numpy(pop).cuda()
    with pytest.raises(morea.MoreaError):
        morea._check(morea.load_library().morea_repair_folds(prob.handle, morea._dev_ptr(t), 16,
                                                              morea._dev_ptr(t), 0, None,
                                                              morea._dev_ptr(t), None))


def test_too_many_points_refused():
    dims = (24, 24, 20)
    pts, tets, fixed = synth.kuhn_grid(dims, (20, 20, 16))          # 6,400 points
    img = np.ones(dims[::-1], np.float32)
    prob = morea.Problem(dims, img, img, tets, pts, np.ones(len(tets), np.float32), [], [], radius=1.0,
                         max_population=1)
    cand = torch.from_numpy(np.ascontiguousarray(np.stack([pts.T, pts.T])[None], dtype=np.float32)).cuda()
    with pytest.raises(morea.MoreaError):
        prob.repair_folds(cand, torch.zeros((1, 1, 64, 3), dtype=torch.float32, device="cuda"))


def test_c2_population():
    """Config 2, population 512 in one launch; the folded candidates (and a few
    others) against the reference; fold-free after repair checked by the GPU
    evaluation."""
    p = synth_problem(2)
    pop = synth.make_population(p)
    draws = np.random.default_rng(5).normal(size=(512, 16, 64, 3)).astype(np.float32)
    prob = morea.Problem.from_synth(p, max_population=512)
    g, info = run(prob, pop, draws, pinned_of(p))
    idx = [c for c in range(512) if c % 16 == 0] + [1, 255, 511]
    o, moves, outcome, _ = R.repair(p.tets, p.ref_points, pop[idx], draws[idx], fixed=pinned_of(p))
    np.testing.assert_array_equal(info[idx, 0], moves)
    np.testing.assert_array_equal(info[idx, 1], outcome)
    np.testing.assert_array_equal(g[idx].view(np.uint32), o.view(np.uint32))
    others = np.setdiff1d(np.arange(512), idx)
    np.testing.assert_array_equal(g[others], pop[others])           # fold-free: untouched
    assert np.all(info[others, 1] == R.NO_FOLD)
    out = prob.eval_full(torch.from_numpy(g).cuda())
    flags = out["flags"].cpu().numpy()
    folded = [c for c in range(512) if c % 16 == 0]
    assert (flags[folded] == 0).sum() >= 24
