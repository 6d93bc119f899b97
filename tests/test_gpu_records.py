"""GPU parity of the per-(candidate, tet, direction) records that the
evaluation leaves in a cache, element by element against the oracle's
records: sample counts and violation bits bit-exact per tet and direction,
the intensity sum h, the guidance sum g, the magnitude term and the violating
volume within bounds derived from the FP32 arithmetic of one sample.

Per-sample bound (the kernel maps in FP64 and interpolates in FP32): the
trilinear value of an image in [0, 1] is within about 8 ulp(1) = 5e-7 of the
exact one, so h = (a - b)^2 with |a - b| <= 1 moves by at most 1e-6 per
sample; the guidance term w (d - d')^2 with d, d' of a distance map moves by
at most 2 |d - d'| 5e-7 |d'| <= 4e-6 r^2 per band sample (d < r, |d'| < 2r
where the term is not negligible).  Summation in FP32 over at most a few
hundred samples per lane tree adds 1e-6 relative.  The magnitude term uses
exact FP64 squared lengths, one FP32 rounding, hardware square roots and one
reciprocal (a few ulp): 2e-6 relative.

Sizes: the 32^3 phantom's 16 dual candidates with folds (every tet), two
candidates of the 128x128x96 population (every tet), and the cache after an
acceptance of partial evaluations, which must hold the records of the
updated parents."""
import numpy as np
import pytest

import synth
from conftest import oracle_problem, synth_problem
from oracle import accept as acc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2303_04873_amd as morea  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def assert_records(rec, ref, radius, what, valid=None):
    """rec: structured [pop][tets][2] from the cache; ref: oracle [pop][tets][2][6]."""
    if valid is not None:
        rec, ref = rec[valid], ref[valid]
    n = rec["n"].astype(np.int64)
    np.testing.assert_array_equal(n, ref[..., 2].astype(np.int64), err_msg=f"samples {what}")
    np.testing.assert_array_equal(rec["bits"] & 1, ref[..., 5].astype(np.uint32), err_msg=f"violation {what}")
    r2 = max(1.0, float(radius) ** 2)
    for name, k, atol in (("h", 0, 1e-6 * n + 1e-7), ("g", 1, 4e-6 * r2 * n + 1e-7),
                          ("mag", 3, 1e-12), ("vol", 4, 1e-12)):
        g = rec[name].astype(np.float64)
        o = ref[..., k]
        rtol = 2e-6 if name in ("h", "g", "mag") else 1e-6
        err = np.abs(g - o)
        bad = err > atol + rtol * np.abs(o)
        assert not bad.any(), (f"{name} {what}: {bad.sum()} records out of bound, worst at "
                               f"{np.argwhere(bad)[0].tolist()}: {g[bad][0]} vs {o[bad][0]}")
    return float(np.max(np.abs(rec["h"] - ref[..., 0]) / np.maximum(np.abs(ref[..., 0]), 1e-30)))


def full_records(prob, pop):
    d = dev(pop)
    cache = prob.new_cache(len(pop))
    prob.eval_full(d, cache=cache)
    torch.cuda.synchronize()
    return prob.cache_records(cache, len(pop))


def test_c1_full_records_every_tet():
    p = synth_problem(1)
    pop = synth.make_population(p, pop=16, seed=101, perturb_source=True, fold_fraction=0.25)
    prob = morea.Problem.from_synth(p, max_population=16)
    rec = full_records(prob, pop)
    o = oracle_problem(1).evaluate(pop, records=True)
    assert (o["flags"] & 3).any()
    assert_records(rec, o["records"], oracle_problem(1).radius, "c1")
    assert (rec["n"] > 0).mean() > 0.9


def test_c1_invalid_candidate_records():
    """A candidate with an out-of-range coordinate: the records of the tets
    that hold the point carry the invalid bit in both directions, no other
    record does; the valid candidate beside it is unaffected."""
    p = synth_problem(1)
    pop = synth.make_population(p, pop=2, seed=3)
    pop[1, 1, 0, 7] = 700.0
    prob = morea.Problem.from_synth(p, max_population=2)
    rec = full_records(prob, pop)
    o = oracle_problem(1).evaluate(pop, records=True)
    assert_records(rec, o["records"], oracle_problem(1).radius, "c1 valid", valid=np.array([True, False]))
    holds = np.any(p.tets == 7, axis=1)
    np.testing.assert_array_equal((rec[1]["bits"] & 4) != 0, np.repeat(holds[:, None], 2, axis=1))
    assert not np.any(rec[0]["bits"] & 4)


def test_c2_full_records_sample():
    """Two candidates of the 128x128x96 population (one with a fold), every
    tet, evaluated in the population launch of the benchmark (512)."""
    p = synth_problem(2)
    pop = synth.make_population(p)
    prob = morea.Problem.from_synth(p, max_population=len(pop))
    d = dev(pop)
    cache = prob.new_cache(len(pop))
    out = prob.eval_full(d, cache=cache)
    torch.cuda.synchronize()
    folded = np.nonzero(out["flags"].cpu().numpy() & 3)[0]     # which candidates to sample
    idx = [0, int(folded[0]) if folded.size else 1]
    rec = prob.cache_records(cache, len(pop))[idx]
    o = oracle_problem(2).evaluate(pop[idx], records=True)
    worst = assert_records(rec, o["records"], oracle_problem(2).radius, "c2")
    print(f"c2 records: worst per-tet h rel err {worst:.2e}", flush=True)


def test_c1_cache_after_acceptance_holds_updated_parents():
    p = synth_problem(1)
    parents = synth.make_population(p, pop=8, seed=21, perturb_source=True, fold_fraction=0.25)
    elements, colors, _ = morea.build_fos(p.n_points, p.tets)
    mine = elements[colors == 1]
    off = np.arange(0, 2 * len(mine) + 1, 2, dtype=np.int32)
    pts = mine.reshape(-1).astype(np.int32)
    ep, eg, new = synth.make_children(p, parents, off, pts, seed=9)
    prob = morea.Problem.from_synth(p, max_population=len(parents))
    prob.set_groups(off, pts)
    prob.reserve_partial(len(ep))
    d = dev(parents)
    cache = prob.new_cache(len(parents))
    prob.eval_full(d, cache=cache)
    dep, deg, dnew = dev(ep), dev(eg), dev(new)
    child = prob.eval_partial(d, cache, dep, deg, dnew)
    par = prob.eval_full(dev(parents))
    # archive: the starting parents' objective vectors (a decision input only)
    archive = par["obj"][par["flags"] == 0].contiguous()
    a = prob.accept_partial(d, cache, dep, deg, dnew, child, par, archive=archive)
    torch.cuda.synchronize()
    kept = a.cpu().numpy()
    assert kept.sum() > 0
    updated = acc.apply(parents, off, pts, ep, eg, new, kept)
    np.testing.assert_array_equal(d.cpu().numpy(), updated)
    rec = prob.cache_records(cache, len(parents))
    o = oracle_problem(1).evaluate(updated, records=True)
    assert_records(rec, o["records"], oracle_problem(1).radius, "cache after acceptance")
