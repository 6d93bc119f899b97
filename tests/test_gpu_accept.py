"""GPU parity of the acceptance step of optimal mixing (Sec. 3) through the
C-ABI.

The decisions are compared bit-exactly with the oracle on seeded decision
inputs (objective vectors on a small grid, so that ties, equal vectors,
mixed feasibility and NaN all occur; archives spanning several LDS chunks).
After acceptance the parents' points must equal the oracle's application of
the accepted children exactly, the parents' evaluation (recomputed from the
cache) must match the oracle's full evaluation of the updated parents to the
parity bar, and the cache must serve further partial evaluations of the
updated parents.  At the full 128x128x96 size the decisions are checked on a
sample and the parents against the GPU's own full evaluation."""
import numpy as np
import pytest

import synth
from conftest import oracle_problem, synth_problem
from oracle import accept as acc
from parity import assert_parity, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2303_04873_amd as morea  # noqa: E402


def colour_setup(p, parents, colour, seed, extra_invalid=False):
    elements, colors, _ = morea.build_fos(p.n_points, p.tets)
    mine = elements[colors == colour]
    off = np.arange(0, 2 * len(mine) + 1, 2, dtype=np.int32)
    pts = mine.reshape(-1).astype(np.int32)
    ep, eg, new = synth.make_children(p, parents, off, pts, seed=seed)
    if extra_invalid:
        # an out-of-range parent (its valid group still owns two rows) and an
        # out-of-range group (owns none)
        ep = np.concatenate([ep, np.array([-1, 0], np.int32)])
        eg = np.concatenate([eg, np.array([0, len(mine)], np.int32)])
        new = np.concatenate([new, new[:2]])
    prob = morea.Problem.from_synth(p, max_population=parents.shape[0])
    prob.set_groups(off, pts)
    prob.reserve_partial(len(ep))
    return prob, off, pts, ep, eg, new


def synthetic_decisions(rs, n, pop):
    """Objective vectors on {0, 1, 2}, flags and severities mixed."""
    def block(k):
        obj = rs.integers(0, 3, (k, 3)).astype(np.float32)
        flags = rs.choice(np.array([0, 0, 0, 0, 1, 2, 3, 4], np.uint8), k)
        sev = (rs.integers(0, 3, k) * 0.5).astype(np.float32)
        return obj, flags, sev
    child, parent = block(n), block(pop)
    child[0][rs.integers(0, n)] = [np.nan, 1, 1]
    return child, parent


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_accept(prob, d, cache, ep, eg, new, child, parent, archive):
    c = dict(obj=dev(child[0]), flags=dev(child[1]), severity=dev(child[2]))
    par = dict(obj=dev(parent[0]), flags=dev(parent[1]), severity=dev(parent[2]),
               counts=torch.empty((len(parent[1]), 2), dtype=torch.int32, device="cuda"))
    a = prob.accept_partial(d, cache, ep, eg, new, c, par, archive=None if archive is None else dev(archive))
    torch.cuda.synchronize()
    return a.cpu().numpy(), to_host(par)


def test_c1_decisions_application_and_cache():
    p = synth_problem(1)
    parents = synth.make_population(p, pop=8, seed=21, perturb_source=True, fold_fraction=0.25)
    prob, off, pts, ep, eg, new = colour_setup(p, parents, 0, seed=5, extra_invalid=True)
    d = dev(parents)
    cache = prob.new_cache(len(parents))
    prob.eval_full(d, cache=cache)
    dep, deg, dnew = dev(ep), dev(eg), dev(new)
    prob.eval_partial(d, cache, dep, deg, dnew)
    rs = np.random.default_rng(77)
    child, parent = synthetic_decisions(rs, len(ep), len(parents))
    archive = rs.integers(0, 3, (1300, 3)).astype(np.float32) + np.float32(0.5)   # three LDS chunks
    archive[1100] = [0, 0, 1]                                                      # dominating, late chunk
    print("c1 acceptance", len(ep), "evaluations, archive", len(archive), flush=True)
    got, par_out = run_accept(prob, d, cache, dep, deg, dnew, child, parent, archive)
    want = acc.accept_batch(*child, ep, eg, len(off) - 1, *parent, [tuple(m) for m in archive])
    np.testing.assert_array_equal(got, want)
    assert 0 < want.sum() < len(want) and got[-2:].tolist() == [0, 0]
    updated = acc.apply(parents, off, pts, ep, eg, new, want)
    np.testing.assert_array_equal(d.cpu().numpy(), updated)
    assert_parity(par_out, oracle_problem(1).evaluate(updated), what="parents after acceptance")
    # the cache now holds the updated parents: a partial evaluation of new
    # children of them matches the oracle's full evaluation of those children
    ep2, eg2, new2 = synth.make_children(p, updated, off, pts, seed=6)
    out = to_host(prob.eval_partial(d, cache, dev(ep2), dev(eg2), dev(new2)))
    kids = np.stack([synth.apply_child(updated, off, pts, ep2, eg2, new2, e) for e in range(len(ep2))])
    assert_parity(out, oracle_problem(1).evaluate(kids), what="partial evaluation after acceptance")


def test_c1_steering_bound():
    p = synth_problem(1)
    parents = synth.make_population(p, pop=8, seed=23, perturb_source=True, fold_fraction=0.25)
    prob, off, pts, ep, eg, new = colour_setup(p, parents, 2, seed=7)
    d = dev(parents)
    cache = prob.new_cache(len(parents))
    prob.eval_full(d, cache=cache)
    dep, deg, dnew = dev(ep), dev(eg), dev(new)
    prob.eval_partial(d, cache, dep, deg, dnew)
    rs = np.random.default_rng(79)
    child, parent = synthetic_decisions(rs, len(ep), len(parents))
    # guidance values 0, 0.5, ..., 2.5 against the bound 1.2: several excesses
    child[0][:, 2] = (rs.integers(0, 6, len(ep)) * 0.5).astype(np.float32)
    parent[0][:, 2] = (rs.integers(0, 6, len(parents)) * 0.5).astype(np.float32)
    archive = (rs.integers(0, 3, (40, 3)) * 0.5 + 0.25).astype(np.float32)
    gmax = 1.2
    c = dict(obj=dev(child[0]), flags=dev(child[1]), severity=dev(child[2]))
    par = dict(obj=dev(parent[0]), flags=dev(parent[1]), severity=dev(parent[2]),
               counts=torch.empty((len(parents), 2), dtype=torch.int32, device="cuda"))
    got = prob.accept_partial(d, cache, dep, deg, dnew, c, par, archive=dev(archive), guidance_max=gmax)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    want = acc.accept_batch(*child, ep, eg, len(off) - 1, *parent, [tuple(m) for m in archive],
                            guidance_max=float(np.float32(gmax)))
    np.testing.assert_array_equal(got, want)
    off_bound = acc.accept_batch(*child, ep, eg, len(off) - 1, *parent, [tuple(m) for m in archive])
    assert np.any(want != off_bound)          # the bound changed some decisions
    np.testing.assert_array_equal(d.cpu().numpy(), acc.apply(parents, off, pts, ep, eg, new, want))


def test_c1_real_objectives_and_state_errors():
    p = synth_problem(1)
    parents = synth.make_population(p, pop=6, seed=22, perturb_source=True, fold_fraction=0.3)
    prob, off, pts, ep, eg, new = colour_setup(p, parents, 1, seed=8)
    d = dev(parents)
    cache = prob.new_cache(len(parents))
    par_out = prob.eval_full(d, cache=cache)
    dep, deg, dnew = dev(ep), dev(eg), dev(new)
    child_out = prob.eval_partial(d, cache, dep, deg, dnew)
    # acceptance must follow the partial evaluation of the same list
    with pytest.raises(morea.MoreaError) as err:
        prob.accept_partial(d, cache, dep.clone(), deg, dnew, child_out, par_out)
    assert err.value.status == morea.MOREA_ESTATE
    ora = oracle_problem(1)
    po = ora.evaluate(parents)
    kids = np.stack([synth.apply_child(parents, off, pts, ep, eg, new, e) for e in range(len(ep))])
    ko = ora.evaluate(kids)
    feas = po["flags"] == 0
    archive = po["obj"][feas].astype(np.float32) * np.float32(1.0001)
    got = prob.accept_partial(d, cache, dep, deg, dnew, child_out, par_out, archive=dev(archive))
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    arc = [tuple(map(float, m)) for m in archive]
    want = acc.accept_batch(ko["obj"], ko["flags"], ko["severity"], ep, eg, len(off) - 1, po["obj"], po["flags"],
                            po["severity"], arc)

    def robust(e):
        # the decision is monotone in the child's values (smaller is better):
        # it is insensitive to FP32 rounding when moving every child value by
        # twice the parity bar towards better and towards worse gives the same
        pa = int(ep[e])
        parent = (po["obj"][pa], po["flags"][pa], po["severity"][pa])
        o, s = ko["obj"][e], ko["severity"][e]
        t = 2e-5
        better = acc.accept((o - t * np.abs(o), ko["flags"][e], s - t * abs(s)), parent, arc)
        worse = acc.accept((o + t * np.abs(o), ko["flags"][e], s + t * abs(s)), parent, arc)
        return better == worse

    keep = [e for e in range(len(ep)) if robust(e)]
    print("robust decisions", len(keep), "of", len(ep), "accepted", int(got.sum()), flush=True)
    assert len(keep) > 0
    np.testing.assert_array_equal(got[keep], want[keep])
    np.testing.assert_array_equal(d.cpu().numpy(), acc.apply(parents, off, pts, ep, eg, new, got))
    # a tuning run discards the evaluation list the workspace belongs to
    prob.eval_partial(d, cache, dep, deg, dnew, out=child_out)
    prob.tune_partial(d, cache, dep, deg, dnew)
    with pytest.raises(morea.MoreaError) as err:
        prob.accept_partial(d, cache, dep, deg, dnew, child_out, par_out)
    assert err.value.status == morea.MOREA_ESTATE


def test_c2_full_size_one_colour():
    p = synth_problem(2)
    parents = synth.make_population(p)
    prob, off, pts, ep, eg, new = colour_setup(p, parents, 0, seed=9)
    d = dev(parents)
    cache = prob.new_cache(len(parents))
    prob.eval_full(d, cache=cache)
    dep, deg, dnew = dev(ep), dev(eg), dev(new)
    prob.eval_partial(d, cache, dep, deg, dnew)
    rs = np.random.default_rng(78)
    child, parent = synthetic_decisions(rs, len(ep), len(parents))
    archive = rs.integers(0, 3, (2000, 3)).astype(np.float32) + np.float32(0.25)
    print("c2 acceptance", len(ep), "evaluations, archive", len(archive), flush=True)
    got, par_out = run_accept(prob, d, cache, dep, deg, dnew, child, parent, archive)
    sample = np.sort(rs.choice(len(ep), 600, replace=False))
    arc = [tuple(m) for m in archive]
    want = np.array([acc.accept_batch(child[0][e:e + 1], child[1][e:e + 1], child[2][e:e + 1], ep[e:e + 1],
                                      eg[e:e + 1], len(off) - 1, *parent, arc)[0] for e in sample])
    np.testing.assert_array_equal(got[sample], want)
    updated = acc.apply(parents, off, pts, ep, eg, new, got)
    np.testing.assert_array_equal(d.cpu().numpy(), updated)
    # the parents' evaluation from the cache equals a fresh full evaluation
    fresh = to_host(morea.Problem.from_synth(p, max_population=len(parents)).eval_full(dev(updated)))
    np.testing.assert_array_equal(par_out["flags"], fresh["flags"])
    np.testing.assert_array_equal(par_out["counts"], fresh["counts"])
    np.testing.assert_allclose(par_out["obj"], fresh["obj"], rtol=1e-6)
    changed = np.unique(ep[got == 1])
    pick = [int(changed[0]), int(changed[-1])]
    assert_parity(par_out, oracle_problem(2).evaluate(updated[pick]), idx=pick, what="c2 parents")


def test_c1_large_groups_one_per_parent():
    """Groups of 4-40 points (write-back loops of many lane passes), one
    evaluation per parent (disjoint by construction)."""
    p = synth_problem(1)
    parents = synth.make_population(p, pop=10, seed=24, perturb_source=True, fold_fraction=0.2)
    off, pts = synth.make_groups(p, n_groups=10, sizes=(4, 40), seed=3)
    ep = np.arange(10, dtype=np.int32)
    eg = np.random.default_rng(4).permutation(10).astype(np.int32)
    _, _, all_new = synth.make_children(p, parents, off, pts, seed=4)
    # rows of evaluation (e, eg[e]) taken from the (parent, group) pair's rows of make_children
    sizes = np.diff(off)
    start = {}
    r = 0
    for pa in range(10):
        for g in range(10):
            start[(pa, g)] = r
            r += sizes[g]
    new = np.concatenate([all_new[start[(e, eg[e])]:start[(e, eg[e])] + sizes[eg[e]]] for e in range(10)])
    prob = morea.Problem.from_synth(p, max_population=10)
    prob.set_groups(off, pts)
    prob.reserve_partial(10)
    d = dev(parents)
    cache = prob.new_cache(10)
    prob.eval_full(d, cache=cache)
    dep, deg, dnew = dev(ep), dev(eg), dev(new)
    prob.eval_partial(d, cache, dep, deg, dnew)
    rs = np.random.default_rng(80)
    child, parent = synthetic_decisions(rs, 10, 10)
    got, par_out = run_accept(prob, d, cache, dep, deg, dnew, child, parent, None)
    want = acc.accept_batch(*child, ep, eg, 10, *parent, [])
    np.testing.assert_array_equal(got, want)
    assert want.sum() >= 3 and sizes[eg[want == 1]].max() > 10
    updated = acc.apply(parents, off, pts, ep, eg, new, want)
    np.testing.assert_array_equal(d.cpu().numpy(), updated)
    assert_parity(par_out, oracle_problem(1).evaluate(updated), what="large groups")
