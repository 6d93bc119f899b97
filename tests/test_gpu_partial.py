"""GPU parity of partial evaluation (persistent, graph-replayed launch).

A partial evaluation of (parent, group) must equal a full evaluation of the
child (parent with the group's points moved): counts, flags and invalidity
exactly, objectives within 1e-5.  Checked against the oracle's full
evaluation of the child, and against the GPU's own full evaluation for many
children at the full 128x128x96 / 3,402-tet / 512 x 64 size."""
import numpy as np
import pytest

import synth
from conftest import oracle_problem, synth_problem
from parity import assert_parity, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2303_04873_amd as morea  # noqa: E402


def setup(p, parents, n_groups, sizes, seed=0):
    off, pts = synth.make_groups(p, n_groups=n_groups, sizes=sizes, seed=seed)
    ep, eg, new = synth.make_children(p, parents, off, pts, seed=seed)
    prob = morea.Problem.from_synth(p, max_population=parents.shape[0])
    prob.set_groups(off, pts)
    prob.reserve_partial(len(ep))
    dev = dict(parents=torch.from_numpy(parents).cuda(), ep=torch.from_numpy(ep).cuda(),
               eg=torch.from_numpy(eg).cuda(), new=torch.from_numpy(new).cuda())
    cache = prob.new_cache(parents.shape[0])
    prob.eval_full(dev["parents"], cache=cache)
    return prob, off, pts, ep, eg, new, dev, cache


def children(parents, off, pts, ep, eg, new, idx):
    return np.stack([synth.apply_child(parents, off, pts, ep, eg, new, e) for e in idx])


def test_partial_c1_against_oracle():
    p = synth_problem(1)
    parents = synth.make_population(p, pop=8, seed=11, perturb_source=True, fold_fraction=0.25)
    prob, off, pts, ep, eg, new, dev, cache = setup(p, parents, 12, (4, 20))
    out = prob.eval_partial(dev["parents"], cache, dev["ep"], dev["eg"], dev["new"])
    torch.cuda.synchronize()
    g = to_host(out)
    idx = np.arange(len(ep))
    kids = children(parents, off, pts, ep, eg, new, idx)
    assert_parity(g, oracle_problem(1).evaluate(kids), what="partial c1")
    # the GPU's own full evaluation of the children agrees exactly on integers
    full = to_host(morea.Problem.from_synth(p, max_population=len(kids)).eval_full(
        torch.from_numpy(kids).cuda()))
    np.testing.assert_array_equal(full["counts"], g["counts"])
    np.testing.assert_array_equal(full["flags"], g["flags"])


def test_partial_graph_replay_and_tuner():
    p = synth_problem(1)
    parents = synth.make_population(p, pop=6, seed=12)
    prob, off, pts, ep, eg, new, dev, cache = setup(p, parents, 10, (4, 16), seed=3)
    out = prob.outputs(len(ep))
    ref = None
    for rep in range(4):
        prob.eval_partial(dev["parents"], cache, dev["ep"], dev["eg"], dev["new"], out=out)
        torch.cuda.synchronize()
        g = to_host(out)
        if ref is None:
            ref = g
        for k in g:
            np.testing.assert_array_equal(g[k], ref[k])
        # unrelated eager work between replays
        junk = torch.randn(1 << 20, device="cuda")
        (junk * 2).sum().item()
        out["obj"].zero_()
    ms, shape = prob.tune_partial(dev["parents"], cache, dev["ep"], dev["eg"], dev["new"])
    assert ms > 0 and ((shape[0] > 0 and shape[1] in (1, 2, 4, 8, 16)) or shape == (0, 0))
    prob.eval_partial(dev["parents"], cache, dev["ep"], dev["eg"], dev["new"], out=out)
    torch.cuda.synchronize()
    g = to_host(out)
    for k in g:
        np.testing.assert_array_equal(g[k], ref[k])
    # both launch forms, several shapes: the same outputs bit for bit
    for shape in [(0, 0), (3, 1), (7, 16), (256, 8)]:
        prob.set_partial_shape(*shape)
        assert prob.partial_shape() == shape
        out["obj"].zero_()
        prob.eval_partial(dev["parents"], cache, dev["ep"], dev["eg"], dev["new"], out=out)
        torch.cuda.synchronize()
        g = to_host(out)
        for k in g:
            np.testing.assert_array_equal(g[k], ref[k], err_msg=f"shape {shape} {k}")
    for bad in [(0, 4), (4, 0), (-1, 1), (4, 65)]:
        with pytest.raises(morea.MoreaError):
            prob.set_partial_shape(*bad)


def test_partial_graph_cache_alternating_sets():
    """Four argument sets alternated (one per colour of a generation) are
    captured once each and then replayed; each replay equals the first
    result of its set; a ninth set evicts the least recently used graph."""
    p = synth_problem(1)
    parents = synth.make_population(p, pop=6, seed=14)
    prob, off, pts, ep, eg, new, dev, cache = setup(p, parents, 10, (4, 16), seed=4)
    h = prob.handle
    n0, c0 = morea.morea_partial_graphs(h)
    assert n0 == 0 and c0 == 0
    sets = []
    for k in range(4):
        sel = torch.arange(k, len(ep), 4, device="cuda")
        rows = []
        eg_h = eg
        starts = np.concatenate([[0], np.cumsum(np.diff(off)[eg_h])])
        for e in sel.cpu().numpy():
            rows.append(np.arange(starts[e], starts[e + 1]))
        new_k = torch.from_numpy(new[np.concatenate(rows)]).cuda()
        sets.append((dev["ep"][sel].contiguous(), dev["eg"][sel].contiguous(), new_k, prob.outputs(len(sel))))
    first = []
    for rnd in range(3):
        for k, (a, b, c, o) in enumerate(sets):
            prob.eval_partial(dev["parents"], cache, a, b, c, out=o)
            torch.cuda.synchronize()
            g = to_host(o)
            if rnd == 0:
                first.append(g)
            else:
                for key in g:
                    np.testing.assert_array_equal(g[key], first[k][key])
            o["obj"].zero_()
    assert morea.morea_partial_graphs(h) == (4, 4)
    # more argument sets than slots: the oldest ones are replaced
    extra = [prob.outputs(len(sets[0][0])) for _ in range(5)]
    for o in extra:
        prob.eval_partial(dev["parents"], cache, sets[0][0], sets[0][1], sets[0][2], out=o)
    torch.cuda.synchronize()
    assert morea.morea_partial_graphs(h) == (8, 9)
    for o in extra:
        for key in ("obj", "flags", "counts"):
            np.testing.assert_array_equal(to_host(o)[key], first[0][key])


def test_partial_invalid_inputs():
    p = synth_problem(1)
    parents = synth.make_population(p, pop=4, seed=13)
    off, pts = synth.make_groups(p, n_groups=4, sizes=(4, 8), seed=5)
    ep, eg, new = synth.make_children(p, parents, off, pts, seed=5)
    # a parent with one invalid coordinate at a point of group eg[1]
    bad_pt = pts[off[eg[1]]]
    parents_bad = parents.copy()
    parents_bad[ep[1], 1, 0, bad_pt] = 900.0
    new = new.copy()
    new[2 * 0 + 0] = np.nan                          # first row of eval 0 invalid
    ep = ep.copy()
    ep[3] = 99                                       # out-of-range parent
    prob = morea.Problem.from_synth(p, max_population=4)
    prob.set_groups(off, pts)
    prob.reserve_partial(len(ep))
    dpar = torch.from_numpy(parents_bad).cuda()
    cache = prob.new_cache(4)
    prob.eval_full(dpar, cache=cache)
    g = to_host(prob.eval_partial(dpar, cache, torch.from_numpy(ep).cuda(), torch.from_numpy(eg).cuda(),
                                  torch.from_numpy(new).cuda()))
    assert g["flags"][0] == 4 and np.isnan(g["obj"][0]).all()
    assert g["flags"][3] == 4
    # eval 1 replaces the invalid coordinate with a valid one: the child is valid
    assert g["flags"][1] & 4 == 0
    kid = synth.apply_child(parents_bad, off, pts, ep, eg, new, 1)[None]
    assert_parity({k: v[1:2] for k, v in g.items()}, oracle_problem(1).evaluate(kid), what="fixed")
    with pytest.raises(morea.MoreaError):
        prob.eval_partial(dpar, cache, torch.zeros(len(ep) + 1, dtype=torch.int32, device="cuda"),
                          torch.zeros(len(ep) + 1, dtype=torch.int32, device="cuda"),
                          torch.from_numpy(new).cuda())


def test_partial_c3_full_size():
    """512 parents x 64 groups of 4-48 points (config 3) in one call."""
    p = synth_problem(3)
    parents = synth.make_population(p)
    prob, off, pts, ep, eg, new, dev, cache = setup(p, parents, synth.N_GROUPS, synth.GROUP_SIZES)
    assert len(ep) == 512 * 64
    g = to_host(prob.eval_partial(dev["parents"], cache, dev["ep"], dev["eg"], dev["new"]))
    # GPU full evaluation of a sample of 512 children: integers exact, objectives close
    rs = np.random.default_rng(0)
    idx = np.sort(rs.choice(len(ep), 512, replace=False))
    kids = children(parents, off, pts, ep, eg, new, idx)
    full = to_host(morea.Problem.from_synth(p, max_population=512).eval_full(torch.from_numpy(kids).cuda()))
    np.testing.assert_array_equal(full["counts"], g["counts"][idx])
    np.testing.assert_array_equal(full["flags"], g["flags"][idx])
    rel = np.abs(full["obj"].astype(np.float64) - g["obj"][idx]) / np.abs(full["obj"])
    assert rel.max() < 2e-5
    # oracle on a few children
    few = idx[:4]
    assert_parity(g, oracle_problem(3).evaluate(children(parents, off, pts, ep, eg, new, few)),
                  idx=few, what="c3")
