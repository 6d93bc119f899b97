"""GPU parity of the optimal-mixing distributions (Sec. 3) through the C-ABI.

Every step is FP64 one operation at a time in the order the reference
states, so the estimates (means, Cholesky factors, fallback decisions) and
the FP32 samples must equal the reference bit for bit: clusters that
overlap, one with fewer members than variables (fallback), one of identical
members (zero covariance), an empty one, one holding an out-of-range member;
pinned axes; evaluations with an out-of-range parent, group or cluster.  At
the full 128x128x96 mesh (400 edges, 10 clusters, 512 solutions) the records
and samples are compared on a sample of pairs and evaluations."""
import numpy as np
import pytest

import synth
from conftest import synth_problem
from oracle import mixing as mx

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2303_04873_amd as morea  # noqa: E402

DIST = np.dtype([("mean", "<f8", 24), ("L", "<f8", 576), ("var", "<i4", 24), ("n_free", "<i4"), ("mode", "<i4"),
                 ("pad", "<i4", 2)])


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def pinned_bits(p):
    fa = p.fixed_axes.astype(np.uint8)
    return (fa[:, 0] | (fa[:, 1] << 1) | (fa[:, 2] << 2)).astype(np.uint8)


def setup(p, n_pop):
    elements, colors, _ = morea.build_fos(p.n_points, p.tets)
    off = np.arange(0, 2 * len(elements) + 1, 2, dtype=np.int32)
    pts = elements.reshape(-1).astype(np.int32)
    prob = morea.Problem.from_synth(p, max_population=n_pop)
    prob.set_groups(off, pts)
    return prob, off, pts, colors


def records(work, n_pairs):
    raw = work.cpu().numpy()[:n_pairs * DIST.itemsize]
    assert DIST.itemsize == 4912
    return raw.view(DIST)


def check_record(rec, ref):
    free, mean, L, mode = ref
    assert rec["mode"] == mode and rec["n_free"] == len(free)
    assert list(rec["var"][:len(free)]) == free
    n = len(free)
    if mode != 2:
        np.testing.assert_array_equal(rec["mean"][:n], np.array(mean))
        np.testing.assert_array_equal(rec["L"].reshape(24, 24)[:n, :n], np.array(L).reshape(n, n))


def test_c1_records_and_samples_bit_exact():
    p = synth_problem(1)
    pop = synth.make_population(p, pop=24, seed=41, perturb_source=True, fold_fraction=0.2)
    prob, off, gpts, colors = setup(p, len(pop))
    n_groups = len(off) - 1
    pinned = pinned_bits(p)
    # clusters: overlapping, rank-deficient, identical members, empty, out-of-range member
    clusters = [list(range(0, 14)), list(range(8, 24)), [0, 1, 2, 3, 4], [7, 7, 7], [], [3, 99]]
    clu_off = np.concatenate([[0], np.cumsum([len(c) for c in clusters])]).astype(np.int32)
    clu_members = np.array(sum(clusters, []), np.int32)
    k = len(clusters)
    rs = np.random.default_rng(12)
    ep = np.repeat(np.arange(len(pop), dtype=np.int32), n_groups)
    eg = np.tile(np.arange(n_groups, dtype=np.int32), len(pop))
    ec = rs.integers(0, k, len(ep)).astype(np.int32)
    ep = np.concatenate([ep, np.array([-1, 3, 5, 2], np.int32)])
    eg = np.concatenate([eg, np.array([0, n_groups, 1, 2], np.int32)])
    ec = np.concatenate([ec, np.array([0, 0, k, -1], np.int32)])
    prob.reserve_partial(len(ep))
    rows = 2 * int(np.sum((eg >= 0) & (eg < n_groups)))
    z = rs.normal(size=(rows, 2, 3)).astype(np.float32)
    mult = rs.uniform(0.5, 2.0, (k, n_groups)).astype(np.float32)
    d = dev(pop)
    work = prob.mixing_workspace(k)
    print("c1 mixing", len(ep), "evaluations,", k, "clusters,", n_groups, "groups", flush=True)
    prob.estimate_distributions(d, dev(clu_off), dev(clu_members), work, pinned=dev(pinned))
    new = prob.sample_partial(d, work, k, dev(ep), dev(eg), dev(ec), dev(z), pinned=dev(pinned), mult=dev(mult))
    torch.cuda.synchronize()
    got = new.cpu().numpy()
    want = mx.sample_batch(pop, clu_off, clu_members, off, gpts, pinned, mult, ep, eg, ec, z)
    np.testing.assert_array_equal(got, want)
    rec = records(work, k * n_groups)
    modes = set()
    for c in range(k):
        members = clusters[c] if all(0 <= i < len(pop) for i in clusters[c]) else [-1]
        for g in range(n_groups):
            ref = mx.estimate(pop, members, [int(v) for v in gpts[off[g]:off[g + 1]]], pinned)
            check_record(rec[c * n_groups + g], ref)
            modes.add(ref[3])
    assert modes == {0, 1, 2}
    # a second estimate from another snapshot replaces the records; pinned
    # coordinates are equal in every candidate, so the reference may take the
    # snapshot for the parents too
    pop2 = pop[::-1].copy()
    fx = p.fixed_axes
    for a in range(3):
        for m in range(2):
            col = pop[:, m, a, fx[:, a]]
            assert np.all(col == col[0])
    prob.estimate_distributions(dev(pop2), dev(clu_off), dev(clu_members), work, pinned=dev(pinned))
    new2 = prob.sample_partial(d, work, k, dev(ep), dev(eg), dev(ec), dev(z), pinned=dev(pinned))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(new2.cpu().numpy(),
                                  mx.sample_batch(pop2, clu_off, clu_members, off, gpts, pinned, None, ep, eg, ec, z))
    # a workspace too small is refused
    with pytest.raises(morea.MoreaError) as err:
        prob.estimate_distributions(d, dev(clu_off), dev(clu_members), work[:100], pinned=dev(pinned))
    assert err.value.status == morea.MOREA_ERANGE


def test_c2_full_mesh_sampled():
    p = synth_problem(2)
    pop = synth.make_population(p)
    prob, off, gpts, colors = setup(p, len(pop))
    n_groups = len(off) - 1
    pinned = pinned_bits(p)
    k = 10
    order = np.random.default_rng(5).permutation(len(pop)).astype(np.int32)
    clu_off = np.linspace(0, len(pop), k + 1).astype(np.int32)
    mine = np.flatnonzero(colors == 0).astype(np.int32)
    ep = np.repeat(np.arange(len(pop), dtype=np.int32), len(mine))
    eg = np.tile(mine, len(pop))
    ec = np.searchsorted(clu_off, np.argsort(order), side="right").astype(np.int32) - 1
    ec = ec[ep]
    prob.reserve_partial(len(ep))
    rs = np.random.default_rng(13)
    z = rs.normal(size=(2 * len(ep), 2, 3)).astype(np.float32)
    d = dev(pop)
    work = prob.mixing_workspace(k)
    print("c2 mixing", len(ep), "evaluations", flush=True)
    prob.estimate_distributions(d, dev(clu_off), dev(order), work, pinned=dev(pinned))
    new = prob.sample_partial(d, work, k, dev(ep), dev(eg), dev(ec), dev(z), pinned=dev(pinned))
    torch.cuda.synchronize()
    got = new.cpu().numpy()
    assert np.all(np.isfinite(got))
    rec = records(work, k * n_groups)
    cache = {}
    for e in np.sort(rs.choice(len(ep), 300, replace=False)):
        c, g = int(ec[e]), int(eg[e])
        gp = [int(v) for v in gpts[off[g]:off[g + 1]]]
        if (c, g) not in cache:
            cache[(c, g)] = mx.estimate(pop, [int(i) for i in order[clu_off[c]:clu_off[c + 1]]], gp, pinned)
            check_record(rec[c * n_groups + g], cache[(c, g)])
        par = [mx.values(pop, int(ep[e]), gp, v) for v in range(12)]
        want = mx.sample(cache[(c, g)], z[2 * e:2 * e + 2].reshape(-1), 1.0, par)
        np.testing.assert_array_equal(got[2 * e:2 * e + 2].reshape(-1), np.array(want, np.float32))
    assert all(v[3] == 0 for v in cache.values())


def test_c1_one_generation_end_to_end():
    """Distributions from a snapshot, then per colour: children sampled (bit
    for bit against the reference), evaluated (against the oracle's full
    evaluation of each child), accepted with an empty archive (every feasible
    child is kept, infeasible ones compare their violations with the
    parent's), written back.  The reference follows its own decisions; they
    must equal the library's, the parents' points after each colour must
    equal the reference's, and the parents' evaluations kept in the caches
    must equal a fresh full evaluation and the oracle's."""
    import oracle
    from oracle import accept as acc
    from parity import assert_parity, to_host
    p = synth_problem(1)
    pop = synth.make_population(p, pop=12, seed=44, perturb_source=True, fold_fraction=0.25)
    prob, off, gpts, colors = setup(p, len(pop))
    n_colors = int(colors.max()) + 1
    pinned = pinned_bits(p)
    k = 3
    clu_off = np.array([0, 4, 8, 12], np.int32)
    members = np.arange(12, dtype=np.int32)
    cluster_of = np.repeat(np.arange(k, dtype=np.int32), 4)
    per_colour = [np.flatnonzero(colors == c).astype(np.int32) for c in range(n_colors)]
    prob.reserve_partial(len(pop) * max(len(g) for g in per_colour))
    ora = oracle.Problem.from_synth(p)
    d = dev(pop)
    cache = prob.new_cache(len(pop))
    par_out = prob.eval_full(d, cache=cache)
    snapshot = pop.copy()
    work = prob.mixing_workspace(k)
    prob.estimate_distributions(dev(snapshot), dev(clu_off), dev(members), work, pinned=dev(pinned))
    rs = np.random.default_rng(15)
    state = pop.copy()
    kept_total = rejected = 0
    for c, g in enumerate(per_colour):
        ep = np.repeat(np.arange(len(pop), dtype=np.int32), len(g))
        eg = np.tile(g, len(pop))
        ec = cluster_of[ep]
        z = rs.normal(size=(2 * len(ep), 2, 3)).astype(np.float32)
        dep, deg = dev(ep), dev(eg)
        new = prob.sample_partial(d, work, k, dep, deg, dev(ec), dev(z), pinned=dev(pinned))
        out = prob.eval_partial(d, cache, dep, deg, new)
        kept = prob.accept_partial(d, cache, dep, deg, new, out, par_out)
        torch.cuda.synchronize()
        new_ref = mx.sample_batch(snapshot, clu_off, members, off, gpts, pinned, None, ep, eg, ec, z)
        np.testing.assert_array_equal(new.cpu().numpy(), new_ref)
        po = ora.evaluate(state)
        kids = np.stack([synth.apply_child(state, off, gpts, ep, eg, new_ref, e) for e in range(len(ep))])
        ko = ora.evaluate(kids)
        assert_parity(to_host(out), ko, what=f"colour {c} children")
        want = acc.accept_batch(ko["obj"], ko["flags"], ko["severity"], ep, eg, len(off) - 1, po["obj"],
                                po["flags"], po["severity"], [])
        np.testing.assert_array_equal(kept.cpu().numpy(), want, err_msg=f"colour {c} decisions")
        kept_total += int(want.sum())
        rejected += int(len(want) - want.sum())
        state = acc.apply(state, off, gpts, ep, eg, new_ref, want)
        np.testing.assert_array_equal(d.cpu().numpy(), state, err_msg=f"colour {c} parents")
    print("kept", kept_total, "rejected", rejected, flush=True)
    assert kept_total > 0 and rejected > 0
    fresh = to_host(morea.Problem.from_synth(p, max_population=len(pop)).eval_full(dev(state)))
    mine = to_host(par_out)
    np.testing.assert_array_equal(mine["flags"], fresh["flags"])
    np.testing.assert_array_equal(mine["counts"], fresh["counts"])
    np.testing.assert_allclose(mine["obj"], fresh["obj"], rtol=1e-6)
    assert_parity(mine, ora.evaluate(state), what="parents after the generation")


def test_c1_groups_of_three_and_four_points():
    """Up to 24 variables per distribution (several passes of the
    covariance lanes and a 24-column factor); groups of 5 points refused."""
    p = synth_problem(1)
    pop = synth.make_population(p, pop=40, seed=45, perturb_source=True)
    off, gpts = synth.make_groups(p, n_groups=12, sizes=(3, 4), seed=5)
    assert set(np.diff(off)) == {3, 4}
    prob = morea.Problem.from_synth(p, max_population=len(pop))
    prob.set_groups(off, gpts)
    n_groups = len(off) - 1
    pinned = pinned_bits(p)
    clusters = [list(range(0, 40)), list(range(10, 30)), [1, 2, 3, 4, 5, 6]]
    clu_off = np.concatenate([[0], np.cumsum([len(c) for c in clusters])]).astype(np.int32)
    clu_members = np.array(sum(clusters, []), np.int32)
    k = len(clusters)
    rs = np.random.default_rng(16)
    ep = np.repeat(np.arange(len(pop), dtype=np.int32), n_groups)
    eg = np.tile(np.arange(n_groups, dtype=np.int32), len(pop))
    ec = rs.integers(0, k, len(ep)).astype(np.int32)
    prob.reserve_partial(len(ep))
    rows = int(np.diff(off)[eg].sum())
    z = rs.normal(size=(rows, 2, 3)).astype(np.float32)
    mult = rs.uniform(0.5, 2.0, (k, n_groups)).astype(np.float32)
    d = dev(pop)
    work = prob.mixing_workspace(k)
    prob.estimate_distributions(d, dev(clu_off), dev(clu_members), work, pinned=dev(pinned))
    new = prob.sample_partial(d, work, k, dev(ep), dev(eg), dev(ec), dev(z), pinned=dev(pinned), mult=dev(mult))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(new.cpu().numpy(), mx.sample_batch(pop, clu_off, clu_members, off, gpts, pinned,
                                                                      mult, ep, eg, ec, z))
    rec = records(work, k * n_groups)
    modes = set()
    for c in range(k):
        for g in range(n_groups):
            ref = mx.estimate(pop, clusters[c], [int(v) for v in gpts[off[g]:off[g + 1]]], pinned)
            check_record(rec[c * n_groups + g], ref)
            modes.add(ref[3])
    assert 0 in modes and 1 in modes
    assert max(int(r["n_free"]) for r in rec) > 12
    # groups of five points are refused
    off5, pts5 = synth.make_groups(p, n_groups=3, sizes=(5, 5), seed=6)
    prob.set_groups(off5, pts5)
    prob.reserve_partial(8)
    with pytest.raises(morea.MoreaError) as err:
        prob.estimate_distributions(d, dev(clu_off), dev(clu_members), prob.mixing_workspace(k))
    assert err.value.status == morea.MOREA_ERANGE


def test_sampling_and_estimation_argument_errors():
    p = synth_problem(1)
    pop = synth.make_population(p, pop=4, seed=46)
    prob, off, gpts, colors = setup(p, len(pop))
    with pytest.raises(morea.MoreaError) as err:
        prob.mixing_workspace(2)                       # no reservation yet
    assert err.value.status == morea.MOREA_ESTATE
    prob.reserve_partial(8)
    work = prob.mixing_workspace(2)
    d = dev(pop)
    ep = np.zeros(9, np.int32)
    eg = np.zeros(9, np.int32)
    z = np.zeros((18, 2, 3), np.float32)
    with pytest.raises(morea.MoreaError) as err:        # more evaluations than reserved
        prob.sample_partial(d, work, 2, dev(ep), dev(eg), dev(ep), dev(z))
    assert err.value.status == morea.MOREA_ERANGE
    with pytest.raises(morea.MoreaError) as err:        # workspace for fewer clusters
        prob.sample_partial(d, work, 3, dev(ep[:8]), dev(eg[:8]), dev(ep[:8]), dev(z[:16]))
    assert err.value.status == morea.MOREA_ERANGE
    torch.cuda.synchronize()
