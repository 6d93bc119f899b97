"""Pins of the elitist-archive reference (Sec. 3, Sec. 4.3.2) and of the
multiplier adaptation.

* Without capacity pressure or a bound, an update equals the classic
  archive that takes offers one at a time (insert unless dominated by or
  equal to a member, then drop the members it dominates), written here
  independently; the result is also checked against a brute-force
  non-dominated filter by NumPy broadcasting.
* Hand-worked cases: dominated offers, equal vectors (the member wins),
  infeasible and invalid offers, slots freed and reused in ascending order.
* Capacity: hand-worked boxes on a line of non-dominated points, and the
  properties every thinning has (at most the capacity, one member per box,
  every dropped candidate shares its box with an earlier kept one).
* Steering: members above the bound are purged, offers above it refused.
* Multipliers: hand-worked sequences of the adaptation.
"""
import math

import numpy as np

from oracle import accept as acc
from oracle import archive as ar


def one_by_one(members, offers):
    arc = [tuple(m) for m in members]
    for o in offers:
        o = tuple(o)
        if any(all(a <= b for a, b in zip(m, o)) for m in arc):
            continue                                  # dominated by or equal to a member
        arc = [m for m in arc if not (all(a <= b for a, b in zip(o, m)) and o != m)] + [o]
    return arc


def nd_filter(v):
    v = np.asarray(v, np.float64)
    le = np.all(v[:, None, :] <= v[None, :, :], axis=2)
    lt = np.any(v[:, None, :] < v[None, :, :], axis=2)
    dominated = np.any(le & lt, axis=0)
    return v[~dominated]


def vectors(arc):
    return sorted(tuple(float(x) for x in arc.obj[s]) for s in arc.members())


def offers(rs, n, grid=4):
    obj = rs.integers(0, grid, (n, 3)).astype(np.float32)
    flags = np.zeros(n, np.uint8)
    sev = np.zeros(n, np.float32)
    return obj, flags, sev


def test_matches_one_by_one_and_brute_force():
    rs = np.random.default_rng(0)
    arc = ar.Archive(4096)
    seen = []
    for step in range(6):
        obj, fl, sv = offers(rs, 60, grid=6)
        before = vectors(arc)
        ins, slot = ar.update(arc, obj, fl, sv)
        seen += [tuple(map(float, o)) for o in obj]
        want = sorted(one_by_one(before, [tuple(map(float, o)) for o in obj]))
        assert vectors(arc) == want
        nd = sorted(set(map(tuple, nd_filter(seen).tolist())))
        assert vectors(arc) == nd
        # inserted offers are exactly the first occurrences of new members
        for i in np.flatnonzero(ins):
            assert tuple(arc.obj[slot[i]]) == tuple(obj[i])
        assert arc.levels == 0


def test_hand_worked_update():
    arc = ar.Archive(4)
    obj = np.array([[1, 2, 3], [2, 2, 3], [1, 2, 3], [3, 1, 3], [0, 5, 5], [0, 0, 0]], np.float32)
    fl = np.array([0, 0, 0, 0, 0, 1], np.uint8)                 # the last one folds: never a member
    sv = np.array([0, 0, 0, 0, 0, 2], np.float32)
    ins, slot = ar.update(arc, obj[:5], fl[:5], sv[:5])
    # [2,2,3] is dominated by [1,2,3]; the second [1,2,3] is a duplicate
    assert ins.tolist() == [1, 0, 0, 1, 1] and slot.tolist() == [0, -1, -1, 1, 2]
    assert arc.stamp.tolist() == [0, 1, 2, -1] and arc.next_stamp == 3
    assert arc.best_guidance() == 3.0
    # an infeasible offer and an invalid one are refused; a dominating one
    # frees the slots of the members it dominates, and takes the first free slot
    obj2 = np.array([[0, 0, 0], [1, 1, 2], [np.nan, 0, 0]], np.float32)
    ins, slot = ar.update(arc, obj2, np.array([1, 0, 0], np.uint8), np.array([2, 0, 0], np.float32))
    assert ins.tolist() == [0, 1, 0]
    assert slot.tolist() == [-1, 0, -1]
    # [1,1,2] dominates [1,2,3] and [3,1,3]; [0,5,5] stays
    assert arc.stamp.tolist() == [3, -1, 2, -1]
    assert np.all(np.isinf(arc.obj[1])) and np.all(np.isinf(arc.obj[3]))
    assert vectors(arc) == [(0.0, 5.0, 5.0), (1.0, 1.0, 2.0)]
    assert list(arc.members()) == [2, 0]                       # stamp order


def test_equal_offer_to_a_member_is_not_inserted():
    arc = ar.Archive(8)
    o = np.array([[1, 1, 1]], np.float32)
    ar.update(arc, o, np.zeros(1, np.uint8), np.zeros(1, np.float32))
    ins, _ = ar.update(arc, np.repeat(o, 3, axis=0), np.zeros(3, np.uint8), np.zeros(3, np.float32))
    assert ins.tolist() == [0, 0, 0] and len(arc.members()) == 1


def test_thinning_hand_worked_line():
    """Six non-dominated points on x + y = 5 (z = 0) and capacity 3: at L = 3
    the x boxes are floor(x / 5 * 3) = 0,0,1,1,2,3->2, i.e. 0,0,1,1,2,2 with y
    mirrored, so 3 boxes: the earliest of each pair stays."""
    arc = ar.Archive(3)
    x = np.arange(6, dtype=np.float32)
    obj = np.stack([x, 5 - x, np.zeros(6, np.float32)], axis=1)
    ins, slot = ar.update(arc, obj, np.zeros(6, np.uint8), np.zeros(6, np.float32))
    assert ar.box_count(obj.astype(np.float64), 3) == 3
    assert ar.box_count(obj.astype(np.float64), 2) == 2
    assert arc.levels == 3
    assert ins.tolist() == [1, 0, 1, 0, 1, 0]
    assert sorted(arc.obj[arc.members(), 0].tolist()) == [0.0, 2.0, 4.0]


def test_thinning_properties():
    rs = np.random.default_rng(3)
    cap = 40
    arc = ar.Archive(cap)
    for step in range(5):
        n = 300
        u = rs.random((n, 2))
        obj = np.stack([u[:, 0], u[:, 1], 2.0 - u[:, 0] - u[:, 1]], axis=1).astype(np.float32)  # a plane: all non-dominated
        before = [tuple(arc.obj[s]) for s in arc.members()]
        ins, slot = ar.update(arc, obj, np.zeros(n, np.uint8), np.zeros(n, np.float32))
        m = arc.members()
        assert 0 < len(m) <= cap and arc.levels >= 1
        kept = arc.obj[m].astype(np.float64)
        cand = np.array(before + [tuple(o) for o in obj], np.float64)
        bx_all = [tuple(b) for b in ar.boxes(cand, arc.levels)]
        # the boxes are those of the candidates' common range: one member each
        keys = {}
        for i, b in enumerate(bx_all):
            keys.setdefault(b, i)
        first = sorted(keys.values())
        assert len(first) == len(m) and len(first) <= cap
        assert sorted(map(tuple, kept.tolist())) == sorted(map(tuple, cand[first].tolist()))
        # a finer resolution would exceed the capacity (the search's last step)
        assert ar.box_count(cand, arc.levels + 1) > cap or arc.levels == min(cap, ar.MAX_LEVELS)


def test_steering_purge_and_refusal():
    arc = ar.Archive(16)
    obj = np.array([[1, 5, 1.0], [2, 4, 2.0], [3, 3, 3.0], [4, 2, 4.0]], np.float32)
    ar.update(arc, obj, np.zeros(4, np.uint8), np.zeros(4, np.float32))
    assert arc.best_guidance() == 1.0
    bound = ar.steering_bound(arc.best_guidance())
    assert bound == 1.5
    off = np.array([[0, 9, 1.4], [0, 0, 1.6]], np.float32)     # the second dominates all but is above the bound
    ins, _ = ar.update(arc, off, np.zeros(2, np.uint8), np.zeros(2, np.float32), guidance_max=bound)
    assert ins.tolist() == [1, 0]
    assert vectors(arc) == [(0.0, 9.0, 1.399999976158142), (1.0, 5.0, 1.0)]
    assert ar.steering_bound(math.inf) == math.inf
    assert ar.steering_bound(0.1) == float(np.float32(1.5) * np.float32(0.1))


def test_archive_members_never_dominate_each_other_and_acceptance_reads_free_slots():
    rs = np.random.default_rng(9)
    arc = ar.Archive(64)
    for _ in range(4):
        obj, fl, sv = offers(rs, 100, grid=8)
        ar.update(arc, obj, fl, sv)
        m = arc.obj[arc.members()]
        for i in range(len(m)):
            for j in range(len(m)):
                assert i == j or not acc.pareto_dominates(m[i], m[j])
        # free slots hold (inf, inf, inf): they dominate no vector
        free = arc.obj[arc.stamp < 0]
        assert all(not acc.pareto_dominates(f, (1e30, 1e30, 1e30)) for f in free)


def test_multiplier_adaptation_hand_worked():
    mult = np.array([[1.0, 1.0, 2.0, 0.5]], np.float32)
    nis = np.array([[0, 24, 0, 3]], np.int64)
    imp = np.array([[1, 0, 0, 1]], np.uint8)
    ar.adapt_multipliers(imp, mult, nis)
    f = np.float32
    assert mult[0, 0] == f(f(1.0) / f(0.9)) and nis[0, 0] == 0            # improvement: up
    assert mult[0, 1] == f(f(0.9) * f(1.0)) and nis[0, 1] == 25           # stretch reached 25: down
    assert mult[0, 2] == f(f(0.9) * f(2.0)) and nis[0, 2] == 0            # above 1: down, no stretch
    assert mult[0, 3] == f(f(1.0) / f(0.9)) and nis[0, 3] == 0            # below 1, improvement: from 1 up
    assert not imp.any()
    # no improvement with c < 1 and a short stretch: reset to 1
    mult = np.array([[0.5]], np.float32)
    nis = np.array([[2]], np.int64)
    ar.adapt_multipliers(np.zeros((1, 1), np.uint8), mult, nis)
    assert mult[0, 0] == 1.0 and nis[0, 0] == 3
    # repeated improvements stop at 10
    mult = np.array([[9.5]], np.float32)
    nis = np.zeros((1, 1), np.int64)
    ar.adapt_multipliers(np.ones((1, 1), np.uint8), mult, nis)
    assert mult[0, 0] == 10.0


def test_mark_improvements():
    imp = np.zeros((2, 3), np.uint8)
    ar.mark_improvements(imp, eval_parent=[0, 1, 1, 2, 5], eval_group=[0, 1, 2, 2, 0],
                         eval_cluster=[1, 0, 0, 1, 0], accepted=[1, 1, 0, 1, 1],
                         parent_inserted=np.array([1, 1, 0], np.uint8))
    # e0 (c1, g0) kept and inserted; e1 (c0, g1); e2 not kept; e3 parent not
    # inserted; e4 parent out of range
    assert imp.tolist() == [[0, 1, 0], [1, 0, 0]]
