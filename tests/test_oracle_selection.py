"""Pins of the selection and clustering reference (Sec. 3).

Fronts are pinned by hand-worked sets and by an independent definition (the
front index is the length of the longest chain of dominating solutions);
the selection by its size and tie rule; the clustering by a hand-worked
one-dimensional case, by the farthest-point property of the leaders, by equal
cluster sizes, and by every solution's cluster leader being its nearest."""
import functools
import math

import numpy as np

from oracle import accept as acc
from oracle import selection as sl


def arrays(objs, flags=None, sev=None):
    n = len(objs)
    return (np.array(objs, np.float32), np.zeros(n, np.uint8) if flags is None else np.array(flags, np.uint8),
            np.zeros(n, np.float32) if sev is None else np.array(sev, np.float32))


def test_hand_worked_fronts_and_selection():
    obj, fl, sv = arrays([(0, 3, 1), (1, 1, 1), (3, 0, 1), (2, 2, 1), (3, 3, 1), (1, 1, 1), (0, 0, 9)])
    assert sl.fronts(obj, fl, sv) == [0, 0, 0, 1, 2, 0, 0]
    # infeasible solutions come after every feasible one, ordered by violation
    obj, fl, sv = arrays([(5, 5, 5), (0, 0, 0), (0, 0, 0), (9, 9, 9), (1, 1, 1)], [0, 1, 2, 0, 4], [0, 2.0, 1.0, 0, 0])
    assert sl.fronts(obj, fl, sv) == [0, 3, 2, 1, None]
    assert sl.select(obj, fl, sv, 2) == [0, 3]
    assert sl.select(obj, fl, sv, 10) == [0, 1, 2, 3]          # the invalid one never
    obj, fl, sv = arrays([(1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 2, 2), (0, 0.5, 0.5)])
    assert sl.select(obj, fl, sv, 2) == [0, 1]                   # last front cut in index order
    # an infinite objective or severity makes a solution invalid: never
    # selected (it would otherwise dominate everything or normalise to NaN)
    inf = float("inf")
    obj, fl, sv = arrays([(-inf, 0, 0), (1, 1, 1), (0, inf, 0), (2, 0, 2), (0, 0, 0)], sev=[0, 0, 0, 0, inf])
    assert sl.fronts(obj, fl, sv) == [None, 0, None, 0, None]
    assert sl.select(obj, fl, sv, 5) == [1, 3]
    sel, leaders, members, cluster_of = sl.clusters(obj, fl, sv, 5, 2)
    assert cluster_of[0] == cluster_of[2] == cluster_of[4] == -1
    assert sorted(map(len, members)) == [2, 2]


def chain_rank(obj, flags, sev):
    sols = [(obj[i], flags[i], sev[i]) for i in range(len(flags))]
    ok = [sl.valid(*s) for s in sols]

    @functools.lru_cache(maxsize=None)
    def rank(i):
        dom = [j for j in range(len(sols)) if ok[j] and j != i and acc.constraint_dominates(sols[j], sols[i])]
        return 0 if not dom else 1 + max(rank(j) for j in dom)
    return [rank(i) if ok[i] else None for i in range(len(sols))]


def test_fronts_equal_longest_dominating_chain():
    rs = np.random.default_rng(9)
    for _ in range(6):
        n = 40
        obj = rs.integers(0, 5, (n, 3)).astype(np.float32)
        fl = rs.choice(np.array([0, 0, 0, 1, 2, 4], np.uint8), n)
        sv = (rs.integers(0, 4, n) * 0.5).astype(np.float32)
        assert sl.fronts(obj, fl, sv) == chain_rank(obj, fl, sv)


def test_one_dimensional_clustering():
    xs = [0.0, 1.0, 2.0, 3.0, 10.0, 4.0, 9.0]
    obj, fl, sv = arrays([(x, 0, 0) for x in xs])
    # equal in the other objectives, every x is a front of its own; all 7 selected
    sel, leaders, members, cluster_of = sl.clusters(obj, fl, sv, 7, 3)
    assert sel == list(range(7))
    # leaders: smallest x (index 0), then the farthest (x = 10, index 4), then
    # the one farthest from both (x = 4, index 5, 4 away from x = 0)
    assert leaders == [0, 4, 5]
    m = math.ceil(2 * 7 / 3)
    assert all(len(c) == m for c in members)
    assert members[0] == [0, 1, 2, 3, 5]                  # nearest 5 to x = 0
    assert members[1] == [2, 3, 4, 5, 6]                  # nearest to x = 10: 10, 9, 4, 3, 2
    assert cluster_of == [0, 0, 0, 2, 1, 2, 1]


def test_clustering_properties():
    rs = np.random.default_rng(11)
    n, k = 60, 5
    obj = rs.normal(size=(n, 3)).astype(np.float32)
    fl = rs.choice(np.array([0, 0, 0, 0, 1, 4], np.uint8), n)
    sv = rs.uniform(0, 1, n).astype(np.float32)
    sel, leaders, members, cluster_of = sl.clusters(obj, fl, sv, 30, k)
    assert len(sel) == 30 and len(set(leaders)) == k
    # normalised over the selection, computed here on its own
    o64 = obj.astype(np.float64)
    lo, hi = o64[sel].min(axis=0), o64[sel].max(axis=0)
    p = {i: list((o64[i] - lo) / (hi - lo)) for i in range(n) if sl.valid(obj[i], fl[i], sv[i])}
    # the second leader is the selected solution farthest from the first
    far = max(sel, key=lambda i: (sl.dist(p[i], p[leaders[0]]), -i))
    assert leaders[1] == far
    m = math.ceil(2 * 30 / k)
    for j in range(k):
        assert len(members[j]) == m and leaders[j] in members[j] and members[j] == sorted(members[j])
        worst = max(sl.dist(p[i], p[leaders[j]]) for i in members[j])
        assert all(sl.dist(p[i], p[leaders[j]]) >= worst for i in sel if i not in members[j])
    for i in range(n):
        if i not in p:
            assert cluster_of[i] == -1
        else:
            d = [sl.dist(p[i], p[leaders[j]]) for j in range(k)]
            assert d[cluster_of[i]] == min(d)
    # fewer selected solutions than clusters: the rest stay empty
    sel, leaders, members, cluster_of = sl.clusters(obj, fl, sv, 3, k)
    assert len(leaders) == 3 and all(members[j] == [] for j in range(3, k))
