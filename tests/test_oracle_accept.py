"""Pins of the acceptance reference (Sec. 3 optimal mixing).

The decision rule is pinned by hand-worked cases, by the order properties
constraint domination must have (irreflexive, antisymmetric, transitive; it
reduces to Pareto domination among feasible solutions and to the violation
order among infeasible ones), and by a textbook 2-D skyline (sort and sweep)
that decides non-domination within an archive by another route.  The
steering bound (Sec. 4.3.2) is pinned by hand-worked cases, by changing
nothing when infinite and by keeping the order properties.  Applying the
accepted children is pinned against building each child on its own."""
import bisect
import functools

import numpy as np

import synth
from oracle import accept as acc
from oracle import fos

F, S, T, BAD = 0, 1, 2, 4     # feasible, fold in S, fold in T, invalid


def sol(obj, flags=F, sev=0.0):
    return (tuple(float(v) for v in obj), flags, float(sev))


def test_hand_worked_cases():
    pd = acc.pareto_dominates
    assert pd((1, 2, 3), (1, 2, 4)) and not pd((1, 2, 4), (1, 2, 3))
    assert not pd((1, 2, 3), (1, 2, 3))                  # equal vectors: neither
    assert not pd((1, 2, 3), (2, 1, 3)) and not pd((2, 1, 3), (1, 2, 3))
    assert pd((0, 0, 0), (1, 1, 1))
    cd = acc.constraint_dominates
    assert cd(sol((9, 9, 9)), sol((0, 0, 0), S, 5.0))    # feasible beats any infeasible
    assert not cd(sol((0, 0, 0), S, 5.0), sol((9, 9, 9)))
    assert cd(sol((9, 9, 9), T, 0.5), sol((0, 0, 0), S, 1.0))
    assert not cd(sol((0, 0, 0), S, 1.0), sol((9, 9, 9), S | T, 1.0))   # equal violation
    assert not cd(sol((1, 1, 1), BAD), sol((9, 9, 9), BAD))             # invalid never wins
    assert cd(sol((9, 9, 9), S, 1e30), sol((0, 0, 0), BAD))
    assert cd(sol((1, 1, 1)), sol((1, float("nan"), 0)))                # NaN counts as invalid
    inf = float("inf")
    assert cd(sol((1, 1, 1)), sol((-inf, 0, 0)))                        # so does an infinity
    assert cd(sol((9, 9, 9), S, 1e30), sol((0, inf, 0)))
    assert not cd(sol((0, 0, inf)), sol((9, 9, 9), S, 1e30))
    assert not acc.accept(sol((-inf, -inf, -inf)), sol((9, 9, 9)), [])  # never kept
    assert acc.violation((0, 0, 0), F, inf) == (False, (inf, inf))      # an infinite severity too
    parent = sol((1, 2, 3))
    trade = sol((0.5, 2.5, 3))                                          # better in one, worse in one
    assert acc.accept(trade, parent, [])                                # vacuously non-dominated
    assert not acc.accept(trade, parent, [(0.5, 2.5, 2.9)])             # dominated in the archive
    assert acc.accept(trade, parent, [(0.5, 2.5, 3.0), (1, 1, 4)])      # an equal member does not dominate
    assert acc.accept(sol((1, 2, 2.5)), parent, [(0, 0, 0)])            # dominates its parent
    assert not acc.accept(sol((0, 0, 0), S, 0.5), sol((1, 1, 1)), [])   # infeasible child, feasible parent
    assert acc.accept(sol((5, 5, 5), S, 0.5), sol((0, 0, 0), T, 0.7), [(0, 0, 0)])
    assert not acc.accept(sol((0, 0, 0), S, 0.5), sol((9, 9, 9), T, 0.4), [])   # archive path needs feasibility
    assert not acc.accept(sol((0, 0, 0), BAD), sol((9, 9, 9), BAD), [])


def random_solutions(rs, n):
    out = []
    for _ in range(n):
        flags = int(rs.choice([F, F, F, S, T, S | T, BAD]))
        out.append(sol(rs.integers(0, 3, 3), flags, float(rs.integers(0, 3)) * 0.5))
    return out


def test_constraint_domination_is_a_strict_order():
    rs = np.random.default_rng(5)
    xs = random_solutions(rs, 60)
    cd = acc.constraint_dominates
    rel = [[cd(a, b) for b in xs] for a in xs]
    for i in range(len(xs)):
        assert not rel[i][i]
        for j in range(len(xs)):
            assert not (rel[i][j] and rel[j][i])
            if rel[i][j]:
                assert all(rel[i][k] for k in range(len(xs)) if rel[j][k])
    # among feasible solutions it is Pareto domination, among infeasible
    # (finite) ones the order of the violations
    for a in xs:
        for b in xs:
            fa, va = acc.violation(*a)
            fb, vb = acc.violation(*b)
            if fa and fb:
                assert cd(a, b) == acc.pareto_dominates(a[0], b[0])
            elif not fa and not fb:
                assert cd(a, b) == (va < vb)


def skyline_dominated(archive, q):
    """q (x, y) is dominated by a member of the archive: sort by x, sweep the
    running minimum of y; members with the same x dominate when y is smaller."""
    pts = sorted(archive)
    xs = [p[0] for p in pts]
    lo = bisect.bisect_left(xs, q[0])
    hi = bisect.bisect_right(xs, q[0])
    run = min((p[1] for p in pts[:lo]), default=np.inf)
    same = min((p[1] for p in pts[lo:hi]), default=np.inf)
    return run <= q[1] or same < q[1]


def test_archive_non_domination_matches_skyline():
    rs = np.random.default_rng(8)
    for _ in range(40):
        archive = [tuple(map(float, rs.integers(0, 6, 2))) + (1.0,) for _ in range(int(rs.integers(0, 12)))]
        for _ in range(20):
            q = tuple(map(float, rs.integers(0, 6, 2))) + (1.0,)
            parent = sol((0, 0, 0))                       # never dominated by the child
            got = acc.accept(sol(q), parent, archive)
            assert got == (not skyline_dominated([a[:2] for a in archive], q[:2]))


def test_batch_guards_and_out_of_range():
    obj = np.array([[1, 1, 1], [0, 0, 0], [0, 0, 0], [0, 0, 0]], np.float32)
    flags = np.zeros(4, np.uint8)
    sev = np.zeros(4, np.float32)
    ep = np.array([0, 1, 2, -1], np.int32)
    eg = np.array([0, 0, 0, 0], np.int32)
    pobj = np.array([[2, 2, 2], [0, 0, 0]], np.float32)
    out = acc.accept_batch(obj, flags, sev, ep, eg, 1, pobj, np.zeros(2, np.uint8), np.zeros(2, np.float32), [])
    # eval 1 equals its parent and the archive is empty: accepted as non-dominated
    assert out.tolist() == [1, 1, 0, 0]
    out = acc.accept_batch(obj, flags, sev, ep, np.array([0, 1, 0, 0], np.int32), 1, pobj,
                           np.zeros(2, np.uint8), np.zeros(2, np.float32), [(0.0, 0.0, 0.0)])
    assert out.tolist() == [1, 0, 0, 0]


@functools.lru_cache(maxsize=None)
def colour_groups(config):
    p = synth.make_problem(config)
    elements, colors = fos.build(p.n_points, p.tets)
    return p, elements, colors


def test_apply_matches_children_built_one_by_one():
    p, elements, colors = colour_groups(1)
    rs = np.random.default_rng(3)
    parents = synth.make_population(p, pop=5, seed=4, perturb_source=True)
    for c in range(max(colors) + 1):
        mine = [e for e, k in zip(elements, colors) if k == c]
        off = np.arange(0, 2 * len(mine) + 1, 2, dtype=np.int32)
        pts = np.array(mine, np.int32).reshape(-1)
        ep, eg, new = synth.make_children(p, parents, off, pts, seed=c)
        mask = (rs.random(len(ep)) < 0.4).astype(np.uint8)
        got = acc.apply(parents, off, pts, ep, eg, new, mask)
        want = parents.copy()
        for e in np.flatnonzero(mask):
            idx = pts[off[eg[e]]:off[eg[e] + 1]]
            want[ep[e]][:, :, idx] = synth.apply_child(parents, off, pts, ep, eg, new, e)[:, :, idx]
        np.testing.assert_array_equal(got, want)
        # untouched points keep their values; none accepted leaves the parents
        np.testing.assert_array_equal(acc.apply(parents, off, pts, ep, eg, new, np.zeros_like(mask)), parents)
        # the order of the evaluations of one colour does not matter
        perm = rs.permutation(len(ep))
        rows = np.concatenate([np.arange(2 * e, 2 * e + 2) for e in perm])
        np.testing.assert_array_equal(acc.apply(parents, off, pts, ep[perm], eg[perm], new[rows], mask[perm]), got)


def test_steering_bound():
    inf = float("inf")
    cd = acc.constraint_dominates
    inside, outside = sol((5, 5, 1.0)), sol((0, 0, 2.0))
    assert cd(inside, outside, 1.5) and not cd(outside, inside, 1.5)      # the bound is a hard constraint
    assert cd(outside, inside, inf) is False and cd(outside, inside) is False
    assert acc.pareto_dominates((0, 0, 1.0), (5, 5, 1.0))
    # both above the bound: the smaller excess wins; a fold outranks any excess
    assert cd(sol((9, 9, 1.6)), sol((0, 0, 1.9)), 1.5)
    assert cd(sol((9, 9, 100.0)), sol((0, 0, 1.0), S, 0.5), 1.5)
    assert not cd(sol((0, 0, 1.0), S, 0.5), sol((9, 9, 100.0)), 1.5)
    assert cd(sol((9, 9, 1.9), S, 0.5), sol((0, 0, 1.6), S, 0.7), 1.5)
    assert cd(sol((9, 9, 1.6), S, 0.5), sol((0, 0, 1.9), S, 0.5), 1.5)
    # equal to the bound is inside; the archive path needs the bound too
    assert acc.violation((0, 0, 1.5), F, 0.0, 1.5)[0]
    assert not acc.accept(sol((0.5, 9, 1.7)), sol((1, 1, 1.0)), [], 1.5)
    assert acc.accept(sol((0.5, 9, 1.4)), sol((1, 1, 1.0)), [], 1.5)
    # the excess is the FP32 difference
    assert acc.violation((0, 0, 1.5000001), F, 0.0, 1.5)[1] == (0.0, float(np.float32(1.5000001) - np.float32(1.5)))


def test_infinite_bound_changes_nothing_and_order_holds():
    rs = np.random.default_rng(6)
    xs = random_solutions(rs, 50)
    arch = [tuple(map(float, rs.integers(0, 3, 3))) for _ in range(6)]
    for a in xs:
        for b in xs:
            assert acc.accept(a, b, arch, float("inf")) == acc.accept(a, b, arch)
    rel = [[acc.constraint_dominates(a, b, 1.0) for b in xs] for a in xs]
    for i in range(len(xs)):
        assert not rel[i][i]
        for j in range(len(xs)):
            assert not (rel[i][j] and rel[j][i])
            if rel[i][j]:
                assert all(rel[i][k] for k in range(len(xs)) if rel[j][k])
