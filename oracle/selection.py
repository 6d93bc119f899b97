"""Selection and clustering at the start of a generation -- plain reference,
test infrastructure only (not part of the library's path).

Sec. 3: each generation starts from a selection of non-dominated solutions
of the population, clustered into k equally sized clusters.  The paper
leaves the details to MO-RV-GOMEA's literature; the readings (listed in the
design notes):
  * domination is the constraint domination of the acceptance (feasibility,
    fold violation and steering excess, then Pareto domination);
  * fronts by peeling: front 0 holds the solutions no other solution
    dominates, front r those no solution outside fronts 0..r-1 dominates;
    the selection takes whole fronts in order and the last one it needs in
    ascending index, until it holds `size` solutions; a solution with invalid
    coordinates or an objective or severity that is not finite (NaN or an
    infinity) is never selected;
  * objectives are normalised over the selection, (v - lo) / (hi - lo), 0
    where hi == lo; distances are squared Euclidean, FP64, summed over the
    three objectives in order;
  * leaders: the first is the selected solution with the smallest first
    objective, each next one the selected solution farthest (largest
    smallest distance) from the leaders so far; ties to the lower index;
    min(k, |S|) leaders;
  * cluster j holds the m = min(|S|, ceil(2 |S| / k)) selected solutions
    nearest to leader j (ties to the lower index), listed in ascending
    index; clusters without a leader are empty;
  * every valid solution of the population is varied with the cluster of its
    nearest leader (ties to the lower cluster), an invalid one with none (-1).
"""
import math

from oracle import accept as acc


def valid(obj, flags, severity):
    return not (int(flags) & acc.INVALID) and all(math.isfinite(float(v)) for v in list(obj) + [severity])


def fronts(obj, flags, sev, guidance_max=math.inf):
    """Front index of every valid solution (None for invalid ones)."""
    n = len(flags)
    sols = [(obj[i], flags[i], sev[i]) for i in range(n)]
    rank = [None] * n
    left = [i for i in range(n) if valid(*sols[i])]
    r = 0
    while left:
        front = [i for i in left
                 if not any(acc.constraint_dominates(sols[j], sols[i], guidance_max) for j in left if j != i)]
        for i in front:
            rank[i] = r
        left = [i for i in left if rank[i] is None]
        r += 1
    return rank


def select(obj, flags, sev, size, guidance_max=math.inf):
    """Indices of the selection, ascending."""
    rank = fronts(obj, flags, sev, guidance_max)
    chosen = []
    r = 0
    while len(chosen) < size and any(x is not None and x >= r for x in rank):
        chosen += [i for i in range(len(rank)) if rank[i] == r][:size - len(chosen)]
        r += 1
    return sorted(chosen)


def normaliser(obj, sel):
    lo = [min(float(obj[i][o]) for i in sel) for o in range(3)]
    hi = [max(float(obj[i][o]) for i in sel) for o in range(3)]

    def norm(v):
        return [((float(v[o]) - lo[o]) / (hi[o] - lo[o])) if hi[o] > lo[o] else 0.0 for o in range(3)]
    return norm


def dist(a, b):
    s = 0.0
    for o in range(3):
        d = a[o] - b[o]
        s = s + d * d
    return s


def clusters(obj, flags, sev, size, k, guidance_max=math.inf):
    """(selection, leaders, members per cluster, cluster of every solution)."""
    sel = select(obj, flags, sev, size, guidance_max)
    n = len(flags)
    if not sel:
        return sel, [], [[] for _ in range(k)], [-1] * n
    norm = normaliser(obj, sel)
    pts = {i: norm(obj[i]) for i in range(n) if valid(obj[i], flags[i], sev[i])}
    first = min(sel, key=lambda i: (pts[i][0], i))
    leaders = [first]
    nearest = {i: dist(pts[i], pts[first]) for i in sel}
    while len(leaders) < min(k, len(sel)):
        nxt = min(sel, key=lambda i: (-nearest[i], i))
        leaders.append(nxt)
        for i in sel:
            d = dist(pts[i], pts[nxt])
            if d < nearest[i]:
                nearest[i] = d
    m = min(len(sel), -(-2 * len(sel) // k))
    members = []
    for j in range(k):
        if j < len(leaders):
            near = sorted(sel, key=lambda i: (dist(pts[i], pts[leaders[j]]), i))[:m]
            members.append(sorted(near))
        else:
            members.append([])
    cluster_of = []
    for i in range(n):
        if i not in pts:
            cluster_of.append(-1)
            continue
        cluster_of.append(min(range(len(leaders)), key=lambda j: (dist(pts[i], pts[leaders[j]]), j)))
    return sel, leaders, members, cluster_of
