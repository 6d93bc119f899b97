"""Elitist archive of the optimizer -- plain reference, test infrastructure
only (not part of the library's path).

Sec. 3: non-dominated solutions are kept across generations in an elitist
archive of a fixed capacity (2000 in the parameter listing of App. C), whose
management the paper takes from its reference on elitist archiving (an
objective space divided into boxes whose size adapts to the capacity).
Sec. 4.3.2: once adaptive steering is on, only solutions whose guidance value
lies in [s_G, 1.5 s_G] are kept, s_G the best guidance value in the archive;
App. D notes that this purges the archive when it switches on.

Readings (listed in the design notes):
  * the archive holds feasible solutions (R24's feasibility: valid, no fold,
    finite objectives and severity) by their objective vectors; each member
    keeps the slot it was given and an insertion stamp that orders members;
  * an update offers solutions (the population after a batch of
    acceptances) and a steering bound (infinite when off); the candidates
    are the members in stamp order, then the feasible offers in index
    order, minus every candidate whose guidance value is above the bound;
  * a candidate stays unless another candidate Pareto-dominates it or an
    earlier candidate has the same objective vector;
  * if more than `capacity` stay, they are thinned by boxes: with lo, hi the
    FP64 minimum and maximum of each objective over them, a value v lies in
    box min(L - 1, floor(((v - lo) / (hi - lo)) * L)) (0 where hi == lo);
    L is found by a binary search over [1, min(capacity, 1024)] for a
    resolution whose number of occupied boxes is at most the capacity
    (mid = (a + b + 1) // 2, kept when it fits), and each occupied box keeps
    its earliest candidate;
  * members that do not stay free their slots; staying offers fill the free
    slots in ascending slot order, in offer order, each taking the next
    stamp; a free slot holds the objective vector (inf, inf, inf), which
    dominates nothing, so the acceptance can read every slot;
  * s_G is the smallest guidance value among the members after the update
    (inf when empty); the steering bound of a generation is fl32(1.5 s_G),
    computed in FP32 from the s_G of the update before it;
  * distribution multipliers (MO-RV-GOMEA's adaptive variance scaling in a
    reduced form; the paper's listing sets no anticipated mean shift): a
    (cluster, element) improves in a generation when a kept child sampled
    from it belongs to a parent that then entered the archive; on
    improvement its no-improvement stretch resets and c = max(c, 1) / 0.9,
    at most 10; otherwise the stretch grows while c <= 1, c = 0.9 c when
    c > 1 or the stretch has reached 25, and a c below 1 with a shorter
    stretch is reset to 1 (FP32 arithmetic).
"""
import math

import numpy as np

from oracle import accept as acc

MAX_LEVELS = 1024        # boxes per objective at most


class Archive:
    """Slots [capacity] of objective vectors and stamps (-1: free)."""

    def __init__(self, capacity):
        self.capacity = int(capacity)
        self.obj = np.full((self.capacity, 3), np.inf, np.float32)
        self.stamp = np.full(self.capacity, -1, np.int64)
        self.next_stamp = 0
        self.levels = 0          # L of the last thinning (0: none)

    def members(self):
        """Occupied slots in stamp order."""
        occ = np.flatnonzero(self.stamp >= 0)
        return occ[np.argsort(self.stamp[occ], kind="stable")]

    def best_guidance(self):
        m = self.members()
        return float(np.min(self.obj[m, 2])) if len(m) else math.inf


def feasible(obj, flags, sev):
    f, _ = acc.violation(obj, flags, sev)
    return f


def boxes(vals, L):
    """Box indices [n][3] of the candidates' objective vectors at resolution L
    (the range is that of the given vectors)."""
    v = np.asarray(vals, np.float64)
    lo, hi = v.min(axis=0), v.max(axis=0)
    out = np.zeros(v.shape, np.int64)
    for o in range(3):
        if hi[o] > lo[o]:
            t = (v[:, o] - lo[o]) / (hi[o] - lo[o])
            out[:, o] = np.minimum(L - 1, np.floor(t * L).astype(np.int64))
    return out


def first_in_box(vals, L):
    """Indices of the earliest candidate of every occupied box, ascending."""
    _, first = np.unique(boxes(vals, L), axis=0, return_index=True)
    return np.sort(first)


def box_count(vals, L):
    return len(first_in_box(vals, L))


def thin(vals, capacity):
    """(indices kept, L): the earliest candidate of every occupied box at the
    resolution the binary search picks."""
    a, b = 1, min(capacity, MAX_LEVELS)
    while a < b:
        mid = (a + b + 1) // 2
        if box_count(vals, mid) <= capacity:
            a = mid
        else:
            b = mid - 1
    return list(first_in_box(vals, a)), a


def stayers(vals):
    """Mask of the candidates that no other candidate Pareto-dominates and
    that no earlier candidate equals (NumPy broadcasting over all pairs)."""
    v = np.asarray(vals, np.float64).reshape(-1, 3)
    n = len(v)
    if n == 0:
        return np.zeros(0, bool)
    le = np.all(v[:, None, :] <= v[None, :, :], axis=2)      # [y][x]: y no worse than x everywhere
    lt = np.any(v[:, None, :] < v[None, :, :], axis=2)       # [y][x]: y better somewhere
    eq = np.all(v[:, None, :] == v[None, :, :], axis=2)
    earlier = np.tril(np.ones((n, n), bool), k=-1).T          # [y][x]: y < x
    dominated = np.any(le & lt, axis=0)
    duplicate = np.any(eq & earlier, axis=0)
    return ~dominated & ~duplicate


def update(arc, offer_obj, offer_flags, offer_sev, guidance_max=math.inf):
    """Update the archive in place; returns inserted [n_offers] (uint8) and
    the slot of every inserted offer (-1 otherwise)."""
    n_off = len(offer_flags)
    cand = []                        # (objective vector, member slot or None, offer index or None)
    for s in arc.members():
        cand.append((arc.obj[s].astype(np.float64), s, None))
    for i in range(n_off):
        if feasible(offer_obj[i], offer_flags[i], offer_sev[i]):
            cand.append((np.asarray(offer_obj[i], np.float32).astype(np.float64), None, i))
    cand = [c for c in cand if not float(np.float32(c[0][2])) > guidance_max]
    mask = stayers([c[0] for c in cand])
    stay = [c for c, m in zip(cand, mask) if m]
    arc.levels = 0
    if len(stay) > arc.capacity:
        keep, arc.levels = thin([c[0] for c in stay], arc.capacity)
        stay = [stay[i] for i in keep]
    kept_slots = {c[1] for c in stay if c[1] is not None}
    for s in arc.members():
        if s not in kept_slots:
            arc.stamp[s] = -1
            arc.obj[s] = np.inf
    free = list(np.flatnonzero(arc.stamp < 0))
    inserted = np.zeros(n_off, np.uint8)
    slot_of = np.full(n_off, -1, np.int64)
    for c in stay:
        if c[2] is None:
            continue
        s = free.pop(0)
        arc.obj[s] = np.asarray(offer_obj[c[2]], np.float32)
        arc.stamp[s] = arc.next_stamp
        arc.next_stamp += 1
        inserted[c[2]] = 1
        slot_of[c[2]] = s
    return inserted, slot_of


def steering_bound(s_g):
    """fl32(1.5 s_G); inf for an empty archive."""
    if not math.isfinite(s_g):
        return math.inf
    return float(np.float32(1.5) * np.float32(s_g))


def mark_improvements(improved, eval_parent, eval_group, eval_cluster, accepted, parent_inserted):
    """Mark (cluster, element) improved [k][n_groups] (uint8, in place) for
    every kept child whose parent entered the archive in the same batch."""
    k, n_groups = improved.shape
    n_parents = len(parent_inserted)
    for e in range(len(accepted)):
        p, g, c = int(eval_parent[e]), int(eval_group[e]), int(eval_cluster[e])
        if accepted[e] and 0 <= p < n_parents and 0 <= g < n_groups and 0 <= c < k and parent_inserted[p]:
            improved[c, g] = 1


def adapt_multipliers(improved, mult, nis):
    """Adaptive variance scaling, reduced (see the module readings): FP32
    multipliers and no-improvement stretches updated in place; the marks are
    cleared."""
    f = np.float32
    for q in np.ndindex(mult.shape):
        c = f(mult[q])
        if improved[q]:
            nis[q] = 0
            c = min(f(max(c, f(1.0)) / f(0.9)), f(10.0))
        else:
            if c <= f(1.0):
                nis[q] += 1
            if c > f(1.0) or nis[q] >= 25:
                c = f(f(0.9) * c)
            elif c < f(1.0):
                c = f(1.0)
        mult[q] = c
        improved[q] = 0
