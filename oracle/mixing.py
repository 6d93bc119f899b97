"""Distributions of optimal mixing -- plain reference, test infrastructure only
(not part of the library's path).

Sec. 3: for each FOS element in each cluster a distribution is estimated from
the cluster's selected solutions, and new partial solutions are sampled from
it.  The paper leaves the distribution to MO-RV-GOMEA's literature, which
uses a normal distribution; the readings (listed in the design notes):
  * variables of an element: for its k-th point, mesh m, axis a, index
    (2 k + m) 3 + a -- the layout of a partial evaluation's new coordinates;
    an axis pinned for a point (bit a of pinned[point]) is not a variable of
    the distribution and keeps the parent's value;
  * maximum-likelihood estimates over the cluster's members in the order
    given: mean = (sum of the values, ascending member order) / m;
    covariance = (sum of products of the centred values) / m;
  * factor: Cholesky-Banachiewicz, row by row, every sum in ascending index
    order; it fails when a pivot is not larger than 1e-12 times its diagonal
    entry, and the distribution then falls back to the diagonal (standard
    deviations sqrt(cov[v][v]));
  * sample: x = mean + sqrt(c) (L z), z the caller's standard normal draws, c
    the distribution multiplier, in FP64, rounded once to FP32;
  * a cluster without members, or with a member index or offsets out of
    range, gives no distribution: its samples are NaN.
All arithmetic is FP64 on Python floats, one operation at a time, in the
order stated, so that the result is fixed to the last bit.
"""
import math

import numpy as np

PIVOT_REL = 1e-12


def free_variables(group_pts, pinned):
    """Indices (2 k + m) 3 + a of the element's free variables, ascending."""
    out = []
    for k, pt in enumerate(group_pts):
        for m in range(2):
            for a in range(3):
                if pinned is None or not (int(pinned[pt]) >> a) & 1:
                    out.append((2 * k + m) * 3 + a)
    return out


def values(pts, member, group_pts, v):
    k, r = divmod(v, 6)
    m, a = divmod(r, 3)
    return float(pts[member][m][a][group_pts[k]])


def estimate(pts, members, group_pts, pinned):
    """(free, mean, L, mode) of one (cluster, element); mode 0 Cholesky,
    1 diagonal fallback, 2 no members."""
    free = free_variables(group_pts, pinned)
    n = len(free)
    if len(members) == 0 or any(not 0 <= i < pts.shape[0] for i in members):
        return free, [math.nan] * n, [[0.0] * n for _ in range(n)], 2
    x = [[values(pts, i, group_pts, v) for v in free] for i in members]
    m = len(members)
    mean = []
    for u in range(n):
        s = 0.0
        for row in x:
            s = s + row[u]
        mean.append(s / m)
    cov = [[0.0] * n for _ in range(n)]
    for u in range(n):
        for v in range(u + 1):
            s = 0.0
            for row in x:
                s = s + (row[u] - mean[u]) * (row[v] - mean[v])
            cov[u][v] = cov[v][u] = s / m
    L = [[0.0] * n for _ in range(n)]
    ok = True
    for i in range(n):
        for j in range(i + 1):
            s = cov[i][j]
            for k in range(j):
                s = s - L[i][k] * L[j][k]
            if i == j:
                if not s > PIVOT_REL * cov[i][i]:
                    ok = False
                    break
                L[i][i] = math.sqrt(s)
            else:
                L[i][j] = s / L[j][j]
        if not ok:
            break
    if not ok:
        L = [[0.0] * n for _ in range(n)]
        for i in range(n):
            L[i][i] = math.sqrt(cov[i][i])
        return free, mean, L, 1
    return free, mean, L, 0


def sample(dist, z_row, mult, parent_vals):
    """New values (FP32) of all 6 |group| variables: z_row and parent_vals are
    indexed by variable; pinned variables keep the parent's value."""
    free, mean, L, mode = dist
    out = [np.float32(v) for v in parent_vals]
    scale = math.sqrt(float(np.float32(mult)))
    for u, var in enumerate(free):
        if mode == 2:
            out[var] = np.float32(math.nan)
            continue
        t = 0.0
        for k in range(u + 1):
            t = t + L[u][k] * float(z_row[free[k]])
        out[var] = np.float32(mean[u] + scale * t)
    return out


def sample_batch(pts, clu_off, clu_members, grp_off, grp_pts, pinned, mult, eval_parent, eval_group,
                 eval_cluster, z):
    """New coordinates [rows][2][3] FP32 of every evaluation: evaluations with
    a valid group own |group| rows in order; an out-of-range parent or
    cluster gives NaN rows.  mult: [n_clusters][n_groups] or None (1)."""
    n_groups = len(grp_off) - 1
    n_clusters = len(clu_off) - 1
    n_pop = pts.shape[0]
    cache = {}
    rows = []
    for e in range(len(eval_group)):
        g = int(eval_group[e])
        if not 0 <= g < n_groups:
            continue
        gp = [int(v) for v in grp_pts[grp_off[g]:grp_off[g + 1]]]
        r0 = len(rows)
        zr = np.asarray(z[r0:r0 + len(gp)], np.float32).reshape(-1)
        p, c = int(eval_parent[e]), int(eval_cluster[e])
        if not (0 <= p < n_pop and 0 <= c < n_clusters):
            rows.extend(np.full((len(gp), 2, 3), np.nan, np.float32))
            continue
        if (c, g) not in cache:
            lo, hi = int(clu_off[c]), int(clu_off[c + 1])
            members = [int(i) for i in clu_members[lo:hi]] if 0 <= lo <= hi <= len(clu_members) else [-1]
            cache[(c, g)] = estimate(pts, members, gp, pinned)
        par = [values(pts, p, gp, v) for v in range(6 * len(gp))]
        cm = 1.0 if mult is None else mult[c][g]
        new = sample(cache[(c, g)], zr, cm, par)
        rows.extend(np.array(new, np.float32).reshape(len(gp), 2, 3))
    return np.array(rows, np.float32).reshape(-1, 2, 3)
