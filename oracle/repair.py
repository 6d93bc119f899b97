"""Fold repair of infeasible candidates -- plain reference, test
infrastructure only (imported by the tests and the benchmark's checks, never
by the product path).  Written from Sec. 4.3.1 of the paper: for each point of
a folded tetrahedron, 64 Gaussian trial moves scaled by the point's estimated
distance to its surrounding polygon; the trial with the best constraint
improvement is applied if there is one, and the repair of the candidate stops
when every trial is worse.  Folds are those of App. A.4 (a signed volume whose
sign differs from the reference mesh's, or zero).

Readings where the passage leaves details open (each listed in the design
notes):
  - coordinates are snapped to 2^-10 voxel as for the evaluation; a move is
    made on that grid, so the constraint is exact integer arithmetic;
  - the constraint of a visited point is the pair (number of folded tets among
    the point's incident tets in its mesh, sum of their |6V|), compared
    lexicographically (so zero-volume folds count);
  - the points visited are the vertices of the tets folded at the start, mesh
    S then mesh T, each in ascending index; a point whose incident tets are no
    longer folded when its turn comes is skipped without using a draw;
  - the surrounding polygon of a point is formed by its neighbours (the
    other vertices of its incident tets, each counted once); its distance to
    it is estimated as the distance from the point to their centroid, rounded
    down to a power of two of grid units (at least 1, at most 2^18):
    sigma = 2^j for the largest j with 4^j n^2 <= |n v - sum_u u|^2, n the
    number of neighbours (exact integers);
  - trial k of visit i moves each free axis by rint(sigma * z[i][k][axis]) grid
    units (ties to even), z the caller's standard normal draws; axes the
    caller pins do not move; a trial that leaves |x| < 512 voxels is never
    chosen;
  - the best trial is the smallest (constraint, k); it is applied when its
    constraint is strictly smaller than the current one; when it equals the
    current one (no trial improves, not all deteriorate, e.g. a point whose
    axes are all pinned) the point is left as it is and the next one visited;
    when every trial is worse, or leaves the coordinate range, the repair of
    the candidate stops ("aborted"); at most K visits (the draws given).

Outcome codes per candidate: 0 no fold at the start, 1 every listed point
visited, 2 aborted, 3 the K draws used up, 4 invalid coordinates (untouched).
"""
import numpy as np

FIX = 1024
LIMIT = 512 * FIX            # |x_fix| < 2^19, as for the evaluation
SIGMA_MAX_LOG2 = 18

NO_FOLD, DONE, ABORTED, OUT_OF_DRAWS, INVALID = 0, 1, 2, 3, 4


def snap(x):
    """rint(x * 1024), ties to even, as a Python int."""
    return int(np.rint(np.float64(x) * 1024.0))


def det6(a, b, c, d):
    """6 x signed volume of four integer points (exact)."""
    u = [b[i] - a[i] for i in range(3)]
    v = [c[i] - a[i] for i in range(3)]
    w = [d[i] - a[i] for i in range(3)]
    return (u[0] * (v[1] * w[2] - v[2] * w[1]) - u[1] * (v[0] * w[2] - v[2] * w[0]) +
            u[2] * (v[0] * w[1] - v[1] * w[0]))


def is_fold(D, ref):
    return D == 0 or (D > 0) != (ref > 0)


def incidence(tets, n_points):
    """For each point, the (tet, slot) pairs of the tets it belongs to."""
    inc = [[] for _ in range(n_points)]
    for t, tv in enumerate(tets):
        for s in range(4):
            inc[int(tv[s])].append((t, s))
    return inc


def constraint(X, tets, refs, inc_v, v, pos):
    """(folded incident tets, sum of their |6V|) with point v at pos."""
    cnt, sev = 0, 0
    for t, s in inc_v:
        P = [pos if k == s else X[int(tets[t][k])] for k in range(4)]
        D = det6(*P)
        if is_fold(D, refs[t]):
            cnt += 1
            sev += abs(D)
    return cnt, sev


def sigma(X, tets, inc_v, v):
    """Power-of-two estimate of v's distance to its surrounding polygon: the
    distance to the centroid of its neighbours."""
    nb = sorted({int(tets[t][k]) for t, s in inc_v for k in range(4) if k != s})
    if not nb:
        return 1
    n = len(nb)
    D = [n * X[v][i] - sum(X[u][i] for u in nb) for i in range(3)]
    d2 = D[0] * D[0] + D[1] * D[1] + D[2] * D[2]
    j = 0
    while j < SIGMA_MAX_LOG2 and (4 ** (j + 1)) * n * n <= d2:
        j += 1
    return 1 << j


def repair_one(tets, refs, inc, cand, noise, fixed):
    """Repair one candidate cand [2][3][P] (float32); returns (new cand,
    moves, outcome, log of visits)."""
    P = cand.shape[2]
    out = cand.copy()
    if not np.all(np.abs(cand.astype(np.float64)) < 512.0):
        return out, 0, INVALID, []
    X = [[[snap(cand[m, a, v]) for a in range(3)] for v in range(P)] for m in range(2)]
    todo = []
    for m in range(2):
        pts = set()
        for t, tv in enumerate(tets):
            if is_fold(det6(*[X[m][int(i)] for i in tv]), refs[t]):
                pts.update(int(i) for i in tv)
        todo += [(m, v) for v in sorted(pts)]
    if not todo:
        return out, 0, NO_FOLD, []
    K = noise.shape[0]
    visit, moves, outcome, log = 0, 0, DONE, []
    for m, v in todo:
        c0 = constraint(X[m], tets, refs, inc[v], v, X[m][v])
        if c0[0] == 0:
            continue
        if visit == K:
            outcome = OUT_OF_DRAWS
            break
        sg = sigma(X[m], tets, inc[v], v)
        best = None
        for k in range(noise.shape[1]):
            pos = list(X[m][v])
            for a in range(3):
                if not (fixed is not None and (int(fixed[v]) >> a) & 1):
                    pos[a] += int(np.rint(float(sg) * float(noise[visit, k, a])))
            if any(abs(x) >= LIMIT for x in pos):
                continue
            ck = constraint(X[m], tets, refs, inc[v], v, pos)
            if best is None or ck < best[0]:
                best = (ck, k, pos)
        visit += 1
        if best is not None and best[0] < c0:
            X[m][v] = best[2]
            for a in range(3):
                out[m, a, v] = np.float32(best[2][a] / FIX)
            moves += 1
            log.append((m, v, sg, c0, best[0], best[1]))
        elif best is not None and best[0] == c0:
            log.append((m, v, sg, c0, best[0], None))
        else:
            log.append((m, v, sg, c0, None if best is None else best[0], None))
            outcome = ABORTED
            break
    return out, moves, outcome, log


def repair(tets, ref_points, pts, noise, fixed=None):
    """Repair candidates pts [pop][2][3][P] float32 with draws noise
    [pop][K][64][3] float32 and an optional per-point mask of pinned axes
    (bit a: axis a).  Returns (new pts, moves [pop], outcome [pop], logs)."""
    tets = np.asarray(tets)
    ref = np.asarray(ref_points, np.float32)
    P = ref.shape[0]
    R = [[snap(ref[v, a]) for a in range(3)] for v in range(P)]
    refs = [det6(*[R[int(i)] for i in tv]) for tv in tets]
    inc = incidence(tets, P)
    pts = np.asarray(pts, np.float32)
    out = pts.copy()
    moves = np.zeros(len(pts), np.int32)
    outcome = np.zeros(len(pts), np.int32)
    logs = []
    for c in range(len(pts)):
        out[c], moves[c], outcome[c], lg = repair_one(tets, refs, inc, pts[c], np.asarray(noise[c], np.float32),
                                                       fixed)
        logs.append(lg)
    return out, moves, outcome, logs
