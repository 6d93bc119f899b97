"""FP64 reference of the surrogate's inputs and training targets -- test
infrastructure (only the tests import it).

The learned pre-screen is this build's own addition: the paper has no
counterpart, so no passage defines these quantities; they are defined here in
plain terms and the GPU kernels are checked against these definitions.

Region statistics, per reference tetrahedron: the voxel centres inside the
tet of the reference mesh (the same tie rule as the objectives' rasterizer,
Sec. 4.1.2 read with exact predicates) index both images at the same grid
positions, and eight numbers describe them:
    0 mean of I_s           1 standard deviation of I_s (population form)
    2 fraction with I_s > 0 3 mean of I_t
    4 std. dev. of I_t      5 fraction with I_t > 0
    6 mean of (I_s - I_t)^2 7 voxel count x n_tets / V (1 on average)
An empty tet gives zeros.

Mean term of (candidate, tet): the tet's mean intensity term per sample over
both directions, (h_S + h_T) / (n_S + n_T) from the full evaluation's per-tet
records (Sec. 4.1.2's objective restricted to one tet); 0 when the tet holds
no sample.  h_scale: the mean of (I_s - I_t)^2 over the grid's voxels (1 when
that is 0).  The training target of (offspring, tet) is the offspring's mean
term minus its parent's, divided by h_scale.

Input row of (offspring, tet), 23 values:
    0..11  the moves of the tet's 4 target-mesh vertices from the parent's,
           (T_v - T_parent,v) / 0.5 voxel, vertex-major
    12..14 the mean of h = (I_s(x) - I_t(y))^2 over a point set of the tet,
           x = S l and y = T l for barycentric coordinates l, in the
           offspring minus that in the parent, over h_scale; the sets: the 4
           vertices, the 6 edge midpoints, 16 interior points (Halton points
           j = 1..16 in bases 2, 3, 5, sorted into a <= b <= c, taken as
           (a, b - a, c - b, 1 - c))
    15..20 region statistics 0..5
    21     region statistic 6 over h_scale
    22     the parent's mean term of the tet over h_scale
each image value the trilinear interpolant at the point clamped into the
image box (oracle.trilinear with clamping).  An offspring without a valid
parent has a row of NaN.

Score of an offspring given per-tet predictions y (in units of h_scale):
sum_t w_t (parent's mean term + h_scale y_t) / sum_t w_t, with w_t the
offspring's |volume| of tet t in the source mesh plus that in the target
mesh (voxel^3).
"""
import numpy as np

from . import tet_voxels, trilinear


def region_stats(problem):
    """stats [n_tets][8] FP64 and counts [n_tets] of the reference mesh's
    tets over the problem's two images (as stored: pass quantized images for
    a reduced-precision problem)."""
    nx, ny, nz = problem.dims
    V = nx * ny * nz
    Is = problem.image_src.reshape(-1).astype(np.float64)
    It = problem.image_tgt.reshape(-1).astype(np.float64)
    ref = problem.ref_points
    out = np.zeros((problem.n_tets, 8), np.float64)
    cnt = np.zeros(problem.n_tets, np.int64)
    for t, tet in enumerate(problem.tets):
        vox = tet_voxels(ref[tet], problem.dims)
        n = vox.size
        cnt[t] = n
        if n == 0:
            continue
        a, b = Is[vox], It[vox]
        out[t] = [a.mean(), a.std(), np.mean(a > 0), b.mean(), b.std(), np.mean(b > 0),
                  np.mean((a - b) ** 2), n * problem.n_tets / V]
    return out, cnt


def mean_terms(records):
    """Per-(candidate, tet) mean terms [pop][n_tets] from the oracle's
    records [pop][n_tets][2][>=3] (h sum at 0, samples at 2)."""
    rec = np.asarray(records, np.float64)
    h = rec[..., 0, 0] + rec[..., 1, 0]
    n = rec[..., 0, 2] + rec[..., 1, 2]
    return np.where(n > 0, h / np.maximum(n, 1.0), 0.0)


def h_scale(problem):
    """The mean of (I_s - I_t)^2 over the grid's voxels, 1 when it is 0."""
    d = problem.image_src.astype(np.float64) - problem.image_tgt.astype(np.float64)
    v = float(np.mean(d * d))
    return v if v > 0 else 1.0


def radical_inverse(j, b):
    r, f = 0.0, 1.0 / b
    while j > 0:
        r += f * (j % b)
        j //= b
        f /= b
    return r


def point_sets():
    """Barycentric coordinates [26][4]: 4 vertices, 6 edge midpoints, 16
    interior Halton points."""
    pts = [np.eye(4)[v] for v in range(4)]
    for a in range(4):
        for b in range(a + 1, 4):
            l = np.zeros(4)
            l[a] = l[b] = 0.5
            pts.append(l)
    for j in range(1, 17):
        u = sorted(radical_inverse(j, b) for b in (2, 3, 5))
        pts.append(np.array([u[0], u[1] - u[0], u[2] - u[1], 1.0 - u[2]]))
    return np.array(pts)


def point_means(problem, cand):
    """Means of h over the three point sets of every tet [n_tets][3] of one
    candidate [2][3][P]."""
    L = point_sets()
    S = np.asarray(cand[0], np.float64).T[problem.tets]                # [n_tets][4][3]
    T = np.asarray(cand[1], np.float64).T[problem.tets]
    out = np.zeros((len(problem.tets), 3))
    for t in range(len(problem.tets)):
        h = np.empty(len(L))
        for j, l in enumerate(L):
            d = trilinear(problem.image_src, l @ S[t], clamp=True) - trilinear(problem.image_tgt, l @ T[t], clamp=True)
            h[j] = d * d
        out[t] = [h[:4].mean(), h[4:10].mean(), h[10:].mean()]
    return out


def targets(records, parent_records, parent_of, scale):
    """Targets [pop][n_tets]: each offspring's mean terms minus those of its
    parent parent_records[parent_of[k]], over `scale` (h_scale); NaN rows
    for an invalid parent."""
    t = mean_terms(records)
    tp = mean_terms(parent_records)
    out = np.full_like(t, np.nan)
    for k, q in enumerate(parent_of):
        if 0 <= q < len(tp):
            out[k] = (t[k] - tp[q]) / scale
    return out


def features(problem, stats, pts, parent_pts, parent_records, parent_of):
    """Input rows [pop][n_tets][23] FP64 of offspring `pts` [pop][2][3][P]
    with parents `parent_pts` [n][2][3][P] whose records are
    `parent_records`; `stats` from region_stats."""
    tets = problem.tets
    hs = h_scale(problem)
    T = np.asarray(pts, np.float64)[:, 1].transpose(0, 2, 1)            # [pop][P][3]
    Tp = np.asarray(parent_pts, np.float64)[:, 1].transpose(0, 2, 1)
    tp = mean_terms(parent_records)
    out = np.full((len(T), len(tets), 23), np.nan)
    pm = {}
    for k, q in enumerate(parent_of):
        if not 0 <= q < len(Tp):
            continue
        if q not in pm:
            pm[q] = point_means(problem, parent_pts[q])
        out[k, :, :12] = ((T[k][tets] - Tp[q][tets]) * 2.0).reshape(len(tets), 12)
        out[k, :, 12:15] = (point_means(problem, pts[k]) - pm[q]) / hs
        out[k, :, 15:21] = stats[:, :6]
        out[k, :, 21] = stats[:, 6] / hs
        out[k, :, 22] = tp[q] / hs
    return out


def weights(problem, cand):
    """|volume| of every tet in the source plus in the target mesh [n_tets]
    of one candidate [2][3][P] (voxel^3)."""
    w = np.zeros(len(problem.tets))
    for m in range(2):
        v = np.asarray(cand[m], np.float64).T[problem.tets]
        e = v[:, 1:] - v[:, :1]
        w += np.abs(np.linalg.det(e)) / 6.0
    return w


def score(problem, pts, parent_records, parent_of, pred):
    """Scores [pop] of offspring from per-tet predictions pred [pop][n_tets]
    (units of h_scale); +inf without a valid parent."""
    hs = h_scale(problem)
    tp = mean_terms(parent_records)
    out = np.full(len(pts), np.inf)
    for k, q in enumerate(parent_of):
        if 0 <= q < len(tp):
            w = weights(problem, pts[k])
            out[k] = (w * (tp[q] + hs * pred[k])).sum() / w.sum()
    return out
