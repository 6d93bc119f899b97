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

Training target of (candidate, tet): the tet's mean intensity term per
sample over both directions, (h_S + h_T) / (n_S + n_T) from the full
evaluation's per-tet records (Sec. 4.1.2's objective restricted to one tet);
0 when the tet holds no sample.
"""
import numpy as np

from . import tet_voxels


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


def targets(records):
    """Per-(candidate, tet) targets [pop][n_tets] from the oracle's records
    [pop][n_tets][2][>=3] (h sum at 0, samples at 2)."""
    rec = np.asarray(records, np.float64)
    h = rec[..., 0, 0] + rec[..., 1, 0]
    n = rec[..., 0, 2] + rec[..., 1, 2]
    return np.where(n > 0, h / np.maximum(n, 1.0), 0.0)
