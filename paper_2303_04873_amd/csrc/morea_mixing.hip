// Distributions of optimal mixing (Sec. 3): for every FOS element in every
// cluster a normal distribution is estimated from the cluster's selected
// solutions, and new partial solutions are sampled from it for partial
// evaluation.
//
// Definitions where the paper leaves the distribution to MO-RV-GOMEA's
// literature:
//   variables of an element: for its k-th point, mesh m, axis a, index
//     (2 k + m) 3 + a (the row layout of a partial evaluation's new
//     coordinates); an axis pinned for a point is not a variable and keeps
//     the parent's value;
//   estimates: maximum likelihood over the members in the given order, mean
//     = (ascending sum) / m, covariance = (ascending sum of products of the
//     centred values) / m, FP64;
//   factor: Cholesky (every entry's sum in ascending index order); a pivot
//     not larger than 1e-12 times its diagonal entry makes it fail, and the
//     distribution falls back to the diagonal (standard deviations);
//   sample: x = mean + sqrt(c) (L z) in FP64 with the caller's standard
//     normal draws z and multiplier c, rounded once to FP32;
//   a cluster without members, or with a member or offset out of range, has
//     no distribution: its samples are NaN.
// Every FP64 operation is done one at a time in the stated order
// (contraction off), so results are fixed to the last bit.
//
// Estimation: one wave per (cluster, element): free variables by ballot,
// means on lanes, the lower triangle of the covariance on lanes, the factor
// column by column (pivot on one lane, the column below it on all lanes).
// Sampling: a prefix over the evaluations (first new-coordinate row of
// each), then one wave per evaluation, its variables on lanes.
#include <math.h>
#include <stdio.h>

#include "morea_internal.h"

namespace morea {
namespace mixing {

constexpr int kMaxVars = 24;                  // groups of at most 4 points
constexpr double kPivotRel = 1e-12;

// Distribution of one (cluster, element) in the caller's workspace.
struct Dist {
  double mean[kMaxVars];
  double L[kMaxVars * kMaxVars];              // lower triangle, row-major over free variables
  int var[kMaxVars];                          // free variables, ascending
  int n_free;
  int mode;                                   // 0 factor, 1 diagonal, 2 none
  int pad[2];
};
static_assert(sizeof(Dist) % 16 == 0, "distribution record alignment");

__device__ __forceinline__ unsigned long long lanes_below(int lane) {
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ double value(const float* pts, int n_points, int member, int pt, int ma) {
  return static_cast<double>(pts[(static_cast<size_t>(member) * 6 + ma) * n_points + pt]);
}

__global__ __launch_bounds__(kWave) void k_estimate(const float* __restrict__ pts, int n_pop, int n_points,
                                                    int n_groups, const int* __restrict__ grp_off,
                                                    const int* __restrict__ grp_pts,
                                                    const int* __restrict__ clu_off,
                                                    const int* __restrict__ clu_members, int n_members,
                                                    const uint8_t* __restrict__ pinned, Dist* __restrict__ out) {
#pragma clang fp contract(off)
  __shared__ double s_mean[kMaxVars];
  __shared__ double s_cov[kMaxVars * kMaxVars];
  __shared__ double s_L[kMaxVars * kMaxVars];
  __shared__ int s_var[kMaxVars];
  __shared__ int s_fail;
  const int g = blockIdx.x % n_groups, c = blockIdx.x / n_groups;
  const int lane = threadIdx.x;
  Dist& D = out[blockIdx.x];
  const int k0 = grp_off[g], np = grp_off[g + 1] - k0;
  // free variables
  bool free_v = false;
  if (lane < 6 * np) {
    const int pt = grp_pts[k0 + lane / 6];
    free_v = !(pinned && ((pinned[pt] >> (lane % 3)) & 1));
  }
  const unsigned long long fm = __ballot(free_v);
  const int n = __popcll(fm);
  if (free_v) s_var[__popcll(fm & lanes_below(lane))] = lane;
  for (int i = lane; i < kMaxVars * kMaxVars; i += kWave) {
    s_L[i] = 0.0;
    s_cov[i] = 0.0;
  }
  if (lane == 0) s_fail = 0;
  __syncthreads();
  // members
  const int lo = clu_off[c], hi = clu_off[c + 1];
  bool bad = !(lo >= 0 && lo < hi && hi <= n_members);
  if (!bad)
    for (int i = lo + lane; i < hi; i += kWave) {
      const int mem = clu_members[i];
      if (mem < 0 || mem >= n_pop) bad = true;
    }
  bad = __ballot(bad) != 0;
  if (lane < kMaxVars) D.var[lane] = lane < n ? s_var[lane] : -1;
  if (lane == 0) D.n_free = n;
  if (bad) {
    for (int i = lane; i < kMaxVars * kMaxVars; i += kWave) D.L[i] = 0.0;
    if (lane < kMaxVars) D.mean[lane] = NAN;
    if (lane == 0) D.mode = 2;
    return;
  }
  const int m = hi - lo;
  const double dm = static_cast<double>(m);
  // means
  if (lane < n) {
    const int v = s_var[lane];
    const int pt = grp_pts[k0 + v / 6], ma = v % 6;
    double s = 0.0;
    for (int i = lo; i < hi; i++) s = s + value(pts, n_points, clu_members[i], pt, ma);
    s_mean[lane] = s / dm;
  }
  __syncthreads();
  // covariance, lower triangle: entry t -> (u, v), v <= u
  for (int t = lane; t < n * (n + 1) / 2; t += kWave) {
    int u = 0;
    while ((u + 1) * (u + 2) / 2 <= t) u++;
    const int v = t - u * (u + 1) / 2;
    const int vu = s_var[u], vv = s_var[v];
    const int pu = grp_pts[k0 + vu / 6], mu = vu % 6, pv = grp_pts[k0 + vv / 6], mv = vv % 6;
    const double au = s_mean[u], av = s_mean[v];
    double s = 0.0;
    for (int i = lo; i < hi; i++) {
      const int mem = clu_members[i];
      const double du = value(pts, n_points, mem, pu, mu) - au;
      const double dv = value(pts, n_points, mem, pv, mv) - av;
      const double pr = du * dv;
      s = s + pr;
    }
    s_cov[u * kMaxVars + v] = s / dm;
  }
  __syncthreads();
  // factor, column by column; every entry's sum runs over ascending k
  for (int j = 0; j < n; j++) {
    if (lane == 0) {
      double s = s_cov[j * kMaxVars + j];
      for (int k = 0; k < j; k++) {
        const double pr = s_L[j * kMaxVars + k] * s_L[j * kMaxVars + k];
        s = s - pr;
      }
      const double lim = kPivotRel * s_cov[j * kMaxVars + j];
      if (!(s > lim))
        s_fail = 1;
      else
        s_L[j * kMaxVars + j] = sqrt(s);
    }
    __syncthreads();
    if (s_fail) break;
    const double piv = s_L[j * kMaxVars + j];
    for (int i = j + 1 + lane; i < n; i += kWave) {
      double s = s_cov[i * kMaxVars + j];
      for (int k = 0; k < j; k++) {
        const double pr = s_L[i * kMaxVars + k] * s_L[j * kMaxVars + k];
        s = s - pr;
      }
      s_L[i * kMaxVars + j] = s / piv;
    }
    __syncthreads();
  }
  const bool fail = s_fail != 0;
  for (int i = lane; i < kMaxVars * kMaxVars; i += kWave) {
    const int r = i / kMaxVars, q = i % kMaxVars;
    double x = 0.0;
    if (r < n && q <= r) x = fail ? (r == q ? sqrt(s_cov[r * kMaxVars + r]) : 0.0) : s_L[i];
    D.L[i] = x;
  }
  if (lane < kMaxVars) D.mean[lane] = lane < n ? s_mean[lane] : 0.0;
  if (lane == 0) D.mode = fail ? 1 : 0;
}

// First new-coordinate row of every evaluation: evaluations with a valid
// group own |group| rows.  Per-block scans of 256 evaluations (block totals
// after the row offsets in the workspace), one block scanning the totals,
// then the block offsets added back.
constexpr int kRowBlock = 256;

__global__ __launch_bounds__(kRowBlock) void k_rows_local(int n_evals, int n_groups,
                                                          const int* __restrict__ eval_group,
                                                          const int* __restrict__ grp_off, int* __restrict__ row_off,
                                                          int* __restrict__ bsum) {
  __shared__ int s_rows[kRowBlock];
  const int tid = threadIdx.x, e = blockIdx.x * kRowBlock + tid;
  int rows = 0;
  if (e < n_evals) {
    const int g = eval_group[e];
    if (g >= 0 && g < n_groups) rows = grp_off[g + 1] - grp_off[g];
  }
  s_rows[tid] = rows;
  __syncthreads();
  for (int d = 1; d < kRowBlock; d <<= 1) {
    const int r = tid >= d ? s_rows[tid - d] : 0;
    __syncthreads();
    s_rows[tid] += r;
    __syncthreads();
  }
  if (e < n_evals) row_off[e] = s_rows[tid] - rows;
  if (tid == kRowBlock - 1) bsum[blockIdx.x] = s_rows[tid];
}

__global__ __launch_bounds__(1024) void k_rows_blocks(int n_blocks, int* __restrict__ bsum) {
  __shared__ int s_rows[1024];
  const int tid = threadIdx.x;
  int carry = 0;
  for (int b0 = 0; b0 < n_blocks; b0 += 1024) {
    const int b = b0 + tid;
    const int r = b < n_blocks ? bsum[b] : 0;
    s_rows[tid] = r;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
      const int x = tid >= d ? s_rows[tid - d] : 0;
      __syncthreads();
      s_rows[tid] += x;
      __syncthreads();
    }
    if (b < n_blocks) bsum[b] = carry + s_rows[tid] - r;
    carry += s_rows[1023];
    __syncthreads();
  }
}

__global__ __launch_bounds__(kRowBlock) void k_rows_add(int n_evals, int* __restrict__ row_off,
                                                        const int* __restrict__ bsum) {
  const int e = blockIdx.x * kRowBlock + threadIdx.x;
  if (e < n_evals) row_off[e] += bsum[blockIdx.x];
}

__global__ __launch_bounds__(256) void k_sample(const float* __restrict__ pts, int n_pop, int n_points,
                                                int n_groups, int n_clusters, const int* __restrict__ grp_off,
                                                const int* __restrict__ grp_pts, const Dist* __restrict__ dist,
                                                const float* __restrict__ mult, int n_evals,
                                                const int* __restrict__ eval_parent,
                                                const int* __restrict__ eval_group,
                                                const int* __restrict__ eval_cluster,
                                                const int* __restrict__ row_off, const float* __restrict__ z,
                                                const uint8_t* __restrict__ pinned,
                                                float* __restrict__ new_coords) {
#pragma clang fp contract(off)
  const int e = blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (e >= n_evals) return;
  const int g = eval_group[e];
  if (g < 0 || g >= n_groups) return;
  const int k0 = grp_off[g], np = grp_off[g + 1] - k0;
  const size_t base = static_cast<size_t>(row_off[e]) * 6;
  const int par = eval_parent[e], c = eval_cluster[e];
  const bool valid = par >= 0 && par < n_pop && c >= 0 && c < n_clusters;
  bool free_v = false;
  int pt = 0;
  if (lane < 6 * np) {
    pt = grp_pts[k0 + lane / 6];
    free_v = !(pinned && ((pinned[pt] >> (lane % 3)) & 1));
  }
  const unsigned long long fm = __ballot(free_v);
  if (lane >= 6 * np) return;
  if (!valid) {
    new_coords[base + lane] = NAN;
    return;
  }
  if (!free_v) {
    new_coords[base + lane] = pts[(static_cast<size_t>(par) * 6 + lane % 6) * n_points + pt];
    return;
  }
  const Dist& D = dist[static_cast<size_t>(c) * n_groups + g];
  if (D.mode == 2) {
    new_coords[base + lane] = NAN;
    return;
  }
  const int u = __popcll(fm & lanes_below(lane));
  const double scale = sqrt(static_cast<double>(mult ? mult[static_cast<size_t>(c) * n_groups + g] : 1.0f));
  double t = 0.0;
  for (int k = 0; k <= u; k++) {
    const double pr = D.L[u * kMaxVars + k] * static_cast<double>(z[base + D.var[k]]);
    t = t + pr;
  }
  const double st = scale * t;
  new_coords[base + lane] = static_cast<float>(D.mean[u] + st);
}

size_t dist_bytes(const morea_problem* p, int n_clusters) {
  return static_cast<size_t>(n_clusters) * p->n_groups * sizeof(Dist);
}

}  // namespace mixing
}  // namespace morea

using namespace morea;

namespace {

morea_status mix_fail(morea_status code, const char* msg) {
  set_error(msg);
  return code;
}

morea_status mix_launch_status(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess) return MOREA_OK;
  char buf[256];
  snprintf(buf, sizeof(buf), "%s: %s", what, hipGetErrorString(e));
  set_error(buf);
  return MOREA_EDEVICE;
}

}  // namespace

extern "C" size_t morea_mixing_bytes(const morea_problem* p, int32_t n_clusters) {
  if (!p || n_clusters < 1 || p->n_groups == 0 || p->max_evals == 0) return 0;
  // distributions, row offsets, block totals of the row scan
  return mixing::dist_bytes(p, n_clusters) +
         (static_cast<size_t>(p->max_evals) + p->max_evals / mixing::kRowBlock + 1) * sizeof(int);
}

extern "C" morea_status morea_estimate_distributions(morea_problem* p, const float* pts, int32_t n_pop,
                                                     int32_t n_clusters, const int32_t* clu_off,
                                                     const int32_t* clu_members, int32_t n_members,
                                                     const uint8_t* pinned, void* work, size_t work_bytes,
                                                     void* stream) {
  if (!p) return mix_fail(MOREA_EINVAL, "problem is NULL");
  if (p->n_groups == 0 || p->max_evals == 0)
    return mix_fail(MOREA_ESTATE, "call morea_set_groups and morea_reserve_partial first");
  if (n_pop < 1 || n_clusters < 1 || n_members < 0) return mix_fail(MOREA_EINVAL, "bad n_pop / n_clusters / n_members");
  if (!pts || !clu_off || (n_members > 0 && !clu_members) || !work) return mix_fail(MOREA_EINVAL, "NULL argument");
  if (p->max_group > 4) return mix_fail(MOREA_ERANGE, "distributions need groups of at most 4 points");
  if (work_bytes < morea_mixing_bytes(p, n_clusters)) return mix_fail(MOREA_ERANGE, "workspace too small");
  if (reinterpret_cast<uintptr_t>(work) % 16 != 0) return mix_fail(MOREA_EINVAL, "workspace must be 16-byte aligned");
  if (static_cast<int64_t>(n_clusters) * p->n_groups > (1 << 30)) return mix_fail(MOREA_ERANGE, "too many pairs");
  {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mix_fail(MOREA_EDEVICE, hipGetErrorString(e));
  }
  hipLaunchKernelGGL(mixing::k_estimate, dim3(n_clusters * p->n_groups), dim3(kWave), 0,
                     static_cast<hipStream_t>(stream), pts, n_pop, p->view.n_points, p->n_groups, p->d_grp_off,
                     p->d_grp_pts, clu_off, clu_members, n_members, pinned, static_cast<mixing::Dist*>(work));
  return mix_launch_status("distribution estimation");
}

extern "C" morea_status morea_sample_partial(morea_problem* p, const float* pts, int32_t n_pop, void* work,
                                             size_t work_bytes, int32_t n_clusters, const float* mult,
                                             int32_t n_evals, const int32_t* eval_parent, const int32_t* eval_group,
                                             const int32_t* eval_cluster, const float* z, const uint8_t* pinned,
                                             float* new_coords, void* stream) {
  if (!p) return mix_fail(MOREA_EINVAL, "problem is NULL");
  if (p->n_groups == 0 || p->max_evals == 0)
    return mix_fail(MOREA_ESTATE, "call morea_set_groups and morea_reserve_partial first");
  if (n_pop < 1 || n_clusters < 1 || n_evals < 0) return mix_fail(MOREA_EINVAL, "bad n_pop / n_clusters / n_evals");
  if (n_evals > p->max_evals) return mix_fail(MOREA_ERANGE, "n_evals beyond the reservation");
  if (n_evals == 0) return MOREA_OK;
  if (!pts || !work || !eval_parent || !eval_group || !eval_cluster || !z || !new_coords)
    return mix_fail(MOREA_EINVAL, "NULL argument");
  if (p->max_group > 4) return mix_fail(MOREA_ERANGE, "distributions need groups of at most 4 points");
  if (work_bytes < morea_mixing_bytes(p, n_clusters)) return mix_fail(MOREA_ERANGE, "workspace too small");
  if (reinterpret_cast<uintptr_t>(work) % 16 != 0) return mix_fail(MOREA_EINVAL, "workspace must be 16-byte aligned");
  {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mix_fail(MOREA_EDEVICE, hipGetErrorString(e));
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const mixing::Dist* dist = static_cast<const mixing::Dist*>(work);
  int* row_off = reinterpret_cast<int*>(static_cast<char*>(work) + mixing::dist_bytes(p, n_clusters));
  int* bsum = row_off + p->max_evals;
  const int row_blocks = (n_evals + mixing::kRowBlock - 1) / mixing::kRowBlock;
  hipLaunchKernelGGL(mixing::k_rows_local, dim3(row_blocks), dim3(mixing::kRowBlock), 0, s, n_evals, p->n_groups,
                     eval_group, p->d_grp_off, row_off, bsum);
  hipLaunchKernelGGL(mixing::k_rows_blocks, dim3(1), dim3(1024), 0, s, row_blocks, bsum);
  hipLaunchKernelGGL(mixing::k_rows_add, dim3(row_blocks), dim3(mixing::kRowBlock), 0, s, n_evals, row_off, bsum);
  morea_status st = mix_launch_status("sampling rows");
  if (st != MOREA_OK) return st;
  constexpr int per_block = 256 / kWave;
  hipLaunchKernelGGL(mixing::k_sample, dim3((n_evals + per_block - 1) / per_block), dim3(256), 0, s, pts, n_pop,
                     p->view.n_points, p->n_groups, n_clusters, p->d_grp_off, p->d_grp_pts, dist, mult, n_evals,
                     eval_parent, eval_group, eval_cluster, row_off, z, pinned, new_coords);
  return mix_launch_status("sampling");
}
