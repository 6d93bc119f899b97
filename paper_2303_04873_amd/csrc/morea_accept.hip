// Acceptance of partial solutions in optimal mixing (Sec. 3): a sampled
// partial solution, inserted into its parent, is kept when the result
// dominates the parent or is not dominated within the current elitist
// archive.  Kept children are written into their parents: the group's new
// coordinates into the parent's points, the dependent tets' records of the
// partial evaluation into the parent's cache, and the parent's totals and
// objectives recomputed from the cache.
//
// Definitions where the paper leaves the details to MO-RV-GOMEA's
// literature (all three objectives are minimised):
//   feasible: flags == 0 in the fold and invalid bits; violation = severity
//     (summed |signed volume| of the violating tets) when a fold bit is set,
//     +inf when the invalid bit is set or an objective or the severity is not
//     finite (NaN or an infinity);
//   child vs parent: constraint domination -- feasible beats infeasible, two
//     infeasible compare violations (strictly smaller wins), two feasible
//     compare by Pareto domination (none worse, one strictly better);
//   archive: feasible objective vectors; a feasible child is non-dominated
//     when no member Pareto-dominates it (an equal member does not);
//   an evaluation whose parent or group index is out of range is rejected;
//   adaptive steering (Sec. 4.3.2): a guidance value above the caller's bound
//     (1.5 times the archive's best) is a hard constraint -- the solution is
//     infeasible and violations compare lexicographically as (fold
//     violation, FP32 excess guidance - bound); an infinite bound is off.
//
// Three launches: the decisions (one thread per evaluation, the archive
// staged through LDS in chunks shared by the block), the write-back (one
// wave per evaluation: 48-byte record pairs as three 16-byte vectors, then
// the group's coordinates), and the per-candidate reduction of the
// evaluation over the parents' caches.
#include <math.h>

#include <algorithm>
#include <stdio.h>
#include <string.h>

#include "morea_internal.h"

namespace morea {
namespace accept {

constexpr int kBlock = 256;
constexpr int kChunk = 512;   // archive members staged per pass (6 KB of LDS)

// Feasibility and the violation pair (fold violation, guidance excess).
__device__ __forceinline__ bool feasible_of(float o0, float o1, float o2, uint8_t f, float sev, float gmax,
                                            float& fold, float& excess) {
  if ((f & 4u) || !isfinite(o0) || !isfinite(o1) || !isfinite(o2) || !isfinite(sev)) {
    fold = excess = INFINITY;
    return false;
  }
  const bool folded = (f & 3u) != 0, over = o2 > gmax;
  fold = folded ? sev : 0.f;
  excess = over ? o2 - gmax : 0.f;
  return !folded && !over;
}

__device__ __forceinline__ bool pareto(float a0, float a1, float a2, float b0, float b1, float b2) {
  return a0 <= b0 && a1 <= b1 && a2 <= b2 && (a0 < b0 || a1 < b1 || a2 < b2);
}

__global__ __launch_bounds__(kBlock) void k_decide(int n_evals, int n_parents, int n_groups,
                                                   const int* __restrict__ eval_parent,
                                                   const int* __restrict__ eval_group,
                                                   const float* __restrict__ child_obj,
                                                   const uint8_t* __restrict__ child_flags,
                                                   const float* __restrict__ child_sev,
                                                   const float* __restrict__ parent_obj,
                                                   const uint8_t* __restrict__ parent_flags,
                                                   const float* __restrict__ parent_sev,
                                                   const float* __restrict__ archive, int n_archive, float gmax,
                                                   uint8_t* __restrict__ accepted) {
  __shared__ float s_arc[kChunk * 3];
  const int e = blockIdx.x * kBlock + threadIdx.x;
  bool decided = true, ok = false;
  float c0 = 0.f, c1 = 0.f, c2 = 0.f;
  if (e < n_evals) {
    const int par = eval_parent[e], g = eval_group[e];
    if (par >= 0 && par < n_parents && g >= 0 && g < n_groups) {
      c0 = child_obj[3 * e];
      c1 = child_obj[3 * e + 1];
      c2 = child_obj[3 * e + 2];
      float fc_fold, fc_exc, fp_fold, fp_exc;
      const bool fc = feasible_of(c0, c1, c2, child_flags[e], child_sev[e], gmax, fc_fold, fc_exc);
      const float p0 = parent_obj[3 * par], p1 = parent_obj[3 * par + 1], p2 = parent_obj[3 * par + 2];
      const bool fp = feasible_of(p0, p1, p2, parent_flags[par], parent_sev[par], gmax, fp_fold, fp_exc);
      const bool less = fc_fold < fp_fold || (fc_fold == fp_fold && fc_exc < fp_exc);
      const bool dom = (fc && fp) ? pareto(c0, c1, c2, p0, p1, p2) : (fc != fp ? fc : less);
      if (dom) {
        ok = true;
      } else if (fc) {
        ok = true;          // until a member of the archive dominates it
        decided = false;
      }
    }
  }
  for (int base = 0; base < n_archive; base += kChunk) {
    if (!__syncthreads_or(decided ? 0 : 1)) break;
    const int m = min(kChunk, n_archive - base);
    for (int i = threadIdx.x; i < 3 * m; i += kBlock) s_arc[i] = archive[3 * static_cast<size_t>(base) + i];
    __syncthreads();
    if (!decided) {
      for (int i = 0; i < m; i++)
        if (pareto(s_arc[3 * i], s_arc[3 * i + 1], s_arc[3 * i + 2], c0, c1, c2)) {
          ok = false;
          decided = true;
          break;
        }
    }
  }
  if (e < n_evals) accepted[e] = ok ? 1 : 0;
}

// One wave per evaluation: the accepted child's dependent-tet records (two
// directions, 48 bytes) into the parent's cache, and its group's new
// coordinates into the parent's points.
__global__ __launch_bounds__(kBlock) void k_write_back(int n_evals, int n_parents, int n_groups, int n_points,
                                                       int n_tets, const int* __restrict__ eval_parent,
                                                       const int* __restrict__ eval_group,
                                                       const uint8_t* __restrict__ accepted,
                                                       const int* __restrict__ row_off,
                                                       const int* __restrict__ item_off,
                                                       const int* __restrict__ grp_off,
                                                       const int* __restrict__ grp_pts,
                                                       const int* __restrict__ dep_off,
                                                       const int* __restrict__ dep_tet,
                                                       const float* __restrict__ new_coords,
                                                       const uint4* __restrict__ new_rec,
                                                       float* __restrict__ parent_pts,
                                                       uint4* __restrict__ parent_rec) {
  const int e = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (e >= n_evals || !accepted[e]) return;
  const int par = eval_parent[e], g = eval_group[e];
  if (par < 0 || par >= n_parents || g < 0 || g >= n_groups) return;
  const int d0 = dep_off[g], nd = dep_off[g + 1] - d0;
  const size_t src = static_cast<size_t>(item_off[e]) * 3;
  for (int i = lane; i < 3 * nd; i += kWave) {
    const int j = i / 3, q = i - 3 * j;
    const size_t dst = (static_cast<size_t>(par) * n_tets + dep_tet[d0 + j]) * 3;
    parent_rec[dst + q] = new_rec[src + 3 * static_cast<size_t>(j) + q];
  }
  const int k0 = grp_off[g], nk = grp_off[g + 1] - k0;
  const size_t row = static_cast<size_t>(row_off[e]);
  for (int i = lane; i < 6 * nk; i += kWave) {
    const int k = i / 6, r = i - 6 * k;   // r = mesh * 3 + axis
    parent_pts[(static_cast<size_t>(par) * 6 + r) * n_points + grp_pts[k0 + k]] = new_coords[(row + k) * 6 + r];
  }
}

// ---------------------------------------------------------------- selection
// Selection and clustering at the start of a generation (Sec. 3: a selection
// of non-dominated solutions of the population, clustered into k equally
// sized clusters), one block of 1024 threads, one solution per thread.
// Definitions where the paper leaves the details to MO-RV-GOMEA's literature:
//   fronts by peeling under the constraint domination above; the selection
//     takes whole fronts in order and the last one it needs in ascending
//     index, up to `size` solutions; invalid solutions are never selected;
//   objectives normalised over the selection, (v - lo) / (hi - lo), 0 where
//     hi == lo; squared Euclidean distances in FP64, contraction off;
//   leaders: the selected solution with the smallest normalised first
//     objective, then repeatedly the one farthest from the leaders so far
//     (ties to the lower index), min(k, |S|) of them;
//   cluster j: the m = min(|S|, ceil(2 |S| / k)) selected solutions nearest
//     to leader j (ties to the lower index), in ascending index;
//   the cluster of a valid solution: its nearest leader (ties to the lower
//     cluster); -1 for an invalid one.
constexpr int kSelThreads = 1024;

struct SelShared {
  double key[kSelThreads];
  int idx[kSelThreads];
  int scan[kSelThreads];
  int count;
};

// Block-wide minimum of (key, idx) (lexicographic); every thread returns it.
__device__ void block_argmin(SelShared& S, double key, int idx, double& out_key, int& out_idx) {
  const int t = threadIdx.x;
  S.key[t] = key;
  S.idx[t] = idx;
  __syncthreads();
  for (int d = kSelThreads / 2; d > 0; d >>= 1) {
    if (t < d) {
      const double k2 = S.key[t + d];
      const int i2 = S.idx[t + d];
      if (k2 < S.key[t] || (k2 == S.key[t] && i2 < S.idx[t])) {
        S.key[t] = k2;
        S.idx[t] = i2;
      }
    }
    __syncthreads();
  }
  out_key = S.key[0];
  out_idx = S.idx[0];
  __syncthreads();
}

// Block-wide exclusive prefix sum of v; *total receives the sum.
__device__ int block_scan(SelShared& S, int v, int* total) {
  const int t = threadIdx.x;
  S.scan[t] = v;
  __syncthreads();
  for (int d = 1; d < kSelThreads; d <<= 1) {
    const int x = t >= d ? S.scan[t - d] : 0;
    __syncthreads();
    S.scan[t] += x;
    __syncthreads();
  }
  const int incl = S.scan[t];
  *total = S.scan[kSelThreads - 1];
  __syncthreads();
  return incl - v;
}

__device__ __forceinline__ double dist3(const double* a, const double* b) {
#pragma clang fp contract(off)
  double s = 0.0;
  for (int o = 0; o < 3; o++) {
    const double d = a[o] - b[o];
    const double p = d * d;
    s = s + p;
  }
  return s;
}

__global__ __launch_bounds__(kSelThreads) void k_select(int n, int size, int k, float gmax,
                                                        const float* __restrict__ obj,
                                                        const uint8_t* __restrict__ flags,
                                                        const float* __restrict__ sev, int* __restrict__ sel_out,
                                                        int* __restrict__ n_sel_out, int* __restrict__ clu_off,
                                                        int* __restrict__ clu_members,
                                                        int* __restrict__ cluster_of) {
#pragma clang fp contract(off)
  __shared__ SelShared S;
  __shared__ float s_o[3][kSelThreads];
  __shared__ float s_fold[kSelThreads], s_exc[kSelThreads];
  __shared__ uint8_t s_feas[kSelThreads], s_left[kSelThreads];
  __shared__ double s_norm[3][kSelThreads];
  __shared__ int s_leader[kSelThreads];
  const int i = threadIdx.x;
  const bool in = i < n;
  float o0 = 0.f, o1 = 0.f, o2 = 0.f, fold = 0.f, exc = 0.f;
  bool valid = false, feas = false;
  if (in) {
    o0 = obj[3 * i];
    o1 = obj[3 * i + 1];
    o2 = obj[3 * i + 2];
    const uint8_t f = flags[i];
    const float sv = sev[i];
    valid = !((f & 4u) || !isfinite(o0) || !isfinite(o1) || !isfinite(o2) || !isfinite(sv));
    feas = feasible_of(o0, o1, o2, f, sv, gmax, fold, exc);
  }
  s_o[0][i] = o0;
  s_o[1][i] = o1;
  s_o[2][i] = o2;
  s_fold[i] = fold;
  s_exc[i] = exc;
  s_feas[i] = feas;
  s_left[i] = valid;
  __syncthreads();
  // dominators of each solution as a bit row (32 words of 32 solutions),
  // then fronts by peeling until `size` solutions are covered: a solution
  // joins the front when none of its dominators is left
  __shared__ uint32_t s_left_bits[kSelThreads / 32];
  if (i < kSelThreads / 32) s_left_bits[i] = 0u;
  __syncthreads();
  if (valid) atomicOr(&s_left_bits[i >> 5], 1u << (i & 31));
  uint32_t dm[kSelThreads / 32];
#pragma unroll
  for (int w = 0; w < kSelThreads / 32; w++) {
    uint32_t bits = 0u;
    if (valid && w * 32 < n)
      for (int b = 0; b < 32; b++) {
        const int j = w * 32 + b;
        if (j >= n || j == i || !s_left[j]) continue;
        bool dom;
        if (s_feas[j] && s_feas[i])
          dom = pareto(s_o[0][j], s_o[1][j], s_o[2][j], s_o[0][i], s_o[1][i], s_o[2][i]);
        else if (s_feas[j] != s_feas[i])
          dom = s_feas[j];
        else
          dom = s_fold[j] < s_fold[i] || (s_fold[j] == s_fold[i] && s_exc[j] < s_exc[i]);
        bits |= dom ? (1u << b) : 0u;
      }
    dm[w] = bits;
  }
  __syncthreads();
  int rank = -1, covered = 0, r = 0;
  bool left = valid;
  while (covered < size) {
    uint32_t hit = 0u;
#pragma unroll
    for (int w = 0; w < kSelThreads / 32; w++) hit |= dm[w] & s_left_bits[w];
    const bool front = left && hit == 0u;
    int n_front;
    const int before = block_scan(S, front ? 1 : 0, &n_front);
    if (n_front == 0) break;
    if (front) {
      left = false;
      atomicAnd(&s_left_bits[i >> 5], ~(1u << (i & 31)));
      // the last front needed is cut in ascending index
      if (covered + before < size) rank = r;
    }
    covered += n_front;
    r++;
    __syncthreads();
  }
  const bool chosen = rank >= 0;
  int n_sel;
  const int pos = block_scan(S, chosen ? 1 : 0, &n_sel);
  if (chosen) sel_out[pos] = i;
  if (i == 0) *n_sel_out = n_sel;
  const int k_eff = min(k, n_sel);
  const int m = n_sel == 0 ? 0 : min(n_sel, (2 * n_sel + k - 1) / k);
  for (int j = i; j <= k; j += kSelThreads) clu_off[j] = min(j, k_eff) * m;
  if (n_sel == 0) {
    if (in) cluster_of[i] = -1;
    return;
  }
  // normalisation over the selection (exact minima and maxima)
  double lo[3], hi[3];
  for (int o = 0; o < 3; o++) {
    double mn, mx;
    int dummy;
    block_argmin(S, chosen ? static_cast<double>(s_o[o][i]) : INFINITY, i, mn, dummy);
    block_argmin(S, chosen ? -static_cast<double>(s_o[o][i]) : INFINITY, i, mx, dummy);
    lo[o] = mn;
    hi[o] = -mx;
  }
  double me[3];
  for (int o = 0; o < 3; o++) {
    const double v = static_cast<double>(s_o[o][i]);
    me[o] = hi[o] > lo[o] ? (v - lo[o]) / (hi[o] - lo[o]) : 0.0;
    s_norm[o][i] = me[o];
  }
  __syncthreads();
  // leaders: smallest first objective, then farthest points
  double kk;
  int first;
  block_argmin(S, chosen ? me[0] : INFINITY, chosen ? i : 0x7fffffff, kk, first);
  if (i == 0) s_leader[0] = first;
  double lead[3] = {s_norm[0][first], s_norm[1][first], s_norm[2][first]};
  double nearest = chosen ? dist3(me, lead) : 0.0;
  for (int j = 1; j < k_eff; j++) {
    int nxt;
    block_argmin(S, chosen ? -nearest : INFINITY, chosen ? i : 0x7fffffff, kk, nxt);
    if (i == 0) s_leader[j] = nxt;
    const double ln[3] = {s_norm[0][nxt], s_norm[1][nxt], s_norm[2][nxt]};
    const double d = dist3(me, ln);
    if (chosen && d < nearest) nearest = d;
  }
  __syncthreads();
  // members of each cluster: the m nearest selected solutions, ascending index
  for (int j = 0; j < k_eff; j++) {
    const int L = s_leader[j];
    const double ln[3] = {s_norm[0][L], s_norm[1][L], s_norm[2][L]};
    const double dme = dist3(me, ln);
    S.key[i] = chosen ? dme : INFINITY;
    __syncthreads();
    int closer = 0;
    if (chosen)
      for (int q = 0; q < n; q++) {
        const double dq = S.key[q];
        closer += (dq < dme || (dq == dme && q < i)) ? 1 : 0;
      }
    const bool member = chosen && closer < m;
    int cnt;
    const int at = block_scan(S, member ? 1 : 0, &cnt);
    // exactly m members by the (distance, index) order; the bound keeps every
    // write inside cluster j's m slots whatever the keys hold
    if (member && at < m) clu_members[j * m + at] = i;
  }
  // cluster of every valid solution: the nearest leader
  if (in) {
    int best = -1;
    double bd = INFINITY;
    if (valid)
      for (int j = 0; j < k_eff; j++) {
        const int L = s_leader[j];
        const double ln[3] = {s_norm[0][L], s_norm[1][L], s_norm[2][L]};
        const double d = dist3(me, ln);
        if (best < 0 || d < bd) {
          bd = d;
          best = j;
        }
      }
    cluster_of[i] = best;
  }
}

}  // namespace accept
}  // namespace morea

using namespace morea;

namespace {

morea_status accept_fail(morea_status code, const char* msg) {
  set_error(msg);
  return code;
}

}  // namespace

extern "C" morea_status morea_select_clusters(const float* obj, const uint8_t* flags, const float* severity,
                                              int32_t n_pop, int32_t size, int32_t k, float guidance_max,
                                              int32_t* selection, int32_t* n_selected, int32_t* clu_off,
                                              int32_t* clu_members, int32_t members_cap, int32_t* cluster_of,
                                              void* stream) {
  if (n_pop < 1 || n_pop > accept::kSelThreads || size < 0 || k < 1 || isnan(guidance_max))
    return accept_fail(MOREA_EINVAL, "need 1 <= n_pop <= 1024, size >= 0, k >= 1, guidance_max not NaN");
  if (!obj || !flags || !severity || !selection || !n_selected || !clu_off || !clu_members || !cluster_of)
    return accept_fail(MOREA_EINVAL, "NULL argument");
  const int64_t s = std::min<int64_t>(size, n_pop);
  if (static_cast<int64_t>(members_cap) < k * ((2 * s + k - 1) / k))
    return accept_fail(MOREA_ERANGE, "members_cap below k * ceil(2 min(size, n_pop) / k)");
  {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return accept_fail(MOREA_EDEVICE, hipGetErrorString(e));
  }
  hipLaunchKernelGGL(accept::k_select, dim3(1), dim3(accept::kSelThreads), 0, static_cast<hipStream_t>(stream),
                     n_pop, static_cast<int>(s), k, guidance_max, obj, flags, severity, selection, n_selected, clu_off,
                     clu_members, cluster_of);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    char buf[256];
    snprintf(buf, sizeof(buf), "selection kernel: %s", hipGetErrorString(e));
    set_error(buf);
    return MOREA_EDEVICE;
  }
  return MOREA_OK;
}

extern "C" morea_status morea_accept_partial(morea_problem* p, float* parent_pts, int32_t n_parents,
                                             void* parent_cache, int32_t n_evals, const int32_t* eval_parent,
                                             const int32_t* eval_group, const float* new_coords,
                                             const float* child_obj, const uint8_t* child_flags,
                                             const float* child_sev, float* parent_obj, uint8_t* parent_flags,
                                             float* parent_sev, uint32_t* parent_counts, const float* archive_obj,
                                             int32_t n_archive, float guidance_max, uint8_t* accepted,
                                             void* stream) {
  if (!p) return accept_fail(MOREA_EINVAL, "problem is NULL");
  if (n_evals < 0 || n_parents < 1 || n_archive < 0)
    return accept_fail(MOREA_EINVAL, "need n_evals >= 0, n_parents >= 1, n_archive >= 0");
  if (isnan(guidance_max)) return accept_fail(MOREA_EINVAL, "guidance_max is NaN");
  if (n_evals == 0) return MOREA_OK;
  if (!parent_pts || !parent_cache || !eval_parent || !eval_group || !new_coords || !child_obj || !child_flags ||
      !child_sev || !parent_obj || !parent_flags || !parent_sev || !parent_counts || !accepted ||
      (n_archive > 0 && !archive_obj))
    return accept_fail(MOREA_EINVAL, "NULL argument");
  if (reinterpret_cast<uintptr_t>(parent_cache) % 16 != 0)
    return accept_fail(MOREA_EINVAL, "parent_cache must be 16-byte aligned");
  // the records and offsets of the partial evaluation live in the library's
  // workspace: they must be those of this evaluation list
  const void* key[5] = {parent_pts, parent_cache, eval_parent, eval_group, new_coords};
  if (!p->last_partial || memcmp(key, p->last_key, sizeof(key)) != 0 || p->last_n[0] != n_parents ||
      p->last_n[1] != n_evals)
    return accept_fail(MOREA_ESTATE, "acceptance must follow morea_eval_partial of the same evaluations");
  {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return accept_fail(MOREA_EDEVICE, hipGetErrorString(e));
  }
  const ProblemView& P = p->view;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(accept::k_decide, dim3((n_evals + accept::kBlock - 1) / accept::kBlock), dim3(accept::kBlock),
                     0, s, n_evals, n_parents, p->n_groups, eval_parent, eval_group, child_obj, child_flags,
                     child_sev, parent_obj, parent_flags, parent_sev, archive_obj, n_archive, guidance_max, accepted);
  Record* rec = static_cast<Record*>(parent_cache);
  Totals* tot = reinterpret_cast<Totals*>(static_cast<char*>(parent_cache) +
                                          static_cast<size_t>(n_parents) * P.n_tets * 2 * sizeof(Record));
  constexpr int per_block = accept::kBlock / kWave;
  hipLaunchKernelGGL(accept::k_write_back, dim3((n_evals + per_block - 1) / per_block), dim3(accept::kBlock), 0, s,
                     n_evals, n_parents, p->n_groups, P.n_points, P.n_tets, eval_parent, eval_group, accepted,
                     p->d_row_off, p->d_item_off, p->d_grp_off, p->d_grp_pts, p->d_dep_off, p->d_dep_tet,
                     new_coords, reinterpret_cast<const uint4*>(p->d_partial_records), parent_pts,
                     reinterpret_cast<uint4*>(rec));
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = launch_finalize(P, parent_pts, n_parents, rec, parent_obj, parent_flags, parent_sev, parent_counts, tot, s);
  if (e != hipSuccess) {
    char buf[256];
    snprintf(buf, sizeof(buf), "acceptance kernels: %s", hipGetErrorString(e));
    set_error(buf);
    return MOREA_EDEVICE;
  }
  return MOREA_OK;
}
