// Elitist archive of the optimizer (Sec. 3: non-dominated solutions kept
// across generations in an archive of fixed capacity, 2000 in App. C's
// parameter listing; Sec. 4.3.2: with adaptive steering on, only guidance
// values up to 1.5 times the archive's best are kept, which purges the
// archive when steering starts) and the adaptation of the distribution
// multipliers of optimal mixing.
//
// Definitions where the paper defers to its references on elitist archiving
// and on MO-RV-GOMEA:
//   members are feasible solutions (valid, no fold, finite objectives and
//     severity) in slots; each carries an insertion stamp that orders them;
//     a free slot has stamp -1 and the objective vector (inf, inf, inf),
//     which dominates nothing, so the acceptance may read every slot;
//   an update's candidates are the members in stamp order, then the feasible
//     offers in index order, less every candidate whose guidance value is
//     above the steering bound; a candidate stays unless another candidate
//     Pareto-dominates it or an earlier one has the same objective vector;
//   above capacity the stayers are thinned by boxes: per objective the range
//     [lo, hi] of the stayers is cut into L equal boxes (FP64, contraction
//     off: box = min(L - 1, floor(((v - lo) / (hi - lo)) * L)), 0 where
//     hi == lo); L is found by a binary search over [1, min(capacity, 1024)]
//     for a resolution whose occupied boxes number at most the capacity, and
//     each occupied box keeps its earliest candidate;
//   members that do not stay free their slots; staying offers fill the free
//     slots in ascending slot order, in offer order, with the next stamps;
//   distribution multipliers (adaptive variance scaling, reduced): a
//     (cluster, element) improves in a generation when a kept child sampled
//     from it belongs to a parent that then entered the archive; on
//     improvement the no-improvement stretch resets and c = max(c, 1) / 0.9
//     (at most 10); otherwise, when c <= 1 the stretch grows, and when c > 1
//     or the stretch has reached 25, c = 0.9 c; a c below 1 whose stretch is
//     under 25 is reset to 1.
//
// The update is one block of 1,024 threads holding up to 4,096 candidates
// in LDS: the members ordered by a bitonic sort of their stamps, domination
// and duplicates by comparisons against LDS (broadcast reads; members only
// against the offers, since they are mutually non-dominated and distinct),
// and each resolution of the thinning's search by a bitonic sort of the
// stayers' (box key, candidate) pairs.
#include <math.h>
#include <stdio.h>

#include "morea_internal.h"

namespace morea {
namespace archive {

constexpr int kThreads = 1024;
constexpr int kMax = 4096;                 // members + offers per update
constexpr int kPer = kMax / kThreads;
constexpr int kMaxLevels = 1024;           // boxes per objective (10-bit fields of a key)
constexpr uint32_t kNoKey = 0xffffffffu;

__device__ __forceinline__ bool pareto(float a0, float a1, float a2, float b0, float b1, float b2) {
  return a0 <= b0 && a1 <= b1 && a2 <= b2 && (a0 < b0 || a1 < b1 || a2 < b2);
}

struct Shared {
  float o[3][kMax];      // candidate objective vectors, in candidate order
  int src[kMax];         // slot of a member, -1 - index of an offer
  // sort keys: (stamp, slot) of the members, then (box key, candidate) of
  // the stayers; afterwards the occupancy of the slots (low words)
  uint64_t sortbuf[kMax];
  int flag[kMax];        // first candidate of its box; then the free slots in ascending order
  int wsum[kThreads / 64];
  float wmin[kThreads / 64];
  float wmax[kThreads / 64];
};

// Ascending bitonic sort of a[0 .. n2) (n2 a power of two, at most kMax) by
// the whole block; ends with a barrier.
__device__ void bitonic_sort(uint64_t* a, int n2) {
  for (int k = 2; k <= n2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n2; i += kThreads) {
        const int l = i ^ j;
        if (l > i) {
          const uint64_t x = a[i], y = a[l];
          if ((x > y) == ((i & k) == 0)) {
            a[i] = y;
            a[l] = x;
          }
        }
      }
      __syncthreads();
    }
}

__device__ __forceinline__ int pow2_at_least(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// Exclusive prefix over the block of one value per thread; *total gets the sum.
__device__ int block_excl(Shared& S, int v, int* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) S.wsum[w] = x;
  __syncthreads();
  int before = 0, all = 0;
  for (int k = 0; k < kThreads / 64; k++) {
    const int s = S.wsum[k];
    before += k < w ? s : 0;
    all += s;
  }
  __syncthreads();
  *total = all;
  return before + x - v;
}

__device__ float block_min(Shared& S, float v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = fminf(v, __shfl_xor(v, d, 64));
  if ((threadIdx.x & 63) == 0) S.wmin[threadIdx.x >> 6] = v;
  __syncthreads();
  float r = INFINITY;
  for (int k = 0; k < kThreads / 64; k++) r = fminf(r, S.wmin[k]);
  __syncthreads();
  return r;
}

__device__ float block_max(Shared& S, float v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, 64));
  if ((threadIdx.x & 63) == 0) S.wmax[threadIdx.x >> 6] = v;
  __syncthreads();
  float r = -INFINITY;
  for (int k = 0; k < kThreads / 64; k++) r = fmaxf(r, S.wmax[k]);
  __syncthreads();
  return r;
}

__device__ __forceinline__ int box_of(float v, double lo, double hi, int L) {
#pragma clang fp contract(off)
  if (!(hi > lo)) return 0;
  const double t = (static_cast<double>(v) - lo) / (hi - lo);
  const double s = t * static_cast<double>(L);
  const int b = static_cast<int>(floor(s));
  return b < L - 1 ? b : L - 1;
}

__global__ __launch_bounds__(kThreads) void k_update(int n_off, const float* __restrict__ offer_obj,
                                                     const uint8_t* __restrict__ offer_flags,
                                                     const float* __restrict__ offer_sev, float gmax, int cap,
                                                     float* __restrict__ arc_obj, int* __restrict__ arc_stamp,
                                                     int* __restrict__ arc_state, float* __restrict__ best_out,
                                                     uint8_t* __restrict__ inserted, int* __restrict__ slot_of) {
  __shared__ Shared S;
  const int t = threadIdx.x;
  // ---- members in stamp order: sort (stamp, slot) of the occupied slots
  const int ncap = pow2_at_least(cap);
  int n_occ_mine = 0;
  for (int s = t; s < ncap; s += kThreads) {
    const int st = s < cap ? arc_stamp[s] : -1;
    S.sortbuf[s] = st >= 0 ? (static_cast<uint64_t>(st) << 32 | static_cast<uint32_t>(s)) : ~0ull;
    n_occ_mine += st >= 0 ? 1 : 0;
  }
  int nm;
  block_excl(S, n_occ_mine, &nm);     // its barriers publish the keys
  bitonic_sort(S.sortbuf, ncap);
  for (int r = t; r < nm; r += kThreads) {
    const int s = static_cast<int>(S.sortbuf[r] & 0xffffffffu);
    S.o[0][r] = arc_obj[3 * s];
    S.o[1][r] = arc_obj[3 * s + 1];
    S.o[2][r] = arc_obj[3 * s + 2];
    S.src[r] = s;
  }
  // ---- feasible offers after them, in index order
  bool feas = false;
  float f0 = 0.f, f1 = 0.f, f2 = 0.f;
  if (t < n_off) {
    f0 = offer_obj[3 * t];
    f1 = offer_obj[3 * t + 1];
    f2 = offer_obj[3 * t + 2];
    const float sv = offer_sev[t];
    feas = offer_flags[t] == 0 && isfinite(f0) && isfinite(f1) && isfinite(f2) && isfinite(sv);
  }
  int n_feas;
  const int at = nm + block_excl(S, feas ? 1 : 0, &n_feas);
  if (feas) {
    S.o[0][at] = f0;
    S.o[1][at] = f1;
    S.o[2][at] = f2;
    S.src[at] = -1 - t;
  }
  const int N = nm + n_feas;
  __syncthreads();
  // ---- stayers: inside the steering window, not dominated, first of equals.
  // The members are mutually non-dominated and distinct (every update leaves
  // them so), so a member can only be dominated by an offer and is never the
  // later of two equal vectors; an offer is tested against every candidate.
  bool stay[kPer];
  int n_stay_mine = 0;
#pragma unroll
  for (int j = 0; j < kPer; j++) {
    const int x = t + j * kThreads;
    bool ok = x < N && !(S.o[2][x] > gmax);
    if (ok) {
      const float a0 = S.o[0][x], a1 = S.o[1][x], a2 = S.o[2][x];
      for (int y = x < nm ? nm : 0; y < N; y++) {
        const float b0 = S.o[0][y], b1 = S.o[1][y], b2 = S.o[2][y];
        if (y == x || b2 > gmax) continue;
        if (pareto(b0, b1, b2, a0, a1, a2) || (y < x && b0 == a0 && b1 == a1 && b2 == a2)) {
          ok = false;
          break;
        }
      }
    }
    stay[j] = ok;
    n_stay_mine += ok ? 1 : 0;
  }
  int n_stay;
  block_excl(S, n_stay_mine, &n_stay);
  // ---- thinning by boxes above capacity: per resolution, the stayers'
  // (box key, candidate) sorted; the first entry of each key is its box's
  // earliest candidate
  int levels = 0;
  if (n_stay > cap) {
    double lo[3], hi[3];
    for (int o = 0; o < 3; o++) {
      float mn = INFINITY, mx = -INFINITY;
#pragma unroll
      for (int j = 0; j < kPer; j++) {
        const int x = t + j * kThreads;
        if (stay[j]) {
          mn = fminf(mn, S.o[o][x]);
          mx = fmaxf(mx, S.o[o][x]);
        }
      }
      lo[o] = block_min(S, mn);
      hi[o] = block_max(S, mx);
    }
    const int n2 = pow2_at_least(N);
    int a = 1, b = cap < kMaxLevels ? cap : kMaxLevels;
    // the last pass (a == b) sorts at the chosen resolution
    for (;;) {
      const int L = a < b ? (a + b + 1) / 2 : a;
      for (int x = t; x < n2; x += kThreads) S.sortbuf[x] = ~0ull;
      __syncthreads();
#pragma unroll
      for (int j = 0; j < kPer; j++) {
        const int x = t + j * kThreads;
        if (x < N && stay[j]) {
          const uint32_t key = static_cast<uint32_t>(box_of(S.o[0][x], lo[0], hi[0], L)) |
                               static_cast<uint32_t>(box_of(S.o[1][x], lo[1], hi[1], L)) << 10 |
                               static_cast<uint32_t>(box_of(S.o[2][x], lo[2], hi[2], L)) << 20;
          S.sortbuf[x] = static_cast<uint64_t>(key) << 32 | static_cast<uint32_t>(x);
        }
      }
      __syncthreads();
      bitonic_sort(S.sortbuf, n2);
      int n_first_mine = 0;
      for (int i = t; i < n2; i += kThreads) {
        const uint64_t v = S.sortbuf[i];
        const bool first = v != ~0ull && (i == 0 || (S.sortbuf[i - 1] >> 32) != (v >> 32));
        n_first_mine += first ? 1 : 0;
      }
      int cnt;
      block_excl(S, n_first_mine, &cnt);    // its barriers also end the key reads
      if (a == b) break;
      if (cnt <= cap) a = L;
      else b = L - 1;
    }
    levels = a;
    // keep the first candidate of each box
    for (int x = t; x < N; x += kThreads) S.flag[x] = 0;
    __syncthreads();
    for (int i = t; i < n2; i += kThreads) {
      const uint64_t v = S.sortbuf[i];
      if (v != ~0ull && (i == 0 || (S.sortbuf[i - 1] >> 32) != (v >> 32)))
        S.flag[static_cast<uint32_t>(v)] = 1;
    }
    __syncthreads();
    n_stay_mine = 0;
#pragma unroll
    for (int j = 0; j < kPer; j++) {
      const int x = t + j * kThreads;
      stay[j] = stay[j] && S.flag[x] != 0;
      n_stay_mine += stay[j] ? 1 : 0;
    }
    block_excl(S, n_stay_mine, &n_stay);
  }
  // ---- slots: occupancy after the update (low words of sortbuf)
  uint32_t* occ = reinterpret_cast<uint32_t*>(S.sortbuf);
  for (int s = t; s < cap; s += kThreads) occ[s] = 0u;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kPer; j++) {
    const int x = t + j * kThreads;
    if (x >= N) continue;
    const int src = S.src[x];
    if (src >= 0) {
      if (stay[j]) {
        occ[src] = 1u;
      } else {
        arc_stamp[src] = -1;
        arc_obj[3 * src] = INFINITY;
        arc_obj[3 * src + 1] = INFINITY;
        arc_obj[3 * src + 2] = INFINITY;
      }
    }
  }
  __syncthreads();
  // free slots in ascending order: thread t scans slots 4t .. 4t + 3
  {
    int fr[kPer], nf = 0;
#pragma unroll
    for (int j = 0; j < kPer; j++) {
      const int s = kPer * t + j;
      fr[j] = (s < cap && occ[s] == 0u) ? 1 : 0;
      nf += fr[j];
    }
    int total;
    int pos = block_excl(S, nf, &total);
#pragma unroll
    for (int j = 0; j < kPer; j++)
      if (fr[j]) S.flag[pos++] = kPer * t + j;
  }
  // staying offers take the free slots in candidate order (x = t + j * 1024,
  // so one pass per j, each ranked by a block prefix)
  if (t < n_off) {
    inserted[t] = 0;
    slot_of[t] = -1;
  }
  __syncthreads();
  const int next = arc_state[1];
  int base = 0;
#pragma unroll
  for (int j = 0; j < kPer; j++) {
    const int x = t + j * kThreads;
    const bool nw = x < N && stay[j] && S.src[x] < 0;
    int cnt;
    const int r = base + block_excl(S, nw ? 1 : 0, &cnt);
    if (nw) {
      const int s = S.flag[r];
      const int i = -1 - S.src[x];
      arc_obj[3 * s] = S.o[0][x];
      arc_obj[3 * s + 1] = S.o[1][x];
      arc_obj[3 * s + 2] = S.o[2][x];
      arc_stamp[s] = next + r;
      inserted[i] = 1;
      slot_of[i] = s;
    }
    base += cnt;
  }
  // best guidance among the members after the update
  float g = INFINITY;
#pragma unroll
  for (int j = 0; j < kPer; j++) {
    const int x = t + j * kThreads;
    if (x < N && stay[j]) g = fminf(g, S.o[2][x]);
  }
  g = block_min(S, g);
  if (t == 0) {
    arc_state[0] = n_stay;
    arc_state[1] = next + base;
    arc_state[2] = levels;
    arc_state[3] = 0;
    best_out[0] = g;
  }
}

// Points of the offers that entered the archive, into their slots.
__global__ void k_copy_points(int n_off, int per, const float* __restrict__ offer_pts,
                              const int* __restrict__ slot_of, float* __restrict__ arc_pts) {
  const int i = blockIdx.x;
  const int s = slot_of[i];
  if (s < 0) return;
  const float* src = offer_pts + static_cast<size_t>(i) * per;
  float* dst = arc_pts + static_cast<size_t>(s) * per;
  for (int q = threadIdx.x; q < per; q += blockDim.x) dst[q] = src[q];
}

__global__ void k_clear(int cap, float* __restrict__ arc_obj, int* __restrict__ arc_stamp,
                        int* __restrict__ arc_state, float* __restrict__ best_out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < cap) {
    arc_stamp[s] = -1;
    arc_obj[3 * s] = INFINITY;
    arc_obj[3 * s + 1] = INFINITY;
    arc_obj[3 * s + 2] = INFINITY;
  }
  if (s < 4) arc_state[s] = 0;
  if (s == 0) best_out[0] = INFINITY;
}

// Improvements of one batch: a kept child whose parent entered the archive
// marks its (cluster, element).
__global__ void k_mark(int n_evals, int n_parents, int n_clusters, int n_groups, const int* __restrict__ eval_parent,
                       const int* __restrict__ eval_group, const int* __restrict__ eval_cluster,
                       const uint8_t* __restrict__ accepted, const uint8_t* __restrict__ parent_inserted,
                       uint8_t* __restrict__ improved) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_evals || !accepted[e]) return;
  const int p = eval_parent[e], g = eval_group[e], c = eval_cluster[e];
  if (p < 0 || p >= n_parents || g < 0 || g >= n_groups || c < 0 || c >= n_clusters) return;
  if (parent_inserted[p]) improved[static_cast<size_t>(c) * n_groups + g] = 1;
}

__global__ void k_adapt(int n, uint8_t* __restrict__ improved, float* __restrict__ mult, int* __restrict__ nis) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  float c = mult[q];
  int s = nis[q];
  if (improved[q]) {
    s = 0;
    c = fminf(fmaxf(c, 1.f) / 0.9f, 10.f);
  } else {
    if (c <= 1.f) s += 1;
    if (c > 1.f || s >= 25) c = 0.9f * c;
    else if (c < 1.f) c = 1.f;
  }
  mult[q] = c;
  nis[q] = s;
  improved[q] = 0;
}

}  // namespace archive
}  // namespace morea

using namespace morea;

namespace {

morea_status arc_fail(morea_status code, const char* msg) {
  set_error(msg);
  return code;
}

morea_status arc_launched(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess) return MOREA_OK;
  char buf[256];
  snprintf(buf, sizeof(buf), "%s: %s", what, hipGetErrorString(e));
  set_error(buf);
  return MOREA_EDEVICE;
}

morea_status arc_pending() {
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess) return MOREA_OK;
  set_error(hipGetErrorString(e));
  return MOREA_EDEVICE;
}

}  // namespace

extern "C" morea_status morea_archive_clear(int32_t capacity, float* arc_obj, int32_t* arc_stamp,
                                            int32_t* arc_state, float* best_guidance, void* stream) {
  if (capacity < 1 || capacity > archive::kMax) return arc_fail(MOREA_EINVAL, "need 1 <= capacity <= 4096");
  if (!arc_obj || !arc_stamp || !arc_state || !best_guidance) return arc_fail(MOREA_EINVAL, "NULL argument");
  if (morea_status st = arc_pending()) return st;
  hipLaunchKernelGGL(archive::k_clear, dim3((capacity + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream),
                     capacity, arc_obj, arc_stamp, arc_state, best_guidance);
  return arc_launched("archive clear kernel");
}

extern "C" morea_status morea_archive_update(int32_t n_offers, const float* offer_obj, const uint8_t* offer_flags,
                                             const float* offer_sev, const float* offer_pts, int32_t n_points,
                                             float guidance_max, int32_t capacity, float* arc_obj,
                                             int32_t* arc_stamp, float* arc_pts, int32_t* arc_state,
                                             float* best_guidance, uint8_t* inserted, int32_t* slot_of,
                                             void* stream) {
  if (capacity < 1 || n_offers < 0 || n_offers > archive::kThreads ||
      static_cast<int64_t>(capacity) + n_offers > archive::kMax)
    return arc_fail(MOREA_ERANGE, "need capacity >= 1, 0 <= n_offers <= 1024, capacity + n_offers <= 4096");
  if (isnan(guidance_max)) return arc_fail(MOREA_EINVAL, "guidance_max is NaN");
  if (!arc_obj || !arc_stamp || !arc_state || !best_guidance || (n_offers > 0 && (!offer_obj || !offer_flags ||
      !offer_sev || !inserted || !slot_of)))
    return arc_fail(MOREA_EINVAL, "NULL argument");
  if ((offer_pts == nullptr) != (arc_pts == nullptr) || (arc_pts && n_points < 1))
    return arc_fail(MOREA_EINVAL, "offer_pts and arc_pts: both NULL, or both set with n_points >= 1");
  if (morea_status st = arc_pending()) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // slot_of is needed by the point copy even when the caller does not want it
  hipLaunchKernelGGL(archive::k_update, dim3(1), dim3(archive::kThreads), 0, s, n_offers, offer_obj, offer_flags,
                     offer_sev, guidance_max, capacity, arc_obj, arc_stamp, arc_state, best_guidance, inserted,
                     slot_of);
  if (morea_status st = arc_launched("archive update kernel")) return st;
  if (arc_pts && n_offers > 0) {
    hipLaunchKernelGGL(archive::k_copy_points, dim3(n_offers), dim3(256), 0, s, n_offers, 6 * n_points, offer_pts,
                       slot_of, arc_pts);
    return arc_launched("archive point copy kernel");
  }
  return MOREA_OK;
}

extern "C" morea_status morea_mark_improvements(int32_t n_evals, const int32_t* eval_parent,
                                                const int32_t* eval_group, const int32_t* eval_cluster,
                                                const uint8_t* accepted, int32_t n_parents,
                                                const uint8_t* parent_inserted, int32_t n_clusters,
                                                int32_t n_groups, uint8_t* improved, void* stream) {
  if (n_evals < 0 || n_parents < 1 || n_clusters < 1 || n_groups < 1)
    return arc_fail(MOREA_EINVAL, "need n_evals >= 0 and n_parents, n_clusters, n_groups >= 1");
  if (n_evals == 0) return MOREA_OK;
  if (!eval_parent || !eval_group || !eval_cluster || !accepted || !parent_inserted || !improved)
    return arc_fail(MOREA_EINVAL, "NULL argument");
  if (morea_status st = arc_pending()) return st;
  hipLaunchKernelGGL(archive::k_mark, dim3((n_evals + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream),
                     n_evals, n_parents, n_clusters, n_groups, eval_parent, eval_group, eval_cluster, accepted,
                     parent_inserted, improved);
  return arc_launched("improvement marking kernel");
}

extern "C" morea_status morea_adapt_multipliers(int32_t n_clusters, int32_t n_groups, uint8_t* improved,
                                                float* mult, int32_t* no_improvement, void* stream) {
  if (n_clusters < 1 || n_groups < 1) return arc_fail(MOREA_EINVAL, "need n_clusters, n_groups >= 1");
  if (!improved || !mult || !no_improvement) return arc_fail(MOREA_EINVAL, "NULL argument");
  if (morea_status st = arc_pending()) return st;
  const int n = n_clusters * n_groups;
  hipLaunchKernelGGL(archive::k_adapt, dim3((n + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream), n,
                     improved, mult, no_improvement);
  return arc_launched("multiplier adaptation kernel");
}
