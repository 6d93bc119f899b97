// Fold repair of infeasible candidates (Sec. 4.3.1): each point of a folded
// tetrahedron (App. A.4) gets 64 Gaussian trial moves scaled by its estimated
// distance to the polygon its neighbours form; the trial with the best
// constraint improvement is applied, and the candidate's repair stops when
// every trial is worse.
//
// Definitions (all on the 2^-10-voxel grid of the evaluation, so every
// comparison is exact integer arithmetic):
//   constraint of a point: (folded tets among its incident tets in its mesh,
//     sum of their |6V|), compared lexicographically;
//   points visited: the vertices of the tets folded at the start, mesh S then
//     mesh T, each ascending; a point no longer in a folded tet is skipped
//     without using a draw; at most K visits (the draws given);
//   step sigma: 2^j for the largest j <= 18 with 4^j n^2 <= |n v - sum u|^2
//     (u the n neighbours of v, each once), at least 1;
//   trial k of visit i: each free axis moves by rint(sigma z[i][k][axis])
//     (ties to even); a trial leaving |x| < 2^19 (512 voxels) is never chosen;
//   the smallest (constraint, k) is applied when strictly below the point's
//     constraint, nothing happens when equal, the repair stops when above.
//
// One 64-lane wave per candidate, the 64 trials on the 64 lanes.  The
// candidate's snapped coordinates and the fold and moved bitmaps live in LDS;
// moved points are written back at the end (others keep their input bits).
#include <math.h>
#include <stdio.h>

#include "morea_internal.h"

namespace morea {
namespace repair {

constexpr int kLimit = 1 << 19;         // |x| < 512 voxels on the 2^-10 grid
constexpr int kSigmaMaxLog2 = 18;
constexpr int kMaxPoints = 6144;        // LDS: 24 B per point + bitmaps
enum Outcome { kNoFold = 0, kDone = 1, kAborted = 2, kOutOfDraws = 3, kInvalid = 4 };

typedef unsigned __int128 u128;

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int64_t det6(const int a[3], const int b[3], const int c[3], const int d[3]) {
  const int64_t u0 = b[0] - a[0], u1 = b[1] - a[1], u2 = b[2] - a[2];
  const int64_t v0 = c[0] - a[0], v1 = c[1] - a[1], v2 = c[2] - a[2];
  const int64_t w0 = d[0] - a[0], w1 = d[1] - a[1], w2 = d[2] - a[2];
  return u0 * (v1 * w2 - v2 * w1) - u1 * (v0 * w2 - v2 * w0) + u2 * (v0 * w1 - v1 * w0);
}

__device__ __forceinline__ bool folded(int64_t D, int ref) { return D == 0 || (D > 0) != (ref > 0); }

__device__ __forceinline__ uint64_t shfl_u64(uint64_t x, int src) {
  const uint32_t lo = __shfl(static_cast<uint32_t>(x), src, 64), hi = __shfl(static_cast<uint32_t>(x >> 32), src, 64);
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ u128 wave_sum_u128(u128 x) {
  for (int d = 32; d >= 1; d >>= 1) {
    const uint64_t lo = static_cast<uint64_t>(x), hi = static_cast<uint64_t>(x >> 64);
    const uint64_t olo = shfl_u64(lo, lane_id() ^ d), ohi = shfl_u64(hi, lane_id() ^ d);
    x += (static_cast<u128>(ohi) << 64) | olo;
  }
  return x;
}

__device__ __forceinline__ int wave_sum_i(int x) {
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

// Lexicographic key of a trial: (valid ? 0 : 1, count, severity, lane).
struct Key {
  uint32_t bad, cnt;
  u128 sev;
  int k;
};

__device__ __forceinline__ bool less(const Key& a, const Key& b) {
  if (a.bad != b.bad) return a.bad < b.bad;
  if (a.cnt != b.cnt) return a.cnt < b.cnt;
  if (a.sev != b.sev) return a.sev < b.sev;
  return a.k < b.k;
}

__device__ __forceinline__ Key wave_min_key(Key x) {
  for (int d = 32; d >= 1; d >>= 1) {
    const int src = lane_id() ^ d;
    Key o;
    o.bad = __shfl(x.bad, src, 64);
    o.cnt = __shfl(x.cnt, src, 64);
    const uint64_t lo = shfl_u64(static_cast<uint64_t>(x.sev), src), hi = shfl_u64(static_cast<uint64_t>(x.sev >> 64), src);
    o.sev = (static_cast<u128>(hi) << 64) | lo;
    o.k = __shfl(x.k, src, 64);
    if (less(o, x)) x = o;
  }
  return x;
}

// LDS: X[2][n][3] snapped coordinates, then the fold and moved bitmaps of
// both meshes ([2][words] each).
__global__ __launch_bounds__(64) void k_repair(ProblemView P, float* pts, const float* draws, int n_draws,
                                             const uint8_t* pinned, const int* inc_off, const int* inc,
                                             const int* nb_off, const int* nb, int* info) {
  extern __shared__ int lds[];
  const int n = P.n_points, words = (n + 31) >> 5;
  int* X = lds;                              // [2][n][3]
  uint32_t* fold_bits = reinterpret_cast<uint32_t*>(lds + 6 * n);   // [2][words]
  uint32_t* moved_bits = fold_bits + 2 * words;                      // [2][words]
  const int c = blockIdx.x, lane = lane_id();
  float* cp = pts + static_cast<size_t>(c) * 6 * n;

  // snap; any coordinate outside |x| < 512 voxels (or not a number) leaves
  // the candidate untouched
  bool ok = true;
  for (int i = lane; i < 6 * n; i += 64) {
    const int m = i / (3 * n), a = (i / n) % 3, v = i % n;
    const float x = cp[i];
    ok = ok && fabsf(x) < kCoordLimit;
    X[(m * n + v) * 3 + a] = ok ? static_cast<int>(rintf(x * kFixOne)) : 0;
  }
  if (__ballot(!ok) != 0ull) {
    if (lane == 0) {
      info[2 * c] = 0;
      info[2 * c + 1] = kInvalid;
    }
    return;
  }
  for (int i = lane; i < 4 * words; i += 64) fold_bits[i] = 0u;
  wave_sync();
  // vertices of the tets folded at the start
  bool any = false;
  for (int t = lane; t < P.n_tets; t += 64) {
    const int4 tv = P.tets[t];
    const int ref = P.ref_sign[t];
#pragma unroll
    for (int m = 0; m < 2; m++) {
      const int* b = X + m * n * 3;
      if (folded(det6(b + 3 * tv.x, b + 3 * tv.y, b + 3 * tv.z, b + 3 * tv.w), ref)) {
        any = true;
        atomicOr(&fold_bits[m * words + (tv.x >> 5)], 1u << (tv.x & 31));
        atomicOr(&fold_bits[m * words + (tv.y >> 5)], 1u << (tv.y & 31));
        atomicOr(&fold_bits[m * words + (tv.z >> 5)], 1u << (tv.z & 31));
        atomicOr(&fold_bits[m * words + (tv.w >> 5)], 1u << (tv.w & 31));
      }
    }
  }
  if (__ballot(any) == 0ull) {
    if (lane == 0) {
      info[2 * c] = 0;
      info[2 * c + 1] = kNoFold;
    }
    return;
  }
  wave_sync();

  int visit = 0, moves = 0, outcome = kDone;
  bool stop = false;
  for (int m = 0; m < 2 && !stop; m++) {
    int* Xm = X + m * n * 3;
    for (int w = 0; w < words && !stop; w++) {
      uint32_t bits = __builtin_amdgcn_readfirstlane(fold_bits[m * words + w]);
      while (bits != 0u && !stop) {
        const int v = 32 * w + __builtin_ctz(bits);
        bits &= bits - 1u;
        const int i0 = inc_off[v], i1 = inc_off[v + 1];
        // the point's constraint now
        int cnt = 0;
        u128 sev = 0;
        for (int e = i0 + lane; e < i1; e += 64) {
          const int t = inc[e] >> 2;
          const int4 tv = P.tets[t];
          const int64_t D = det6(Xm + 3 * tv.x, Xm + 3 * tv.y, Xm + 3 * tv.z, Xm + 3 * tv.w);
          if (folded(D, P.ref_sign[t])) {
            cnt += 1;
            sev += static_cast<u128>(D < 0 ? -D : D);
          }
        }
        const int cnt0 = wave_sum_i(cnt);
        const u128 sev0 = wave_sum_u128(sev);
        if (cnt0 == 0) continue;
        if (visit == n_draws) {
          outcome = kOutOfDraws;
          stop = true;
          break;
        }
        // step: distance to the neighbours' centroid, as a power of two
        const int j0 = nb_off[v], j1 = nb_off[v + 1];
        int64_t s[3] = {0, 0, 0};
        for (int e = j0 + lane; e < j1; e += 64) {
          const int u = nb[e];
#pragma unroll
          for (int a = 0; a < 3; a++) s[a] += Xm[3 * u + a];
        }
        int64_t dvec[3];
        const int64_t nn = j1 - j0;
#pragma unroll
        for (int a = 0; a < 3; a++) {
          int64_t t = s[a];
          for (int d = 32; d >= 1; d >>= 1) t += static_cast<int64_t>(shfl_u64(static_cast<uint64_t>(t), lane ^ d));
          dvec[a] = nn * Xm[3 * v + a] - t;
        }
        const u128 d2 = static_cast<u128>(static_cast<__int128>(dvec[0]) * dvec[0]) +
                        static_cast<u128>(static_cast<__int128>(dvec[1]) * dvec[1]) +
                        static_cast<u128>(static_cast<__int128>(dvec[2]) * dvec[2]);
        int jl = 0;
        if (nn > 0)
          while (jl < kSigmaMaxLog2 && (static_cast<u128>(nn * nn) << (2 * (jl + 1))) <= d2) jl++;
        const double sigma = static_cast<double>(1 << jl);
        // trial of this lane
        const float* z = draws + ((static_cast<size_t>(c) * n_draws + visit) * 64 + lane) * 3;
        const unsigned pin = pinned ? pinned[v] : 0u;
        int pos[3];
        bool valid = true;
#pragma unroll
        for (int a = 0; a < 3; a++) {
          const double step = (pin >> a) & 1u ? 0.0 : sigma * static_cast<double>(z[a]);
          // |step| >= 2^20 grid units always leaves the range (and is not a number otherwise)
          valid = valid && fabs(step) < 1048576.0;
          const int64_t q = Xm[3 * v + a] + (valid ? static_cast<int64_t>(rint(step)) : 0);
          valid = valid && q > -kLimit && q < kLimit;
          pos[a] = static_cast<int>(q);
        }
        int tc = 0;
        u128 ts = 0;
        for (int e = i0; e < i1; e++) {
          const int t = inc[e] >> 2, slot = inc[e] & 3;
          const int4 tv = P.tets[t];
          int q0[3], q1[3], q2[3], q3[3];
#pragma unroll
          for (int a = 0; a < 3; a++) {
            q0[a] = slot == 0 ? pos[a] : Xm[3 * tv.x + a];
            q1[a] = slot == 1 ? pos[a] : Xm[3 * tv.y + a];
            q2[a] = slot == 2 ? pos[a] : Xm[3 * tv.z + a];
            q3[a] = slot == 3 ? pos[a] : Xm[3 * tv.w + a];
          }
          const int64_t D = det6(q0, q1, q2, q3);
          if (folded(D, P.ref_sign[t])) {
            tc += 1;
            ts += static_cast<u128>(D < 0 ? -D : D);
          }
        }
        const Key best = wave_min_key(Key{valid ? 0u : 1u, static_cast<uint32_t>(tc), ts, lane});
        visit += 1;
        const bool improves = best.bad == 0u && (best.cnt < static_cast<uint32_t>(cnt0) ||
                                                 (best.cnt == static_cast<uint32_t>(cnt0) && best.sev < sev0));
        const bool equal = best.bad == 0u && best.cnt == static_cast<uint32_t>(cnt0) && best.sev == sev0;
        if (improves) {
          if (lane == best.k) {
#pragma unroll
            for (int a = 0; a < 3; a++) Xm[3 * v + a] = pos[a];
            moved_bits[m * words + (v >> 5)] |= 1u << (v & 31);
          }
          moves += 1;
          wave_sync();
        } else if (!equal) {
          outcome = kAborted;
          stop = true;
        }
      }
    }
  }
  wave_sync();
  // write the moved points back (exact: grid value * 2^-10)
  for (int i = lane; i < 2 * n; i += 64) {
    const int m = i / n, v = i % n;
    if ((moved_bits[m * words + (v >> 5)] >> (v & 31)) & 1u)
#pragma unroll
      for (int a = 0; a < 3; a++) cp[(m * 3 + a) * n + v] = static_cast<float>(X[(m * n + v) * 3 + a]) * 0x1p-10f;
  }
  if (lane == 0) {
    info[2 * c] = moves;
    info[2 * c + 1] = outcome;
  }
}

}  // namespace repair
}  // namespace morea

using namespace morea;

extern "C" morea_status morea_repair_folds(morea_problem* p, float* pts, int32_t pop, const float* draws,
                                           int32_t n_draws, const uint8_t* pinned, int32_t* info, void* stream) {
  if (!p) {
    set_error("problem is NULL");
    return MOREA_EINVAL;
  }
  if (pop < 0 || n_draws < 1) {
    set_error("need pop >= 0 and n_draws >= 1");
    return MOREA_EINVAL;
  }
  if (pop == 0) return MOREA_OK;
  if (!pts || !draws || !info) {
    set_error("NULL argument");
    return MOREA_EINVAL;
  }
  const ProblemView& P = p->view;
  if (P.n_points > repair::kMaxPoints) {
    set_error("fold repair keeps a candidate in LDS: at most 6144 points per mesh");
    return MOREA_ERANGE;
  }
  {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      set_error(hipGetErrorString(e));
      return MOREA_EDEVICE;
    }
  }
  const int words = (P.n_points + 31) / 32;
  const size_t lds = sizeof(int) * (6 * static_cast<size_t>(P.n_points) + 4 * static_cast<size_t>(words));
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(repair::k_repair),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (e == hipSuccess) {
    hipLaunchKernelGGL(repair::k_repair, dim3(pop), dim3(64), lds, static_cast<hipStream_t>(stream), P, pts, draws,
                       n_draws, pinned, p->d_pinc_off, p->d_pinc, p->d_nb_off, p->d_nb, info);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    char buf[256];
    snprintf(buf, sizeof(buf), "fold repair: %s", hipGetErrorString(e));
    set_error(buf);
    return MOREA_EDEVICE;
  }
  return MOREA_OK;
}
