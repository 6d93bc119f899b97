// Deformation vector fields of one candidate, rasterized from its two meshes
// (Sec. 5.4 compares registrations through a forward DVF on the source grid
// and an inverse DVF on the target grid).  A voxel centre p of tet t of the
// sampled mesh (the centres of the evaluation: exact signed volumes, a centre
// on a face belonging to the tet that holds p + (e, e^2, e^3)) gets q - p,
// q its barycentric image in the other mesh.  A centre covered by several
// tets (a folded mesh) takes the tet of smallest index, a centre covered by
// none the displacement 0; a tet with a vertex coordinate that is not finite
// or has |x| >= 512 voxels is skipped.
//
// Two passes of one 64-lane wave per (direction, tet), lanes over the voxels
// of the tet's bounding box: the first claims each covered centre with an
// atomic minimum of the tet index and counts the covering tets, the second
// lets the owner write the displacement (FP64 barycentric image, rounded once
// to FP32).
//
// The same exact point location gives the point-based guidance error of the
// paper's prior work, which Sec. 4.1.3 replaces by the continuous form: every
// point c of C_s is located in the source mesh (smallest tet index if
// several), mapped to the target mesh through its barycentric coordinates,
// and its squared distance to the nearest point of the set's C_t taken; the
// value is the mean over all points of all sets (sets weighted |C_i| / |G|);
// points in no tet are left out and counted.
#include <math.h>
#include <stdio.h>

#include <mutex>

#include "morea_internal.h"

namespace morea {
namespace dvf {

typedef __int128 i128;

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// 6 x signed volume (exact in 128 bits for any coordinates below 2^21)
__device__ __forceinline__ i128 vol6(const int64_t a[3], const int64_t b[3], const int64_t c[3], const int64_t d[3]) {
  const i128 u0 = b[0] - a[0], u1 = b[1] - a[1], u2 = b[2] - a[2];
  const i128 v0 = c[0] - a[0], v1 = c[1] - a[1], v2 = c[2] - a[2];
  const i128 w0 = d[0] - a[0], w1 = d[1] - a[1], w2 = d[2] - a[2];
  return u0 * (v1 * w2 - v2 * w1) - u1 * (v0 * w2 - v2 * w0) + u2 * (v0 * w1 - v1 * w0);
}

// Face value of vertex i (the volume with vertex i replaced by p), oriented
// positive inside.
__device__ __forceinline__ i128 face(const int64_t v[4][3], int i, const int64_t p[3], int sgn) {
  const int64_t* q0 = i == 0 ? p : v[0];
  const int64_t* q1 = i == 1 ? p : v[1];
  const int64_t* q2 = i == 2 ? p : v[2];
  const int64_t* q3 = i == 3 ? p : v[3];
  const i128 s = vol6(q0, q1, q2, q3);
  return sgn > 0 ? s : -s;
}

// Inside test with the tie rule: on a face plane the sign of the face value
// at p + (e, e^2, e^3) decides, i.e. the first nonzero component of its
// gradient (the change for a unit step along x, then y, then z).
__device__ __forceinline__ bool inside(const int64_t v[4][3], int sgn, const int64_t p[3], i128 val[4]) {
  bool in = true;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    val[i] = face(v, i, p, sgn);
    if (val[i] < 0) in = false;
  }
  if (!in) return false;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    if (val[i] != 0) continue;
    int sgrad = 0;
    for (int k = 0; k < 3 && sgrad == 0; k++) {
      int64_t pk[3] = {p[0], p[1], p[2]};
      pk[k] += 1;
      const i128 g = face(v, i, pk, sgn) - val[i];
      sgrad = (g > 0) - (g < 0);
    }
    if (sgrad <= 0) return false;
  }
  return true;
}

__global__ void k_dvf_clear(size_t V, int* owner, uint32_t* cover, float* fwd, float* inv) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= 2 * V) return;
  owner[i] = 0x7fffffff;
  cover[i] = 0u;
  float* out = i < V ? fwd + 3 * i : inv + 3 * (i - V);
  out[0] = out[1] = out[2] = 0.f;
}

template <bool WRITE>
__global__ __launch_bounds__(256) void k_dvf_pass(ProblemView P, const float* cand, int* owner, uint32_t* cover,
                                                float* fwd, float* inv) {
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int item = blockIdx.x * 4 + wave;
  if (item >= 2 * P.n_tets) return;
  const int d = item / P.n_tets, t = item % P.n_tets;
  const int lane = lane_id();
  // lane l < 24: mesh (l < 12 ? sampled : other), vertex (l % 12) / 3, axis l % 3
  const int4 tv = P.tets[t];
  float x = 0.f;
  if (lane < 24) {
    const int i = (lane % 12) / 3, k = lane % 3;
    const int pt = i == 0 ? tv.x : (i == 1 ? tv.y : (i == 2 ? tv.z : tv.w));
    const int mesh = lane < 12 ? d : 1 - d;
    x = cand[(mesh * 3 + k) * P.n_points + pt];
  }
  if (__ballot(lane < 24 && !(fabsf(x) < kCoordLimit)) != 0ull) return;
  const int fix = lane < 24 ? static_cast<int>(rintf(x * kFixOne)) : 0;
  int64_t own[4][3], oth[4][3];
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int k = 0; k < 3; k++) {
      own[i][k] = __builtin_amdgcn_readlane(fix, 3 * i + k);
      oth[i][k] = __builtin_amdgcn_readlane(fix, 12 + 3 * i + k);
    }
  const i128 D = vol6(own[0], own[1], own[2], own[3]);
  if (D == 0) return;
  const int sgn = D > 0 ? 1 : -1;
  const double inv_absD = 1.0 / static_cast<double>(D > 0 ? D : -D);
  const int dims[3] = {P.nx, P.ny, P.nz};
  int lo[3], ext[3];
#pragma unroll
  for (int k = 0; k < 3; k++) {
    int64_t mn = own[0][k], mx = own[0][k];
#pragma unroll
    for (int i = 1; i < 4; i++) {
      mn = min(mn, own[i][k]);
      mx = max(mx, own[i][k]);
    }
    // ceil(mn / 1024) and floor(mx / 1024), clipped to the grid
    const int64_t c = mn >= 0 ? (mn + 1023) / 1024 : -((-mn) / 1024);
    const int64_t f = mx >= 0 ? mx / 1024 : -((-mx + 1023) / 1024);
    lo[k] = static_cast<int>(max<int64_t>(c, 0));
    ext[k] = static_cast<int>(min<int64_t>(f, dims[k] - 1)) - lo[k] + 1;
  }
  if (ext[0] <= 0 || ext[1] <= 0 || ext[2] <= 0) return;
  const size_t V = static_cast<size_t>(P.nx) * P.ny * P.nz;
  const int64_t box = static_cast<int64_t>(ext[0]) * ext[1] * ext[2];
  for (int64_t q = lane; q < box; q += 64) {
    const int xv = lo[0] + static_cast<int>(q % ext[0]);
    const int yv = lo[1] + static_cast<int>((q / ext[0]) % ext[1]);
    const int zv = lo[2] + static_cast<int>(q / (static_cast<int64_t>(ext[0]) * ext[1]));
    const int64_t p[3] = {static_cast<int64_t>(xv) * 1024, static_cast<int64_t>(yv) * 1024,
                          static_cast<int64_t>(zv) * 1024};
    i128 val[4];
    if (!inside(own, sgn, p, val)) continue;
    const size_t v = (static_cast<size_t>(zv) * P.ny + yv) * P.nx + xv;
    if (!WRITE) {
      atomicMin(&owner[d * V + v], t);
      atomicAdd(&cover[d * V + v], 1u);
    } else if (owner[d * V + v] == t) {
      float* out = (d == 0 ? fwd : inv) + 3 * v;
      const int pv[3] = {xv, yv, zv};
#pragma unroll
      for (int a = 0; a < 3; a++) {
        double qa = static_cast<double>(oth[0][a]);
#pragma unroll
        for (int i = 1; i < 4; i++)
          qa += static_cast<double>(val[i]) * inv_absD * static_cast<double>(oth[i][a] - oth[0][a]);
        out[a] = static_cast<float>(qa * (1.0 / 1024.0) - pv[a]);
      }
    }
  }
}

// Point-based guidance: one block of 4 waves per candidate; wave w takes the
// source guidance points w, w + 4, ... in order and sums their squared
// distances in FP64; the 4 sums are added in wave order.
__global__ __launch_bounds__(256) void k_point_guidance(ProblemView P, const float* pts, const int* off_s,
                                                      const int* fix_s, const int* off_t, const int* fix_t,
                                                      float* f, int* unmapped) {
  extern __shared__ int X[];                 // [2][n][3] snapped coordinates
  __shared__ double wsum[4];
  __shared__ int wcnt[4], wun[4], bad;
  const int n = P.n_points, c = blockIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6)), lane = lane_id();
  const float* cp = pts + static_cast<size_t>(c) * 6 * n;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < 6 * n; i += blockDim.x) {
    const int m = i / (3 * n), a = (i / n) % 3, v = i % n;
    const float x = cp[i];
    if (!(fabsf(x) < kCoordLimit)) bad = 1;
    X[(m * n + v) * 3 + a] = fabsf(x) < kCoordLimit ? static_cast<int>(rintf(x * kFixOne)) : 0;
  }
  __syncthreads();
  if (bad) {
    if (threadIdx.x == 0) {
      f[c] = __builtin_nanf("");
      unmapped[c] = 0;
    }
    return;
  }
  const int G = P.n_sets > 0 ? off_s[P.n_sets] : 0;
  double sum = 0.0;
  int cnt = 0, un = 0;
  for (int g = wave; g < G; g += 4) {
    int s = 0;
    while (off_s[s + 1] <= g) s++;
    const int64_t cpt[3] = {fix_s[3 * g], fix_s[3 * g + 1], fix_s[3 * g + 2]};
    // the smallest tet of the source mesh that holds the point
    int hit_t = -1;
    for (int base = 0; base < P.n_tets && hit_t < 0; base += 64) {
      const int t = base + lane;
      bool hit = false;
      if (t < P.n_tets) {
        const int4 tv = P.tets[t];
        const int vi[4] = {tv.x, tv.y, tv.z, tv.w};
        int64_t own[4][3];
        bool in_box = true;
#pragma unroll
        for (int k = 0; k < 3; k++) {
          int64_t mn = INT64_MAX, mx = INT64_MIN;
#pragma unroll
          for (int i = 0; i < 4; i++) {
            own[i][k] = X[3 * vi[i] + k];
            mn = min(mn, own[i][k]);
            mx = max(mx, own[i][k]);
          }
          in_box = in_box && cpt[k] >= mn && cpt[k] <= mx;
        }
        if (in_box) {
          const i128 D = vol6(own[0], own[1], own[2], own[3]);
          i128 val[4];
          hit = D != 0 && inside(own, D > 0 ? 1 : -1, cpt, val);
        }
      }
      const uint64_t m = __ballot(hit);
      if (m != 0ull) hit_t = base + __builtin_ctzll(m);
    }
    if (hit_t < 0) {
      un += 1;
      continue;
    }
    // its image in the target mesh (every lane, the same tet)
    const int4 tv = P.tets[hit_t];
    const int vi[4] = {tv.x, tv.y, tv.z, tv.w};
    int64_t own[4][3], oth[4][3];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
      for (int k = 0; k < 3; k++) {
        own[i][k] = X[3 * vi[i] + k];
        oth[i][k] = X[3 * (n + vi[i]) + k];
      }
    const i128 D = vol6(own[0], own[1], own[2], own[3]);
    i128 val[4];
    (void)inside(own, D > 0 ? 1 : -1, cpt, val);
    const double inv_absD = 1.0 / static_cast<double>(D > 0 ? D : -D);
    double q[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
      double qa = static_cast<double>(oth[0][a]);
#pragma unroll
      for (int i = 1; i < 4; i++)
        qa += static_cast<double>(val[i]) * inv_absD * static_cast<double>(oth[i][a] - oth[0][a]);
      q[a] = qa * (1.0 / 1024.0);
    }
    // nearest point of the set's C_t
    double best = INFINITY;
    for (int k = off_t[s] + lane; k < off_t[s + 1]; k += 64) {
      double d2 = 0.0;
#pragma unroll
      for (int a = 0; a < 3; a++) {
        const double diff = q[a] - static_cast<double>(fix_t[3 * k + a]) * (1.0 / 1024.0);
        d2 = fma(diff, diff, d2);
      }
      best = fmin(best, d2);
    }
    for (int dd = 32; dd >= 1; dd >>= 1) best = fmin(best, __shfl_xor(best, dd, 64));
    sum += best;
    cnt += 1;
  }
  if (lane == 0) {
    wsum[wave] = sum;
    wcnt[wave] = cnt;
    wun[wave] = un;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double total = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
    const int nn = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    f[c] = nn > 0 ? static_cast<float>(total / nn) : __builtin_nanf("");
    unmapped[c] = wun[0] + wun[1] + wun[2] + wun[3];
  }
}

}  // namespace dvf
}  // namespace morea

using namespace morea;

namespace morea {
namespace dvf {

// Owner workspace of the allocation-free DVF entry point: one int32 per
// voxel centre of both grids, 16 MiB, so grids of at most 2,097,152 voxels.
// Every GPU the library runs on holds its own copy until the process ends;
// calls on one GPU share it (calls that overlap on one GPU race), and every
// call clears the part it uses with a kernel first.
constexpr size_t kScratchInts = static_cast<size_t>(1) << 22;
static __device__ __align__(256) int32_t scratch[kScratchInts];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int32_t* g_scratch[kMaxDevices] = {};

}  // namespace dvf

// Device address of the scratch array on the current device (looked up once
// per device, with that device current).  The array's name is only a
// host-side stand-in: kernels get this address.
morea_status static_scratch_init(int device) {
  if (device < 0 || device >= dvf::kMaxDevices) {
    set_error("device index beyond the scratch table");
    return MOREA_EINVAL;
  }
  std::lock_guard<std::mutex> lock(dvf::g_scratch_mu);
  if (dvf::g_scratch[device]) return MOREA_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(dvf::scratch));
  if (e != hipSuccess || !ptr) {
    char buf[256];
    snprintf(buf, sizeof(buf), "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    set_error(buf);
    return MOREA_EDEVICE;
  }
  dvf::g_scratch[device] = static_cast<int32_t*>(ptr);
  return MOREA_OK;
}

}  // namespace morea

namespace {

morea_status launch_dvf(morea_problem* p, const float* cand, float* fwd, float* inv, uint32_t* cover, int32_t* work,
                        hipStream_t s) {
  const ProblemView& P = p->view;
  const size_t V = static_cast<size_t>(P.nx) * P.ny * P.nz;
  const int items = 2 * P.n_tets;
  hipLaunchKernelGGL(dvf::k_dvf_clear, dim3(static_cast<unsigned>((2 * V + 255) / 256)), dim3(256), 0, s, V, work,
                     cover, fwd, inv);
  hipLaunchKernelGGL(dvf::k_dvf_pass<false>, dim3((items + 3) / 4), dim3(256), 0, s, P, cand, work, cover, fwd, inv);
  hipLaunchKernelGGL(dvf::k_dvf_pass<true>, dim3((items + 3) / 4), dim3(256), 0, s, P, cand, work, cover, fwd, inv);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    char buf[256];
    snprintf(buf, sizeof(buf), "DVF rasterization: %s", hipGetErrorString(e));
    set_error(buf);
    return MOREA_EDEVICE;
  }
  return MOREA_OK;
}

}  // namespace

extern "C" morea_status morea_rasterize_dvf_static(morea_problem* p, const float* cand, float* fwd, float* inv,
                                                   uint32_t* cover, void* stream) {
  if (!p || !cand || !fwd || !inv || !cover) {
    set_error("NULL argument");
    return MOREA_EINVAL;
  }
  const ProblemView& P = p->view;
  const size_t V = static_cast<size_t>(P.nx) * P.ny * P.nz;
  if (2 * V > dvf::kScratchInts) {
    char buf[160];
    snprintf(buf, sizeof(buf), "allocation-free DVF: %zu voxels per grid exceed the scratch limit of %zu", V,
             dvf::kScratchInts / 2);
    set_error(buf);
    return MOREA_ERANGE;
  }
  {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      set_error(hipGetErrorString(e));
      return MOREA_EDEVICE;
    }
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    set_error("hipGetDevice failed");
    return MOREA_EDEVICE;
  }
  if (dev < 0 || dev >= dvf::kMaxDevices || !dvf::g_scratch[dev]) {
    // first call on this device (problems created on it normally did this)
    if (morea_status st = static_scratch_init(dev)) return st;
  }
  return launch_dvf(p, cand, fwd, inv, cover, dvf::g_scratch[dev], static_cast<hipStream_t>(stream));
}

extern "C" morea_status morea_rasterize_dvf(morea_problem* p, const float* cand, float* fwd, float* inv,
                                            uint32_t* cover, int32_t* work, void* stream) {
  if (!p || !cand || !fwd || !inv || !cover || !work) {
    set_error("NULL argument");
    return MOREA_EINVAL;
  }
  {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      set_error(hipGetErrorString(e));
      return MOREA_EDEVICE;
    }
  }
  return launch_dvf(p, cand, fwd, inv, cover, work, static_cast<hipStream_t>(stream));
}

extern "C" morea_status morea_point_guidance(morea_problem* p, const float* pts, int32_t pop, float* f,
                                             int32_t* unmapped, void* stream) {
  if (!p || pop < 0) {
    set_error("bad argument");
    return MOREA_EINVAL;
  }
  if (pop == 0) return MOREA_OK;
  if (!pts || !f || !unmapped) {
    set_error("NULL argument");
    return MOREA_EINVAL;
  }
  const ProblemView& P = p->view;
  if (P.n_points > 6144) {
    set_error("point-based guidance keeps a candidate in LDS: at most 6144 points per mesh");
    return MOREA_ERANGE;
  }
  {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      set_error(hipGetErrorString(e));
      return MOREA_EDEVICE;
    }
  }
  const size_t lds = sizeof(int) * 6 * static_cast<size_t>(P.n_points);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(dvf::k_point_guidance),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (e == hipSuccess) {
    hipLaunchKernelGGL(dvf::k_point_guidance, dim3(pop), dim3(256), lds, static_cast<hipStream_t>(stream), P, pts,
                       p->d_set_off[0], p->d_set_fix[0], p->d_set_off[1], p->d_set_fix[1], f, unmapped);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    char buf[256];
    snprintf(buf, sizeof(buf), "point-based guidance: %s", hipGetErrorString(e));
    set_error(buf);
    return MOREA_EDEVICE;
  }
  return MOREA_OK;
}
