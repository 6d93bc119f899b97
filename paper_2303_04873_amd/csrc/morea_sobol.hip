// Sobol-sampled objective evaluation: the paper's own estimator of the
// intensity and guidance terms (App. A.2).  Each tet of each mesh is sampled
// at N random points spread uniformly through its barycentric coordinates,
// N = round(rate * volume); a point takes four numbers r_j of a Sobol
// sequence seeded from the tet's coordinates, lambda_j = -ln r_j / sum_k
// (-ln r_k), and is p = v_0 + sum_{i>=1} lambda_i (v_i - v_0) in the sampled
// tet and q = w_0 + sum_{i>=1} lambda_i (w_i - w_0) in the other mesh's
// tet.  h (Sec. 4.1.2) compares the trilinear values of the two images at p
// and q, with foreground decided on each stencil's exact support; the
// guidance term (Sec. 4.1.3) compares the two distance maps at p and q for
// the sets whose interpolated own distance is below the radius.  Magnitude
// and folds are those of the full evaluation (Sec. 4.1.1, App. A.4).
//
// The sequence: 4 dimensions with 32-bit direction numbers from the
// primitive polynomials 1, x + 1, x^2 + x + 1, x^3 + x + 1 (initial
// numbers (1), (1, 3), (1, 3, 1)), point n in natural order (the XOR of the
// direction numbers of the set bits of n), randomised by a digital shift of
// four words from a SplitMix64 hash of the seed, the direction and the
// tet's 12 fixed-point coordinates.  r_j = (2 floor(u_j / 2^9) + 1) 2^-24.
// -ln is the FP32 atanh series of ln m, m in [sqrt(1/2), sqrt(2)], to s^11.
// The points are formed in FP32 with explicit FMAs and correctly rounded
// divisions, contraction off: which trilinear corners a point's stencil
// supports depends on its bits, and these are the bits the definition
// fixes.
//
// One 64-lane wave per (candidate, tet); both directions in turn; sample n
// of a direction is taken by lane n % 64.  Since lane < 64, the Sobol
// integer of n = 64 k + lane is the XOR of that of the lane (per lane, once
// per direction) and that of 64 k (wave-uniform, scalar, once per batch).
#include <math.h>
#include <stdio.h>

#include "morea_internal.h"

namespace morea {
namespace sobol {

constexpr int kMaxSamples = 1 << 20;          // per tet and direction
constexpr uint64_t kGolden = 0x9e3779b97f4a7c15ull;

struct DirTable {
  uint32_t v[4][32];
};

// Direction numbers V_j[b] = m_{b+1} 2^(31-b), m_k = m_{k-s} XOR
// (XOR over i = 1..s of c_i 2^i m_{k-i}) with c_i the coefficient of
// x^(s-i) of the degree-s primitive polynomial (c_s = 1).
constexpr DirTable make_directions() {
  DirTable t{};
  for (int b = 0; b < 32; b++) t.v[0][b] = 0x80000000u >> b;
  const uint32_t poly[3] = {0x3u, 0x7u, 0xbu};   // x + 1, x^2 + x + 1, x^3 + x + 1
  const int degree[3] = {1, 2, 3};
  const uint64_t first[3][3] = {{1, 0, 0}, {1, 3, 0}, {1, 3, 1}};
  for (int j = 0; j < 3; j++) {
    const int s = degree[j];
    uint64_t m[33] = {};
    for (int k = 1; k <= s; k++) m[k] = first[j][k - 1];
    for (int k = s + 1; k <= 32; k++) {
      uint64_t x = m[k - s];
      for (int i = 1; i <= s; i++)
        if ((poly[j] >> (s - i)) & 1u) x ^= m[k - i] << i;
      m[k] = x;
    }
    for (int b = 0; b < 32; b++) t.v[j + 1][b] = static_cast<uint32_t>(m[b + 1] << (31 - b));
  }
  return t;
}

__constant__ DirTable kDir = make_directions();

__device__ __forceinline__ uint64_t splitmix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ __forceinline__ float wave_sum(float v) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ double wave_sum_d(double v) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// -ln(r) for r in (0, 1]: r = m 2^e, m in [sqrt(1/2), sqrt(2)], ln m =
// 2 atanh(s) with s = (m - 1) / (m + 1) and the series s (1 + s^2/3 + ... +
// s^10/11).
__device__ __forceinline__ float neg_log(float r) {
#pragma clang fp contract(off)
  const uint32_t u = __float_as_uint(r);
  int e = static_cast<int>(u >> 23) - 127;
  float m = __uint_as_float((u & 0x007fffffu) | 0x3f800000u);
  if (m > 0x1.6a09e6p+0f) {
    m = m * 0.5f;
    e = e + 1;
  }
  const float s = (m - 1.0f) / (m + 1.0f);
  const float s2 = s * s;
  float c = __builtin_fmaf(s2, 0x1.745d18p-4f, 0x1.c71c72p-4f);
  c = __builtin_fmaf(s2, c, 0x1.24924ap-3f);
  c = __builtin_fmaf(s2, c, 0x1.99999ap-3f);
  c = __builtin_fmaf(s2, c, 0x1.555556p-2f);
  c = __builtin_fmaf(s2, c, 1.0f);
  const float ln_m = (s + s) * c;
  return -__builtin_fmaf(static_cast<float>(e), 0x1.62e430p-1f, ln_m);
}

template <int ST>
__device__ __forceinline__ float ld(const void* base, int idx) {
  if constexpr (ST == kF32) {
    return static_cast<const float*>(base)[idx];
  } else if constexpr (ST == kBF16) {
    return __uint_as_float(static_cast<uint32_t>(static_cast<const uint16_t*>(base)[idx]) << 16);
  } else {
    return static_cast<float>(static_cast<const _Float16*>(base)[idx]);
  }
}

// Trilinear value and exact-support foreground of an image (zero padding) at
// an FP32 point in grid coordinates.
template <int ST>
__device__ __forceinline__ float image_at(const ProblemView& P, const void* img, const uint8_t* fgc, float x,
                                          float y, float z, bool& fg) {
  const float kx = floorf(x), ky = floorf(y), kz = floorf(z);
  const float fx = x - kx, fy = y - ky, fz = z - kz;
  const int ix = static_cast<int>(kx), iy = static_cast<int>(ky), iz = static_cast<int>(kz);
  fg = false;
  // both corners of an axis lie outside the grid when k <= -2 or k >= n
  if (kx < -1.f || ky < -1.f || kz < -1.f || ix > P.nx - 1 || iy > P.ny - 1 || iz > P.nz - 1) return 0.f;
  const int i0 = (iz + 1) * P.pxy + (iy + 1) * P.px + ix + 1;
  // a cell without a positive corner is background whatever the support
  const unsigned code = fgc[i0];
  if (!(code & 1u)) return 0.f;
  const int i1 = i0 + P.pxy;
  const float c000 = ld<ST>(img, i0), c100 = ld<ST>(img, i0 + 1);
  const float c010 = ld<ST>(img, i0 + P.px), c110 = ld<ST>(img, i0 + P.px + 1);
  const float c001 = ld<ST>(img, i1), c101 = ld<ST>(img, i1 + 1);
  const float c011 = ld<ST>(img, i1 + P.px), c111 = ld<ST>(img, i1 + P.px + 1);
  if (code & 2u) {
    fg = true;    // every corner is positive, so is every supported one
  } else {
    const bool ux = fx > 0.f, uy = fy > 0.f, uz = fz > 0.f;
    const bool f0 = c000 > 0.f || (ux && c100 > 0.f) || (uy && c010 > 0.f) || (ux && uy && c110 > 0.f);
    const bool f1 = c001 > 0.f || (ux && c101 > 0.f) || (uy && c011 > 0.f) || (ux && uy && c111 > 0.f);
    fg = f0 || (uz && f1);
    if (!fg) return 0.f;
  }
  const float x00 = fmaf(fx, c100 - c000, c000), x10 = fmaf(fx, c110 - c010, c010);
  const float x01 = fmaf(fx, c101 - c001, c001), x11 = fmaf(fx, c111 - c011, c011);
  const float y0 = fmaf(fy, x10 - x00, x00), y1 = fmaf(fy, x11 - x01, x01);
  return fmaf(fz, y1 - y0, y0);
}

// Stencil of a distance map (edge clamping): the point clamped into
// [0, n - 1] per axis, the cell below it capped at n - 2 (at 0 for n = 1),
// its first padded element and fractions.
struct MapCell {
  int i0;
  float fx, fy, fz;
};

__device__ __forceinline__ MapCell map_cell(const ProblemView& P, float x, float y, float z) {
  const float cx = fminf(fmaxf(x, 0.f), static_cast<float>(P.nx - 1));
  const float cy = fminf(fmaxf(y, 0.f), static_cast<float>(P.ny - 1));
  const float cz = fminf(fmaxf(z, 0.f), static_cast<float>(P.nz - 1));
  const int ix = max(min(static_cast<int>(floorf(cx)), P.nx - 2), 0);
  const int iy = max(min(static_cast<int>(floorf(cy)), P.ny - 2), 0);
  const int iz = max(min(static_cast<int>(floorf(cz)), P.nz - 2), 0);
  return MapCell{(iz + 1) * P.pxy + (iy + 1) * P.px + ix + 1, cx - static_cast<float>(ix),
                 cy - static_cast<float>(iy), cz - static_cast<float>(iz)};
}

__device__ __forceinline__ float map_at(const ProblemView& P, const float* m, const MapCell& c) {
  const int i0 = c.i0, i1 = c.i0 + P.pxy;
  const float x00 = fmaf(c.fx, m[i0 + 1] - m[i0], m[i0]);
  const float x10 = fmaf(c.fx, m[i0 + P.px + 1] - m[i0 + P.px], m[i0 + P.px]);
  const float x01 = fmaf(c.fx, m[i1 + 1] - m[i1], m[i1]);
  const float x11 = fmaf(c.fx, m[i1 + P.px + 1] - m[i1 + P.px], m[i1 + P.px]);
  const float y0 = fmaf(c.fy, x10 - x00, x00), y1 = fmaf(c.fy, x11 - x01, x01);
  return fmaf(c.fz, y1 - y0, y0);
}

// 6 x signed volume of snapped vertices (exact: coordinates below 2^19).
__device__ __forceinline__ int64_t det6(const int v[4][3]) {
  const int64_t a0 = v[1][0] - v[0][0], a1 = v[1][1] - v[0][1], a2 = v[1][2] - v[0][2];
  const int64_t b0 = v[2][0] - v[0][0], b1 = v[2][1] - v[0][1], b2 = v[2][2] - v[0][2];
  const int64_t c0 = v[3][0] - v[0][0], c1 = v[3][1] - v[0][1], c2 = v[3][2] - v[0][2];
  return a0 * (b1 * c2 - b2 * c1) - a1 * (b0 * c2 - b2 * c0) + a2 * (b0 * c1 - b1 * c0);
}

// Blocks of 4 waves; each XCD (blocks dealt round-robin) gets one contiguous
// range of items, so neighbouring tets share its L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb / 8, rem = nb % 8;
  const int x = b % 8, pos = b / 8;
  return x < rem ? x * (q + 1) + pos : rem * (q + 1) + (x - rem) * q + pos;
}

template <int ST>
__global__ __launch_bounds__(256, 6) void k_eval_sobol(ProblemView P, const float* pts, int pop, double inv_pop,
                                                  double count_scale, uint64_t seed, const uint8_t* cells0,
                                                  const uint8_t* cells1, const uint8_t* fgc0, const uint8_t* fgc1,
                                                  Record* rec, int n_items) {
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int item = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
  if (item >= n_items) return;
  int tet = static_cast<int>(static_cast<double>(item) * inv_pop);
  int cand = item - tet * pop;
  if (cand < 0) {
    tet -= 1;
    cand += pop;
  } else if (cand >= pop) {
    tet += 1;
    cand -= pop;
  }
  tet = __builtin_amdgcn_readfirstlane(tet);
  cand = __builtin_amdgcn_readfirstlane(cand);
  const int lane = lane_id();
  Record* out = rec + (static_cast<size_t>(cand) * P.n_tets + tet) * 2;

  // snap (lane l < 24: mesh l / 12, vertex (l % 12) / 3, axis l % 3)
  const int4 tv = P.tets[tet];
  float coord = 0.f;
  if (lane < 24) {
    const int i = (lane % 12) / 3, k = lane % 3;
    const int v = i == 0 ? tv.x : (i == 1 ? tv.y : (i == 2 ? tv.z : tv.w));
    coord = pts[((static_cast<size_t>(cand) * 2 + lane / 12) * 3 + k) * P.n_points + v];
  }
  const bool ok = lane >= 24 || fabsf(coord) < kCoordLimit;
  if (__ballot(ok) != ~0ull) {
    if (lane < 2) out[lane] = Record{0.f, 0.f, 0u, 0.f, 0.f, 4u};
    return;
  }
  // snapped coordinate of lane l < 24: mesh l / 12, vertex (l % 12) / 3, axis l % 3
  const int fix = lane < 24 ? static_cast<int>(rintf(coord * kFixOne)) : 0;

  // magnitude (Sec. 4.1.1): lane e < 10 takes edge e (6 edges, then the 4
  // spokes from the centroid), squared lengths exact in FP64
  double term = 0.0;
  {
    const int e = lane < 10 ? lane : 0;
    const int va = e < 3 ? 0 : (e < 5 ? 1 : (e < 6 ? 2 : e - 6));
    const int vb = e < 3 ? e + 1 : (e < 5 ? e - 1 : 3);
    double ls = 0.0, lt = 0.0;
#pragma unroll
    for (int k = 0; k < 3; k++) {
      const int sa = __shfl(fix, 3 * va + k, 64), sb = __shfl(fix, 3 * vb + k, 64);
      const int ta = __shfl(fix, 12 + 3 * va + k, 64), tb = __shfl(fix, 12 + 3 * vb + k, 64);
      double ds, dt;
      if (e < 6) {
        ds = static_cast<double>(sa - sb);
        dt = static_cast<double>(ta - tb);
      } else {   // 4 v_a - (v_0 + v_1 + v_2 + v_3), exact
        const int ss = __builtin_amdgcn_readlane(fix, k) + __builtin_amdgcn_readlane(fix, 3 + k) +
                       __builtin_amdgcn_readlane(fix, 6 + k) + __builtin_amdgcn_readlane(fix, 9 + k);
        const int st = __builtin_amdgcn_readlane(fix, 12 + k) + __builtin_amdgcn_readlane(fix, 15 + k) +
                       __builtin_amdgcn_readlane(fix, 18 + k) + __builtin_amdgcn_readlane(fix, 21 + k);
        ds = 4.0 * sa - ss;
        dt = 4.0 * ta - st;
      }
      ls = fma(ds, ds, ls);
      lt = fma(dt, dt, lt);
    }
    if (lane < 10) {
      const double den = sqrt(ls) + sqrt(lt);
      const double d = den > 0.0 ? (ls - lt) / den * (e < 6 ? 1.0 / 1024.0 : 1.0 / 4096.0) : 0.0;
      term = d * d;
    }
  }
  const float mag = static_cast<float>(static_cast<double>(P.elasticity[tet]) * wave_sum_d(term));

  // shift words of both directions: lane d < 2 hashes direction d's tet
  uint64_t w0 = 0, w1 = 0;
  {
    const int m = lane < 2 ? lane : 0;
    uint64_t hsh = splitmix(seed + kGolden * static_cast<uint64_t>(m + 1));
#pragma unroll
    for (int i = 0; i < 12; i++) {
      const int c = __shfl(fix, 12 * m + i, 64);
      hsh = splitmix(hsh + kGolden + static_cast<uint64_t>(static_cast<uint32_t>(c)));
    }
    w0 = splitmix(hsh + kGolden);
    w1 = splitmix(hsh + 2 * kGolden);
  }
  const int ref = P.ref_sign[tet];

#pragma unroll 1
  for (int d = 0; d < 2; d++) {
    // the sampled tet and the other one (wave-uniform)
    int own[4][3], oth[4][3];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
      for (int k = 0; k < 3; k++) {
        own[i][k] = __builtin_amdgcn_readlane(fix, 12 * d + 3 * i + k);
        oth[i][k] = __builtin_amdgcn_readlane(fix, 12 * (1 - d) + 3 * i + k);
      }
    const int64_t D = det6(own);
    const int sg = (D > 0) - (D < 0);
    const bool viol = sg == 0 || sg != ref;
    const int64_t absD = D < 0 ? -D : D;
    const float vol = viol ? static_cast<float>(static_cast<double>(absD) * (1.0 / 6442450944.0)) : 0.f;
    int N = 0;
    if (D != 0) {
      const double x = floor(static_cast<double>(absD) * count_scale + 0.5);
      N = x > 0.0 ? (x >= kMaxSamples ? kMaxSamples : static_cast<int>(x)) : 0;
    }
    float h = 0.f, g = 0.f;
    if (N > 0) {
      // this lane's Sobol integers (its 6 low bits) with the shift applied
      const uint32_t s0 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<uint32_t>(w0), d));
      const uint32_t s1 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<uint32_t>(w0 >> 32), d));
      const uint32_t s2 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<uint32_t>(w1), d));
      const uint32_t s3 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<uint32_t>(w1 >> 32), d));
      uint32_t xl[4] = {s0, s1, s2, s3};
#pragma unroll
      for (int b = 0; b < 6; b++)
        if ((lane >> b) & 1)
#pragma unroll
          for (int j = 0; j < 4; j++) xl[j] ^= kDir.v[j][b];
      // FP32 base vertex and edge vectors of both tets, in voxels (exact)
      float bo[3], eo[3][3], bt[3], et[3][3];
#pragma unroll
      for (int a = 0; a < 3; a++) {
        bo[a] = static_cast<float>(own[0][a]) * 0x1p-10f;
        bt[a] = static_cast<float>(oth[0][a]) * 0x1p-10f;
#pragma unroll
        for (int i = 0; i < 3; i++) {
          eo[i][a] = static_cast<float>(own[i + 1][a] - own[0][a]) * 0x1p-10f;
          et[i][a] = static_cast<float>(oth[i + 1][a] - oth[0][a]) * 0x1p-10f;
        }
      }
      const void* img_own = d == 0 ? P.img[0] : P.img[1];
      const void* img_oth = d == 0 ? P.img[1] : P.img[0];
      const uint8_t* cells = d == 0 ? cells0 : cells1;
      const uint8_t* fgc_own = d == 0 ? fgc0 : fgc1;
      const uint8_t* fgc_oth = d == 0 ? fgc1 : fgc0;
      const float* map_own = d == 0 ? P.dmap[0] : P.dmap[1];
      const float* map_oth = d == 0 ? P.dmap[1] : P.dmap[0];
      const float* set_w = P.set_w + d * kMaxSets;
      for (int base = 0; base < N; base += kWave) {
        // Sobol integers of 64 k (wave-uniform)
        uint32_t xk[4] = {0u, 0u, 0u, 0u};
        for (uint32_t t = static_cast<uint32_t>(base) >> 6; t != 0u; t &= t - 1u) {
          const int b = __builtin_ctz(t) + 6;
#pragma unroll
          for (int j = 0; j < 4; j++) xk[j] ^= kDir.v[j][b];
        }
        if (base + lane >= N) break;
        float p[3], q[3];
        {
#pragma clang fp contract(off)
          float e[4];
#pragma unroll
          for (int j = 0; j < 4; j++) {
            const uint32_t u = xl[j] ^ xk[j];
            e[j] = neg_log(static_cast<float>(2u * (u >> 9) + 1u) * 0x1p-24f);
          }
          const float sum = ((e[0] + e[1]) + e[2]) + e[3];
          const float l1 = e[1] / sum, l2 = e[2] / sum, l3 = e[3] / sum;
#pragma unroll
          for (int a = 0; a < 3; a++) {
            p[a] = __builtin_fmaf(l3, eo[2][a], __builtin_fmaf(l2, eo[1][a], __builtin_fmaf(l1, eo[0][a], bo[a])));
            q[a] = __builtin_fmaf(l3, et[2][a], __builtin_fmaf(l2, et[1][a], __builtin_fmaf(l1, et[0][a], bt[a])));
          }
        }
        bool fa, fb;
        const float a = image_at<ST>(P, img_own, fgc_own, p[0], p[1], p[2], fa);
        const float b = image_at<ST>(P, img_oth, fgc_oth, q[0], q[1], q[2], fb);
        h += (fa && fb) ? (a - b) * (a - b) : (fa == fb ? 0.f : 1.f);
        if (P.n_sets > 0) {
          const MapCell cp = map_cell(P, p[0], p[1], p[2]);
          // sets within the radius at one of the stencil's corners (if at
          // none, the interpolated distance is not below it either)
          unsigned bits = cells[cp.i0];
          if (bits) {
            const MapCell cq = map_cell(P, q[0], q[1], q[2]);
            for (; bits; bits &= bits - 1u) {
              const int s = __builtin_ctz(bits);
              const float dn = map_at(P, map_own + static_cast<size_t>(s) * P.pvox, cp);
              if (dn < P.radius) {
                const float dq = map_at(P, map_oth + static_cast<size_t>(s) * P.pvox, cq);
                const float diff = dn - dq;
                g = fmaf(set_w[s] * (P.radius - dn) * P.inv_radius, diff * diff, g);
              }
            }
          }
        }
      }
      h = wave_sum(h);
      g = wave_sum(g);
    }
    if (lane == 0)
      out[d] = Record{h, g, static_cast<uint32_t>(N), d == 0 ? mag : 0.f, vol, viol ? 1u : 0u};
  }
}

// Band mask per grid cell (lower corner at padded element i): the OR of the
// band bytes of its 8 corners; elements that are no cell's lower corner hold 0.
__global__ void k_band_cells(ProblemView P, const uint8_t* band, uint8_t* cells) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= static_cast<int>(P.pvox)) return;
  const int x = i % P.px - 1, y = (i / P.px) % (P.ny + 2) - 1, z = i / P.pxy - 1;
  uint8_t v = 0;
  if (x >= 0 && y >= 0 && z >= 0 && x <= max(P.nx - 2, 0) && y <= max(P.ny - 2, 0) && z <= max(P.nz - 2, 0)) {
    const int j = i + P.pxy;
    v = band[i] | band[i + 1] | band[i + P.px] | band[i + P.px + 1] | band[j] | band[j + 1] | band[j + P.px] |
        band[j + P.px + 1];
  }
  cells[i] = v;
}

morea_status fail(morea_status s, const char* msg) {
  set_error(msg);
  return s;
}

morea_status device_fail(hipError_t e, const char* what) {
  char buf[256];
  snprintf(buf, sizeof(buf), "%s: %s", what, hipGetErrorString(e));
  set_error(buf);
  return MOREA_EDEVICE;
}

// Foreground code per cell (lower corner at padded element i): bit 0 when a
// corner of the cell holds a value > 0, bit 1 when all eight do.
template <int ST>
__global__ void k_fg_cells(ProblemView P, const void* img, uint8_t* cells) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= static_cast<int>(P.pvox)) return;
  const int x = i % P.px, y = (i / P.px) % (P.ny + 2), z = i / P.pxy;
  uint8_t v = 0;
  if (x + 1 < P.px && y + 1 < P.ny + 2 && z + 1 < P.nz + 2) {
    const int j = i + P.pxy;
    const int idx[8] = {i, i + 1, i + P.px, i + P.px + 1, j, j + 1, j + P.px, j + P.px + 1};
    bool any = false, all = true;
#pragma unroll
    for (int k = 0; k < 8; k++) {
      const bool pos = ld<ST>(img, idx[k]) > 0.f;
      any = any || pos;
      all = all && pos;
    }
    v = static_cast<uint8_t>((any ? 1 : 0) | (all ? 2 : 0));
  }
  cells[i] = v;
}

}  // namespace sobol

hipError_t launch_fg_cells(const ProblemView& P, int storage, const void* img, uint8_t* cells, hipStream_t s) {
  const dim3 grid((P.pvox + 255) / 256);
  switch (storage) {
    case kF32: hipLaunchKernelGGL(sobol::k_fg_cells<kF32>, grid, dim3(256), 0, s, P, img, cells); break;
    case kBF16: hipLaunchKernelGGL(sobol::k_fg_cells<kBF16>, grid, dim3(256), 0, s, P, img, cells); break;
    default: hipLaunchKernelGGL(sobol::k_fg_cells<kF16>, grid, dim3(256), 0, s, P, img, cells); break;
  }
  return hipGetLastError();
}

hipError_t launch_band_cells(const ProblemView& P, const uint8_t* band, uint8_t* cells, hipStream_t s) {
  hipLaunchKernelGGL(sobol::k_band_cells, dim3((P.pvox + 255) / 256), dim3(256), 0, s, P, band, cells);
  return hipGetLastError();
}

}  // namespace morea

using namespace morea;

extern "C" morea_status morea_eval_sobol(morea_problem* p, const float* pts, int32_t pop, float rate,
                                         uint64_t seed, float* obj, uint8_t* flags, float* severity,
                                         uint32_t* counts, void* stream) {
  if (!p) return sobol::fail(MOREA_EINVAL, "problem is NULL");
  if (pop < 0) return sobol::fail(MOREA_EINVAL, "pop < 0");
  if (pop > p->max_population) return sobol::fail(MOREA_ERANGE, "pop above max_population");
  if (!(rate > 0.f) || !(rate < INFINITY)) return sobol::fail(MOREA_EINVAL, "rate must be finite and > 0");
  if (pop == 0) return MOREA_OK;
  if (!pts || !obj || !flags || !severity || !counts) return sobol::fail(MOREA_EINVAL, "NULL argument");
  {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return sobol::device_fail(e, "earlier device work failed");
  }
  const ProblemView& P = p->view;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t n_items = static_cast<size_t>(pop) * P.n_tets;
  if (n_items > 0) {
    const int blocks = static_cast<int>((n_items + 3) / 4);
    const double count_scale = static_cast<double>(rate) / 6442450944.0;   // rate / (6 * 2^30)
    const double inv_pop = 1.0 / pop;
    switch (p->storage) {
      case kF32:
        hipLaunchKernelGGL(sobol::k_eval_sobol<kF32>, dim3(blocks), dim3(256), 0, s, P, pts, pop, inv_pop,
                           count_scale, seed, p->band_cell[0], p->band_cell[1], p->fg_cell[0], p->fg_cell[1],
                           p->work_records,
                           static_cast<int>(n_items));
        break;
      case kBF16:
        hipLaunchKernelGGL(sobol::k_eval_sobol<kBF16>, dim3(blocks), dim3(256), 0, s, P, pts, pop, inv_pop,
                           count_scale, seed, p->band_cell[0], p->band_cell[1], p->fg_cell[0], p->fg_cell[1],
                           p->work_records,
                           static_cast<int>(n_items));
        break;
      default:
        hipLaunchKernelGGL(sobol::k_eval_sobol<kF16>, dim3(blocks), dim3(256), 0, s, P, pts, pop, inv_pop,
                           count_scale, seed, p->band_cell[0], p->band_cell[1], p->fg_cell[0], p->fg_cell[1],
                           p->work_records,
                           static_cast<int>(n_items));
        break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return sobol::device_fail(e, "Sobol evaluation");
  }
  hipError_t e = launch_finalize(P, pts, pop, p->work_records, obj, flags, severity, counts, nullptr, s);
  if (e != hipSuccess) return sobol::device_fail(e, "Sobol evaluation");
  return MOREA_OK;
}
