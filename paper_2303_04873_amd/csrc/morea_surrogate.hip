// Learned pre-screen of offspring: a per-tetrahedron multilayer perceptron
// 23 -> 128 -> 128 -> 1 (ReLU) that predicts how an offspring's mean
// intensity term of a tet (the sum of h over the tet's samples in both
// directions divided by their number, Sec. 4.1.2) differs from its parent's,
// from how the tet's vertices moved away from the parent's, the tet's region
// statistics, the parent's exact term and samples of the target image.
// Trained on records produced by the exact evaluator for offspring and
// parents; a batch of offspring is ranked by the parent's exact terms plus
// the predicted changes before only the best are evaluated exactly.  The
// surrogate has no counterpart in the paper; it sits in front of the exact
// evaluation, which stays the judge of every selected candidate.
//
// Dense layers run on the matrix cores: v_mfma_f32_32x32x8_bf16 with BF16
// operands and FP32 accumulation, one 64-lane wave per tile of 32 rows.
// Lane l holds row (A) / column (B) l % 32 and the k-quad 4 * (l / 32);
// accumulator element r of lane l is row 8 (r / 4) + 4 (l / 32) + r % 4,
// column l % 32.  Master weights, gradients and the Adam state are FP32.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <random>
#include <string>
#include <vector>

#include "morea_internal.h"

namespace morea {
namespace surr {

constexpr int kIn = 23, kInPad = 24, kHid = 128;
constexpr int oW1 = 0, oB1 = oW1 + kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid,
              oW3 = oB2 + kHid, oB3 = oW3 + kHid, kParams = oB3 + 1;   // 19,713
constexpr int kRowTile = 32;
constexpr int kWavePart = 3 * kHid + 2;   // per-wave partials: dw3, db2, db1, db3, loss
constexpr int kSplitK = 16;
constexpr int kGradTiles = 20;            // 16 tiles of W2, 4 of W1

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef unsigned short bf16;

__device__ __forceinline__ bf16 f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<bf16>(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16 b) { return __uint_as_float(static_cast<uint32_t>(b) << 16); }
__device__ __forceinline__ s4 ld4(const bf16* p) { return *reinterpret_cast<const s4*>(p); }
__device__ __forceinline__ f16v mma(s4 a, s4 b, f16v c) {
  return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ int acc_row(int r, int kh) { return 8 * (r >> 2) + 4 * kh + (r & 3); }
__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Weights staged in LDS by every block that runs the network.
struct alignas(16) NetLds {
  bf16 w1[kHid][kInPad];   // W1[j][k], k padded with zeros
  bf16 w2[kHid][kHid];     // W2[j][k]
  float b1[kHid], b2[kHid], w3[kHid];
  float b3;
};

// Per-wave tile buffers.  For inference the output reduction reuses the
// layer-1 activations' space (dead once layer 2 has consumed them).
typedef float RedTile[kRowTile][kRowTile + 1];
struct alignas(16) TileLds {
  bf16 x[kRowTile][kInPad];
  union {
    bf16 h1[kRowTile][kHid];
    RedTile red;
  };
  float y[kRowTile];
};

__device__ void load_net(NetLds* N, const bf16* w1b, const bf16* w2b, const float* params) {
  for (int i = threadIdx.x; i < kHid * kInPad; i += blockDim.x) (&N->w1[0][0])[i] = w1b[i];
  for (int i = threadIdx.x; i < kHid * kHid / 4; i += blockDim.x)
    reinterpret_cast<s4*>(&N->w2[0][0])[i] = reinterpret_cast<const s4*>(w2b)[i];
  for (int i = threadIdx.x; i < kHid; i += blockDim.x) {
    N->b1[i] = params[oB1 + i];
    N->b2[i] = params[oB2 + i];
    N->w3[i] = params[oW3 + i];
  }
  if (threadIdx.x == 0) N->b3 = params[oB3];
}

// Forward pass of one tile of 32 rows (T->x filled).  Leaves relu(z1) in
// T->h1 (BF16) unless `red` overlays it, returns the layer-2
// pre-activations (4 column tiles) in z2 and writes y to T->y.
__device__ void tile_forward(const NetLds* N, TileLds* T, RedTile& red, f16v z2[4]) {
  const int lane = lane_id(), i = lane & 31, kh = lane >> 5;
#pragma unroll
  for (int n = 0; n < 4; n++) {
    f16v acc = {};
#pragma unroll
    for (int s = 0; s < kInPad / 8; s++)
      acc = mma(ld4(&T->x[i][8 * s + 4 * kh]), ld4(&N->w1[32 * n + i][8 * s + 4 * kh]), acc);
    const float bias = N->b1[32 * n + i];
#pragma unroll
    for (int r = 0; r < 16; r++) T->h1[acc_row(r, kh)][32 * n + i] = f2bf(fmaxf(acc[r] + bias, 0.f));
  }
  wave_sync();
  float part[16];
#pragma unroll
  for (int r = 0; r < 16; r++) part[r] = 0.f;
#pragma unroll
  for (int n = 0; n < 4; n++) {
    f16v acc = {};
#pragma unroll
    for (int s = 0; s < kHid / 8; s++)
      acc = mma(ld4(&T->h1[i][8 * s + 4 * kh]), ld4(&N->w2[32 * n + i][8 * s + 4 * kh]), acc);
    const float bias = N->b2[32 * n + i], w = N->w3[32 * n + i];
#pragma unroll
    for (int r = 0; r < 16; r++) {
      acc[r] += bias;
      part[r] = fmaf(fmaxf(acc[r], 0.f), w, part[r]);
    }
    z2[n] = acc;
  }
  // y[row] = sum over the 128 columns: this lane holds column i of 16 rows
  wave_sync();
#pragma unroll
  for (int r = 0; r < 16; r++) red[acc_row(r, kh)][i] = part[r];
  wave_sync();
  if (lane < kRowTile) {
    float y = N->b3;
    for (int c = 0; c < kRowTile; c++) y += red[lane][c];
    T->y[lane] = y;
  }
  wave_sync();
}

// ------------------------------------------------------------- features

// Features of (offspring, tet), relative to the offspring's parent (whose
// exact evaluation is known: its per-tet records are in its cache):
//   0..11  the move of the tet's 4 target-mesh vertices from the parent's,
//          (T_v - T_parent,v) / 0.5 voxel (the scale of the offspring's
//          perturbation, well resolved in BF16);
//   12..14 estimates of the change of the tet's mean intensity term, each
//          the mean of h = (I_s(x) - I_t(y))^2 over a fixed set of points of
//          the tet, x and y at the same barycentric coordinates in the
//          offspring's source and target tets, minus the same mean for the
//          parent: over the 4 vertices, the 6 edge midpoints, and 16
//          interior points (Halton points in barycentric form); divided by
//          h_scale;
//   15..21 the first 7 of the tet's 8 source-region statistics, the 7th
//          (the mean of (I_s - I_t)^2) divided by h_scale;
//   22     the parent's exact mean intensity term of the tet, (h_S + h_T) /
//          (n_S + n_T) from its records (0 without samples), divided by
//          h_scale.
// h_scale is the mean of (I_s - I_t)^2 over the grid's voxels (1 when that is
// 0), so that the h-valued features and the targets are of order 1.  Image
// values are trilinear interpolants at the point clamped into the image box,
// so every feature is continuous in the vertex positions.
constexpr float kRelScale = 2.0f;
constexpr int kHalton = 16;

// The parents of a batch of offspring: points [n][2][3][n_points], per-tet
// records of their full evaluation [n][n_tets][2], the parent of each
// offspring.
struct Parents {
  const float* pts;
  const Record* rec;
  const int* of;
  int n;
};

// Trilinear interpolant at (x, y, z) clamped into [0, n - 1] on each axis,
// from a quad copy `q` of a padded image (entry e holds the FP32 voxels e,
// e + 1, e + px, e + px + 1 of the padded volume, voxel (i, j, k) at
// (k + 1) pxy + (j + 1) px + i + 1), so a sample reads two aligned 16-byte
// entries instead of eight scattered values.  The cell is the one below the
// point, capped at n - 2, so the upper corner always lies in the volume or,
// for an axis of size 1, on its zero border with weight 0.
__device__ __forceinline__ float sample_clamped(const ProblemView& P, const float4* q, float x, float y, float z) {
  const float p[3] = {fminf(fmaxf(x, 0.f), static_cast<float>(P.nx - 1)),
                      fminf(fmaxf(y, 0.f), static_cast<float>(P.ny - 1)),
                      fminf(fmaxf(z, 0.f), static_cast<float>(P.nz - 1))};
  const int n[3] = {P.nx, P.ny, P.nz};
  int c[3];
  float f[3];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    c[a] = max(min(static_cast<int>(floorf(p[a])), n[a] - 2), 0);
    f[a] = p[a] - static_cast<float>(c[a]);
  }
  const size_t e = static_cast<size_t>(c[2] + 1) * P.pxy + static_cast<size_t>(c[1] + 1) * P.px + c[0] + 1;
  const float4 b = q[e], b1 = q[e + P.pxy];
  const float x00 = fmaf(f[0], b.y - b.x, b.x), x10 = fmaf(f[0], b.w - b.z, b.z);
  const float x01 = fmaf(f[0], b1.y - b1.x, b1.x), x11 = fmaf(f[0], b1.w - b1.z, b1.z);
  const float y0 = fmaf(f[1], x10 - x00, x00), y1 = fmaf(f[1], x11 - x01, x01);
  return fmaf(f[2], y1 - y0, y0);
}

// A tet's vertices in one candidate: mesh 0 (source) or 1 (target).
__device__ __forceinline__ void tet_vertices(const ProblemView& P, const float* cand, int tet, int mesh,
                                             float d[4][3]) {
  const int4 tv = P.tets[tet];
  const int vs[4] = {tv.x, tv.y, tv.z, tv.w};
#pragma unroll
  for (int v = 0; v < 4; v++)
#pragma unroll
    for (int a = 0; a < 3; a++) d[v][a] = cand[(3 * mesh + a) * P.n_points + vs[v]];
}

// h at barycentric coordinates l of the tet: (I_s(S l) - I_t(T l))^2.
__device__ __forceinline__ float h_at(const ProblemView& P, const float4* img_s, const float4* img_t,
                                      const float S[4][3], const float T[4][3], const float l[4]) {
  float x[3], y[3];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    x[a] = fmaf(l[0], S[0][a], fmaf(l[1], S[1][a], fmaf(l[2], S[2][a], l[3] * S[3][a])));
    y[a] = fmaf(l[0], T[0][a], fmaf(l[1], T[1][a], fmaf(l[2], T[2][a], l[3] * T[3][a])));
  }
  const float d = sample_clamped(P, img_s, x[0], x[1], x[2]) - sample_clamped(P, img_t, y[0], y[1], y[2]);
  return d * d;
}

// Sums of h over points [j0, j1) of a tet's 26 (the 4 vertices, the edge
// midpoints (0,1) (0,2) (0,3) (1,2) (1,3) (2,3), then the 16 interior points
// `bary`) into acc: [0] vertices, [1] edges, [2] interior.  One point at a
// time.
__device__ __forceinline__ void point_sums(const ProblemView& P, const float4* img_s, const float4* img_t,
                                           const float S[4][3], const float T[4][3], const float4* bary, int j0,
                                           int j1, float acc[3]) {
  acc[0] = acc[1] = acc[2] = 0.f;
#pragma unroll 1
  for (int j = j0; j < j1; j++) {
    float l[4] = {0.f, 0.f, 0.f, 0.f};
    if (j < 4) {
      l[0] = j == 0 ? 1.f : 0.f;
      l[1] = j == 1 ? 1.f : 0.f;
      l[2] = j == 2 ? 1.f : 0.f;
      l[3] = j == 3 ? 1.f : 0.f;
    } else if (j < 10) {
      const int e = j - 4, a = e < 3 ? 0 : (e < 5 ? 1 : 2), b = e < 3 ? e + 1 : (e < 5 ? e - 1 : 3);
#pragma unroll
      for (int v = 0; v < 4; v++) l[v] = (v == a || v == b) ? .5f : 0.f;
    } else {
      const float4 q = bary[j - 10];
      l[0] = q.x;
      l[1] = q.y;
      l[2] = q.z;
      l[3] = q.w;
    }
    const float hv = h_at(P, img_s, img_t, S, T, l);
    acc[j < 4 ? 0 : (j < 10 ? 1 : 2)] += hv;
  }
}

// The points are summed in two parts, [0, 13) and [13, 26), added at the end:
// the pre-screen splits them over two lane halves in the same way, so both
// paths give the same values.
constexpr int kPointSplit = 13, kPoints = 10 + kHalton;

__device__ __forceinline__ void combine_means(const float a[3], const float b[3], float m[3]) {
  m[0] = (a[0] + b[0]) * 0.25f;
  m[1] = (a[1] + b[1]) * (1.f / 6.f);
  m[2] = (a[2] + b[2]) * (1.f / kHalton);
}

// Means of h over the tet's point sets in one candidate: m[0] the 4
// vertices, m[1] the 6 edge midpoints, m[2] the 16 interior points.
__device__ __forceinline__ void point_means(const ProblemView& P, const float4* img_s, const float4* img_t,
                                            const float* cand, int tet, const float4* bary, float m[3]) {
  float S[4][3], T[4][3];
  tet_vertices(P, cand, tet, 0, S);
  tet_vertices(P, cand, tet, 1, T);
  float a[3], b[3];
  point_sums(P, img_s, img_t, S, T, bary, 0, kPointSplit, a);
  point_sums(P, img_s, img_t, S, T, bary, kPointSplit, kPoints, b);
  combine_means(a, b, m);
}

// |signed volume| of a tet's source and target (voxel^3): the expected
// samples of the tet in both directions.
__device__ __forceinline__ float tet_weight(const ProblemView& P, const float* cand, int tet) {
  float w = 0.f;
#pragma unroll
  for (int mesh = 0; mesh < 2; mesh++) {
    float d[4][3];
    tet_vertices(P, cand, tet, mesh, d);
    float e[3][3];
#pragma unroll
    for (int k = 0; k < 3; k++)
#pragma unroll
      for (int a = 0; a < 3; a++) e[k][a] = d[k + 1][a] - d[0][a];
    const float det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                      e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                      e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
    w += fabsf(det) * (1.f / 6.f);
  }
  return w;
}

// Mean intensity term per sample of a tet over both directions, from its
// two records.
__device__ __forceinline__ float tet_mean_h(const Record* rec, int tet) {
  const Record a = rec[2 * static_cast<size_t>(tet)], b = rec[2 * static_cast<size_t>(tet) + 1];
  const uint32_t n = a.n + b.n;
  return n ? (a.h + b.h) / static_cast<float>(n) : 0.f;
}

// Value of stored voxel e of image `which` as FP32 (0 beyond the volume).
template <int ST>
__device__ __forceinline__ float stored_voxel(const ProblemView& P, int which, size_t e) {
  if (e >= P.pvox) return 0.f;
  if constexpr (ST == kF32) {
    return static_cast<const float*>(P.img[which])[e];
  } else if constexpr (ST == kBF16) {
    return bf2f(static_cast<const bf16*>(P.img[which])[e]);
  } else {
    return static_cast<float>(static_cast<const _Float16*>(P.img[which])[e]);
  }
}

// Quad copy of image `which` (0 source, 1 target; any storage): entry e
// holds the padded voxels e, e + 1, e + px, e + px + 1 as FP32.
template <int ST>
__global__ void k_image_quads(ProblemView P, int which, float4* out) {
  const size_t e = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= P.pvox) return;
  out[e] = make_float4(stored_voxel<ST>(P, which, e), stored_voxel<ST>(P, which, e + 1),
                       stored_voxel<ST>(P, which, e + P.px), stored_voxel<ST>(P, which, e + P.px + 1));
}

template <int ST>
__global__ void k_tet_stats(ProblemView P, const float* ref, float* stats, int* counts, float inv_mean) {
  const int tet = blockIdx.x;
  const int lane = threadIdx.x;
  const int4 tv = P.tets[tet];
  const int vs[4] = {tv.x, tv.y, tv.z, tv.w};
  double v[4][3];
  for (int i = 0; i < 4; i++)
    for (int a = 0; a < 3; a++) v[i][a] = rint(static_cast<double>(ref[3 * vs[i] + a]) * 1024.0);
  double e[3][3];
  for (int i = 0; i < 3; i++)
    for (int a = 0; a < 3; a++) e[i][a] = v[i + 1][a] - v[0][a];
  const double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                     e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                     e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
  const double sg = det > 0 ? 1.0 : -1.0;
  // inward face normals n_i and a vertex r_i on each face (face i omits v_i)
  double n[4][3], r[4][3];
  for (int i = 0; i < 4; i++) {
    const int b0 = i == 0 ? 1 : 0, u0 = i == 0 ? 2 : (i == 1 ? 2 : (i == 2 ? 3 : 1)),
              w0 = i == 0 ? 3 : (i == 1 ? 3 : (i == 2 ? 1 : 2));
    double u[3], w[3];
    for (int a = 0; a < 3; a++) {
      r[i][a] = v[b0][a];
      u[a] = v[u0][a] - v[b0][a];
      w[a] = v[w0][a] - v[b0][a];
    }
    const double f = (i == 0 ? -sg : sg);
    n[i][0] = f * (u[1] * w[2] - u[2] * w[1]);
    n[i][1] = f * (u[2] * w[0] - u[0] * w[2]);
    n[i][2] = f * (u[0] * w[1] - u[1] * w[0]);
  }
  int lo[3], hi[3];
  const int dims[3] = {P.nx, P.ny, P.nz};
  for (int a = 0; a < 3; a++) {
    double mn = v[0][a], mx = v[0][a];
    for (int i = 1; i < 4; i++) {
      mn = fmin(mn, v[i][a]);
      mx = fmax(mx, v[i][a]);
    }
    lo[a] = max(0, static_cast<int>(ceil(mn / 1024.0)));
    hi[a] = min(dims[a] - 1, static_cast<int>(floor(mx / 1024.0)));
  }
  const int wx = max(0, hi[0] - lo[0] + 1), wy = max(0, hi[1] - lo[1] + 1), wz = max(0, hi[2] - lo[2] + 1);
  const long long nbox = det != 0.0 ? static_cast<long long>(wx) * wy * wz : 0;
  float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // n, Is, Is^2, fg_s, It, It^2, fg_t, (Is-It)^2
  for (long long q = lane; q < nbox; q += 64) {
    const int x = lo[0] + static_cast<int>(q % wx), y = lo[1] + static_cast<int>((q / wx) % wy),
              z = lo[2] + static_cast<int>(q / (static_cast<long long>(wx) * wy));
    const double p[3] = {x * 1024.0, y * 1024.0, z * 1024.0};
    bool in = true;
    for (int i = 0; i < 4 && in; i++) {
      const double val = n[i][0] * (p[0] - r[i][0]) + n[i][1] * (p[1] - r[i][1]) + n[i][2] * (p[2] - r[i][2]);
      if (val < 0) in = false;
      else if (val == 0)
        in = n[i][0] > 0 || (n[i][0] == 0 && (n[i][1] > 0 || (n[i][1] == 0 && n[i][2] > 0)));
    }
    if (!in) continue;
    const int vi = (z + 1) * P.pxy + (y + 1) * P.px + x + 1;   // padded volumes
    float is, it;
    if constexpr (ST == kF32) {
      is = static_cast<const float*>(P.img[0])[vi];
      it = static_cast<const float*>(P.img[1])[vi];
    } else if constexpr (ST == kBF16) {
      is = bf2f(static_cast<const bf16*>(P.img[0])[vi]);
      it = bf2f(static_cast<const bf16*>(P.img[1])[vi]);
    } else {
      is = static_cast<float>(static_cast<const _Float16*>(P.img[0])[vi]);
      it = static_cast<float>(static_cast<const _Float16*>(P.img[1])[vi]);
    }
    s[0] += 1.f;
    s[1] += is;
    s[2] += is * is;
    s[3] += is > 0.f;
    s[4] += it;
    s[5] += it * it;
    s[6] += it > 0.f;
    s[7] += (is - it) * (is - it);
  }
  for (int k = 0; k < 8; k++)
    for (int d = 32; d >= 1; d >>= 1) s[k] += __shfl_xor(s[k], d, 64);
  if (lane == 0) {
    const float cnt = s[0], inv_n = cnt > 0.f ? 1.f / cnt : 0.f;
    const float ms = s[1] * inv_n, mt = s[4] * inv_n;
    float* o = stats + 8 * tet;
    o[0] = ms;
    o[1] = sqrtf(fmaxf(s[2] * inv_n - ms * ms, 0.f));
    o[2] = s[3] * inv_n;
    o[3] = mt;
    o[4] = sqrtf(fmaxf(s[5] * inv_n - mt * mt, 0.f));
    o[5] = s[6] * inv_n;
    o[6] = s[7] * inv_n;
    o[7] = cnt * inv_mean;
    counts[tet] = static_cast<int>(cnt);
  }
}

// Images and constants the features read.
struct FeatureInputs {
  const float4* img_s;  // quad copies of the two images
  const float4* img_t;
  const float4* bary;   // [16] interior points, barycentric
  const float* stats;   // [n_tets][8]
  float h_scale;
  float inv_h;          // 1 / h_scale
};

// One thread per (offspring, tet) row: the 23 features in order.  Threads in
// tet-major order, so that the threads in flight read the same part of the
// images.
__global__ void k_features(ProblemView P, const float* pts, Parents Q, FeatureInputs F, int pop, float* feats) {
  const long long r = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= static_cast<long long>(pop) * P.n_tets) return;
  const int tet = static_cast<int>(r / pop), cand = static_cast<int>(r % pop);
  float* o = feats + (static_cast<size_t>(cand) * P.n_tets + tet) * kIn;
  const int par = Q.of[cand];
  if (par < 0 || par >= Q.n) {   // no parent: the row has no features
    for (int k = 0; k < kIn; k++) o[k] = __builtin_nanf("");
    return;
  }
  const float* cp = pts + static_cast<size_t>(cand) * 6 * P.n_points;
  const float* pp = Q.pts + static_cast<size_t>(par) * 6 * P.n_points;
  float d[4][3], dp[4][3];
  tet_vertices(P, cp, tet, 1, d);
  tet_vertices(P, pp, tet, 1, dp);
#pragma unroll
  for (int v = 0; v < 4; v++)
#pragma unroll
    for (int a = 0; a < 3; a++) o[3 * v + a] = (d[v][a] - dp[v][a]) * kRelScale;
  float mc[3], mp[3];
  point_means(P, F.img_s, F.img_t, cp, tet, F.bary, mc);
  point_means(P, F.img_s, F.img_t, pp, tet, F.bary, mp);
#pragma unroll
  for (int k = 0; k < 3; k++) o[12 + k] = (mc[k] - mp[k]) * F.inv_h;
#pragma unroll
  for (int k = 0; k < 6; k++) o[15 + k] = F.stats[8 * tet + k];
  o[21] = F.stats[8 * tet + 6] * F.inv_h;
  o[22] = tet_mean_h(Q.rec + static_cast<size_t>(par) * P.n_tets * 2, tet) * F.inv_h;
}

// Target of (offspring, tet): its mean intensity term minus its parent's
// (both from their caches' records), divided by h_scale; NaN without a valid
// parent.
__global__ void k_targets(const Record* rec, int n_tets, int rows, Parents Q, float inv_h, float* t) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int cand = r / n_tets, tet = r - cand * n_tets;
  const int par = Q.of[cand];
  if (par < 0 || par >= Q.n) {
    t[r] = __builtin_nanf("");
    return;
  }
  t[r] = (tet_mean_h(rec + static_cast<size_t>(cand) * n_tets * 2, tet) -
          tet_mean_h(Q.rec + static_cast<size_t>(par) * n_tets * 2, tet)) * inv_h;
}

// Point means of every (parent, tet): out [n][n_tets] (m0, m1, m2, 0).
// Threads in tet-major order, so that the threads in flight read the same
// part of the images.
__global__ void k_parent_means(ProblemView P, const float* pts, int n, FeatureInputs F, float4* out) {
  const long long r = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= static_cast<long long>(n) * P.n_tets) return;
  const int tet = static_cast<int>(r / n), cand = static_cast<int>(r % n);
  float m[3];
  point_means(P, F.img_s, F.img_t, pts + static_cast<size_t>(cand) * 6 * P.n_points, tet, F.bary, m);
  out[static_cast<size_t>(cand) * P.n_tets + tet] = make_float4(m[0], m[1], m[2], 0.f);
}

// ------------------------------------------------------------ prescreen
// The pre-screen runs both dense layers transposed, Z^T = W X^T, on
// v_mfma_f32_32x32x16_bf16 (BF16 operands, FP32 accumulation): the weights
// are the A operand (lane l: output unit 32 n + l % 32, k = 8 (l / 32) .. +7
// of a 16-wide slice), the tets the B operand (lane l: tet l % 32 of the
// tile, the same k range), and the accumulator of lane l holds tet l % 32
// and units 8 (r / 4) + 4 (l / 32) + r % 4 of the output tile (r = 0..15).
// Accumulators r = 8 g .. 8 g + 7 of layer 1 are therefore, after bias, ReLU
// and BF16 rounding, one 16-wide k-slice of layer 2's B operand, in the unit
// order  slot kk of lane half h -> unit 4 h + kk (kk < 4), 8 + 4 h + kk - 4
// (kk >= 4)  within the slice; W2's columns are stored in that order, so no
// activation passes through LDS.  Layer 1's bias rides on constant features
// (features 23..25 = 1, W1 columns 23..25 = b1 split into three BF16 terms
// that sum to it in the FP32 accumulator); layer 2's accumulators start at b2.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));

constexpr int kPreIn = 32;                 // features padded: 23 + three constant 1s + zeros
constexpr int kTetRun = 8;                 // tets per pre-screen work item
constexpr int kW1Row = kPreIn + 8;         // LDS row strides padded against bank conflicts
constexpr int kW2Row = kHid + 8;

struct alignas(16) PreLds {
  bf16 w1[kHid][kW1Row];   // W1 | b1 (three terms) | 0
  bf16 w2[kHid][kW2Row];   // W2, columns permuted per 16-wide slice
  float b2[kHid];
  float w3[kHid];
};

__device__ __forceinline__ int slot_unit(int j) {   // 16-wide slice: slot j -> unit
  const int h = j >> 3, kk = j & 7;
  return kk < 4 ? 4 * h + kk : 8 + 4 * h + (kk - 4);
}

__device__ __forceinline__ bf8 ld8(const bf16* p) { return *reinterpret_cast<const bf8*>(p); }

__device__ __forceinline__ bf8 pack8(const float v[8]) {
  u4v w;
  w.x = static_cast<uint32_t>(f2bf(v[0])) | (static_cast<uint32_t>(f2bf(v[1])) << 16);
  w.y = static_cast<uint32_t>(f2bf(v[2])) | (static_cast<uint32_t>(f2bf(v[3])) << 16);
  w.z = static_cast<uint32_t>(f2bf(v[4])) | (static_cast<uint32_t>(f2bf(v[5])) << 16);
  w.w = static_cast<uint32_t>(f2bf(v[6])) | (static_cast<uint32_t>(f2bf(v[7])) << 16);
  return __builtin_bit_cast(bf8, w);
}

// Score of each offspring: the predicted intensity objective,
// sum_tet (parent_tet + h_scale pred_tet) w_tet / sum_tet w_tet with
// parent_tet the parent's exact mean term (FP32, from its records), pred_tet
// the network's predicted change (in units of h_scale) and w_tet the
// offspring's |volume| of the tet's source plus that of its target (voxel^3,
// the samples the tet contributes in the two directions).  Blocks of 4 waves loop over candidates; each wave takes tiles of
// 32 tets; fixed-order reductions.
__global__ __launch_bounds__(256, 3) void k_prescreen(ProblemView P, const float* pts, Parents Q, FeatureInputs F,
                                                    const float4* pmeans, const float* params, int pop,
                                                    float2* partial) {
  __shared__ PreLds N;
  for (int e = threadIdx.x; e < kHid * kPreIn; e += blockDim.x) {
    const int j = e / kPreIn, k = e % kPreIn;
    if (k < kIn) {
      N.w1[j][k] = f2bf(params[oW1 + j * kIn + k]);
    } else if (k < kIn + 3) {
      // b1 = hi + mid + lo, three BF16 terms carrying its 24-bit mantissa
      const float b = params[oB1 + j];
      const bf16 hi = f2bf(b), mid = f2bf(b - bf2f(hi)), lo = f2bf(b - bf2f(hi) - bf2f(mid));
      N.w1[j][k] = k == kIn ? hi : (k == kIn + 1 ? mid : lo);
    } else {
      N.w1[j][k] = 0;
    }
  }
  for (int e = threadIdx.x; e < kHid * kHid; e += blockDim.x) {
    const int j = e / kHid, k = e % kHid;
    N.w2[j][k] = f2bf(params[oW2 + j * kHid + (k & ~15) + slot_unit(k & 15)]);
  }
  for (int e = threadIdx.x; e < kHid; e += blockDim.x) {
    N.b2[e] = params[oB2 + e];
    N.w3[e] = params[oW3 + e];
  }
  const float b3 = params[oB3];
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = lane_id(), i = lane & 31, h = lane >> 5;
  const int n_groups = (pop + kRowTile - 1) / kRowTile;
  const int n_runs = (P.n_tets + kTetRun - 1) / kTetRun;
  const long long n_items = static_cast<long long>(n_runs) * n_groups;
  const long long n_waves = static_cast<long long>(gridDim.x) * 4;
  // work items (run of kTetRun tets, group of 32 offspring), run-major, one
  // per wave at a time: a tile of the network is one tet of 32 offspring, so
  // the lanes of a wave read nearly the same image positions and the waves
  // in flight share a few runs of tets
  for (long long w = static_cast<long long>(blockIdx.x) * 4 + wave; w < n_items; w += n_waves) {
    const int run = static_cast<int>(w / n_groups), grp = static_cast<int>(w % n_groups);
    const int cand = grp * kRowTile + i;
    const int par = cand < pop ? Q.of[cand] : -1;
    const bool ok = par >= 0 && par < Q.n;   // no parent: scored by the reduction
    const float* cp = pts + static_cast<size_t>(ok ? cand : 0) * 6 * P.n_points;
    const float* pp = Q.pts + static_cast<size_t>(ok ? par : 0) * 6 * P.n_points;
    const Record* prec = Q.rec + static_cast<size_t>(ok ? par : 0) * P.n_tets * 2;
    const float4* pmr = pmeans + static_cast<size_t>(ok ? par : 0) * P.n_tets;
    float acc_s = 0.f, cnt = 0.f;
    const int t_end = min(P.n_tets, (run + 1) * kTetRun);
    for (int tet = run * kTetRun; tet < t_end; tet++) {
      // this lane's half of the tet's features (natural order: 12 vertex
      // moves, 3 estimated changes, 7 statistics, the parent's mean term,
      // three constant 1s, zeros): h = 0 holds features 0..7 and 16..23,
      // h = 1 features 8..15 and 24..31.  The offspring's 26 points behind
      // the estimated changes are split over the halves (h = 0 points
      // 0..12, h = 1 points 13..25) and combined in the upper half, which
      // subtracts the parent's means computed beforehand.
      float f0[8], f1[8];
#pragma unroll
      for (int k = 0; k < 8; k++) f0[k] = f1[k] = 0.f;
      float acc[3] = {0.f, 0.f, 0.f};
      float pterm = 0.f, wt = 0.f;
      float4 pm = make_float4(0.f, 0.f, 0.f, 0.f);
      if (ok) {
        float d[4][3], dp[4][3];
        tet_vertices(P, cp, tet, 1, d);
        tet_vertices(P, pp, tet, 1, dp);
        {
          float sv[4][3];
          tet_vertices(P, cp, tet, 0, sv);
          point_sums(P, F.img_s, F.img_t, sv, d, F.bary, h == 0 ? 0 : kPointSplit, h == 0 ? kPointSplit : kPoints,
                     acc);
        }
        if (h == 1) pm = pmr[tet];
        if (h == 0) {
#pragma unroll
          for (int k = 0; k < 8; k++) {
            const int v = k / 3, a = k % 3;
            f0[k] = (d[v][a] - dp[v][a]) * kRelScale;
          }
#pragma unroll
          for (int k = 0; k < 5; k++) f1[k] = F.stats[8 * tet + 1 + k];
          f1[5] = F.stats[8 * tet + 6] * F.inv_h;
          pterm = tet_mean_h(prec, tet);
          f1[6] = pterm * F.inv_h;
          f1[7] = 1.f;   // the first term of b1
          wt = tet_weight(P, cp, tet);
        } else {
#pragma unroll
          for (int k = 0; k < 4; k++) {
            const int fk = 8 + k, v = fk / 3, a = fk % 3;
            f0[k] = (d[v][a] - dp[v][a]) * kRelScale;
          }
          f0[7] = F.stats[8 * tet];
          f1[0] = f1[1] = 1.f;   // the other two terms of b1
        }
      }
      {
        float lo[3], m[3];
#pragma unroll
        for (int k = 0; k < 3; k++) lo[k] = __shfl_xor(acc[k], 32, 64);
        if (h == 1) {
          combine_means(lo, acc, m);
          f0[4] = (m[0] - pm.x) * F.inv_h;
          f0[5] = (m[1] - pm.y) * F.inv_h;
          f0[6] = (m[2] - pm.z) * F.inv_h;
        }
      }
      const bf8 xb0 = pack8(f0), xb1 = pack8(f1);
      // layer 1: 4 output tiles of 32 units, K = 32 (two slices)
      bf8 hb[8];
#pragma unroll
      for (int n = 0; n < 4; n++) {
        f16v z = {};
        z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ld8(&N.w1[32 * n + i][8 * h]), xb0, z, 0, 0, 0);
        z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ld8(&N.w1[32 * n + i][16 + 8 * h]), xb1, z, 0, 0, 0);
        float v0[8], v1[8];
#pragma unroll
        for (int r = 0; r < 8; r++) {
          v0[r] = fmaxf(z[r], 0.f);
          v1[r] = fmaxf(z[8 + r], 0.f);
        }
        hb[2 * n] = pack8(v0);
        hb[2 * n + 1] = pack8(v1);
      }
      // layer 2 (K = 128, eight slices) and the output layer
      float part = 0.f;
#pragma unroll 1
      for (int n = 0; n < 4; n++) {
        f16v z;
#pragma unroll
        for (int r = 0; r < 16; r++) z[r] = N.b2[32 * n + 8 * (r >> 2) + 4 * h + (r & 3)];
#pragma unroll
        for (int sl = 0; sl < 8; sl++)
          z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ld8(&N.w2[32 * n + i][16 * sl + 8 * h]), hb[sl], z, 0, 0,
                                                      0);
#pragma unroll
        for (int r = 0; r < 16; r++)
          part = fmaf(fmaxf(z[r], 0.f), N.w3[32 * n + 8 * (r >> 2) + 4 * h + (r & 3)], part);
      }
      const float y = part + __shfl_xor(part, 32, 64) + b3;   // the two halves hold different units
      if (h == 0 && ok) {
        // the parent's exact term plus the predicted change, weighted by the
        // offspring's expected samples of the tet
        acc_s = fmaf(wt, fmaf(y, F.h_scale, pterm), acc_s);
        cnt += wt;
      }
    }
    if (h == 0 && cand < pop) partial[static_cast<size_t>(run) * pop + cand] = make_float2(acc_s, cnt);
  }
}

// Scores from the per-(run, offspring) partial sums, added in run order.
__global__ void k_prescreen_reduce(const float2* partial, int n_runs, int pop, Parents Q, float* score) {
  const int cand = blockIdx.x * blockDim.x + threadIdx.x;
  if (cand >= pop) return;
  const int par = Q.of[cand];
  if (par < 0 || par >= Q.n) {   // no parent: never preferred
    score[cand] = INFINITY;
    return;
  }
  float a = 0.f, c = 0.f;
  for (int t = 0; t < n_runs; t++) {
    const float2 v = partial[static_cast<size_t>(t) * pop + cand];
    a += v.x;
    c += v.y;
  }
  score[cand] = c > 0.f ? a / c : 0.f;
}

// Predictions for explicit feature rows (one wave per 32 rows).
__global__ __launch_bounds__(256) void k_predict_rows(const float* X, int n, const bf16* w1b,
                                                       const bf16* w2b, const float* params, float* y) {
  __shared__ NetLds N;
  __shared__ TileLds Tl[4];
  load_net(&N, w1b, w2b, params);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = lane_id(), i = lane & 31, kh = lane >> 5;
  const int row0 = (blockIdx.x * 4 + wave) * kRowTile;
  if (row0 >= n) return;
  TileLds* T = &Tl[wave];
  const bool valid = row0 + i < n;
  for (int k = kh * 12; k < (kh ? kInPad : 12); k++)
    T->x[i][k] = f2bf(valid && k < kIn ? X[static_cast<size_t>(row0 + i) * kIn + k] : 0.f);
  wave_sync();
  f16v z2[4];
  tile_forward(&N, T, T->red, z2);
  if (lane < kRowTile && row0 + lane < n) y[row0 + lane] = T->y[lane];
}

// ------------------------------------------------------------- training

struct TrainBuf {
  bf16* xT;     // [kInPad][Bpad]
  bf16* h1T;    // [kHid][Bpad]
  bf16* dz2T;   // [kHid][Bpad]
  bf16* dz1T;   // [kHid][Bpad]
  float* wpart; // [n_waves][kWavePart]
  float* gpart; // [kSplitK][kGradTiles][32][32]
  int bpad;
};

// Forward and backward (data) pass of one tile of 32 training rows.
__global__ __launch_bounds__(128) void k_train_rows(const float* X, const float* t, int n,
                                                     const bf16* w1b, const bf16* w2b,
                                                     const float* params, TrainBuf B) {
  __shared__ NetLds N;
  __shared__ TileLds Tl[2];
  __shared__ alignas(16) bf16 w2t[kHid][kHid];     // W2 transposed: w2t[k][j] = W2[j][k]
  __shared__ alignas(16) bf16 dz2s[2][kRowTile][kHid];
  __shared__ float dys[2][kRowTile];
  __shared__ RedTile reds[2];
  load_net(&N, w1b, w2b, params);
  for (int q = threadIdx.x; q < kHid * kHid; q += blockDim.x) {
    const int j = q / kHid, k = q % kHid;
    w2t[k][j] = w2b[q];
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = lane_id(), i = lane & 31, kh = lane >> 5;
  const int gw = blockIdx.x * 2 + wave;
  const int row0 = gw * kRowTile;
  float* wp = B.wpart + static_cast<size_t>(gw) * kWavePart;
  if (row0 >= B.bpad) return;
  TileLds* T = &Tl[wave];
  const bool valid = row0 + i < n;
  for (int k = kh * 12; k < (kh ? kInPad : 12); k++) {
    const bf16 v = f2bf(valid && k < kIn ? X[static_cast<size_t>(row0 + i) * kIn + k] : 0.f);
    T->x[i][k] = v;
    B.xT[static_cast<size_t>(k) * B.bpad + row0 + i] = v;
  }
  wave_sync();
  f16v z2[4];
  tile_forward(&N, T, reds[wave], z2);
  // output gradient of the mean squared error
  float lossp = 0.f, dyp = 0.f;
  if (lane < kRowTile) {
    const bool v = row0 + lane < n;
    const float diff = v ? T->y[lane] - t[row0 + lane] : 0.f;
    dys[wave][lane] = 2.f * diff / static_cast<float>(n);
    lossp = diff * diff;
    dyp = 2.f * diff / static_cast<float>(n);
  }
  wave_sync();
  // layer 2 backward: dz2 = dy w3 relu'(z2); dw3 = sum dy h2; db2 = sum dz2
#pragma unroll
  for (int nt = 0; nt < 4; nt++) {
    const int col = 32 * nt + i;
    const float w = N.w3[col];
    float gw3 = 0.f, gb2 = 0.f;
#pragma unroll
    for (int r = 0; r < 16; r++) {
      const int row = acc_row(r, kh);
      const float z = z2[nt][r];
      const float dy = dys[wave][row];
      const float dz = z > 0.f ? dy * w : 0.f;
      gw3 = fmaf(dy, fmaxf(z, 0.f), gw3);
      gb2 += dz;
      const bf16 dzb = f2bf(dz);
      dz2s[wave][row][col] = dzb;
      B.dz2T[static_cast<size_t>(col) * B.bpad + row0 + row] = dzb;
    }
    gw3 += __shfl_xor(gw3, 32, 64);
    gb2 += __shfl_xor(gb2, 32, 64);
    if (kh == 0) {
      wp[col] = gw3;
      wp[kHid + col] = gb2;
    }
  }
  // h1 transposed for the weight gradients
  for (int q = lane; q < kRowTile * kHid; q += 64) {
    const int row = q % kRowTile, k = q / kRowTile;
    B.h1T[static_cast<size_t>(k) * B.bpad + row0 + row] = T->h1[row][k];
  }
  wave_sync();
  // layer 1 backward: dh1 = dz2 W2 (MFMA with B[k=j][col] = W2[j][col]),
  // dz1 = dh1 relu'(z1); db1 = sum dz1
#pragma unroll
  for (int nt = 0; nt < 4; nt++) {
    f16v acc = {};
#pragma unroll
    for (int s = 0; s < kHid / 8; s++)
      acc = mma(ld4(&dz2s[wave][i][8 * s + 4 * kh]), ld4(&w2t[32 * nt + i][8 * s + 4 * kh]), acc);
    const int col = 32 * nt + i;
    float gb1 = 0.f;
#pragma unroll
    for (int r = 0; r < 16; r++) {
      const int row = acc_row(r, kh);
      const float dz = bf2f(T->h1[row][col]) > 0.f ? acc[r] : 0.f;
      gb1 += dz;
      B.dz1T[static_cast<size_t>(col) * B.bpad + row0 + row] = f2bf(dz);
    }
    gb1 += __shfl_xor(gb1, 32, 64);
    if (kh == 0) wp[2 * kHid + col] = gb1;
  }
  for (int d = 32; d >= 1; d >>= 1) {
    lossp += __shfl_xor(lossp, d, 64);
    dyp += __shfl_xor(dyp, d, 64);
  }
  if (lane == 0) {
    wp[3 * kHid] = dyp;
    wp[3 * kHid + 1] = lossp;
  }
}

// Weight gradients as GEMMs over the batch (K = rows), split into kSplitK
// chunks: tile 0..15 = W2 (32 x 32 blocks), 16..19 = W1 (rows 32 tr..).
__global__ __launch_bounds__(64) void k_weight_grads(TrainBuf B) {
  const int tile = blockIdx.x % kGradTiles, split = blockIdx.x / kGradTiles;
  const int lane = lane_id(), i = lane & 31, kh = lane >> 5;
  const int chunk = (B.bpad / kSplitK + 7) / 8 * 8;
  const int k0 = split * chunk, k1 = min(B.bpad, k0 + chunk);
  const bf16 *A, *Bm;
  bool bvalid = true;
  if (tile < 16) {
    const int tr = tile / 4, tc = tile % 4;
    A = B.dz2T + static_cast<size_t>(32 * tr + i) * B.bpad;
    Bm = B.h1T + static_cast<size_t>(32 * tc + i) * B.bpad;
  } else {
    const int tr = tile - 16;
    A = B.dz1T + static_cast<size_t>(32 * tr + i) * B.bpad;
    bvalid = i < kInPad;
    Bm = B.xT + static_cast<size_t>(bvalid ? i : 0) * B.bpad;
  }
  f16v acc = {};
  const s4 zero = {0, 0, 0, 0};
  for (int k = k0; k < k1; k += 8) {
    const s4 a = ld4(A + k + 4 * kh);
    const s4 b = bvalid ? ld4(Bm + k + 4 * kh) : zero;
    acc = mma(a, b, acc);
  }
  float* out = B.gpart + (static_cast<size_t>(split) * kGradTiles + tile) * 1024;
#pragma unroll
  for (int r = 0; r < 16; r++) out[acc_row(r, kh) * 32 + i] = acc[r];
}

// Gradient of every parameter (fixed-order sums of the partials), then
// either the Adam update (FP32 master, BF16 copies refreshed) or a copy of
// the gradient to `grad_out`.
__global__ void k_reduce_update(TrainBuf B, int n_waves, float* params, float* m, float* v,
                                bf16* w1b, bf16* w2b, float lr, float c1, float c2, float* grad_out,
                                float* loss_out, int n) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0 && loss_out) {
    float l = 0.f;
    for (int w = 0; w < n_waves; w++) l += B.wpart[static_cast<size_t>(w) * kWavePart + 3 * kHid + 1];
    *loss_out = l / static_cast<float>(n);
  }
  if (p >= kParams) return;
  float g = 0.f;
  if (p < oB1) {                       // W1[j][k]
    const int j = (p - oW1) / kIn, k = (p - oW1) % kIn;
    for (int s = 0; s < kSplitK; s++)
      g += B.gpart[(static_cast<size_t>(s) * kGradTiles + 16 + j / 32) * 1024 + (j % 32) * 32 + k];
  } else if (p < oW2) {                // b1
    for (int w = 0; w < n_waves; w++) g += B.wpart[static_cast<size_t>(w) * kWavePart + 2 * kHid + (p - oB1)];
  } else if (p < oB2) {                // W2[j][k]
    const int j = (p - oW2) / kHid, k = (p - oW2) % kHid;
    const int tile = (j / 32) * 4 + k / 32;
    for (int s = 0; s < kSplitK; s++)
      g += B.gpart[(static_cast<size_t>(s) * kGradTiles + tile) * 1024 + (j % 32) * 32 + (k % 32)];
  } else if (p < oW3) {                // b2
    for (int w = 0; w < n_waves; w++) g += B.wpart[static_cast<size_t>(w) * kWavePart + kHid + (p - oB2)];
  } else if (p < oB3) {                // w3
    for (int w = 0; w < n_waves; w++) g += B.wpart[static_cast<size_t>(w) * kWavePart + (p - oW3)];
  } else {                             // b3
    for (int w = 0; w < n_waves; w++) g += B.wpart[static_cast<size_t>(w) * kWavePart + 3 * kHid];
  }
  if (grad_out) {
    grad_out[p] = g;
    return;
  }
  const float b1 = 0.9f, b2 = 0.999f;
  const float mm = b1 * m[p] + (1.f - b1) * g;
  const float vv = b2 * v[p] + (1.f - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  const float w = params[p] - lr * (mm * c1) / (sqrtf(vv * c2) + 1e-8f);
  params[p] = w;
  if (p < oB1) {
    const int j = (p - oW1) / kIn, k = (p - oW1) % kIn;
    w1b[j * kInPad + k] = f2bf(w);
  } else if (p >= oW2 && p < oB2) {
    w2b[p - oW2] = f2bf(w);
  }
}

__global__ void k_refresh_bf16(const float* params, bf16* w1b, bf16* w2b) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < kHid * kInPad) {
    const int j = q / kInPad, k = q % kInPad;
    w1b[q] = k < kIn ? f2bf(params[oW1 + j * kIn + k]) : static_cast<bf16>(0);
  }
  if (q < kHid * kHid) w2b[q] = f2bf(params[oW2 + q]);
}

// --------------------------------------------------------- selection

// Indices of the k lowest scores (ties: lower index first), one block,
// bitonic sort of (score, index) pairs in LDS; n <= 8192.
__global__ __launch_bounds__(1024) void k_select(const float* score, int n, int k, int* idx_out) {
  __shared__ float key[8192];
  __shared__ int val[8192];
  int m = 1;
  while (m < n) m <<= 1;
  for (int q = threadIdx.x; q < m; q += blockDim.x) {
    key[q] = q < n ? score[q] : INFINITY;
    val[q] = q;
  }
  __syncthreads();
  for (int size = 2; size <= m; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int q = threadIdx.x; q < m; q += blockDim.x) {
        const int o = q ^ stride;
        if (o > q) {
          const bool up = (q & size) == 0;
          const float a = key[q], b = key[o];
          const int ia = val[q], ib = val[o];
          const bool greater = (a > b) || (a == b && ia > ib) || (a != a && b == b);
          if (greater == up) {
            key[q] = b; key[o] = a;
            val[q] = ib; val[o] = ia;
          }
        }
      }
      __syncthreads();
    }
  for (int q = threadIdx.x; q < k; q += blockDim.x) idx_out[q] = val[q];
}

__global__ void k_gather(const float* pts, const int* idx, int k, int per_cand, float* out) {
  for (size_t q = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
       q < static_cast<size_t>(k) * per_cand; q += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const size_t c = q / per_cand, e = q % per_cand;
    out[q] = pts[static_cast<size_t>(idx[c]) * per_cand + e];
  }
}

}  // namespace surr
}  // namespace morea

using namespace morea;
using namespace morea::surr;

struct morea_surrogate {
  morea_problem* p = nullptr;
  int max_rows = 0;
  float* params = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  bf16* w1b = nullptr;
  bf16* w2b = nullptr;
  float* stats = nullptr;
  int* counts = nullptr;
  float* ref = nullptr;
  float4* img_s = nullptr;  // quad copies of the source and target images
  float4* img_t = nullptr;
  float4* bary = nullptr;   // [16] interior sample points of a tet, barycentric
  float h_scale = 1.f;      // mean of (I_s - I_t)^2 over the grid (1 when 0)
  void* work = nullptr;     // pre-screen workspace: the parents' point means,
  size_t work_cap = 0;      // then the per-(tile, offspring) partial sums (bytes)
  TrainBuf tb{};
  int steps = 0;
  std::vector<void*> allocs;
};

namespace {
thread_local std::string s_error;
morea_status sfail(morea_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  s_error = buf;
  morea::set_error(buf);
  return s;
}

template <typename T>
morea_status salloc(morea_surrogate* s, T** dst, size_t bytes) {
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, bytes ? bytes : 4);
  if (e != hipSuccess) return sfail(MOREA_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  s->allocs.push_back(d);
  *dst = static_cast<T*>(d);
  return MOREA_OK;
}

morea_status sdev(hipError_t e, const char* what) {
  if (e == hipSuccess) return MOREA_OK;
  return sfail(MOREA_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

hipError_t launch_stats(morea_surrogate* s, const float* ref_dev) {
  const ProblemView& P = s->p->view;
  const float inv_mean = static_cast<float>(P.n_tets) / static_cast<float>(P.nx * P.ny * P.nz);
  switch (s->p->storage) {
    case kF32: hipLaunchKernelGGL(k_tet_stats<kF32>, dim3(P.n_tets), dim3(64), 0, 0, P, ref_dev, s->stats, s->counts, inv_mean); break;
    case kBF16: hipLaunchKernelGGL(k_tet_stats<kBF16>, dim3(P.n_tets), dim3(64), 0, 0, P, ref_dev, s->stats, s->counts, inv_mean); break;
    default: hipLaunchKernelGGL(k_tet_stats<kF16>, dim3(P.n_tets), dim3(64), 0, 0, P, ref_dev, s->stats, s->counts, inv_mean); break;
  }
  return hipGetLastError();
}

hipError_t launch_image_copies(morea_surrogate* s) {
  const ProblemView& P = s->p->view;
  const dim3 grid((P.pvox + 255) / 256);
  for (int which = 0; which < 2; which++) {
    float4* out = which ? s->img_t : s->img_s;
    switch (s->p->storage) {
      case kF32: hipLaunchKernelGGL(k_image_quads<kF32>, grid, dim3(256), 0, 0, P, which, out); break;
      case kBF16: hipLaunchKernelGGL(k_image_quads<kBF16>, grid, dim3(256), 0, 0, P, which, out); break;
      default: hipLaunchKernelGGL(k_image_quads<kF16>, grid, dim3(256), 0, 0, P, which, out); break;
    }
  }
  return hipGetLastError();
}

// Radical inverse of j in base b (van der Corput).
double radical_inverse(int j, int b) {
  double r = 0.0, f = 1.0 / b;
  for (; j > 0; j /= b, f /= b) r += f * (j % b);
  return r;
}

// The interior sample points: Halton points j = 1..16 in bases 2, 3, 5,
// each (u1, u2, u3) sorted into a <= b <= c and mapped to the barycentric
// coordinates (a, b - a, c - b, 1 - c) (the spacings of sorted uniforms,
// uniform on the simplex).
std::vector<float4> interior_points() {
  std::vector<float4> out;
  for (int j = 1; j <= kHalton; j++) {
    double u[3] = {radical_inverse(j, 2), radical_inverse(j, 3), radical_inverse(j, 5)};
    std::sort(u, u + 3);
    out.push_back(make_float4(static_cast<float>(u[0]), static_cast<float>(u[1] - u[0]),
                              static_cast<float>(u[2] - u[1]), static_cast<float>(1.0 - u[2])));
  }
  return out;
}

FeatureInputs feature_inputs(const morea_surrogate* s) {
  return FeatureInputs{s->img_s, s->img_t, s->bary, s->stats, s->h_scale, 1.f / s->h_scale};
}

morea_status train_launch(morea_surrogate* s, const float* X, const float* t, int n, float lr,
                          float* grad_out, float* loss_out, hipStream_t st) {
  if (!s || !X || !t) return sfail(MOREA_EINVAL, "NULL argument");
  if (n < 1 || n > s->max_rows) return sfail(MOREA_ERANGE, "rows %d outside [1, %d]", n, s->max_rows);
  TrainBuf B = s->tb;
  B.bpad = (n + kRowTile - 1) / kRowTile * kRowTile;
  B.bpad = (B.bpad + 8 * kSplitK - 1) / (8 * kSplitK) * (8 * kSplitK);
  const int n_waves = B.bpad / kRowTile;
  hipLaunchKernelGGL(k_train_rows, dim3((n_waves + 1) / 2), dim3(128), 0, st, X, t, n, s->w1b, s->w2b,
                     s->params, B);
  hipLaunchKernelGGL(k_weight_grads, dim3(kGradTiles * kSplitK), dim3(64), 0, st, B);
  float c1 = 1.f, c2 = 1.f;
  if (!grad_out) {
    s->steps += 1;
    c1 = 1.f / (1.f - powf(0.9f, static_cast<float>(s->steps)));
    c2 = 1.f / (1.f - powf(0.999f, static_cast<float>(s->steps)));
  }
  hipLaunchKernelGGL(k_reduce_update, dim3((kParams + 255) / 256), dim3(256), 0, st, B, n_waves,
                     s->params, s->adam_m, s->adam_v, s->w1b, s->w2b, lr, c1, c2, grad_out, loss_out, n);
  return sdev(hipGetLastError(), "training kernels");
}
}  // namespace

extern "C" {

int32_t morea_surrogate_num_params(void) { return kParams; }
int32_t morea_surrogate_num_features(void) { return kIn; }

morea_status morea_surrogate_create(morea_problem* p, int32_t max_rows, uint64_t seed,
                                    morea_surrogate** out) {
  if (!out) return sfail(MOREA_EINVAL, "out is NULL");
  *out = nullptr;
  if (!p) return sfail(MOREA_EINVAL, "problem is NULL");
  if (max_rows < 1 || max_rows > (1 << 24)) return sfail(MOREA_EINVAL, "max_rows %d outside [1, 2^24]", max_rows);
  morea_surrogate* s = new morea_surrogate();
  s->p = p;
  s->max_rows = max_rows;
  const int NT = p->view.n_tets;
  const int bmax = ((max_rows + 8 * kSplitK - 1) / (8 * kSplitK) + 1) * (8 * kSplitK) + kRowTile;
  s->tb.bpad = bmax;
  morea_status st = MOREA_OK;
  auto ok = [&](morea_status r) { if (st == MOREA_OK) st = r; return st == MOREA_OK; };
  ok(salloc(s, &s->params, sizeof(float) * kParams));
  ok(salloc(s, &s->adam_m, sizeof(float) * kParams));
  ok(salloc(s, &s->adam_v, sizeof(float) * kParams));
  ok(salloc(s, &s->w1b, sizeof(bf16) * kHid * kInPad));
  ok(salloc(s, &s->w2b, sizeof(bf16) * kHid * kHid));
  ok(salloc(s, &s->stats, sizeof(float) * 8 * NT));
  ok(salloc(s, &s->counts, sizeof(int) * NT));
  ok(salloc(s, &s->tb.xT, sizeof(bf16) * kInPad * static_cast<size_t>(bmax)));
  ok(salloc(s, &s->tb.h1T, sizeof(bf16) * kHid * static_cast<size_t>(bmax)));
  ok(salloc(s, &s->tb.dz2T, sizeof(bf16) * kHid * static_cast<size_t>(bmax)));
  ok(salloc(s, &s->tb.dz1T, sizeof(bf16) * kHid * static_cast<size_t>(bmax)));
  ok(salloc(s, &s->tb.wpart, sizeof(float) * kWavePart * static_cast<size_t>(bmax / kRowTile + 4)));
  ok(salloc(s, &s->tb.gpart, sizeof(float) * kSplitK * kGradTiles * 1024));
  ok(salloc(s, &s->ref, sizeof(float) * 3 * p->view.n_points));
  ok(salloc(s, &s->img_s, sizeof(float4) * static_cast<size_t>(p->view.pvox)));
  ok(salloc(s, &s->img_t, sizeof(float4) * static_cast<size_t>(p->view.pvox)));
  ok(salloc(s, &s->bary, sizeof(float4) * kHalton));
  float* ref_dev = s->ref;
  if (st == MOREA_OK) {
    // He-normal initial weights, zero biases, from the given seed
    std::vector<float> h(kParams, 0.f);
    std::mt19937_64 rng(seed);
    std::normal_distribution<float> n1(0.f, sqrtf(2.f / kIn)), n2(0.f, sqrtf(2.f / kHid)), n3(0.f, sqrtf(1.f / kHid));
    for (int q = oW1; q < oB1; q++) h[q] = n1(rng);
    for (int q = oW2; q < oB2; q++) h[q] = n2(rng);
    for (int q = oW3; q < oB3; q++) h[q] = n3(rng);
    std::vector<float> z(kParams, 0.f);
    ok(sdev(hipMemcpy(s->params, h.data(), sizeof(float) * kParams, hipMemcpyHostToDevice), "upload"));
    ok(sdev(hipMemcpy(s->adam_m, z.data(), sizeof(float) * kParams, hipMemcpyHostToDevice), "upload"));
    ok(sdev(hipMemcpy(s->adam_v, z.data(), sizeof(float) * kParams, hipMemcpyHostToDevice), "upload"));
    ok(sdev(hipMemcpy(ref_dev, p->ref_host.data(), sizeof(float) * p->ref_host.size(), hipMemcpyHostToDevice), "upload"));
  }
  if (st == MOREA_OK) {
    hipLaunchKernelGGL(k_refresh_bf16, dim3((kHid * kHid + 255) / 256), dim3(256), 0, 0, s->params, s->w1b, s->w2b);
    ok(sdev(hipGetLastError(), "refresh"));
    ok(sdev(launch_stats(s, ref_dev), "tet statistics"));
    ok(sdev(launch_image_copies(s), "image copies"));
    const std::vector<float4> bary = interior_points();
    ok(sdev(hipMemcpy(s->bary, bary.data(), sizeof(float4) * kHalton, hipMemcpyHostToDevice), "upload"));
    ok(sdev(hipDeviceSynchronize(), "surrogate set-up"));
  }
  if (st == MOREA_OK) {
    // h_scale: the count-weighted mean of the tets' mean (I_s - I_t)^2 (the
    // reference mesh tiles the grid, so this is the mean over its voxels)
    std::vector<float> hs(8 * static_cast<size_t>(NT));
    std::vector<int> hc(NT);
    ok(sdev(hipMemcpy(hs.data(), s->stats, sizeof(float) * hs.size(), hipMemcpyDeviceToHost), "copy"));
    ok(sdev(hipMemcpy(hc.data(), s->counts, sizeof(int) * hc.size(), hipMemcpyDeviceToHost), "copy"));
    double num = 0.0, den = 0.0;
    for (int t = 0; t < NT; t++) {
      num += static_cast<double>(hc[t]) * hs[8 * static_cast<size_t>(t) + 6];
      den += hc[t];
    }
    const double hsc = den > 0.0 ? num / den : 0.0;
    s->h_scale = hsc > 0.0 && std::isfinite(hsc) ? static_cast<float>(hsc) : 1.f;
  }
  if (st != MOREA_OK) {
    for (void* a : s->allocs) (void)hipFree(a);
    delete s;
    return st;
  }
  *out = s;
  return MOREA_OK;
}

void morea_surrogate_destroy(morea_surrogate* s) {
  if (!s) return;
  (void)hipDeviceSynchronize();
  for (void* a : s->allocs) (void)hipFree(a);
  if (s->work) (void)hipFree(s->work);
  delete s;
}

morea_status morea_surrogate_features(morea_surrogate* s, const float* pts, int32_t pop, const float* parent_pts,
                                      int32_t n_parents, const void* parent_cache, const int32_t* parent_of,
                                      float* feats, void* stream) {
  if (!s || pop < 0 || n_parents < 0) return sfail(MOREA_EINVAL, "bad argument");
  const long long rows = static_cast<long long>(pop) * s->p->view.n_tets;
  if (rows == 0) return MOREA_OK;
  if (!pts || !feats || !parent_of || (n_parents > 0 && (!parent_pts || !parent_cache)))
    return sfail(MOREA_EINVAL, "NULL argument");
  if (rows > (1LL << 31) / 4) return sfail(MOREA_ERANGE, "too many rows");
  const Parents Q{parent_pts, static_cast<const Record*>(parent_cache), parent_of, n_parents};
  hipLaunchKernelGGL(k_features, dim3(static_cast<unsigned>((rows + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), s->p->view, pts, Q, feature_inputs(s), pop, feats);
  return sdev(hipGetLastError(), "features");
}

morea_status morea_surrogate_targets(morea_surrogate* s, const void* cache, int32_t pop, const void* parent_cache,
                                     int32_t n_parents, const int32_t* parent_of, float* targets, void* stream) {
  if (!s || pop < 0 || n_parents < 0) return sfail(MOREA_EINVAL, "bad argument");
  const long long rows = static_cast<long long>(pop) * s->p->view.n_tets;
  if (rows == 0) return MOREA_OK;
  if (!cache || !targets || !parent_of || (n_parents > 0 && !parent_cache))
    return sfail(MOREA_EINVAL, "NULL argument");
  if (rows > (1LL << 31) - 256) return sfail(MOREA_ERANGE, "too many rows");
  const Parents Q{nullptr, static_cast<const Record*>(parent_cache), parent_of, n_parents};
  hipLaunchKernelGGL(k_targets, dim3(static_cast<unsigned>((rows + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), static_cast<const Record*>(cache), s->p->view.n_tets,
                     static_cast<int>(rows), Q, 1.f / s->h_scale, targets);
  return sdev(hipGetLastError(), "targets");
}

morea_status morea_surrogate_train_step(morea_surrogate* s, const float* feats, const float* targets,
                                        int32_t n_rows, float lr, float* loss_out, void* stream) {
  return train_launch(s, feats, targets, n_rows, lr, nullptr, loss_out, static_cast<hipStream_t>(stream));
}

morea_status morea_surrogate_gradients(morea_surrogate* s, const float* feats, const float* targets,
                                       int32_t n_rows, float* grads, float* loss_out, void* stream) {
  if (!grads) return sfail(MOREA_EINVAL, "grads is NULL");
  return train_launch(s, feats, targets, n_rows, 0.f, grads, loss_out, static_cast<hipStream_t>(stream));
}

morea_status morea_surrogate_predict_rows(morea_surrogate* s, const float* feats, int32_t n_rows,
                                          float* pred, void* stream) {
  if (!s || !feats || !pred || n_rows < 0) return sfail(MOREA_EINVAL, "bad argument");
  if (n_rows == 0) return MOREA_OK;
  const int waves = (n_rows + kRowTile - 1) / kRowTile;
  hipLaunchKernelGGL(k_predict_rows, dim3((waves + 3) / 4), dim3(256), 0, static_cast<hipStream_t>(stream),
                     feats, n_rows, s->w1b, s->w2b, s->params, pred);
  return sdev(hipGetLastError(), "predict");
}

morea_status morea_surrogate_prescreen(morea_surrogate* s, const float* pts, int32_t pop, const float* parent_pts,
                                       int32_t n_parents, const void* parent_cache, const int32_t* parent_of,
                                       float* score, void* stream) {
  if (!s || pop < 0 || n_parents < 0) return sfail(MOREA_EINVAL, "bad argument");
  if (pop == 0) return MOREA_OK;
  if (!pts || !score || !parent_of || (n_parents > 0 && (!parent_pts || !parent_cache)))
    return sfail(MOREA_EINVAL, "NULL argument");
  const ProblemView& P = s->p->view;
  const int n_runs = (P.n_tets + kTetRun - 1) / kTetRun;
  const size_t rows = static_cast<size_t>(n_parents) * P.n_tets;
  const size_t pm_bytes = (sizeof(float4) * rows + 255) / 256 * 256;
  const size_t need = pm_bytes + sizeof(float2) * static_cast<size_t>(n_runs) * pop;
  if (need > s->work_cap) {   // grow the workspace (hipFree waits for the device)
    if (s->work) (void)hipFree(s->work);
    s->work = nullptr;
    s->work_cap = 0;
    void* d = nullptr;
    const hipError_t e = hipMalloc(&d, need);
    if (e != hipSuccess) return sfail(MOREA_ENOMEM, "hipMalloc(%zu): %s", need, hipGetErrorString(e));
    s->work = d;
    s->work_cap = need;
  }
  float4* pmeans = static_cast<float4*>(s->work);
  float2* partial = reinterpret_cast<float2*>(static_cast<char*>(s->work) + pm_bytes);
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const FeatureInputs F = feature_inputs(s);
  if (rows > 0)
    hipLaunchKernelGGL(k_parent_means, dim3(static_cast<unsigned>((rows + 255) / 256)), dim3(256), 0, st, P,
                       parent_pts, n_parents, F, pmeans);
  const Parents Q{parent_pts, static_cast<const Record*>(parent_cache), parent_of, n_parents};
  const long long items = static_cast<long long>(n_runs) * ((pop + kRowTile - 1) / kRowTile);
  const int blocks = static_cast<int>(std::min<long long>((items + 3) / 4, 768));
  hipLaunchKernelGGL(k_prescreen, dim3(blocks), dim3(256), 0, st, P, pts, Q, F, pmeans, s->params, pop, partial);
  hipLaunchKernelGGL(k_prescreen_reduce, dim3((pop + 255) / 256), dim3(256), 0, st, partial, n_runs, pop, Q, score);
  return sdev(hipGetLastError(), "prescreen");
}

morea_status morea_surrogate_select(const float* score, int32_t n, int32_t k, const float* pts,
                                    int32_t n_points, int32_t* idx_out, float* selected_pts, void* stream) {
  if (!score || !idx_out || n < 1 || n > 8192 || k < 1 || k > n)
    return sfail(MOREA_EINVAL, "need 1 <= k <= n <= 8192 and non-NULL arrays");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, st, score, n, k, idx_out);
  if (pts && selected_pts) {
    const int per = 6 * n_points;
    hipLaunchKernelGGL(k_gather, dim3(1024), dim3(256), 0, st, pts, idx_out, k, per, selected_pts);
  }
  return sdev(hipGetLastError(), "select");
}

morea_status morea_surrogate_get_params(morea_surrogate* s, float* host_params) {
  if (!s || !host_params) return sfail(MOREA_EINVAL, "bad argument");
  return sdev(hipMemcpy(host_params, s->params, sizeof(float) * kParams, hipMemcpyDeviceToHost), "copy");
}

morea_status morea_surrogate_set_params(morea_surrogate* s, const float* host_params) {
  if (!s || !host_params) return sfail(MOREA_EINVAL, "bad argument");
  morea_status st = sdev(hipMemcpy(s->params, host_params, sizeof(float) * kParams, hipMemcpyHostToDevice), "copy");
  if (st != MOREA_OK) return st;
  hipLaunchKernelGGL(k_refresh_bf16, dim3((kHid * kHid + 255) / 256), dim3(256), 0, 0, s->params, s->w1b, s->w2b);
  st = sdev(hipGetLastError(), "refresh");
  if (st == MOREA_OK) st = sdev(hipDeviceSynchronize(), "set params");
  return st;
}

morea_status morea_surrogate_scale(const morea_surrogate* s, float* h_scale) {
  if (!s || !h_scale) return sfail(MOREA_EINVAL, "bad argument");
  *h_scale = s->h_scale;
  return MOREA_OK;
}

morea_status morea_surrogate_stats(morea_surrogate* s, float* host_stats, int32_t* host_counts) {
  if (!s || !host_stats) return sfail(MOREA_EINVAL, "bad argument");
  const int NT = s->p->view.n_tets;
  morea_status st = sdev(hipMemcpy(host_stats, s->stats, sizeof(float) * 8 * NT, hipMemcpyDeviceToHost), "copy");
  if (st == MOREA_OK && host_counts)
    st = sdev(hipMemcpy(host_counts, s->counts, sizeof(int) * NT, hipMemcpyDeviceToHost), "copy");
  return st;
}

}  // extern "C"
