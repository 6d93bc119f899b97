// Device code of libmorea: per-(candidate, tetrahedron, direction) evaluation
// by one 64-lane wavefront, per-candidate reductions, and the set-up kernel
// that builds the guidance distance maps.
//
// One wave owns one work item: a tetrahedron of one candidate in one
// direction.  Direction 0 rasterizes the source tet on I_s's voxel grid, maps
// each sample into the target tet and samples I_t; direction 1 does the same
// with the roles of the two meshes and images exchanged (the symmetric
// objective of Sec. 4.1.2 and the dual-dynamic model of Sec. 4.2.1).
//
// Rasterization is exact.  Coordinates are snapped to 2^-10 voxel; each face
// plane value s_i(p) = D * lambda_i(p) is an integer (units 2^-30 voxel^3),
// computed exactly in FP64 when the tet's extent is at most 2^16 units (64
// voxels: every product and partial sum stays below 2^53) and in int64
// otherwise (extent < 2^20 keeps |s_i| < 6 E^3 < 2^63).  A centre on a face
// belongs to the tet iff the face's inward normal is lexicographically
// positive, i.e. p + (e, e^2, e^3) is strictly inside.
//
// Each wave walks the bounding box row by row: 64 rows at a time, one per
// lane, it solves the x-interval of each row exactly (a division estimate
// corrected by exact evaluation), compacts the non-empty rows into LDS and
// then streams the row samples 64 at a time, so every lane holds one voxel.
#include "morea_internal.h"

namespace morea {

// ------------------------------------------------------------------ helpers

template <int ST>
__device__ __forceinline__ float ld_img(const void* base, int idx) {
  if constexpr (ST == kF32) {
    return static_cast<const float*>(base)[idx];
  } else if constexpr (ST == kBF16) {
    return __uint_as_float(static_cast<uint32_t>(static_cast<const uint16_t*>(base)[idx]) << 16);
  } else {
    return static_cast<float>(static_cast<const _Float16*>(base)[idx]);
  }
}

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ __forceinline__ int bits_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int wave_excl_scan(int v) {
  const int lane = lane_id();
  int x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x - v;
}

// Butterfly sum: every lane ends with the same value, in a fixed order.
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ int64_t floor_div_pos(int64_t a, int64_t b) {  // b > 0
  int64_t q = a / b;
  return (q * b > a) ? q - 1 : q;
}

// Compensated (double-float) accumulation: value = hi + lo.
__device__ __forceinline__ void df_add(float& hi, float& lo, float x) {
  float s = hi + x;
  float bb = s - hi;
  float err = (hi - (s - bb)) + (x - bb);
  hi = s;
  lo += err;
}

// 6 x signed volume with integer coordinates (|coord| < 2^19: exact in int64).
__device__ __forceinline__ int64_t det_i64(const int v[4][3]) {
  int64_t a0 = v[1][0] - v[0][0], a1 = v[1][1] - v[0][1], a2 = v[1][2] - v[0][2];
  int64_t b0 = v[2][0] - v[0][0], b1 = v[2][1] - v[0][1], b2 = v[2][2] - v[0][2];
  int64_t c0 = v[3][0] - v[0][0], c1 = v[3][1] - v[0][1], c2 = v[3][2] - v[0][2];
  return a0 * (b1 * c2 - b2 * c1) - a1 * (b0 * c2 - b2 * c0) + a2 * (b0 * c1 - b1 * c0);
}

// LDS scratch of one wave.
struct WaveLds {
  int row_x0[kWave];
  int row_yz[kWave];
  int row_off[kWave];
  int mark[kWave];
  int vert[24];   // snapped own tet (12), then other tet (12)
};

// Exact support test of the trilinear stencil (rare path, taken only when
// the FP32 mapped coordinate is within its error bound of an integer on some
// axis).  Recomputes D * lambda_i(p) exactly, forms the mapped coordinate as
// the rational N / (|D| 2^10) in 128-bit integers and finds its exact floor
// k: if N / (|D| 2^10) == k only corner k carries weight on that axis,
// otherwise corners k and k + 1 do.  Returns whether any supported in-grid
// corner is > 0.
template <int ST>
__device__ __noinline__ bool exact_foreground(const void* img, int nx, int ny, int nz,
                                              const int* vert, int sigma, int64_t absD, int x,
                                              int y, int z, float q0, float q1, float q2,
                                              int amb) {
  int own[4][3], oth[4][3];
  for (int i = 0; i < 4; i++)
    for (int k = 0; k < 3; k++) {
      own[i][k] = vert[3 * i + k];
      oth[i][k] = vert[12 + 3 * i + k];
    }
  const int p[3] = {x * 1024, y * 1024, z * 1024};
  int64_t s[4];
  for (int i = 0; i < 4; i++) {
    int w[4][3];
    for (int j = 0; j < 4; j++)
      for (int k = 0; k < 3; k++) w[j][k] = (j == i) ? p[k] : own[j][k];
    s[i] = sigma * det_i64(w);
  }
  const __int128 den = static_cast<__int128>(absD) * 1024;
  const float q[3] = {q0, q1, q2};
  int lo[3], hi[3];
  for (int a = 0; a < 3; a++) {
    if (amb & (1 << a)) {
      __int128 num = 0;
      for (int i = 0; i < 4; i++) num += static_cast<__int128>(s[i]) * oth[i][a];
      // exact floor k of num / den, starting from the FP32 estimate; the
      // mapped point is a convex combination of valid vertices, so
      // |k| <= 513 and the corrections terminate.
      int k = static_cast<int>(floorf(q[a]));
      k = min(max(k, -600), 600);
      while (static_cast<__int128>(k) * den > num) k--;
      while (static_cast<__int128>(k + 1) * den <= num) k++;
      const bool on_grid = static_cast<__int128>(k) * den == num;
      lo[a] = k;
      hi[a] = on_grid ? k : k + 1;
    } else {
      lo[a] = static_cast<int>(floorf(q[a]));
      hi[a] = lo[a] + 1;
    }
  }
  bool fg = false;
  for (int cz = lo[2]; cz <= hi[2]; cz++)
    for (int cy = lo[1]; cy <= hi[1]; cy++)
      for (int cx = lo[0]; cx <= hi[0]; cx++)
        if (cx >= 0 && cy >= 0 && cz >= 0 && cx < nx && cy < ny && cz < nz)
          fg |= ld_img<ST>(img, (cz * ny + cy) * nx + cx) > 0.0f;
  return fg;
}

// Exact x-interval [js, je] (relative to the row start x0, clipped to
// [0, W]) of one row for one face: the set of j with a*j + b + lex > 0.
// T is double (exact for extents <= 2^16) or int64_t.
template <typename T>
__device__ __forceinline__ void clip_face(T a, T bl, int W, int& js, int& je) {
  if (a > 0) {
    double t = -static_cast<double>(bl) / static_cast<double>(a);
    t = fmin(fmax(t, -2.0), W + 1.0);
    int j = static_cast<int>(floor(t)) + 1;
    if (a * static_cast<T>(j - 1) + bl > 0) j -= 1;
    if (a * static_cast<T>(j) + bl <= 0) j += 1;
    js = max(js, j);
  } else if (a < 0) {
    double t = static_cast<double>(bl) / -static_cast<double>(a);
    t = fmin(fmax(t, -2.0), W + 1.0);
    int j = static_cast<int>(ceil(t)) - 1;
    if (a * static_cast<T>(j + 1) + bl > 0) j += 1;
    if (a * static_cast<T>(j) + bl <= 0) j -= 1;
    je = min(je, j);
  } else if (!(bl > 0)) {
    je = -1;
  }
}

struct Planes {
  // s_i(x0 + j, y, z) = A[i] * j + Cx[i] + NY[i] * (1024 y - RY[i]) + NZ[i] * (1024 z - RZ[i])
  int64_t A[4], Cx[4], NY[4], NZ[4], RY[4], RZ[4];
  int lex[4];
};

template <typename T>
__device__ __forceinline__ void row_span(const Planes& pl, int y, int z, int W, int& js, int& je) {
  js = 0;
  je = W;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    T b = static_cast<T>(pl.Cx[i]) + static_cast<T>(pl.NY[i]) * static_cast<T>(1024 * (int64_t)y - pl.RY[i]) +
          static_cast<T>(pl.NZ[i]) * static_cast<T>(1024 * (int64_t)z - pl.RZ[i]) + static_cast<T>(pl.lex[i]);
    clip_face<T>(static_cast<T>(pl.A[i]), b, W, js, je);
  }
}

// Evaluate one (tet, direction) for the candidate whose vertex coordinates
// are held by lanes 0..23 (`coord`: lanes 0..11 own tet v0x v0y v0z v1x ...,
// lanes 12..23 the other tet).  The wave writes one Record.
template <int ST>
__device__ void eval_tet_dir(const ProblemView& P, int tet, int dir, float coord, WaveLds* L,
                             Record* out) {
  const int lane = lane_id();
  // ---- snap and validate (the loading lane snaps its own coordinate)
  const bool in_range = lane >= 24 || fabsf(coord) < kCoordLimit;
  const bool all_ok = __ballot(in_range) == ~0ull;
  const int fix = (lane < 24 && in_range) ? static_cast<int>(rintf(coord * kFixOne)) : 0;
  if (!all_ok) {
    if (lane == 0) *out = Record{0.f, 0.f, 0u, 0.f, 0.f, 4u};
    return;
  }
  if (lane < 24) L->vert[lane] = fix;
  int own[4][3], oth[4][3];
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int k = 0; k < 3; k++) {
      own[i][k] = __builtin_amdgcn_readlane(fix, 3 * i + k);
      oth[i][k] = __builtin_amdgcn_readlane(fix, 12 + 3 * i + k);
    }

  // ---- fold check (App. A.4): exact signed volume vs the reference sign
  const int64_t D = det_i64(own);
  const int ref = P.ref_sign[tet];
  const int sgnD = (D > 0) - (D < 0);
  const bool viol = (sgnD == 0) || (sgnD != ref);
  const int64_t absD = D < 0 ? -D : D;
  Record rec{0.f, 0.f, 0u, 0.f, 0.f, viol ? 1u : 0u};
  if (viol) rec.vol = static_cast<float>(static_cast<double>(absD) * (1.0 / (6.0 * 1073741824.0)));

  // ---- deformation magnitude (Sec. 4.1.1), computed once, by direction 0:
  // |e_s| - |e_t| = (|e_s|^2 - |e_t|^2) / (|e_s| + |e_t|) with the squared
  // lengths exact in int64, so small differences do not cancel.
  if (dir == 0) {
    float acc = 0.f;
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
      for (int j = i + 1; j < 4; j++) {
        int64_t ls = 0, lt = 0;
#pragma unroll
        for (int k = 0; k < 3; k++) {
          int64_t ds = own[i][k] - own[j][k], dt = oth[i][k] - oth[j][k];
          ls += ds * ds;
          lt += dt * dt;
        }
        float den = sqrtf(static_cast<float>(ls)) + sqrtf(static_cast<float>(lt));
        float d = den > 0.f ? static_cast<float>(ls - lt) / den * (1.0f / kFixOne) : 0.f;
        acc += d * d;
      }
#pragma unroll
    for (int i = 0; i < 4; i++) {
      int64_t ls = 0, lt = 0;
#pragma unroll
      for (int k = 0; k < 3; k++) {
        int64_t ds = 4 * (int64_t)own[i][k] - (own[0][k] + own[1][k] + own[2][k] + own[3][k]);
        int64_t dt = 4 * (int64_t)oth[i][k] - (oth[0][k] + oth[1][k] + oth[2][k] + oth[3][k]);
        ls += ds * ds;
        lt += dt * dt;
      }
      float den = sqrtf(static_cast<float>(ls)) + sqrtf(static_cast<float>(lt));
      float d = den > 0.f ? static_cast<float>(ls - lt) / den * (1.0f / (4.0f * kFixOne)) : 0.f;
      acc += d * d;
    }
    rec.mag = P.elasticity[tet] * acc;
  }

  // ---- bounding box on this direction's grid
  int lo[3], hi[3], ext = 0;
  const int dims[3] = {P.nx, P.ny, P.nz};
#pragma unroll
  for (int k = 0; k < 3; k++) {
    int mn = min(min(own[0][k], own[1][k]), min(own[2][k], own[3][k]));
    int mx = max(max(own[0][k], own[1][k]), max(own[2][k], own[3][k]));
    ext = max(ext, mx - mn);
    lo[k] = max(0, -static_cast<int>(floor_div_pos(-static_cast<int64_t>(mn), 1024)));
    hi[k] = min(dims[k] - 1, static_cast<int>(floor_div_pos(mx, 1024)));
  }
  const bool empty = D == 0 || lo[0] > hi[0] || lo[1] > hi[1] || lo[2] > hi[2];
  if (empty) {
    if (lane == 0) *out = rec;
    return;
  }
  const int sigma = D > 0 ? 1 : -1;

  // ---- face planes: gradient n_i of D * lambda_i (inward after sigma) and a
  // reference vertex r_i on the face.
  Planes pl;
  {
    int64_t e[3][3];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int k = 0; k < 3; k++) e[i][k] = own[i + 1][k] - own[0][k];
    int64_t n[4][3];
    auto cross = [](const int64_t* u, const int64_t* v, int64_t* r) {
      r[0] = u[1] * v[2] - u[2] * v[1];
      r[1] = u[2] * v[0] - u[0] * v[2];
      r[2] = u[0] * v[1] - u[1] * v[0];
    };
    cross(e[1], e[2], n[1]);
    cross(e[2], e[0], n[2]);
    cross(e[0], e[1], n[3]);
#pragma unroll
    for (int k = 0; k < 3; k++) n[0][k] = -(n[1][k] + n[2][k] + n[3][k]);
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int rv = (i == 0) ? 1 : 0;
      int64_t nx_ = sigma * n[i][0], ny_ = sigma * n[i][1], nz_ = sigma * n[i][2];
      pl.A[i] = nx_ * 1024;
      pl.Cx[i] = nx_ * (1024 * (int64_t)lo[0] - own[rv][0]);
      pl.NY[i] = ny_;
      pl.NZ[i] = nz_;
      pl.RY[i] = own[rv][1];
      pl.RZ[i] = own[rv][2];
      pl.lex[i] = (nx_ > 0 || (nx_ == 0 && (ny_ > 0 || (ny_ == 0 && nz_ > 0)))) ? 1 : 0;
    }
  }

  // ---- affine map of this direction: q = M (p - p_lo) + q_lo (FP32), with
  // M = B adj(A) / D from the exact edge matrices, and a per-axis bound
  // `guard` on the FP32 error of q.
  float M[3][3], qlo[3], guard[3];
  {
    double inv = 1.0 / static_cast<double>(D);
    // rows of adj(A) are n_1, n_2, n_3 (before sigma): recompute them here
    int64_t e[3][3], b[3][3];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int k = 0; k < 3; k++) {
        e[i][k] = own[i + 1][k] - own[0][k];
        b[i][k] = oth[i + 1][k] - oth[0][k];
      }
    double adj[3][3];
    adj[0][0] = (double)(e[1][1] * e[2][2] - e[1][2] * e[2][1]);
    adj[0][1] = (double)(e[1][2] * e[2][0] - e[1][0] * e[2][2]);
    adj[0][2] = (double)(e[1][0] * e[2][1] - e[1][1] * e[2][0]);
    adj[1][0] = (double)(e[2][1] * e[0][2] - e[2][2] * e[0][1]);
    adj[1][1] = (double)(e[2][2] * e[0][0] - e[2][0] * e[0][2]);
    adj[1][2] = (double)(e[2][0] * e[0][1] - e[2][1] * e[0][0]);
    adj[2][0] = (double)(e[0][1] * e[1][2] - e[0][2] * e[1][1]);
    adj[2][1] = (double)(e[0][2] * e[1][0] - e[0][0] * e[1][2]);
    adj[2][2] = (double)(e[0][0] * e[1][1] - e[0][1] * e[1][0]);
    double Md[3][3];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
      for (int c = 0; c < 3; c++)
        Md[a][c] = ((double)b[0][a] * adj[0][c] + (double)b[1][a] * adj[1][c] + (double)b[2][a] * adj[2][c]) * inv;
    const double pl0[3] = {lo[0] - own[0][0] / 1024.0, lo[1] - own[0][1] / 1024.0, lo[2] - own[0][2] / 1024.0};
#pragma unroll
    for (int a = 0; a < 3; a++) {
      double q = oth[0][a] / 1024.0 + Md[a][0] * pl0[0] + Md[a][1] * pl0[1] + Md[a][2] * pl0[2];
      qlo[a] = static_cast<float>(q);
      double bound = fabs(q) + 1.0;
#pragma unroll
      for (int c = 0; c < 3; c++) {
        M[a][c] = static_cast<float>(Md[a][c]);
        bound += fabs(Md[a][c]) * (hi[c] - lo[c]);
      }
      guard[a] = static_cast<float>(bound * (1.0 / 1048576.0));   // 2^-20 * bound >= 4x the error
    }
  }

  const int W = hi[0] - lo[0];
  const int NYb = hi[1] - lo[1] + 1;
  const int R = NYb * (hi[2] - lo[2] + 1);
  const bool fast = ext <= kFastExtent;
  const void* img_own = P.img[dir];
  const void* img_oth = P.img[1 - dir];
  const uint8_t* band_own = P.band[dir];
  const float* map_own = P.dmap[dir];
  const float* map_oth = P.dmap[1 - dir];
  const int V = P.nx * P.ny * P.nz;
  const float r = P.radius, inv_r = P.inv_radius;
  const bool guided = P.n_sets > 0;

  float h_acc = 0.f, g_acc = 0.f;
  int n_acc = 0;
  wave_sync();   // vertex table visible to the exact path

  for (int rb = 0; rb < R; rb += kWave) {
    const int rr = rb + lane;
    int js = 1, je = 0, y = 0, z = 0;
    if (rr < R) {
      const int zr = rr / NYb;
      z = lo[2] + zr;
      y = lo[1] + (rr - zr * NYb);
      if (fast)
        row_span<double>(pl, y, z, W, js, je);
      else
        row_span<int64_t>(pl, y, z, W, js, je);
    }
    const int len = max(0, je - js + 1);
    const uint64_t rows_mask = __ballot(len > 0);
    if (rows_mask == 0) continue;
    const int nrows = __popcll(rows_mask);
    const int off = wave_excl_scan(len);
    const int total = __shfl(off + len, 63, 64);
    if (len > 0) {
      const int ci = bits_below(rows_mask);
      L->row_x0[ci] = lo[0] + js;
      L->row_yz[ci] = y | (z << 16);
      L->row_off[ci] = off;
    }
    wave_sync();
    const int my_off = lane < nrows ? L->row_off[lane] : 0x7fffffff;

    for (int sb = 0; sb < total; sb += kWave) {
      // row of each lane's sample: rows starting at or before sb, plus rows
      // starting inside (sb, sb + lane]
      const int first = __popcll(__ballot(my_off <= sb)) - 1;
      L->mark[lane] = 0;
      wave_sync();
      const int rel = my_off - sb;
      if (rel > 0 && rel < kWave) L->mark[rel] = 1;
      wave_sync();
      const uint64_t starts = __ballot(L->mark[lane] != 0);
      const int ri = first + bits_below(starts) + static_cast<int>((starts >> lane) & 1ull);
      const int s = sb + lane;
      if (s < total) {
        const int x = L->row_x0[ri] + (s - L->row_off[ri]);
        const int yz = L->row_yz[ri];
        const int yy = yz & 0xffff, zz = yz >> 16;
        const int vi = (zz * P.ny + yy) * P.nx + x;
        const float a = ld_img<ST>(img_own, vi);
        const float dx = static_cast<float>(x - lo[0]);
        const float dy = static_cast<float>(yy - lo[1]);
        const float dz = static_cast<float>(zz - lo[2]);
        float q[3], f[3];
        int c[3];
        int amb = 0;
#pragma unroll
        for (int k = 0; k < 3; k++) {
          q[k] = fmaf(M[k][0], dx, fmaf(M[k][1], dy, fmaf(M[k][2], dz, qlo[k])));
          const float fl = floorf(q[k]);
          f[k] = q[k] - fl;
          c[k] = static_cast<int>(fl);
          if (f[k] <= guard[k] || f[k] >= 1.0f - guard[k]) amb |= 1 << k;
        }
        const bool x0ok = c[0] >= 0 && c[0] < P.nx, x1ok = c[0] + 1 >= 0 && c[0] + 1 < P.nx;
        const bool y0ok = c[1] >= 0 && c[1] < P.ny, y1ok = c[1] + 1 >= 0 && c[1] + 1 < P.ny;
        const bool z0ok = c[2] >= 0 && c[2] < P.nz, z1ok = c[2] + 1 >= 0 && c[2] + 1 < P.nz;
        const int base = (c[2] * P.ny + c[1]) * P.nx + c[0];
        const int sy = P.nx, sz = P.nx * P.ny;
        const float v000 = (z0ok && y0ok && x0ok) ? ld_img<ST>(img_oth, base) : 0.f;
        const float v001 = (z0ok && y0ok && x1ok) ? ld_img<ST>(img_oth, base + 1) : 0.f;
        const float v010 = (z0ok && y1ok && x0ok) ? ld_img<ST>(img_oth, base + sy) : 0.f;
        const float v011 = (z0ok && y1ok && x1ok) ? ld_img<ST>(img_oth, base + sy + 1) : 0.f;
        const float v100 = (z1ok && y0ok && x0ok) ? ld_img<ST>(img_oth, base + sz) : 0.f;
        const float v101 = (z1ok && y0ok && x1ok) ? ld_img<ST>(img_oth, base + sz + 1) : 0.f;
        const float v110 = (z1ok && y1ok && x0ok) ? ld_img<ST>(img_oth, base + sz + sy) : 0.f;
        const float v111 = (z1ok && y1ok && x1ok) ? ld_img<ST>(img_oth, base + sz + sy + 1) : 0.f;
        const float e00 = fmaf(f[0], v001 - v000, v000), e01 = fmaf(f[0], v011 - v010, v010);
        const float e10 = fmaf(f[0], v101 - v100, v100), e11 = fmaf(f[0], v111 - v110, v110);
        const float e0 = fmaf(f[1], e01 - e00, e00), e1 = fmaf(f[1], e11 - e10, e10);
        float b = fmaf(f[2], e1 - e0, e0);
        bool fg_b = (v000 > 0.f) | (v001 > 0.f) | (v010 > 0.f) | (v011 > 0.f) | (v100 > 0.f) |
                    (v101 > 0.f) | (v110 > 0.f) | (v111 > 0.f);
        if (amb)
          fg_b = exact_foreground<ST>(img_oth, P.nx, P.ny, P.nz, L->vert, sigma, absD, x, yy, zz,
                                      q[0], q[1], q[2], amb);
        const bool fg_a = a > 0.f;
        float h;
        if (fg_a && fg_b) {
          const float dd = a - b;
          h = dd * dd;
        } else {
          h = (fg_a != fg_b) ? 1.f : 0.f;
        }
        h_acc += h;
        n_acc += 1;

        if (guided) {
          unsigned bandbits = band_own[vi];
          if (bandbits) {
            const int cx0 = min(max(c[0], 0), P.nx - 1), cx1 = min(max(c[0] + 1, 0), P.nx - 1);
            const int cy0 = min(max(c[1], 0), P.ny - 1), cy1 = min(max(c[1] + 1, 0), P.ny - 1);
            const int cz0 = min(max(c[2], 0), P.nz - 1), cz1 = min(max(c[2] + 1, 0), P.nz - 1);
            const int i00 = (cz0 * P.ny + cy0) * P.nx, i01 = (cz0 * P.ny + cy1) * P.nx;
            const int i10 = (cz1 * P.ny + cy0) * P.nx, i11 = (cz1 * P.ny + cy1) * P.nx;
            while (bandbits) {
              const int sidx = __builtin_ctz(bandbits);
              bandbits &= bandbits - 1;
              const float* mo = map_oth + static_cast<size_t>(sidx) * V;
              const float d = map_own[static_cast<size_t>(sidx) * V + vi];
              const float u00 = fmaf(f[0], mo[i00 + cx1] - mo[i00 + cx0], mo[i00 + cx0]);
              const float u01 = fmaf(f[0], mo[i01 + cx1] - mo[i01 + cx0], mo[i01 + cx0]);
              const float u10 = fmaf(f[0], mo[i10 + cx1] - mo[i10 + cx0], mo[i10 + cx0]);
              const float u11 = fmaf(f[0], mo[i11 + cx1] - mo[i11 + cx0], mo[i11 + cx0]);
              const float u0 = fmaf(f[1], u01 - u00, u00), u1 = fmaf(f[1], u11 - u10, u10);
              const float d2 = fmaf(f[2], u1 - u0, u0);
              const float diff = d - d2;
              g_acc += P.set_w[dir][sidx] * ((r - d) * inv_r) * diff * diff;
            }
          }
        }
      }
      wave_sync();
    }
  }
  rec.h = wave_sum(h_acc);
  rec.g = wave_sum(g_acc);
  rec.n = static_cast<uint32_t>(wave_sum_i(n_acc));
  if (lane == 0) *out = rec;
}

// Block index remap so that each of the 8 XCDs (which receive blocks
// round-robin) works through one contiguous range of logical blocks: the
// items of neighbouring tets then share that XCD's L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb / 8, rem = nb % 8;
  const int x = b % 8, pos = b / 8;
  return x < rem ? x * (q + 1) + pos : rem * (q + 1) + (x - rem) * q + pos;
}

// ------------------------------------------------------------------ kernels

// Full evaluation: item = (tet * pop + candidate) * 2 + direction.
template <int ST>
__global__ __launch_bounds__(256) void k_eval_full(ProblemView P, FullItems F, Record* rec,
                                                    int n_items) {
  __shared__ WaveLds lds[4];
  const int wave = threadIdx.x >> 6;
  const int item = xcd_block(blockIdx.x, gridDim.x) * 4 + wave;
  if (item >= n_items) return;
  const int dir = item & 1;
  const int rest = item >> 1;
  const int cand = rest % F.pop;
  const int tet = rest / F.pop;
  const int lane = lane_id();
  float coord = 0.f;
  if (lane < 24) {
    const int4 tv = P.tets[tet];
    const int i = (lane % 12) / 3, k = lane % 3;
    const int v = i == 0 ? tv.x : (i == 1 ? tv.y : (i == 2 ? tv.z : tv.w));
    const int mesh = lane < 12 ? dir : 1 - dir;
    coord = F.pts[((static_cast<size_t>(cand) * 2 + mesh) * 3 + k) * P.n_points + v];
  }
  eval_tet_dir<ST>(P, tet, dir, coord, &lds[wave], &rec[(static_cast<size_t>(cand) * P.n_tets + tet) * 2 + dir]);
}

template __global__ void k_eval_full<kF32>(ProblemView, FullItems, Record*, int);
template __global__ void k_eval_full<kBF16>(ProblemView, FullItems, Record*, int);
template __global__ void k_eval_full<kF16>(ProblemView, FullItems, Record*, int);

// Per-candidate reduction over all tets in a fixed order, with compensated
// sums; writes the objective vector, flags, severity, counts and (when
// `totals` is non-null) the candidate totals of the cache.
__global__ __launch_bounds__(256) void k_finalize(ProblemView P, const float* pts, const Record* rec,
                                                   float* obj, uint8_t* flags, float* severity,
                                                   uint32_t* counts, Totals* totals) {
  const int cand = blockIdx.x;
  const int tid = threadIdx.x;
  float hh = 0.f, hl = 0.f, gh = 0.f, gl = 0.f, mh = 0.f, ml = 0.f, vh = 0.f, vl = 0.f;
  uint32_t ns = 0, nt = 0, vs = 0, vt = 0, bad = 0;
  const Record* rc = rec + static_cast<size_t>(cand) * P.n_tets * 2;
  for (int t = tid; t < P.n_tets; t += blockDim.x) {
    const Record a = rc[2 * t], b = rc[2 * t + 1];
    df_add(hh, hl, a.h);
    df_add(hh, hl, b.h);
    df_add(gh, gl, a.g);
    df_add(gh, gl, b.g);
    df_add(mh, ml, a.mag);
    df_add(vh, vl, a.vol);
    df_add(vh, vl, b.vol);
    ns += a.n;
    nt += b.n;
    vs += a.bits & 1u;
    vt += b.bits & 1u;
  }
  const float* cp = pts + static_cast<size_t>(cand) * 6 * P.n_points;
  for (int i = tid; i < 6 * P.n_points; i += blockDim.x) bad += !(fabsf(cp[i]) < kCoordLimit);

  __shared__ float sf[8][256];
  __shared__ uint32_t su[5][256];
  sf[0][tid] = hh; sf[1][tid] = hl; sf[2][tid] = gh; sf[3][tid] = gl;
  sf[4][tid] = mh; sf[5][tid] = ml; sf[6][tid] = vh; sf[7][tid] = vl;
  su[0][tid] = ns; su[1][tid] = nt; su[2][tid] = vs; su[3][tid] = vt; su[4][tid] = bad;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) {
#pragma unroll
      for (int k = 0; k < 8; k += 2) {
        float h = sf[k][tid], l = sf[k + 1][tid];
        df_add(h, l, sf[k][tid + s]);
        l += sf[k + 1][tid + s];
        sf[k][tid] = h;
        sf[k + 1][tid] = l;
      }
#pragma unroll
      for (int k = 0; k < 5; k++) su[k][tid] += su[k][tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const uint32_t Ns = su[0][0], Nt = su[1][0];
    const bool invalid = su[4][0] != 0;
    const float H = sf[0][0] + sf[1][0], G = sf[2][0] + sf[3][0];
    const float Mg = sf[4][0] + sf[5][0], Vv = sf[6][0] + sf[7][0];
    const float N = static_cast<float>(Ns) + static_cast<float>(Nt);
    if (invalid) {
      const float nan = __builtin_nanf("");
      obj[3 * cand] = obj[3 * cand + 1] = obj[3 * cand + 2] = nan;
      flags[cand] = 4;
      severity[cand] = nan;
      counts[2 * cand] = counts[2 * cand + 1] = 0;
    } else {
      obj[3 * cand + 0] = H / N;
      obj[3 * cand + 1] = Mg / (10.0f * static_cast<float>(P.n_tets));
      obj[3 * cand + 2] = G / N;
      flags[cand] = static_cast<uint8_t>((su[2][0] ? 1 : 0) | (su[3][0] ? 2 : 0));
      severity[cand] = Vv;
      counts[2 * cand] = Ns;
      counts[2 * cand + 1] = Nt;
    }
    if (totals) {
      Totals T;
      T.h_hi = sf[0][0]; T.h_lo = sf[1][0]; T.g_hi = sf[2][0]; T.g_lo = sf[3][0];
      T.m_hi = sf[4][0]; T.m_lo = sf[5][0]; T.v_hi = sf[6][0]; T.v_lo = sf[7][0];
      T.n[0] = Ns; T.n[1] = Nt; T.viol[0] = su[2][0]; T.viol[1] = su[3][0];
      T.bad = su[4][0];
      T.pad[0] = T.pad[1] = T.pad[2] = 0;
      totals[cand] = T;
    }
  }
}

// Guidance distance maps: d(p, C) for every set and voxel centre, from the
// set points snapped like mesh coordinates (exact squared distances in
// int64, square root in FP64, rounded to FP32), plus the per-voxel band mask
// of the sets with d < r.
__global__ void k_distance_maps(int nx, int ny, int nz, int n_sets, const int* set_off,
                                const int* pts_fix, float radius, float* dmap, uint8_t* band) {
  const size_t V = static_cast<size_t>(nx) * ny * nz;
  for (size_t v = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; v < V;
       v += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int x = static_cast<int>(v % nx), y = static_cast<int>((v / nx) % ny),
              z = static_cast<int>(v / (static_cast<size_t>(nx) * ny));
    const int64_t px = (int64_t)x * 1024, py = (int64_t)y * 1024, pz = (int64_t)z * 1024;
    unsigned bits = 0;
    for (int s = 0; s < n_sets; s++) {
      int64_t best = INT64_MAX;
      for (int j = set_off[s]; j < set_off[s + 1]; j++) {
        const int64_t dx = px - pts_fix[3 * j], dy = py - pts_fix[3 * j + 1], dz = pz - pts_fix[3 * j + 2];
        const int64_t d2 = dx * dx + dy * dy + dz * dz;
        best = d2 < best ? d2 : best;
      }
      const float d = static_cast<float>(sqrt(static_cast<double>(best)) / 1024.0);
      dmap[static_cast<size_t>(s) * V + v] = d;
      if (d < radius) bits |= 1u << s;
    }
    band[v] = static_cast<uint8_t>(bits);
  }
}

}  // namespace morea

namespace morea {

hipError_t launch_distance_maps(int nx, int ny, int nz, int n_sets, const int* set_off,
                                const int* pts_fix, float radius, float* dmap, uint8_t* band,
                                hipStream_t s) {
  const size_t V = static_cast<size_t>(nx) * ny * nz;
  const int blocks = static_cast<int>(std::min<size_t>((V + 255) / 256, 65536));
  hipLaunchKernelGGL(k_distance_maps, dim3(blocks), dim3(256), 0, s, nx, ny, nz, n_sets, set_off,
                     pts_fix, radius, dmap, band);
  return hipGetLastError();
}

hipError_t launch_eval_full(const ProblemView& P, int storage, const float* pts, int pop,
                            Record* rec, hipStream_t s) {
  const size_t n_items = static_cast<size_t>(pop) * P.n_tets * 2;
  if (n_items == 0) return hipSuccess;
  const int blocks = static_cast<int>((n_items + 3) / 4);
  FullItems F{pts, pop};
  switch (storage) {
    case kF32:
      hipLaunchKernelGGL(k_eval_full<kF32>, dim3(blocks), dim3(256), 0, s, P, F, rec, (int)n_items);
      break;
    case kBF16:
      hipLaunchKernelGGL(k_eval_full<kBF16>, dim3(blocks), dim3(256), 0, s, P, F, rec, (int)n_items);
      break;
    default:
      hipLaunchKernelGGL(k_eval_full<kF16>, dim3(blocks), dim3(256), 0, s, P, F, rec, (int)n_items);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_finalize(const ProblemView& P, const float* pts, int pop, const Record* rec,
                           float* obj, uint8_t* flags, float* severity, uint32_t* counts,
                           Totals* totals, hipStream_t s) {
  if (pop == 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3(pop), dim3(256), 0, s, P, pts, rec, obj, flags, severity,
                     counts, totals);
  return hipGetLastError();
}

}  // namespace morea
