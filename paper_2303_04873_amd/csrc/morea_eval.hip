// Device code of libmorea: per-(candidate, tetrahedron) evaluation by one
// 64-lane wavefront, per-candidate reductions, partial evaluation, and the
// set-up kernel that builds the guidance distance maps.
//
// One wave owns one work item: a tetrahedron of one candidate, evaluated in
// both directions.  Direction 0 rasterizes the source tet on I_s's voxel
// grid, maps each sample into the target tet and samples I_t; direction 1
// does the same with the roles of the two meshes and images exchanged (the
// symmetric objective of Sec. 4.1.2 and the dual-dynamic model of
// Sec. 4.2.1).
//
// Rasterization is exact.  Coordinates are snapped to 2^-10 voxel; each face
// plane value s_i(p) = D * lambda_i(p) is an integer (units 2^-30 voxel^3),
// computed exactly in FP64 when the tet's extent is at most 2^16 units (64
// voxels: every product and partial sum stays below 2^53) and in int64
// otherwise (extent < 2^20 keeps |s_i| < 6 E^3 < 2^63).  A centre on a face
// belongs to the tet iff the face's inward normal is lexicographically
// positive, i.e. p + (e, e^2, e^3) is strictly inside.
//
// Per direction the rows of each slice that can meet the tet are solved 64
// at a time (one per lane); non-empty rows enter a ring in LDS whose samples
// form one stream of two-sample units, consumed 64 units per batch (one per
// lane).  Samples whose mapped point lies within its error bound of a grid
// plane, and samples inside a guidance band, are queued and resolved a full
// wave at a time.
#include <type_traits>

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

// Exclusive prefix sum over the 64 lanes: inclusive scan within each row of
// 16 lanes by DPP row shifts (1, 2, 4, 8), then the row broadcasts of lanes
// 15 and 31 carry it across rows.  Lanes a DPP source does not reach add 0.
__device__ __forceinline__ int wave_excl_scan(int v) {
  int x = v;
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);   // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);   // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);   // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);   // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);   // row_bcast:15 -> rows 1, 3
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);   // row_bcast:31 -> rows 2, 3
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

// 1 / x in FP64: the hardware estimate refined by two Newton steps (relative
// error near 2^-52; every use below carries a margin of at least 2^4 ulp).
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}

__device__ __forceinline__ int64_t floor_div_pos(int64_t a, int64_t b) {  // b > 0
  int64_t q = a / b;
  return (q * b > a) ? q - 1 : q;
}

// Two consecutive floats read by one 8-byte load at 4-byte alignment.
struct __attribute__((aligned(4))) F2 {
  float a, b;
};

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

// Per-direction constants of a work item, written once into the wave's LDS
// and read back by the row and sample loops.  Direction 0 rasterizes the
// source tet S on I_s and samples I_t; direction 1 the target tet T on I_t
// and samples I_s.  Face plane i of the rasterized tet evaluated at voxel
// (lo0 + j, lo1 + yr, lo2 + zr), plus its tie-break bit lex_i, is
//   s_i + lex_i = A_i j + PY_i yr + PZ_i zr + B0_i      (exact integers)
// and the mapped point is q = qlo + M (p - lo).
struct DirConst {
  union {
    struct {
      double A[4], PY[4], PZ[4], B0[4];        // exact in FP64 when the extent is <= 2^16
    };
    struct {
      long long Ai[4], PYi[4], PZi[4], B0i[4]; // int64 form for wider tets (fast == 0)
    };
  };
  double invA[4];
  // x position of face i's plane on row (yr, zr): t_i = TA yr + TB zr + TG
  // (= -(PY yr + PZ zr + B0) / A); for a face with A = 0 the same three
  // numbers hold PY, PZ, B0 (so "t" is the face value itself).  TE bounds the
  // FP64 error of t.
  double TA[4], TB[4], TG[4], TE[4];
  int kind[4];                                 // sign of A_i
  int lex[4];                                  // tie-break bit of face i
  double M[3][3];
  double qlo[3];
  double gthr[3];                              // 0.5 - FP64 error bound of q: near-grid iff |frac(q) - 0.5| >= gthr
  float thr_f[3];                              // the same test on the FP32 fraction (wider margin)
  int64_t absD;
  int fast;                                    // extent <= 2^16: FP64 plane arithmetic
  int sigma;                                   // orientation sign of the rasterized tet
  // bounding box of the rasterized tet on its grid and the row count
  int lo[3], hi[3];
  int W, NYb, R;                               // box width - 1, rows per slice, rows
  int active;                                  // the direction has voxels to visit
  int inner;                                   // mapped points stay inside the padded volume
  // the direction's record, completed by the sample loop
  float h, g, mag, vol;
  uint32_t samples, bits;
};

// 6 x signed volume in FP64: exact when every coordinate difference is
// <= 2^16 (the result is below 6 * 2^48).
__device__ __forceinline__ double det_f64(const int v[4][3]) {
  const double a0 = v[1][0] - v[0][0], a1 = v[1][1] - v[0][1], a2 = v[1][2] - v[0][2];
  const double b0 = v[2][0] - v[0][0], b1 = v[2][1] - v[0][1], b2 = v[2][2] - v[0][2];
  const double c0 = v[3][0] - v[0][0], c1 = v[3][1] - v[0][1], c2 = v[3][2] - v[0][2];
  return a0 * (b1 * c2 - b2 * c1) - a1 * (b0 * c2 - b2 * c0) + a2 * (b0 * c1 - b1 * c0);
}

constexpr int kDeferCap = 64;   // a wave's worth: every append adds at most 64

// Per-item constants in LDS: both directions and the snapped vertices.
struct ItemLds {
  DirConst c[2];
  int vert[24];            // snapped S (12), then T (12)
};

// LDS scratch of one wave: the constants of its two items (the set-up runs
// for both at once, one per half-wave) and the row and sample tables of the
// item being evaluated.
struct WaveLds {
  ItemLds it[2];
  int4 row[kWave];         // padded element of the first sample, the row's first unit in
                           // the unit stream, jx | jy << 10 | jz << 20 (box-relative), length
  union {
    double rowq[kWave][3]; // mapped point of each row's first sample
    struct {               // set-up only, per (half, direction): oriented face normals and
      double n[2][2][4][3];        // the absolute map terms behind the error bound of q
      double Mabs[2][2][3][3];
    } su;
  };
  int4 slice[kWave];       // non-empty slices of a group: z, first row y, first row index, rows
  int mark[kWave];         // row starts inside the current batch, tagged with the batch
  // samples left to the slow paths, resolved a wave at a time; the first
  // word is the box-relative position jx | jy << 10 | jz << 20 | dir << 30:
  //   near-grid: (position, a, b, 0)
  //   in band:   (position, band bits, 0, 1)
  int4 defer[kDeferCap];
  int pre_rows[4], pre_ns[4];   // per (item, direction) unit: rows and non-empty slices of its table
};

// Exact support test of the trilinear stencil (rare path, taken only when
// the mapped coordinate is within its error bound of an integer on some
// axis).  The face values s_i(p) = D * lambda_i(p) come exactly from the
// stored plane constants; the mapped coordinate is the rational
// N / (|D| 2^10), N = sum_i s_i * other_i, in 128-bit integers, and its exact
// floor k decides: if N / (|D| 2^10) == k only corner k carries weight on that
// axis, otherwise corners k and k + 1 do.  Returns whether any supported
// in-grid corner is > 0.
template <int ST>
__device__ __forceinline__ bool exact_foreground(const ProblemView& P, const void* img,
                                                 const ItemLds* I, int d, int jx, int jy, int jz,
                                                 const double q[3], int amb) {
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const DirConst& c = I->c[d];
  const int* oth = I->vert + (d == 0 ? 12 : 0);
  int64_t s[4];
#pragma unroll
  for (int i = 0; i < 4; i++) {
    if (c.fast)
      s[i] = static_cast<int64_t>(fma(c.A[i], jx, fma(c.PY[i], jy, fma(c.PZ[i], jz, c.B0[i]))));
    else
      s[i] = c.Ai[i] * jx + c.PYi[i] * jy + c.PZi[i] * jz + c.B0i[i];
    s[i] -= c.lex[i];
  }
  const __int128 den = static_cast<__int128>(c.absD) * 1024;
  int lo[3], hi[3];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    int k = static_cast<int>(floor(q[a])) - 1;     // q is in padded coordinates
    bool on_grid = false;
    if (amb & (1 << a)) {
      __int128 num = 0;
#pragma unroll
      for (int i = 0; i < 4; i++) num += static_cast<__int128>(s[i]) * oth[3 * i + a];
      // exact floor of num / den from the FP64 estimate; the mapped point is
      // a convex combination of valid vertices, so |k| <= 513
      k = min(max(k, -600), 600);
      while (static_cast<__int128>(k) * den > num) k--;
      while (static_cast<__int128>(k + 1) * den <= num) k++;
      on_grid = static_cast<__int128>(k) * den == num;
    }
    lo[a] = k;
    hi[a] = on_grid ? k : k + 1;
  }
  bool fg = false;
  for (int cz = lo[2]; cz <= hi[2]; cz++)
    for (int cy = lo[1]; cy <= hi[1]; cy++)
      for (int cx = lo[0]; cx <= hi[0]; cx++)
        if (cx >= 0 && cy >= 0 && cz >= 0 && cx < nx && cy < ny && cz < nz)
          fg |= ld_img<ST>(img, (cz + 1) * P.pxy + (cy + 1) * P.px + cx + 1) > 0.0f;
  return fg;
}

// Exact x-interval update for one face: the j with A j + b > 0.  The FP64
// quotient estimate is corrected by one exact evaluation on each side; T is
// double (exact for extents <= 2^16) or int64.
template <typename T>
__device__ __forceinline__ void clip_face(int kind, T A, double invA, T b, int W, int& js, int& je) {
  if (kind > 0) {
    const double t = fmin(fmax(-static_cast<double>(b) * invA, -2.0), W + 1.0);
    int j = static_cast<int>(floor(t)) + 1;
    if (A * static_cast<T>(j) + b <= 0) j += 1;
    else if (A * static_cast<T>(j - 1) + b > 0) j -= 1;
    js = max(js, j);
  } else if (kind < 0) {
    const double t = fmin(fmax(-static_cast<double>(b) * invA, -2.0), W + 1.0);
    int j = static_cast<int>(ceil(t)) - 1;
    if (A * static_cast<T>(j) + b <= 0) j -= 1;
    else if (A * static_cast<T>(j + 1) + b > 0) j += 1;
    je = min(je, j);
  } else if (!(b > 0)) {
    je = -1;
  }
}

// x-interval [js, je] (relative to the box start, within [0, W]) of row
// (yr, zr) of one direction, for tets with extent <= 2^16 (exact FP64 plane
// values).  Face i with kind != 0 crosses zero at the box-relative x position
// t_i = TA yr + TB zr + TG.  The first voxel inside a face with kind > 0 is
// floor(t) + 1 and the last inside a face with kind < 0 is ceil(t) - 1 (a
// centre on the plane is outside once the tie-break bit is folded in), unless
// t is within its FP64 error bound TE of an integer r: then the exact plane
// value at r decides between r and its neighbour.  Branch-free per face.
__device__ __forceinline__ void row_span_fast(const DirConst& c, int yr, int zr, int W, int& js, int& je) {
  js = 0;
  je = W;
  const double y = yr, z = zr;
  bool empty = false;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    // the face's orientation is the same for the whole wave (one item and
    // direction): scalar branches, one rounding path per face
    const int kind = uniform_i(c.kind[i]);
    const double t = fma(c.TA[i], y, fma(c.TB[i], z, c.TG[i]));
    if (kind == 0) {
      // face parallel to x: t holds the plane value itself
      empty = empty || !(t > 0.0);
      continue;
    }
    // a crossing beyond [-2, W + 1] leaves the row full or empty either way:
    // floor / ceil of the clamped value decide it without the exact test
    const double tc = fmin(fmax(t, -2.0), W + 1.0);
    const double r = rint(tc);
    const bool near = tc == t && fabs(tc - r) <= c.TE[i];
    int j = kind > 0 ? static_cast<int>(floor(tc)) + 1 : static_cast<int>(ceil(tc)) - 1;
    if (__ballot(near)) {
      // rare: the exact plane value (+ tie-break bit) at x = r decides;
      // |terms| < 2^50
      const double e = fma(c.A[i], r, fma(c.PY[i], y, fma(c.PZ[i], z, c.B0[i])));
      const int ri = static_cast<int>(r);
      const int jx = kind > 0 ? (e > 0.0 ? ri : ri + 1) : (e > 0.0 ? ri : ri - 1);
      j = near ? jx : j;
    }
    if (kind > 0)
      js = max(js, j);
    else
      je = min(je, j);
  }
  if (empty) je = -1;
}

// The same for wider tets, in int64 (extent < 2^20 keeps |s_i| < 2^63).
__device__ __forceinline__ void row_span_wide(const DirConst& c, int yr, int zr, int W, int& js, int& je) {
  js = 0;
  je = W;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    const long long b = c.PYi[i] * yr + c.PZi[i] * zr + c.B0i[i];
    clip_face<long long>(c.kind[i], c.Ai[i], c.invA[i], b, W, js, je);
  }
}

// Rows of one slice that can hold samples: the y-range of the cross-section
// of the tet (vertices `v`, fixed point) with the plane z = Z, from the
// intersections of its 6 edges with the plane, widened by 1/16 voxel (the
// FP32 error is below one fixed-point unit) and clipped to [ylo, yhi].
// Every sample of the slice lies in this range; the row spans decide
// exactly.  Returns the first row relative to ylo and the row count.
__device__ __forceinline__ void slice_rows(const int* v, int Z, int ylo, int yhi, int& y0, int& cnt) {
  const int zf = Z * 1024;
  float mn = 3.0e38f, mx = -3.0e38f;
#pragma unroll
  for (int e = 0; e < 6; e++) {
    const int i = e < 3 ? 0 : (e < 5 ? 1 : 2);
    const int j = e < 3 ? e + 1 : (e < 5 ? e - 1 : 3);
    const int zi = v[3 * i + 2] - zf, zj = v[3 * j + 2] - zf;
    const float yi = static_cast<float>(v[3 * i + 1]), yj = static_cast<float>(v[3 * j + 1]);
    if ((zi <= 0 && zj >= 0) || (zi >= 0 && zj <= 0)) {
      if (zi == zj) {
        mn = fminf(mn, fminf(yi, yj));
        mx = fmaxf(mx, fmaxf(yi, yj));
      } else {
        const float t = static_cast<float>(-zi) * __builtin_amdgcn_rcpf(static_cast<float>(zj - zi));
        const float y = fmaf(t, yj - yi, yi);
        mn = fminf(mn, y);
        mx = fmaxf(mx, y);
      }
    }
  }
  const int a = max(ylo, static_cast<int>(ceilf((mn - 64.f) * (1.f / 1024.f))));
  const int b = min(yhi, static_cast<int>(floorf((mx + 64.f) * (1.f / 1024.f))));
  y0 = a - ylo;
  cnt = max(0, b - a + 1);
}

// Buffer resources over padded volumes: element i is byte offset i * size.
// A buffer load outside the resource returns 0 instead of faulting.
template <int ST>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t image_rsrc(const void* img, unsigned pvox) {
  constexpr unsigned esize = ST == kF32 ? 4 : 2;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(img), static_cast<short>(0),
                                           static_cast<int>(pvox * esize), 0x00020000);
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t byte_rsrc(const uint8_t* p, unsigned n) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(p), static_cast<short>(0),
                                           static_cast<int>(n), 0x00020000);
}

template <int ST>
__device__ __forceinline__ float ld_buf(__amdgpu_buffer_rsrc_t r, int idx) {
  if constexpr (ST == kF32) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, static_cast<unsigned>(idx) * 4u, 0, 0));
  } else {
    const unsigned short u = __builtin_amdgcn_raw_buffer_load_b16(r, static_cast<unsigned>(idx) * 2u, 0, 0);
    if constexpr (ST == kBF16)
      return __uint_as_float(static_cast<uint32_t>(u) << 16);
    else
      return static_cast<float>(__builtin_bit_cast(_Float16, u));
  }
}

// Two consecutive FP32 voxels (idx, idx + 1) in one 8-byte buffer load; the
// scalar offset `soff` (bytes) selects the row of the pair.
__device__ __forceinline__ F2 ld_pair(__amdgpu_buffer_rsrc_t r, int idx, int soff) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  const f2v v = __builtin_bit_cast(
      f2v, __builtin_amdgcn_raw_buffer_load_b64(r, static_cast<unsigned>(idx) * 4u, soff, 0));
  return F2{v.x, v.y};
}

// Two consecutive 2-byte voxels (idx, idx + 1) as one 32-bit word (idx in
// the low half): one 8-byte load of the 4-element window that starts at the
// even element idx & ~1 (4-byte aligned, as every row and slice offset `soff`
// of a 2-byte volume), then a 16-bit funnel shift when idx is odd.
__device__ __forceinline__ uint32_t ld_pair16(__amdgpu_buffer_rsrc_t r, int idx, int soff, uint32_t shift) {
  typedef unsigned u2v __attribute__((ext_vector_type(2)));
  const u2v w = __builtin_bit_cast(
      u2v, __builtin_amdgcn_raw_buffer_load_b64(r, static_cast<unsigned>(idx & ~1) * 2u, soff, 0));
  return __builtin_amdgcn_alignbit(w.y, w.x, shift);
}

template <int ST>
__device__ __forceinline__ float lo16(uint32_t w) {
  if constexpr (ST == kBF16)
    return __uint_as_float(w << 16);
  else
    return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<unsigned short>(w)));
}

template <int ST>
__device__ __forceinline__ float hi16(uint32_t w) {
  if constexpr (ST == kBF16)
    return __uint_as_float(w & 0xffff0000u);
  else
    return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<unsigned short>(w >> 16)));
}

__device__ __forceinline__ double uniform_d(double v) {
  const uint64_t b = static_cast<uint64_t>(__double_as_longlong(v));
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(b));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(b >> 32));
  return __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(hi) << 32) | lo));
}

__device__ __forceinline__ float uniform_f(float v) {
  return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(v)));
}

// Wave-uniform constants of one direction's sample loop (scalar registers).
struct SampleConst {
  double m0, m1, m2;    // M[:, 0]: step of the mapped point per voxel along x
  float thr;            // near-grid threshold on max_a |frac(q_a) - 1/2|
};

// One voxel sample of direction d whose mapped points may leave the padded
// volume (a tet near or beyond the image border): the centre at padded
// element vi, its mapped point (padded coordinates) q = q_row + k * M[:, 0]
// (q_row of the sample's row, k its offset in the row).  Samples the other
// image trilinearly (zero outside the grid, corners clamped for the distance
// maps), adds h (Sec. 4.1.2) and, inside the guidance band, the set-weighted
// guidance term (Sec. 4.1.3, App. A.3).  Returns true when the mapped point
// is within its error bound of a grid plane on some axis: that sample's h is
// left to the exact path (a_out and b_out carry what it needs).
template <int ST>
__device__ __forceinline__ bool sample_one(const ProblemView& P, const SampleConst& U,
                                           __amdgpu_buffer_rsrc_t r_own, __amdgpu_buffer_rsrc_t r_oth,
                                           __amdgpu_buffer_rsrc_t r_band, int d, int vi,
                                           const double qr[3], int k, float& h_acc, float& g_acc,
                                           float& a_out, float& b_out) {
  const float a = ld_buf<ST>(r_own, vi);
  const double kd = static_cast<double>(k);
  const double q[3] = {fma(U.m0, kd, qr[0]), fma(U.m1, kd, qr[1]), fma(U.m2, kd, qr[2])};
  float f[3];
  int c[3];
#pragma unroll
  for (int t = 0; t < 3; t++) {
    const double fl = floor(q[t]);
    c[t] = static_cast<int>(fl);
    f[t] = static_cast<float>(q[t] - fl);
  }
  const bool amb = fabsf(f[0] - 0.5f) >= U.thr || fabsf(f[1] - 0.5f) >= U.thr || fabsf(f[2] - 0.5f) >= U.thr;

  // corner indices (padded elements): x pair ix0/ix1, row offsets ry0/ry1,
  // slice offsets rz0/rz1.  The padded index range per axis is [0, n + 1];
  // corners beyond it are outside the image (value 0) and clamp for the
  // distance maps
  const int n0 = P.nx + 1, n1 = P.ny + 1, n2 = P.nz + 1;
  const int ix0 = min(max(c[0], 0), n0), ix1 = min(max(c[0] + 1, 0), n0);
  const int cy0 = min(max(c[1], 0), n1), cy1 = min(max(c[1] + 1, 0), n1);
  const int cz0 = min(max(c[2], 0), n2), cz1 = min(max(c[2] + 1, 0), n2);
  const int ry0 = __umul24(cy0, P.px), ry1 = __umul24(cy1, P.px);
  const int rz0 = __umul24(cz0, P.pxy), rz1 = __umul24(cz1, P.pxy);
  const bool vx0 = c[0] >= 0 && c[0] <= n0, vx1 = c[0] >= -1 && c[0] < n0;
  const bool vy0 = c[1] >= 0 && c[1] <= n1, vy1 = c[1] >= -1 && c[1] < n1;
  const bool vz0 = c[2] >= 0 && c[2] <= n2, vz1 = c[2] >= -1 && c[2] < n2;
  float v000 = ld_buf<ST>(r_oth, rz0 + ry0 + ix0), v001 = ld_buf<ST>(r_oth, rz0 + ry0 + ix1);
  float v010 = ld_buf<ST>(r_oth, rz0 + ry1 + ix0), v011 = ld_buf<ST>(r_oth, rz0 + ry1 + ix1);
  float v100 = ld_buf<ST>(r_oth, rz1 + ry0 + ix0), v101 = ld_buf<ST>(r_oth, rz1 + ry0 + ix1);
  float v110 = ld_buf<ST>(r_oth, rz1 + ry1 + ix0), v111 = ld_buf<ST>(r_oth, rz1 + ry1 + ix1);
  v000 = (vz0 && vy0 && vx0) ? v000 : 0.f;
  v001 = (vz0 && vy0 && vx1) ? v001 : 0.f;
  v010 = (vz0 && vy1 && vx0) ? v010 : 0.f;
  v011 = (vz0 && vy1 && vx1) ? v011 : 0.f;
  v100 = (vz1 && vy0 && vx0) ? v100 : 0.f;
  v101 = (vz1 && vy0 && vx1) ? v101 : 0.f;
  v110 = (vz1 && vy1 && vx0) ? v110 : 0.f;
  v111 = (vz1 && vy1 && vx1) ? v111 : 0.f;
  // any corner > 0 (the images are >= 0: any non-zero magnitude bit)
  const uint32_t ob = __float_as_uint(v000) | __float_as_uint(v001) | __float_as_uint(v010) |
                      __float_as_uint(v011) | __float_as_uint(v100) | __float_as_uint(v101) |
                      __float_as_uint(v110) | __float_as_uint(v111);
  const bool fg8 = (ob << 1) != 0u;
  const float e00 = fmaf(f[0], v001 - v000, v000), e01 = fmaf(f[0], v011 - v010, v010);
  const float e10 = fmaf(f[0], v101 - v100, v100), e11 = fmaf(f[0], v111 - v110, v110);
  const float e0 = fmaf(f[1], e01 - e00, e00), e1 = fmaf(f[1], e11 - e10, e10);
  const float b = fmaf(f[2], e1 - e0, e0);

  if (P.n_sets > 0) {
    unsigned bandbits = __builtin_amdgcn_raw_buffer_load_b8(r_band, static_cast<unsigned>(vi), 0, 0);
    if (bandbits) {
      const float r = P.radius, inv_r = P.inv_radius;
      const float* map_own = d ? P.dmap[1] : P.dmap[0];
      const float* map_oth = d ? P.dmap[0] : P.dmap[1];
      const int i00 = rz0 + ry0, i01 = rz0 + ry1, i10 = rz1 + ry0, i11 = rz1 + ry1;
      while (bandbits) {
        const int sidx = __builtin_ctz(bandbits);
        bandbits &= bandbits - 1;
        const float* mo = map_oth + static_cast<size_t>(sidx) * P.pvox;
        const float dist = map_own[static_cast<size_t>(sidx) * P.pvox + vi];
        const float u00 = fmaf(f[0], mo[i00 + ix1] - mo[i00 + ix0], mo[i00 + ix0]);
        const float u01 = fmaf(f[0], mo[i01 + ix1] - mo[i01 + ix0], mo[i01 + ix0]);
        const float u10 = fmaf(f[0], mo[i10 + ix1] - mo[i10 + ix0], mo[i10 + ix0]);
        const float u11 = fmaf(f[0], mo[i11 + ix1] - mo[i11 + ix0], mo[i11 + ix0]);
        const float u0 = fmaf(f[1], u01 - u00, u00), u1 = fmaf(f[1], u11 - u10, u10);
        const float d2 = fmaf(f[2], u1 - u0, u0);
        const float diff = dist - d2;
        g_acc += P.set_w[d * kMaxSets + sidx] * ((r - dist) * inv_r) * diff * diff;
      }
    }
  }
  // foreground of the interpolated sample: any of the 8 corners, unless the
  // mapped point is within its error bound of a grid plane (rare): then the
  // exact support decides, later, from the deferred queue
  a_out = a;
  b_out = b;
  if (amb) return true;
  const bool fg_a = a > 0.f;
  const float dd = a - b;
  h_acc += (fg_a && fg8) ? dd * dd : ((fg_a != fg8) ? 1.f : 0.f);
  return false;
}

// Guidance term of one in-band sample (Sec. 4.1.3, App. A.3): for every set
// whose band holds the sample, the set-weighted (r - d)/r (d - d')^2 with d
// from the own map at vi and d' the trilinear value of the other map (corner
// rows i00..i11, x pair ix0/ix1, fractions f).
__device__ __forceinline__ void guidance(const ProblemView& P, int d, unsigned bandbits, int vi, int i00,
                                         int i01, int i10, int i11, int ix0, int ix1, const float f[3],
                                         float& g_acc) {
  const float r = P.radius, inv_r = P.inv_radius;
  const float* map_own = d ? P.dmap[1] : P.dmap[0];
  const float* map_oth = d ? P.dmap[0] : P.dmap[1];
  while (bandbits) {
    const int sidx = __builtin_ctz(bandbits);
    bandbits &= bandbits - 1;
    const float* mo = map_oth + static_cast<size_t>(sidx) * P.pvox;
    const float dist = map_own[static_cast<size_t>(sidx) * P.pvox + vi];
    const float u00 = fmaf(f[0], mo[i00 + ix1] - mo[i00 + ix0], mo[i00 + ix0]);
    const float u01 = fmaf(f[0], mo[i01 + ix1] - mo[i01 + ix0], mo[i01 + ix0]);
    const float u10 = fmaf(f[0], mo[i10 + ix1] - mo[i10 + ix0], mo[i10 + ix0]);
    const float u11 = fmaf(f[0], mo[i11 + ix1] - mo[i11 + ix0], mo[i11 + ix0]);
    const float u0 = fmaf(f[1], u01 - u00, u00), u1 = fmaf(f[1], u11 - u10, u10);
    const float d2 = fmaf(f[2], u1 - u0, u0);
    const float diff = dist - d2;
    g_acc += P.set_w[d * kMaxSets + sidx] * ((r - dist) * inv_r) * diff * diff;
  }
}

// Two consecutive samples of one row (x offsets k and k + 1, padded
// elements vi + k and vi + k + 1) for a direction whose mapped points stay
// inside the padded volume.  Straight-line: both samples' loads are issued
// before either is interpolated; loads for an invalid sample read whatever
// in-resource memory its address names (a buffer load cannot fault) and are
// discarded.  For each valid sample h is added unless the mapped point is
// within its error bound of a grid plane (amb: left to the exact path with
// a, b); its band bits are returned for the guidance term, which the
// slow-path queue adds (band is 0 for an invalid sample).
template <int ST>
__device__ __forceinline__ void sample_pair_inner(const ProblemView& P, const SampleConst& U,
                                                  __amdgpu_buffer_rsrc_t r_own, __amdgpu_buffer_rsrc_t r_oth,
                                                  __amdgpu_buffer_rsrc_t r_band, int d, int vi, const double qr[3],
                                                  int k, bool v0, bool v1, float& h_acc, bool amb[2],
                                                  float a[2], float b[2], unsigned band[2]) {
  const int e0 = vi + k;
  float f[2][3];
  int base[2];
#pragma unroll
  for (int s = 0; s < 2; s++) {
    const double kd = static_cast<double>(k + s);
    int c[3];
#pragma unroll
    for (int t = 0; t < 3; t++) {
      const double q = fma(t == 0 ? U.m0 : (t == 1 ? U.m1 : U.m2), kd, qr[t]);
      c[t] = static_cast<int>(q);     // q > 0 for a valid sample: truncation is the floor
      f[s][t] = static_cast<float>(__builtin_amdgcn_fract(q));
    }
    base[s] = __umul24(c[2], P.pxy) + __umul24(c[1], P.px) + c[0];
    amb[s] = fabsf(f[s][0] - 0.5f) >= U.thr || fabsf(f[s][1] - 0.5f) >= U.thr || fabsf(f[s][2] - 0.5f) >= U.thr;
  }
  // loads: own voxels (one pair), the 2 x 4 corner pairs, the two band bytes
  float v[2][8];
  bool fg8[2];
  constexpr int esize = ST == kF32 ? 4 : 2;
  const int sy = P.px * esize, sz = P.pxy * esize;   // row and slice offsets in bytes
  if constexpr (ST == kF32) {
    const F2 own = ld_pair(r_own, e0, 0);
    a[0] = own.a;
    a[1] = own.b;
#pragma unroll
    for (int s = 0; s < 2; s++) {
      const F2 p00 = ld_pair(r_oth, base[s], 0), p01 = ld_pair(r_oth, base[s], sy);
      const F2 p10 = ld_pair(r_oth, base[s], sz), p11 = ld_pair(r_oth, base[s], sy + sz);
      v[s][0] = p00.a; v[s][1] = p00.b; v[s][2] = p01.a; v[s][3] = p01.b;
      v[s][4] = p10.a; v[s][5] = p10.b; v[s][6] = p11.a; v[s][7] = p11.b;
    }
  } else {
    const uint32_t own = ld_pair16(r_own, e0, 0, static_cast<uint32_t>(e0 & 1) << 4);
    a[0] = lo16<ST>(own);
    a[1] = hi16<ST>(own);
#pragma unroll
    for (int s = 0; s < 2; s++) {
      const uint32_t sh = static_cast<uint32_t>(base[s] & 1) << 4;
      const uint32_t w00 = ld_pair16(r_oth, base[s], 0, sh), w01 = ld_pair16(r_oth, base[s], sy, sh);
      const uint32_t w10 = ld_pair16(r_oth, base[s], sz, sh), w11 = ld_pair16(r_oth, base[s], sy + sz, sh);
      v[s][0] = lo16<ST>(w00); v[s][1] = hi16<ST>(w00); v[s][2] = lo16<ST>(w01); v[s][3] = hi16<ST>(w01);
      v[s][4] = lo16<ST>(w10); v[s][5] = hi16<ST>(w10); v[s][6] = lo16<ST>(w11); v[s][7] = hi16<ST>(w11);
      if (!P.fg_from_b) fg8[s] = ((w00 | w01 | w10 | w11) & 0x7fff7fffu) != 0u;
    }
  }
  // the band mask is all zero when the problem has no guidance sets
  band[0] = __builtin_amdgcn_raw_buffer_load_b8(r_band, static_cast<unsigned>(e0), 0, 0);
  band[1] = __builtin_amdgcn_raw_buffer_load_b8(r_band, static_cast<unsigned>(e0) + 1u, 0, 0);
#pragma unroll
  for (int s = 0; s < 2; s++) {
    const float* w = v[s];
    const float e00 = fmaf(f[s][0], w[1] - w[0], w[0]), e01 = fmaf(f[s][0], w[3] - w[2], w[2]);
    const float e10 = fmaf(f[s][0], w[5] - w[4], w[4]), e11 = fmaf(f[s][0], w[7] - w[6], w[6]);
    const float ea = fmaf(f[s][1], e01 - e00, e00), eb = fmaf(f[s][1], e11 - e10, e10);
    b[s] = fmaf(f[s][2], eb - ea, ea);
    if (P.fg_from_b) {
      fg8[s] = b[s] > 0.f;
    } else if constexpr (ST == kF32) {
      const uint32_t ob = __float_as_uint(w[0]) | __float_as_uint(w[1]) | __float_as_uint(w[2]) |
                          __float_as_uint(w[3]) | __float_as_uint(w[4]) | __float_as_uint(w[5]) |
                          __float_as_uint(w[6]) | __float_as_uint(w[7]);
      fg8[s] = (ob << 1) != 0u;
    }
    const bool fg_a = a[s] > 0.f;
    const float dd = a[s] - b[s];
    const float hv = (fg_a && fg8[s]) ? dd * dd : ((fg_a != fg8[s]) ? 1.f : 0.f);
    const bool valid = s == 0 ? v0 : v1;
    amb[s] = amb[s] && valid;
    if (!valid) band[s] = 0u;
    if (valid && !amb[s]) h_acc += hv;
  }
}

// Resolve the queued samples of a wave, one per lane; the mapped point is
// recomputed in FP64 from the item constants.  Near-grid samples: the axes
// near a grid plane are found again and the foreground is decided on the
// exact support; h is added.  In-band samples (queued only by directions
// whose mapped points stay inside the padded volume): the guidance term is
// added.
template <int ST>
__device__ __forceinline__ void flush_deferred(const ProblemView& P, const WaveLds* L, const ItemLds* I,
                                               int count, float& h_acc, float& g_acc) {
  const int lane = lane_id();
  for (int base = 0; base < count; base += kWave) {
    const int e = base + lane;
    if (e >= count) continue;
    const int4 q4 = L->defer[e];
    const int jx = q4.x & 1023, jy = (q4.x >> 10) & 1023, jz = (q4.x >> 20) & 1023, d = (q4.x >> 30) & 1;
    const DirConst& C = I->c[d];
    double q[3];
#pragma unroll
    for (int k = 0; k < 3; k++)
      q[k] = fma(C.M[k][0], static_cast<double>(jx),
                 fma(C.M[k][1], static_cast<double>(jy), fma(C.M[k][2], static_cast<double>(jz), C.qlo[k])));
    if (q4.w != 0) {
      int c[3];
      float f[3];
#pragma unroll
      for (int k = 0; k < 3; k++) {
        c[k] = static_cast<int>(q[k]);
        f[k] = static_cast<float>(__builtin_amdgcn_fract(q[k]));
      }
      const int vi = (C.lo[2] + jz + 1) * P.pxy + (C.lo[1] + jy + 1) * P.px + C.lo[0] + jx + 1;
      const int i00 = c[2] * P.pxy + c[1] * P.px;
      guidance(P, d, static_cast<unsigned>(q4.y), vi, i00, i00 + P.px, i00 + P.pxy, i00 + P.pxy + P.px, c[0],
               c[0] + 1, f, g_acc);
      continue;
    }
    const float a = __int_as_float(q4.y), b = __int_as_float(q4.z);
    int axes = 0;
#pragma unroll
    for (int k = 0; k < 3; k++)
      if (fabs(q[k] - floor(q[k]) - 0.5) >= C.gthr[k]) axes |= 1 << k;
    const bool fg_b = exact_foreground<ST>(P, d ? P.img[0] : P.img[1], I, d, jx, jy, jz, q, axes);
    const bool fg_a = a > 0.f;
    const float dd = a - (fg_b ? b : 0.f);
    h_acc += (fg_a && fg_b) ? dd * dd : ((fg_a != fg_b) ? 1.f : 0.f);
  }
}

// Evaluate two items (a tet of a candidate each) in both directions.  The
// set-up runs for both at once, item s on half-wave s (lanes 32 s .. 32 s +
// 31); rows and samples then take one item after the other on the whole
// wave.  Lanes 0..11 of a half hold the source tet's coordinates (v0x v0y
// v0z v1x ...), lanes 12..23 the target tet's (`coord`).  Item s writes
// out_s[0] (direction 0) and out_s[1]; item 1 exists only when has1.
template <int ST>
__device__ void eval_tet(const ProblemView& P, int tet0, int tet1, bool has1, float coord, WaveLds* L,
                         Record* out0, Record* out1) {
  // the lane index is made opaque so that values derived from it are not
  // hoisted out of the persistent partial-evaluation loop (they would stay
  // live across every item and cost registers, i.e. occupancy)
  int lane = lane_id();
  asm volatile("" : "+v"(lane));
  const int half = lane >> 5, hl = lane & 31;
  ItemLds* I = &L->it[half];
  const int tet = half ? tet1 : tet0;
  // ---- snap and validate (the loading lane snaps its own coordinate)
  const bool in_range = hl >= 24 || fabsf(coord) < kCoordLimit;
  const uint64_t ok_mask = __ballot(in_range);
  const bool ok0 = static_cast<uint32_t>(ok_mask) == 0xffffffffu;
  const bool ok1 = has1 && static_cast<uint32_t>(ok_mask >> 32) == 0xffffffffu;
  const int fix = (hl < 24 && in_range) ? static_cast<int>(rintf(coord * kFixOne)) : 0;
  if (!ok0 && lane < 2) out0[lane] = Record{0.f, 0.f, 0u, 0.f, 0.f, 4u};
  if (has1 && !ok1 && lane >= 32 && lane < 34) out1[lane - 32] = Record{0.f, 0.f, 0u, 0.f, 0.f, 4u};
  if (!ok0 && !ok1) return;
  if (hl < 24) I->vert[hl] = fix;
  wave_sync();
  // ---- per direction: box on its grid, fold check (App. A.4), interior
  // flag; lanes 0..15 of a half take mesh 0, lanes 16..31 mesh 1.  The
  // values go to the item's LDS block so that only the current direction's
  // copy is live in the sample loop.
  const int dims[3] = {P.nx, P.ny, P.nz};
  const int ref = P.ref_sign[tet];
  bool active;
  {
    const int m = hl >> 4;
    int V[4][3];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
      for (int k = 0; k < 3; k++) V[i][k] = I->vert[12 * m + 3 * i + k];
    int ext = 0, lo[3], hi[3];
    bool interior = true;
#pragma unroll
    for (int k = 0; k < 3; k++) {
      const int mn = min(min(V[0][k], V[1][k]), min(V[2][k], V[3][k]));
      const int mx = max(max(V[0][k], V[1][k]), max(V[2][k], V[3][k]));
      ext = max(ext, mx - mn);
      lo[k] = max(0, -static_cast<int>(floor_div_pos(-static_cast<int64_t>(mn), 1024)));
      hi[k] = min(dims[k] - 1, static_cast<int>(floor_div_pos(mx, 1024)));
      // the tet of mesh m is sampled by direction 1 - m: every trilinear
      // corner of a mapped point lies in the padded volume when the tet is
      // inside (-1, n) by at least 2^-10 voxel
      interior = interior && mn >= -1023 && mx <= 1024 * dims[k] - 1;
    }
    const bool fast = ext <= kFastExtent;
    // FP64 is exact for extents <= 2^16: |6V| <= 6 E^3 < 2^53
    const int64_t D = fast ? static_cast<int64_t>(det_f64(V)) : det_i64(V);
    const int sg = (D > 0) - (D < 0);
    const bool viol = (sg == 0) || (sg != ref);
    const int64_t absD = D < 0 ? -D : D;
    active = D != 0 && lo[0] <= hi[0] && lo[1] <= hi[1] && lo[2] <= hi[2];
    if ((hl & 15) == 0) {
      DirConst& C = I->c[m];
      C.absD = absD;
      C.fast = fast ? 1 : 0;
      C.sigma = D > 0 ? 1 : -1;
#pragma unroll
      for (int k = 0; k < 3; k++) {
        C.lo[k] = lo[k];
        C.hi[k] = hi[k];
      }
      C.W = hi[0] - lo[0];
      C.NYb = hi[1] - lo[1] + 1;
      C.R = active ? C.NYb * (hi[2] - lo[2] + 1) : 0;
      C.active = active ? 1 : 0;
      I->c[1 - m].inner = interior ? 1 : 0;
      C.h = 0.f;
      C.g = 0.f;
      C.samples = 0u;
      C.mag = 0.f;
      C.vol = viol ? static_cast<float>(static_cast<double>(absD) * (1.0 / (6.0 * 1073741824.0))) : 0.f;
      C.bits = viol ? 1u : 0u;
    }
  }
  // items with samples to visit (a half-wave value made wave-uniform)
  const uint64_t act_mask = __ballot(active && (half ? ok1 : ok0));
  const bool act0 = (act_mask & 0xffffffffull) != 0, act1 = (act_mask >> 32) != 0;

  wave_sync();   // the box constants are read below

  // ---- one pass over lanes 0..17 of each half: set-up phase 1 on lanes
  // 0..7 (below) and the deformation magnitude on lanes 8..17.
  // Deformation magnitude (Sec. 4.1.1), one edge per lane:
  // |e_s| - |e_t| = (|e_s|^2 - |e_t|^2) / (|e_s| + |e_t|) with the squared
  // lengths exact in FP64 (components < 2^22, sums < 2^46).
  {
    float term = 0.f;
    const int e = hl - 8;   // the magnitude's edge (lanes 8..17 of the half)
    if (e >= 0 && e < 10) {
      double ls = 0.0, lt = 0.0;
      float scale;
      if (e < 6) {
        const int i = e < 3 ? 0 : (e < 5 ? 1 : 2);
        const int j = e < 3 ? e + 1 : (e < 5 ? e - 1 : 3);
#pragma unroll
        for (int k = 0; k < 3; k++) {
          const double ds = I->vert[3 * i + k] - I->vert[3 * j + k];
          const double dt = I->vert[12 + 3 * i + k] - I->vert[12 + 3 * j + k];
          ls = fma(ds, ds, ls);
          lt = fma(dt, dt, lt);
        }
        scale = 1.0f / kFixOne;
      } else {
        const int v = e - 6;
#pragma unroll
        for (int k = 0; k < 3; k++) {
          const int ss = I->vert[k] + I->vert[3 + k] + I->vert[6 + k] + I->vert[9 + k];
          const int st = I->vert[12 + k] + I->vert[15 + k] + I->vert[18 + k] + I->vert[21 + k];
          const double ds = 4 * I->vert[3 * v + k] - ss;
          const double dt = 4 * I->vert[12 + 3 * v + k] - st;
          ls = fma(ds, ds, ls);
          lt = fma(dt, dt, lt);
        }
        scale = 1.0f / (4.0f * kFixOne);
      }
      // hardware square root and reciprocal (about 1 ulp each)
      const float den = __builtin_amdgcn_sqrtf(static_cast<float>(ls)) + __builtin_amdgcn_sqrtf(static_cast<float>(lt));
      const float dd = den > 0.f ? static_cast<float>(ls - lt) * __builtin_amdgcn_rcpf(den) * scale : 0.f;
      term = dd * dd;
    }
    // the sum within each half-wave (butterfly over lane bits 0..4)
#pragma unroll
    for (int d = 16; d >= 1; d >>= 1) term += __shfl_xor(term, d, 64);
    const float mag = P.elasticity[tet] * term;
    if (hl == 0) I->c[0].mag = mag;
  }
  // set-up phase 1, lanes 0..7 of each half (direction d = hl / 4, face
  // i): face plane (gradient of D * lambda_i oriented inwards, its value at
  // the box corner, the row-boundary estimate)
  if (hl < 8) {
    const int d = hl >> 2, i = hl & 3;
    DirConst& C = I->c[d];
    const int* own = I->vert + 12 * d;
    const int sigma = C.sigma;
    const int b0 = i == 0 ? 1 : 0;                            // base vertex on the face
    const int u0 = i == 0 ? 2 : (i == 1 ? 2 : (i == 2 ? 3 : 1));
    const int w0 = i == 0 ? 3 : (i == 1 ? 3 : (i == 2 ? 1 : 2));
    double u[3], w[3], r[3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
      const int rk = own[3 * b0 + k];
      r[k] = rk;
      u[k] = own[3 * u0 + k] - rk;
      w[k] = own[3 * w0 + k] - rk;
    }
    // cross product: |components| < 2^41, exact in FP64
    const double sg = (i == 0 ? -sigma : sigma);
    const double nx_ = sg * (u[1] * w[2] - u[2] * w[1]);
    const double ny_ = sg * (u[2] * w[0] - u[0] * w[2]);
    const double nz_ = sg * (u[0] * w[1] - u[1] * w[0]);
    L->su.n[half][d][i][0] = nx_;
    L->su.n[half][d][i][1] = ny_;
    L->su.n[half][d][i][2] = nz_;
    const int lex = (nx_ > 0 || (nx_ == 0 && (ny_ > 0 || (ny_ == 0 && nz_ > 0)))) ? 1 : 0;
    const double ox = 1024.0 * C.lo[0] - r[0], oy = 1024.0 * C.lo[1] - r[1], oz = 1024.0 * C.lo[2] - r[2];
    const double A = nx_ * 1024.0, PY = ny_ * 1024.0, PZ = nz_ * 1024.0;
    C.A[i] = A;
    C.PY[i] = PY;
    C.PZ[i] = PZ;
    const double invA = nx_ != 0 ? rcp64(A) : 0.0;
    C.invA[i] = invA;
    const int kind = (nx_ > 0) - (nx_ < 0);
    C.kind[i] = kind;
    C.lex[i] = lex;
    if (C.fast) {
      // |terms| <= 2 E^3 <= 2^49: exact
      const double B0 = fma(nx_, ox, fma(ny_, oy, nz_ * oz)) + lex;
      C.B0[i] = B0;
      if (kind != 0) {
        const double ta = -PY * invA, tb = -PZ * invA, tg = -B0 * invA;
        C.TA[i] = ta;
        C.TB[i] = tb;
        C.TG[i] = tg;
        C.TE[i] = (fabs(ta) * C.NYb + fabs(tb) * (C.hi[2] - C.lo[2] + 1) + fabs(tg) + 128.0) * 0x1p-48;
      } else {
        C.TA[i] = PY;
        C.TB[i] = PZ;
        C.TG[i] = B0;
        C.TE[i] = 0.0;
      }
    } else {
      const long long nxi = static_cast<long long>(nx_), nyi = static_cast<long long>(ny_),
                      nzi = static_cast<long long>(nz_);
      C.Ai[i] = nxi * 1024;
      C.PYi[i] = nyi * 1024;
      C.PZi[i] = nzi * 1024;
      C.B0i[i] = nxi * static_cast<long long>(ox) + nyi * static_cast<long long>(oy) +
                 nzi * static_cast<long long>(oz) + lex;
    }
  }
  wave_sync();
  if (!act0 && !act1) {
    if (ok0 && lane < 2) {
      const DirConst& C = L->it[0].c[lane];
      out0[lane] = Record{0.f, 0.f, 0u, C.mag, C.vol, C.bits};
    }
    if (ok1 && lane >= 32 && lane < 34) {
      const DirConst& C = L->it[1].c[lane - 32];
      out1[lane - 32] = Record{0.f, 0.f, 0u, C.mag, C.vol, C.bits};
    }
    return;
  }
  // phase 2, lanes 0..17 of each half: map entry M[a][c] of direction
  // d = hl / 9: sum_i b_i[a] adj_i[c] / D with b_i = oth_i - oth_0 and
  // adj_i = sigma n_i (i = 1..3), the rows of adj(E)
  if (hl < 18) {
    const int d = hl / 9, a = (hl % 9) / 3, cc = hl % 3;
    DirConst& C = I->c[d];
    const int* oth = I->vert + 12 * (1 - d);
    const double sigma = C.sigma;
    const double invD = sigma * rcp64(static_cast<double>(C.absD != 0 ? C.absD : 1));
    const double oth0 = oth[a];
    double num = 0.0, mag = 0.0;
#pragma unroll
    for (int i = 0; i < 3; i++) {
      const double bi = static_cast<double>(oth[3 * (i + 1) + a]) - oth0;
      const double t = bi * (sigma * L->su.n[half][d][i + 1][cc]);
      num += t;
      mag += fabs(t);
    }
    C.M[a][cc] = num * invD;
    L->su.Mabs[half][d][a][cc] = mag * fabs(invD);
  }
  wave_sync();
  // phase 3, lanes 0..5 of each half: q at the box corner (padded
  // coordinates: grid coordinate + 1) and the FP64 error bound of q
  if (hl < 6) {
    const int d = hl / 3, a = hl % 3;
    DirConst& C = I->c[d];
    const int* own = I->vert + 12 * d;
    const int* oth = I->vert + 12 * (1 - d);
    double q = oth[a] * (1.0 / 1024.0) + 1.0;
    double bound = fabs(q) + 1.0;
#pragma unroll
    for (int cc = 0; cc < 3; cc++) {
      const double off = C.lo[cc] - own[cc] * (1.0 / 1024.0);
      q += C.M[a][cc] * off;
      bound += L->su.Mabs[half][d][a][cc] * (fabs(off) + (C.hi[cc] - C.lo[cc]));
    }
    C.qlo[a] = q;
    C.gthr[a] = 0.5 - bound * 0x1p-40;
    // FP32 fraction: rounding it and subtracting 1/2 moves the test value by
    // < 2^-24; the margin 2^-22 also covers rounding the threshold
    C.thr_f[a] = static_cast<float>(0.5 - bound * 0x1p-40 - 0x1p-22);
  }
  wave_sync();

  // ---- the slices of all four (item, direction) units at once when each
  // has at most 16: unit u = 2 s + d on lanes 16 u .. 16 u + 15, one slice z
  // per lane; unit u's non-empty slices go to slice[16 u ..] in ascending z
  // (with their first row index, an exclusive scan within the 16 lanes).
  // Otherwise every unit takes its slices in groups of 64 as it goes.
  bool pre = false;
  {
    const int u = lane >> 4, zl = lane & 15;
    const ItemLds* IU = &L->it[u >> 1];
    const DirConst& CU = IU->c[u & 1];
    const bool uact = ((u >> 1) ? act1 : act0) && CU.active != 0;
    const int unzb = CU.hi[2] - CU.lo[2] + 1;
    pre = __ballot(uact && unzb > 16) == 0ull;
    if (pre) {
      int y0 = 0, cnt = 0;
      if (uact && zl < unzb) slice_rows(IU->vert + 12 * (u & 1), CU.lo[2] + zl, CU.lo[1], CU.lo[1] + CU.NYb - 1, y0, cnt);
      const uint64_t ne = __ballot(cnt > 0);
      const uint64_t seg = 0xffffull << (16 * u);
      int x = cnt;   // inclusive scan within each row of 16 lanes
      x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);   // row_shr:1
      x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);   // row_shr:2
      x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);   // row_shr:4
      x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);   // row_shr:8
      if (cnt > 0) L->slice[16 * u + bits_below(ne & seg)] = make_int4(zl, y0, x - cnt, cnt);
      if (zl == 15) {
        L->pre_rows[u] = x;
        L->pre_ns[u] = __popcll(ne & seg);
      }
    }
  }
  wave_sync();

  // ---- rows and samples, one direction at a time (wave-uniform d).  Rows
  // are solved 64 at a time; non-empty rows enter a table of up to 64 rows.
  // Each row is cut into units of two consecutive samples (the last unit of
  // an odd row holds one); the units of the table form one stream, consumed
  // in batches of 64 units, one per lane.  The stream carries over from one
  // chunk of rows to the next, so only the direction's last batch runs
  // part-empty.
  L->mark[lane] = 0;
  int tag = 0;          // batch tags: unique within the wave's call
  for (int s = 0; s < 2; s++) {
  if (!(s ? act1 : act0)) continue;
  ItemLds* IT = &L->it[s];
  for (int d = 0; d < 2; d++) {
    const DirConst& Cd = IT->c[d];
    if (!uniform_i(Cd.active)) continue;
    const int nyb = uniform_i(Cd.NYb), Wd = uniform_i(Cd.W);
    const int lox = uniform_i(Cd.lo[0]), loy = uniform_i(Cd.lo[1]), loz = uniform_i(Cd.lo[2]);
    const bool inner = uniform_i(Cd.inner) != 0;
    const bool fast = uniform_i(Cd.fast) != 0;
    SampleConst U;
    U.m0 = uniform_d(Cd.M[0][0]);
    U.m1 = uniform_d(Cd.M[1][0]);
    U.m2 = uniform_d(Cd.M[2][0]);
    U.thr = uniform_f(fminf(fminf(Cd.thr_f[0], Cd.thr_f[1]), Cd.thr_f[2]));
    const __amdgpu_buffer_rsrc_t r_own = image_rsrc<ST>(P.img[d], P.pvox);
    const __amdgpu_buffer_rsrc_t r_oth = image_rsrc<ST>(P.img[1 - d], P.pvox);
    const __amdgpu_buffer_rsrc_t r_band = byte_rsrc(P.band[d], P.pvox);
    float h = 0.f, g = 0.f;
    int n = 0, n_defer = 0;
    // row table: a ring of 64 slots; the row of rank r (in stream order)
    // sits in slot (head + r) & 63.  Units are numbered from the start of
    // the direction; `cons` units are consumed, `tab_end` appended.
    int head = 0, n_tab = 0, cons = 0, tab_end = 0;

    // one sample of the current batch for directions whose mapped points may
    // leave the padded volume; a near-grid one joins the deferred queue
    auto sample = [&](bool valid, int vi, const double qr[3], int k, int jbase) {
      bool amb = false;
      float a = 0.f, b = 0.f;
      if (valid) {
        amb = sample_one<ST>(P, U, r_own, r_oth, r_band, d, vi + k, qr, k, h, g, a, b);
        n += 1;
      }
      const uint64_t amb_mask = __ballot(amb);
      if (amb_mask) {
        if (n_defer + __popcll(amb_mask) > kDeferCap) {
          wave_sync();
          flush_deferred<ST>(P, L, IT, n_defer, h, g);
          n_defer = 0;
          wave_sync();
        }
        if (amb) {
          const int slot = n_defer + bits_below(amb_mask);
          L->defer[slot] = make_int4((jbase + k) | (d << 30), __float_as_int(a), __float_as_int(b), 0);
        }
        n_defer += __popcll(amb_mask);
      }
    };

    // consume units [cons, limit) in batches of 64 (one unit per lane), then
    // drop the rows that end by `limit` (a prefix of the ring)
    auto run_batches_t = [&](auto inner_tag, int limit) {
      constexpr bool kInner = decltype(inner_tag)::value;
      const bool valid = ((lane - head) & (kWave - 1)) < n_tab;
      const int my_off = valid ? L->row[lane].y : 0x7fffffff;
      for (int sb = cons; sb < limit; sb += kWave) {
        // rank of each lane's row: rows starting at or before sb, plus rows
        // starting inside (sb, sb + lane] (marked with this batch's tag)
        tag += 1;
        const int first = __popcll(__ballot(my_off <= sb)) - 1;
        const int rel = my_off - sb;
        if (rel > 0 && rel < kWave) L->mark[rel] = tag;
        wave_sync();
        const uint64_t starts = __ballot(L->mark[lane] == tag);
        const int rank = first + bits_below(starts) + static_cast<int>((starts >> lane) & 1ull);
        const int slot = (head + rank) & (kWave - 1);
        const int u = sb + lane;
        const bool ok = u < limit;
        const int4 rw = L->row[slot];
        const double qr[3] = {L->rowq[slot][0], L->rowq[slot][1], L->rowq[slot][2]};
        const int k = 2 * (u - rw.y);
        const bool ok2 = ok && k + 1 < rw.w;
        if constexpr (kInner) {
          bool amb[2];
          float a[2], b[2];
          unsigned band[2];
          sample_pair_inner<ST>(P, U, r_own, r_oth, r_band, d, rw.x, qr, k, ok, ok2, h, amb, a, b, band);
          n += static_cast<int>(ok) + static_cast<int>(ok2);
          // near-grid and in-band samples join the queue, at most one wave's
          // worth (64, the queue's capacity) at a time, a flush first when
          // they would not fit
#pragma unroll
          for (int s2 = 0; s2 < 4; s2++) {
            const bool want = (s2 & 1) ? band[s2 >> 1] != 0u : amb[s2 >> 1];
            const uint64_t m = __ballot(want);
            if (m) {
              const int nq = __popcll(m);
              if (n_defer + nq > kDeferCap) {
                wave_sync();
                flush_deferred<ST>(P, L, IT, n_defer, h, g);
                n_defer = 0;
                wave_sync();
              }
              if (want) {
                const int j = rw.z + k + (s2 >> 1);
                L->defer[n_defer + bits_below(m)] =
                    (s2 & 1) ? make_int4(j | (d << 30), static_cast<int>(band[s2 >> 1]), 0, 1)
                             : make_int4(j | (d << 30), __float_as_int(a[s2 >> 1]), __float_as_int(b[s2 >> 1]), 0);
              }
              n_defer += nq;
            }
          }
        } else {
          sample(ok, rw.x, qr, k, rw.z);
          sample(ok2, rw.x, qr, k + 1, rw.z);
        }
        wave_sync();
      }
      // a row ends where the next one (in ring order) starts; the last at tab_end
      const int nxt = __shfl(my_off, (lane + 1) & (kWave - 1), 64);
      const int last = (head + n_tab - 1) & (kWave - 1);
      const int end = lane == last ? tab_end : nxt;
      const int done = __popcll(__ballot(valid && end <= limit));
      head = (head + done) & (kWave - 1);
      n_tab -= done;
      cons = limit;
    };
    // the mapped points stay inside the padded volume (no clamps) or not:
    // one specialised batch loop each
    auto run_batches = [&](int limit) {
      if (inner)
        run_batches_t(std::true_type{}, limit);
      else
        run_batches_t(std::false_type{}, limit);
    };

    // rows: slices in groups of 64 (one per lane), the rows of the non-empty
    // slices of a group enumerated 64 at a time
    const int nzb = uniform_i(Cd.hi[2]) - loz + 1;
    const int* own_v = IT->vert + 12 * d;
    const int unit = 2 * s + d;
    const int sbase = pre ? 16 * unit : 0;
    for (int zb = 0; zb < (pre ? 1 : nzb); zb += kWave) {
      int ns, Rg;
      if (pre) {
        ns = uniform_i(L->pre_ns[unit]);
        Rg = uniform_i(L->pre_rows[unit]);
      } else {
        int y0 = 0, cnt = 0;
        if (zb + lane < nzb) slice_rows(own_v, loz + zb + lane, loy, loy + nyb - 1, y0, cnt);
        const uint64_t ne = __ballot(cnt > 0);
        ns = __popcll(ne);
        const int sexcl = wave_excl_scan(cnt);
        Rg = __builtin_amdgcn_readlane(sexcl + cnt, 63);
        if (cnt > 0) L->slice[bits_below(ne)] = make_int4(zb + lane, y0, sexcl, cnt);
        wave_sync();
      }
      const int my_soff = lane < ns ? L->slice[sbase + lane].z : 0x7fffffff;
      for (int rb = 0; rb < Rg; rb += kWave) {
        const int rr = rb + lane;
        // slice of each lane's row: the mark trick over the slices' first rows
        tag += 1;
        const int sfirst = __popcll(__ballot(my_soff <= rb)) - 1;
        const int srel = my_soff - rb;
        if (srel > 0 && srel < kWave) L->mark[srel] = tag;
        wave_sync();
        const uint64_t sst = __ballot(L->mark[lane] == tag);
        const int si = sfirst + bits_below(sst) + static_cast<int>((sst >> lane) & 1ull);
        int js = 1, je = 0, yr = 0, zr = 0;
        if (rr < Rg) {
          const int4 sl = L->slice[sbase + si];
          zr = sl.x;
          yr = sl.y + (rr - sl.z);
          if (fast)
            row_span_fast(Cd, yr, zr, Wd, js, je);
          else
            row_span_wide(Cd, yr, zr, Wd, js, je);
        }
        const int len = max(0, je - js + 1);
        // the row's box-relative position, packed (it stays live while the
        // table is consumed)
        const int jp = js | (yr << 10) | (zr << 20);
        uint64_t want = __ballot(len > 0);
        while (want) {
          // append as many of this chunk's rows as the ring holds
          const int space = kWave - n_tab;
          const int ci = bits_below(want);
          const bool take = ((want >> lane) & 1ull) && ci < space;
          const uint64_t took = __ballot(take);
          const int tl = take ? (len + 1) >> 1 : 0;     // units of the row
          const int excl = wave_excl_scan(tl);
          const int added = __builtin_amdgcn_readlane(excl + tl, 63);
          if (take) {
            const int slot = (head + n_tab + ci) & (kWave - 1);
            const int jx = jp & 1023, jy = (jp >> 10) & 1023, jz = jp >> 20;
            const int vi_row = __umul24(loz + jz + 1, P.pxy) + __umul24(loy + jy + 1, P.px) + lox + jx + 1;
            L->row[slot] = make_int4(vi_row, tab_end + excl, jp, len);
#pragma unroll
            for (int t = 0; t < 3; t++)
              L->rowq[slot][t] = fma(Cd.M[t][0], static_cast<double>(jx),
                                     fma(Cd.M[t][1], static_cast<double>(jy),
                                         fma(Cd.M[t][2], static_cast<double>(jz), Cd.qlo[t])));
          }
          n_tab += __popcll(took);
          tab_end += added;
          want &= ~took;
          wave_sync();
          if (tab_end - cons >= kWave) run_batches(cons + ((tab_end - cons) & ~(kWave - 1)));
        }
      }
      wave_sync();   // the slice table is rewritten by the next group
    }
    if (tab_end > cons) run_batches(tab_end);
    if (n_defer > 0) {
      wave_sync();
      flush_deferred<ST>(P, L, IT, n_defer, h, g);
    }
    h = wave_sum(h);
    g = wave_sum(g);
    n = wave_sum_i(n);
    if (lane == 0) {
      IT->c[d].h = h;
      IT->c[d].g = g;
      IT->c[d].samples = static_cast<uint32_t>(n);
    }
  }
  }
  wave_sync();
  if (ok0 && lane < 2) {
    const DirConst& C = L->it[0].c[lane];
    out0[lane] = Record{C.h, C.g, C.samples, C.mag, C.vol, C.bits};
  }
  if (ok1 && lane >= 32 && lane < 34) {
    const DirConst& C = L->it[1].c[lane - 32];
    out1[lane - 32] = Record{C.h, C.g, C.samples, C.mag, C.vol, C.bits};
  }
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

// Full evaluation: one wave per two (candidate, tet) items, item = tet * pop
// + candidate, so the 4 waves of a block take 8 consecutive candidates of one
// tet (fewer at a tet boundary).
__device__ __forceinline__ void split_item(const FullItems& F, int item, int& tet, int& cand) {
  // item = tet * pop + cand, split with the reciprocal (wave-uniform values)
  tet = static_cast<int>(static_cast<double>(item) * F.inv_pop);
  cand = item - tet * F.pop;
  if (cand < 0) {
    tet -= 1;
    cand += F.pop;
  } else if (cand >= F.pop) {
    tet += 1;
    cand -= F.pop;
  }
  tet = uniform_i(tet);
  cand = uniform_i(cand);
}

template <int ST>
__global__ __launch_bounds__(256, 5) void k_eval_full(ProblemView P, FullItems F, Record* rec,
                                                    int n_items) {
  __shared__ WaveLds lds[4];
  const int wave = uniform_i(static_cast<int>(threadIdx.x >> 6));
  const int item0 = 2 * (xcd_block(blockIdx.x, gridDim.x) * 4 + wave);
  if (item0 >= n_items) return;
  const bool has1 = item0 + 1 < n_items;
  int tet0, cand0, tet1 = 0, cand1 = 0;
  split_item(F, item0, tet0, cand0);
  if (has1) split_item(F, item0 + 1, tet1, cand1);
  const int lane = lane_id();
  const int half = lane >> 5, hl = lane & 31;
  float coord = 0.f;
  if (hl < 24 && (half == 0 || has1)) {
    const int tet = half ? tet1 : tet0, cand = half ? cand1 : cand0;
    const int4 tv = P.tets[tet];
    const int i = (hl % 12) / 3, k = hl % 3;
    const int v = i == 0 ? tv.x : (i == 1 ? tv.y : (i == 2 ? tv.z : tv.w));
    const int mesh = hl < 12 ? 0 : 1;
    coord = F.pts[((static_cast<size_t>(cand) * 2 + mesh) * 3 + k) * P.n_points + v];
  }
  eval_tet<ST>(P, tet0, tet1, has1, coord, &lds[wave], &rec[(static_cast<size_t>(cand0) * P.n_tets + tet0) * 2],
               &rec[(static_cast<size_t>(cand1) * P.n_tets + tet1) * 2]);
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
// of the sets with d < r.  Both are written padded: a border element holds
// the value of the nearest grid voxel (edge clamping).
__global__ void k_distance_maps(int nx, int ny, int nz, int n_sets, const int* set_off,
                                const int* pts_fix, float radius, float* dmap, uint8_t* band) {
  const int px = padded_row(nx), py = ny + 2;
  const size_t PV = static_cast<size_t>(px) * py * (nz + 2);
  for (size_t v = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; v < PV;
       v += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int x = min(max(static_cast<int>(v % px) - 1, 0), nx - 1);
    const int y = min(max(static_cast<int>((v / px) % py) - 1, 0), ny - 1);
    const int z = min(max(static_cast<int>(v / (static_cast<size_t>(px) * py)) - 1, 0), nz - 1);
    const int64_t qx = (int64_t)x * 1024, qy = (int64_t)y * 1024, qz = (int64_t)z * 1024;
    unsigned bits = 0;
    for (int s = 0; s < n_sets; s++) {
      int64_t best = INT64_MAX;
      for (int j = set_off[s]; j < set_off[s + 1]; j++) {
        const int64_t dx = qx - pts_fix[3 * j], dy = qy - pts_fix[3 * j + 1], dz = qz - pts_fix[3 * j + 2];
        const int64_t d2 = dx * dx + dy * dy + dz * dz;
        best = d2 < best ? d2 : best;
      }
      const float d = static_cast<float>(sqrt(static_cast<double>(best)) / 1024.0);
      dmap[static_cast<size_t>(s) * PV + v] = d;
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
  const size_t PV = static_cast<size_t>(padded_row(nx)) * (ny + 2) * (nz + 2);
  const int blocks = static_cast<int>(std::min<size_t>((PV + 255) / 256, 65536));
  hipLaunchKernelGGL(k_distance_maps, dim3(blocks), dim3(256), 0, s, nx, ny, nz, n_sets, set_off,
                     pts_fix, radius, dmap, band);
  return hipGetLastError();
}

hipError_t launch_eval_full(const ProblemView& P, int storage, const float* pts, int pop,
                            Record* rec, hipStream_t s) {
  const size_t n_items = static_cast<size_t>(pop) * P.n_tets;
  if (n_items == 0) return hipSuccess;
  const int blocks = static_cast<int>((n_items + 7) / 8);
  FullItems F{pts, pop, 1.0 / pop};
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

// ------------------------------------------------------- partial evaluation
namespace morea {

// Prefix sums of the evaluation list: first new-coordinate row of each
// evaluation and first record (dependent tet).  An evaluation with an
// out-of-range group owns no new-coordinate rows; one with an out-of-range
// parent or group gets no work items and is reported invalid by the finalize
// kernel.  Then the evaluations are bucketed by group (rank within the
// group; the ranks' order does not affect any result) and each group's first
// processing position is the prefix of evaluations x dependent tets over the
// groups.  Four launches: per-block scans of 256 evaluations (block totals
// into the head of the item-info array, which the item kernel fills only
// afterwards), one block scanning the block totals (and clearing the group
// counters and the work queue), the block offsets added back with the ranks
// taken, and one block for the group bases.
constexpr int kPrepBlock = 256;

__device__ __forceinline__ void eval_sizes(const PartialItems& I, int e, int n_parents, int n_groups, int& rows,
                                           int& items) {
  rows = items = 0;
  const int g = I.eval_group[e], par = I.eval_parent[e];
  if (g >= 0 && g < n_groups) {
    rows = I.grp_off[g + 1] - I.grp_off[g];
    if (par >= 0 && par < n_parents) items = I.dep_off[g + 1] - I.dep_off[g];
  }
}

__global__ __launch_bounds__(kPrepBlock) void k_prep_local(PartialItems I, int n_parents, int n_groups) {
  __shared__ int s_rows[kPrepBlock], s_items[kPrepBlock];
  const int tid = threadIdx.x, e = blockIdx.x * kPrepBlock + tid;
  int rows = 0, items = 0;
  if (e < I.n_evals) eval_sizes(I, e, n_parents, n_groups, rows, items);
  s_rows[tid] = rows;
  s_items[tid] = items;
  __syncthreads();
  for (int d = 1; d < kPrepBlock; d <<= 1) {
    const int r = tid >= d ? s_rows[tid - d] : 0, it = tid >= d ? s_items[tid - d] : 0;
    __syncthreads();
    s_rows[tid] += r;
    s_items[tid] += it;
    __syncthreads();
  }
  if (e < I.n_evals) {
    const_cast<int*>(I.row_off)[e] = s_rows[tid] - rows;
    const_cast<int*>(I.item_off)[e] = s_items[tid] - items;
  }
  if (tid == kPrepBlock - 1) {
    int* bsum = reinterpret_cast<int*>(I.item_info);
    bsum[2 * blockIdx.x] = s_rows[tid];
    bsum[2 * blockIdx.x + 1] = s_items[tid];
  }
}

__global__ __launch_bounds__(1024) void k_prep_blocks(PartialItems I, int n_blocks, int n_groups, int* queue) {
  __shared__ int s_rows[1024], s_items[1024];
  const int tid = threadIdx.x;
  int* bsum = reinterpret_cast<int*>(I.item_info);
  int carry_r = 0, carry_i = 0;
  for (int b0 = 0; b0 < n_blocks; b0 += 1024) {
    const int b = b0 + tid;
    const int r = b < n_blocks ? bsum[2 * b] : 0, it = b < n_blocks ? bsum[2 * b + 1] : 0;
    s_rows[tid] = r;
    s_items[tid] = it;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
      const int x = tid >= d ? s_rows[tid - d] : 0, y = tid >= d ? s_items[tid - d] : 0;
      __syncthreads();
      s_rows[tid] += x;
      s_items[tid] += y;
      __syncthreads();
    }
    if (b < n_blocks) {
      bsum[2 * b] = carry_r + s_rows[tid] - r;
      bsum[2 * b + 1] = carry_i + s_items[tid] - it;
    }
    carry_r += s_rows[1023];
    carry_i += s_items[1023];
    __syncthreads();
  }
  if (tid == 0) {
    const_cast<int*>(I.item_off)[I.n_evals] = carry_i;
    *queue = 0;
  }
  for (int g = tid; g < n_groups; g += 1024) I.grp_count[g] = 0;
}

__global__ __launch_bounds__(kPrepBlock) void k_prep_offsets(PartialItems I, int n_parents, int n_groups) {
  const int e = blockIdx.x * kPrepBlock + threadIdx.x;
  if (e >= I.n_evals) return;
  const int* bsum = reinterpret_cast<const int*>(I.item_info);
  const_cast<int*>(I.row_off)[e] += bsum[2 * blockIdx.x];
  const_cast<int*>(I.item_off)[e] += bsum[2 * blockIdx.x + 1];
  const int g = I.eval_group[e], par = I.eval_parent[e];
  if (g >= 0 && g < n_groups && par >= 0 && par < n_parents) I.eval_rank[e] = atomicAdd(&I.grp_count[g], 1);
}

// Group bases: exclusive prefix of count x dependent tets, 1024 groups per pass.
__global__ __launch_bounds__(1024) void k_prep_groups(PartialItems I, int n_groups) {
  __shared__ int s_items[1024];
  const int tid = threadIdx.x;
  int carry = 0;
  for (int g0 = 0; g0 < n_groups; g0 += 1024) {
    const int g = g0 + tid;
    int v = 0;
    if (g < n_groups) v = I.grp_count[g] * (I.dep_off[g + 1] - I.dep_off[g]);
    s_items[tid] = v;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
      const int t = tid >= d ? s_items[tid - d] : 0;
      __syncthreads();
      s_items[tid] += t;
      __syncthreads();
    }
    if (g < n_groups) I.grp_base[g] = carry + s_items[tid] - v;
    carry += s_items[1023];
    __syncthreads();
  }
}

// Per-item records of the partial launch, one wave per evaluation: for
// dependent tet j of evaluation e (rank r in its group g of c evaluations)
// the processing position is grp_base[g] + j c + r; the record there names
// the dependent-tet slot, the tet, the parent and the evaluation's first
// new-coordinate row, and its destination item_off[e] + j.  Evaluations with
// an out-of-range parent or group own no items.
__global__ __launch_bounds__(256) void k_partial_items(PartialItems I, int n_parents, int n_groups) {
  const int e = blockIdx.x * 4 + static_cast<int>(threadIdx.x >> 6);
  const int lane = lane_id();
  if (e >= I.n_evals) return;
  const int g = I.eval_group[e], par = I.eval_parent[e];
  if (g < 0 || g >= n_groups || par < 0 || par >= n_parents) return;
  const int first = I.dep_off[g], n = I.dep_off[g + 1] - first;
  const int c = I.grp_count[g], pos0 = I.grp_base[g] + I.eval_rank[e];
  const int dest0 = I.item_off[e], row = I.row_off[e];
  for (int j = lane; j < n; j += kWave) {
    const int pos = pos0 + j * c;
    I.item_info[pos] = make_int4(first + j, I.dep_tet[first + j], par, row);
    I.item_dest[pos] = dest0 + j;
  }
}

// Persistent evaluation of all (evaluation, dependent tet) items, both
// directions per item: each wave takes `chunk` consecutive items from a
// device work queue until the list is exhausted.  Every wave leaves the loop
// once the queue passes the end of the list.
// Child coordinate of lane `lane` for the item pair (idx, idx + 1): lanes
// 0..23 of each half hold the 24 coordinates of their item's tet (mesh 0
// then 1, vertex-major), from the group's new coordinates or the parent.
__device__ __forceinline__ float partial_coord(const ProblemView& P, const PartialItems& I, int4 it0, int4 it1,
                                               bool has1, int lane) {
  const int half = lane >> 5, hl = lane & 31;
  const int4 it = half ? it1 : it0;
  float coord = 0.f;
  if (hl < 24 && (half == 0 || has1)) {
    const int slot = it.x, tet = it.y, par = it.z, row = it.w;
    const int i = (hl % 12) / 3, k = hl % 3;
    const int mesh = hl < 12 ? 0 : 1;
    const int loc = I.dep_local[4 * slot + i];
    if (loc >= 0) {
      coord = I.new_coords[((static_cast<size_t>(row) + loc) * 2 + mesh) * 3 + k];
    } else {
      const int4 tv = P.tets[tet];
      const int v = i == 0 ? tv.x : (i == 1 ? tv.y : (i == 2 ? tv.z : tv.w));
      coord = I.parent_pts[((static_cast<size_t>(par) * 2 + mesh) * 3 + k) * P.n_points + v];
    }
  }
  return coord;
}

// Persistent form: every wave takes `chunk` items at a time from the queue
// (items in processing order) until none is left.
template <int ST>
__global__ __launch_bounds__(256, 4) void k_eval_partial(ProblemView P, PartialItems I, Record* out,
                                                       int* queue, int chunk) {
  __shared__ WaveLds lds[4];
  const int wave = threadIdx.x >> 6;
  const int lane = lane_id();
  const int total = I.item_off[I.n_evals];
  while (true) {
    int base = 0;
    if (lane == 0) base = atomicAdd(queue, chunk);
    base = __shfl(base, 0, 64);
    if (base >= total) break;
    const int end = min(total, base + chunk);
    for (int idx = base; idx < end; idx += 2) {
      const bool has1 = idx + 1 < end;
      const int4 it0 = I.item_info[idx];
      const int4 it1 = has1 ? I.item_info[idx + 1] : it0;
      const int tet0 = uniform_i(it0.y), tet1 = uniform_i(it1.y);
      const float coord = partial_coord(P, I, it0, it1, has1, lane);
      const int dest0 = uniform_i(I.item_dest[idx]);
      const int dest1 = has1 ? uniform_i(I.item_dest[idx + 1]) : dest0;
      eval_tet<ST>(P, tet0, tet1, has1, coord, &lds[wave], &out[static_cast<size_t>(dest0) * 2],
                   &out[static_cast<size_t>(dest1) * 2]);
    }
  }
}

// Grid form: wave w evaluates items 2 w and 2 w + 1 (in processing order);
// the grid covers a bound of the item count known on the host, and the
// waves beyond the actual count return at once.  Without the persistent
// loop the kernel fits five waves per SIMD.
template <int ST>
__global__ __launch_bounds__(256, 5) void k_eval_partial_grid(ProblemView P, PartialItems I, Record* out) {
  __shared__ WaveLds lds[4];
  const int wave = uniform_i(static_cast<int>(threadIdx.x >> 6));
  const int lane = lane_id();
  const int total = I.item_off[I.n_evals];
  const long long idx_l = 2 * (static_cast<long long>(blockIdx.x) * 4 + wave);
  if (idx_l >= total) return;
  const int idx = static_cast<int>(idx_l);
  const bool has1 = idx + 1 < total;
  const int4 it0 = I.item_info[idx];
  const int4 it1 = has1 ? I.item_info[idx + 1] : it0;
  const int tet0 = uniform_i(it0.y), tet1 = uniform_i(it1.y);
  const float coord = partial_coord(P, I, it0, it1, has1, lane);
  const int dest0 = uniform_i(I.item_dest[idx]);
  const int dest1 = has1 ? uniform_i(I.item_dest[idx + 1]) : dest0;
  eval_tet<ST>(P, tet0, tet1, has1, coord, &lds[wave], &out[static_cast<size_t>(dest0) * 2],
               &out[static_cast<size_t>(dest1) * 2]);
}

template __global__ void k_eval_partial<kF32>(ProblemView, PartialItems, Record*, int*, int);
template __global__ void k_eval_partial<kBF16>(ProblemView, PartialItems, Record*, int*, int);
template __global__ void k_eval_partial<kF16>(ProblemView, PartialItems, Record*, int*, int);
template __global__ void k_eval_partial_grid<kF32>(ProblemView, PartialItems, Record*);
template __global__ void k_eval_partial_grid<kBF16>(ProblemView, PartialItems, Record*);
template __global__ void k_eval_partial_grid<kF16>(ProblemView, PartialItems, Record*);

__device__ __forceinline__ void df_wave_sum(float& hi, float& lo) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const float h2 = __shfl_xor(hi, d, 64), l2 = __shfl_xor(lo, d, 64);
    df_add(hi, lo, h2);
    lo += l2;
  }
}

// Child totals = parent totals - parent records of the dependent tets + new
// records, in compensated arithmetic; counts, violations and invalid
// coordinates are exact integer deltas.  One wave per evaluation.
__global__ __launch_bounds__(256) void k_finalize_partial(ProblemView P, PartialItems I,
                                                           const Record* parent_rec,
                                                           const Totals* parent_tot, int n_parents,
                                                           int n_groups, const Record* new_rec,
                                                           float* obj, uint8_t* flags,
                                                           float* severity, uint32_t* counts) {
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (e >= I.n_evals) return;
  const int lane = lane_id();
  const int g = I.eval_group[e], par = I.eval_parent[e];
  if (g < 0 || g >= n_groups || par < 0 || par >= n_parents) {
    if (lane == 0) {
      const float nan = __builtin_nanf("");
      obj[3 * e] = obj[3 * e + 1] = obj[3 * e + 2] = nan;
      flags[e] = 4;
      severity[e] = nan;
      counts[2 * e] = counts[2 * e + 1] = 0;
    }
    return;
  }
  const Totals T = parent_tot[par];
  float hh = lane == 0 ? T.h_hi : 0.f, hl = lane == 0 ? T.h_lo : 0.f;
  float gh = lane == 0 ? T.g_hi : 0.f, gl = lane == 0 ? T.g_lo : 0.f;
  float mh = lane == 0 ? T.m_hi : 0.f, ml = lane == 0 ? T.m_lo : 0.f;
  float vh = lane == 0 ? T.v_hi : 0.f, vl = lane == 0 ? T.v_lo : 0.f;
  int dns = 0, dnt = 0, dvs = 0, dvt = 0, dbad = 0;
  const int n_dep = I.item_off[e + 1] - I.item_off[e];
  const Record* pr = parent_rec + static_cast<size_t>(par) * P.n_tets * 2;
  const Record* nr = new_rec + static_cast<size_t>(I.item_off[e]) * 2;
  for (int j = lane; j < n_dep; j += 64) {
    const int tet = I.dep_tet[I.dep_off[g] + j];
    const Record o0 = pr[2 * tet], o1 = pr[2 * tet + 1];
    const Record n0 = nr[2 * j], n1 = nr[2 * j + 1];
    df_add(hh, hl, -o0.h); df_add(hh, hl, -o1.h); df_add(hh, hl, n0.h); df_add(hh, hl, n1.h);
    df_add(gh, gl, -o0.g); df_add(gh, gl, -o1.g); df_add(gh, gl, n0.g); df_add(gh, gl, n1.g);
    df_add(mh, ml, -o0.mag); df_add(mh, ml, n0.mag);
    df_add(vh, vl, -o0.vol); df_add(vh, vl, -o1.vol); df_add(vh, vl, n0.vol); df_add(vh, vl, n1.vol);
    dns += static_cast<int>(n0.n) - static_cast<int>(o0.n);
    dnt += static_cast<int>(n1.n) - static_cast<int>(o1.n);
    dvs += static_cast<int>(n0.bits & 1u) - static_cast<int>(o0.bits & 1u);
    dvt += static_cast<int>(n1.bits & 1u) - static_cast<int>(o1.bits & 1u);
  }
  // invalid coordinates: the group's old coordinates leave, the new ones enter
  const int g0 = I.grp_off[g], size = I.grp_off[g + 1] - g0;
  const float* pp = I.parent_pts + static_cast<size_t>(par) * 6 * P.n_points;
  for (int k = lane; k < size * 6; k += 64) {
    const float nv = I.new_coords[static_cast<size_t>(I.row_off[e]) * 6 + k];
    const int pt = I.grp_pts[g0 + k / 6], ma = k % 6;   // ma = mesh * 3 + axis
    const float ov = pp[static_cast<size_t>(ma) * P.n_points + pt];
    dbad += static_cast<int>(!(fabsf(nv) < kCoordLimit)) - static_cast<int>(!(fabsf(ov) < kCoordLimit));
  }
  df_wave_sum(hh, hl);
  df_wave_sum(gh, gl);
  df_wave_sum(mh, ml);
  df_wave_sum(vh, vl);
  dns = wave_sum_i(dns);
  dnt = wave_sum_i(dnt);
  dvs = wave_sum_i(dvs);
  dvt = wave_sum_i(dvt);
  dbad = wave_sum_i(dbad);
  if (lane == 0) {
    const uint32_t Ns = T.n[0] + dns, Nt = T.n[1] + dnt;
    const int bad = static_cast<int>(T.bad) + dbad;
    if (bad > 0) {
      const float nan = __builtin_nanf("");
      obj[3 * e] = obj[3 * e + 1] = obj[3 * e + 2] = nan;
      flags[e] = 4;
      severity[e] = nan;
      counts[2 * e] = counts[2 * e + 1] = 0;
    } else {
      const float N = static_cast<float>(Ns) + static_cast<float>(Nt);
      obj[3 * e + 0] = (hh + hl) / N;
      obj[3 * e + 1] = (mh + ml) / (10.0f * static_cast<float>(P.n_tets));
      obj[3 * e + 2] = (gh + gl) / N;
      flags[e] = static_cast<uint8_t>((T.viol[0] + dvs ? 1 : 0) | (T.viol[1] + dvt ? 2 : 0));
      severity[e] = vh + vl;
      counts[2 * e] = Ns;
      counts[2 * e + 1] = Nt;
    }
  }
}

}  // namespace morea

namespace morea {

hipError_t launch_partial(const ProblemView& P, int storage, const PartialItems& I, int n_parents,
                          int n_groups, const Record* parent_rec, const Totals* parent_tot,
                          Record* new_rec, int* queue, int blocks, int chunk, float* obj,
                          uint8_t* flags, float* severity, uint32_t* counts, hipStream_t s) {
  if (I.n_evals == 0) return hipSuccess;
  const int prep_blocks = (I.n_evals + kPrepBlock - 1) / kPrepBlock;
  hipLaunchKernelGGL(k_prep_local, dim3(prep_blocks), dim3(kPrepBlock), 0, s, I, n_parents, n_groups);
  hipLaunchKernelGGL(k_prep_blocks, dim3(1), dim3(1024), 0, s, I, prep_blocks, n_groups, queue);
  hipLaunchKernelGGL(k_prep_offsets, dim3(prep_blocks), dim3(kPrepBlock), 0, s, I, n_parents, n_groups);
  hipLaunchKernelGGL(k_prep_groups, dim3(1), dim3(1024), 0, s, I, n_groups);
  hipLaunchKernelGGL(k_partial_items, dim3((I.n_evals + 3) / 4), dim3(256), 0, s, I, n_parents, n_groups);
  if (chunk == 0) {   // grid form: `blocks` covers the bound of the item count
    switch (storage) {
      case kF32: hipLaunchKernelGGL(k_eval_partial_grid<kF32>, dim3(blocks), dim3(256), 0, s, P, I, new_rec); break;
      case kBF16: hipLaunchKernelGGL(k_eval_partial_grid<kBF16>, dim3(blocks), dim3(256), 0, s, P, I, new_rec); break;
      default: hipLaunchKernelGGL(k_eval_partial_grid<kF16>, dim3(blocks), dim3(256), 0, s, P, I, new_rec); break;
    }
  } else {
    switch (storage) {
      case kF32:
        hipLaunchKernelGGL(k_eval_partial<kF32>, dim3(blocks), dim3(256), 0, s, P, I, new_rec, queue, chunk);
        break;
      case kBF16:
        hipLaunchKernelGGL(k_eval_partial<kBF16>, dim3(blocks), dim3(256), 0, s, P, I, new_rec, queue, chunk);
        break;
      default:
        hipLaunchKernelGGL(k_eval_partial<kF16>, dim3(blocks), dim3(256), 0, s, P, I, new_rec, queue, chunk);
        break;
    }
  }
  hipLaunchKernelGGL(k_finalize_partial, dim3((I.n_evals + 3) / 4), dim3(256), 0, s, P, I,
                     parent_rec, parent_tot, n_parents, n_groups, new_rec, obj, flags, severity,
                     counts);
  return hipGetLastError();
}

}  // namespace morea

namespace morea {
int partial_blocks_per_cu(int storage) {
  int n = 0;
  hipError_t e;
  if (storage == kF32)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(&k_eval_partial<kF32>), 256, 0);
  else if (storage == kBF16)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(&k_eval_partial<kBF16>), 256, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(&k_eval_partial<kF16>), 256, 0);
  return e == hipSuccess ? n : 1;
}
}  // namespace morea
