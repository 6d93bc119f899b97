/*
 * MOREA objective evaluation -- plain CPU oracle (test infrastructure only).
 *
 * This file is the slow, obviously-correct reference against which the GPU
 * evaluator is checked.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it; the product path never does.  It
 * shares no code with the HIP library.
 *
 * Everything is computed from the plain definitions of the paper, for each
 * candidate, each direction, each tetrahedron and each voxel centre of the
 * tetrahedron's bounding box, in FP64 with exact __int128 geometric
 * predicates:
 *
 *   f_magnitude  Sec. 4.1.1 (equation for f_magnitude): per tet, elasticity
 *                c_delta times the sum over 10 edges (6 edges + 4 spokes) of
 *                (|e_s| - |e_t|)^2, normalised by 10 |Delta|.
 *   f_intensity  Sec. 4.1.2 (equations for f_intensity and h): sum of h over
 *                the sample points of both images, normalised by |P_s|+|P_t|.
 *   f_guidance   Sec. 4.1.3 (equations for f_guidance and g) with the
 *                distance-map reading of App. A.3.
 *   folds        Sec. 4.1.4 and App. A.4: sign of each tet's signed volume
 *                against the reference sign of the initial mesh; severity is
 *                the absolute violating volume.
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *   - sample points are the voxel centres inside each tet (rasterization, the
 *     prototype's association of App. A.2) instead of random samples;
 *   - coordinates are snapped to the fixed-point grid 2^-10 voxel
 *     (x_hat = rint_half_even(x * 1024)) so every predicate is exact;
 *   - a voxel centre p lies in tet delta iff p + (e, e^2, e^3) is strictly
 *     inside for infinitesimal e > 0 (a watertight tie rule);
 *   - "interpolated intensity > 0" is decided on the exact support of the
 *     trilinear stencil (corners with positive exact weight);
 *   - intensities outside the image are 0; distance maps are edge-clamped;
 *   - the guidance radius r is compared with a strict '<' against the stored
 *     FP32 distance map, and set weights are |C|/|G| as printed;
 *   - spokes join the centroid to each vertex; a zero volume is a fold;
 *   - magnitude is in voxel units (isotropic voxels).
 *
 * oracle_eval_sobol evaluates the same objectives from the paper's own
 * estimator, random barycentric samples from a seeded Sobol sequence
 * (App. A.2); its readings are listed where it is defined below.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

#define FRAC_BITS 10
#define FIX_ONE ((int64_t)1 << FRAC_BITS)
#define COORD_LIMIT 512.0

typedef struct {
  int nx, ny, nz;
  const float *img_s, *img_t;      /* [nz][ny][nx], stored values */
  int n_points, n_tets;
  const int32_t *tets;             /* [n_tets][4] */
  const float *ref_points;         /* [n_points][3] */
  const float *elasticity;         /* [n_tets] */
  int n_sets;
  const int32_t *set_off_s, *set_off_t;  /* [n_sets+1] */
  const float *dmap_s, *dmap_t;    /* [n_sets][nz][ny][nx] stored distance maps */
  float radius;
} oracle_problem;

/* ------------------------------------------------------------------ helpers */

static int64_t snap(float x) { return (int64_t)rint((double)x * (double)FIX_ONE); }

static i128 det3(const i128 a[3], const i128 b[3], const i128 c[3]) {
  return a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
         a[2] * (b[0] * c[1] - b[1] * c[0]);
}

/* 6 x signed volume of (v0, v1, v2, v3) in fixed-point units (2^-30 voxel^3) */
static i128 orient(const int64_t v[4][3]) {
  i128 a[3], b[3], c[3];
  for (int k = 0; k < 3; k++) {
    a[k] = (i128)v[1][k] - v[0][k];
    b[k] = (i128)v[2][k] - v[0][k];
    c[k] = (i128)v[3][k] - v[0][k];
  }
  return det3(a, b, c);
}

/* orient() with vertex i replaced by point p: D * lambda_i(p) */
static i128 orient_replaced(const int64_t v[4][3], int i, const int64_t p[3]) {
  int64_t w[4][3];
  memcpy(w, v, sizeof(w));
  for (int k = 0; k < 3; k++) w[i][k] = p[k];
  return orient(w);
}

static i128 floor_div(i128 a, i128 b) { /* b > 0 */
  i128 q = a / b;
  if ((a % b) != 0 && a < 0) q -= 1;
  return q;
}

static int64_t floor_div64(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b) != 0 && a < 0) q -= 1;
  return q;
}

static int64_t ceil_div64(int64_t a, int64_t b) { return -floor_div64(-a, b); }

static int sgn128(i128 x) { return (x > 0) - (x < 0); }

/* Is p (fixed-point) inside the tet under the tie rule?  On return lam[i]
 * holds |D| * lambda_i (all >= 0 when inside). */
static int inside_tie(const int64_t v[4][3], i128 D, const int64_t p[3], i128 lam[4]) {
  int s = sgn128(D);
  for (int i = 0; i < 4; i++) {
    i128 val = s * orient_replaced(v, i, p);
    lam[i] = val;
    if (val > 0) continue;
    if (val < 0) return 0;
    /* on the face plane: decide by the sign of the value at p + (e, e^2, e^3),
     * i.e. lexicographically by the gradient (dx, dy, dz) of the affine
     * function; the gradient is the difference for a unit step of p. */
    int64_t q[3];
    i128 grad[3];
    for (int k = 0; k < 3; k++) {
      memcpy(q, p, sizeof(q));
      q[k] += 1;
      grad[k] = s * orient_replaced(v, i, q) - val;
    }
    int pos = grad[0] > 0 || (grad[0] == 0 && (grad[1] > 0 || (grad[1] == 0 && grad[2] > 0)));
    if (!pos) return 0;
  }
  return 1;
}

static double fetch_zero(const float *img, int nx, int ny, int nz, int64_t x, int64_t y, int64_t z) {
  if (x < 0 || y < 0 || z < 0 || x >= nx || y >= ny || z >= nz) return 0.0;
  return (double)img[((size_t)z * ny + y) * nx + x];
}

static double fetch_clamp(const float *img, int nx, int ny, int nz, int64_t x, int64_t y, int64_t z) {
  x = x < 0 ? 0 : (x >= nx ? nx - 1 : x);
  y = y < 0 ? 0 : (y >= ny ? ny - 1 : y);
  z = z < 0 ? 0 : (z >= nz ? nz - 1 : z);
  return (double)img[((size_t)z * ny + y) * nx + x];
}

/* Trilinear interpolation with corner k + d (d in {0,1}) weighted by
 * (d ? f : 1 - f) per axis. */
static double trilinear(const float *img, int nx, int ny, int nz, const int64_t k[3],
                        const double f[3], int clamp) {
  double acc = 0.0;
  for (int dz = 0; dz < 2; dz++)
    for (int dy = 0; dy < 2; dy++)
      for (int dx = 0; dx < 2; dx++) {
        double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
        double val = clamp ? fetch_clamp(img, nx, ny, nz, k[0] + dx, k[1] + dy, k[2] + dz)
                           : fetch_zero(img, nx, ny, nz, k[0] + dx, k[1] + dy, k[2] + dz);
        acc += w * val;
      }
  return acc;
}

/* Mapped position of an inside point: q = sum_i lambda_i * other_i with
 * lambda_i = lam[i] / |D|.  Per axis: k = floor(q) exactly, f = q - k,
 * exact = (q is an integer).  */
static void map_point(const i128 lam[4], i128 absD, const int64_t oth[4][3], int64_t k[3],
                      double f[3], int exact[3], double q[3]) {
  i128 den = absD * FIX_ONE;
  for (int a = 0; a < 3; a++) {
    i128 num = 0;
    for (int i = 0; i < 4; i++) num += lam[i] * (i128)oth[i][a];
    i128 kk = floor_div(num, den);
    i128 r = num - kk * den;
    k[a] = (int64_t)kk;
    exact[a] = (r == 0);
    f[a] = (double)r / (double)den;
    q[a] = (double)kk + f[a];
  }
}

/* ------------------------------------------------------------ distance maps */

/* d(p, C) at every voxel centre: Euclidean distance to the nearest point of
 * the set (points snapped like mesh coordinates), rounded to FP32. */
void oracle_distance_map(int nx, int ny, int nz, int n, const float *pts, float *out) {
  int64_t *c = (int64_t *)malloc(sizeof(int64_t) * 3 * (n > 0 ? n : 1));
  for (int i = 0; i < 3 * n; i++) c[i] = snap(pts[i]);
#pragma omp parallel for schedule(static)
  for (int z = 0; z < nz; z++)
    for (int y = 0; y < ny; y++)
      for (int x = 0; x < nx; x++) {
        int64_t best = INT64_MAX;
        for (int j = 0; j < n; j++) {
          int64_t dx = (int64_t)x * FIX_ONE - c[3 * j], dy = (int64_t)y * FIX_ONE - c[3 * j + 1],
                  dz = (int64_t)z * FIX_ONE - c[3 * j + 2];
          int64_t d2 = dx * dx + dy * dy + dz * dz;
          if (d2 < best) best = d2;
        }
        out[((size_t)z * ny + y) * nx + x] = (float)(sqrt((double)best) / (double)FIX_ONE);
      }
  free(c);
}

/* --------------------------------------------------------------- evaluation */

typedef struct {
  double h;      /* sum of h over the tet's samples, this direction */
  double g;      /* set-weighted guidance sum, this direction */
  int64_t n;     /* number of samples */
  int viol;      /* signed-volume sign differs from the reference (or is 0) */
  double vol;    /* |signed volume| in voxel^3 */
} dir_record;

static void eval_direction(const oracle_problem *P, const int64_t own[4][3], const int64_t oth[4][3],
                           int ref_sign, int dir, const double *set_w, dir_record *rec) {
  const float *img_own = dir == 0 ? P->img_s : P->img_t;
  const float *img_oth = dir == 0 ? P->img_t : P->img_s;
  const float *map_own = dir == 0 ? P->dmap_s : P->dmap_t;
  const float *map_oth = dir == 0 ? P->dmap_t : P->dmap_s;
  const size_t V = (size_t)P->nx * P->ny * P->nz;
  const int dims[3] = {P->nx, P->ny, P->nz};
  memset(rec, 0, sizeof(*rec));
  i128 D = orient(own);
  rec->viol = (sgn128(D) == 0) || (sgn128(D) != ref_sign);
  i128 absD = D < 0 ? -D : D;
  rec->vol = (double)absD / 6.0 / (double)((int64_t)1 << (3 * FRAC_BITS));
  if (D == 0) return;

  int64_t lo[3], hi[3];
  for (int a = 0; a < 3; a++) {
    int64_t mn = own[0][a], mx = own[0][a];
    for (int i = 1; i < 4; i++) {
      if (own[i][a] < mn) mn = own[i][a];
      if (own[i][a] > mx) mx = own[i][a];
    }
    lo[a] = ceil_div64(mn, FIX_ONE);
    hi[a] = floor_div64(mx, FIX_ONE);
    if (lo[a] < 0) lo[a] = 0;
    if (hi[a] > dims[a] - 1) hi[a] = dims[a] - 1;
  }
  const double r = (double)P->radius;
  for (int64_t z = lo[2]; z <= hi[2]; z++)
    for (int64_t y = lo[1]; y <= hi[1]; y++)
      for (int64_t x = lo[0]; x <= hi[0]; x++) {
        int64_t p[3] = {x * FIX_ONE, y * FIX_ONE, z * FIX_ONE};
        i128 lam[4];
        if (!inside_tie(own, D, p, lam)) continue;
        rec->n += 1;
        int64_t k[3];
        double f[3], q[3];
        int exact[3];
        map_point(lam, absD, oth, k, f, exact, q);
        size_t vi = ((size_t)z * P->ny + y) * P->nx + x;

        /* intensity: h(a, b) */
        double a = (double)img_own[vi];
        int fg_b = 0;
        for (int dz = 0; dz <= !exact[2]; dz++)
          for (int dy = 0; dy <= !exact[1]; dy++)
            for (int dx = 0; dx <= !exact[0]; dx++)
              if (fetch_zero(img_oth, P->nx, P->ny, P->nz, k[0] + dx, k[1] + dy, k[2] + dz) > 0.0)
                fg_b = 1;
        double b = fg_b ? trilinear(img_oth, P->nx, P->ny, P->nz, k, f, 0) : 0.0;
        int fg_a = a > 0.0;
        double h;
        if (fg_a && fg_b)
          h = (a - b) * (a - b);
        else if (!fg_a && !fg_b)
          h = 0.0;
        else
          h = 1.0;
        rec->h += h;

        /* guidance: each set whose own distance is inside the radius */
        for (int s = 0; s < P->n_sets; s++) {
          double d = (double)map_own[(size_t)s * V + vi];
          if (!(d < r)) continue;
          double d2 = trilinear(map_oth + (size_t)s * V, P->nx, P->ny, P->nz, k, f, 1);
          rec->g += set_w[s] * ((r - d) / r) * (d - d2) * (d - d2);
        }
      }
}

/* ------------------------------------------- Sobol-sampled estimator
 *
 * App. A.2: each tet is sampled at N points drawn uniformly through its
 * barycentric coordinates, N set by the tet's volume; each point takes four
 * numbers r_j in (0, 1], e_j = -log(r_j), lambda_j = e_j / sum(e), from a
 * Sobol sequence seeded from the tet's coordinates.  Sec. 4.1.2 and 4.1.3
 * then give h and the guidance term at each point, as for the rasterized
 * samples.  Readings where the paper leaves the construction open:
 *   - N = floor(rate * |V| + 1/2), |V| the exact volume in voxel^3, at most
 *     2^20 per tet and direction (rate = 1 in the paper's configuration);
 *   - the 4-dimensional Sobol sequence in natural order (point n XORs the
 *     direction numbers of the set bits of n), 32-bit direction numbers from
 *     the primitive polynomials 1 (van der Corput), x + 1, x^2 + x + 1 and
 *     x^3 + x + 1 with initial numbers (1), (1, 3), (1, 3, 1) -- the first
 *     four dimensions of Joe and Kuo's table -- randomised by a digital
 *     shift: XOR with four 32-bit words of a SplitMix64 hash of a global
 *     seed, the direction and the tet's 12 snapped coordinates;
 *   - r_j = (2 floor(u_j / 2^9) + 1) 2^-24, exact in FP32;
 *   - the point is p = v_0 + sum_{i=1..3} lambda_i (v_i - v_0) in the
 *     sampled tet and q = w_0 + sum_{i=1..3} lambda_i (w_i - w_0) in the
 *     other one.  Which corners support a value depends on the bits of p and
 *     q, so they are formed in FP32 in the order written here (the GPU forms
 *     the same bits), with -log from the atanh series below;
 *   - both values are trilinear with zero padding and the exact-support
 *     foreground rule; the guidance band test d < r uses the interpolated own
 *     distance; both distance maps are read edge-clamped. */

#define SOBOL_MAX_N ((int64_t)1 << 20)
#define SM_GAMMA 0x9e3779b97f4a7c15ULL

static uint32_t sobol_dir[4][32];
static int sobol_dir_ready = 0;

static void sobol_init(void) {
  if (sobol_dir_ready) return;
  const int degree[4] = {0, 1, 2, 3};
  const uint32_t inner[4] = {0, 0, 1, 1};        /* a_1 .. a_{s-1}, a_1 the high bit */
  const uint64_t m_first[4][3] = {{1, 0, 0}, {1, 0, 0}, {1, 3, 0}, {1, 3, 1}};
  for (int b = 0; b < 32; b++) sobol_dir[0][b] = 1u << (31 - b);
  for (int j = 1; j < 4; j++) {
    const int s = degree[j];
    uint64_t m[33];
    for (int k = 1; k <= s; k++) m[k] = m_first[j][k - 1];
    for (int k = s + 1; k <= 32; k++) {
      /* m_k = 2 a_1 m_{k-1} ^ ... ^ 2^{s-1} a_{s-1} m_{k-s+1} ^ 2^s m_{k-s} ^ m_{k-s} */
      uint64_t v = m[k - s] ^ (m[k - s] << s);
      for (int i = 1; i < s; i++)
        if ((inner[j] >> (s - 1 - i)) & 1u) v ^= m[k - i] << i;
      m[k] = v;
    }
    for (int k = 1; k <= 32; k++) sobol_dir[j][k - 1] = (uint32_t)(m[k] << (32 - k));
  }
  sobol_dir_ready = 1;
}

static uint32_t sobol_coord(int j, uint32_t n) {
  uint32_t x = 0;
  for (int b = 0; n != 0; b++, n >>= 1)
    if (n & 1u) x ^= sobol_dir[j][b];
  return x;
}

static uint64_t splitmix_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

/* -ln(r), r in (0, 1], in FP32: r = m 2^k with m in [sqrt(1/2), sqrt(2)],
 * ln m = 2 atanh(s), s = (m - 1) / (m + 1), by the series s + s^3/3 + ... +
 * s^11/11 (|s| <= 0.172: truncation below 2e-11). */
static float neg_ln_f32(float r) {
  uint32_t bits;
  memcpy(&bits, &r, sizeof(bits));
  int k = (int)(bits >> 23) - 127;
  const uint32_t mbits = (bits & 0x7fffffu) | 0x3f800000u;
  float m;
  memcpy(&m, &mbits, sizeof(m));
  if (m > 0x1.6a09e6p+0f) {
    m = m * 0.5f;
    k += 1;
  }
  const float s = (m - 1.0f) / (m + 1.0f);
  const float t = s * s;
  float poly = fmaf(t, 0x1.745d18p-4f, 0x1.c71c72p-4f);   /* 1/11, 1/9 */
  poly = fmaf(t, poly, 0x1.24924ap-3f);                   /* 1/7 */
  poly = fmaf(t, poly, 0x1.99999ap-3f);                   /* 1/5 */
  poly = fmaf(t, poly, 0x1.555556p-2f);                   /* 1/3 */
  poly = fmaf(t, poly, 1.0f);
  const float ln_m = (s + s) * poly;
  return -fmaf((float)k, 0x1.62e430p-1f, ln_m);           /* ln 2 */
}

/* Sample count of a tet (|D| = 6 |V| 2^30) at the given rate. */
static int64_t sobol_count(i128 absD, double rate) {
  const double scale = rate / 6442450944.0;   /* rate / (6 * 2^30) */
  const double x = floor((double)absD * scale + 0.5);
  if (!(x > 0.0)) return 0;
  return x >= (double)SOBOL_MAX_N ? SOBOL_MAX_N : (int64_t)x;
}

/* The four shift words of a tet's sequence. */
static void sobol_shift(const int64_t own[4][3], int dir, uint64_t seed, uint32_t shift[4]) {
  uint64_t h = splitmix_mix(seed + SM_GAMMA * (uint64_t)(dir + 1));
  for (int i = 0; i < 4; i++)
    for (int k = 0; k < 3; k++) h = splitmix_mix(h + SM_GAMMA + (uint64_t)(uint32_t)(int32_t)own[i][k]);
  const uint64_t w0 = splitmix_mix(h + SM_GAMMA), w1 = splitmix_mix(h + 2 * SM_GAMMA);
  shift[0] = (uint32_t)w0;
  shift[1] = (uint32_t)(w0 >> 32);
  shift[2] = (uint32_t)w1;
  shift[3] = (uint32_t)(w1 >> 32);
}

/* Point n of a tet's sequence: p in the sampled tet, q in the other. */
static void sobol_point(uint32_t n, const uint32_t shift[4], const float base_own[3],
                        const float edge_own[3][3], const float base_oth[3], const float edge_oth[3][3],
                        float p[3], float q[3]) {
  float e[4];
  for (int j = 0; j < 4; j++) {
    const uint32_t u = sobol_coord(j, n) ^ shift[j];
    const float r = (float)(2u * (u >> 9) + 1u) * 0x1p-24f;
    e[j] = neg_ln_f32(r);
  }
  const float sum = ((e[0] + e[1]) + e[2]) + e[3];
  const float l1 = e[1] / sum, l2 = e[2] / sum, l3 = e[3] / sum;
  for (int a = 0; a < 3; a++) {
    p[a] = fmaf(l3, edge_own[2][a], fmaf(l2, edge_own[1][a], fmaf(l1, edge_own[0][a], base_own[a])));
    q[a] = fmaf(l3, edge_oth[2][a], fmaf(l2, edge_oth[1][a], fmaf(l1, edge_oth[0][a], base_oth[a])));
  }
}

/* FP32 base vertex and edge vectors of a snapped tet, in voxels (exact). */
static void tet_f32(const int64_t v[4][3], float base[3], float edge[3][3]) {
  for (int a = 0; a < 3; a++) {
    base[a] = (float)v[0][a] * 0x1p-10f;
    for (int i = 0; i < 3; i++) edge[i][a] = (float)(v[i + 1][a] - v[0][a]) * 0x1p-10f;
  }
}

/* Cell and fractions of an FP32 point: k = floor(x), f = x - k (exact). */
static void cell_of(const float x[3], int64_t k[3], double f[3]) {
  for (int a = 0; a < 3; a++) {
    const double xd = (double)x[a];
    const double fl = floor(xd);
    k[a] = (int64_t)fl;
    f[a] = xd - fl;
  }
}

/* Foreground by the exact support: a corner with positive weight (the lower
 * corner always, the upper one where f > 0) holding a value > 0. */
static int support_foreground(const float *img, int nx, int ny, int nz, const int64_t k[3],
                              const double f[3]) {
  for (int cz = 0; cz < 2; cz++)
    for (int cy = 0; cy < 2; cy++)
      for (int cx = 0; cx < 2; cx++) {
        if ((cx && !(f[0] > 0.0)) || (cy && !(f[1] > 0.0)) || (cz && !(f[2] > 0.0))) continue;
        if (fetch_zero(img, nx, ny, nz, k[0] + cx, k[1] + cy, k[2] + cz) > 0.0) return 1;
      }
  return 0;
}

static void eval_direction_sobol(const oracle_problem *P, const int64_t own[4][3], const int64_t oth[4][3],
                                 int ref_sign, int dir, const double *set_w, double rate, uint64_t seed,
                                 dir_record *rec) {
  const float *img_own = dir == 0 ? P->img_s : P->img_t;
  const float *img_oth = dir == 0 ? P->img_t : P->img_s;
  const float *map_own = dir == 0 ? P->dmap_s : P->dmap_t;
  const float *map_oth = dir == 0 ? P->dmap_t : P->dmap_s;
  const size_t V = (size_t)P->nx * P->ny * P->nz;
  memset(rec, 0, sizeof(*rec));
  const i128 D = orient(own);
  rec->viol = sgn128(D) == 0 || sgn128(D) != ref_sign;   /* App. A.4, as for the voxel samples */
  const i128 absD = D < 0 ? -D : D;
  rec->vol = (double)absD / 6.0 / (double)((int64_t)1 << (3 * FRAC_BITS));
  const int64_t N = D == 0 ? 0 : sobol_count(absD, rate);
  rec->n = N;
  if (N == 0) return;
  uint32_t shift[4];
  sobol_shift(own, dir, seed, shift);
  float bo[3], eo[3][3], bt[3], et[3][3];
  tet_f32(own, bo, eo);
  tet_f32(oth, bt, et);
  const double radius = (double)P->radius;
  for (int64_t n = 0; n < N; n++) {
    float p[3], q[3];
    sobol_point((uint32_t)n, shift, bo, eo, bt, et, p, q);
    int64_t kp[3], kq[3];
    double fp[3], fq[3];
    cell_of(p, kp, fp);
    cell_of(q, kq, fq);
    const int fa = support_foreground(img_own, P->nx, P->ny, P->nz, kp, fp);
    const int fb = support_foreground(img_oth, P->nx, P->ny, P->nz, kq, fq);
    const double a = fa ? trilinear(img_own, P->nx, P->ny, P->nz, kp, fp, 0) : 0.0;
    const double b = fb ? trilinear(img_oth, P->nx, P->ny, P->nz, kq, fq, 0) : 0.0;
    /* h of Sec. 4.1.2: squared difference inside both foregrounds, 0 in
     * both backgrounds, 1 across */
    rec->h += (fa && fb) ? (a - b) * (a - b) : (fa == fb ? 0.0 : 1.0);
    for (int s = 0; s < P->n_sets; s++) {
      const double d_own = trilinear(map_own + (size_t)s * V, P->nx, P->ny, P->nz, kp, fp, 1);
      if (d_own >= radius) continue;
      const double d_oth = trilinear(map_oth + (size_t)s * V, P->nx, P->ny, P->nz, kq, fq, 1);
      const double diff = d_own - d_oth;
      rec->g += set_w[s] * (radius - d_own) / radius * diff * diff;
    }
  }
}

static double edge_len(const int64_t a[3], const int64_t b[3], double scale) {
  double s = 0.0;
  for (int k = 0; k < 3; k++) {
    double d = (double)(a[k] - b[k]) / scale;
    s += d * d;
  }
  return sqrt(s);
}

/* c_delta * sum over the 6 edges and 4 centroid spokes of (|e_s| - |e_t|)^2 */
static double tet_magnitude(const int64_t S[4][3], const int64_t T[4][3], double c) {
  double acc = 0.0;
  for (int i = 0; i < 4; i++)
    for (int j = i + 1; j < 4; j++) {
      double d = edge_len(S[i], S[j], FIX_ONE) - edge_len(T[i], T[j], FIX_ONE);
      acc += d * d;
    }
  /* spokes: 4 v_i - sum(v) is exact; its length / 4 is |v_i - centroid| */
  int64_t cs[3] = {0, 0, 0}, ct[3] = {0, 0, 0};
  for (int i = 0; i < 4; i++)
    for (int k = 0; k < 3; k++) {
      cs[k] += S[i][k];
      ct[k] += T[i][k];
    }
  for (int i = 0; i < 4; i++) {
    int64_t s4[3], t4[3];
    for (int k = 0; k < 3; k++) {
      s4[k] = 4 * S[i][k];
      t4[k] = 4 * T[i][k];
    }
    double d = edge_len(s4, cs, 4.0 * FIX_ONE) - edge_len(t4, ct, 4.0 * FIX_ONE);
    acc += d * d;
  }
  return c * acc;
}

static int candidate_valid(const float *cand, int n_points) {
  for (int i = 0; i < 6 * n_points; i++) {
    float x = cand[i];
    if (!(fabs((double)x) < COORD_LIMIT)) return 0; /* also rejects NaN */
  }
  return 1;
}

/* Records per (candidate, tet, direction): h, g, n, magnitude (direction 0
 * only), violation volume (0 when no violation), violation (1 or 0). */
typedef struct {
  double rate;
  uint64_t seed;
} sobol_cfg;

static int eval_all(const oracle_problem *P, const float *pts, int pop, const sobol_cfg *sc, double *obj,
                    uint8_t *flags, double *severity, int64_t *counts, double *tet_rec) {
  const int NP = P->n_points, NT = P->n_tets;
  int *ref = (int *)malloc(sizeof(int) * (NT > 0 ? NT : 1));
  for (int t = 0; t < NT; t++) {
    int64_t v[4][3];
    for (int i = 0; i < 4; i++)
      for (int k = 0; k < 3; k++) v[i][k] = snap(P->ref_points[3 * P->tets[4 * t + i] + k]);
    ref[t] = sgn128(orient(v));
  }
  double w_s[64], w_t[64];
  int Gs = 0, Gt = 0;
  for (int s = 0; s < P->n_sets; s++) {
    Gs += P->set_off_s[s + 1] - P->set_off_s[s];
    Gt += P->set_off_t[s + 1] - P->set_off_t[s];
  }
  for (int s = 0; s < P->n_sets && s < 64; s++) {
    w_s[s] = (double)(P->set_off_s[s + 1] - P->set_off_s[s]) / (double)Gs;
    w_t[s] = (double)(P->set_off_t[s + 1] - P->set_off_t[s]) / (double)Gt;
  }
  size_t n_items = (size_t)pop * NT;
  dir_record *recs = (dir_record *)calloc(2 * n_items + 1, sizeof(dir_record));
  double *mags = (double *)calloc(n_items + 1, sizeof(double));
  char *valid = (char *)malloc(pop + 1);
  for (int c = 0; c < pop; c++) valid[c] = (char)candidate_valid(pts + (size_t)c * 6 * NP, NP);

#pragma omp parallel for schedule(dynamic, 1)
  for (long long it = 0; it < (long long)n_items; it++) {
    int c = (int)(it / NT), t = (int)(it % NT);
    if (!valid[c]) continue;
    const float *cand = pts + (size_t)c * 6 * NP;
    int64_t S[4][3], T[4][3];
    for (int i = 0; i < 4; i++) {
      int v = P->tets[4 * t + i];
      for (int k = 0; k < 3; k++) {
        S[i][k] = snap(cand[(0 * 3 + k) * NP + v]);
        T[i][k] = snap(cand[(1 * 3 + k) * NP + v]);
      }
    }
    if (sc) {
      eval_direction_sobol(P, S, T, ref[t], 0, w_s, sc->rate, sc->seed, &recs[2 * it + 0]);
      eval_direction_sobol(P, T, S, ref[t], 1, w_t, sc->rate, sc->seed, &recs[2 * it + 1]);
    } else {
      eval_direction(P, S, T, ref[t], 0, w_s, &recs[2 * it + 0]);
      eval_direction(P, T, S, ref[t], 1, w_t, &recs[2 * it + 1]);
    }
    mags[it] = tet_magnitude(S, T, (double)P->elasticity[t]);
  }

  for (int c = 0; c < pop; c++) {
    double H = 0, G = 0, M = 0, sev = 0;
    int64_t Ns = 0, Nt = 0;
    int fl = 0;
    for (int t = 0; t < NT; t++) {
      size_t it = (size_t)c * NT + t;
      for (int m = 0; m < 2; m++) {
        dir_record *r = &recs[2 * it + m];
        H += r->h;
        G += r->g;
        if (m == 0) Ns += r->n; else Nt += r->n;
        if (r->viol) {
          fl |= 1 << m;
          sev += r->vol;
        }
        if (tet_rec) {
          double *o = tet_rec + (it * 2 + m) * 6;
          o[0] = r->h;
          o[1] = r->g;
          o[2] = (double)r->n;
          o[3] = m == 0 ? mags[it] : 0.0;
          o[4] = r->viol ? r->vol : 0.0;
          o[5] = r->viol ? 1.0 : 0.0;
        }
      }
      M += mags[it];
    }
    if (!valid[c]) {
      obj[3 * c + 0] = obj[3 * c + 1] = obj[3 * c + 2] = NAN;
      flags[c] = 4;
      severity[c] = NAN;
      counts[2 * c] = counts[2 * c + 1] = 0;
      continue;
    }
    double N = (double)(Ns + Nt);
    obj[3 * c + 0] = H / N;                          /* intensity */
    obj[3 * c + 1] = M / (10.0 * (double)NT);        /* magnitude */
    obj[3 * c + 2] = G / N;                          /* guidance */
    flags[c] = (uint8_t)fl;
    severity[c] = sev;
    counts[2 * c] = Ns;
    counts[2 * c + 1] = Nt;
  }
  free(ref);
  free(recs);
  free(mags);
  free(valid);
  return 0;
}

int oracle_eval(const oracle_problem *P, const float *pts, int pop, double *obj, uint8_t *flags,
                double *severity, int64_t *counts, double *tet_rec) {
  return eval_all(P, pts, pop, NULL, obj, flags, severity, counts, tet_rec);
}

/* The same objectives from the Sobol-sampled estimator (counts are the
 * numbers of sample points). */
int oracle_eval_sobol(const oracle_problem *P, const float *pts, int pop, double rate, uint64_t seed,
                      double *obj, uint8_t *flags, double *severity, int64_t *counts, double *tet_rec) {
  if (!(rate > 0.0)) return -1;
  sobol_init();
  const sobol_cfg sc = {rate, seed};
  return eval_all(P, pts, pop, &sc, obj, flags, severity, counts, tet_rec);
}

/* ------------------------------------------------- probes used by the pins */

/* Voxel centres (flat indices) inside one tet under the tie rule. */
int oracle_tet_voxels(const float v[12], int nx, int ny, int nz, int32_t *out, int cap) {
  int64_t w[4][3];
  for (int i = 0; i < 4; i++)
    for (int k = 0; k < 3; k++) w[i][k] = snap(v[3 * i + k]);
  i128 D = orient(w);
  if (D == 0) return 0;
  int n = 0;
  const int dims[3] = {nx, ny, nz};
  int64_t lo[3], hi[3];
  for (int a = 0; a < 3; a++) {
    int64_t mn = w[0][a], mx = w[0][a];
    for (int i = 1; i < 4; i++) {
      if (w[i][a] < mn) mn = w[i][a];
      if (w[i][a] > mx) mx = w[i][a];
    }
    lo[a] = ceil_div64(mn, FIX_ONE);
    hi[a] = floor_div64(mx, FIX_ONE);
    if (lo[a] < 0) lo[a] = 0;
    if (hi[a] > dims[a] - 1) hi[a] = dims[a] - 1;
  }
  for (int64_t z = lo[2]; z <= hi[2]; z++)
    for (int64_t y = lo[1]; y <= hi[1]; y++)
      for (int64_t x = lo[0]; x <= hi[0]; x++) {
        int64_t p[3] = {x * FIX_ONE, y * FIX_ONE, z * FIX_ONE};
        i128 lam[4];
        if (!inside_tie(w, D, p, lam)) continue;
        if (n < cap) out[n] = (int32_t)(((int64_t)z * ny + y) * nx + x);
        n++;
      }
  return n;
}

/* Map a point p (integer voxel, must lie in the own tet) to the other tet:
 * q in FP64 and the per-axis exactness flags of the mapped coordinate. */
int oracle_map(const float own_f[12], const float oth_f[12], const int32_t p_in[3], double q[3],
               int32_t exact_out[3]) {
  int64_t own[4][3], oth[4][3];
  for (int i = 0; i < 4; i++)
    for (int k = 0; k < 3; k++) {
      own[i][k] = snap(own_f[3 * i + k]);
      oth[i][k] = snap(oth_f[3 * i + k]);
    }
  i128 D = orient(own);
  if (D == 0) return -1;
  int64_t p[3] = {(int64_t)p_in[0] * FIX_ONE, (int64_t)p_in[1] * FIX_ONE, (int64_t)p_in[2] * FIX_ONE};
  i128 lam[4];
  int s = sgn128(D);
  for (int i = 0; i < 4; i++) lam[i] = s * orient_replaced(own, i, p);
  int64_t k[3];
  double f[3];
  int ex[3];
  map_point(lam, D < 0 ? -D : D, oth, k, f, ex, q);
  for (int a = 0; a < 3; a++) exact_out[a] = ex[a];
  return 0;
}

/* Trilinear sample at an arbitrary FP64 point (zero padding or clamping). */
double oracle_trilinear(const float *img, int nx, int ny, int nz, const double q[3], int clamp) {
  int64_t k[3];
  double f[3];
  for (int a = 0; a < 3; a++) {
    double fl = floor(q[a]);
    k[a] = (int64_t)fl;
    f[a] = q[a] - fl;
  }
  return trilinear(img, nx, ny, nz, k, f, clamp);
}

/* Exact 6 x signed volume of one tet in units of 2^-30 voxel^3 (as double). */
double oracle_orient(const float v[12]) {
  int64_t w[4][3];
  for (int i = 0; i < 4; i++)
    for (int k = 0; k < 3; k++) w[i][k] = snap(v[3 * i + k]);
  return (double)orient(w);
}

/* Number of threads the OpenMP loops above run with (reported beside the
 * oracle's timings). */
int oracle_threads(void) { return omp_get_max_threads(); }

void oracle_set_threads(int n) { omp_set_num_threads(n); }

/* Coordinate j of point n of the unshifted Sobol sequence (natural order). */
uint32_t oracle_sobol_coord(int j, uint32_t n) {
  sobol_init();
  return sobol_coord(j, n);
}

float oracle_neg_ln_f32(float r) { return neg_ln_f32(r); }

/* The sample points p (in the sampled tet own) and q (in oth) of one tet and
 * direction: writes min(N, cap) points and returns N (-1 on a bad rate). */
int64_t oracle_sobol_points(const float own_f[12], const float oth_f[12], int dir, uint64_t seed, double rate,
                            float *p_out, float *q_out, int64_t cap) {
  if (!(rate > 0.0)) return -1;
  sobol_init();
  int64_t own[4][3], oth[4][3];
  for (int i = 0; i < 4; i++)
    for (int k = 0; k < 3; k++) {
      own[i][k] = snap(own_f[3 * i + k]);
      oth[i][k] = snap(oth_f[3 * i + k]);
    }
  const i128 D = orient(own);
  const int64_t N = D == 0 ? 0 : sobol_count(D < 0 ? -D : D, rate);
  uint32_t shift[4];
  sobol_shift(own, dir, seed, shift);
  float bo[3], eo[3][3], bt[3], et[3][3];
  tet_f32(own, bo, eo);
  tet_f32(oth, bt, et);
  for (int64_t n = 0; n < N && n < cap; n++)
    sobol_point((uint32_t)n, shift, bo, eo, bt, et, p_out + 3 * n, q_out + 3 * n);
  return N;
}

/* ---------------------------------------------------- deformation vector fields
 *
 * Sec. 5.4 compares registrations through a forward DVF on the source grid
 * and an inverse DVF on the target grid, rasterized from MOREA's two meshes.
 * Readings: the voxel centres of a tet are those of the evaluation (the tie
 * rule above); a centre p of tet t of the sampled mesh gets the displacement
 * q - p with q its barycentric image in the other mesh (exact rational,
 * rounded once); a centre covered by several tets (a folded mesh) takes the
 * tet of smallest index, one covered by none the displacement 0; a tet with a
 * vertex coordinate that is not finite or has |x| >= 512 voxels is skipped.
 * cover[d][v] counts the tets that contain centre v. */
int oracle_dvf(const oracle_problem *P, const float *cand, double *fwd, double *inv, int32_t *cover) {
  const int NP = P->n_points;
  const size_t V = (size_t)P->nx * P->ny * P->nz;
  const int dims[3] = {P->nx, P->ny, P->nz};
  int32_t *owner = (int32_t *)malloc(sizeof(int32_t) * (V > 0 ? V : 1));
  for (int d = 0; d < 2; d++) {
    double *out = d == 0 ? fwd : inv;
    int32_t *cov = cover + (size_t)d * V;
    for (size_t v = 0; v < V; v++) {
      owner[v] = -1;
      cov[v] = 0;
      out[3 * v] = out[3 * v + 1] = out[3 * v + 2] = 0.0;
    }
    for (int t = 0; t < P->n_tets; t++) {
      int64_t own[4][3], oth[4][3];
      int good = 1;
      for (int i = 0; i < 4; i++) {
        const int pt = P->tets[4 * t + i];
        for (int k = 0; k < 3; k++) {
          const float xo = cand[(d * 3 + k) * NP + pt], xt = cand[((1 - d) * 3 + k) * NP + pt];
          if (!(fabs((double)xo) < COORD_LIMIT) || !(fabs((double)xt) < COORD_LIMIT)) good = 0;
          own[i][k] = good ? snap(xo) : 0;
          oth[i][k] = good ? snap(xt) : 0;
        }
      }
      if (!good) continue;
      const i128 D = orient(own);
      if (D == 0) continue;
      const i128 absD = D < 0 ? -D : D;
      int64_t lo[3], hi[3];
      for (int a = 0; a < 3; a++) {
        int64_t mn = own[0][a], mx = own[0][a];
        for (int i = 1; i < 4; i++) {
          if (own[i][a] < mn) mn = own[i][a];
          if (own[i][a] > mx) mx = own[i][a];
        }
        lo[a] = ceil_div64(mn, FIX_ONE);
        hi[a] = floor_div64(mx, FIX_ONE);
        if (lo[a] < 0) lo[a] = 0;
        if (hi[a] > dims[a] - 1) hi[a] = dims[a] - 1;
      }
      for (int64_t z = lo[2]; z <= hi[2]; z++)
        for (int64_t y = lo[1]; y <= hi[1]; y++)
          for (int64_t x = lo[0]; x <= hi[0]; x++) {
            const int64_t p[3] = {x * FIX_ONE, y * FIX_ONE, z * FIX_ONE};
            i128 lam[4];
            if (!inside_tie(own, D, p, lam)) continue;
            const size_t v = ((size_t)z * P->ny + y) * P->nx + x;
            cov[v] += 1;
            if (owner[v] >= 0) continue;
            owner[v] = t;
            int64_t kq[3];
            double fq[3], q[3];
            int ex[3];
            map_point(lam, absD, oth, kq, fq, ex, q);
            const int64_t pv[3] = {x, y, z};
            for (int a = 0; a < 3; a++) out[3 * v + a] = (double)(kq[a] - pv[a]) + fq[a];
          }
    }
  }
  free(owner);
  return 0;
}

/* ----------------------------------------------------- point-based guidance
 *
 * The guidance error of the paper's prior work, which Sec. 4.1.3 replaces by
 * the continuous form: every point c of C_s is located in the source mesh,
 * mapped to the target mesh through its barycentric coordinates, and its
 * distance to the closest point of the set's C_t taken.  Readings: points are
 * snapped like mesh coordinates; a point belongs to the tet that holds it
 * under the tie rule of the evaluation (the smallest index if several, a
 * folded mesh); the value is the mean of the squared distances over all
 * points of all sets (each set weighted by |C_i| / |G| as in the continuous
 * form); points in no tet are left out and counted.  pts_s and pts_t are the
 * concatenated sets (CSR offsets of the problem). */
int oracle_point_guidance(const oracle_problem *P, const float *set_pts_s, const float *set_pts_t,
                          const float *pts, int pop, double *f, int32_t *unmapped) {
  const int NP = P->n_points, NT = P->n_tets;
  const int G = P->n_sets > 0 ? P->set_off_s[P->n_sets] : 0;
  for (int c = 0; c < pop; c++) {
    const float *cand = pts + (size_t)c * 6 * NP;
    f[c] = NAN;
    unmapped[c] = 0;
    if (!candidate_valid(cand, NP)) continue;
    double total = 0.0;
    int n = 0;
    for (int s = 0; s < P->n_sets; s++)
      for (int j = P->set_off_s[s]; j < P->set_off_s[s + 1]; j++) {
        const int64_t cp[3] = {snap(set_pts_s[3 * j]), snap(set_pts_s[3 * j + 1]), snap(set_pts_s[3 * j + 2])};
        int found = 0;
        double q[3] = {0, 0, 0};
        for (int t = 0; t < NT && !found; t++) {
          int64_t S[4][3], T[4][3];
          for (int i = 0; i < 4; i++)
            for (int k = 0; k < 3; k++) {
              S[i][k] = snap(cand[k * NP + P->tets[4 * t + i]]);
              T[i][k] = snap(cand[(3 + k) * NP + P->tets[4 * t + i]]);
            }
          const i128 D = orient(S);
          if (D == 0) continue;
          i128 lam[4];
          if (!inside_tie(S, D, cp, lam)) continue;
          int64_t kq[3];
          double fq[3];
          int ex[3];
          map_point(lam, D < 0 ? -D : D, T, kq, fq, ex, q);
          found = 1;
        }
        if (!found) {
          unmapped[c] += 1;
          continue;
        }
        double best = INFINITY;
        for (int k = P->set_off_t[s]; k < P->set_off_t[s + 1]; k++) {
          double d2 = 0.0;
          for (int a = 0; a < 3; a++) {
            const double diff = q[a] - (double)snap(set_pts_t[3 * k + a]) / (double)FIX_ONE;
            d2 += diff * diff;
          }
          if (d2 < best) best = d2;
        }
        total += best;
        n += 1;
      }
    (void)G;
    f[c] = n > 0 ? total / n : NAN;
  }
  return 0;
}
