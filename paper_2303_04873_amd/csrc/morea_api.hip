// Host side of libmorea: the C-ABI entry points declared in include/morea.h.
// Argument validation, conversion of the images to their storage type,
// device uploads, set-up kernels and kernel launches.  No entry point that
// evaluates candidates allocates memory or synchronises the host.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "morea_internal.h"

using namespace morea;

namespace {

thread_local std::string g_error;

morea_status fail(morea_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
  return s;
}

morea_status hip_fail(hipError_t e, const char* what) {
  return fail(MOREA_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Round-to-nearest-even conversions of the stored images.
uint16_t to_bf16(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  u = u + 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

uint16_t to_f16(float f) {
  _Float16 h = static_cast<_Float16>(f);
  uint16_t u;
  memcpy(&u, &h, 2);
  return u;
}

int64_t snap_host(float x) { return static_cast<int64_t>(rint(static_cast<double>(x) * 1024.0)); }

bool coord_ok(float x) { return fabsf(x) < kCoordLimit; }

template <typename T>
morea_status upload(morea_problem* p, T** dst, const void* src, size_t bytes) {
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, bytes ? bytes : 4);
  if (e != hipSuccess) return fail(MOREA_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  p->allocations.push_back(d);
  if (src && bytes) {
    e = hipMemcpy(d, src, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  }
  *dst = static_cast<T*>(d);
  return MOREA_OK;
}

morea_status check_pending() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "earlier device work failed");
  return MOREA_OK;
}

void free_all(morea_problem* p) {
  for (void* a : p->allocations) (void)hipFree(a);
  p->allocations.clear();
}

}  // namespace

namespace morea {
void set_error(const char* msg) { g_error = msg; }

void ensure_partial_shape(morea_problem* p) {
  if (p->partial_chunk >= 0) return;   // chosen already (a default or the tuner's)
  int cus = 0, per_cu = 0;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
  per_cu = partial_blocks_per_cu(p->storage);
  // the tuner's choice on the 128x128x96 workloads: 4 blocks per compute
  // unit (at most the occupancy limit), 8 items per queue pop
  p->partial_blocks = std::max(1, cus) * std::max(1, std::min(4, per_cu));
  p->partial_chunk = 8;
}
}  // namespace morea

extern "C" {

const char* morea_last_error(void) { return g_error.c_str(); }

morea_status morea_problem_create(const morea_problem_desc* d, morea_problem** out) {
  if (!out) return fail(MOREA_EINVAL, "out is NULL");
  *out = nullptr;
  if (!d) return fail(MOREA_EINVAL, "desc is NULL");
  for (int k = 0; k < 3; k++)
    if (d->dims[k] < 1 || d->dims[k] > 1024) return fail(MOREA_EINVAL, "dims[%d]=%d outside [1,1024]", k, d->dims[k]);
  if (!d->image_src || !d->image_tgt) return fail(MOREA_EINVAL, "image pointer is NULL");
  if (d->storage < 0 || d->storage > 2) return fail(MOREA_EINVAL, "storage %d unknown", d->storage);
  if (d->n_points < 4 || d->n_tets < 1) return fail(MOREA_EINVAL, "need >= 4 points and >= 1 tet");
  if (d->n_points > (1 << 28) || d->n_tets > (1 << 28)) return fail(MOREA_EINVAL, "more than 2^28 points or tets");
  if (!d->tets || !d->ref_points || !d->elasticity) return fail(MOREA_EINVAL, "mesh pointer is NULL");
  if (d->n_sets < 0 || d->n_sets > kMaxSets) return fail(MOREA_EINVAL, "n_sets %d outside [0,%d]", d->n_sets, kMaxSets);
  if (d->max_population < 1) return fail(MOREA_EINVAL, "max_population must be >= 1");
  const int nx = d->dims[0], ny = d->dims[1], nz = d->dims[2];
  const size_t V = static_cast<size_t>(nx) * ny * nz;
  if (V > (static_cast<size_t>(1) << 29))
    return fail(MOREA_EINVAL, "%zu voxels per image exceed the limit 2^29", V);
  float min_pos = INFINITY;   // smallest positive value of either image
  for (size_t i = 0; i < V; i++) {
    float a = d->image_src[i], b = d->image_tgt[i];
    if (!(a >= 0.f && a < INFINITY) || !(b >= 0.f && b < INFINITY))
      return fail(MOREA_EINVAL, "image value at %zu is negative or not finite", i);
    if (a > 0.f && a < min_pos) min_pos = a;
    if (b > 0.f && b < min_pos) min_pos = b;
  }
  for (int i = 0; i < 3 * d->n_points; i++)
    if (!coord_ok(d->ref_points[i])) return fail(MOREA_EINVAL, "ref_points[%d] out of range", i);
  std::vector<int8_t> ref_sign(d->n_tets);
  for (int t = 0; t < d->n_tets; t++) {
    int64_t v[4][3];
    for (int i = 0; i < 4; i++) {
      int idx = d->tets[4 * t + i];
      if (idx < 0 || idx >= d->n_points) return fail(MOREA_EINVAL, "tet %d has vertex index %d", t, idx);
      for (int k = 0; k < 3; k++) v[i][k] = snap_host(d->ref_points[3 * idx + k]);
    }
    int64_t a[3], b[3], c[3];
    for (int k = 0; k < 3; k++) {
      a[k] = v[1][k] - v[0][k];
      b[k] = v[2][k] - v[0][k];
      c[k] = v[3][k] - v[0][k];
    }
    int64_t det = a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
                  a[2] * (b[0] * c[1] - b[1] * c[0]);
    if (det == 0) return fail(MOREA_EINVAL, "reference tet %d is flat", t);
    ref_sign[t] = det > 0 ? 1 : -1;
    float c_d = d->elasticity[t];
    if (!(c_d > 0.f && c_d < INFINITY)) return fail(MOREA_EINVAL, "elasticity[%d] not positive", t);
  }
  std::vector<int> set_off[2];
  std::vector<int> set_fix[2];
  float set_w[2][kMaxSets] = {};
  if (d->n_sets > 0) {
    const int32_t* offs[2] = {d->set_off_src, d->set_off_tgt};
    const float* pts[2] = {d->set_pts_src, d->set_pts_tgt};
    for (int m = 0; m < 2; m++) {
      if (!offs[m] || !pts[m]) return fail(MOREA_EINVAL, "guidance set pointer is NULL");
      if (offs[m][0] != 0) return fail(MOREA_EINVAL, "set offsets must start at 0");
      for (int s = 0; s < d->n_sets; s++)
        if (offs[m][s + 1] <= offs[m][s]) return fail(MOREA_EINVAL, "guidance set %d of image %d is empty", s, m);
      const int total = offs[m][d->n_sets];
      set_off[m].assign(offs[m], offs[m] + d->n_sets + 1);
      set_fix[m].resize(3 * static_cast<size_t>(total));
      for (int i = 0; i < 3 * total; i++) {
        if (!coord_ok(pts[m][i])) return fail(MOREA_EINVAL, "guidance point coordinate %d out of range", i);
        set_fix[m][i] = static_cast<int>(snap_host(pts[m][i]));
      }
      for (int s = 0; s < d->n_sets; s++)
        set_w[m][s] = static_cast<float>(static_cast<double>(offs[m][s + 1] - offs[m][s]) / total);
    }
  }
  float radius = d->radius > 0.f ? d->radius : 0.025f * static_cast<float>(nx);
  if (!(radius < INFINITY)) return fail(MOREA_EINVAL, "radius not finite");

  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  morea_problem* p = new morea_problem();
  p->device = dev;
  p->storage = d->storage;
  p->max_population = d->max_population;
  p->voxels = V;
  p->tets_host.assign(d->tets, d->tets + 4 * static_cast<size_t>(d->n_tets));
  p->ref_host.assign(d->ref_points, d->ref_points + 3 * static_cast<size_t>(d->n_points));
  ProblemView& P = p->view;
  P.nx = nx;
  P.ny = ny;
  P.nz = nz;
  P.px = padded_row(nx);
  P.pxy = P.px * (ny + 2);
  const size_t PV = static_cast<size_t>(P.pxy) * (nz + 2);
  P.pvox = static_cast<unsigned>(PV);
  P.n_points = d->n_points;
  P.n_tets = d->n_tets;
  P.n_sets = d->n_sets;
  P.radius = radius;
  P.inv_radius = 1.0f / radius;
  // inputs >= 2^-39 stay >= 2^-40 after BF16 rounding; FP16 keeps positive
  // values >= 2^-24 or rounds them to 0
  P.fg_from_b = min_pos >= 0x1p-39f ? 1 : 0;

  morea_status st = MOREA_OK;
  auto guard = [&](morea_status s) {
    if (s != MOREA_OK && st == MOREA_OK) st = s;
    return s == MOREA_OK;
  };
  // images in their storage type
  for (int m = 0; m < 2 && st == MOREA_OK; m++) {
    const float* img = m == 0 ? d->image_src : d->image_tgt;
    void* dst = nullptr;
    // padded copy: a border of zeros one voxel wide on every side
    std::vector<float> pad(PV, 0.f);
    for (int z = 0; z < nz; z++)
      for (int y = 0; y < ny; y++)
        memcpy(pad.data() + ((static_cast<size_t>(z) + 1) * (ny + 2) + (y + 1)) * P.px + 1,
               img + (static_cast<size_t>(z) * ny + y) * nx, nx * sizeof(float));
    if (d->storage == kF32) {
      guard(upload(p, &dst, pad.data(), PV * sizeof(float)));
    } else {
      std::vector<uint16_t> q(PV);
      for (size_t i = 0; i < PV; i++) q[i] = d->storage == kBF16 ? to_bf16(pad[i]) : to_f16(pad[i]);
      guard(upload(p, &dst, q.data(), PV * sizeof(uint16_t)));
    }
    P.img[m] = dst;
  }
  float* sw = nullptr;
  if (st == MOREA_OK) guard(upload(p, &sw, set_w, sizeof(set_w)));
  P.set_w = sw;
  int4* tets = nullptr;
  int8_t* rs = nullptr;
  float* el = nullptr;
  if (st == MOREA_OK) guard(upload(p, &tets, d->tets, sizeof(int4) * d->n_tets));
  if (st == MOREA_OK) guard(upload(p, &rs, ref_sign.data(), d->n_tets));
  if (st == MOREA_OK) guard(upload(p, &el, d->elasticity, sizeof(float) * d->n_tets));
  P.tets = tets;
  P.ref_sign = rs;
  P.elasticity = el;
  for (int m = 0; m < 2 && st == MOREA_OK; m++) {
    float* dm = nullptr;
    uint8_t* band = nullptr;
    guard(upload(p, &dm, nullptr, sizeof(float) * PV * std::max(d->n_sets, 1)));
    if (st == MOREA_OK) guard(upload(p, &band, nullptr, PV));
    if (st != MOREA_OK) break;
    if (d->n_sets > 0) {
      int* doff = nullptr;
      int* dpts = nullptr;
      guard(upload(p, &doff, set_off[m].data(), sizeof(int) * set_off[m].size()));
      if (st == MOREA_OK) guard(upload(p, &dpts, set_fix[m].data(), sizeof(int) * set_fix[m].size()));
      if (st != MOREA_OK) break;
      e = launch_distance_maps(nx, ny, nz, d->n_sets, doff, dpts, radius, dm, band, nullptr);
      if (e != hipSuccess) guard(hip_fail(e, "distance map kernel"));
      p->d_set_off[m] = doff;
      p->d_set_fix[m] = dpts;
    } else {
      e = hipMemset(band, 0, PV);
      if (e != hipSuccess) guard(hip_fail(e, "hipMemset"));
    }
    P.dmap[m] = dm;
    P.band[m] = band;
    uint8_t* cells = nullptr;
    guard(upload(p, &cells, nullptr, PV));
    if (st != MOREA_OK) break;
    e = launch_band_cells(P, band, cells, nullptr);
    if (e != hipSuccess) guard(hip_fail(e, "band cell kernel"));
    p->band_cell[m] = cells;
    uint8_t* fgc = nullptr;
    guard(upload(p, &fgc, nullptr, PV));
    if (st != MOREA_OK) break;
    e = launch_fg_cells(P, d->storage, P.img[m], fgc, nullptr);
    if (e != hipSuccess) guard(hip_fail(e, "foreground cell kernel"));
    p->fg_cell[m] = fgc;
  }
  if (st == MOREA_OK) {
    const size_t nrec = static_cast<size_t>(d->max_population) * d->n_tets * 2;
    guard(upload(p, &p->work_records, nullptr, nrec * sizeof(Record)));
    if (st == MOREA_OK) guard(upload(p, &p->work_totals, nullptr, sizeof(Totals) * d->max_population));
  }
  if (st == MOREA_OK) {
    // point -> incident tets and point -> neighbours, for fold repair
    const int NP = d->n_points;
    std::vector<int> inc_off(NP + 1, 0), inc(4 * static_cast<size_t>(d->n_tets));
    for (int t = 0; t < d->n_tets; t++)
      for (int i = 0; i < 4; i++) inc_off[p->tets_host[4 * t + i] + 1]++;
    for (int v = 0; v < NP; v++) inc_off[v + 1] += inc_off[v];
    std::vector<int> fill(inc_off.begin(), inc_off.end() - 1);
    std::vector<std::vector<int>> nbs(NP);
    for (int t = 0; t < d->n_tets; t++)
      for (int i = 0; i < 4; i++) {
        const int v = p->tets_host[4 * t + i];
        inc[fill[v]++] = (t << 2) | i;
        for (int k = 0; k < 4; k++)
          if (k != i) nbs[v].push_back(p->tets_host[4 * t + k]);
      }
    std::vector<int> nb_off(NP + 1, 0), nb;
    for (int v = 0; v < NP; v++) {
      std::sort(nbs[v].begin(), nbs[v].end());
      nbs[v].erase(std::unique(nbs[v].begin(), nbs[v].end()), nbs[v].end());
      nb.insert(nb.end(), nbs[v].begin(), nbs[v].end());
      nb_off[v + 1] = static_cast<int>(nb.size());
    }
    guard(upload(p, &p->d_pinc_off, inc_off.data(), sizeof(int) * inc_off.size()));
    if (st == MOREA_OK) guard(upload(p, &p->d_pinc, inc.data(), sizeof(int) * inc.size()));
    if (st == MOREA_OK) guard(upload(p, &p->d_nb_off, nb_off.data(), sizeof(int) * nb_off.size()));
    if (st == MOREA_OK) guard(upload(p, &p->d_nb, nb.data(), sizeof(int) * nb.size()));
  }
  if (st == MOREA_OK) {
    e = hipDeviceSynchronize();
    if (e != hipSuccess) guard(hip_fail(e, "set-up"));
  }
  // the device address of the allocation-free entry point's scratch, once
  // per device, with the problem's device current
  if (st == MOREA_OK) guard(static_scratch_init(dev));
  if (st != MOREA_OK) {
    std::string msg = g_error;
    free_all(p);
    delete p;
    g_error = msg;
    return st;
  }
  *out = p;
  return MOREA_OK;
}

void morea_problem_destroy(morea_problem* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  for (auto& g : p->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
  for (void* a : p->partial_allocs) (void)hipFree(a);
  for (void* a : p->group_allocs) (void)hipFree(a);
  free_all(p);
  delete p;
}

size_t morea_cache_bytes(const morea_problem* p, int32_t pop) {
  if (!p || pop < 0) return 0;
  return static_cast<size_t>(pop) * p->view.n_tets * 2 * sizeof(Record) +
         static_cast<size_t>(pop) * sizeof(Totals);
}

morea_status morea_eval_full(morea_problem* p, const float* pts, int32_t pop, float* obj,
                             uint8_t* flags, float* severity, uint32_t* counts, void* cache,
                             void* stream) {
  if (!p) return fail(MOREA_EINVAL, "problem is NULL");
  if (pop < 0) return fail(MOREA_EINVAL, "pop %d < 0", pop);
  if (pop > p->max_population) return fail(MOREA_ERANGE, "pop %d > max_population %d", pop, p->max_population);
  if (pop == 0) return MOREA_OK;
  if (!pts || !obj || !flags || !severity || !counts) return fail(MOREA_EINVAL, "NULL argument");
  morea_status st = check_pending();
  if (st != MOREA_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Record* rec = p->work_records;
  Totals* tot = nullptr;
  if (cache) {
    rec = static_cast<Record*>(cache);
    tot = reinterpret_cast<Totals*>(static_cast<char*>(cache) +
                                    static_cast<size_t>(pop) * p->view.n_tets * 2 * sizeof(Record));
  }
  hipError_t e = launch_eval_full(p->view, p->storage, pts, pop, rec, s);
  if (e != hipSuccess) return hip_fail(e, "eval kernel launch");
  e = launch_finalize(p->view, pts, pop, rec, obj, flags, severity, counts, tot, s);
  if (e != hipSuccess) return hip_fail(e, "finalize kernel launch");
  return MOREA_OK;
}

morea_status morea_debug_distance_map(morea_problem* p, int32_t image, int32_t set, float* host_out,
                                      uint8_t* band_out) {
  if (!p || !host_out || image < 0 || image > 1 || set < 0 || set >= p->view.n_sets)
    return fail(MOREA_EINVAL, "bad argument");
  // the stored volumes are padded: copy them whole and return the grid part
  const ProblemView& P = p->view;
  std::vector<float> dm(P.pvox);
  std::vector<uint8_t> bd(P.pvox);
  hipError_t e = hipMemcpy(dm.data(), P.dmap[image] + static_cast<size_t>(set) * P.pvox,
                           P.pvox * sizeof(float), hipMemcpyDeviceToHost);
  if (e == hipSuccess && band_out)
    e = hipMemcpy(bd.data(), P.band[image], P.pvox, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  for (int z = 0; z < P.nz; z++)
    for (int y = 0; y < P.ny; y++) {
      const size_t src = (static_cast<size_t>(z + 1) * (P.ny + 2) + (y + 1)) * P.px + 1;
      const size_t dst = (static_cast<size_t>(z) * P.ny + y) * P.nx;
      memcpy(host_out + dst, dm.data() + src, P.nx * sizeof(float));
      if (band_out) memcpy(band_out + dst, bd.data() + src, P.nx);
    }
  return MOREA_OK;
}

}  // extern "C"

namespace {

void free_list(std::vector<void*>& v) {
  for (void* a : v) (void)hipFree(a);
  v.clear();
}

template <typename T>
morea_status upload_to(std::vector<void*>& list, T** dst, const void* src, size_t bytes) {
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, bytes ? bytes : 4);
  if (e != hipSuccess) return fail(MOREA_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  list.push_back(d);
  if (src && bytes) {
    e = hipMemcpy(d, src, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  }
  *dst = static_cast<T*>(d);
  return MOREA_OK;
}

void drop_graph(morea_problem* p) {
  for (auto& g : p->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g = morea_problem::GraphSlot{};
  }
  p->last_partial = false;
}

void drop_partial(morea_problem* p) {
  drop_graph(p);
  (void)hipDeviceSynchronize();
  free_list(p->partial_allocs);
  p->max_evals = 0;
  p->d_row_off = p->d_item_off = p->d_queue = nullptr;
  p->d_partial_records = nullptr;
  p->d_item_info = nullptr;
  p->d_item_dest = p->d_grp_count = p->d_grp_base = p->d_eval_rank = nullptr;
}

}  // namespace

extern "C" {

morea_status morea_set_groups(morea_problem* p, int32_t n_groups, const int32_t* grp_off,
                              const int32_t* grp_pts) {
  if (!p) return fail(MOREA_EINVAL, "problem is NULL");
  if (n_groups < 1 || !grp_off || !grp_pts) return fail(MOREA_EINVAL, "need n_groups >= 1 and CSR arrays");
  const int NP = p->view.n_points, NT = p->view.n_tets;
  if (grp_off[0] != 0) return fail(MOREA_EINVAL, "grp_off[0] must be 0");
  for (int g = 0; g < n_groups; g++)
    if (grp_off[g + 1] <= grp_off[g]) return fail(MOREA_EINVAL, "group %d is empty", g);
  // point -> incident tets
  std::vector<int> inc_off(NP + 1, 0), inc;
  for (int t = 0; t < NT; t++)
    for (int i = 0; i < 4; i++) inc_off[p->tets_host[4 * t + i] + 1]++;
  for (int v = 0; v < NP; v++) inc_off[v + 1] += inc_off[v];
  inc.resize(inc_off[NP]);
  {
    std::vector<int> fill(inc_off.begin(), inc_off.end() - 1);
    for (int t = 0; t < NT; t++)
      for (int i = 0; i < 4; i++) {
        const int v = p->tets_host[4 * t + i];
        inc[fill[v]++] = t;
      }
  }
  std::vector<int> pos(NP, -1), tet_mark(NT, -1), dep_off(1, 0), dep_tet;
  std::vector<int8_t> dep_local;
  int max_dep = 0, max_group = 0;
  for (int g = 0; g < n_groups; g++) {
    const int b = grp_off[g], e = grp_off[g + 1];
    if (e - b > 127) return fail(MOREA_EINVAL, "group %d has %d points (at most 127)", g, e - b);
    max_group = std::max(max_group, e - b);
    std::vector<int> tl;
    for (int k = b; k < e; k++) {
      const int v = grp_pts[k];
      if (v < 0 || v >= NP) return fail(MOREA_EINVAL, "group %d point %d out of range", g, v);
      if (pos[v] >= 0) return fail(MOREA_EINVAL, "group %d repeats point %d", g, v);
      pos[v] = k - b;
      for (int q = inc_off[v]; q < inc_off[v + 1]; q++)
        if (tet_mark[inc[q]] != g) {
          tet_mark[inc[q]] = g;
          tl.push_back(inc[q]);
        }
    }
    std::sort(tl.begin(), tl.end());
    for (int t : tl) {
      dep_tet.push_back(t);
      for (int i = 0; i < 4; i++) dep_local.push_back(static_cast<int8_t>(pos[p->tets_host[4 * t + i]]));
    }
    for (int k = b; k < e; k++) pos[grp_pts[k]] = -1;
    dep_off.push_back(static_cast<int>(dep_tet.size()));
    max_dep = std::max(max_dep, static_cast<int>(tl.size()));
  }
  drop_partial(p);
  free_list(p->group_allocs);
  morea_status st = upload_to(p->group_allocs, &p->d_grp_off, grp_off, sizeof(int) * (n_groups + 1));
  if (st == MOREA_OK)
    st = upload_to(p->group_allocs, &p->d_grp_pts, grp_pts, sizeof(int) * grp_off[n_groups]);
  if (st == MOREA_OK) st = upload_to(p->group_allocs, &p->d_dep_off, dep_off.data(), sizeof(int) * dep_off.size());
  if (st == MOREA_OK) st = upload_to(p->group_allocs, &p->d_dep_tet, dep_tet.data(), sizeof(int) * dep_tet.size());
  if (st == MOREA_OK) st = upload_to(p->group_allocs, &p->d_dep_local, dep_local.data(), dep_local.size());
  if (st != MOREA_OK) {
    free_list(p->group_allocs);
    p->n_groups = 0;
    return st;
  }
  p->n_groups = n_groups;
  p->max_dep = max_dep;
  p->max_group = max_group;
  return MOREA_OK;
}

morea_status morea_reserve_partial(morea_problem* p, int32_t max_evals) {
  if (!p) return fail(MOREA_EINVAL, "problem is NULL");
  if (p->n_groups == 0) return fail(MOREA_ESTATE, "call morea_set_groups first");
  if (max_evals < 1) return fail(MOREA_EINVAL, "max_evals must be >= 1");
  drop_partial(p);
  morea_status st = upload_to(p->partial_allocs, &p->d_row_off, nullptr, sizeof(int) * max_evals);
  if (st == MOREA_OK) st = upload_to(p->partial_allocs, &p->d_item_off, nullptr, sizeof(int) * (max_evals + 1));
  if (st == MOREA_OK) st = upload_to(p->partial_allocs, &p->d_queue, nullptr, sizeof(int) * 64);
  if (st == MOREA_OK)
    st = upload_to(p->partial_allocs, &p->d_partial_records, nullptr,
                   sizeof(Record) * 2 * static_cast<size_t>(max_evals) * p->max_dep);
  if (st == MOREA_OK)
    // at least room for the prefix kernels' block totals (two ints per 256
    // evaluations), which use the head of this array before the items fill it
    st = upload_to(p->partial_allocs, &p->d_item_info, nullptr,
                   sizeof(int4) * std::max(static_cast<size_t>(max_evals) * p->max_dep,
                                           static_cast<size_t>(max_evals) / 128 + 2));
  if (st == MOREA_OK)
    st = upload_to(p->partial_allocs, &p->d_item_dest, nullptr,
                   sizeof(int) * static_cast<size_t>(max_evals) * p->max_dep);
  if (st == MOREA_OK) st = upload_to(p->partial_allocs, &p->d_grp_count, nullptr, sizeof(int) * p->n_groups);
  if (st == MOREA_OK) st = upload_to(p->partial_allocs, &p->d_grp_base, nullptr, sizeof(int) * p->n_groups);
  if (st == MOREA_OK) st = upload_to(p->partial_allocs, &p->d_eval_rank, nullptr, sizeof(int) * max_evals);
  if (st != MOREA_OK) {
    free_list(p->partial_allocs);
    return st;
  }
  if (!p->capture_stream) {
    hipError_t e = hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
  }
  ensure_partial_shape(p);
  p->max_evals = max_evals;
  return MOREA_OK;
}

static morea_status partial_args(morea_problem* p, const float* parent_pts, int32_t n_parents,
                                 const void* parent_cache, int32_t n_evals,
                                 const int32_t* eval_parent, const int32_t* eval_group,
                                 const float* new_coords, float* obj, uint8_t* flags,
                                 float* severity, uint32_t* counts) {
  if (!p) return fail(MOREA_EINVAL, "problem is NULL");
  if (p->n_groups == 0) return fail(MOREA_ESTATE, "call morea_set_groups first");
  if (p->max_evals == 0) return fail(MOREA_ESTATE, "call morea_reserve_partial first");
  if (n_evals < 0 || n_parents < 1) return fail(MOREA_EINVAL, "bad n_evals / n_parents");
  if (n_evals > p->max_evals) return fail(MOREA_ERANGE, "n_evals %d > reserved %d", n_evals, p->max_evals);
  if (n_evals > 0 && (!parent_pts || !parent_cache || !eval_parent || !eval_group || !new_coords ||
                      !obj || !flags || !severity || !counts))
    return fail(MOREA_EINVAL, "NULL argument");
  return MOREA_OK;
}

static hipError_t partial_launch(morea_problem* p, const float* parent_pts, int32_t n_parents,
                                 const void* parent_cache, int32_t n_evals,
                                 const int32_t* eval_parent, const int32_t* eval_group,
                                 const float* new_coords, float* obj, uint8_t* flags,
                                 float* severity, uint32_t* counts, int blocks, int chunk,
                                 hipStream_t s) {
  PartialItems I;
  I.parent_pts = parent_pts;
  I.eval_parent = eval_parent;
  I.eval_group = eval_group;
  I.new_coords = new_coords;
  I.row_off = p->d_row_off;
  I.item_off = p->d_item_off;
  I.grp_off = p->d_grp_off;
  I.grp_pts = p->d_grp_pts;
  I.dep_off = p->d_dep_off;
  I.dep_tet = p->d_dep_tet;
  I.dep_local = p->d_dep_local;
  I.item_info = p->d_item_info;
  I.item_dest = p->d_item_dest;
  I.grp_count = p->d_grp_count;
  I.grp_base = p->d_grp_base;
  I.eval_rank = p->d_eval_rank;
  I.n_evals = n_evals;
  const Record* prec = static_cast<const Record*>(parent_cache);
  const Totals* ptot = reinterpret_cast<const Totals*>(
      static_cast<const char*>(parent_cache) + static_cast<size_t>(n_parents) * p->view.n_tets * 2 * sizeof(Record));
  if (chunk == 0) {   // grid form: one wave per item pair up to the bound n_evals x max_dep
    const long long bound = static_cast<long long>(n_evals) * std::max(p->max_dep, 1);
    blocks = static_cast<int>(std::min<long long>((bound + 7) / 8, 0x7fffffffLL));
  }
  return launch_partial(p->view, p->storage, I, n_parents, p->n_groups, prec, ptot,
                        p->d_partial_records, p->d_queue, blocks, chunk, obj, flags, severity,
                        counts, s);
}

morea_status morea_eval_partial(morea_problem* p, const float* parent_pts, int32_t n_parents,
                                const void* parent_cache, int32_t n_evals,
                                const int32_t* eval_parent, const int32_t* eval_group,
                                const float* new_coords, float* obj, uint8_t* flags,
                                float* severity, uint32_t* counts, void* stream) {
  morea_status st = partial_args(p, parent_pts, n_parents, parent_cache, n_evals, eval_parent,
                                 eval_group, new_coords, obj, flags, severity, counts);
  if (st != MOREA_OK) return st;
  if (n_evals == 0) return MOREA_OK;
  st = check_pending();
  if (st != MOREA_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const void* key[9] = {parent_pts, parent_cache, eval_parent, eval_group, new_coords, obj, flags,
                        severity, counts};
  const int key_n[4] = {n_parents, n_evals, p->partial_blocks, p->partial_chunk};
  morea_problem::GraphSlot* slot = nullptr;
  for (auto& g : p->graphs)
    if (g.exec && memcmp(key, g.key, sizeof(key)) == 0 && memcmp(key_n, g.key_n, sizeof(key_n)) == 0) slot = &g;
  if (!slot) {
    // capture into the least recently used slot (an empty one first)
    slot = &p->graphs[0];
    for (auto& g : p->graphs)
      if (!g.exec || (slot->exec && g.used < slot->used)) {
        slot = &g;
        if (!g.exec) break;
      }
    if (slot->exec) (void)hipGraphExecDestroy(slot->exec);
    *slot = morea_problem::GraphSlot{};
    hipError_t e = hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t le = partial_launch(p, parent_pts, n_parents, parent_cache, n_evals, eval_parent,
                                   eval_group, new_coords, obj, flags, severity, counts,
                                   p->partial_blocks, p->partial_chunk, p->capture_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(p->capture_stream, &g);
    if (le != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hip_fail(le, "partial kernels");
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&slot->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      slot->exec = nullptr;
      return hip_fail(e, "hipGraphInstantiate");
    }
    memcpy(slot->key, key, sizeof(key));
    memcpy(slot->key_n, key_n, sizeof(key_n));
    p->graph_captures++;
  }
  slot->used = ++p->graph_clock;
  p->last_partial = false;
  hipError_t e = hipGraphLaunch(slot->exec, s);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  memcpy(p->last_key, key, sizeof(p->last_key));
  p->last_n[0] = n_parents;
  p->last_n[1] = n_evals;
  p->last_partial = true;
  return MOREA_OK;
}

morea_status morea_tune_partial(morea_problem* p, const float* parent_pts, int32_t n_parents,
                                const void* parent_cache, int32_t n_evals,
                                const int32_t* eval_parent, const int32_t* eval_group,
                                const float* new_coords, float* obj, uint8_t* flags,
                                float* severity, uint32_t* counts, void* stream,
                                float* best_ms) {
  morea_status st = partial_args(p, parent_pts, n_parents, parent_cache, n_evals, eval_parent,
                                 eval_group, new_coords, obj, flags, severity, counts);
  if (st != MOREA_OK) return st;
  if (n_evals == 0) return MOREA_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int cus = 0, per_cu = 0;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
  per_cu = partial_blocks_per_cu(p->storage);
  cus = std::max(cus, 1);
  per_cu = std::max(per_cu, 1);
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
    return fail(MOREA_EDEVICE, "hipEventCreate");
  float best = 1e30f;
  int best_blocks = p->partial_blocks, best_chunk = p->partial_chunk;
  const int chunks[5] = {1, 2, 4, 8, 16};
  // every persistent shape, then the grid form (chunk 0)
  for (int bpc = 1; bpc <= per_cu + 1; bpc++)
    for (int c = 0; c < (bpc <= per_cu ? 5 : 1); c++) {
      const int blocks = bpc <= per_cu ? bpc * cus : 0, chunk = bpc <= per_cu ? chunks[c] : 0;
      float total = 0.f;
      hipError_t e = hipSuccess;
      for (int rep = 0; rep < 3 && e == hipSuccess; rep++) {
        e = hipEventRecord(a, s);
        if (e == hipSuccess)
          e = partial_launch(p, parent_pts, n_parents, parent_cache, n_evals, eval_parent, eval_group,
                             new_coords, obj, flags, severity, counts, blocks, chunk, s);
        if (e == hipSuccess) e = hipEventRecord(b, s);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (rep > 0) total += ms;   // first repetition is a warm-up
      }
      if (e != hipSuccess) {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        return hip_fail(e, "tuning run");
      }
      if (total < best) {
        best = total;
        best_blocks = blocks;
        best_chunk = chunk;
      }
    }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  p->partial_blocks = best_blocks;
  p->partial_chunk = best_chunk;
  drop_graph(p);
  if (best_ms) *best_ms = best / 2.0f;
  return MOREA_OK;
}

morea_status morea_partial_graphs(const morea_problem* p, int32_t* cached, int64_t* captures) {
  if (!p || !cached || !captures) return fail(MOREA_EINVAL, "NULL argument");
  int n = 0;
  for (const auto& g : p->graphs) n += g.exec ? 1 : 0;
  *cached = n;
  *captures = static_cast<int64_t>(p->graph_captures);
  return MOREA_OK;
}

morea_status morea_set_partial_shape(morea_problem* p, int32_t blocks, int32_t chunk) {
  if (!p) return fail(MOREA_EINVAL, "NULL argument");
  const bool grid = blocks == 0 && chunk == 0;
  if (!grid && (blocks < 1 || chunk < 1 || chunk > 64)) return fail(MOREA_EINVAL, "bad launch shape");
  if (p->partial_blocks != blocks || p->partial_chunk != chunk) drop_graph(p);
  p->partial_blocks = blocks;
  p->partial_chunk = chunk;
  return MOREA_OK;
}

morea_status morea_partial_shape(const morea_problem* p, int32_t* blocks, int32_t* chunk) {
  if (!p || !blocks || !chunk) return fail(MOREA_EINVAL, "NULL argument");
  *blocks = p->partial_blocks;
  *chunk = p->partial_chunk;
  return MOREA_OK;
}

}  // extern "C"
