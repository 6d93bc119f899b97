// Internal types shared by the libmorea HIP sources.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/morea.h"

namespace morea {

constexpr int kFracBits = 10;                 // fixed-point snap: 2^-10 voxel
constexpr float kFixOne = 1024.0f;
constexpr float kCoordLimit = 512.0f;         // |x| < 512 voxels keeps every extent < 2^20
constexpr int kFastExtent = 1 << 16;          // tets up to 64 voxels: exact plane tests in FP64
constexpr int kMaxSets = 8;
constexpr int kWave = 64;

// Per-(candidate, tet, direction) partial objective record.  Direction 0
// rasterizes the source tet on I_s and samples I_t; direction 1 rasterizes
// the target tet on I_t and samples I_s.
struct Record {
  float h;        // sum of h over this tet's samples
  float g;        // set-weighted guidance sum
  uint32_t n;     // samples
  float mag;      // magnitude term of the tet (direction 0 only, else 0)
  float vol;      // |signed volume| (voxel^3) when the tet violates, else 0
  uint32_t bits;  // bit0: violation of this direction's mesh; bit2: invalid vertex
};
static_assert(sizeof(Record) == 24, "record layout");

// Per-candidate totals kept after the records in a cache (compensated
// double-float sums: value = hi + lo).
struct Totals {
  float h_hi, h_lo, g_hi, g_lo, m_hi, m_lo, v_hi, v_lo;
  uint32_t n[2];
  uint32_t viol[2];   // violating tets per mesh
  uint32_t bad;       // invalid coordinates of the candidate
  uint32_t pad[3];
};
static_assert(sizeof(Totals) == 64, "totals layout");

enum Store { kF32 = 0, kBF16 = 1, kF16 = 2 };

// Device view of a problem, passed by value to kernels.
//
// Every stored volume (images, distance maps, band masks) carries a border of
// at least one voxel on each side: padded dimensions (px, ny + 2, nz + 2) with
// the row length px = nx + 2 rounded up to even (so that every row and slice
// of a 2-byte volume starts 4-byte aligned), voxel (x, y, z) of the grid at
// element (z + 1) * pxy + (y + 1) * px + (x + 1).  Image borders hold 0 (the
// zero padding of the intensity term), distance map borders repeat the
// nearest grid value (edge clamping), so trilinear corners in [-1, n] per
// axis need no clamping.
__host__ __device__ inline int padded_row(int nx) { return (nx + 3) & ~1; }

struct ProblemView {
  int nx, ny, nz;
  int px, pxy;                   // padded row and slice strides: padded_row(nx), px (ny + 2)
  unsigned pvox;                 // padded voxels per volume
  int n_points, n_tets, n_sets;
  float radius, inv_radius;
  // every positive stored image value is >= 2^-40: then a sample whose
  // mapped point is not near a grid plane (trilinear weights >= 2^-22) has
  // b > 0 exactly when one of its 8 corners is > 0 (b >= 2^-106 stays normal)
  int fg_from_b;
  const void* img[2];            // [0] = I_s, [1] = I_t, storage type, padded
  const float* dmap[2];          // [n_sets][pvox] distance maps on each image grid, padded
  const uint8_t* band[2];        // [pvox] bit s set where dmap[s] < radius
  const float* set_w;            // [2][kMaxSets] |C_i| / |G| per direction (device memory)
  const int4* tets;
  const int8_t* ref_sign;
  const float* elasticity;
};

// Work item of one wave: candidate geometry source.
struct FullItems {
  const float* pts;   // [pop][2][3][n_points]
  int pop;
  double inv_pop;     // 1 / pop, for the item -> (tet, candidate) split
};

struct PartialItems {
  const float* parent_pts;     // [n_parents][2][3][n_points]
  const int* eval_parent;      // [n_evals]
  const int* eval_group;       // [n_evals]
  const float* new_coords;     // [rows][2][3]
  const int* row_off;          // [n_evals] first new-coordinate row of each evaluation
  const int* item_off;         // [n_evals + 1] prefix of dependent tets per evaluation
  const int* grp_off;          // [n_groups + 1] CSR into grp_pts
  const int* grp_pts;          // group points
  const int* dep_off;          // [n_groups + 1] CSR into dep_tet / dep_local
  const int* dep_tet;          // dependent tets per group
  const int8_t* dep_local;     // [.][4] position of each tet vertex in the group, -1 if none
  // items are processed group by group, dependent tet by dependent tet, the
  // group's evaluations innermost (neighbouring waves share a tet's image
  // region); a record still lands at item_off[e] + j
  int4* item_info;             // [items] in processing order: dependent-tet slot, tet, parent, first row
  int* item_dest;              // [items] in processing order: record index item_off[e] + j
  int* grp_count;              // [n_groups] evaluations of each group
  int* grp_base;               // [n_groups] first processing position of each group
  int* eval_rank;              // [n_evals] rank of each evaluation within its group
  int n_evals;
};

}  // namespace morea

struct morea_problem {
  int device = 0;
  morea::ProblemView view{};
  int storage = 0;
  int max_population = 0;
  size_t voxels = 0;
  std::vector<void*> allocations;
  std::vector<void*> group_allocs;
  std::vector<void*> partial_allocs;
  std::vector<int> tets_host;
  std::vector<float> ref_host;
  morea::Record* work_records = nullptr;   // [max_population][n_tets][2]
  // per image: at padded element i (the lower corner of a grid cell), the OR
  // of the band bits of the cell's 8 corners i + {0, 1} + {0, px} + {0, pxy}
  uint8_t* band_cell[2] = {nullptr, nullptr};
  // per image: at padded element i (the lower corner of a cell, i + {0, 1} +
  // {0, px} + {0, pxy}, for every cell of the padded volume), bit 0 set when
  // a corner holds a value > 0, bit 1 when all eight do
  uint8_t* fg_cell[2] = {nullptr, nullptr};
  // point -> incident tets (entries tet << 2 | slot) and point -> neighbours
  // (the other vertices of its incident tets, each once, ascending), CSR
  int* d_pinc_off = nullptr;
  int* d_pinc = nullptr;
  int* d_nb_off = nullptr;
  int* d_nb = nullptr;
  // guidance sets per image: CSR offsets [n_sets + 1] and snapped points [*][3]
  int* d_set_off[2] = {nullptr, nullptr};
  int* d_set_fix[2] = {nullptr, nullptr};
  morea::Totals* work_totals = nullptr;    // [max_population]
  // family of subsets
  int n_groups = 0;
  int max_group = 0;
  int* d_grp_off = nullptr;
  int* d_grp_pts = nullptr;
  int* d_dep_off = nullptr;
  int* d_dep_tet = nullptr;
  int8_t* d_dep_local = nullptr;
  int max_dep = 0;
  // partial workspace
  int max_evals = 0;
  int* d_row_off = nullptr;
  int* d_item_off = nullptr;
  morea::Record* d_partial_records = nullptr;  // [max_evals * max_dep][2]
  int4* d_item_info = nullptr;                 // [max_evals * max_dep]
  int* d_item_dest = nullptr;                  // [max_evals * max_dep]
  int* d_grp_count = nullptr;                  // [n_groups]
  int* d_grp_base = nullptr;                   // [n_groups]
  int* d_eval_rank = nullptr;                  // [max_evals]
  int* d_queue = nullptr;
  hipStream_t capture_stream = nullptr;
  // autotuned persistent launch shape
  int partial_blocks = 0;    // persistent blocks, or 0 with partial_chunk 0: the grid form
  int partial_chunk = -1;    // items per queue pop; -1 until a shape is chosen
  // captured partial-evaluation graphs, each with the arguments it bakes in;
  // a call whose arguments match an entry replays it, otherwise the least
  // recently used entry is replaced (a generation alternates one argument set
  // per colour)
  static constexpr int kGraphSlots = 8;
  struct GraphSlot {
    hipGraphExec_t exec = nullptr;
    const void* key[9] = {};
    int key_n[4] = {};
    uint64_t used = 0;   // call counter at the last replay
  };
  GraphSlot graphs[kGraphSlots];
  uint64_t graph_clock = 0;
  uint64_t graph_captures = 0;   // graphs captured so far (for tests)
  // arguments of the last launched partial evaluation, whose records and
  // offsets the workspace holds (the acceptance reads them)
  bool last_partial = false;
  const void* last_key[5] = {};
  int last_n[2] = {};
};

namespace morea {
// Kernel launchers (defined with the kernels).
hipError_t launch_distance_maps(int nx, int ny, int nz, int n_sets, const int* set_off,
                                const int* pts_fix, float radius, float* dmap, uint8_t* band,
                                hipStream_t s);
hipError_t launch_eval_full(const ProblemView& P, int storage, const float* pts, int pop,
                            Record* rec, hipStream_t s);
hipError_t launch_finalize(const ProblemView& P, const float* pts, int pop, const Record* rec,
                           float* obj, uint8_t* flags, float* severity, uint32_t* counts,
                           Totals* totals, hipStream_t s);
int partial_blocks_per_cu(int storage);
hipError_t launch_band_cells(const ProblemView& P, const uint8_t* band, uint8_t* cells, hipStream_t s);
hipError_t launch_fg_cells(const ProblemView& P, int storage, const void* img, uint8_t* cells, hipStream_t s);
void set_error(const char* msg);   // message returned by morea_last_error() on this thread
// device address of the allocation-free entry point's static scratch on the
// current device (looked up once per device)
morea_status static_scratch_init(int device);
void ensure_partial_shape(morea_problem* p);   // untuned persistent launch shape, once
hipError_t launch_partial(const ProblemView& P, int storage, const PartialItems& I, int n_parents,
                          int n_groups, const Record* parent_rec, const Totals* parent_tot,
                          Record* new_rec, int* queue, int blocks, int chunk, float* obj,
                          uint8_t* flags, float* severity, uint32_t* counts, hipStream_t s);
}  // namespace morea
