/*
 * libmorea -- batched evaluation of MOREA's registration objectives on one
 * AMD Instinct MI355X (gfx950).
 *
 * A candidate registration is a dual-dynamic tetrahedral mesh: two point sets
 * with one shared connectivity, S on the source image I_s and T on the target
 * image I_t (Sec. 4.2.1; the mesh is duplicated into the target space).  The
 * pair defines the piecewise-affine map T (source -> target) and its inverse
 * T' through barycentric coordinates, so every evaluation is symmetric
 * (Sec. 2.1, Sec. 4.1.2).  For each candidate the library returns
 *
 *   obj[0]  f_intensity  Sec. 4.1.2, equations for f_intensity and h
 *   obj[1]  f_magnitude  Sec. 4.1.1, equation for f_magnitude
 *   obj[2]  f_guidance   Sec. 4.1.3, equations for f_guidance and g, with the
 *                        distance-map form of App. A.3
 *   flags   fold constraint of Sec. 4.1.4 / App. A.4 (sign of every tet's
 *           signed volume against the sign in the initial mesh)
 *   severity  sum of |signed volume| of the violating tets (App. A.4)
 *   counts  |P_s| and |P_t|, the numbers of sample points
 *
 * Sample points are the voxel centres inside each tetrahedron (the voxel
 * association of App. A.2), found by an exact, watertight rasterization:
 * coordinates are snapped to 2^-10 voxel, and a centre that lies on a face
 * belongs to the tet that contains it after an infinitesimal move by
 * (e, e^2, e^3).  Every centre inside a fold-free mesh is therefore sampled
 * exactly once per direction.
 *
 * Coordinates are voxel index units: voxel (i, j, k) has its centre at
 * (i, j, k).  Images are [nz][ny][nx] with x fastest; both images share the
 * grid (the pair is cropped to a common box, Sec. 5.1).  Intensity 0 is
 * background and must be exactly 0; foreground is > 0.
 *
 * Conventions for every call:
 *   - status codes are returned synchronously for argument errors; errors of
 *     earlier asynchronous device work surface as MOREA_EDEVICE on a later
 *     call; morea_last_error() returns a message for the calling thread;
 *   - evaluation calls are asynchronous on the given stream (a hipStream_t,
 *     NULL for the default stream), perform no host synchronisation and no
 *     allocation; their pointer arguments are DEVICE pointers that the caller
 *     owns and keeps alive until the stream has completed the call;
 *   - a candidate with any coordinate that is not finite or has |x| >= 512
 *     voxels is invalid: flags bit 2, NaN objectives and severity, zero
 *     counts;
 *   - results are deterministic: the same inputs give bitwise-identical
 *     outputs (fixed reduction order, no floating-point atomics).
 */
#ifndef MOREA_H
#define MOREA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MOREA_OK = 0,
  MOREA_EINVAL = -1,  /* invalid argument (NULL pointer, bad size, bad index) */
  MOREA_ENOMEM = -2,  /* device allocation failed */
  MOREA_EDEVICE = -3, /* HIP runtime / kernel error */
  MOREA_ERANGE = -4,  /* size beyond what the problem was created for */
  MOREA_ESTATE = -5   /* call order violated (e.g. partial without groups) */
} morea_status;

typedef enum {
  MOREA_STORE_F32 = 0, /* images kept as FP32 */
  MOREA_STORE_BF16 = 1, /* images rounded (nearest, ties to even) to bfloat16 */
  MOREA_STORE_F16 = 2  /* images rounded (nearest, ties to even) to IEEE half */
} morea_store;

typedef struct morea_problem morea_problem; /* opaque; owns all device copies */

/* Problem description.  Every pointer is a HOST pointer; the library copies
 * what it needs during morea_problem_create and keeps no reference.  */
typedef struct {
  int32_t dims[3];              /* nx, ny, nz; each in [1, 1024], nx*ny*nz <= 2^29 */
  const float *image_src;       /* I_s, [nz][ny][nx], finite, >= 0 */
  const float *image_tgt;       /* I_t, same shape */
  int32_t storage;              /* morea_store */
  int32_t n_points;             /* points per mesh (4 .. 2^28) */
  int32_t n_tets;               /* tetrahedra (1 .. 2^28) */
  const int32_t *tets;          /* [n_tets][4] point indices */
  const float *ref_points;      /* [n_points][3] initial mesh: reference signs
                                   of App. A.4; no reference tet may be flat */
  const float *elasticity;      /* [n_tets] c_delta > 0 (Sec. 4.1.1, App. A.1) */
  int32_t n_sets;               /* guidance set pairs <C_s, C_t>, 0..8 */
  const int32_t *set_off_src;   /* CSR offsets [n_sets+1] into set_pts_src */
  const int32_t *set_off_tgt;   /* CSR offsets [n_sets+1] into set_pts_tgt */
  const float *set_pts_src;     /* [*][3] points of C_s (on I_s) */
  const float *set_pts_tgt;     /* [*][3] points of C_t (on I_t) */
  float radius;                 /* truncation radius r in voxels; <= 0 selects
                                   2.5% of the image width, 0.025 * nx (App. A.3) */
  int32_t max_population;       /* largest pop of morea_eval_full (workspace) */
} morea_problem_desc;

/* Validate the description, copy images (converted to the storage type),
 * mesh and guidance sets to the current device, and compute the distance
 * map d(p, C) of every guidance set at every voxel centre (App. A.3).
 * Blocks until the set-up work is complete.
 * Errors: MOREA_EINVAL (bad description), MOREA_ENOMEM, MOREA_EDEVICE. */
morea_status morea_problem_create(const morea_problem_desc *desc, morea_problem **out);

/* Free all device memory of the problem (synchronises the device first).
 * NULL is accepted. */
void morea_problem_destroy(morea_problem *p);

/* Bytes of a per-tetrahedron cache for `pop` candidates (App. A.2's partial
 * objective values per tet, kept so that partial evaluations can reuse
 * them, Sec. 4.2.1).  Layout: pop * n_tets * 2 records of 24 bytes,
 * candidate-major, then tet, then direction (0: the source tet rasterized on
 * I_s and mapped into I_t; 1: the target tet on I_t mapped into I_s), each
 *   float h      sum of the intensity term h over the tet's samples
 *   float g      set-weighted guidance sum (weights |C_i| / |G|)
 *   uint32 n     samples (voxel centres, or points of the sampled estimator)
 *   float mag    the tet's magnitude term c * sum (|e_S| - |e_T|)^2
 *                (direction 0; 0 in direction 1)
 *   float vol    |signed volume| (voxel^3) when the direction's tet violates
 *                its reference orientation, else 0
 *   uint32 bits  bit0 violation, bit2 a vertex of the tet has an invalid
 *                coordinate
 * followed by pop blocks of 64 bytes of per-candidate totals (internal). */
size_t morea_cache_bytes(const morea_problem *p, int32_t pop);

/* Full evaluation of `pop` candidates (Sec. 4.1).
 *   pts       [pop][2][3][n_points] FP32, mesh 0 = S, mesh 1 = T,
 *             coordinate-major (x row, y row, z row) per mesh
 *   obj       [pop][3]  intensity, magnitude, guidance (FP32)
 *   flags     [pop]     bit0 fold in S, bit1 fold in T, bit2 invalid
 *   severity  [pop]     sum of violating |signed volume|, voxel^3 (FP32)
 *   counts    [pop][2]  |P_s|, |P_t|
 *   cache     NULL, or morea_cache_bytes(p, pop) bytes of device memory that
 *             receives the per-tet records for later partial evaluations
 *   stream    hipStream_t or NULL
 * 0 <= pop <= max_population.  Errors: MOREA_EINVAL, MOREA_ERANGE,
 * MOREA_EDEVICE. */
morea_status morea_eval_full(morea_problem *p, const float *pts, int32_t pop, float *obj,
                             uint8_t *flags, float *severity, uint32_t *counts, void *cache,
                             void *stream);

/* Full evaluation with the paper's random-sampling estimator (App. A.2)
 * instead of voxel centres: each tet of each mesh is sampled at
 * N = floor(rate * |V| + 1/2) points (|V| its exact volume in voxel^3, at
 * most 2^20) spread uniformly through its barycentric coordinates,
 * lambda_j = -ln r_j / sum_k (-ln r_k) from four numbers r_j of a Sobol
 * sequence seeded from `seed`, the direction and the tet's fixed-point
 * coordinates (the same tet always gets the same points).  The point p in the
 * sampled tet and its image q in the other mesh's tet are formed in FP32 from
 * the same lambda; h (Sec. 4.1.2) compares the trilinear image values at p and
 * q (zero padding, foreground on each stencil's exact support) and the
 * guidance term (Sec. 4.1.3) the two distance maps (edge clamped) where the
 * own distance is below the radius.  Magnitude, flags and severity are those
 * of morea_eval_full; counts are the numbers of sample points.  Sequence:
 * 4-D Sobol, natural order, direction numbers of the primitive polynomials
 * 1, x + 1, x^2 + x + 1, x^3 + x + 1 (initial numbers (1), (1, 3),
 * (1, 3, 1)), digital shift by four 32-bit words of a SplitMix64 hash;
 * r_j = (2 floor(u_j / 2^9) + 1) 2^-24.  Arguments as morea_eval_full
 * (no cache); rate finite and > 0.  Errors: MOREA_EINVAL, MOREA_ERANGE,
 * MOREA_EDEVICE. */
morea_status morea_eval_sobol(morea_problem *p, const float *pts, int32_t pop, float rate, uint64_t seed,
                              float *obj, uint8_t *flags, float *severity, uint32_t *counts,
                              void *stream);

/* Fold repair (Sec. 4.3.1) of candidates, in place.  For each point of a
 * folded tet (App. A.4) -- the vertices of the tets folded when the call
 * starts, mesh S then mesh T, each ascending; a point no longer in a folded
 * tet when its turn comes is skipped -- 64 trial moves are tried, trial k of
 * the candidate's i-th visited point moving each free axis by
 * rint(sigma * draws[c][i][k][axis]) grid units of 2^-10 voxel (ties to even),
 * sigma the point's distance to the centroid of its neighbours (the other
 * vertices of its incident tets) rounded down to a power of two of grid units
 * (1 .. 2^18).  The constraint of the point is (folded incident tets, sum of
 * their |6V|), compared lexicographically; the trial with the smallest
 * (constraint, k) is applied when it is strictly below the point's constraint,
 * nothing changes when it is equal, and the candidate's repair stops when it
 * is above (every trial worse or out of the |x| < 512 voxel range).  Moved
 * coordinates are written as their grid values (exact FP32); all others keep
 * their input bits.
 *   pts     [pop][2][3][n_points] FP32, read and written
 *   draws   [pop][n_draws][64][3] FP32 standard normal draws (finite), one
 *           [64][3] block per visited point; at most n_draws points are
 *           visited per candidate
 *   pinned  [n_points] bit a set: axis a of the point never moves (e.g. the
 *           normal axis of boundary points), or NULL
 *   info    [pop][2] int32: moves applied, outcome (0 no fold at the start,
 *           1 every listed point visited, 2 stopped because every trial was
 *           worse, 3 n_draws used up, 4 invalid coordinates, left untouched)
 * n_points <= 6144 (a candidate is held in LDS).  Asynchronous on `stream`;
 * no allocation.  Errors: MOREA_EINVAL, MOREA_ERANGE, MOREA_EDEVICE. */
morea_status morea_repair_folds(morea_problem *p, float *pts, int32_t pop, const float *draws, int32_t n_draws,
                                const uint8_t *pinned, int32_t *info, void *stream);

/* Deformation vector fields of one candidate (Sec. 5.4: registrations are
 * compared through a forward DVF on the source grid and an inverse DVF on the
 * target grid; MOREA's are rasterized from its two meshes).  A voxel centre p
 * of a tet of the sampled mesh -- the centres of the evaluation, a centre on a
 * face belonging to the tet that holds p + (e, e^2, e^3) -- gets the
 * displacement q - p, q its barycentric image in the other mesh (computed in
 * FP64 from exact signed volumes, rounded once to FP32).  A centre covered by
 * several tets (a folded mesh) takes the tet of smallest index; one covered
 * by none gets 0; a tet with a vertex coordinate that is not finite or has
 * |x| >= 512 voxels is skipped.
 *   cand   [2][3][n_points] FP32, one candidate (layout of morea_eval_full)
 *   fwd    [nz][ny][nx][3] FP32 T(p) - p on the I_s grid
 *   inv    [nz][ny][nx][3] FP32 T'(y) - y on the I_t grid
 *   cover  [2][nz][ny][nx] tets containing each centre (source, target grid)
 *   work   [2][nz][ny][nx] int32 workspace (owner of each centre)
 * Asynchronous on `stream`; no allocation.  Errors: MOREA_EINVAL,
 * MOREA_EDEVICE. */
morea_status morea_rasterize_dvf(morea_problem *p, const float *cand, float *fwd, float *inv, uint32_t *cover,
                                 int32_t *work, void *stream);

/* The same DVF rasterization for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc): no workspace argument and no allocation; the owner of every
 * centre lives in a static 16 MiB device array of the library (one per GPU,
 * held until the process ends), so grids of at most 2,097,152 voxels.  Calls
 * on one GPU share that array: calls that overlap on one GPU (different
 * streams, threads) race.  Arguments and outputs as morea_rasterize_dvf.
 * Errors: MOREA_EINVAL, MOREA_ERANGE (grid above the limit), MOREA_EDEVICE. */
morea_status morea_rasterize_dvf_static(morea_problem *p, const float *cand, float *fwd, float *inv,
                                        uint32_t *cover, void *stream);

/* Point-based guidance error of `pop` candidates: the guidance measure of
 * the paper's prior work, which Sec. 4.1.3 replaces by the continuous form.
 * Every point c of the problem's C_s sets is located in the candidate's
 * source mesh (the tet that holds it under the tie rule of the evaluation,
 * the smallest index if several), mapped to the target mesh through its
 * barycentric coordinates, and its squared distance (voxel^2) to the nearest
 * point of the set's C_t taken; f[c] is the mean over all points of all sets
 * (each set weighted |C_i| / |G|), NaN for an invalid candidate or when no
 * point is located; unmapped[c] counts the points in no tet.
 *   pts       [pop][2][3][n_points] FP32 (layout of morea_eval_full)
 *   f         [pop] FP32
 *   unmapped  [pop] int32
 * n_points <= 6144 (a candidate is held in LDS).  Asynchronous on `stream`;
 * no allocation.  Errors: MOREA_EINVAL, MOREA_ERANGE, MOREA_EDEVICE. */
morea_status morea_point_guidance(morea_problem *p, const float *pts, int32_t pop, float *f, int32_t *unmapped,
                                  void *stream);

/* Linkage model of the optimizer's parallel variation (Sec. 4.2.1): the mesh
 * edges are the FOS elements; a greedy set cover (the edge covering the most
 * uncovered points, ties to the lexicographically smallest (a, b), a < b)
 * keeps edges until every point of a tet is covered; two elements interact
 * when their dependent tets (those holding one of their points) overlap;
 * DSATUR colours the interaction graph (largest saturation, then degree, then
 * smaller index; smallest free colour), so the elements of one colour can be
 * varied and evaluated in parallel -- e.g. registered with morea_set_groups
 * and evaluated for every (solution, element of the colour) pair in one
 * morea_eval_partial call.  Host code; all pointers are HOST pointers.
 *   tets       [n_tets][4] point indices in [0, n_points)
 *   elem_pts   [capacity][2] receives the elements (a < b), in cover order
 *   color      [capacity] receives each element's colour
 *   n_elements, n_colors  receive the counts
 * Errors: MOREA_EINVAL, MOREA_ERANGE (more elements than capacity; at most
 * n_points are needed). */
morea_status morea_build_fos(int32_t n_points, int32_t n_tets, const int32_t *tets, int32_t capacity,
                             int32_t *elem_pts, int32_t *color, int32_t *n_elements, int32_t *n_colors);

/* Register the family of subsets: n_groups point groups in CSR form (host
 * pointers).  For every group the library builds the list of dependent
 * tetrahedra, those with at least one vertex in the group (Sec. 4.2.1), and
 * the position of each of their vertices in the group.  A group may not repeat
 * a point.  Synchronous.  Errors: MOREA_EINVAL, MOREA_ENOMEM, MOREA_EDEVICE. */
morea_status morea_set_groups(morea_problem *p, int32_t n_groups, const int32_t *grp_off,
                              const int32_t *grp_pts);

/* Maximum number of evaluations that one morea_eval_partial call accepts;
 * allocates the partial-evaluation workspace (per-item records for
 * max_evals times the largest dependent-tet list).  Call after every
 * morea_set_groups.  Synchronous.  Errors: MOREA_ESTATE, MOREA_EINVAL,
 * MOREA_ENOMEM, MOREA_EDEVICE. */
morea_status morea_reserve_partial(morea_problem *p, int32_t max_evals);

/* Partial evaluation (Sec. 3 optimal mixing; Sec. 4.2.1 dependent
 * tetrahedra): evaluation e is the candidate parent_pts[eval_parent[e]] with
 * the points of group eval_group[e] moved to new coordinates.  Only the
 * dependent tets of the group are evaluated; all others come from the
 * parent's cache (written by morea_eval_full with the same parent_pts).  The
 * results equal a full evaluation of the child up to FP32 rounding; counts,
 * flags and invalidity are exact.
 *   parent_pts    [n_parents][2][3][n_points]
 *   parent_cache  cache of morea_eval_full for parent_pts
 *   eval_parent   [n_evals] in [0, n_parents)
 *   eval_group    [n_evals] in [0, n_groups)
 *   new_coords    [sum over e of |group e|][2][3]: group points in group order,
 *                 evaluations in order; [k][m][a] = mesh m, axis a (an
 *                 evaluation whose group index is out of range owns no rows)
 *   obj, flags, severity, counts: [n_evals] as in morea_eval_full
 * All arrays are device pointers.  The three kernels of a call (list prefix
 * sums, one persistent launch that takes (evaluation, dependent tet,
 * direction) items from a device work queue, and the per-evaluation
 * reduction) are captured into a HIP graph and replayed while the pointer
 * arguments and sizes match one of the last 8 argument sets (see
 * morea_partial_graphs); other calls capture a new graph.  Out-of-range eval_parent / eval_group entries give
 * that evaluation flags bit 2 and NaN objectives.  The evaluation list is
 * staged through a library-owned device workspace, so calls on one problem
 * must not overlap (use one stream per problem).  Errors: MOREA_ESTATE (no groups or no
 * reservation), MOREA_ERANGE (n_evals or rows beyond the reservation),
 * MOREA_EINVAL, MOREA_EDEVICE. */
morea_status morea_eval_partial(morea_problem *p, const float *parent_pts, int32_t n_parents,
                                const void *parent_cache, int32_t n_evals,
                                const int32_t *eval_parent, const int32_t *eval_group,
                                const float *new_coords, float *obj, uint8_t *flags,
                                float *severity, uint32_t *counts, void *stream);

/* Acceptance of the evaluated partial solutions (Sec. 3 optimal mixing): a
 * child (parent with its group's points moved) is kept when it dominates its
 * parent or is not dominated within the elitist archive; kept children are
 * written into their parents.  All three objectives are minimised.
 *   domination child vs parent: constraint domination -- a feasible solution
 *     (flags & 7 == 0) beats an infeasible one; two infeasible ones compare
 *     their violation (severity; +inf with flags bit 2 or an objective or
 *     severity that is not finite), the strictly smaller wins; two feasible
 *     ones compare by Pareto domination (no objective worse, one strictly
 *     better);
 *   archive: feasible objective vectors; a feasible child is non-dominated
 *     when no member Pareto-dominates it (a member equal to it does not);
 *   an evaluation with an out-of-range parent or group is rejected;
 *   adaptive steering (Sec. 4.3.2): with a finite guidance_max (the caller
 *     passes 1.5 times the best guidance value in the archive) a solution
 *     whose guidance objective exceeds it is infeasible too, and violations
 *     compare lexicographically as (severity of folds, FP32 excess
 *     guidance - guidance_max); INFINITY switches steering off.
 * For every kept evaluation e the group's new coordinates are written into
 * parent_pts[eval_parent[e]] and the partial evaluation's records of the
 * group's dependent tets into the parent's cache; then the totals in the
 * cache and the parents' obj / flags / severity / counts are recomputed from
 * the cached records of every parent (as morea_eval_full reports them).
 *   parent_pts, n_parents, parent_cache, n_evals, eval_parent, eval_group,
 *   new_coords   exactly the arguments (and contents) of the preceding
 *                morea_eval_partial on this problem, whose records are read
 *                from the library's workspace (MOREA_ESTATE otherwise, or
 *                after morea_tune_partial / morea_set_groups /
 *                morea_reserve_partial); parent_cache 16-byte aligned
 *   child_obj, child_flags, child_sev   [n_evals] decision inputs, normally
 *                the outputs of that call (layout of morea_eval_full)
 *   parent_obj, parent_flags, parent_sev, parent_counts   [n_parents] the
 *                parents' evaluation: read for the decisions, rewritten
 *   archive_obj  [n_archive][3] FP32 (NULL when n_archive == 0)
 *   guidance_max steering bound, or INFINITY (not NaN)
 *   accepted     [n_evals] receives 1 (kept) or 0
 * The kept evaluations of one parent must have pairwise disjoint dependent
 * tets (e.g. the elements of one colour of morea_build_fos); otherwise which
 * child's values a shared tet or point keeps is unspecified (every write
 * still stays inside the parent's arrays).  All arrays are device pointers;
 * asynchronous on `stream`; no allocation.  Errors: MOREA_EINVAL,
 * MOREA_ESTATE, MOREA_EDEVICE. */
morea_status morea_accept_partial(morea_problem *p, float *parent_pts, int32_t n_parents, void *parent_cache,
                                  int32_t n_evals, const int32_t *eval_parent, const int32_t *eval_group,
                                  const float *new_coords, const float *child_obj, const uint8_t *child_flags,
                                  const float *child_sev, float *parent_obj, uint8_t *parent_flags,
                                  float *parent_sev, uint32_t *parent_counts, const float *archive_obj,
                                  int32_t n_archive, float guidance_max, uint8_t *accepted, void *stream);

/* Selection and clustering at the start of a generation (Sec. 3: a
 * selection of non-dominated solutions of the population, clustered into k
 * equally sized clusters).  Solutions are ordered by the constraint
 * domination of morea_accept_partial (with the same steering bound); fronts
 * by peeling; the selection takes whole fronts in order and the last one it
 * needs in ascending index, up to `size` solutions (invalid ones -- flags
 * bit 2, or an objective or severity that is not finite -- never).
 * Objectives are normalised over the selection ((v - lo) / (hi - lo), 0 where
 * hi == lo) and compared by squared Euclidean distance in FP64.  Leaders: the
 * selected solution with the smallest normalised first objective, then
 * repeatedly the one farthest from the leaders so far (ties to the lower
 * index), min(k, |S|) of them.  Cluster j holds the m = min(|S|,
 * ceil(2 |S| / k)) selected solutions nearest to leader j (ties to the lower
 * index) in ascending index; clusters without a leader are empty.  Every
 * valid solution is assigned the cluster of its nearest leader (ties to the
 * lower cluster), an invalid one -1.
 *   obj, flags, severity   [n_pop] (layout of morea_eval_full)
 *   selection    [n_pop] receives the selected indices, ascending
 *   n_selected   [1] receives |S|
 *   clu_off      [k + 1] receives CSR offsets into clu_members
 *   clu_members  [members_cap] receives the clusters' members
 *   cluster_of   [n_pop] receives each solution's cluster or -1
 * The outputs feed morea_estimate_distributions (clu_off, clu_members with
 * n_members = members_cap) and morea_sample_partial (cluster_of gathered per
 * evaluation).  n_pop <= 1024 (one block); members_cap >= k * ceil(2 min(size,
 * n_pop) / k).  All arrays are device pointers; asynchronous on `stream`; no
 * allocation.  Errors: MOREA_EINVAL, MOREA_ERANGE, MOREA_EDEVICE. */
morea_status morea_select_clusters(const float *obj, const uint8_t *flags, const float *severity, int32_t n_pop,
                                   int32_t size, int32_t k, float guidance_max, int32_t *selection,
                                   int32_t *n_selected, int32_t *clu_off, int32_t *clu_members, int32_t members_cap,
                                   int32_t *cluster_of, void *stream);

/* Elitist archive (Sec. 3: non-dominated solutions kept across generations
 * in an archive of fixed capacity, 2000 in App. C; Sec. 4.3.2: with adaptive
 * steering only guidance values up to 1.5 times the archive's best are kept).
 * The archive is caller-owned device memory of `capacity` slots:
 *   arc_obj    [capacity][3] FP32 objective vectors; a free slot holds
 *              (inf, inf, inf), which dominates nothing, so the slot array
 *              can be passed whole as morea_accept_partial's archive
 *   arc_stamp  [capacity] insertion stamps (order of the members), -1 free
 *   arc_pts    [capacity][2][3][n_points] FP32 members' points, or NULL
 *   arc_state  [4] int32: members, next stamp, boxes per objective of the
 *              last thinning (0: none), 0
 *   best_guidance [1] FP32: the members' smallest guidance value (inf when
 *              empty); the next generation's steering bound is 1.5 times it
 * morea_archive_clear empties it (kernels only: no memset, so a captured
 * graph may hold it).  1 <= capacity <= 4096.  Errors: MOREA_EINVAL,
 * MOREA_EDEVICE. */
morea_status morea_archive_clear(int32_t capacity, float *arc_obj, int32_t *arc_stamp, int32_t *arc_state,
                                 float *best_guidance, void *stream);

/* Archive update with a batch of offered solutions (the population after a
 * batch of acceptances).  The candidates are the members in stamp order, then
 * the feasible offers (flags == 0, finite objectives and severity) in index
 * order, less those whose guidance value is above guidance_max (the steering
 * bound, inf when off: members above it are purged); a candidate stays unless
 * another Pareto-dominates it or an earlier one has the same objective vector.
 * If more than `capacity` stay, the objective range of the stayers is cut
 * into L boxes per objective (FP64: min(L - 1, floor((v - lo) / (hi - lo) *
 * L)), 0 where hi == lo), L found by binary search over [1, min(capacity,
 * 1024)] for at most `capacity` occupied boxes, and each box keeps its
 * earliest candidate.  Members that do not stay free their slots; staying
 * offers take the free slots in ascending order with the next stamps.
 *   offer_obj, offer_flags, offer_sev   [n_offers] (layout of morea_eval_full)
 *   offer_pts  [n_offers][2][3][n_points] or NULL (then arc_pts NULL too)
 *   inserted   [n_offers] receives 1 for offers that entered, else 0
 *   slot_of    [n_offers] receives the slot of an entered offer, else -1
 * 0 <= n_offers <= 1024, capacity + n_offers <= 4096.  All arrays are device
 * pointers; asynchronous on `stream` (one block); no allocation.  Errors:
 * MOREA_EINVAL, MOREA_ERANGE, MOREA_EDEVICE. */
morea_status morea_archive_update(int32_t n_offers, const float *offer_obj, const uint8_t *offer_flags,
                                  const float *offer_sev, const float *offer_pts, int32_t n_points,
                                  float guidance_max, int32_t capacity, float *arc_obj, int32_t *arc_stamp,
                                  float *arc_pts, int32_t *arc_state, float *best_guidance, uint8_t *inserted,
                                  int32_t *slot_of, void *stream);

/* Improvements of a batch for the distribution multipliers (MO-RV-GOMEA's
 * adaptive variance scaling, to which Sec. 3 defers): improved[c][g] is set
 * to 1 for every kept child (accepted[e] != 0) of cluster eval_cluster[e] and
 * element eval_group[e] whose parent entered the archive in the batch's
 * update (parent_inserted[eval_parent[e]] != 0); out-of-range indices are
 * skipped.  Device pointers; asynchronous on `stream`.  Errors:
 * MOREA_EINVAL, MOREA_EDEVICE. */
morea_status morea_mark_improvements(int32_t n_evals, const int32_t *eval_parent, const int32_t *eval_group,
                                     const int32_t *eval_cluster, const uint8_t *accepted, int32_t n_parents,
                                     const uint8_t *parent_inserted, int32_t n_clusters, int32_t n_groups,
                                     uint8_t *improved, void *stream);

/* End-of-generation adaptation of the multipliers mult [n_clusters][n_groups]
 * (FP32, morea_sample_partial's `mult`) with no-improvement stretches
 * [n_clusters][n_groups] int32: improved -> stretch 0, c = min(max(c, 1) /
 * 0.9, 10); otherwise the stretch grows while c <= 1, c = 0.9 c when c > 1 or
 * the stretch has reached 25, and a c below 1 with a shorter stretch is reset
 * to 1.  The marks are cleared.  Device pointers; asynchronous on `stream`.
 * Errors: MOREA_EINVAL, MOREA_EDEVICE. */
morea_status morea_adapt_multipliers(int32_t n_clusters, int32_t n_groups, uint8_t *improved, float *mult,
                                     int32_t *no_improvement, void *stream);

/* Bytes of the caller-owned workspace of the optimal-mixing distributions
 * for n_clusters clusters of the registered groups (one record per
 * (cluster, group) plus the row offsets of the reserved evaluations); 0 before
 * morea_set_groups / morea_reserve_partial. */
size_t morea_mixing_bytes(const morea_problem *p, int32_t n_clusters);

/* Distributions of optimal mixing (Sec. 3): for every registered group g and
 * cluster c, a normal distribution over the group's free variables estimated
 * from the cluster's members.  Variable (2 k + m) 3 + a is axis a of mesh m
 * of the group's k-th point (the row layout of morea_eval_partial's
 * new_coords); an axis whose bit is set in pinned[point] is no variable.
 * Mean and covariance are the maximum-likelihood estimates (sums over the
 * members in the given order, divided by m), the factor is Cholesky (each
 * entry's sum in ascending index order) in FP64; a pivot not above 1e-12
 * times its diagonal entry makes the distribution fall back to the diagonal
 * (standard deviations).  A cluster with no members, or with a member outside
 * [0, n_pop) or offsets outside [0, n_members], has no distribution.
 *   pts          [n_pop][2][3][n_points] FP32, the selection's snapshot
 *   clu_off      [n_clusters + 1] CSR offsets into clu_members
 *   clu_members  [n_members] indices into pts
 *   pinned       [n_points] bit a: axis a fixed, or NULL
 *   work         morea_mixing_bytes(p, n_clusters) bytes, 16-byte aligned;
 *                receives the distributions, read by morea_sample_partial
 * Groups of at most 4 points (MOREA_ERANGE otherwise).  All arrays are device
 * pointers; asynchronous on `stream`; no allocation.  Errors: MOREA_EINVAL,
 * MOREA_ESTATE, MOREA_ERANGE, MOREA_EDEVICE. */
morea_status morea_estimate_distributions(morea_problem *p, const float *pts, int32_t n_pop, int32_t n_clusters,
                                          const int32_t *clu_off, const int32_t *clu_members, int32_t n_members,
                                          const uint8_t *pinned, void *work, size_t work_bytes, void *stream);

/* New partial solutions sampled from the distributions of the preceding
 * morea_estimate_distributions (Sec. 3): evaluation e draws the free
 * variables of group eval_group[e] from cluster eval_cluster[e]'s
 * distribution, x = mean + sqrt(mult[c][g]) (L z) in FP64, rounded once to
 * FP32; pinned variables keep parent eval_parent[e]'s values.  Evaluations
 * with a valid group own |group| rows of new_coords in evaluation order (the
 * layout morea_eval_partial reads); an out-of-range parent or cluster, or a
 * cluster without a distribution, gives NaN for the sampled rows.
 *   pts          [n_pop][2][3][n_points] FP32, the parents
 *   work         the workspace of morea_estimate_distributions (the same
 *                n_clusters); its tail receives the evaluations' row offsets
 *   mult         [n_clusters][n_groups] FP32 distribution multipliers, or
 *                NULL (1)
 *   eval_parent, eval_group, eval_cluster   [n_evals]
 *   z            [rows][2][3] FP32 standard normal draws (row layout of
 *                new_coords; entries of pinned variables are not read)
 *   pinned       as for the estimation
 *   new_coords   [rows][2][3] FP32 output
 * n_evals <= the reservation of morea_reserve_partial.  All arrays are device
 * pointers; asynchronous on `stream`; no allocation.  Errors: MOREA_EINVAL,
 * MOREA_ESTATE, MOREA_ERANGE, MOREA_EDEVICE. */
morea_status morea_sample_partial(morea_problem *p, const float *pts, int32_t n_pop, void *work, size_t work_bytes,
                                  int32_t n_clusters, const float *mult, int32_t n_evals, const int32_t *eval_parent,
                                  const int32_t *eval_group, const int32_t *eval_cluster, const float *z,
                                  const uint8_t *pinned, float *new_coords, void *stream);

/* Copy the distance map d(p, C) of guidance set `set` on image `image`
 * (0 = I_s grid with C_s, 1 = I_t grid with C_t) to host memory `host_out`
 * ([nz][ny][nx] FP32), and, when `band_out` is not NULL, the per-voxel band
 * mask (bit s set where map s < r) of that image.  Synchronous; for
 * verification of the set-up (App. A.3).  Errors: MOREA_EINVAL, MOREA_EDEVICE. */
morea_status morea_debug_distance_map(morea_problem *p, int32_t image, int32_t set, float *host_out,
                                      uint8_t *band_out);

/* Autotuner of the partial-evaluation launch: with the same arguments as
 * morea_eval_partial, times every launch shape (persistent blocks per compute
 * unit up to the occupancy limit x work items taken per queue pop in
 * {1, 2, 4, 8, 16}, and the grid form: one wave per two items over a grid
 * that covers n_evals x the largest dependent-tet count of a group, the
 * waves beyond the actual item count returning at once) on the given inputs
 * with HIP events and keeps the fastest for later morea_eval_partial calls.
 * Synchronous; overwrites the output arrays.  *best_ms (may be NULL) receives
 * the best time.  Untuned, the shape is 4 persistent blocks per compute unit
 * (at most the occupancy limit) and 8 items per pop.  Errors as
 * morea_eval_partial. */
morea_status morea_tune_partial(morea_problem *p, const float *parent_pts, int32_t n_parents,
                                const void *parent_cache, int32_t n_evals,
                                const int32_t *eval_parent, const int32_t *eval_group,
                                const float *new_coords, float *obj, uint8_t *flags,
                                float *severity, uint32_t *counts, void *stream, float *best_ms);

/* Current launch shape of partial evaluation: persistent blocks of 256
 * threads and items per queue pop, or *chunk = 0 (and *blocks = 0) for the
 * grid form.  Errors: MOREA_EINVAL. */
morea_status morea_partial_shape(const morea_problem *p, int32_t *blocks, int32_t *chunk);

/* Set the launch shape of partial evaluation (as morea_tune_partial would):
 * blocks >= 1 persistent blocks and 1 <= chunk <= 64 items per queue pop, or
 * blocks = chunk = 0 for the grid form.  Errors: MOREA_EINVAL. */
morea_status morea_set_partial_shape(morea_problem *p, int32_t blocks, int32_t chunk);

/* Graph cache of morea_eval_partial: up to 8 captured graphs are kept, one
 * per argument set (pointers, sizes, launch shape); a call that matches one
 * replays it, any other captures a new graph in place of the least recently
 * used.  *cached receives the graphs held, *captures the graphs captured
 * since the problem was created.  Errors: MOREA_EINVAL. */
morea_status morea_partial_graphs(const morea_problem *p, int32_t *cached, int64_t *captures);

/* ------------------------------------------------------------------------
 * Learned pre-screen of offspring.  A per-tetrahedron multilayer perceptron
 * 23 -> 128 -> 128 -> 1 (ReLU) predicts the change of a tet's mean intensity
 * term (the sum of h, Sec. 4.1.2, over the tet's samples in both directions
 * divided by their number) from an offspring's parent, whose exact
 * evaluation is known, to the offspring, in units of h_scale, the mean of
 * (I_s - I_t)^2 over the grid's voxels (1 when that is 0).  Inputs per
 * (offspring, tet), in order:
 *   0..11  the moves of the tet's 4 target-mesh vertices from the parent's,
 *          (T_v - T_parent,v) / 0.5 voxel, vertex-major;
 *   12..14 three cheap estimates of the change: the mean of
 *          h = (I_s(x) - I_t(y))^2 over a fixed point set of the tet (x, y
 *          at the same barycentric coordinates in the source and target
 *          tets) in the offspring minus that in the parent, over the 4
 *          vertices, the 6 edge midpoints, and 16 interior points (Halton
 *          points j = 1..16 in bases 2, 3, 5, each sorted into a <= b <= c
 *          and taken as barycentric coordinates (a, b - a, c - b, 1 - c));
 *          divided by h_scale;
 *   15..21 statistics of the tet's region in the reference mesh: mean, std
 *          and foreground fraction of I_s and of I_t over its voxels, and
 *          their mean squared difference divided by h_scale;
 *   22     the parent's exact mean term of the tet, (h_S + h_T) / (n_S + n_T)
 *          from its cache records (0 without samples), divided by h_scale.
 * Image values are trilinear interpolants at the point clamped into
 * [0, n - 1] per axis, in the cell below it capped at n - 2.  An offspring's
 * score is sum_tet w_tet (parent term + h_scale prediction) / sum_tet w_tet
 * with w_tet the offspring's |volume| of the tet's source plus that of its
 * target (voxel^3: the samples the tet contributes in the two directions), a
 * predicted f_intensity; the best-scoring offspring are then evaluated
 * exactly.  Dense
 * layers run on the matrix cores with BF16 operands and FP32 accumulation;
 * master weights, gradients and Adam state are FP32.  The surrogate is an
 * addition of this library; the paper has no counterpart.  Parameters are
 * one FP32 vector: W1 [128][23], b1 [128], W2 [128][128], b2 [128],
 * w3 [128], b3 [1] (19,713 values).
 * All array arguments are device pointers unless named host_*; calls with a
 * stream are asynchronous on it. */
typedef struct morea_surrogate morea_surrogate;

int32_t morea_surrogate_num_params(void);     /* 19,713 */
int32_t morea_surrogate_num_features(void);   /* 23 inputs per row */

/* Create a surrogate for problem p (which must outlive it): He-normal
 * weights from `seed`, zero Adam state, the per-tet statistics of the
 * reference mesh, h_scale, FP32 copies of I_s and I_t (whatever the
 * problem's image storage; 16 bytes per padded voxel, the four voxels of a
 * cell face read by one aligned load), and a training workspace for batches of up to max_rows rows.
 * Synchronous.  Errors: MOREA_EINVAL, MOREA_ENOMEM, MOREA_EDEVICE. */
morea_status morea_surrogate_create(morea_problem *p, int32_t max_rows, uint64_t seed,
                                    morea_surrogate **out);
void morea_surrogate_destroy(morea_surrogate *s);

/* Input rows of every (offspring, tet): feats [pop][n_tets][23] FP32.
 *   pts           [pop][2][3][n_points] the offspring
 *   parent_pts    [n_parents][2][3][n_points] their parents
 *   parent_cache  the parents' cache (morea_eval_full of parent_pts)
 *   parent_of     [pop] int32 parent of each offspring; an index outside
 *                 [0, n_parents) gives a row of NaN */
morea_status morea_surrogate_features(morea_surrogate *s, const float *pts, int32_t pop, const float *parent_pts,
                                      int32_t n_parents, const void *parent_cache, const int32_t *parent_of,
                                      float *feats, void *stream);

/* Training targets of `pop` offspring: targets [pop][n_tets] FP32, the
 * offspring's mean term of each tet minus its parent's (a term is 0 for a tet
 * without samples), divided by h_scale; NaN for an offspring whose parent_of
 * is outside [0, n_parents).
 *   cache         the offspring's cache (morea_eval_full)
 *   parent_cache  the parents' cache (morea_eval_full), n_parents of them
 *   parent_of     [pop] int32 */
morea_status morea_surrogate_targets(morea_surrogate *s, const void *cache, int32_t pop, const void *parent_cache,
                                     int32_t n_parents, const int32_t *parent_of, float *targets, void *stream);

/* One Adam step (beta 0.9 / 0.999, eps 1e-8) on the mean squared error of
 * n_rows <= max_rows rows; *loss_out (device, may be NULL) receives the loss
 * before the step.  Errors: MOREA_EINVAL, MOREA_ERANGE, MOREA_EDEVICE. */
morea_status morea_surrogate_train_step(morea_surrogate *s, const float *feats,
                                        const float *targets, int32_t n_rows, float lr,
                                        float *loss_out, void *stream);

/* Gradient of that loss without an update: grads [19,713] FP32 (device). */
morea_status morea_surrogate_gradients(morea_surrogate *s, const float *feats,
                                       const float *targets, int32_t n_rows, float *grads,
                                       float *loss_out, void *stream);

/* Predictions pred [n_rows] for explicit input rows. */
morea_status morea_surrogate_predict_rows(morea_surrogate *s, const float *feats, int32_t n_rows,
                                          float *pred, void *stream);

/* Pre-screen: score [pop] of offspring pts [pop][2][3][n_points] with their
 * parents as for morea_surrogate_features (features built on the fly: one
 * launch for the parents' point means, one for the offspring); an offspring
 * without a valid parent scores +inf.  The parents' point means go to a
 * workspace of the surrogate (16 bytes per (parent, tet)), allocated again
 * (hipMalloc, after waiting for the device) when a call needs more than
 * every earlier one; calls on one surrogate that overlap on different
 * streams race on it. */
morea_status morea_surrogate_prescreen(morea_surrogate *s, const float *pts, int32_t pop, const float *parent_pts,
                                       int32_t n_parents, const void *parent_cache, const int32_t *parent_of,
                                       float *score, void *stream);

/* Indices of the k lowest scores (ties: lower index first) into idx_out [k],
 * 1 <= k <= n <= 8192; when pts and selected_pts are not NULL the selected
 * candidates are copied to selected_pts [k][2][3][n_points] in that order. */
morea_status morea_surrogate_select(const float *score, int32_t n, int32_t k, const float *pts,
                                    int32_t n_points, int32_t *idx_out, float *selected_pts,
                                    void *stream);

/* Copy the FP32 parameter vector out / in (host arrays of 19,713 floats;
 * checkpoints).  Synchronous. */
morea_status morea_surrogate_get_params(morea_surrogate *s, float *host_params);
morea_status morea_surrogate_set_params(morea_surrogate *s, const float *host_params);

/* h_scale of the surrogate's problem into *h_scale (host). */
morea_status morea_surrogate_scale(const morea_surrogate *s, float *h_scale);

/* The per-tet statistics host_stats [n_tets][8] and reference voxel counts
 * host_counts [n_tets] (may be NULL).  Synchronous. */
morea_status morea_surrogate_stats(morea_surrogate *s, float *host_stats, int32_t *host_counts);

/* Message for the last non-OK status returned on the calling thread. */
const char *morea_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MOREA_H */
