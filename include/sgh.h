/*
 * sgh.h -- C ABI of a gfx950 (AMD Instinct MI355X) library that hierarchizes
 * the combination grids of the sparse grid combination technique, after
 * P. Hupp, "Hierarchization for the Sparse Grid Combination Technique",
 * arXiv:1309.0392.
 *
 * Grid model (paper, Section 2, "The Combination Technique"): a combination
 * grid is completely described by its level vector l = (l_0, ..., l_{d-1});
 * level 1 is a single point, so axis k holds n_k = 2^{l_k} - 1 interior
 * points.  Boundary values are zero and are not stored.  Storage is dense and
 * row major with axis 0 (the paper's x_1) changing fastest (Section 3,
 * "Unrolling and Vectorization"): the point with 1-based positions
 * (p_0, ..., p_{d-1}) is element  sum_k (p_k - 1) * S_k,  S_k = prod_{j<k} n_j.
 *
 * All entry points are plain C: host pointers to descriptors, device pointers
 * to grid data, a HIP stream passed as void* (NULL = the default stream).
 * The caller owns every grid buffer; the library never allocates or frees
 * caller data.  The library owns plans, their graphs, device task lists and
 * tuning state.
 *
 * Errors: every call returns SGH_OK (0) or a negative SGH_ERR_* code.  All
 * descriptors of a call are validated on the host before anything is
 * launched (all or nothing: on a validation error no kernel runs and no data
 * is touched).  sgh_last_error_message() gives a human-readable detail for
 * the calling thread's last failure.  Device faults surface, as in HIP, at
 * the next synchronization of the stream.
 *
 * Concurrency: grids of one call must not overlap in memory (SGH_ERR_OVERLAP).
 * Calls are asynchronous with respect to the host and ordered on `stream`.
 */
#ifndef SGH_H
#define SGH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SGH_MAX_DIM 16   /* the paper's experiments go up to d = 10 (Section 4, Fig. 8) */
#define SGH_MAX_LEVEL 30 /* per axis; positions fit in int32 */

/* element types of grid data */
#define SGH_F32 0
#define SGH_F64 1

/* operations */
#define SGH_OP_HIERARCHIZE 0   /* nodal -> hierarchical surpluses (Algorithm 1) */
#define SGH_OP_DEHIERARCHIZE 1 /* hierarchical -> nodal (its exact inverse) */
#define SGH_OP_ADJOINT 2       /* transpose of the hierarchization map */

/* return codes */
#define SGH_OK 0
#define SGH_ERR_ARG (-1)         /* null pointer, bad dim/level/op, size overflow */
#define SGH_ERR_DTYPE (-2)       /* dtype is neither SGH_F32 nor SGH_F64 */
#define SGH_ERR_ALIGN (-3)       /* data not aligned to its element size */
#define SGH_ERR_OVERLAP (-4)     /* two grids of one call share memory */
#define SGH_ERR_HIP (-5)         /* a HIP runtime call or kernel launch failed */
#define SGH_ERR_NOMEM (-6)       /* the library could not allocate its own state */
#define SGH_ERR_UNSUPPORTED (-7) /* valid request that this build does not handle */

/* Grid descriptor.  level[k] for k >= dim is ignored.  data is a device
 * pointer to prod_k (2^{level[k]} - 1) elements of the given dtype. */
typedef struct sgh_grid {
    int32_t dim;                 /* 1 .. SGH_MAX_DIM */
    int32_t level[SGH_MAX_DIM];  /* 1 .. SGH_MAX_LEVEL */
    int32_t dtype;               /* SGH_F32 or SGH_F64 */
    void *data;                  /* device pointer, aligned to the element size */
} sgh_grid;

/* ---- one-shot transforms (in place) -------------------------------------
 *
 * sgh_hierarchize: Algorithm 1 (Section 3).  Along every axis k, each point
 * turns into its hierarchical surplus: its nodal value minus half of each of
 * its two hierarchical predecessors (the nearest coarser points to its left
 * and right in the binary-tree picture of Fig. 3), all read as nodal values,
 * with zero for a predecessor on the boundary.  Axes commute.
 *
 * sgh_dehierarchize: the inverse base change back to the nodal basis, used
 * after the scatter step of the iterated combination technique (Section 2,
 * Fig. 2): levels coarse to fine, each point adds half of its (already nodal)
 * predecessors.
 *
 * sgh_hierarchize_adjoint: the transposed map: each point subtracts half of
 * the values of all points whose predecessor it is (gradient of a loss of the
 * hierarchized grid with respect to the nodal values).
 *
 * grids: host array of n descriptors (n >= 0; n == 0 is a no-op).  Each grid is
 * transformed in place.  FP64 data is computed in FP64; FP32 data in FP32.
 */
int sgh_hierarchize(const sgh_grid *grids, int32_t n, void *stream);
int sgh_dehierarchize(const sgh_grid *grids, int32_t n, void *stream);
int sgh_hierarchize_adjoint(const sgh_grid *grids, int32_t n, void *stream);

/* Same as the three above, selected by op (SGH_OP_*). */
int sgh_transform(int32_t op, const sgh_grid *grids, int32_t n, void *stream);

/* Out of place: dst[i] receives op applied to src[i], which is left
 * unchanged.  src[i] and dst[i] have the same dim, levels and dtype; no
 * destination may overlap any source or another destination, except that
 * dst[i].data == src[i].data is allowed and means in place for that grid
 * (SGH_ERR_OVERLAP otherwise; SGH_ERR_ARG for differing shapes).  The first
 * launch of each grid's schedule reads the source and writes the
 * destination, so the result costs no more HBM traffic than in place; for
 * the hierarchization a fused launch also takes the axis after its walked
 * axis (its one-shot stencil reads the predecessor planes, which stay nodal
 * in the source), one HBM round trip fewer than in place. */
int sgh_transform_out(int32_t op, const sgh_grid *src, const sgh_grid *dst, int32_t n, void *stream);

/* ---- batched plans ------------------------------------------------------
 *
 * A plan fixes an operation and a list of grids (shapes, dtypes and data
 * pointers), builds a device task list and, with SGH_PLAN_GRAPH, captures
 * all of its launches into one HIP graph.  Grids that fit the on-chip tile
 * are transformed by one kernel launch with one workgroup per grid (largest
 * grids first), each grid loaded into LDS, transformed along all axes and
 * stored once.  A set of many such grids (4096 or more of one dtype by
 * default, see sgh_set_batch_classes) is split into size classes by bytes
 * (up to 8, 16, 32 and 64 KiB), one launch each, so that each launch's
 * workgroups and LDS tiles fit its grids.  Medium grids (too large for the
 * tile, at most 2^18 points by default, at least 16 of them per dtype) go to
 * a second launch with one workgroup per grid that takes the grid's axes in
 * passes through its tile.
 * The remaining grids get their own launches, captured in the same graph.
 * This is the coarse "all combination grids in parallel" level of the
 * combination technique (Section 2).
 *
 * flags: SGH_PLAN_GRAPH   capture into a hipGraph at creation when the plan
 *                          needs more than one launch (a single launch is
 *                          issued directly)
 *        SGH_PLAN_AUTOTUNE time candidate tile configurations on scratch
 *                          buffers at creation and keep the fastest (results
 *                          are cached per device, op, dtype and level set).
 *        SGH_PLAN_RELATIVE the descriptors' data fields are byte offsets
 *                          (0 allowed, aligned to the element size) into one
 *                          buffer that is named at each execution
 *                          (sgh_plan_execute_at); such a plan never captures
 *                          a graph.  For callers that keep a whole set in one
 *                          allocation whose address changes between calls
 *                          (autograd buffers), without re-uploading the task
 *                          list or synchronizing.
 * The plan does not own the grid buffers; they must outlive every execute.
 */
#define SGH_PLAN_GRAPH 1u
#define SGH_PLAN_AUTOTUNE 2u
#define SGH_PLAN_RELATIVE 4u

typedef struct sgh_plan sgh_plan;

int sgh_plan_create(sgh_plan **plan, int32_t op, const sgh_grid *grids, int32_t n, uint32_t flags);
/* Executes a plan on `stream` (NULL = default stream).  SGH_ERR_ARG for a
 * relative plan. */
int sgh_plan_execute(sgh_plan *plan, void *stream);
/* Executes a relative plan (SGH_PLAN_RELATIVE) on the grids at base + offset:
 * base is a device pointer aligned to every grid's element size; the buffer
 * must hold every grid of the plan.  Allocates nothing; the same launches as
 * sgh_plan_execute.  SGH_ERR_ARG for a plan created without the flag or a
 * null base, SGH_ERR_ALIGN for a misaligned base. */
int sgh_plan_execute_at(sgh_plan *plan, void *base, void *stream);
/* A relative plan out of place: the grids at src_base + offset are
 * transformed into dst_base + offset (the source is left unchanged).  The
 * two buffers must not overlap over the plan's extent (SGH_ERR_OVERLAP);
 * equal bases mean in place.  Allocates nothing. */
int sgh_plan_execute_out(sgh_plan *plan, const void *src_base, void *dst_base, void *stream);
/* Repoint the plan to new buffers of identical shapes and dtypes (same n,
 * same order).  Synchronizes the device first (an execute in flight may still
 * read the old task list), then rewrites the device task list; the graph is
 * re-captured only when the plan holds grids too large for the batch kernel. */
int sgh_plan_set_data(sgh_plan *plan, const sgh_grid *grids, int32_t n);
/* Writes a short JSON description of the plan (launches, tiles, graph) into
 * buf (NUL-terminated, truncated to len).  Returns the full length needed. */
int sgh_plan_describe(const sgh_plan *plan, char *buf, int32_t len);
void sgh_plan_destroy(sgh_plan *plan);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops): op applied in place to every grid in one call, with
 * no plan and no allocation.  The grids that fit the on-chip tile (at most
 * SGH_STATIC_TASKS of them, else SGH_ERR_UNSUPPORTED before anything is
 * launched) go to the batch launch, whose task list is copied into a
 * fixed-size device array that the library holds on every device it has
 * run on (about 1.4 MB, until the process ends); larger grids get their own
 * launches, which use no device memory beyond the grid.  The array is
 * shared by every call on a device and keeps the last call's contents:
 * calls on one stream are ordered, but calls on one device from different
 * streams or threads that overlap in time race for it.  Same results, bit
 * for bit, as a plan without autotuning (sgh_plan_create + execute). */
#define SGH_STATIC_TASKS 4096
int sgh_transform_batch_static(int32_t op, const sgh_grid *grids, int32_t n, void *stream);

/* ---- combination technique: sparse grid of a combination set ------------
 *
 * Hierarchization is what makes the combination technique's communication
 * phase cheap (Section 2, "Hierarchization as preprocessing"): in the
 * hierarchical basis a point that a combination grid does not hold has
 * surplus zero, so the sparse grid's surplus at a point is the coefficient-
 * weighted sum of the surpluses of the grids that hold it (Fig. 1 shows the
 * +1/-1 weights in 2-d), with no interpolation.
 *
 * A combination object fixes a list of grids (one dim and one dtype; shapes,
 * data pointers) and one coefficient per grid, and builds the sparse-grid
 * layout on the host: every hierarchical subspace m (m_k >= 1) that lies in at
 * least one grid (m <= l componentwise), ordered by |m|_1 and then
 * lexicographically with m_0 compared first.  Subspace m stores its
 * prod_k 2^(m_k - 1) points densely, axis 0 fastest; point i of axis k sits at
 * the odd position 2 i + 1 of 1-d level m_k.  The sparse array is a device
 * buffer of sgh_combi_sparse_points elements of the grids' dtype, owned by
 * the caller.  The object does not own the grid buffers.
 *
 * flags: SGH_PLAN_GRAPH    sgh_combi_reduce replays one captured HIP graph
 *                          (re-captured when the sparse pointer changes)
 *        SGH_PLAN_AUTOTUNE autotune the hierarchize / dehierarchize plans.
 * Errors: SGH_ERR_ARG for a null pointer, n < 1, or grids of mixed dim or
 * dtype; descriptor errors as sgh_validate; SGH_ERR_UNSUPPORTED when the
 * dense level table (prod_k max_l l_k entries) exceeds 2^26 entries.
 * Calls on one object must not overlap in time (they share device state).
 */
typedef struct sgh_combi sgh_combi;

int sgh_combi_create(sgh_combi **combi, const sgh_grid *grids, int32_t n, const double *coefs, uint32_t flags);
/* Points of the sparse grid (length of the sparse array), -1 for null. */
int64_t sgh_combi_sparse_points(const sgh_combi *combi);
/* Number of subspaces S, -1 for null. */
int32_t sgh_combi_num_subspaces(const sgh_combi *combi);
/* Copies the layout to host arrays: sub_levels[S * dim] (level vector of
 * subspace s at s * dim, axis 0 first) and offsets[S] (first element). */
int sgh_combi_layout(const sgh_combi *combi, int32_t *sub_levels, int64_t *offsets);
/* sparse[point] = sum over the grids holding the point, in list order, of
 * coef * grid value (the grids must already hold surpluses).  Every element is
 * written.  Products and sums are rounded separately, in the grids' dtype.
 * Asynchronous on `stream` (NULL = default stream). */
int sgh_combi_gather(sgh_combi *combi, void *sparse, void *stream);
/* Every point of every grid takes the sparse grid's value at that point
 * (overwrites all grid values).  Asynchronous on `stream`. */
int sgh_combi_scatter(sgh_combi *combi, const void *sparse, void *stream);
/* One step of the iterated combination technique without the solver
 * (Section 2): hierarchize every grid, gather into `sparse`, scatter back,
 * dehierarchize every grid.  Leaves the sparse surpluses in `sparse`. */
int sgh_combi_reduce(sgh_combi *combi, void *sparse, void *stream);
/* Repoint to new grid buffers of identical shapes (same n and order).
 * Synchronizes the device first and drops a captured graph. */
int sgh_combi_set_data(sgh_combi *combi, const sgh_grid *grids, int32_t n);
void sgh_combi_destroy(sgh_combi *combi);

/* ---- host utilities (no device access) ---------------------------------- */

/* Validates descriptors exactly as the transforms do; touches no memory
 * behind data.  Returns SGH_OK or the first error. */
int sgh_validate(const sgh_grid *grids, int32_t n);
/* Number of stored points of a grid, or -1 on an invalid descriptor. */
int64_t sgh_num_points(const sgh_grid *grid);
/* Sparse-grid layout of a combination set, exactly as sgh_combi_create builds
 * it (same checks on the grids; host only).  Writes the first min(S, capacity)
 * subspaces to sub_levels[s * dim ..] and offsets[s] (either may be NULL), the
 * subspace count S to *num_subspaces and the total points to *points. */
int sgh_sparse_layout(const sgh_grid *grids, int32_t n, int32_t capacity, int32_t *sub_levels, int64_t *offsets,
                      int32_t *num_subspaces, int64_t *points);
/* Describes the launch schedule the library would use for one grid (JSON),
 * in place and out of place (sgh_transform_out). */
int sgh_schedule_describe(int32_t op, const sgh_grid *grid, char *buf, int32_t len);
int sgh_schedule_describe_out(int32_t op, const sgh_grid *grid, char *buf, int32_t len);
const char *sgh_error_string(int code);
const char *sgh_last_error_message(void);
/* Library version, e.g. "0.1.0". */
const char *sgh_version(void);

/* Tuning knob: poles of level `level` on strided axes are kept in registers
 * as dyadic blocks of span 2^block_exponent (the block boundaries are the
 * coarse points, transformed last; Section 3's binary-tree predecessors of a
 * block's interior points all lie inside the block).  Applies to schedules
 * and plans built after the call; 0 restores the default (or the autotuned)
 * choice.  Returns SGH_ERR_UNSUPPORTED for pairs this build has no kernel for. */
int sgh_set_pole_block(int32_t level, int32_t block_exponent);

/* Tuning knob: poles of level `level` on strided axes use the three-level
 * register walk: 2^top_exponent super-blocks of 2^block_exponent blocks of
 * span 2^block_exponent (level = top_exponent + 2 * block_exponent), with the
 * next group of rows prefetched when `prefetch` is 1.  block_exponent 0
 * removes the override.  Returns SGH_ERR_UNSUPPORTED for splits this build has
 * no kernel for. */
int sgh_set_pole_split(int32_t level, int32_t top_exponent, int32_t block_exponent, int32_t prefetch);

/* Tuning knob for poles too long for one pass (contiguous axes beyond the LDS
 * tile, strided axes beyond the register kernels), which are cut into dyadic
 * blocks: the block boundaries are the coarse points, transformed in later
 * launches on a lattice of spacing 2^(sum of the earlier spans) (Section 3's
 * binary-tree predecessors of a block's interior lie in the block or on its
 * boundary).  `fine` is the span exponent of the first launch, `coarse` that of
 * the later ones; each is capped to what fits a 64 KiB tile; 0 restores the
 * defaults (a 32 KiB tile first, then spans of 2^7).  Applies to schedules and
 * plans built after the call. */
int sgh_set_split_spans(int32_t fine, int32_t coarse);

/* Tuning knob for runs of consecutive small strided axes, which one launch
 * transforms together: each workgroup loads W adjacent columns times the full
 * extent of those axes into LDS (axes commute, Algorithm 1's outer loop may
 * take them in any grouping).  A run is formed only while the box stays within
 * `max_bytes` with rows (W elements) of at least `min_row_bytes`; 0 restores a
 * default (64 KiB boxes, 128-byte rows).  Applies to schedules and plans
 * built after the call; fusion level 0 forms no boxes. */
int sgh_set_box_limits(int32_t max_bytes, int32_t min_row_bytes);

/* Tuning knob for plans: grids larger than the on-chip tile with at most
 * `max_points` points (0..2^24; 0 turns the medium launch off) go to the
 * one-workgroup-per-grid medium launch when a plan holds at least `min_grids`
 * (>= 1) of them of one dtype; otherwise each gets its own launches.  Defaults
 * 2^18 and 16.  Applies to plans built after the call. */
int sgh_set_medium_limits(int64_t max_points, int32_t min_grids);

/* Tuning knob for plans: the small grids of one dtype are split into size
 * classes (one batch launch per class of up to 8, 16, 32, 64 KiB per grid)
 * when there are at least `min_grids` of them (0: never split); a class of
 * fewer than `min_per_class` (>= 1) grids joins the next larger class.  With
 * `concurrent` = 1 the class launches after the first go out on streams of
 * the plan's own, forked from the caller's stream and joined back to it (so
 * that they overlap); 0 issues them one after another on the caller's
 * stream.  Defaults 4096, 1024, 0.  Applies to plans built after the call. */
int sgh_set_batch_classes(int32_t min_grids, int32_t min_per_class, int32_t concurrent);

/* Schedule switch: level 1 (default) fuses the leading LDS-tile axes with one
 * strided axis walked in registers into a single launch (one HBM round trip
 * for both); level 2 does the same but keeps the walk two-level; level 0 keeps
 * one launch for the tile axes and one per strided axis.  Axes commute
 * (Algorithm 1's outer loop may take the dimensions in any order), so all give
 * the same map.  Applies to schedules and plans built after the call. */
int sgh_set_fusion(int32_t level);

/* Schedule switch for out-of-place hierarchization (sgh_transform_out,
 * sgh_plan_execute_out): 1 (default) folds the axis right after a fused
 * launch's walked axis into that launch.  Along an axis the hierarchization
 * is a one-shot stencil on nodal values (Algorithm 1 reads each point's
 * predecessors before they change), and the axes commute, so a pencil that
 * is one plane of that axis is first combined, as its rows are read, with
 * the same rows of its two hierarchical predecessor planes (x - a/2 - b/2),
 * then transformed along the tile and walked axes: one HBM write per point
 * for all of these axes; the predecessor rows are read again by other
 * workgroups at about the same time and mostly come from the caches.  In
 * place this is never done (the predecessor planes would be overwritten
 * while they are read).  0 keeps a separate launch for that axis.  Applies
 * to schedules and plans built after the call. */
int sgh_set_outer_stencil(int32_t on);

/* Launch-order switch for fused launches: 1 deals consecutive pencils to one
 * XCD (its L2 then holds the rows that neighbouring pencils share), 0
 * (default) keeps the hardware's round-robin order. */
int sgh_set_xcd_order(int32_t on);

/* Which strided axis the fused launch walks when several qualify and no
 * autotuned choice exists: 0 (default) the one with the smallest stride (each
 * workgroup then streams one contiguous slab), 1 the one with the largest. */
int sgh_set_walk_preference(int32_t pref);

/* ---- measurement support ------------------------------------------------
 *
 * With timing on, every kernel the library launches is bracketed by HIP
 * events recorded on the stream it is launched on; sgh_timing_report sums
 * their durations per kernel name (it synchronizes those events).  Off by
 * default; costs two event records per launch when on.  Graph executions are
 * timed as one unit named "graph".
 */
int sgh_timing_enable(int32_t on);
int sgh_timing_reset(void);
/* JSON object {name: {"count": c, "ms": total}, ...}; returns needed length. */
int sgh_timing_report(char *buf, int32_t len);

#ifdef __cplusplus
}
#endif

#endif /* SGH_H */
