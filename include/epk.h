/*
 * epk.h - edge-partitioned kernels for MI355X (gfx950).
 *
 * C ABI of libepk, an implementation of the edge-centric data-affinity model of
 * "A Graph-based Model for GPU Caching Problems" (arXiv 1605.02043):
 *
 *   - a data object is a vertex and a task is an edge using two objects
 *     (Section 3.1, Definition 1);
 *   - tasks are grouped into workgroups by a balanced edge partition that
 *     minimises the vertex-cut cost C = sum_v (p_v - 1), the number of
 *     redundant loads (Section 3.1, Definition 2, Eq. 1), solved through the
 *     clone-and-connect transform and a balanced vertex partition
 *     (Section 3.2, Definitions 3-4);
 *   - data are repacked along the new task order and every workgroup stages
 *     its distinct vertices in on-chip memory with coalesced loads
 *     (Section 4, Section 4.1).
 *
 * Conventions (every function):
 *   - Return value: an epk_status; EPK_OK is 0, errors are negative.  After a
 *     non-OK status, epk_last_error() returns a message (thread-local).
 *   - Host arrays passed in are owned by the caller and only read during the
 *     call; the library copies what it keeps.
 *   - Device pointers are borrowed: the caller allocates and frees them.  The
 *     library never allocates device memory.
 *   - stream is a hipStream_t passed as void* (NULL = the default stream).
 *     Device functions enqueue work on that stream and return without
 *     synchronising; validation of every argument happens before any launch.
 *   - Vertex ids are int32, counts int64.  Vertex state is row-major
 *     [n][5] float32 (rho, m1, m2, m3, E), indexed by PACKED vertex id.
 *   - Nothing here aborts or throws across the ABI.
 *   - A plan may be used from several streams at once only with distinct
 *     workspaces and outputs.
 */
#ifndef EPK_H
#define EPK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EPK_OK = 0,
  EPK_EINVAL = -1, /* null pointer, vertex id out of range, self-loop, cap < 1, bad enum */
  EPK_ERANGE = -2, /* sizes beyond what the kernels support (LDS budget, 16-bit local ids) */
  EPK_EHIP = -3,   /* HIP runtime or launch error */
  EPK_ESTATE = -4, /* plan/batch not uploaded, or used with the wrong kind */
  EPK_ENOMEM = -5, /* host allocation failed */
  EPK_ECANCELED = -6 /* a background partition was cancelled */
} epk_status;

typedef enum {
  /* edge partition through the transformed graph (Section 3.2): multilevel
   * vertex partition of the contracted clone-and-connect graph; at most cap
   * edges per part, k = ceil(m / (cap - cap/20)) parts (some may be empty),
   * tasks in ascending edge id inside a part */
  EPK_ORDER_EP = 0,
  /* default schedule: consecutive tasks per block, part = e / cap (Section 1) */
  EPK_ORDER_INPUT = 1,
  /* single-pass greedy growing on the same transform: k = ceil(m / cap),
   * parts 0..k-2 hold exactly cap edges, tasks in placement order */
  EPK_ORDER_GGP = 2,
  /* baselines of Section 3.3's comparison (PowerGraph's vertex cuts), same
   * k = ceil(m / cap) and capacity: random placement (edges sorted by the
   * SplitMix64 hash of their id, consecutive blocks of cap) and greedy
   * placement (edges in id order onto the least loaded part already holding
   * an endpoint, preferring parts holding both); see baselines.cpp */
  EPK_ORDER_RANDOM = 3,
  EPK_ORDER_GREEDY = 4
} epk_order;

typedef enum {
  EPK_FLUX5 = 0, /* cfd-style pairwise interaction on 5-component states */
  EPK_SPMV = 1   /* y_i += w_e x_j on the bipartite SpMV graph (Section 5.2) */
} epk_kind;

/* Partition quality and overhead (Definition 2; Section 3.2 balance factor).
 * loads L = sum_i |V(P_i)|, cost C = L - n_active, replicated R = #{p_v >= 2},
 * slots S = sum_{p_v >= 2} p_v, aux_cut = cut auxiliary edges of the
 * index-order transform, balance = max part size / (m / k).              */
typedef struct {
  int64_t n_parts, loads, cost, replicated, slots, aux_cut, n_active;
  int64_t max_part_edges, max_part_vertices;
  double balance, partition_seconds, plan_seconds;
} epk_stats;

/* A data-affinity graph (Definition 1).
 * FLUX5: edge e = (u, v), geometry = the unit normal from u to v (+ area):
 *        geom_ncomp 2 -> (nx, ny), area 1;  4 -> (nx, ny, nz, area).  The
 *        plan stores 3D geometry as the area vector area*(nx, ny, nz) (the
 *        Euler normal flux is linear in the normal) and recovers the area as
 *        its length; the normal must therefore have unit length.
 * SPMV : vertices [0, n_x) are x, [n_x, n_vertices) are y; edge e must be
 *        (j, n_x + i) for nonzero A[i][j]; geom_ncomp 1 -> the weight A[i][j].
 * edge_uv is host [n_edges][2], edge_geom host [n_edges][geom_ncomp].      */
typedef struct {
  int32_t n_vertices;
  int32_t n_x; /* SPMV only; 0 for FLUX5 */
  int64_t n_edges;
  const int32_t *edge_uv;
  const float *edge_geom;
  int32_t geom_ncomp;
} epk_graph;

typedef struct epk_plan epk_plan;
typedef struct epk_batch epk_batch;

/* ------------------------------------------------------------------ host */

/* The paper's problem (Eq. 1): graph + capacity in, edge -> part and cost out.
 * Every part holds at most `capacity` edges; k and the order inside a part
 * depend on the order (see epk_order).  part_of_edge[m] and task_order[m]
 * are caller-allocated (task_order may be NULL): task_order lists the edges
 * part by part (parts ascending).
 * Host only, synchronous; geometry is not read.                          */
int epk_partition(const epk_graph *g, int32_t capacity, int32_t order, int32_t *part_of_edge,
                  int32_t *task_order, epk_stats *stats);
/* The same with per-class vertex weights, EP order only: the partition
 * minimises sum_v w(v) (p_v - 1), Definition 2's cost with each replicated
 * copy of a vertex weighted by its class, through the same transform
 * (Section 3.2) with every chain link of vertex v weighing w(v).
 * class_weight[2] = {x, y}: x are vertices below n_x, y the rest (FLUX5
 * graphs have n_x = 0, so class_weight[1] applies to all).  {1, 1} (or
 * NULL) is the paper's uniform cost.  For SpMV a replicated y costs a
 * partial write, a read and a reduction step where a replicated x costs one
 * 4-byte gather, so {1, 4} trades x copies for y copies.  Weights 1..64;
 * EPK_EINVAL for other orders with weights other than {1, 1}.  stats
 * report the unweighted cost.                                             */
int epk_partition_weighted(const epk_graph *g, int32_t capacity, int32_t order, const int32_t *class_weight,
                           int32_t *part_of_edge, int32_t *task_order, epk_stats *stats);

/* The EP order after a hub split, for graphs whose degrees follow a power
 * law (an extension of Section 3.2's partition; the paper has no such
 * step).  An edge is a hub edge when its class-y endpoint (vertex id >=
 * g->n_x; of two such endpoints the one of larger degree, ties to the
 * smaller id) has degree above hub_degree.  The hub edges, sorted by (that
 * endpoint, the other endpoint, edge id), fill parts 0 .. kh-1 in runs of
 * `capacity` edges, so a hub of degree d lands in at most ceil(d/capacity)
 * + 1 parts, a bound the multilevel heuristic does not keep on such
 * graphs.  The other edges, in ascending id, form a graph that the EP
 * order (multilevel, with class_weight as in epk_partition_weighted)
 * splits into parts kh, kh+1, ...; task order: the hub parts, then that
 * partition's task order.  With no hub edge the result equals
 * epk_partition_weighted's.  hub_degree >= 1, else EPK_EINVAL; other
 * arguments and errors as epk_partition_weighted.                        */
int epk_partition_hub(const epk_graph *g, int32_t capacity, const int32_t *class_weight, int32_t hub_degree,
                      int32_t *part_of_edge, int32_t *task_order, epk_stats *stats);

/* Plan = partition + data packing along the task order (Section 4.1) + the
 * device image the kernels read.  Host only, synchronous.                */
int epk_plan_create(const epk_graph *g, int32_t capacity, int32_t order, int32_t kind, epk_plan **out);
/* epk_plan_create with per-class vertex weights (see epk_partition_weighted). */
int epk_plan_create_weighted(const epk_graph *g, int32_t capacity, int32_t order, int32_t kind,
                             const int32_t *class_weight, epk_plan **out);
/* epk_plan_create with the hub-split EP partition (epk_partition_hub).   */
int epk_plan_create_hub(const epk_graph *g, int32_t capacity, int32_t kind, const int32_t *class_weight,
                        int32_t hub_degree, epk_plan **out);
/* The same plan from a partition the caller made (Definition 2's output,
 * e.g. from an offline partitioner): part_of_edge[m] in [0, n_parts);
 * task_order[m] lists the edges part by part, parts ascending (NULL:
 * ascending edge id inside a part).  Both host, caller-owned, read during
 * the call.  EPK_EINVAL for an entry outside [0, n_parts) or a task order
 * that is not such a permutation; EPK_ERANGE if a part holds more than
 * `capacity` edges (a part's records fill one block of `capacity` slots).
 * Host only, synchronous.                                                 */
int epk_plan_create_partitioned(const epk_graph *g, int32_t capacity, int64_t n_parts, const int32_t *part_of_edge,
                                const int32_t *task_order, int32_t kind, epk_plan **out);
/* Bytes of the device image and of the per-call workspace (replicated-vertex
 * partials).  Both are caller-allocated; alignment 256 bytes.             */
int epk_plan_device_bytes(const epk_plan *p, size_t *image_bytes, size_t *workspace_bytes);
/* Copy the image to d_image (borrowed for the plan's lifetime) on stream.
 * The image also holds the single-launch reduction's per-part counters
 * (zero as uploaded; every launch leaves them zero): calls on one plan that
 * overlap in time must switch that reduction off (epk_plan_set_fused).    */
int epk_plan_upload(epk_plan *p, void *d_image, void *stream);
/* packed_to_orig[n]: original id of each packed vertex id.               */
int epk_plan_vertex_perm(const epk_plan *p, int32_t *packed_to_orig);
/* part_of_edge[m], task_order[m] as epk_partition returns them.          */
int epk_plan_part_of_edge(const epk_plan *p, int32_t *part_of_edge, int32_t *task_order);
/* Per part and vertex class (FLUX5: 1 class; SPMV: x then y, 2 classes):
 * own_begin/own_count[k * ncls] = the contiguous packed range the part owns
 * (its first-touched vertices); foreign_offset[k * ncls + 1] and
 * foreign_ids[cost] = the packed ids of the part's other vertices,
 * ascending.  Any pointer may be NULL.                                    */
int epk_plan_layout(const epk_plan *p, int32_t *own_begin, int32_t *own_count, int64_t *foreign_offset,
                    int32_t *foreign_ids);
/* The plan's partition quality and overhead (Definition 2: loads, cost,
 * replication; Eq. 1's balance), as epk_partition reports them.          */
int epk_plan_stats(const epk_plan *p, epk_stats *s);
/* Kernel-side sizes: [0] = n_parts, [1] = dynamic LDS bytes of the forward,
 * [2] = of the adjoint, [3] = workgroup size, [4] = vertex classes,
 * [5] = algorithmic HBM bytes of one forward (fwd + reduce),
 * [6] = algorithmic HBM bytes of one adjoint (bwd + reduce),
 * [7] = forward-kernel-only bytes, [8] = adjoint-kernel-only bytes,
 * [9] = max foreign vertices of a part, [10] = pipelined launch setting
 * (0: off), [11] / [12] = its forward / adjoint grid, [13] = its adjoint
 * LDS bytes, [14] = workspace layout in use (0 part-major, 1 vertex-major),
 * [15] = state staging (1 LDS, 0 caches only), [16] = single-launch
 * reduction in use (1) or not (0).  The byte counts follow the layout in
 * use; with the single launch, [7] / [8] hold the whole pass.             */
int epk_plan_info(const epk_plan *p, int64_t *info, int32_t n_info);
/* Launch shape for later calls: workgroup size wg (64..1024, multiple of
 * 64; FLUX5 requires capacity <= 8 wg, SPMV capacity <= 4 wg: each
 * lane then takes ceil(capacity / wg) consecutive edges of its part (the
 * SpMV default is four; the SpMV adjoint always runs one edge per lane);
 * 0 keeps the current one) and
 * xcd_swizzle (1: XCD x runs the consecutive parts [x*ceil(k/8),
 * (x+1)*ceil(k/8)), so parts sharing vertices share an L2; 0: part =
 * workgroup id; -1 keeps the current one).  Host only.                   */
int epk_plan_set_launch(epk_plan *p, int32_t wg, int32_t xcd_swizzle);
/* FLUX5 only: run the part kernels as a software-pipelined persistent
 * launch.  A grid of blocks_per_cu workgroups per CU (-1: as many as fit;
 * 0: back to one workgroup per part) walks the parts; each workgroup loads
 * the header, foreign ids and rows of its next parts while it computes the
 * current one, so the three dependent loads of a part (Section 4's
 * per-block staging) overlap the work of others.  Results are bitwise those
 * of the one-part-per-workgroup launch.  Needs wg <= 256 and the current
 * device (the grid is sized from its CU count and the kernels' occupancy);
 * epk_plan_set_launch switches it off again.  EPK_ERANGE if the double
 * buffers do not fit in a workgroup's LDS.                                */
int epk_plan_set_pipeline(epk_plan *p, int32_t blocks_per_cu);
/* Layout of the replicated vertices' partials in the workspace (d_ws):
 * 0 part-major (each part writes its foreign partials as one block and the
 * reduction gathers a vertex's partials through a slot list), 1 vertex-major
 * (each part scatters its partials so that a vertex's partials sit side by
 * side and the reduction reads them as one run), -1 automatic (FLUX5:
 * vertex-major when the reduced class has more than four partials per
 * replicated vertex; SPMV: vertex-major while the partials number at most
 * one per eight edges, part-major above).  The sum order, ascending part id, and hence
 * every result bit, is the same under both.  Host only; takes effect at the
 * next launch.  The vertex-major layout also stages each part's slot
 * indices in LDS: EPK_ERANGE (layout unchanged) if they no longer fit.   */
int epk_plan_set_slot_layout(epk_plan *p, int32_t layout);
/* FLUX5 only: staged = 1 (default) stages each part's vertex states in LDS,
 * one fetch per distinct vertex (Section 4); staged = 0 runs the paper's
 * cache-only alternative (Section 5.2's texture-cache variant): the same
 * parts, task order and packed layout, each edge reading its endpoints'
 * states from global memory through L1/L2.  The same results up to
 * rounding: the kernels are compiled separately, and the compiler may fuse
 * a multiply and an add differently.  Switches the pipelined launch off.
 * EPK_ERANGE if its LDS does not fit.                                     */
int epk_plan_set_staging(epk_plan *p, int32_t staged);
/* FLUX5 only: sum the replicated vertices' partials inside the part kernel
 * (on = 1) or in a second launch (on = 0, the default: on MI355X the
 * single launch is slower, since the sums' two dependent loads then extend
 * every workgroup's lifetime instead of running massively parallel).  In the single launch each workgroup stores its replicated
 * partials at device scope and then signals the part owning each of those
 * vertices (and itself) with a relaxed device-scope atomic add on that
 * part's counter (in the plan's image); the workgroup that completes a part's
 * count sums that part's replicated vertices in ascending part order, the
 * same arithmetic as the second launch, so results are bitwise the same.
 * Applies to the direct staged kernels with the part-major workspace (not
 * to the pipelined or cache-only launches, which keep two launches).
 * EPK_ESTATE (setting unchanged) if the plan does not allow it: a vertex
 * with more partials than one thread sums, a part signalling more than 64
 * parts, or arrays beyond 2 GiB.  Host only.                               */
int epk_plan_set_fused(epk_plan *p, int32_t on);
/* Frees the plan's host memory (NULL is ignored).  The device image and
 * workspace belong to the caller and are not touched.                     */
void epk_plan_destroy(epk_plan *p);

/* ---------------------------------------------------------------- device */

/* FLUX5 forward on packed states: r = sum of a_e F_e over the incident
 * edges (+ at u, - at v) and, if q_new != NULL, q_new = q + dt r.  The task
 * is Section 1's cfd interaction (Figure 1: one task per pair of adjacent
 * particles, reading both and updating both), run in the partition's task
 * order; each workgroup loads its part's distinct vertices into on-chip
 * memory with coalesced loads, as Section 4's software-cache kernel does, so
 * each vertex of a part is fetched once (Definition 2's loads L).
 * q, r, q_new: device [n][5] float32; d_ws: workspace_bytes.  Each
 * workgroup stages its part's vertices in LDS, accumulates per-vertex
 * partials there, writes owned vertices directly and replicated partials to
 * the workspace; those are summed in ascending part order, by the
 * workgroup that completes them or by a second kernel (epk_plan_set_fused).
 * EPK_ESTATE before upload or for an SpMV plan, EPK_EINVAL for a NULL
 * state, output or (when the cost is nonzero) workspace, EPK_EHIP if a
 * launch fails.                                                           */
int epk_forward(const epk_plan *p, const float *q, float *r, float dt, float *q_new, void *d_ws, void *stream);
/* epk_forward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same kernels and results, bit for bit, with the replicated-vertex
 * partials in a fixed 16 MiB array inside the library instead of d_ws.  No
 * allocation of any kind.  The array is per device (held from module load
 * until the process ends) and shared by every call on that device: calls
 * that overlap on one device race.  stream must belong to the current
 * device.  EPK_ERANGE if the plan's workspace_bytes exceed 16 MiB (tet55 at
 * capacity 256 needs 8.8 MB); otherwise as epk_forward.                   */
int epk_forward_scratch(const epk_plan *p, const float *q, float *r, float dt, float *q_new, void *stream);
/* FLUX5 adjoint: g_q = (dr/dq)^T g_r on packed q, g_r, g_q (device
 * [n][5] float32), on the same partition, staging (Section 4) and reduction
 * as the forward: the upstream gradients are gathered per part like the
 * states, and each part's vertex-state gradients are summed in LDS.  The
 * paper has no adjoint; this is the forward's transpose on its schedule.
 * Errors as epk_forward (g_r must not be NULL).                          */
int epk_backward(const epk_plan *p, const float *q, const float *g_r, float *g_q, void *d_ws, void *stream);
/* SPMV: y[n_y] = A x[n_x] in packed x / y ids (y packed id - n_x), the
 * paper's sparse-matrix workload (Section 5.2: one vertex per element of x
 * and of y, one task per nonzero).  x: device [n_x] float32, y: device
 * [n_y] float32, d_ws: workspace_bytes.  EPK_ESTATE for a FLUX5 plan or
 * before upload, EPK_EINVAL for NULL buffers.                             */
int epk_spmv(const epk_plan *p, const float *x, float *y, void *d_ws, void *stream);
/* The two launches behind epk_forward / epk_backward / epk_spmv (Section 4
 * staging, then the replicated vertices' fixed-order sums), for callers
 * that time or schedule them apart.  stage 0: the part kernel
 * (owned outputs, workspace partials); stage 1: the reduction (adds the
 * partials of replicated vertices in ascending part order, zeroes untouched
 * vertices, finishes q_new).  Stage 1 must follow stage 0 on the same stream
 * with the same buffers.  With the single-launch reduction stage 0 does
 * both and stage 1 launches nothing.  kind-specific arguments as above;
 * unused ones may be NULL (g_r for forward/spmv, dt/q_new for
 * backward/spmv).                                                         */
int epk_run_stage(const epk_plan *p, int32_t op, int32_t stage, const float *in, const float *g_r, float *out,
                  float dt, float *q_new, void *d_ws, void *stream);
/* epk_run_stage for benchmarking the stage's kernel (the measurements of
 * Section 5 are kernel times): the kernel is launched with start and stop
 * events that take the dispatch's own timestamps (hipExtLaunchKernel), and
 * *ms (host) receives its duration as the GPU ran it, without the dispatch
 * latency and event overheads that events recorded around the call would
 * add.  Blocks the host until the kernel ends; work enqueued earlier on the
 * stream (a cache scrub, say) runs first and is not counted.  *ms = 0 if the
 * stage launches no kernel.  Not for use under stream capture.  EPK_EINVAL
 * for a NULL ms; other errors as epk_run_stage.                          */
int epk_run_stage_timed(const epk_plan *p, int32_t op, int32_t stage, const float *in, const float *g_r, float *out,
                        float dt, float *q_new, void *d_ws, void *stream, float *ms);
/* op codes of epk_run_stage */
#define EPK_OP_FORWARD 0
#define EPK_OP_BACKWARD 1
#define EPK_OP_SPMV 2
/* SpMV adjoint on the same plan (Section 5.2's graph, transposed; the
 * paper has no adjoint): g_x = A^T g_y (g_x[j] = sum over the
 * nonzeros (i, j) of w g_y[i]) and, if g_w != NULL, the weight gradient
 * g_w[e] = g_y[i] x[j] for every edge e in ORIGINAL edge order.  x: packed
 * [n_x] (only read for g_w; may be NULL otherwise), g_y: packed [n - n_x],
 * g_x: packed [n_x], g_w: [m]; d_ws as for epk_spmv (the adjoint's x-class
 * partials share it, so do not overlap it with a forward on the same
 * workspace).  Two launches: the part kernel (per-part incidence lists over
 * x, fixed ascending order) and the x-class reduction (ascending part
 * order).                                                                 */
int epk_spmv_adjoint(const epk_plan *p, const float *x, const float *g_y, float *g_x, float *g_w, void *d_ws,
                     void *stream);
/* dst[i] = src[idx[i]] (inverse = 0) or dst[idx[i]] = src[i] (inverse = 1),
 * rows of ncomp float32 (device, n_rows rows each; idx device int32
 * [n_rows]); packs states into / out of the packed order, the data layout
 * transformation that follows the new task order (Section 4.1, cpack).
 * EPK_EINVAL for NULL buffers or ncomp < 1.                               */
int epk_permute_rows(const float *src, float *dst, const int32_t *idx, int64_t n_rows, int32_t ncomp,
                     int32_t inverse, void *stream);

/* -------------------------------------------------------------- adaptive */

/* Adaptive overhead control (the paper's EP-adapt, Sections 4.2 and 5): the
 * edge partition and plan are built on a background CPU thread while the
 * caller keeps running its default order; the caller polls, takes the plan
 * when it is ready and keeps whichever order times faster.  A reuse
 * pre-check runs first: every order loads at least n_active vertex copies,
 * so 1 - n_active / L_input (L_input: the default order's loads at this
 * capacity) bounds the fraction of loads any partition can save; below
 * min_saving the partition is skipped.  The graph arrays are copied; the
 * handle owns its thread.  Host only.                                     */
typedef struct epk_adaptive epk_adaptive;
int epk_adaptive_start(const epk_graph *g, int32_t capacity, int32_t kind, double min_saving, epk_adaptive **out);
/* state: 0 running, 1 plan ready, 2 skipped by the pre-check, 3 failed or
 * cancelled; saving_bound: the pre-check's bound; seconds: partition + plan
 * time once finished.  Any output pointer may be NULL.                    */
int epk_adaptive_poll(epk_adaptive *a, int32_t *state, double *saving_bound, double *seconds);
/* Hand over the EP plan (the caller destroys it); wait = 1 blocks until the
 * thread finishes.  EPK_ESTATE while running, after a skip or once taken.  */
int epk_adaptive_take(epk_adaptive *a, int32_t wait, epk_plan **plan);
/* Cancel an unfinished partition (it stops at its next coarsening level or
 * refinement pass, returning EPK_ECANCELED inside), join, free.           */
void epk_adaptive_destroy(epk_adaptive *a);

/* --------------------------------------------------------------- batched */

/* Many FLUX5 graphs in one launch per pass: every (graph, part) item is one
 * workgroup's block of tasks with its data staged as in Section 4, and the
 * launch shape is the thread-block size that Section 5.2 and Section 5.3
 * study.  Differs from a per-graph pointer list: the states of all graphs
 * are one concatenated array.  States of graph g live at
 * rows [vertex_offset(g), vertex_offset(g) + n_g) of one [sum n][5] array,
 * in graph g's packed order.  The plans must be FLUX5 with 4 geometry
 * components; the batch copies what it needs, the plans may be destroyed.
 * Work items (graph, part) run one workgroup each when every plan has the
 * same capacity, else they are dealt round-robin, largest first, to the
 * workgroups of one pipelined persistent launch (see epk_plan_set_pipeline;
 * epk_batch_set_launch picks either).                                     */
int epk_batch_create(int32_t n_graphs, epk_plan *const *plans, epk_batch **out);
/* Bytes of the batch's device image and workspace (caller-allocated,
 * 256-byte aligned), as epk_plan_device_bytes.                           */
int epk_batch_device_bytes(const epk_batch *b, size_t *image_bytes, size_t *workspace_bytes);
/* Copy the image to d_image (borrowed for the batch's lifetime) and size
 * the grids for the current device.                                       */
int epk_batch_upload(epk_batch *b, void *d_image, void *stream);
/* Launch shape of the batch.  wg: workgroup size (64..256, multiple of 64,
 * at least capacity / 8; 0 keeps the current one).  direct: 1 runs one
 * workgroup per (graph, part) item, as the single-plan kernels do (needs one
 * capacity for all graphs, else EPK_ESTATE; the default where possible); 0
 * the pipelined persistent launch (the default for mixed capacities); -1
 * keeps the current kind.  The grids follow at once
 * if the batch is uploaded, else at upload.  Results do not depend on the
 * shape (the per-vertex sums run in a fixed order).  Host only; EPK_EINVAL
 * for a size out of range.                                                */
int epk_batch_set_launch(epk_batch *b, int32_t wg, int32_t direct);
/* vertex_offset[n_graphs + 1] (rows), total in [n_graphs].               */
int epk_batch_vertex_offsets(const epk_batch *b, int64_t *vertex_offset);
/* [0] items, [1] forward grid, [2] forward LDS bytes, [3] / [4] algorithmic
 * bytes of one forward / adjoint, [5] workgroup size, [6] edges,
 * [7] adjoint grid (the pipelined launch's grids), [8] one workgroup per
 * item (1) or pipelined (0), [9] whether one workgroup per item is
 * possible for this batch.                                                */
int epk_batch_info(const epk_batch *b, int64_t *info, int32_t n_info);
/* Forward / adjoint of every graph of the batch: as epk_forward (dt = 0,
 * no q_new) and epk_backward, on the concatenated packed states q, r, g_r,
 * g_q (device [sum n][5] float32) and a workspace of workspace_bytes.  One
 * part kernel launch and one reduction launch per call.  EPK_ESTATE before
 * upload, EPK_EINVAL for NULL buffers, EPK_EHIP if a launch fails.        */
int epk_batch_forward(const epk_batch *b, const float *q, float *r, void *d_ws, void *stream);
int epk_batch_backward(const epk_batch *b, const float *q, const float *g_r, float *g_q, void *d_ws,
                       void *stream);
/* Frees the batch's host memory (NULL is ignored); the plans it was merged
 * from and the caller's device buffers stay as they are.                  */
void epk_batch_destroy(epk_batch *b);

/* Capacity and launch-shape selection for a batch (the block-size study of
 * Section 5.2 and Section 5.3, done by measurement on this GPU): for each capacity in caps[n_caps],
 * build every graph's EP plan at that capacity, merge them into one batch
 * and time its forward + adjoint launch (median of 5 timings of 5 passes)
 * in each launch shape: one workgroup per item and the pipelined persistent
 * launch, each at 256, 128 and 64 lanes where that leaves at most two edges
 * per lane.  The fastest (capacity, shape) is chosen for all graphs, since a
 * batched launch sizes every workgroup's LDS for its largest parts.
 * Timings within 2% of the fastest count as ties, won by the fewest
 * algorithmic bytes, then by the capacity listed first, one workgroup per
 * item and the larger workgroup.  Results are cached in cache_path (a text
 * file of key|cap wg direct lines, NULL = no cache).  d_scratch
 * (scratch_bytes) is caller-allocated device memory for the trials (a whole
 * batch's image, workspace and three state arrays); a capacity that does
 * not fit is skipped, EPK_ERANGE if none fits.  Plans are built on up to 16
 * host threads.  Synchronises the stream.  chosen_cap[n_graphs] out;
 * chosen_wg[n_graphs] and chosen_direct[n_graphs] (1: one workgroup per
 * item, 0: pipelined; see epk_batch_set_launch) may be NULL.              */
int epk_autotune(const epk_graph *gs, int32_t n_graphs, const int32_t *caps, int32_t n_caps,
                 const char *cache_path, void *d_scratch, size_t scratch_bytes, void *stream,
                 int32_t *chosen_cap, int32_t *chosen_wg, int32_t *chosen_direct);

/* Message of the last non-OK status on the calling thread (empty after a
 * successful call); the string belongs to the library and stays valid until
 * this thread's next call.                                                */
const char *epk_last_error(void);
/* Library name, version and target ("epk 0.1 (gfx950)"); static string.   */
const char *epk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EPK_H */
