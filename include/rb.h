/*
 * rb.h -- exact readability metrics of straight-line graph layouts on AMD
 * Instinct MI355X (gfx950).
 *
 * Implements the five metrics of Section 2.1 of "Scalable Readability
 * Evaluation for Graph Layouts: 2D Geometric Distributed Algorithms"
 * (arXiv 2411.09809) by the exact procedures of Section 3.1 (Algorithms 1-5):
 * node occlusion N_c, minimum angle M_a, edge length variation M_l, edge
 * crossing E_c and crossing angle E_ca.
 *
 * ------------------------------------------------------------------ layout
 * A layout is given as structure-of-arrays in DEVICE memory:
 *   x, y      float[n_nodes]   node coordinates.  Every value must be an
 *                              integer with |value| <= 2^20 (so the geometric
 *                              predicates are evaluated exactly);
 *   src, dst  int32[n_edges]   the two end node ids of each undirected edge,
 *                              0 <= id < n_nodes, src != dst, and no edge
 *                              listed twice (in either orientation).
 * These preconditions are not checked by the metric calls (their results are
 * only defined for valid input); rb_validate_layout checks all of them.  With
 * the environment variable RB_VALIDATE set (to anything but "" or "0"),
 * every call that takes a rb_workspace_size workspace checks them first and
 * returns RB_EDOMAIN on a violation; those calls then synchronise `stream`
 * and cannot be captured into a hipGraph (a debugging aid).
 * Limits: 0 <= n_nodes <= 2^31-1, 0 <= n_edges <= 2^30.
 *
 * ------------------------------------------------------------------ calls
 * Every metric call only ENQUEUES work on `stream` (a hipStream_t passed as
 * void*; NULL means the null stream) and returns.  It does not synchronise,
 * does not allocate and keeps no pointer after returning, so a sequence of
 * calls can be captured into a hipGraph.  Results are written to DEVICE
 * memory (out_* pointers are device pointers; the ones documented as
 * optional may be NULL) when the enqueued work completes.
 *
 * Scratch memory is supplied by the caller: `ws` is a device buffer of
 * `ws_bytes` bytes, at least rb_workspace_size(n_nodes, n_edges), 256-byte
 * aligned.  One workspace serves every call on the same layout size; calls
 * that run concurrently need separate workspaces.  All buffers stay owned by
 * the caller.
 *
 * ------------------------------------------------------------------ errors
 * Argument errors (NULL required pointer, negative or too large size, a bad
 * parameter, a workspace too small or misaligned) return RB_EINVAL or
 * RB_EWORKSPACE before anything is enqueued.  A failing HIP runtime call
 * returns RB_EHIP; a failed allocation of the library's own resources (a
 * batch plan, a graph) RB_ENOMEM.  rb_last_error() then describes the
 * failure (per host thread; valid until the next call on that thread).
 *
 * ------------------------------------------------------- fault injection
 * For tests of callers' error paths, the environment variable RB_FAULT (a
 * comma-separated list, read at each call) makes the library fail on
 * purpose: "launch" -- every call that enqueues GPU work returns RB_EHIP
 * after its argument checks and before its first HIP call (nothing is
 * enqueued, outputs are untouched); "alloc" -- rb_batch_create and
 * rb_batch_graph_create return RB_ENOMEM before allocating; "capture" --
 * rb_batch_graph_create fails inside its stream capture (the capture is
 * ended and discarded) and returns RB_EHIP.  rb_last_error() names the
 * injected fault.
 */
#ifndef RB_H
#define RB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rb_status {
    RB_OK = 0,
    RB_EINVAL = 1,      /* bad argument                                     */
    RB_EWORKSPACE = 2,  /* workspace NULL, misaligned or too small          */
    RB_EDOMAIN = 3,     /* layout violates the preconditions (validation)   */
    RB_EHIP = 4,        /* a HIP runtime call or kernel launch failed       */
    RB_ENOMEM = 5       /* the library could not allocate its own resources */
} rb_status;

/* Library version string, e.g. "rb 1.0.0 gfx950". */
const char *rb_version(void);

/* Text of the last error on the calling host thread ("" if none). */
const char *rb_last_error(void);

/* Bytes of workspace needed by every call below for a layout of this size
 * (a multiple of 256).  Returns 0 for negative or too large sizes. */
size_t rb_workspace_size(int64_t n_nodes, int64_t n_edges);

/* Node occlusion N_c (Section 2.1; Algorithm 1, Section 3.1.1): the number
 * of unordered node pairs {v,u}, v != u, whose Euclidean distance is
 * strictly less than `diameter` (the paper's 2r), evaluated exactly on the
 * integer coordinates.  diameter must be finite and >= 0.
 * out_count: device uint64[1]. */
rb_status rb_node_occlusion(const float *x, const float *y, int64_t n_nodes,
                            double diameter, uint64_t *out_count,
                            void *ws, size_t ws_bytes, void *stream);

/* Edge crossing E_c (Section 2.1; Algorithm 4, Section 3.1.4): the number
 * of unordered pairs of edges that do not share an end node and whose
 * closed segments intersect.  This is Algorithm 4's test -- both products
 * of CCW orientations <= 0 -- where, when both products are zero
 * (collinear or touching ends), the two bounding boxes must also overlap.
 * out_count:  device uint64[1] -- E_c.
 * out_proper: device uint64[1] or NULL -- pairs whose segments cross at a
 *             single point interior to both (both products < 0).         */
rb_status rb_edge_crossing(const float *x, const float *y, int64_t n_nodes,
                           const int32_t *src, const int32_t *dst, int64_t n_edges,
                           uint64_t *out_count, uint64_t *out_proper,
                           void *ws, size_t ws_bytes, void *stream);

/* Crossing angle E_ca (Section 2.1; Algorithm 5, Section 3.1.5): over the
 * crossing pairs of rb_edge_crossing, a = the acute angle between the two
 * edge lines (in [0, pi/2]; 0 for parallel lines and zero-length edges),
 * E_ca = 1 - mean(|ideal_angle - a| / ideal_angle); 1 when nothing
 * crosses.  ideal_angle in radians, 0 < ideal_angle <= pi/2 (the paper
 * uses 70 degrees).  The sweep evaluates a on line angles rounded to
 * multiples of pi / 2^26: each deviation is within 1.5 pi / 2^26 (7.0e-8)
 * of its value on the exact angles, so E_ca is within 7.0e-8 / ideal_angle
 * and the deviation sum within E_c times that.
 * out_metric:  device double[1] -- E_ca.
 * out_count:   device uint64[1] or NULL -- the crossing count E_c.
 * out_dev_sum: device double[1] or NULL -- sum of |ideal - a| / ideal.    */
rb_status rb_crossing_angle(const float *x, const float *y, int64_t n_nodes,
                            const int32_t *src, const int32_t *dst, int64_t n_edges,
                            double ideal_angle, double *out_metric,
                            uint64_t *out_count, double *out_dev_sum,
                            void *ws, size_t ws_bytes, void *stream);

/* rb_crossing_angle without a workspace, for callers that cannot allocate
 * device memory (code under hipGraph capture, tight serving loops, hosts
 * that forbid hipMalloc).  Same arguments and results as rb_crossing_angle
 * (identical kernels, so identical outputs), minus ws / ws_bytes: the edge
 * records and the sweep's partial slots live in a static device array of
 * the library, about 68 MB, which each device that runs this call holds
 * from its first call until the process ends (its address is looked up
 * once per device; `stream` must belong to the current device).  It calls
 * no allocator.  n_edges <= 1,000,000, else RB_EINVAL before anything is
 * enqueued.  All calls on one device share that array, and every call
 * rewrites all of it that it reads, so calls whose work overlaps in time on
 * one device (two streams, two host threads) race and give undefined
 * results; calls ordered on one stream are safe.                          */
rb_status rb_crossing_angle_noalloc(const float *x, const float *y, int64_t n_nodes,
                                    const int32_t *src, const int32_t *dst, int64_t n_edges,
                                    double ideal_angle, double *out_metric,
                                    uint64_t *out_count, double *out_dev_sum, void *stream);

/* Grid-pruned exact paths.  They return exactly what the brute-force calls
 * return (integer counts bit for bit) while skipping pairs that cannot
 * count, and they use their own workspace: rb_grid_workspace_size(V, E)
 * bytes, 256-byte aligned, caller-owned (it covers both calls below).
 * rb_node_occlusion_grid: N_c as rb_node_occlusion, by the grid method of
 *   Section 3.2.1 (cells of side >= d; each node meets the nodes of its own
 *   and four neighbour cells).  Work is O(|V| log |V| + candidate pairs).
 *   Below 2^16 nodes it runs the all-pairs sweep of rb_node_occlusion
 *   instead (the grid's sort and count passes cost more there); the count
 *   is the same either way.
 * rb_crossing_angle_pruned: E_ca, E_c and the deviation sum as
 *   rb_crossing_angle (Algorithms 4 and 5), skipping the tiles of the pair
 *   triangle whose edges' bounding boxes cannot meet: edges are ordered by
 *   bounding-box size class and the Morton code of the box centre first.
 *   Counts equal the brute-force counts; the deviation sum is added in
 *   another order (equal to rounding).  n_edges <= 2^24.  The gain depends
 *   on the layout: large for short edges, none for edges spanning the layout.
 * Errors as for the brute-force calls (RB_EWORKSPACE for a short or
 * misaligned workspace).                                                  */
size_t rb_grid_workspace_size(int64_t n_nodes, int64_t n_edges);
rb_status rb_node_occlusion_grid(const float *x, const float *y, int64_t n_nodes,
                                 double diameter, uint64_t *out_count, void *ws,
                                 size_t ws_bytes, void *stream);
rb_status rb_crossing_angle_pruned(const float *x, const float *y, int64_t n_nodes,
                                   const int32_t *src, const int32_t *dst, int64_t n_edges,
                                   double ideal_angle, double *out_metric, uint64_t *out_count,
                                   double *out_dev_sum, void *ws, size_t ws_bytes,
                                   void *stream);
/* rb_loss_grad_pruned: loss, gradient and crossing count as rb_loss_grad,
 * with the same culled sweep (the per-edge integer adjoint sums are the same
 * integers; the node gradients are the same sums added in another order).
 * Uses the rb_grid_workspace_size workspace.  n_edges <= 2^24.            */
rb_status rb_loss_grad_pruned(const float *x, const float *y, int64_t n_nodes,
                              const int32_t *src, const int32_t *dst, int64_t n_edges,
                              double ideal_angle, double w_angle, double w_length,
                              double w_min_angle, double *out_loss, double *out_grad_x,
                              double *out_grad_y, uint64_t *out_count, void *ws,
                              size_t ws_bytes, void *stream);

/* Approximate mode: the strip method of the enhanced edge-crossing and
 * crossing-angle algorithms (Sections 3.2.2 and 3.2.3).  The plane is cut
 * into strips of integer `width` starting at the smallest node coordinate
 * (vertical strips, or horizontal ones if `horizontal` != 0); in each strip
 * the edges that span it are compared, and a pair counts when the order of
 * their coordinates at the strip's two lines is strictly reversed.  Crossings
 * near an edge's end (inside a strip it does not span) or exactly on a strip
 * line are missed, so the count is a lower bound of E_c.  Outputs (device):
 * out_metric double[1] (1 - mean deviation, 1 if no pair), out_count
 * uint64[1] or NULL, out_dev_sum double[1] or NULL; *out_pieces (host, may
 * be NULL) receives the number of edge pieces.  The call synchronizes
 * `stream` once (to read the piece count).  Workspace:
 * rb_enhanced_workspace_size(n_edges, pieces) bytes; with less than that the
 * call returns RB_EWORKSPACE after writing *out_pieces, so a caller can
 * retry with rb_enhanced_workspace_size(n_edges, *out_pieces).  width in
 * [1, 2^22]; fewer than 2^32 pieces.                                       */
size_t rb_enhanced_workspace_size(int64_t n_edges, uint64_t n_pieces);
rb_status rb_enhanced_crossing(const float *x, const float *y, int64_t n_nodes,
                               const int32_t *src, const int32_t *dst, int64_t n_edges,
                               int64_t width, int horizontal, double ideal_angle,
                               double *out_metric, uint64_t *out_count, double *out_dev_sum,
                               uint64_t *out_pieces, void *ws, size_t ws_bytes, void *stream);

/* Shards of the two all-pairs sweeps, for splitting one layout across
 * devices or processes (each computes its shards; the sums of the shard
 * results are the full results) and for checking a slice of a large
 * layout.  The rows of the pair triangle (edges for the crossing test,
 * nodes for occlusion) are cut at the sweep's row-tile boundaries into
 * n_shards contiguous ranges of about equal pair counts (later shards may be
 * empty when there are more shards than tiles).  Shard k covers the pairs
 * (i, j) with row_begin <= i < row_end and i < j < n; *out_row_begin and
 * *out_row_end (host, may be NULL) report that range.  The ranges depend on
 * the sweep variant in use (see rb_tune_*), so all participants must use the
 * same one.
 * rb_crossing_angle_shard: out_count device uint64[1] (crossings in the
 *   shard), out_dev_sum device double[1] or NULL (sum of |ideal - a| / ideal).
 * rb_node_occlusion_shard: out_count device uint64[1].                     */
rb_status rb_crossing_angle_shard(const float *x, const float *y, int64_t n_nodes,
                                  const int32_t *src, const int32_t *dst, int64_t n_edges,
                                  double ideal_angle, int64_t shard, int64_t n_shards,
                                  uint64_t *out_count, double *out_dev_sum,
                                  int64_t *out_row_begin, int64_t *out_row_end,
                                  void *ws, size_t ws_bytes, void *stream);
rb_status rb_node_occlusion_shard(const float *x, const float *y, int64_t n_nodes,
                                  double diameter, int64_t shard, int64_t n_shards,
                                  uint64_t *out_count, int64_t *out_row_begin,
                                  int64_t *out_row_end, void *ws, size_t ws_bytes, void *stream);

/* Minimum angle M_a (Section 2.1; Algorithm 2, Section 3.1.2): for each
 * node v of degree deg(v) >= 1, the directions v->u of its incident edges
 * as angles in [0, 2 pi), phi_min(v) = the smallest gap between
 * circularly consecutive angles (the wrap-around gap included),
 * d_v = (2 pi/deg - phi_min) / (2 pi/deg); M_a = 1 - mean of d_v over the
 * nodes of degree >= 1 (1 when there are none).
 * out_metric: device double[1];  out_sum_dv: device double[1] or NULL;
 * out_n_used: device uint64[1] or NULL (number of nodes of degree >= 1).  */
rb_status rb_min_angle(const float *x, const float *y, int64_t n_nodes,
                       const int32_t *src, const int32_t *dst, int64_t n_edges,
                       double *out_metric, double *out_sum_dv, uint64_t *out_n_used,
                       void *ws, size_t ws_bytes, void *stream);

/* Edge length variation M_l (Section 2.1; Algorithm 3, Section 3.1.3):
 * l_e the Euclidean edge lengths, N = n_edges, mu = mean(l),
 * M_l = sqrt(sum (l_e - mu)^2 / (N mu^2)) / sqrt(N - 1); 0 when N < 2 or
 * mu = 0.  out_metric: device double[1]; out_mean: device double[1] or NULL. */
rb_status rb_edge_length_variation(const float *x, const float *y, int64_t n_nodes,
                                   const int32_t *src, const int32_t *dst, int64_t n_edges,
                                   double *out_metric, double *out_mean,
                                   void *ws, size_t ws_bytes, void *stream);

/* Layout-optimisation loss and its gradient (the application the paper's
 * Conclusion names; the loss is this library's choice, built from the
 * Algorithm 5, Algorithm 3 and Algorithm 2 metrics):
 *     L = w_angle (1 - E_ca) + w_length M_l + w_min_angle (1 - M_a)
 * with the crossing set S of the current layout held fixed, and
 * d L / d(x, y) of every node, computed exactly as the chain rule through
 * each crossing pair's acute angle, each edge's length and, at each vertex,
 * the two edge directions that bound its smallest gap (M_a averages
 * phi_v deg_v / 2 pi over the vertices of degree >= 1; the term is 0 when
 * there are none).  Kinks (a pair at exactly the ideal angle, perpendicular
 * or parallel lines, equal edge lengths, zero-length edges, a smallest gap
 * that is zero or attained more than once) contribute 0.  w_min_angle = 0
 * skips the M_a passes.  The coordinates must satisfy the layout
 * preconditions (the crossing set is exact on integers).  Weights finite.
 * out_loss: device double[1]; out_grad_x, out_grad_y: device double[n_nodes]
 * (overwritten); out_count: device uint64[1] or NULL -- |S| = E_c. */
rb_status rb_loss_grad(const float *x, const float *y, int64_t n_nodes,
                       const int32_t *src, const int32_t *dst, int64_t n_edges,
                       double ideal_angle, double w_angle, double w_length,
                       double w_min_angle, double *out_loss, double *out_grad_x,
                       double *out_grad_y, uint64_t *out_count, void *ws, size_t ws_bytes,
                       void *stream);

/* Checks the layout preconditions listed above on the GPU and waits for the
 * result (this call synchronises `stream`).  Returns RB_OK or RB_EDOMAIN;
 * *out_flags (host int32, may be NULL) receives a bit set:
 *   1 a coordinate is not an integer, 2 a coordinate exceeds 2^20 in
 *   magnitude, 4 an edge end id is out of range, 8 a self-loop,
 *   16 an edge listed twice.                                              */
rb_status rb_validate_layout(const float *x, const float *y, int64_t n_nodes,
                             const int32_t *src, const int32_t *dst, int64_t n_edges,
                             int32_t *out_flags, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------ batches
 * Many layouts of uneven size in one evaluation.  The layouts are
 * concatenated: x, y hold the nodes of layout 0, then layout 1, ...;
 * src, dst the edges likewise, with end ids LOCAL to their layout
 * (0 <= id < nodes of that layout).  node_off / edge_off (host int64,
 * n_layouts + 1 entries, starting at 0, nondecreasing) give each layout's
 * range.  Each all-pairs sweep runs as ONE launch over the unit lists of
 * all layouts; per-layout results are combined in a fixed order.
 *
 * rb_batch_create builds the host plan (diameters: host double[n_layouts]).
 * rb_batch_upload writes the plan's tables into the workspace (at least
 * rb_batch_workspace_size bytes, 256-byte aligned) and synchronises
 * `stream`; evaluations must use that same workspace.
 * rb_batch_evaluate only enqueues kernels (capturable): outputs are device
 * arrays of n_layouts entries, each may be NULL to skip that metric --
 * node occlusion N_c, crossing count E_c, crossing angle E_ca, minimum
 * angle M_a, edge length variation M_l, with the per-layout definitions of
 * the single-layout calls.
 * rb_batch_autotune times the sweep variants on this batch, keeps the
 * fastest in the plan and the tuning table, re-uploads; it synchronises.
 * rb_batch_graph_create captures rb_batch_evaluate with these arguments into
 * a hipGraph (on a private stream); rb_graph_launch replays it on `stream`.
 * The graph reuses the given pointers: keep them valid while it is used.
 * A graph records the plan it was captured from: a later rb_batch_upload or
 * rb_batch_autotune of that batch rewrites the plan's tables (possibly for
 * another sweep variant), after which rb_graph_launch returns RB_EINVAL
 * and the graph must be captured again.  Destroy graphs before their batch. */
typedef struct rb_batch rb_batch;
typedef struct rb_graph rb_graph;
rb_status rb_batch_create(int64_t n_layouts, const int64_t *node_off, const int64_t *edge_off,
                          const double *diameters, rb_batch **out);
size_t rb_batch_workspace_size(const rb_batch *batch);
rb_status rb_batch_upload(rb_batch *batch, void *ws, size_t ws_bytes, void *stream);
rb_status rb_batch_evaluate(const rb_batch *batch, const float *x, const float *y,
                            const int32_t *src, const int32_t *dst, double ideal_angle,
                            uint64_t *out_occlusion, uint64_t *out_crossings,
                            double *out_crossing_angle, double *out_min_angle, double *out_elv,
                            void *ws, size_t ws_bytes, void *stream);
rb_status rb_batch_autotune(rb_batch *batch, const float *x, const float *y, const int32_t *src,
                            const int32_t *dst, double ideal_angle, int repeats,
                            double *out_best_ms, void *ws, size_t ws_bytes, void *stream);
rb_status rb_batch_variants(const rb_batch *batch, int *cross_rows, int *cross_waves,
                            int *occl_rows, int *occl_waves);
void rb_batch_destroy(rb_batch *batch);
rb_status rb_batch_graph_create(const rb_batch *batch, const float *x, const float *y,
                                const int32_t *src, const int32_t *dst, double ideal_angle,
                                uint64_t *out_occlusion, uint64_t *out_crossings,
                                double *out_crossing_angle, double *out_min_angle,
                                double *out_elv, void *ws, size_t ws_bytes, rb_graph **out);
rb_status rb_graph_launch(rb_graph *graph, void *stream);
void rb_graph_destroy(rb_graph *graph);

/* Autotuning of the all-pairs sweeps.  The sweeps come in variants (rows
 * of the pair matrix held per thread, waves per SIMD and, for the node
 * sweep, how many units each 256-column chunk is split into); all variants
 * give identical results.  Each call above picks the variant recorded for the
 * layout's size class (floor(log2) of its edge count, node count for the
 * occlusion sweep); built-in defaults apply until tuned.
 *   kind: 0 = edge crossing, 1 = crossing angle, 2 = node occlusion,
 *         3 = pruned crossing angle (rb_crossing_angle_pruned; not timed by
 *         rb_autotune; default 256 edges per row tile below 2^17 edges,
 *         512 above);
 *   batch: 0 = single-layout calls, 1 = rb_batch_* calls.
 * rb_autotune times every variant of the three sweeps on the given layout
 * (`repeats` timed launches each, after one untimed launch), records the
 * fastest for its size classes and returns the sum of the three best mean
 * launch times in *out_best_ms (host, may be NULL).  It synchronises
 * `stream`.  rb_tune_set forces a variant index (0 .. variants-1) for a size
 * class (the batched edge sweeps do not offer variant 3, 4 rows per thread:
 * RB_EINVAL); rb_tune_query reports the rows, waves and column split (1, 4 or
 * 8; 1 for the edge sweeps) of the variant in use (each out pointer may be
 * NULL).
 * rb_tune_save / rb_tune_load write and read the table as text (a load
 * replaces the whole table: classes the file does not list return to the
 * built-in defaults); the file
 * named by the environment variable RB_TUNE_CACHE is loaded on first use. */
rb_status rb_autotune(const float *x, const float *y, int64_t n_nodes,
                      const int32_t *src, const int32_t *dst, int64_t n_edges,
                      double diameter, double ideal_angle, int repeats, double *out_best_ms,
                      void *ws, size_t ws_bytes, void *stream);
rb_status rb_tune_set(int kind, int batch, int64_t n_items, int variant);
rb_status rb_tune_query(int kind, int batch, int64_t n_items, int *rows, int *waves,
                        int *col_split);
rb_status rb_tune_save(const char *path);
rb_status rb_tune_load(const char *path);

/* Attainable FP64 FMA rate of the current device, the practical ceiling the
 * sweeps are measured against: one untimed and `repeats` timed launches of
 * a kernel of independent FMA chains (`iters` FMAs per chain) on `stream`,
 * timed with HIP events; the call synchronizes.  *out_lane_ops_per_s (host)
 * receives FMA lane-operations per second; sink is a device double the
 * kernel never writes in practice (it keeps the chains from being removed).
 * iters in [1, 2^24], repeats in [1, 1000].                               */
rb_status rb_valu_probe(int iters, int repeats, double *out_lane_ops_per_s, double *sink,
                        void *stream);

/* Kernel timing for measurement.  While enabled, the library records a HIP
 * event pair on the caller's stream around each launch of its all-pairs
 * sweep kernels.  rb_timing_read waits for the recorded events and returns
 * the summed duration in milliseconds and the number of launches of one
 * kind: 0 = edge-pair sweep (crossing / crossing angle), 1 = node-pair
 * sweep (occlusion), 2 = grid occlusion (all its kernels), 3 = pruned
 * edge-pair path (all its kernels), 4 = the fused forward + adjoint
 * edge-pair sweep of rb_loss_grad (that kernel only).  rb_timing_reset
 * clears the sums.                                                        */
rb_status rb_timing_enable(int enable);
rb_status rb_timing_reset(void);
rb_status rb_timing_read(int kernel, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* RB_H */
