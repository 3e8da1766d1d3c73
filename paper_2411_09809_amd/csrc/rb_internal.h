// Internal declarations of the HIP implementation behind include/rb.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rb.h"

namespace rb {

// ------------------------------------------------------------------ records
//
// Per-edge record written by the edge-preparation kernel: the first end
// point P = (x, y), the direction D = (dx, dy) = Q - P, the line constant
// c = dx*y - dy*x, the line angle th in [0, pi) and the end ids.  With integer
// coordinates |.| <= 2^20 every field but th is an integer below 2^43 in
// magnitude, hence exact in double, and so is every orientation value the
// sweep derives from them (Algorithm 4's CCW).
// tq is the line angle as an integer (see quantize_angle).
struct __align__(16) EdgeRec {
    double x, y;
    double dx, dy;
    double c, th;
    int32_t s, t;
    uint32_t tq;
    int32_t pad1;
};
static_assert(sizeof(EdgeRec) == 64, "edge record is 64 bytes");

// The crossing sweeps' angle term runs on line angles held as integers in
// units of u = pi / 2^26 (so pi/2 is exactly 2^25 u): tq = rint(th / u) in
// [0, 2^26].  With a = pi/2 - ||tq_e - tq_f| - 2^25| and beta = pi/2 -
// ideal in the same units, each crossing's deviation |ideal - a| is three
// v_sad_u32 operations (|x - y| + z) in exact integer arithmetic.  Against
// the same expression on the double angles, a is off by at most u (both
// roundings) and beta by u/2, so each deviation by at most 1.5 u = 7.0e-8.
constexpr uint32_t kHalfPiQ = 1u << 25;
constexpr double kAngleUnit = 3.14159265358979323846 / 67108864.0;
__host__ __device__ inline uint32_t quantize_angle(double th) {
    return (uint32_t)rint(th * (67108864.0 / 3.14159265358979323846));
}

// Record i of a layout segment of n records, or a padding edge at and past
// its end: a row tile (256 * rows records) need not divide the segment.
__device__ __forceinline__ EdgeRec edge_row(const EdgeRec *__restrict__ seg, int64_t i, int64_t n) {
    if (i < n) return seg[i];
    EdgeRec r;
    r.x = 0.0; r.y = 0.0; r.dx = 0.0; r.dy = 0.0; r.c = -1.0; r.th = 0.0;
    r.s = -1; r.t = -1; r.tq = 0; r.pad1 = 0;
    return r;
}

// An edge record as the pair sweeps hold it (rows in registers, columns in
// LDS): x and y become the end-point sums x1 + x2 = 2x + dx and y1 + y2, and c
// becomes 2c; dx, dy, th and the ids stay.  Exact: integers below 2^44.  The
// padding record keeps c != 0, so it never meets another edge's line.
__device__ __forceinline__ EdgeRec sweep_form(EdgeRec e) {
    e.x = fma(2.0, e.x, e.dx);
    e.y = fma(2.0, e.y, e.dy);
    e.c = 2.0 * e.c;
    return e;
}

// Per-node record for the occlusion sweep.  With n = x^2 + y^2 and T the
// largest integer below d^2, the test |p_u - p_v|^2 <= T is rewritten as
//     x_u x_v + y_u y_v + q_v >= h_u,   q = -n/2,  h = (n - T)/2,
// which is exact in double (all terms are multiples of 1/2 below 2^45).
struct __align__(16) NodeRec {
    double x, y, q, h;
};
static_assert(sizeof(NodeRec) == 32, "node record is 32 bytes");

// Partial results of one (block, layout) segment of a sweep.
struct __align__(16) CrossPartial {
    unsigned long long proper, touch;   // proper crossings, other closed crossings
    double dev;                         // sum of |ideal - a| (radians)
    double pad;
};
struct __align__(16) OcclPartial {
    unsigned long long count;
    unsigned long long pad;
};

// ------------------------------------------------------------------ tiling
constexpr int kBlock = 256;          // threads per sweep block (4 waves)
constexpr int kChunk = 256;          // column records staged in LDS per unit
constexpr int kMaxRows = 16;         // largest rows-per-thread of any variant
constexpr int kRecPad = kBlock * kMaxRows;   // record segments padded to this
// Blocks of one sweep launch, each with its own partial-result slot.  A sweep
// cuts its unit list into min(units, kMaxPartials) equal contiguous ranges,
// one per block: far more blocks than fit on the chip at once, so the
// hardware dispatcher hands ranges to compute units as they free up, which
// evens out uneven unit costs and clocks.
constexpr int kMaxPartials = 131072;
// A sweep over a unit list whose length only the device knows (the pruned
// paths) launches this many blocks per resident block slot, capped at
// kMaxPartials; blocks whose range is empty write a zero partial and exit.
constexpr int kListBlocksPerSlot = 8;
constexpr int kSmallDeg = 16;        // min-angle: thread-per-node up to this degree
constexpr int kLdsDeg = 2048;        // min-angle: block sort in LDS up to this degree

// One layout inside a sweep's unit list.  Row tile I (R = 256*K records)
// meets column chunks c = I*K*S .. n_chunks-1 of W = 256/S records each
// (S = 2^col_shift: the node sweep splits chunks when a layout has too few
// units to fill the chip; the edge sweeps keep S = 1); the layout's units
// are numbered from unit_off in that order.
struct SweepLayout {
    int64_t unit_off;       // first global unit of this layout
    int64_t rec_off;        // first record of this layout (multiple of kRecPad)
    int64_t n_row_tiles;
    int64_t n_chunks;
    int64_t col_shift;
};

// Kernel arguments of a sweep.  A single layout travels by value; a batch
// reads its table (n_layouts + 1 entries, the last holding only unit_off =
// total units) from device memory.
struct SweepArgs {
    const SweepLayout *table;
    SweepLayout single;
    int64_t n_layouts;
    int64_t n_units;        // units this launch covers ...
    int64_t unit_base;      // ... starting at this global unit (single layout only)
};

// Sweep kernel variants: rows per thread, minimum waves per SIMD and the
// column split of the unit list (log2 S; node sweep only).
struct SweepVariant {
    int rows;
    int waves;
    int col_shift;
};
constexpr int kCrossVariants = 4;
constexpr int kOcclVariants = 12;
SweepVariant cross_variant(int v);
SweepVariant occl_variant(int v);
// The batched edge sweep offers every crossing variant but the 4-row one:
// in batch form its table walk does not fit the register budget of 5 waves
// per SIMD and would be spilled to scratch memory in every block.
constexpr int kBatchCrossExcluded = 3;
inline bool variant_offered(int kind, bool batch, int v) {
    return !(batch && (kind == 0 || kind == 1) && v == kBatchCrossExcluded);
}

// Layout of the caller's workspace for one layout (byte offsets, 256-aligned).
struct WsLayout {
    size_t edge_rec, node_rec, partial, scalars;
    size_t deg, cursor, offs, angles, nbr, dv, big_list, hash, kacc, fwd;
    // hub order of the edge records (empty below kHubSortMinEdges edges)
    size_t hub_deg, hub_keys, hub_vals, hub_keys2, hub_vals2, hub_hist, hub_hist_off, hub_scan;
    size_t total;
    int64_t n_edge_pad, n_node_pad, hash_size;
};
bool ws_layout(int64_t n_nodes, int64_t n_edges, WsLayout *L);

// Grid-pruned paths (grid.hip): cell parameters on the device and the
// workspace they use (byte offsets, 256-aligned).
struct __align__(16) GridParams {
    int32_t xmin, ymin, xmax, ymax;   // bounding box of the node coordinates
    int32_t shift;                    // cell side 2^shift
    int32_t pad[3];
};
struct GridWs {
    size_t params, keys, vals, keys2, vals2, pos, hist, hist_off, scan_tile, partial;
    size_t rec, box, tile_cnt, tile_off, list;   // pruned edge sweep
    size_t kacc, scalars, fwd;                    // pruned loss and gradient
    size_t deg, cursor, offs, angles, nbr, dv, big_list;   // minimum-angle term
    size_t node_rec;                              // sweep records below kGridMinNodes
    size_t total;
    int64_t n_sort_blocks, n_edge_pad, max_units;
};
// largest edge count of the pruned edge sweep (its unit list is indexed in 32 bits)
constexpr int64_t kMaxPrunedEdges = 1ll << 24;
// below this many nodes the grid occlusion call runs the all-pairs sweep: its
// sort and count passes cost 0.13-0.14 ms up to about 65,000 nodes, where
// the sweep costs as much (50,000 nodes: 0.09 ms)
constexpr int64_t kGridMinNodes = 1ll << 16;
bool grid_ws_layout(int64_t n_nodes, int64_t n_edges, GridWs *G);

// Small device scalars used between kernels of one call.
struct __align__(16) Scalars {
    double mean;            // edge length mean
    double sum_dv;
    unsigned long long n_used;
    unsigned long long big_count;
    double ml;              // forward values used by the gradient pass
    double eca;
    unsigned long long count;
    int32_t flags;
    int32_t pad;
};

// Forward results kept between the passes of the loss-and-gradient calls
// (the call's `fwd` region, 8 words).
struct Fwd {
    unsigned long long count;   // E_c
    double eca, ml, ma;         // E_ca, M_l, M_a
    unsigned long long n_used;  // vertices of degree >= 1
    unsigned long long big_count;
    double sum_dv;
    double pad;
};

// Buffers of the minimum-angle pass: per-node degree, fill cursor, CSR
// offsets, per-half-edge direction angle and far end, per-node d_v, the
// queue of high-degree nodes, the scalar block and the reduction partials.
struct MinAngleBufs {
    uint32_t *deg, *cursor, *offs;
    double *ang, *dv;
    int32_t *nbr, *big;
    Scalars *sc;
    double *partial;
};
inline MinAngleBufs min_angle_bufs(const WsLayout &L, char *w) {
    return {(uint32_t *)(w + L.deg),  (uint32_t *)(w + L.cursor), (uint32_t *)(w + L.offs),
            (double *)(w + L.angles), (double *)(w + L.dv),       (int32_t *)(w + L.nbr),
            (int32_t *)(w + L.big_list), (Scalars *)(w + L.scalars), (double *)(w + L.partial)};
}
inline MinAngleBufs min_angle_bufs(const GridWs &G, char *w) {
    return {(uint32_t *)(w + G.deg),  (uint32_t *)(w + G.cursor), (uint32_t *)(w + G.offs),
            (double *)(w + G.angles), (double *)(w + G.dv),       (int32_t *)(w + G.nbr),
            (int32_t *)(w + G.big_list), (Scalars *)(w + G.scalars), (double *)(w + G.partial)};
}

// Fault injection (RB_FAULT, see rb.h): nonzero when `site` is listed;
// then the error text names `where` and the site.
bool fault_listed(const char *site);
int inject_fault(const char *site, const char *where);

// ------------------------------------------------------------------ plans
struct SweepPlan {
    int variant;
    int rows;
    int grid;
    int64_t n_units;
    SweepLayout single;
};
// Unit list of one layout of n_items records for a variant.
SweepLayout sweep_layout(int64_t n_items, int rows, int64_t unit_off, int64_t rec_off,
                         int col_shift = 0);
int64_t sweep_units(int64_t n_items, int rows, int col_shift = 0);
// Largest grid (blocks) of a sweep variant; a launch uses min(units, this),
// one equal contiguous range of the unit list per block.
int cross_grid(int variant, bool angle);
// Grid of a single layout's node sweep over n_units units: one unit per
// block (up to the partial slots), but two consecutive units per block for
// the split-chunk variants from kTwoUnitNodes nodes, where the units far
// outnumber the chip's block slots: the block's start-up (position, row
// loads) then serves two units, and the second unit's chunk is fetched while
// the first is swept.
constexpr int64_t kTwoUnitNodes = 1ll << 15;
int occl_grid(int variant, int64_t n_units, int64_t n_nodes);

// ------------------------------------------------------------------ launches
// Every launcher enqueues on `st` and returns the launch status.
hipError_t launch_edge_prep(const float *x, const float *y, const int32_t *src,
                            const int32_t *dst, int64_t n_nodes, int64_t n_edges, int64_t n_pad,
                            EdgeRec *rec, hipStream_t st);
hipError_t launch_edge_prep_ordered(const float *x, const float *y, const int32_t *src,
                                    const int32_t *dst, int64_t n_nodes, int64_t n_edges,
                                    int64_t n_pad, const int32_t *order, EdgeRec *rec,
                                    hipStream_t st);
hipError_t launch_node_prep(const float *x, const float *y, int64_t n_nodes, int64_t n_pad,
                            double T, NodeRec *rec, hipStream_t st);

hipError_t launch_cross_sweep(int variant, bool angle, const EdgeRec *rec, const SweepArgs &a,
                              int grid, double ideal, CrossPartial *part, hipStream_t st);
// The finalize calls sum n_part slots in a fixed order.  Above kFoldSpan
// slots a first kernel folds each span of kFoldSpan slots into its first
// slot (in place: the slots' contents are consumed), then one block adds
// the span totals.
constexpr int kFoldSpan = 2048;
hipError_t launch_cross_finalize(CrossPartial *part, int n_part, double ideal,
                                 unsigned long long *out_count, unsigned long long *out_proper,
                                 double *out_metric, double *out_dev_sum, hipStream_t st);
// The node sweep's slots hold twice the count of their units (the diagonal
// squares are counted as ordered pairs); its finalize takes doubled = true.
hipError_t launch_occl_sweep(int variant, const NodeRec *rec, const SweepArgs &a, int grid,
                             OcclPartial *part, hipStream_t st);
hipError_t launch_occl_finalize(OcclPartial *part, int n_part, unsigned long long *out_count,
                                bool doubled, hipStream_t st);

hipError_t launch_elv(const float *x, const float *y, const int32_t *src, const int32_t *dst,
                      int64_t n_nodes, int64_t n_edges, double *partial, Scalars *sc,
                      double *out_metric, double *out_mean, hipStream_t st);

hipError_t launch_min_angle(const float *x, const float *y, int64_t n_nodes,
                            const int32_t *src, const int32_t *dst, int64_t n_edges,
                            const MinAngleBufs &B, double *out_metric, double *out_sum_dv,
                            unsigned long long *out_n_used, hipStream_t st);
// Loss term w_m (1 - M_a) and its gradient, after launch_min_angle wrote M_a
// to *ma and the used-vertex count to *n_used: adds the term to *out_loss and
// scatters its gradient into gx, gy (which already hold the other terms).
hipError_t launch_min_angle_grad(const float *x, const float *y, int64_t n_nodes,
                                 const int32_t *src, const int32_t *dst, int64_t n_edges,
                                 const MinAngleBufs &B, double w_m, const double *ma,
                                 const unsigned long long *n_used,
                                 unsigned long long *big_count, double *out_loss, double *gx,
                                 double *gy, hipStream_t st);

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t st);
hipError_t launch_zero_scalars(Scalars *sc, hipStream_t st);
// deg[v] = number of end points of valid edges at node v (deg holds max(n_nodes, 1) words)
hipError_t launch_degrees(const int32_t *src, const int32_t *dst, int64_t n_nodes,
                          int64_t n_edges, uint32_t *deg, hipStream_t st);
// exclusive scan of deg[0..n) into offs[0..n] (tile: ceil(n/2048) scratch words)
hipError_t launch_scan(const uint32_t *deg, int64_t n, unsigned long long *tile, uint32_t *offs,
                       hipStream_t st);
// d_v of every node from its CSR segment of direction angles (sorts in place)
hipError_t launch_min_angle_nodes(const uint32_t *deg, const uint32_t *offs, double *ang,
                                  int64_t n_nodes, double *dv, int32_t *big, Scalars *sc,
                                  hipStream_t st);

// Stable LSD radix sort of (key, value) pairs, four 8-bit passes; the result
// ends in keys, vals.  hist and hist_off hold 256 ceil(n / kSortTile) words
// (hist_off one more), scan_tile ceil(that / 2048) + 1.
constexpr int kSortTile = 2048;
hipError_t launch_radix_sort(uint32_t *keys, int32_t *vals, uint32_t *keys2, int32_t *vals2,
                             int64_t n, uint32_t *hist, uint32_t *hist_off,
                             unsigned long long *scan_tile, hipStream_t st);

// Hub order of the edge records.  An edge pair that shares an end id has
// both orientation products zero, so the sweep's rare path runs for every
// wave-column holding one.  In input order the incident pairs of a
// power-law graph's hubs are spread over every wave-column (about one in 25
// holds one); sorted by the end point of larger degree, a hub's edges are
// consecutive records and its incident pairs fill a few tiles instead.  The
// sort costs about a millisecond, so single-layout sweeps of at least
// kHubSortMinEdges edges use it.
constexpr int64_t kHubSortMinEdges = 1ll << 20;
struct HubSortBufs {
    uint32_t *deg, *keys, *keys2, *hist, *hist_off;
    int32_t *vals, *vals2;
    unsigned long long *scan_tile;
};
// vals[0..n_edges) = the edge ids ordered by (hub id, edge id), where the
// hub of an edge is its end point of larger degree (the smaller id on a
// tie); edges with ids out of range go first.
hipError_t launch_hub_order(const int32_t *src, const int32_t *dst, int64_t n_nodes,
                            int64_t n_edges, const HubSortBufs &B, hipStream_t st);
hipError_t launch_grid_bounds(const float *x, const float *y, int64_t n, GridParams *gp,
                              int min_shift, int axis_bits, hipStream_t st);
// Sweep over an explicit unit list: tile I meets chunks list[tile_off[I] ..
// tile_off[I+1]); rows at and past n_rec are padding (cross.hip).
int cross_list_grid(int variant);
hipError_t launch_cross_list(int variant, const EdgeRec *rec, const int32_t *list,
                             const uint32_t *tile_off, int64_t n_tiles, int64_t n_rec, int grid,
                             double ideal, CrossPartial *part, hipStream_t st);
// Plan of the pruned edge sweep: records in Hilbert order, chunk boxes and the
// unit list of tiles of 256*K edges (grid.hip).
hipError_t launch_prune_plan(const float *x, const float *y, int64_t n_nodes,
                             const int32_t *src, const int32_t *dst, int64_t m, int K,
                             const GridWs &G, char *w, hipStream_t st);
hipError_t launch_loss_grad_pruned(const float *x, const float *y, int64_t n_nodes,
                                   const int32_t *src, const int32_t *dst, int64_t n_edges,
                                   double ideal, double w_a, double w_l, double w_m,
                                   double *out_loss, double *gx, double *gy,
                                   unsigned long long *out_count, const GridWs &G, char *w,
                                   hipStream_t st);
hipError_t launch_crossing_pruned(const float *x, const float *y, int64_t n_nodes,
                                  const int32_t *src, const int32_t *dst, int64_t n_edges,
                                  double ideal, const GridWs &G, char *w, int variant,
                                  double *out_metric, unsigned long long *out_count,
                                  double *out_dev_sum, hipStream_t st);
// Strip approximation of Sections 3.2.2 / 3.2.3 (strip.hip).
size_t strip_ws_bytes(int64_t m, int64_t n_pieces);
hipError_t launch_strip_count(const float *x, const float *y, const int32_t *src,
                              const int32_t *dst, int64_t n_nodes, int64_t m, int64_t w,
                              char *ws, hipStream_t st);
const unsigned long long *strip_total_ptr(const char *ws);
hipError_t launch_strip_crossing(const float *x, const float *y, const int32_t *src,
                                 const int32_t *dst, int64_t n_nodes, int64_t m, int64_t w,
                                 int64_t n_pieces, double ideal, char *ws, double *out_metric,
                                 unsigned long long *out_count, double *out_dev_sum,
                                 hipStream_t st);
hipError_t launch_occlusion_grid(const float *x, const float *y, int64_t n, double T,
                                 const GridWs &G, char *w, unsigned long long *out_count,
                                 hipStream_t st);
// loss w_a (1 - E_ca) + w_l M_l + w_m (1 - M_a) and its gradient with respect to x, y
hipError_t launch_loss_grad(const float *x, const float *y, int64_t n_nodes, const int32_t *src,
                            const int32_t *dst, int64_t n_edges, double ideal, double w_a,
                            double w_l, double w_m, double *out_loss, double *gx, double *gy,
                            unsigned long long *out_count, const WsLayout &L, char *w,
                            hipStream_t st);

hipError_t launch_validate(const float *x, const float *y, int64_t n_nodes,
                           const int32_t *src, const int32_t *dst, int64_t n_edges,
                           const WsLayout &L, char *ws, hipStream_t st);

int device_cu_count();

// FP64 FMA issue-rate probe (probe.hip): one launch of independent FMA
// chains; *out_lane_ops receives the FMA lane-operations it performs.
// rb_timing_* hooks for launches made outside the entry-point file: while
// timing is on, an event pair around the launch is kept for rb_timing_read.
struct TimedEvents {
    int kind;
    hipStream_t st;
    hipEvent_t a, b;
};
TimedEvents timed_begin(int kind, hipStream_t st);
void timed_end(TimedEvents &t);
hipError_t launch_valu_probe(int iters, double *sink, double *out_lane_ops, hipStream_t st);

// Error text of the calling host thread (api.hip); set_error and hip_error
// return the status they were given (RB_EHIP for hip_error).
int set_error(int status, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int hip_error(hipError_t e, const char *what);
void clear_error();

// Largest integer T with T < d^2 (d finite, >= 0): the squared-distance
// threshold of the occlusion test.  fma(d, d, -n) carries the exact sign of
// d^2 - n.  Squared distances are below 2^43, so T is capped at 2^44.
double occlusion_threshold(double d);

// Autotuning table (plan.hip).  kind: 0 crossing, 1 crossing + angle,
// 2 occlusion; n: records per layout (mean per layout for a batch).
int tuned_variant(int kind, bool batch, int64_t n);
void set_tuned_variant(int kind, bool batch, int64_t n, int variant);
bool save_tuning(const char *path);
bool load_tuning(const char *path);

// ------------------------------------------------------------------ helpers
// Block b of a grid of G blocks owns units [U*b/G, U*(b+1)/G).
__host__ __device__ inline int64_t block_first_unit(int64_t U, int64_t G, int64_t b) {
    return U * b / G;
}

// A batch table entry read into scalar registers.  The sweep kernels store
// to global memory, so the compiler cannot use a scalar load for the table
// and would keep the entry in vector registers, live across the whole sweep
// of a unit.
__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ SweepLayout table_entry(const SweepLayout *tab, int64_t L) {
    const SweepLayout t = tab[L];
    SweepLayout l;
    l.unit_off = uniform64(t.unit_off);
    l.rec_off = uniform64(t.rec_off);
    l.n_row_tiles = uniform64(t.n_row_tiles);
    l.n_chunks = uniform64(t.n_chunks);
    l.col_shift = uniform64(t.col_shift);
    return l;
}

// Units of the row tiles before tile I of a triangular sweep whose tile i
// meets chunks i*KS .. nC-1 (KS chunks span one row tile).
__device__ __forceinline__ int64_t units_before(int64_t I, int64_t nC, int64_t KS) {
    return I * nC - KS * I * (I - 1) / 2;
}

// block_first_unit for a kernel: a double-precision estimate corrected in
// integers.  The 64-bit division the compiler emits otherwise is a sequence
// of some hundred scalar instructions, run by every wave of every block, and
// the scalar unit is shared by the whole CU.
__device__ __forceinline__ int64_t first_unit(int64_t U, int64_t G, int64_t b) {
    const int64_t p = U * b;
    int64_t q = (int64_t)((double)U * (double)b * __builtin_amdgcn_rcp((double)G));
    while (q > 0 && q * G > p) --q;
    while ((q + 1) * G <= p) ++q;
    return q;
}

// tile_of_unit for operands below 2^31 (one unit per block: lu is a block
// index), with 32-bit conversions in place of the 64-bit ones.
__device__ __forceinline__ int64_t tile_of_unit32(int lu, int nI, int nC, int KS) {
    const double B = (double)nC + 0.5 * (double)KS;
    const double disc = fmax(B * B - 2.0 * (double)KS * (double)lu, 0.0);
    int I = (int)((B - sqrt(disc)) * __builtin_amdgcn_rcp((double)KS));
    I = I < 0 ? 0 : (I > nI - 1 ? nI - 1 : I);
    while (I > 0 && units_before(I, nC, KS) > lu) --I;
    while (I + 1 < nI && units_before(I + 1, nC, KS) <= lu) ++I;
    return I;
}

// Row tile of local unit lu: the largest I < nI with units_before(I) <= lu,
// from the smaller root of units_before(I) = lu (a quadratic in I) corrected
// in integers, in place of a binary search over the tiles.
__device__ __forceinline__ int64_t tile_of_unit(int64_t lu, int64_t nI, int64_t nC, int64_t KS) {
    const double B = (double)nC + 0.5 * (double)KS;
    const double disc = fmax(B * B - 2.0 * (double)KS * (double)lu, 0.0);
    int64_t I = (int64_t)((B - sqrt(disc)) * __builtin_amdgcn_rcp((double)KS));
    I = I < 0 ? 0 : (I > nI - 1 ? nI - 1 : I);
    while (I > 0 && units_before(I, nC, KS) > lu) --I;
    while (I + 1 < nI && units_before(I + 1, nC, KS) <= lu) ++I;
    return I;
}

}  // namespace rb
