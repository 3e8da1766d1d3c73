// C-ABI entry points of librb (declared in include/rb.h): argument checks,
// workspace carving and the launch sequence of each metric.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "rb.h"
#include "rb_internal.h"

namespace rb {
namespace {

thread_local std::string g_err;

rb_status fail(rb_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
rb_status fail(rb_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

rb_status hip_fail(hipError_t e, const char *what) {
    return fail(RB_EHIP, "%s: %s", what, hipGetErrorString(e));
}

constexpr int64_t kMaxNodes = 2147483647LL;
constexpr int64_t kMaxEdges = 1LL << 30;

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Timing of the sweep kernels (rb_timing_*): 0 edge-pair sweep, 1 node-pair
// sweep, 2 grid occlusion, 3 pruned edge sweep, 4 fused forward + adjoint
// sweep.
constexpr int kTimedKinds = 5;
struct Timing {
    std::mutex mu;
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[kTimedKinds];
    double ms[kTimedKinds] = {};
    int64_t n[kTimedKinds] = {};
} g_timing;

struct TimedLaunch {
    int kind;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    TimedLaunch(int k, hipStream_t s) : kind(k), st(s) {
        std::lock_guard<std::mutex> g(g_timing.mu);
        if (!g_timing.on) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            a = b = nullptr;
            return;
        }
        (void)hipEventRecord(a, st);
    }
    void done() {
        if (!a) return;
        (void)hipEventRecord(b, st);
        std::lock_guard<std::mutex> g(g_timing.mu);
        g_timing.ev[kind].emplace_back(a, b);
        a = b = nullptr;
    }
};

}  // namespace

TimedEvents timed_begin(int kind, hipStream_t st) {
    TimedEvents t{kind, st, nullptr, nullptr};
    std::lock_guard<std::mutex> g(g_timing.mu);
    if (!g_timing.on || kind < 0 || kind >= kTimedKinds) return t;
    if (hipEventCreate(&t.a) != hipSuccess || hipEventCreate(&t.b) != hipSuccess) {
        t.a = t.b = nullptr;
        return t;
    }
    (void)hipEventRecord(t.a, st);
    return t;
}

void timed_end(TimedEvents &t) {
    if (!t.a) return;
    (void)hipEventRecord(t.b, t.st);
    std::lock_guard<std::mutex> g(g_timing.mu);
    g_timing.ev[t.kind].emplace_back(t.a, t.b);
    t.a = t.b = nullptr;
}

namespace {

rb_status check_sizes(int64_t n_nodes, int64_t n_edges) {
    if (n_nodes < 0 || n_nodes > kMaxNodes)
        return fail(RB_EINVAL, "n_nodes = %lld out of range [0, 2^31-1]", (long long)n_nodes);
    if (n_edges < 0 || n_edges > kMaxEdges)
        return fail(RB_EINVAL, "n_edges = %lld out of range [0, 2^30]", (long long)n_edges);
    return RB_OK;
}

rb_status check_layout(const float *x, const float *y, int64_t n_nodes, const int32_t *src,
                       const int32_t *dst, int64_t n_edges) {
    rb_status s = check_sizes(n_nodes, n_edges);
    if (s) return s;
    if (n_nodes > 0 && (!x || !y)) return fail(RB_EINVAL, "x or y is NULL");
    if (n_edges > 0 && (!src || !dst)) return fail(RB_EINVAL, "src or dst is NULL");
    if (n_edges > 0 && n_nodes < 2) return fail(RB_EINVAL, "edges need at least two nodes");
    return RB_OK;
}

rb_status check_ws(void *ws, size_t ws_bytes, int64_t n_nodes, int64_t n_edges, WsLayout *L) {
    if (!ws_layout(n_nodes, n_edges, L)) return fail(RB_EINVAL, "layout too large");
    if (!ws) return fail(RB_EWORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws & 255u) != 0) return fail(RB_EWORKSPACE, "workspace not 256-byte aligned");
    if (ws_bytes < L->total)
        return fail(RB_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, L->total);
    return RB_OK;
}

int g_cu_count[64];

}  // namespace

// The layout checks of rb_validate_layout on `st`, waited for: RB_OK, or
// RB_EDOMAIN with the violations named in the error text.
rb_status validate_now(const float *x, const float *y, int64_t n_nodes, const int32_t *src,
                       const int32_t *dst, int64_t n_edges, const WsLayout &L, char *w,
                       hipStream_t st, int32_t *out_flags) {
    hipError_t e = launch_validate(x, y, n_nodes, src, dst, n_edges, L, w, st);
    if (e != hipSuccess) return hip_fail(e, "validate launch");
    Scalars sc;
    e = hipMemcpyAsync(&sc, w + L.scalars, sizeof sc, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return hip_fail(e, "validate copy");
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "validate synchronize");
    if (out_flags) *out_flags = sc.flags;
    if (sc.flags) {
        std::string msg = "invalid layout:";
        if (sc.flags & 1) msg += " non-integer coordinate;";
        if (sc.flags & 2) msg += " coordinate beyond 2^20;";
        if (sc.flags & 4) msg += " edge end out of range;";
        if (sc.flags & 8) msg += " self-loop;";
        if (sc.flags & 16) msg += " duplicate edge;";
        g_err = msg;
        return RB_EDOMAIN;
    }
    return RB_OK;
}

// RB_VALIDATE set to anything but "" or "0": the calls that take a
// rb_workspace_size workspace check the layout first (synchronously).
rb_status validate_if_requested(const float *x, const float *y, int64_t n_nodes,
                                const int32_t *src, const int32_t *dst, int64_t n_edges,
                                const WsLayout &L, char *w, hipStream_t st) {
    const char *v = getenv("RB_VALIDATE");
    if (!v || !*v || (v[0] == '0' && v[1] == 0)) return RB_OK;
    return validate_now(x, y, n_nodes, src, dst, n_edges, L, w, st, nullptr);
}

int set_error(int status, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return status;
}

int hip_error(hipError_t e, const char *what) { return hip_fail(e, what); }

bool fault_listed(const char *site) {
    const char *v = getenv("RB_FAULT");
    if (!v || !*v) return false;
    const size_t n = strlen(site);
    for (const char *p = v; *p;) {
        const char *q = strchr(p, ',');
        const size_t len = q ? (size_t)(q - p) : strlen(p);
        if (len == n && strncmp(p, site, n) == 0) return true;
        if (!q) break;
        p = q + 1;
    }
    return false;
}

int inject_fault(const char *site, const char *where) {
    if (!fault_listed(site)) return RB_OK;
    const rb_status s = strcmp(site, "alloc") == 0 ? RB_ENOMEM : RB_EHIP;
    return fail(s, "%s: injected failure (RB_FAULT=%s); nothing was enqueued", where, site);
}

void clear_error() { g_err.clear(); }

double occlusion_threshold(double d) {
    if (d <= 0.0) return -1.0;
    if (d < 1.0) return 0.0;
    if (d >= 4194304.0) return 17592186044416.0;   // d >= 2^22: T = 2^44 covers all
    double t = std::ceil(d * d) - 1.0;
    while (std::fma(d, d, -(t + 1.0)) > 0.0) t += 1.0;
    while (std::fma(d, d, -t) <= 0.0) t -= 1.0;
    return t;
}

int device_cu_count() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (g_cu_count[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            n <= 0)
            n = 256;
        g_cu_count[dev] = n;
    }
    return g_cu_count[dev];
}

bool ws_layout(int64_t n_nodes, int64_t n_edges, WsLayout *L) {
    if (n_nodes < 0 || n_nodes > kMaxNodes || n_edges < 0 || n_edges > kMaxEdges) return false;
    const int64_t V = n_nodes > 0 ? n_nodes : 1;
    const int64_t E = n_edges > 0 ? n_edges : 1;
    L->n_edge_pad = (int64_t)round_up((size_t)E, kRecPad);
    L->n_node_pad = (int64_t)round_up((size_t)V, kRecPad);
    int64_t h = 1024;
    while (h < 2 * E) h <<= 1;
    L->hash_size = h;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = round_up(off + bytes, 256);
        return o;
    };
    L->edge_rec = take(sizeof(EdgeRec) * (size_t)L->n_edge_pad);
    L->node_rec = take(sizeof(NodeRec) * (size_t)L->n_node_pad);
    L->partial = take(sizeof(CrossPartial) * (size_t)kMaxPartials);
    L->scalars = take(sizeof(Scalars));
    L->deg = take(sizeof(uint32_t) * (size_t)V);
    L->cursor = take(sizeof(uint32_t) * (size_t)V);
    L->offs = take(sizeof(uint32_t) * (size_t)(V + 1));
    L->angles = take(sizeof(double) * (size_t)(2 * E));
    L->nbr = take(sizeof(int32_t) * (size_t)(2 * E));
    L->dv = take(sizeof(double) * (size_t)V);
    L->big_list = take(sizeof(int32_t) * (size_t)V);
    L->hash = take(sizeof(unsigned long long) * (size_t)h);
    L->kacc = take(sizeof(int32_t) * (size_t)L->n_edge_pad);
    L->fwd = take(sizeof(Fwd));
    // hub order (rare-path pruning of large single-layout edge sweeps)
    const int64_t hs = n_edges >= kHubSortMinEdges ? E : 0;
    const int64_t n_hist = hs > 0 ? 256 * ((hs + kSortTile - 1) / kSortTile) : 0;
    L->hub_deg = take(hs > 0 ? sizeof(uint32_t) * (size_t)V : 0);
    L->hub_keys = take(sizeof(uint32_t) * (size_t)hs);
    L->hub_vals = take(sizeof(int32_t) * (size_t)hs);
    L->hub_keys2 = take(sizeof(uint32_t) * (size_t)hs);
    L->hub_vals2 = take(sizeof(int32_t) * (size_t)hs);
    L->hub_hist = take(sizeof(uint32_t) * (size_t)n_hist);
    L->hub_hist_off = take(hs > 0 ? sizeof(uint32_t) * (size_t)(n_hist + 1) : 0);
    L->hub_scan = take(hs > 0 ? sizeof(unsigned long long) * (size_t)((n_hist + 2047) / 2048 + 1)
                              : 0);
    L->total = off;
    return true;
}

// The hub-sort buffers of a workspace, or NULL where it has none.
static const HubSortBufs *hub_bufs(const WsLayout &L, char *w, int64_t n_edges,
                                   HubSortBufs *B) {
    if (n_edges < kHubSortMinEdges) return nullptr;
    B->deg = (uint32_t *)(w + L.hub_deg);
    B->keys = (uint32_t *)(w + L.hub_keys);
    B->vals = (int32_t *)(w + L.hub_vals);
    B->keys2 = (uint32_t *)(w + L.hub_keys2);
    B->vals2 = (int32_t *)(w + L.hub_vals2);
    B->hist = (uint32_t *)(w + L.hub_hist);
    B->hist_off = (uint32_t *)(w + L.hub_hist_off);
    B->scan_tile = (unsigned long long *)(w + L.hub_scan);
    return B;
}

}  // namespace rb

using namespace rb;

extern "C" {

const char *rb_version(void) { return "rb 1.0.0 gfx950"; }

const char *rb_last_error(void) { return g_err.c_str(); }

size_t rb_workspace_size(int64_t n_nodes, int64_t n_edges) {
    WsLayout L;
    if (!ws_layout(n_nodes, n_edges, &L)) return 0;
    return L.total;
}

static rb_status occlusion_launch(const float *x, const float *y, int64_t n_nodes,
                                  double diameter, uint64_t *out_count, NodeRec *rec,
                                  int64_t n_node_pad, OcclPartial *part, hipStream_t st,
                                  int timed_kind);

rb_status rb_node_occlusion(const float *x, const float *y, int64_t n_nodes, double diameter,
                            uint64_t *out_count, void *ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    rb_status s = check_sizes(n_nodes, 0);
    if (s) return s;
    if (n_nodes > 0 && (!x || !y)) return fail(RB_EINVAL, "x or y is NULL");
    if (!out_count) return fail(RB_EINVAL, "out_count is NULL");
    if (!(diameter >= 0.0) || !std::isfinite(diameter))
        return fail(RB_EINVAL, "diameter must be finite and >= 0");
    WsLayout L;
    if ((s = check_ws(ws, ws_bytes, n_nodes, 0, &L))) return s;
    if (const int f = inject_fault("launch", "rb_node_occlusion")) return (rb_status)f;
    if ((s = validate_if_requested(x, y, n_nodes, nullptr, nullptr, 0, L, (char *)ws,
                                   (hipStream_t)stream)))
        return s;
    char *w = (char *)ws;
    return occlusion_launch(x, y, n_nodes, diameter, out_count, (NodeRec *)(w + L.node_rec),
                            L.n_node_pad, (OcclPartial *)(w + L.partial), (hipStream_t)stream, 1);
}

// Node preparation, the all-pairs node sweep and its finalize into the given
// record (n_node_pad entries) and partial-slot (kMaxPartials) buffers; the
// sweep's launch is timed as `timed_kind`.
static rb_status occlusion_launch(const float *x, const float *y, int64_t n_nodes,
                                  double diameter, uint64_t *out_count, NodeRec *rec,
                                  int64_t n_node_pad, OcclPartial *part, hipStream_t st,
                                  int timed_kind) {
    if (const int f = inject_fault("launch", "rb_node_occlusion")) return (rb_status)f;
    const int v = tuned_variant(2, false, n_nodes);
    const int rows = occl_variant(v).rows, shift = occl_variant(v).col_shift;
    SweepArgs a;
    a.table = nullptr;
    a.single = sweep_layout(n_nodes, rows, 0, 0, shift);
    a.n_layouts = 1;
    a.n_units = sweep_units(n_nodes, rows, shift);
    a.unit_base = 0;
    const int grid = occl_grid(v, a.n_units, n_nodes);
    hipError_t e = launch_node_prep(x, y, n_nodes, n_node_pad, occlusion_threshold(diameter),
                                    rec, st);
    if (e != hipSuccess) return hip_fail(e, "node_prep launch");
    TimedLaunch tl(timed_kind, st);
    e = launch_occl_sweep(v, rec, a, grid, part, st);
    tl.done();
    if (e != hipSuccess) return hip_fail(e, "occlusion sweep launch");
    e = launch_occl_finalize(part, grid, (unsigned long long *)out_count, true, st);
    if (e != hipSuccess) return hip_fail(e, "occlusion finalize launch");
    return RB_OK;
}

static rb_status crossing_launch(const float *x, const float *y, int64_t n_nodes,
                                 const int32_t *src, const int32_t *dst, int64_t n_edges,
                                 bool angle, double ideal, uint64_t *out_count,
                                 uint64_t *out_proper, double *out_metric, double *out_dev_sum,
                                 EdgeRec *rec, int64_t n_edge_pad, CrossPartial *part,
                                 const HubSortBufs *hub, hipStream_t st);

static rb_status crossing_common(const float *x, const float *y, int64_t n_nodes,
                                 const int32_t *src, const int32_t *dst, int64_t n_edges,
                                 bool angle, double ideal, uint64_t *out_count,
                                 uint64_t *out_proper, double *out_metric, double *out_dev_sum,
                                 void *ws, size_t ws_bytes, void *stream) {
    rb_status s = check_layout(x, y, n_nodes, src, dst, n_edges);
    if (s) return s;
    WsLayout L;
    if ((s = check_ws(ws, ws_bytes, n_nodes, n_edges, &L))) return s;
    if (const int f = inject_fault("launch", "rb_edge_crossing / rb_crossing_angle")) return (rb_status)f;
    if ((s = validate_if_requested(x, y, n_nodes, src, dst, n_edges, L, (char *)ws,
                                   (hipStream_t)stream)))
        return s;
    char *w = (char *)ws;
    HubSortBufs hb;
    return crossing_launch(x, y, n_nodes, src, dst, n_edges, angle, ideal, out_count, out_proper,
                           out_metric, out_dev_sum, (EdgeRec *)(w + L.edge_rec), L.n_edge_pad,
                           (CrossPartial *)(w + L.partial), hub_bufs(L, w, n_edges, &hb),
                           (hipStream_t)stream);
}

// Edge preparation (in hub order when hub is not NULL), the all-pairs sweep
// and its finalize into caller-chosen record (n_edge_pad entries) and
// partial-slot (kMaxPartials) buffers.  The pairs and so the results do not
// depend on the record order, apart from the rounding of the angle sums.
static rb_status crossing_launch(const float *x, const float *y, int64_t n_nodes,
                                 const int32_t *src, const int32_t *dst, int64_t n_edges,
                                 bool angle, double ideal, uint64_t *out_count,
                                 uint64_t *out_proper, double *out_metric, double *out_dev_sum,
                                 EdgeRec *rec, int64_t n_edge_pad, CrossPartial *part,
                                 const HubSortBufs *hub, hipStream_t st) {
    if (const int f = inject_fault("launch", "rb_edge_crossing / rb_crossing_angle")) return (rb_status)f;
    const int v = tuned_variant(angle ? 1 : 0, false, n_edges);
    const int rows = cross_variant(v).rows;
    SweepArgs a;
    a.table = nullptr;
    a.single = sweep_layout(n_edges, rows, 0, 0);
    a.n_layouts = 1;
    a.n_units = sweep_units(n_edges, rows);
    a.unit_base = 0;
    const int grid = (int)std::min<int64_t>(a.n_units, cross_grid(v, angle));
    hipError_t e = hipSuccess;
    if (hub && (e = launch_hub_order(src, dst, n_nodes, n_edges, *hub, st)) != hipSuccess)
        return hip_fail(e, "hub order launch");
    e = launch_edge_prep_ordered(x, y, src, dst, n_nodes, n_edges, n_edge_pad,
                                 hub ? hub->vals : nullptr, rec, st);
    if (e != hipSuccess) return hip_fail(e, "edge_prep launch");
    TimedLaunch tl(0, st);
    e = launch_cross_sweep(v, angle, rec, a, grid, ideal, part, st);
    tl.done();
    if (e != hipSuccess) return hip_fail(e, "crossing sweep launch");
    e = launch_cross_finalize(part, grid, ideal, (unsigned long long *)out_count,
                              (unsigned long long *)out_proper, out_metric, out_dev_sum, st);
    if (e != hipSuccess) return hip_fail(e, "crossing finalize launch");
    return RB_OK;
}

// Tile-aligned, equal-work shard k of n of a single-layout unit list:
// row tiles [t_k, t_k+1) where t_k is the first tile whose preceding units
// reach ceil(k U / n).
static void shard_tiles(int64_t n_items, int rows, int col_shift, int64_t k, int64_t n,
                        int64_t *tile_b, int64_t *tile_e, int64_t *unit_b, int64_t *unit_e) {
    const SweepLayout l = sweep_layout(n_items, rows, 0, 0, col_shift);
    auto before = [&](int64_t I) {
        return I * l.n_chunks - ((int64_t)rows << col_shift) * I * (I - 1) / 2;
    };
    const int64_t U = before(l.n_row_tiles);
    auto first_tile = [&](int64_t q) {   // smallest I with before(I) >= ceil(q U / n)
        const int64_t target = (int64_t)(((__int128)q * U + n - 1) / n);
        int64_t lo = 0, hi = l.n_row_tiles;
        while (lo < hi) {
            const int64_t mid = (lo + hi) / 2;
            if (before(mid) >= target) hi = mid;
            else lo = mid + 1;
        }
        return lo;
    };
    *tile_b = first_tile(k);
    *tile_e = first_tile(k + 1);
    *unit_b = before(*tile_b);
    *unit_e = before(*tile_e);
}

rb_status rb_crossing_angle_shard(const float *x, const float *y, int64_t n_nodes,
                                  const int32_t *src, const int32_t *dst, int64_t n_edges,
                                  double ideal_angle, int64_t shard, int64_t n_shards,
                                  uint64_t *out_count, double *out_dev_sum, int64_t *out_row_begin,
                                  int64_t *out_row_end, void *ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    rb_status s = check_layout(x, y, n_nodes, src, dst, n_edges);
    if (s) return s;
    if (!out_count) return fail(RB_EINVAL, "out_count is NULL");
    if (!(ideal_angle > 0.0) || !(ideal_angle <= 1.5707963267948966))
        return fail(RB_EINVAL, "ideal_angle must be in (0, pi/2]");
    if (n_shards < 1 || shard < 0 || shard >= n_shards)
        return fail(RB_EINVAL, "need 0 <= shard < n_shards");
    WsLayout L;
    if ((s = check_ws(ws, ws_bytes, n_nodes, n_edges, &L))) return s;
    if (const int f = inject_fault("launch", "rb_crossing_angle_shard")) return (rb_status)f;
    if ((s = validate_if_requested(x, y, n_nodes, src, dst, n_edges, L, (char *)ws,
                                   (hipStream_t)stream)))
        return s;
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)ws;
    EdgeRec *rec = (EdgeRec *)(w + L.edge_rec);
    CrossPartial *part = (CrossPartial *)(w + L.partial);
    const int v = tuned_variant(1, false, n_edges);
    const int rows = cross_variant(v).rows;
    int64_t tb, te, ub, ue;
    shard_tiles(n_edges, rows, 0, shard, n_shards, &tb, &te, &ub, &ue);
    const int64_t R = (int64_t)kBlock * rows;
    if (out_row_begin) *out_row_begin = std::min<int64_t>(tb * R, n_edges);
    if (out_row_end) *out_row_end = std::min<int64_t>(te * R, n_edges);
    SweepArgs a;
    a.table = nullptr;
    a.single = sweep_layout(n_edges, rows, 0, 0);
    a.n_layouts = 1;
    a.n_units = ue - ub;
    a.unit_base = ub;
    const int grid = (int)std::min<int64_t>(a.n_units, cross_grid(v, true));
    hipError_t e = launch_edge_prep(x, y, src, dst, n_nodes, n_edges, L.n_edge_pad, rec, st);
    if (e != hipSuccess) return hip_fail(e, "edge_prep launch");
    if (grid > 0) {
        e = launch_cross_sweep(v, true, rec, a, grid, ideal_angle, part, st);
        if (e != hipSuccess) return hip_fail(e, "crossing sweep launch");
    }
    e = launch_cross_finalize(part, grid, ideal_angle, (unsigned long long *)out_count, nullptr,
                              nullptr, out_dev_sum, st);
    if (e != hipSuccess) return hip_fail(e, "crossing finalize launch");
    return RB_OK;
}

rb_status rb_node_occlusion_shard(const float *x, const float *y, int64_t n_nodes,
                                  double diameter, int64_t shard, int64_t n_shards,
                                  uint64_t *out_count, int64_t *out_row_begin,
                                  int64_t *out_row_end, void *ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    rb_status s = check_sizes(n_nodes, 0);
    if (s) return s;
    if (n_nodes > 0 && (!x || !y)) return fail(RB_EINVAL, "x or y is NULL");
    if (!out_count) return fail(RB_EINVAL, "out_count is NULL");
    if (!(diameter >= 0.0) || !std::isfinite(diameter))
        return fail(RB_EINVAL, "diameter must be finite and >= 0");
    if (n_shards < 1 || shard < 0 || shard >= n_shards)
        return fail(RB_EINVAL, "need 0 <= shard < n_shards");
    WsLayout L;
    if ((s = check_ws(ws, ws_bytes, n_nodes, 0, &L))) return s;
    if (const int f = inject_fault("launch", "rb_node_occlusion_shard")) return (rb_status)f;
    if ((s = validate_if_requested(x, y, n_nodes, nullptr, nullptr, 0, L, (char *)ws,
                                   (hipStream_t)stream)))
        return s;
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)ws;
    NodeRec *rec = (NodeRec *)(w + L.node_rec);
    OcclPartial *part = (OcclPartial *)(w + L.partial);
    const int v = tuned_variant(2, false, n_nodes);
    const int rows = occl_variant(v).rows, shift = occl_variant(v).col_shift;
    int64_t tb, te, ub, ue;
    shard_tiles(n_nodes, rows, shift, shard, n_shards, &tb, &te, &ub, &ue);
    const int64_t R = (int64_t)kBlock * rows;
    if (out_row_begin) *out_row_begin = std::min<int64_t>(tb * R, n_nodes);
    if (out_row_end) *out_row_end = std::min<int64_t>(te * R, n_nodes);
    SweepArgs a;
    a.table = nullptr;
    a.single = sweep_layout(n_nodes, rows, 0, 0, shift);
    a.n_layouts = 1;
    a.n_units = ue - ub;
    a.unit_base = ub;
    const int grid = occl_grid(v, a.n_units, n_nodes);
    hipError_t e = launch_node_prep(x, y, n_nodes, L.n_node_pad, occlusion_threshold(diameter),
                                    rec, st);
    if (e != hipSuccess) return hip_fail(e, "node_prep launch");
    if (grid > 0) {
        e = launch_occl_sweep(v, rec, a, grid, part, st);
        if (e != hipSuccess) return hip_fail(e, "occlusion sweep launch");
    }
    e = launch_occl_finalize(part, grid, (unsigned long long *)out_count, true, st);
    if (e != hipSuccess) return hip_fail(e, "occlusion finalize launch");
    return RB_OK;
}

size_t rb_grid_workspace_size(int64_t n_nodes, int64_t n_edges) {
    GridWs G;
    if (!grid_ws_layout(n_nodes, n_edges, &G)) return 0;
    return G.total;
}

rb_status rb_node_occlusion_grid(const float *x, const float *y, int64_t n_nodes,
                                 double diameter, uint64_t *out_count, void *ws,
                                 size_t ws_bytes, void *stream) {
    g_err.clear();
    rb_status s = check_sizes(n_nodes, 0);
    if (s) return s;
    if (n_nodes > 0 && (!x || !y)) return fail(RB_EINVAL, "x or y is NULL");
    if (!out_count) return fail(RB_EINVAL, "out_count is NULL");
    if (!(diameter >= 0.0) || !std::isfinite(diameter))
        return fail(RB_EINVAL, "diameter must be finite and >= 0");
    GridWs G;
    if (!grid_ws_layout(n_nodes, 0, &G)) return fail(RB_EINVAL, "layout too large");
    if (!ws) return fail(RB_EWORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws & 255u) != 0) return fail(RB_EWORKSPACE, "workspace not 256-byte aligned");
    if (ws_bytes < G.total)
        return fail(RB_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, G.total);
    if (const int f = inject_fault("launch", "rb_node_occlusion_grid")) return (rb_status)f;
    hipStream_t st = (hipStream_t)stream;
    if (n_nodes < kGridMinNodes) {     // the sweep costs less than the grid's passes
        const int64_t pad = (std::max<int64_t>(n_nodes, 1) + kRecPad - 1) / kRecPad * kRecPad;
        return occlusion_launch(x, y, n_nodes, diameter, out_count,
                                (NodeRec *)((char *)ws + G.node_rec), pad,
                                (OcclPartial *)((char *)ws + G.partial), st, 2);
    }
    TimedLaunch tl(2, st);
    hipError_t e = launch_occlusion_grid(x, y, n_nodes, occlusion_threshold(diameter), G,
                                         (char *)ws, (unsigned long long *)out_count, st);
    tl.done();
    if (e != hipSuccess) return hip_fail(e, "grid occlusion launch");
    return RB_OK;
}

rb_status rb_crossing_angle_pruned(const float *x, const float *y, int64_t n_nodes,
                                   const int32_t *src, const int32_t *dst, int64_t n_edges,
                                   double ideal_angle, double *out_metric, uint64_t *out_count,
                                   double *out_dev_sum, void *ws, size_t ws_bytes,
                                   void *stream) {
    g_err.clear();
    rb_status s = check_layout(x, y, n_nodes, src, dst, n_edges);
    if (s) return s;
    if (!out_metric) return fail(RB_EINVAL, "out_metric is NULL");
    if (!(ideal_angle > 0.0) || !(ideal_angle <= 1.5707963267948966))
        return fail(RB_EINVAL, "ideal_angle must be in (0, pi/2]");
    if (n_edges > kMaxPrunedEdges)
        return fail(RB_EINVAL, "n_edges = %lld above the pruned path's limit 2^24",
                    (long long)n_edges);
    GridWs G;
    if (!grid_ws_layout(n_nodes, n_edges, &G)) return fail(RB_EINVAL, "layout too large");
    if (!ws) return fail(RB_EWORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws & 255u) != 0) return fail(RB_EWORKSPACE, "workspace not 256-byte aligned");
    if (ws_bytes < G.total)
        return fail(RB_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, G.total);
    if (const int f = inject_fault("launch", "rb_crossing_angle_pruned")) return (rb_status)f;
    hipStream_t st = (hipStream_t)stream;
    const int v = tuned_variant(3, false, n_edges);
    TimedLaunch tl(3, st);
    hipError_t e = launch_crossing_pruned(x, y, n_nodes, src, dst, n_edges, ideal_angle, G,
                                          (char *)ws, v, out_metric,
                                          (unsigned long long *)out_count, out_dev_sum, st);
    tl.done();
    if (e != hipSuccess) return hip_fail(e, "pruned crossing launch");
    return RB_OK;
}

rb_status rb_edge_crossing(const float *x, const float *y, int64_t n_nodes, const int32_t *src,
                           const int32_t *dst, int64_t n_edges, uint64_t *out_count,
                           uint64_t *out_proper, void *ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    if (!out_count) return fail(RB_EINVAL, "out_count is NULL");
    return crossing_common(x, y, n_nodes, src, dst, n_edges, false, 1.0, out_count, out_proper,
                           nullptr, nullptr, ws, ws_bytes, stream);
}

rb_status rb_crossing_angle(const float *x, const float *y, int64_t n_nodes, const int32_t *src,
                            const int32_t *dst, int64_t n_edges, double ideal_angle,
                            double *out_metric, uint64_t *out_count, double *out_dev_sum,
                            void *ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    if (!out_metric) return fail(RB_EINVAL, "out_metric is NULL");
    if (!(ideal_angle > 0.0) || !(ideal_angle <= 1.5707963267948966))
        return fail(RB_EINVAL, "ideal_angle must be in (0, pi/2]");
    return crossing_common(x, y, n_nodes, src, dst, n_edges, true, ideal_angle, out_count,
                           nullptr, out_metric, out_dev_sum, ws, ws_bytes, stream);
}

}  // extern "C"

// ------------------------------------------------ allocation-free variant
// rb_crossing_angle_noalloc keeps the edge records and the sweep's partial
// slots in this file-scope device array instead of a caller workspace.  In
// host code the array's name only stands in for the symbol: kernels get the
// device address that hipGetSymbolAddress returns, looked up once per device.
namespace rb {

constexpr int64_t kNoAllocMaxEdges = 1000000;
constexpr int64_t kNoAllocEdgePad = (kNoAllocMaxEdges + kRecPad - 1) / kRecPad * kRecPad;
constexpr size_t kNoAllocRecBytes = sizeof(EdgeRec) * (size_t)kNoAllocEdgePad;
constexpr size_t kNoAllocBytes = kNoAllocRecBytes + sizeof(CrossPartial) * (size_t)kMaxPartials;
static_assert(kNoAllocRecBytes % 256 == 0, "the partial slots start 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

std::mutex g_scratch_mu;
char *g_scratch_ptr[64];

// Device address of `scratch` on the current device.
rb_status scratch_address(char **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return fail(RB_EINVAL, "device %d: only devices 0..63", dev);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p || ((uintptr_t)p & 255u) != 0)
            return fail(RB_EHIP, "static scratch is not 256-byte aligned");
        g_scratch_ptr[dev] = (char *)p;
    }
    *out = g_scratch_ptr[dev];
    return RB_OK;
}

}  // namespace
}  // namespace rb

extern "C" {

rb_status rb_crossing_angle_noalloc(const float *x, const float *y, int64_t n_nodes,
                                    const int32_t *src, const int32_t *dst, int64_t n_edges,
                                    double ideal_angle, double *out_metric, uint64_t *out_count,
                                    double *out_dev_sum, void *stream) {
    g_err.clear();
    if (!out_metric) return fail(RB_EINVAL, "out_metric is NULL");
    if (!(ideal_angle > 0.0) || !(ideal_angle <= 1.5707963267948966))
        return fail(RB_EINVAL, "ideal_angle must be in (0, pi/2]");
    rb_status s = check_layout(x, y, n_nodes, src, dst, n_edges);
    if (s) return s;
    if (n_edges > kNoAllocMaxEdges)
        return fail(RB_EINVAL, "n_edges = %lld exceeds the %lld edges the static scratch holds",
                    (long long)n_edges, (long long)kNoAllocMaxEdges);
    if (const int f = inject_fault("launch", "rb_crossing_angle_noalloc")) return (rb_status)f;
    char *w = nullptr;
    if ((s = scratch_address(&w))) return s;
    const int64_t pad = (int64_t)round_up((size_t)std::max<int64_t>(n_edges, 1), kRecPad);
    return crossing_launch(x, y, n_nodes, src, dst, n_edges, true, ideal_angle, out_count,
                           nullptr, out_metric, out_dev_sum, (EdgeRec *)w, pad,
                           (CrossPartial *)(w + kNoAllocRecBytes), nullptr, (hipStream_t)stream);
}

rb_status rb_min_angle(const float *x, const float *y, int64_t n_nodes, const int32_t *src,
                       const int32_t *dst, int64_t n_edges, double *out_metric,
                       double *out_sum_dv, uint64_t *out_n_used, void *ws, size_t ws_bytes,
                       void *stream) {
    g_err.clear();
    rb_status s = check_layout(x, y, n_nodes, src, dst, n_edges);
    if (s) return s;
    if (!out_metric) return fail(RB_EINVAL, "out_metric is NULL");
    WsLayout L;
    if ((s = check_ws(ws, ws_bytes, n_nodes, n_edges, &L))) return s;
    if (const int f = inject_fault("launch", "rb_min_angle")) return (rb_status)f;
    if ((s = validate_if_requested(x, y, n_nodes, src, dst, n_edges, L, (char *)ws,
                                   (hipStream_t)stream)))
        return s;
    hipError_t e = launch_min_angle(x, y, n_nodes, src, dst, n_edges,
                                    min_angle_bufs(L, (char *)ws), out_metric, out_sum_dv,
                                    (unsigned long long *)out_n_used, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "min_angle launch");
    return RB_OK;
}

rb_status rb_edge_length_variation(const float *x, const float *y, int64_t n_nodes,
                                   const int32_t *src, const int32_t *dst, int64_t n_edges,
                                   double *out_metric, double *out_mean, void *ws,
                                   size_t ws_bytes, void *stream) {
    g_err.clear();
    rb_status s = check_layout(x, y, n_nodes, src, dst, n_edges);
    if (s) return s;
    if (!out_metric) return fail(RB_EINVAL, "out_metric is NULL");
    WsLayout L;
    if ((s = check_ws(ws, ws_bytes, n_nodes, n_edges, &L))) return s;
    if (const int f = inject_fault("launch", "rb_edge_length_variation")) return (rb_status)f;
    if ((s = validate_if_requested(x, y, n_nodes, src, dst, n_edges, L, (char *)ws,
                                   (hipStream_t)stream)))
        return s;
    char *w = (char *)ws;
    hipError_t e = launch_elv(x, y, src, dst, n_nodes, n_edges, (double *)(w + L.partial),
                              (Scalars *)(w + L.scalars), out_metric, out_mean,
                              (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "edge_length_variation launch");
    return RB_OK;
}

rb_status rb_loss_grad(const float *x, const float *y, int64_t n_nodes, const int32_t *src,
                       const int32_t *dst, int64_t n_edges, double ideal_angle, double w_angle,
                       double w_length, double w_min_angle, double *out_loss, double *out_grad_x,
                       double *out_grad_y, uint64_t *out_count, void *ws, size_t ws_bytes,
                       void *stream) {
    g_err.clear();
    rb_status s = check_layout(x, y, n_nodes, src, dst, n_edges);
    if (s) return s;
    if (!out_loss || (n_nodes > 0 && (!out_grad_x || !out_grad_y)))
        return fail(RB_EINVAL, "out_loss, out_grad_x or out_grad_y is NULL");
    if (!(ideal_angle > 0.0) || !(ideal_angle <= 1.5707963267948966))
        return fail(RB_EINVAL, "ideal_angle must be in (0, pi/2]");
    if (!std::isfinite(w_angle) || !std::isfinite(w_length) || !std::isfinite(w_min_angle))
        return fail(RB_EINVAL, "weights must be finite");
    WsLayout L;
    if ((s = check_ws(ws, ws_bytes, n_nodes, n_edges, &L))) return s;
    if (const int f = inject_fault("launch", "rb_loss_grad")) return (rb_status)f;
    if ((s = validate_if_requested(x, y, n_nodes, src, dst, n_edges, L, (char *)ws,
                                   (hipStream_t)stream)))
        return s;
    hipError_t e = launch_loss_grad(x, y, n_nodes, src, dst, n_edges, ideal_angle, w_angle,
                                    w_length, w_min_angle, out_loss, out_grad_x, out_grad_y,
                                    (unsigned long long *)out_count, L, (char *)ws,
                                    (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "rb_loss_grad launch");
    return RB_OK;
}

rb_status rb_loss_grad_pruned(const float *x, const float *y, int64_t n_nodes,
                              const int32_t *src, const int32_t *dst, int64_t n_edges,
                              double ideal_angle, double w_angle, double w_length,
                              double w_min_angle, double *out_loss, double *out_grad_x,
                              double *out_grad_y, uint64_t *out_count, void *ws, size_t ws_bytes,
                              void *stream) {
    g_err.clear();
    rb_status s = check_layout(x, y, n_nodes, src, dst, n_edges);
    if (s) return s;
    if (!out_loss || (n_nodes > 0 && (!out_grad_x || !out_grad_y)))
        return fail(RB_EINVAL, "out_loss, out_grad_x or out_grad_y is NULL");
    if (!(ideal_angle > 0.0) || !(ideal_angle <= 1.5707963267948966))
        return fail(RB_EINVAL, "ideal_angle must be in (0, pi/2]");
    if (!std::isfinite(w_angle) || !std::isfinite(w_length) || !std::isfinite(w_min_angle))
        return fail(RB_EINVAL, "weights must be finite");
    if (n_edges > kMaxPrunedEdges)
        return fail(RB_EINVAL, "n_edges = %lld above the pruned path's limit 2^24",
                    (long long)n_edges);
    GridWs G;
    if (!grid_ws_layout(n_nodes, n_edges, &G)) return fail(RB_EINVAL, "layout too large");
    if (!ws) return fail(RB_EWORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws & 255u) != 0) return fail(RB_EWORKSPACE, "workspace not 256-byte aligned");
    if (ws_bytes < G.total)
        return fail(RB_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, G.total);
    if (const int f = inject_fault("launch", "rb_loss_grad_pruned")) return (rb_status)f;
    hipError_t e = launch_loss_grad_pruned(x, y, n_nodes, src, dst, n_edges, ideal_angle,
                                           w_angle, w_length, w_min_angle, out_loss, out_grad_x,
                                           out_grad_y,
                                           (unsigned long long *)out_count, G, (char *)ws,
                                           (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "rb_loss_grad_pruned launch");
    return RB_OK;
}

size_t rb_enhanced_workspace_size(int64_t n_edges, uint64_t n_pieces) {
    if (n_edges < 0 || n_edges > kMaxEdges || n_pieces >= (1ull << 32)) return 0;
    return strip_ws_bytes(n_edges, (int64_t)n_pieces);
}

rb_status rb_enhanced_crossing(const float *x, const float *y, int64_t n_nodes,
                               const int32_t *src, const int32_t *dst, int64_t n_edges,
                               int64_t width, int horizontal, double ideal_angle,
                               double *out_metric, uint64_t *out_count, double *out_dev_sum,
                               uint64_t *out_pieces, void *ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    rb_status s = check_layout(x, y, n_nodes, src, dst, n_edges);
    if (s) return s;
    if (!out_metric) return fail(RB_EINVAL, "out_metric is NULL");
    if (width < 1 || width > (1ll << 22)) return fail(RB_EINVAL, "width must be in [1, 2^22]");
    if (!(ideal_angle > 0.0) || !(ideal_angle <= 1.5707963267948966))
        return fail(RB_EINVAL, "ideal_angle must be in (0, pi/2]");
    if (!ws) return fail(RB_EWORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws & 255u) != 0) return fail(RB_EWORKSPACE, "workspace not 256-byte aligned");
    if (ws_bytes < strip_ws_bytes(n_edges, 0))
        return fail(RB_EWORKSPACE, "workspace of %zu bytes, %zu needed to count pieces", ws_bytes,
                    strip_ws_bytes(n_edges, 0));
    if (const int f = inject_fault("launch", "rb_enhanced_crossing")) return (rb_status)f;
    hipStream_t st = (hipStream_t)stream;
    const float *px = horizontal ? y : x, *py = horizontal ? x : y;   // strips across x
    hipError_t e = launch_strip_count(px, py, src, dst, n_nodes, n_edges, width, (char *)ws, st);
    if (e != hipSuccess) return hip_fail(e, "strip count launch");
    unsigned long long P = 0;
    e = hipMemcpyAsync(&P, strip_total_ptr((const char *)ws), sizeof P, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "piece count copy");
    if (out_pieces) *out_pieces = P;
    if (P >= (1ull << 32))
        return fail(RB_EINVAL, "%llu strip pieces: widen the strips", (unsigned long long)P);
    const size_t need = strip_ws_bytes(n_edges, (int64_t)P);
    if (ws_bytes < need)
        return fail(RB_EWORKSPACE, "workspace of %zu bytes, %zu needed for %llu pieces", ws_bytes,
                    need, (unsigned long long)P);
    TimedLaunch tl(3, st);
    e = launch_strip_crossing(px, py, src, dst, n_nodes, n_edges, width, (int64_t)P, ideal_angle,
                              (char *)ws, out_metric, (unsigned long long *)out_count, out_dev_sum,
                              st);
    tl.done();
    if (e != hipSuccess) return hip_fail(e, "strip crossing launch");
    return RB_OK;
}

rb_status rb_validate_layout(const float *x, const float *y, int64_t n_nodes, const int32_t *src,
                             const int32_t *dst, int64_t n_edges, int32_t *out_flags, void *ws,
                             size_t ws_bytes, void *stream) {
    g_err.clear();
    rb_status s = check_layout(x, y, n_nodes, src, dst, n_edges);
    if (s) return s;
    WsLayout L;
    if ((s = check_ws(ws, ws_bytes, n_nodes, n_edges, &L))) return s;
    if (const int f = inject_fault("launch", "rb_validate_layout")) return (rb_status)f;
    return validate_now(x, y, n_nodes, src, dst, n_edges, L, (char *)ws, (hipStream_t)stream,
                        out_flags);
}

rb_status rb_autotune(const float *x, const float *y, int64_t n_nodes, const int32_t *src,
                      const int32_t *dst, int64_t n_edges, double diameter, double ideal_angle,
                      int repeats, double *out_best_ms, void *ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    rb_status s = check_layout(x, y, n_nodes, src, dst, n_edges);
    if (s) return s;
    if (!(diameter >= 0.0) || !std::isfinite(diameter))
        return fail(RB_EINVAL, "diameter must be finite and >= 0");
    if (!(ideal_angle > 0.0) || !(ideal_angle <= 1.5707963267948966))
        return fail(RB_EINVAL, "ideal_angle must be in (0, pi/2]");
    if (repeats < 1 || repeats > 1000) return fail(RB_EINVAL, "repeats must be in [1, 1000]");
    WsLayout L;
    if ((s = check_ws(ws, ws_bytes, n_nodes, n_edges, &L))) return s;
    if (const int f = inject_fault("launch", "rb_autotune")) return (rb_status)f;
    if ((s = validate_if_requested(x, y, n_nodes, src, dst, n_edges, L, (char *)ws,
                                   (hipStream_t)stream)))
        return s;
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)ws;
    EdgeRec *erec = (EdgeRec *)(w + L.edge_rec);
    NodeRec *nrec = (NodeRec *)(w + L.node_rec);
    hipError_t e = launch_edge_prep(x, y, src, dst, n_nodes, n_edges, L.n_edge_pad, erec, st);
    if (e == hipSuccess)
        e = launch_node_prep(x, y, n_nodes, L.n_node_pad, occlusion_threshold(diameter), nrec, st);
    if (e != hipSuccess) return hip_fail(e, "autotune prep");
    hipEvent_t ea, eb;
    if ((e = hipEventCreate(&ea)) != hipSuccess) return hip_fail(e, "autotune event");
    if ((e = hipEventCreate(&eb)) != hipSuccess) {
        (void)hipEventDestroy(ea);
        return hip_fail(e, "autotune event");
    }
    auto timed = [&](auto &&launch, float *ms) -> hipError_t {
        hipError_t r = launch();                    // untimed: first-launch costs
        if (r != hipSuccess) return r;
        if ((r = hipEventRecord(ea, st)) != hipSuccess) return r;
        for (int k = 0; k < repeats && r == hipSuccess; ++k) r = launch();
        if (r != hipSuccess) return r;
        if ((r = hipEventRecord(eb, st)) != hipSuccess) return r;
        if ((r = hipEventSynchronize(eb)) != hipSuccess) return r;
        if ((r = hipEventElapsedTime(ms, ea, eb)) != hipSuccess) return r;
        *ms /= repeats;
        return hipSuccess;
    };
    double best_total = 0.0;
    for (int kind = 0; kind < 3 && e == hipSuccess; ++kind) {
        const bool occl = kind == 2, angle = kind == 1;
        const int nv = occl ? kOcclVariants : kCrossVariants;
        const int64_t n = occl ? n_nodes : n_edges;
        int best = -1;
        float best_ms = 0.f;
        for (int v = 0; v < nv && e == hipSuccess; ++v) {
            const SweepVariant sv = occl ? occl_variant(v) : cross_variant(v);
            SweepArgs a;
            a.table = nullptr;
            a.single = sweep_layout(n, sv.rows, 0, 0, sv.col_shift);
            a.n_layouts = 1;
            a.n_units = sweep_units(n, sv.rows, sv.col_shift);
            a.unit_base = 0;
            const int grid = occl ? occl_grid(v, a.n_units, n)
                                  : (int)std::min<int64_t>(a.n_units, cross_grid(v, angle));
            float ms = 0.f;
            if (occl)
                e = timed([&] { return launch_occl_sweep(v, nrec, a, grid, (OcclPartial *)(w + L.partial), st); }, &ms);
            else
                e = timed([&] { return launch_cross_sweep(v, angle, erec, a, grid, ideal_angle, (CrossPartial *)(w + L.partial), st); }, &ms);
            if (e == hipSuccess && (best < 0 || ms < best_ms)) {
                best = v;
                best_ms = ms;
            }
        }
        if (e == hipSuccess) {
            set_tuned_variant(kind, false, n, best);
            best_total += best_ms;
        }
    }
    (void)hipEventDestroy(ea);
    (void)hipEventDestroy(eb);
    if (e != hipSuccess) return hip_fail(e, "autotune");
    if (out_best_ms) *out_best_ms = best_total;
    return RB_OK;
}

rb_status rb_tune_set(int kind, int batch, int64_t n_items, int variant) {
    g_err.clear();
    if (kind < 0 || kind > 3) return fail(RB_EINVAL, "kind must be 0, 1, 2 or 3");
    if (n_items < 0) return fail(RB_EINVAL, "n_items must be >= 0");
    const int nv = kind == 2 ? kOcclVariants : kCrossVariants;
    if (variant < 0 || variant >= nv) return fail(RB_EINVAL, "variant must be in [0, %d)", nv);
    if (!variant_offered(kind, batch != 0, variant))
        return fail(RB_EINVAL, "variant %d is not offered for batched crossing sweeps", variant);
    set_tuned_variant(kind, batch != 0, n_items, variant);
    return RB_OK;
}

rb_status rb_tune_query(int kind, int batch, int64_t n_items, int *rows, int *waves,
                        int *col_split) {
    g_err.clear();
    if (kind < 0 || kind > 3) return fail(RB_EINVAL, "kind must be 0, 1, 2 or 3");
    if (n_items < 0) return fail(RB_EINVAL, "n_items must be >= 0");
    const int v = tuned_variant(kind, batch != 0, n_items);
    const SweepVariant sv = kind == 2 ? occl_variant(v) : cross_variant(v);
    if (rows) *rows = sv.rows;
    if (waves) *waves = sv.waves;
    if (col_split) *col_split = 1 << sv.col_shift;
    return RB_OK;
}

rb_status rb_tune_save(const char *path) {
    g_err.clear();
    if (!path) return fail(RB_EINVAL, "path is NULL");
    if (!save_tuning(path)) return fail(RB_EINVAL, "cannot write %s", path);
    return RB_OK;
}

rb_status rb_tune_load(const char *path) {
    g_err.clear();
    if (!path) return fail(RB_EINVAL, "path is NULL");
    if (!load_tuning(path)) return fail(RB_EINVAL, "cannot read %s", path);
    return RB_OK;
}

rb_status rb_timing_enable(int enable) {
    std::lock_guard<std::mutex> g(g_timing.mu);
    g_timing.on = enable != 0;
    return RB_OK;
}

rb_status rb_timing_reset(void) {
    std::lock_guard<std::mutex> g(g_timing.mu);
    for (int k = 0; k < kTimedKinds; ++k) {
        for (auto &p : g_timing.ev[k]) {
            (void)hipEventDestroy(p.first);
            (void)hipEventDestroy(p.second);
        }
        g_timing.ev[k].clear();
        g_timing.ms[k] = 0.0;
        g_timing.n[k] = 0;
    }
    return RB_OK;
}

rb_status rb_valu_probe(int iters, int repeats, double *out_lane_ops_per_s, double *sink,
                        void *stream) {
    g_err.clear();
    if (iters < 1 || iters > (1 << 24) || repeats < 1 || repeats > 1000)
        return fail(RB_EINVAL, "iters must be in [1, 2^24] and repeats in [1, 1000]");
    if (!out_lane_ops_per_s || !sink) return fail(RB_EINVAL, "out_lane_ops_per_s or sink is NULL");
    if (const int f = inject_fault("launch", "rb_valu_probe")) return (rb_status)f;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double ops = 0.0;
    hipError_t e = launch_valu_probe(iters, sink, &ops, st);          // untimed first launch
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int r = 0; r < repeats && e == hipSuccess; ++r) e = launch_valu_probe(iters, sink, nullptr, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "rb_valu_probe");
    *out_lane_ops_per_s = ms > 0.f ? ops * repeats / (ms * 1e-3) : 0.0;
    return RB_OK;
}

rb_status rb_timing_read(int kernel, double *total_ms, int64_t *launches) {
    g_err.clear();
    if (kernel < 0 || kernel >= kTimedKinds)
        return fail(RB_EINVAL, "kernel must be in 0 .. %d", kTimedKinds - 1);
    std::lock_guard<std::mutex> g(g_timing.mu);
    for (auto &p : g_timing.ev[kernel]) {
        hipError_t e = hipEventSynchronize(p.second);
        if (e != hipSuccess) return hip_fail(e, "timing event");
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, p.first, p.second);
        if (e != hipSuccess) return hip_fail(e, "timing elapsed");
        g_timing.ms[kernel] += ms;
        g_timing.n[kernel] += 1;
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    g_timing.ev[kernel].clear();
    if (total_ms) *total_ms = g_timing.ms[kernel];
    if (launches) *launches = g_timing.n[kernel];
    return RB_OK;
}

}  // extern "C"
