// Batched evaluation: the five metrics of many layouts of uneven size with
// one launch per all-pairs sweep, capturable into a hipGraph.
//
// The layouts are concatenated (node and edge arrays with offsets; edge ends
// stay local to their layout).  Every layout gets a record segment padded to
// kRecPad, and the units of all layouts' pair triangles form one list
// (SweepLayout table in the workspace), which one launch splits into equal
// contiguous ranges, one per block.  Per-layout results are combined from
// per-(block, layout) partial slots in a fixed order, one finalize block per
// layout.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "rb.h"
#include "rb_device.h"
#include "rb_internal.h"

using namespace rb;

struct rb_batch {
    int64_t B = 0;
    std::vector<int64_t> node_off, edge_off;      // B + 1, into the concatenated arrays
    std::vector<int64_t> erec_off, nrec_off;      // B + 1, record segments
    std::vector<double> T;                        // occlusion threshold per layout
    int cross_var = 1, occl_var = 0;
    // set by upload: unit counts and grid sizes of the two sweeps
    int64_t cross_units = 0, occl_units = 0;
    int cross_grid_n = 1, occl_grid_n = 1;
    // workspace carve (byte offsets, 256-aligned)
    size_t o_erec = 0, o_nrec = 0, o_ctab = 0, o_otab = 0, o_noff = 0, o_eoff = 0, o_ereco = 0,
           o_nreco = 0, o_T = 0, o_cpart = 0, o_opart = 0, o_deg = 0, o_cursor = 0, o_offs = 0,
           o_ang = 0, o_dv = 0, o_big = 0, o_sc = 0, total = 0;
    int64_t n_nodes = 0, n_edges = 0;
    const void *uploaded = nullptr;               // workspace holding the current tables
    // incremented by every upload (rb_batch_upload, rb_batch_autotune): a
    // graph captured under another generation walks tables that no longer
    // match the kernels and grid it recorded, and is refused
    uint64_t plan_gen = 0;
    // second stream (default priority) for the metrics that overlap the edge
    // sweep, and the fork / join events; made on first use, on the device of
    // that call
    mutable hipStream_t side = nullptr;
    mutable hipEvent_t fork = nullptr, join = nullptr;
    mutable int side_device = -1;
    ~rb_batch() {
        if (join) (void)hipEventDestroy(join);
        if (fork) (void)hipEventDestroy(fork);
        if (side) (void)hipStreamDestroy(side);
    }
};

struct rb_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const rb_batch *batch = nullptr;              // the plan it was captured from ...
    uint64_t plan_gen = 0;                        // ... and that plan's generation
};

namespace rb {
namespace {

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// first block whose unit range contains unit u (blocks own [U*b/G, U*(b+1)/G))
__device__ __forceinline__ int64_t block_of_unit(int64_t U, int64_t G, int64_t u) {
    int64_t b = (u * G) / U;
    while (b + 1 < G && block_first_unit(U, G, b + 1) <= u) ++b;
    while (b > 0 && block_first_unit(U, G, b) > u) --b;
    return b;
}

__global__ __launch_bounds__(256) void batch_edge_prep_kernel(
    const float *__restrict__ x, const float *__restrict__ y, const int32_t *__restrict__ src,
    const int32_t *__restrict__ dst, const int64_t *__restrict__ noff,
    const int64_t *__restrict__ eoff, const int64_t *__restrict__ ereco, int64_t B,
    int64_t n_rec, EdgeRec *__restrict__ rec) {
    for (int64_t slot = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; slot < n_rec;
         slot += (int64_t)gridDim.x * blockDim.x) {
        const int64_t L = dev::owner(ereco, B, slot);
        const int64_t k = slot - ereco[L];
        const int64_t nV = noff[L + 1] - noff[L];
        EdgeRec r;
        bool real = false;
        if (k < eoff[L + 1] - eoff[L]) {
            const int64_t e = eoff[L] + k;
            const int32_t s = src[e], t = dst[e];
            if (dev::valid_ids(s, t, nV)) {
                const int64_t gs = noff[L] + s, gt = noff[L] + t;
                const double px = x[gs], py = y[gs];
                const double dx = (double)x[gt] - px, dy = (double)y[gt] - py;
                r.x = px; r.y = py; r.dx = dx; r.dy = dy;
                r.c = fma(dx, py, -(dy * px));
                const bool flip = (dy < 0.0) | ((dy == 0.0) & (dx < 0.0));
                r.th = atan2(flip ? -dy : dy, flip ? -dx : dx);
                r.s = (int32_t)gs;
                r.t = (int32_t)gt;
                real = true;
            }
        }
        if (!real) {
            r.x = 0.0; r.y = 0.0; r.dx = 0.0; r.dy = 0.0; r.c = -1.0; r.th = 0.0;
            r.s = -1; r.t = -1;
        }
        r.tq = quantize_angle(r.th);
        r.pad1 = 0;
        rec[slot] = r;
    }
}

__global__ __launch_bounds__(256) void batch_node_prep_kernel(
    const float *__restrict__ x, const float *__restrict__ y, const int64_t *__restrict__ noff,
    const int64_t *__restrict__ nreco, const double *__restrict__ T, int64_t B, int64_t n_rec,
    NodeRec *__restrict__ rec) {
    for (int64_t slot = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; slot < n_rec;
         slot += (int64_t)gridDim.x * blockDim.x) {
        const int64_t L = dev::owner(nreco, B, slot);
        const int64_t k = slot - nreco[L];
        NodeRec r;
        if (k < noff[L + 1] - noff[L]) {
            const int64_t v = noff[L] + k;
            const double px = x[v], py = y[v];
            const double n = fma(px, px, py * py);
            r.x = px; r.y = py; r.q = -0.5 * n; r.h = 0.5 * (n - T[L]);
        } else {
            r.x = 0.0; r.y = 0.0; r.q = -0x1p100; r.h = 0x1p100;
        }
        rec[slot] = r;
    }
}

// One block per layout: the slots of the blocks whose ranges meet the
// layout's units, summed strided per thread and then as a tree (a fixed order).
__global__ __launch_bounds__(256) void batch_cross_finalize_kernel(
    const CrossPartial *__restrict__ part, const SweepLayout *__restrict__ tab, int64_t U,
    int64_t G, double ideal, unsigned long long *out_count, double *out_metric) {
    __shared__ unsigned long long sc[256];
    __shared__ double sd[256];
    const int64_t L = blockIdx.x;
    const int tid = threadIdx.x;
    unsigned long long c = 0;
    double d = 0.0;
    if (tab[L + 1].unit_off > tab[L].unit_off) {
        const int64_t b0 = block_of_unit(U, G, tab[L].unit_off);
        const int64_t b1 = block_of_unit(U, G, tab[L + 1].unit_off - 1);
        for (int64_t b = b0 + tid; b <= b1; b += 256) {
            c += part[b + L].proper + part[b + L].touch;
            d += part[b + L].dev;
        }
    }
    sc[tid] = c;
    sd[tid] = d;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            sc[tid] += sc[tid + s];
            sd[tid] += sd[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        if (out_count) out_count[L] = sc[0];
        if (out_metric) out_metric[L] = sc[0] ? 1.0 - (sd[0] / ideal) / (double)sc[0] : 1.0;
    }
}

__global__ __launch_bounds__(256) void batch_occl_finalize_kernel(
    const OcclPartial *__restrict__ part, const SweepLayout *__restrict__ tab, int64_t U,
    int64_t G, unsigned long long *out_count) {
    __shared__ unsigned long long sc[256];
    const int64_t L = blockIdx.x;
    const int tid = threadIdx.x;
    unsigned long long c = 0;
    if (tab[L + 1].unit_off > tab[L].unit_off) {
        const int64_t b0 = block_of_unit(U, G, tab[L].unit_off);
        const int64_t b1 = block_of_unit(U, G, tab[L + 1].unit_off - 1);
        for (int64_t b = b0 + tid; b <= b1; b += 256) c += part[b + L].count;
    }
    sc[tid] = c;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) sc[tid] += sc[tid + s];
        __syncthreads();
    }
    if (tid == 0) out_count[L] = sc[0] >> 1;       // the sweep's slots hold twice the count
}

// Algorithm 3 for one layout per block: mean, then the spread about it.
__global__ __launch_bounds__(256) void batch_elv_kernel(
    const float *__restrict__ x, const float *__restrict__ y, const int32_t *__restrict__ src,
    const int32_t *__restrict__ dst, const int64_t *__restrict__ noff,
    const int64_t *__restrict__ eoff, double *__restrict__ out) {
    __shared__ double sh[256];
    const int64_t L = blockIdx.x;
    const int64_t e0 = eoff[L], e1 = eoff[L + 1], v0 = noff[L], nV = noff[L + 1] - v0;
    double acc = 0.0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
        const int32_t s = src[e], t = dst[e];
        if (dev::valid_ids(s, t, nV)) acc += dev::edge_length(x, y, v0 + s, v0 + t);
    }
    const double N = (double)(e1 - e0);
    const double mu = e1 > e0 ? dev::block_sum(acc, sh) / N : 0.0;
    acc = 0.0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
        const int32_t s = src[e], t = dst[e];
        if (dev::valid_ids(s, t, nV)) {
            const double d = dev::edge_length(x, y, v0 + s, v0 + t) - mu;
            acc = fma(d, d, acc);
        }
    }
    const double ss = dev::block_sum(acc, sh);
    if (threadIdx.x == 0) {
        double m = 0.0;
        if (e1 - e0 >= 2 && mu > 0.0) m = sqrt(ss / (N * mu * mu)) / sqrt(N - 1.0);
        out[L] = m;
    }
}

__global__ __launch_bounds__(256) void batch_degree_kernel(
    const int32_t *__restrict__ src, const int32_t *__restrict__ dst,
    const int64_t *__restrict__ noff, const int64_t *__restrict__ eoff, int64_t B,
    int64_t n_edges, uint32_t *deg) {
    for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < n_edges; e += (int64_t)gridDim.x * 256) {
        const int64_t L = dev::owner(eoff, B, e);
        const int32_t s = src[e], t = dst[e];
        if (!dev::valid_ids(s, t, noff[L + 1] - noff[L])) continue;
        atomicAdd(&deg[noff[L] + s], 1u);
        atomicAdd(&deg[noff[L] + t], 1u);
    }
}

__global__ __launch_bounds__(256) void batch_fill_angles_kernel(
    const float *__restrict__ x, const float *__restrict__ y, const int32_t *__restrict__ src,
    const int32_t *__restrict__ dst, const int64_t *__restrict__ noff,
    const int64_t *__restrict__ eoff, int64_t B, int64_t n_edges,
    const uint32_t *__restrict__ offs, uint32_t *cursor, double *__restrict__ ang) {
    for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < n_edges; e += (int64_t)gridDim.x * 256) {
        const int64_t L = dev::owner(eoff, B, e);
        const int32_t ls = src[e], lt = dst[e];
        if (!dev::valid_ids(ls, lt, noff[L + 1] - noff[L])) continue;
        const int64_t s = noff[L] + ls, t = noff[L] + lt;
        const double dx = (double)x[t] - (double)x[s], dy = (double)y[t] - (double)y[s];
        const double rdx = (double)x[s] - (double)x[t], rdy = (double)y[s] - (double)y[t];
        const uint32_t ps = offs[s] + atomicAdd(&cursor[s], 1u);
        const uint32_t pt = offs[t] + atomicAdd(&cursor[t], 1u);
        ang[ps] = dev::direction_angle(dx, dy);
        ang[pt] = dev::direction_angle(rdx, rdy);
    }
}

// M_a of one layout per block: mean of d_v over its nodes of degree >= 1.
__global__ __launch_bounds__(256) void batch_dv_kernel(const uint32_t *__restrict__ deg,
                                                       const double *__restrict__ dv,
                                                       const int64_t *__restrict__ noff,
                                                       double *__restrict__ out) {
    __shared__ double sh[256];
    const int64_t L = blockIdx.x;
    double acc = 0.0, used = 0.0;
    for (int64_t v = noff[L] + threadIdx.x; v < noff[L + 1]; v += 256) {
        if (deg[v] > 0) {
            acc += dv[v];
            used += 1.0;
        }
    }
    const double s = dev::block_sum(acc, sh);
    const double n = dev::block_sum(used, sh);
    if (threadIdx.x == 0) out[L] = n > 0.0 ? 1.0 - s / n : 1.0;
}

int grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (int)g;
}

#define RB_TRY(expr)                          \
    do {                                      \
        hipError_t _e = (expr);               \
        if (_e != hipSuccess) return _e;      \
    } while (0)

// sweep tables of the batch for its current variants
void build_tables(const rb_batch *b, std::vector<SweepLayout> *ct, std::vector<SweepLayout> *ot,
                  int64_t *cu, int64_t *ou) {
    const int rc = cross_variant(b->cross_var).rows, ro = occl_variant(b->occl_var).rows;
    const int so = occl_variant(b->occl_var).col_shift;
    ct->resize(b->B + 1);
    ot->resize(b->B + 1);
    int64_t uc = 0, uo = 0;
    for (int64_t L = 0; L < b->B; ++L) {
        const int64_t E = b->edge_off[L + 1] - b->edge_off[L];
        const int64_t V = b->node_off[L + 1] - b->node_off[L];
        (*ct)[L] = sweep_layout(E, rc, uc, b->erec_off[L]);
        (*ot)[L] = sweep_layout(V, ro, uo, b->nrec_off[L], so);
        uc += sweep_units(E, rc);
        uo += sweep_units(V, ro, so);
    }
    (*ct)[b->B] = SweepLayout{uc, b->erec_off[b->B], 0, 0};
    (*ot)[b->B] = SweepLayout{uo, b->nrec_off[b->B], 0, 0};
    *cu = uc;
    *ou = uo;
}

struct BatchIO {
    const float *x, *y;
    const int32_t *src, *dst;
    double ideal;
    unsigned long long *occl, *cross;
    double *angle, *min_angle, *elv;
};

hipError_t enqueue_cross(const rb_batch *b, char *w, const BatchIO &io, bool with_finalize,
                         hipStream_t st) {
    const int64_t U = b->cross_units;
    const int grid = b->cross_grid_n;
    CrossPartial *part = (CrossPartial *)(w + b->o_cpart);
    RB_TRY(launch_fill_u64((unsigned long long *)part, (int64_t)(grid + b->B) * 4, 0ull, st));
    SweepArgs a;
    a.table = (const SweepLayout *)(w + b->o_ctab);
    a.single = SweepLayout{0, 0, 0, 0};
    a.n_layouts = b->B;
    a.n_units = U;
    a.unit_base = 0;
    RB_TRY(launch_cross_sweep(b->cross_var, true, (const EdgeRec *)(w + b->o_erec), a, grid,
                              io.ideal, part, st));
    if (!with_finalize) return hipSuccess;
    hipLaunchKernelGGL(batch_cross_finalize_kernel, dim3(b->B), dim3(256), 0, st, part, a.table,
                       U, (int64_t)grid, io.ideal, io.cross, io.angle);
    return hipGetLastError();
}

hipError_t enqueue_occl(const rb_batch *b, char *w, const BatchIO &io, bool with_finalize,
                        hipStream_t st) {
    const int64_t U = b->occl_units;
    const int grid = b->occl_grid_n;
    OcclPartial *part = (OcclPartial *)(w + b->o_opart);
    RB_TRY(launch_fill_u64((unsigned long long *)part, (int64_t)(grid + b->B) * 2, 0ull, st));
    SweepArgs a;
    a.table = (const SweepLayout *)(w + b->o_otab);
    a.single = SweepLayout{0, 0, 0, 0};
    a.n_layouts = b->B;
    a.n_units = U;
    a.unit_base = 0;
    RB_TRY(launch_occl_sweep(b->occl_var, (const NodeRec *)(w + b->o_nrec), a, grid, part, st));
    if (!with_finalize) return hipSuccess;
    hipLaunchKernelGGL(batch_occl_finalize_kernel, dim3(b->B), dim3(256), 0, st, part, a.table, U,
                       (int64_t)grid, io.occl);
    return hipGetLastError();
}

hipError_t enqueue_prep(const rb_batch *b, char *w, const BatchIO &io, hipStream_t st) {
    const int64_t *noff = (const int64_t *)(w + b->o_noff);
    const int64_t *eoff = (const int64_t *)(w + b->o_eoff);
    const int64_t n_erec = b->erec_off[b->B], n_nrec = b->nrec_off[b->B];
    hipLaunchKernelGGL(batch_edge_prep_kernel, dim3(grid_for(n_erec)), dim3(256), 0, st, io.x,
                       io.y, io.src, io.dst, noff, eoff, (const int64_t *)(w + b->o_ereco), b->B,
                       n_erec, (EdgeRec *)(w + b->o_erec));
    RB_TRY(hipGetLastError());
    hipLaunchKernelGGL(batch_node_prep_kernel, dim3(grid_for(n_nrec)), dim3(256), 0, st, io.x,
                       io.y, noff, (const int64_t *)(w + b->o_nreco),
                       (const double *)(w + b->o_T), b->B, n_nrec, (NodeRec *)(w + b->o_nrec));
    return hipGetLastError();
}

hipError_t side_stream(const rb_batch *b, hipStream_t *out) {
    int dev = 0;
    RB_TRY(hipGetDevice(&dev));
    if (b->side && b->side_device != dev) return hipErrorInvalidDevice;
    if (!b->side) {
        RB_TRY(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
        RB_TRY(hipEventCreateWithFlags(&b->join, hipEventDisableTiming));
        RB_TRY(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
        b->side_device = dev;
    }
    *out = b->side;
    return hipSuccess;
}

// The edge sweep runs on `main` and the node sweep, edge lengths and
// minimum angle on the batch's second stream, forked from `main` after the
// record prep and joined back at the end; their workspace regions are
// disjoint.  A graph captured from `main` holds the same fork as two
// branches.
hipError_t enqueue_all(const rb_batch *b, char *w, const BatchIO &io, hipStream_t main) {
    const int64_t *noff = (const int64_t *)(w + b->o_noff);
    const int64_t *eoff = (const int64_t *)(w + b->o_eoff);
    const bool need_cross = io.cross || io.angle;
    RB_TRY(enqueue_prep(b, w, io, main));
    hipStream_t st = main;
    RB_TRY(side_stream(b, &st));
    RB_TRY(hipEventRecord(b->fork, main));
    RB_TRY(hipStreamWaitEvent(st, b->fork, 0));
    if (io.occl) RB_TRY(enqueue_occl(b, w, io, true, st));
    if (io.elv) {
        hipLaunchKernelGGL(batch_elv_kernel, dim3((unsigned)b->B), dim3(256), 0, st, io.x, io.y,
                           io.src, io.dst, noff, eoff, io.elv);
        RB_TRY(hipGetLastError());
    }
    if (io.min_angle) {
        const int64_t V = b->n_nodes > 0 ? b->n_nodes : 1;
        uint32_t *deg = (uint32_t *)(w + b->o_deg);
        uint32_t *cursor = (uint32_t *)(w + b->o_cursor);
        uint32_t *offs = (uint32_t *)(w + b->o_offs);
        double *ang = (double *)(w + b->o_ang);
        double *dv = (double *)(w + b->o_dv);
        Scalars *sc = (Scalars *)(w + b->o_sc);
        RB_TRY(launch_zero_scalars(sc, st));
        RB_TRY(launch_fill_u32(deg, V, 0u, st));
        RB_TRY(launch_fill_u32(cursor, V, 0u, st));
        if (b->n_edges > 0) {
            hipLaunchKernelGGL(batch_degree_kernel, dim3(grid_for(b->n_edges)), dim3(256), 0, st,
                               io.src, io.dst, noff, eoff, b->B, b->n_edges, deg);
            RB_TRY(hipGetLastError());
        }
        RB_TRY(launch_scan(deg, V, (unsigned long long *)dv, offs, st));
        if (b->n_edges > 0) {
            hipLaunchKernelGGL(batch_fill_angles_kernel, dim3(grid_for(b->n_edges)), dim3(256), 0,
                               st, io.x, io.y, io.src, io.dst, noff, eoff, b->B, b->n_edges, offs,
                               cursor, ang);
            RB_TRY(hipGetLastError());
        }
        RB_TRY(launch_min_angle_nodes(deg, offs, ang, b->n_nodes, dv,
                                      (int32_t *)(w + b->o_big), sc, st));
        hipLaunchKernelGGL(batch_dv_kernel, dim3((unsigned)b->B), dim3(256), 0, st, deg, dv, noff,
                           io.min_angle);
        RB_TRY(hipGetLastError());
    }
    if (need_cross) RB_TRY(enqueue_cross(b, w, io, true, main));
    RB_TRY(hipEventRecord(b->join, st));
    return hipStreamWaitEvent(main, b->join, 0);
}

void carve(rb_batch *b) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = round_up(off + (bytes ? bytes : 1), 256);
        return o;
    };
    const int64_t B = b->B;
    const int64_t V = b->n_nodes > 0 ? b->n_nodes : 1;
    const int64_t E = b->n_edges > 0 ? b->n_edges : 1;
    b->o_erec = take(sizeof(EdgeRec) * (size_t)b->erec_off[B]);
    b->o_nrec = take(sizeof(NodeRec) * (size_t)b->nrec_off[B]);
    b->o_ctab = take(sizeof(SweepLayout) * (size_t)(B + 1));
    b->o_otab = take(sizeof(SweepLayout) * (size_t)(B + 1));
    b->o_noff = take(sizeof(int64_t) * (size_t)(B + 1));
    b->o_eoff = take(sizeof(int64_t) * (size_t)(B + 1));
    b->o_ereco = take(sizeof(int64_t) * (size_t)(B + 1));
    b->o_nreco = take(sizeof(int64_t) * (size_t)(B + 1));
    b->o_T = take(sizeof(double) * (size_t)B);
    b->o_cpart = take(sizeof(CrossPartial) * (size_t)(kMaxPartials + B));
    b->o_opart = take(sizeof(OcclPartial) * (size_t)(kMaxPartials + B));
    b->o_deg = take(sizeof(uint32_t) * (size_t)V);
    b->o_cursor = take(sizeof(uint32_t) * (size_t)V);
    b->o_offs = take(sizeof(uint32_t) * (size_t)(V + 1));
    b->o_ang = take(sizeof(double) * (size_t)(2 * E));
    b->o_dv = take(sizeof(double) * (size_t)V);
    b->o_big = take(sizeof(int32_t) * (size_t)V);
    b->o_sc = take(sizeof(Scalars));
    b->total = off;
}

hipError_t upload(rb_batch *b, void *ws, hipStream_t st) {
    std::vector<SweepLayout> ct, ot;
    int64_t cu, ou;
    build_tables(b, &ct, &ot, &cu, &ou);
    char *w = (char *)ws;
    struct Piece {
        size_t off;
        const void *src;
        size_t bytes;
    } pieces[] = {
        {b->o_ctab, ct.data(), sizeof(SweepLayout) * ct.size()},
        {b->o_otab, ot.data(), sizeof(SweepLayout) * ot.size()},
        {b->o_noff, b->node_off.data(), sizeof(int64_t) * b->node_off.size()},
        {b->o_eoff, b->edge_off.data(), sizeof(int64_t) * b->edge_off.size()},
        {b->o_ereco, b->erec_off.data(), sizeof(int64_t) * b->erec_off.size()},
        {b->o_nreco, b->nrec_off.data(), sizeof(int64_t) * b->nrec_off.size()},
        {b->o_T, b->T.data(), sizeof(double) * b->T.size()},
    };
    for (const Piece &p : pieces) {
        if (p.bytes == 0) continue;
        RB_TRY(hipMemcpyAsync(w + p.off, p.src, p.bytes, hipMemcpyHostToDevice, st));
    }
    RB_TRY(hipStreamSynchronize(st));
    b->cross_units = cu;
    b->occl_units = ou;
    b->cross_grid_n = (int)std::min<int64_t>(cu, cross_grid(b->cross_var, true));
    b->occl_grid_n = (int)std::min<int64_t>(ou, kMaxPartials);   // one unit per block
    b->uploaded = ws;
    ++b->plan_gen;
    return hipSuccess;
}

rb_status check_io(const rb_batch *b, const BatchIO &io, void *ws, size_t ws_bytes) {
    if (!b) return (rb_status)set_error(RB_EINVAL, "batch is NULL");
    if (b->n_nodes > 0 && (!io.x || !io.y)) return (rb_status)set_error(RB_EINVAL, "x or y is NULL");
    if (b->n_edges > 0 && (!io.src || !io.dst))
        return (rb_status)set_error(RB_EINVAL, "src or dst is NULL");
    if (!(io.ideal > 0.0) || !(io.ideal <= 1.5707963267948966))
        return (rb_status)set_error(RB_EINVAL, "ideal_angle must be in (0, pi/2]");
    if (!ws) return (rb_status)set_error(RB_EWORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws & 255u) != 0)
        return (rb_status)set_error(RB_EWORKSPACE, "workspace not 256-byte aligned");
    if (ws_bytes < b->total)
        return (rb_status)set_error(RB_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes,
                                    b->total);
    if (b->uploaded != ws)
        return (rb_status)set_error(RB_EINVAL, "call rb_batch_upload with this workspace first");
    return RB_OK;
}

}  // namespace
}  // namespace rb

extern "C" {

rb_status rb_batch_create(int64_t n_layouts, const int64_t *node_off, const int64_t *edge_off,
                          const double *diameters, rb_batch **out) {
    clear_error();
    if (!out) return (rb_status)set_error(RB_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_layouts < 1 || n_layouts > (1 << 24))
        return (rb_status)set_error(RB_EINVAL, "n_layouts must be in [1, 2^24]");
    if (!node_off || !edge_off || !diameters)
        return (rb_status)set_error(RB_EINVAL, "offsets or diameters are NULL");
    if (node_off[0] != 0 || edge_off[0] != 0)
        return (rb_status)set_error(RB_EINVAL, "offsets must start at 0");
    for (int64_t L = 0; L < n_layouts; ++L) {
        const int64_t V = node_off[L + 1] - node_off[L], E = edge_off[L + 1] - edge_off[L];
        if (V < 0 || E < 0) return (rb_status)set_error(RB_EINVAL, "offsets must be nondecreasing");
        if (E > 0 && V < 2)
            return (rb_status)set_error(RB_EINVAL, "layout %lld has edges but < 2 nodes",
                                        (long long)L);
        if (!(diameters[L] >= 0.0) || !std::isfinite(diameters[L]))
            return (rb_status)set_error(RB_EINVAL, "diameter of layout %lld invalid", (long long)L);
    }
    if (node_off[n_layouts] > 2147483647LL || edge_off[n_layouts] > (1LL << 30))
        return (rb_status)set_error(RB_EINVAL, "batch too large");
    if (const int f = inject_fault("alloc", "rb_batch_create")) return (rb_status)f;
    rb_batch *b = new (std::nothrow) rb_batch;
    if (!b) return (rb_status)set_error(RB_ENOMEM, "rb_batch_create: out of host memory");
    try {
    b->B = n_layouts;
    b->node_off.assign(node_off, node_off + n_layouts + 1);
    b->edge_off.assign(edge_off, edge_off + n_layouts + 1);
    b->n_nodes = node_off[n_layouts];
    b->n_edges = edge_off[n_layouts];
    b->T.resize(n_layouts);
    b->erec_off.assign(n_layouts + 1, 0);
    b->nrec_off.assign(n_layouts + 1, 0);
    for (int64_t L = 0; L < n_layouts; ++L) {
        const int64_t V = node_off[L + 1] - node_off[L], E = edge_off[L + 1] - edge_off[L];
        b->erec_off[L + 1] = b->erec_off[L] + (int64_t)round_up((size_t)std::max<int64_t>(E, 1), kRecPad);
        b->nrec_off[L + 1] = b->nrec_off[L] + (int64_t)round_up((size_t)std::max<int64_t>(V, 1), kRecPad);
        b->T[L] = occlusion_threshold(diameters[L]);
    }
    const int64_t mean_e = std::max<int64_t>(1, b->n_edges / n_layouts);
    const int64_t mean_v = std::max<int64_t>(1, b->n_nodes / n_layouts);
    b->cross_var = tuned_variant(1, true, mean_e);
    b->occl_var = tuned_variant(2, true, mean_v);
    carve(b);
    } catch (const std::bad_alloc &) {
        delete b;
        return (rb_status)set_error(RB_ENOMEM, "rb_batch_create: out of host memory");
    }
    *out = b;
    return RB_OK;
}

size_t rb_batch_workspace_size(const rb_batch *b) { return b ? b->total : 0; }

rb_status rb_batch_upload(rb_batch *b, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    if (!b) return (rb_status)set_error(RB_EINVAL, "batch is NULL");
    if (!ws || ((uintptr_t)ws & 255u) != 0 || ws_bytes < b->total)
        return (rb_status)set_error(RB_EWORKSPACE, "workspace NULL, misaligned or below %zu bytes",
                                    b->total);
    if (const int f = inject_fault("launch", "rb_batch_upload")) return (rb_status)f;
    hipError_t e = upload(b, ws, (hipStream_t)stream);
    if (e != hipSuccess) return (rb_status)hip_error(e, "rb_batch_upload");
    return RB_OK;
}

rb_status rb_batch_evaluate(const rb_batch *b, const float *x, const float *y, const int32_t *src,
                            const int32_t *dst, double ideal_angle, uint64_t *out_occlusion,
                            uint64_t *out_crossings, double *out_crossing_angle,
                            double *out_min_angle, double *out_elv, void *ws, size_t ws_bytes,
                            void *stream) {
    clear_error();
    BatchIO io{x, y, src, dst, ideal_angle, (unsigned long long *)out_occlusion,
               (unsigned long long *)out_crossings, out_crossing_angle, out_min_angle, out_elv};
    rb_status s = check_io(b, io, ws, ws_bytes);
    if (s) return s;
    if (const int f = inject_fault("launch", "rb_batch_evaluate")) return (rb_status)f;
    hipError_t e = enqueue_all(b, (char *)ws, io, (hipStream_t)stream);
    if (e != hipSuccess) return (rb_status)hip_error(e, "rb_batch_evaluate");
    return RB_OK;
}

rb_status rb_batch_autotune(rb_batch *b, const float *x, const float *y, const int32_t *src,
                            const int32_t *dst, double ideal_angle, int repeats,
                            double *out_best_ms, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    BatchIO io{x, y, src, dst, ideal_angle, nullptr, nullptr, nullptr, nullptr, nullptr};
    rb_status s = check_io(b, io, ws, ws_bytes);
    if (s) return s;
    if (repeats < 1 || repeats > 1000)
        return (rb_status)set_error(RB_EINVAL, "repeats must be in [1, 1000]");
    if (const int f = inject_fault("launch", "rb_batch_autotune")) return (rb_status)f;
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)ws;
    hipError_t e = enqueue_prep(b, w, io, st);
    hipEvent_t ea = nullptr, eb = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&ea);
    if (e == hipSuccess) e = hipEventCreate(&eb);
    double best_total = 0.0;
    for (int kind = 0; kind < 2 && e == hipSuccess; ++kind) {
        const bool occl = kind == 1;
        const int nv = occl ? kOcclVariants : kCrossVariants;
        int best = -1;
        float best_ms = 0.f;
        for (int v = 0; v < nv && e == hipSuccess; ++v) {
            if (!variant_offered(occl ? 2 : 1, true, v)) continue;
            if (occl) b->occl_var = v;
            else b->cross_var = v;
            e = upload(b, ws, st);
            auto launch = [&]() {
                return occl ? enqueue_occl(b, w, io, false, st) : enqueue_cross(b, w, io, false, st);
            };
            if (e == hipSuccess) e = launch();
            if (e == hipSuccess) e = hipEventRecord(ea, st);
            for (int k = 0; k < repeats && e == hipSuccess; ++k) e = launch();
            if (e == hipSuccess) e = hipEventRecord(eb, st);
            if (e == hipSuccess) e = hipEventSynchronize(eb);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ea, eb);
            ms /= repeats;
            if (e == hipSuccess && (best < 0 || ms < best_ms)) {
                best = v;
                best_ms = ms;
            }
        }
        if (e == hipSuccess) {
            if (occl) b->occl_var = best;
            else b->cross_var = best;
            const int64_t mean = std::max<int64_t>(
                1, occl ? b->n_nodes / b->B : b->n_edges / b->B);
            set_tuned_variant(occl ? 2 : 1, true, mean, best);
            best_total += best_ms;
        }
    }
    if (e == hipSuccess) e = upload(b, ws, st);
    if (ea) (void)hipEventDestroy(ea);
    if (eb) (void)hipEventDestroy(eb);
    if (e != hipSuccess) return (rb_status)hip_error(e, "rb_batch_autotune");
    if (out_best_ms) *out_best_ms = best_total;
    return RB_OK;
}

rb_status rb_batch_variants(const rb_batch *b, int *cross_rows, int *cross_waves, int *occl_rows,
                            int *occl_waves) {
    clear_error();
    if (!b) return (rb_status)set_error(RB_EINVAL, "batch is NULL");
    const SweepVariant c = cross_variant(b->cross_var), o = occl_variant(b->occl_var);
    if (cross_rows) *cross_rows = c.rows;
    if (cross_waves) *cross_waves = c.waves;
    if (occl_rows) *occl_rows = o.rows;
    if (occl_waves) *occl_waves = o.waves;
    return RB_OK;
}

void rb_batch_destroy(rb_batch *b) { delete b; }

rb_status rb_batch_graph_create(const rb_batch *b, const float *x, const float *y,
                                const int32_t *src, const int32_t *dst, double ideal_angle,
                                uint64_t *out_occlusion, uint64_t *out_crossings,
                                double *out_crossing_angle, double *out_min_angle,
                                double *out_elv, void *ws, size_t ws_bytes, rb_graph **out) {
    clear_error();
    if (!out) return (rb_status)set_error(RB_EINVAL, "out is NULL");
    *out = nullptr;
    BatchIO io{x, y, src, dst, ideal_angle, (unsigned long long *)out_occlusion,
               (unsigned long long *)out_crossings, out_crossing_angle, out_min_angle, out_elv};
    rb_status s = check_io(b, io, ws, ws_bytes);
    if (s) return s;
    if (const int f = inject_fault("alloc", "rb_batch_graph_create")) return (rb_status)f;
    rb_graph *g = new (std::nothrow) rb_graph;
    if (!g) return (rb_status)set_error(RB_ENOMEM, "rb_batch_graph_create: out of host memory");
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete g;
        return (rb_status)hip_error(e, "capture stream");
    }
    hipGraph_t graph = nullptr;
    bool injected = false;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        injected = fault_listed("capture");
        hipError_t e2 = injected ? hipErrorUnknown : enqueue_all(b, (char *)ws, io, cs);
        e = hipStreamEndCapture(cs, &graph);
        if (e2 != hipSuccess) e = e2;
    }
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        delete g;
        if (injected)
            return (rb_status)set_error(RB_EHIP, "rb_batch_graph_create: injected failure "
                                                 "(RB_FAULT=capture) inside the capture");
        return (rb_status)hip_error(e, "rb_batch_graph_create");
    }
    g->graph = graph;
    g->exec = exec;
    g->batch = b;
    g->plan_gen = b->plan_gen;
    *out = g;
    return RB_OK;
}

rb_status rb_graph_launch(rb_graph *g, void *stream) {
    clear_error();
    if (!g) return (rb_status)set_error(RB_EINVAL, "graph is NULL");
    if (g->batch->plan_gen != g->plan_gen)
        return (rb_status)set_error(RB_EINVAL,
                                    "the batch plan was uploaded again (rb_batch_upload or "
                                    "rb_batch_autotune) after this graph was captured: "
                                    "capture a new graph");
    if (const int f = inject_fault("launch", "rb_graph_launch")) return (rb_status)f;
    hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    if (e != hipSuccess) return (rb_status)hip_error(e, "rb_graph_launch");
    return RB_OK;
}

void rb_graph_destroy(rb_graph *g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

}  // extern "C"
