// Grid-pruned exact sweeps.
//
// Node occlusion on a uniform grid (the grid method of Section 3.2.1): with
// cells of side s >= d, every pair closer than d lies in one cell or in two
// neighbouring cells.  Nodes are sorted by the Morton code of their cell;
// each node then counts its partners among the later nodes of its own cell
// and all nodes of four neighbour cells (east, north-east, north, north-west:
// half of the eight, so that each unordered pair of cells is visited once).
// The distance test is the exact integer one of Algorithm 1, so the count is
// the brute-force count; only pairs that cannot occlude are skipped.  The
// paper instead maps each node to every cell its disc overlaps and removes
// duplicate pairs afterwards; the half stencil needs no duplicate removal.
//
// Edge crossings with unit culling: every crossing pair of closed segments
// has intersecting bounding boxes, so a (row tile, column chunk) unit of the
// all-pairs sweep whose two boxes (the unions of their edges' boxes) are
// disjoint holds no crossing and can be skipped.  To make the boxes small,
// edges are first ordered along a Hilbert curve by their box centre, the
// edges longer than 1/16 of the layout after the others in octave classes.  The kept units
// run through the same sweep body as the brute-force path, so every count is
// the brute-force count; only the order of the floating-point sum changes.
//
// The sort is a stable least-significant-digit radix sort of (key, value)
// pairs with 8-bit digits written here: per-block digit histograms, one
// exclusive scan over (digit, block), and a scatter that ranks items of equal
// digit by wave ballots, so the order is deterministic.
#include <climits>

#include "rb_device.h"
#include "rb_internal.h"

namespace rb {
namespace {

constexpr int kSortPer = kSortTile / 256;    // items per thread and pass

__global__ __launch_bounds__(256) void sort_hist_kernel(const uint32_t *__restrict__ keys,
                                                        int64_t n, int shift,
                                                        uint32_t *__restrict__ hist, int64_t nb) {
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int k = 0; k < kSortPer; ++k) {
        const int64_t i = base + (int64_t)k * 256 + tid;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)tid * nb + blockIdx.x] = h[tid];
}

__global__ __launch_bounds__(256) void sort_scatter_kernel(
    const uint32_t *__restrict__ keys, const int32_t *__restrict__ vals, int64_t n, int shift,
    const uint32_t *__restrict__ off, int64_t nb, uint32_t *__restrict__ keys_out,
    int32_t *__restrict__ vals_out) {
    __shared__ uint32_t run[256];            // items of each digit already placed by this block
    __shared__ uint32_t wcnt[4][256];        // items of each digit in each wave this round
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    run[tid] = 0;
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int k = 0; k < kSortPer; ++k) {
        // round k takes items base + 256 k + tid: thread order is item order
        const int64_t i = base + (int64_t)k * 256 + tid;
        const bool valid = i < n;
        const uint32_t key = valid ? keys[i] : 0u;
        const int32_t val = valid ? vals[i] : 0;
        const uint32_t d = (key >> shift) & 255u;
#pragma unroll
        for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        unsigned long long same = __builtin_amdgcn_ballot_w64(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool set = (d >> bit) & 1u;
            const unsigned long long m = __builtin_amdgcn_ballot_w64(set);
            same &= set ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(same & below);
        if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(same);
        __syncthreads();
        if (valid) {
            uint32_t before = run[d];
            for (int w = 0; w < wave; ++w) before += wcnt[w][d];
            const uint32_t pos = off[(int64_t)d * nb + blockIdx.x] + before + rank;
            keys_out[pos] = key;
            vals_out[pos] = val;
        }
        __syncthreads();
        run[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
    }
}

// ---------------------------------------------------------------- grid setup

__global__ void bounds_init_kernel(GridParams *gp) {
    if (threadIdx.x == 0) {
        gp->xmin = INT_MAX;
        gp->ymin = INT_MAX;
        gp->xmax = INT_MIN;
        gp->ymax = INT_MIN;
        gp->shift = 0;
    }
}

__global__ __launch_bounds__(256) void bounds_kernel(const float *__restrict__ x,
                                                     const float *__restrict__ y, int64_t n,
                                                     GridParams *gp) {
    int x0 = INT_MAX, y0 = INT_MAX, x1 = INT_MIN, y1 = INT_MIN;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int xi = (int)x[i], yi = (int)y[i];
        x0 = min(x0, xi);
        y0 = min(y0, yi);
        x1 = max(x1, xi);
        y1 = max(y1, yi);
    }
    for (int off = 32; off > 0; off >>= 1) {
        x0 = min(x0, __shfl_xor(x0, off, 64));
        y0 = min(y0, __shfl_xor(y0, off, 64));
        x1 = max(x1, __shfl_xor(x1, off, 64));
        y1 = max(y1, __shfl_xor(y1, off, 64));
    }
    // one atomic per block and bound
    __shared__ int4 w[4];
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = make_int4(x0, y0, x1, y1);
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < 4; ++k) {
            x0 = min(x0, w[k].x); y0 = min(y0, w[k].y);
            x1 = max(x1, w[k].z); y1 = max(y1, w[k].w);
        }
        atomicMin(&gp->xmin, x0);
        atomicMin(&gp->ymin, y0);
        atomicMax(&gp->xmax, x1);
        atomicMax(&gp->ymax, y1);
    }
}

// cell side 2^shift: at least 2^min_shift and at most 2^16 cells per axis
__global__ void grid_shift_kernel(GridParams *gp, int min_shift, int axis_bits) {
    if (threadIdx.x != 0) return;
    int shift = min_shift;
    if (gp->xmin <= gp->xmax) {
        const long long span =
            max((long long)gp->xmax - gp->xmin, (long long)gp->ymax - gp->ymin);
        while ((span >> shift) >= (1ll << axis_bits)) ++shift;
    }
    gp->shift = shift;
}

__device__ __forceinline__ uint32_t spread16(uint32_t v) {
    v &= 0xffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

__device__ __forceinline__ uint32_t morton(uint32_t cx, uint32_t cy) {
    return spread16(cx) | (spread16(cy) << 1);
}

__device__ __forceinline__ uint32_t compact16(uint32_t v) {
    v &= 0x55555555u;
    v = (v | (v >> 1)) & 0x33333333u;
    v = (v | (v >> 2)) & 0x0f0f0f0fu;
    v = (v | (v >> 4)) & 0x00ff00ffu;
    v = (v | (v >> 8)) & 0x0000ffffu;
    return v;
}

__global__ __launch_bounds__(256) void node_key_kernel(const float *__restrict__ x,
                                                       const float *__restrict__ y, int64_t n,
                                                       const GridParams *__restrict__ gp,
                                                       uint32_t *__restrict__ keys,
                                                       int32_t *__restrict__ vals) {
    const int shift = gp->shift;
    const int x0 = gp->xmin, y0 = gp->ymin;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t cx = (uint32_t)(((long long)(int)x[i] - x0) >> shift);
        const uint32_t cy = (uint32_t)(((long long)(int)y[i] - y0) >> shift);
        keys[i] = morton(cx, cy);
        vals[i] = (int32_t)i;
    }
}

__global__ __launch_bounds__(256) void gather_nodes_kernel(const float *__restrict__ x,
                                                           const float *__restrict__ y,
                                                           int64_t n,
                                                           const int32_t *__restrict__ order,
                                                           int2 *__restrict__ pos) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = order[p];
        pos[p] = make_int2((int)x[i], (int)y[i]);
    }
}

// first index in keys[0, n) whose key is >= k
__device__ __forceinline__ int64_t lower_bound(const uint32_t *keys, int64_t n, uint32_t k) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < k) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ unsigned long long count_range(const int2 *__restrict__ pos,
                                                          int64_t b, int64_t e, int2 p,
                                                          long long T) {
    unsigned long long c = 0;
    for (int64_t q = b; q < e; ++q) {
        const int2 o = pos[q];
        const long long dx = (long long)p.x - o.x, dy = (long long)p.y - o.y;
        c += (dx * dx + dy * dy <= T) ? 1ull : 0ull;
    }
    return c;
}

__global__ __launch_bounds__(256) void occl_grid_count_kernel(const uint32_t *__restrict__ keys,
                                                              const int2 *__restrict__ pos,
                                                              int64_t n, long long T,
                                                              OcclPartial *__restrict__ part) {
    __shared__ unsigned long long red[4];
    unsigned long long c = 0;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t k = keys[p];
        const int2 me = pos[p];
        // later nodes of the own cell
        int64_t e = p + 1;
        while (e < n && keys[e] == k) ++e;
        c += count_range(pos, p + 1, e, me, T);
        const int cx = (int)compact16(k), cy = (int)compact16(k >> 1);
        const int ncx[4] = {cx + 1, cx + 1, cx, cx - 1};
        const int ncy[4] = {cy, cy + 1, cy + 1, cy + 1};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (ncx[s] < 0 || ncx[s] > 0xffff || ncy[s] > 0xffff) continue;
            const uint32_t nk = morton((uint32_t)ncx[s], (uint32_t)ncy[s]);
            const int64_t b = lower_bound(keys, n, nk);
            int64_t q = b;
            while (q < n && keys[q] == nk) ++q;
            c += count_range(pos, b, q, me, T);
        }
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        OcclPartial P;
        P.count = red[0] + red[1] + red[2] + red[3];
        P.pad = 0;
        part[blockIdx.x] = P;
    }
}

// index of cell (x, y) along the Hilbert curve over a 2^14 x 2^14 grid: cells
// close on the curve are close in the plane, with none of the Morton
// order's jumps, so a run of edges in this order has a compact box
__device__ __forceinline__ uint32_t hilbert14(uint32_t x, uint32_t y) {
    constexpr uint32_t n = 1u << 14;
    uint32_t d = 0;
    for (uint32_t s = n >> 1; s > 0; s >>= 1) {
        const uint32_t rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
        d += s * s * ((3u * rx) ^ ry);
        if (ry == 0) {                        // rotate the quadrant
            if (rx == 1) {
                x = n - 1 - x;
                y = n - 1 - y;
            }
            const uint32_t t = x;
            x = y;
            y = t;
        }
    }
    return d;
}

// key of an edge: edges whose box side is at most 1/16 of the layout's span
// first, in Hilbert order of their box centre; longer edges after them in
// classes by octave of their side (one long edge in a tile of short ones
// would widen that tile's box), each class again in Hilbert order; edges
// with bad ids after all others
// key of edge e = its hub: the end point of larger degree, the smaller id
// on a tie (0 for an edge with ids out of range, which the sweep skips)
__global__ __launch_bounds__(256) void hub_key_kernel(const int32_t *__restrict__ src,
                                                      const int32_t *__restrict__ dst,
                                                      int64_t n_nodes, int64_t m,
                                                      const uint32_t *__restrict__ deg,
                                                      uint32_t *__restrict__ keys,
                                                      int32_t *__restrict__ vals) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t s = src[e], t = dst[e];
        uint32_t key = 0;
        if (dev::valid_ids(s, t, n_nodes)) {
            const uint32_t ds = deg[s], dt = deg[t];
            key = (uint32_t)((ds > dt || (ds == dt && s <= t)) ? s : t);
        }
        keys[e] = key;
        vals[e] = (int32_t)e;
    }
}

__global__ __launch_bounds__(256) void edge_key_kernel(const float *__restrict__ x,
                                                       const float *__restrict__ y,
                                                       const int32_t *__restrict__ src,
                                                       const int32_t *__restrict__ dst,
                                                       int64_t n_nodes, int64_t m,
                                                       const GridParams *__restrict__ gp,
                                                       uint32_t *__restrict__ keys,
                                                       int32_t *__restrict__ vals) {
    const int shift = gp->shift;
    const long long x0 = gp->xmin, y0 = gp->ymin;
    const long long span = max((long long)gp->xmax - x0, (long long)gp->ymax - y0);
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t s = src[e], t = dst[e];
        uint32_t key = 0xffffffffu;
        if (dev::valid_ids(s, t, n_nodes)) {
            const long long xs = (int)x[s], ys = (int)y[s], xt = (int)x[t], yt = (int)y[t];
            const long long bx0 = min(xs, xt), bx1 = max(xs, xt);
            const long long by0 = min(ys, yt), by1 = max(ys, yt);
            const long long r = 16 * max(bx1 - bx0, by1 - by0);
            uint32_t cls = 0;
            while (span > 0 && cls < 7 && r > (span << cls)) ++cls;
            const uint32_t cx = (uint32_t)((bx0 - x0 + bx1 - x0) >> (shift + 1));
            const uint32_t cy = (uint32_t)((by0 - y0 + by1 - y0) >> (shift + 1));
            key = (cls << 28) | hilbert14(cx & 0x3fffu, cy & 0x3fffu);
        }
        keys[e] = key;
        vals[e] = (int32_t)e;
    }
}

// bounding box of the edges of each 256-record chunk (padding records excluded)
__global__ __launch_bounds__(256) void chunk_box_kernel(const EdgeRec *__restrict__ rec,
                                                        int4 *__restrict__ box) {
    const EdgeRec r = rec[(int64_t)blockIdx.x * 256 + threadIdx.x];
    int x0 = INT_MAX, y0 = INT_MAX, x1 = INT_MIN, y1 = INT_MIN;
    if (r.s >= 0) {
        const int ax = (int)r.x, ay = (int)r.y;
        const int bx = (int)(r.x + r.dx), by = (int)(r.y + r.dy);
        x0 = min(ax, bx); x1 = max(ax, bx);
        y0 = min(ay, by); y1 = max(ay, by);
    }
    for (int off = 32; off > 0; off >>= 1) {
        x0 = min(x0, __shfl_xor(x0, off, 64));
        y0 = min(y0, __shfl_xor(y0, off, 64));
        x1 = max(x1, __shfl_xor(x1, off, 64));
        y1 = max(y1, __shfl_xor(y1, off, 64));
    }
    __shared__ int4 w[4];
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = make_int4(x0, y0, x1, y1);
    __syncthreads();
    if (threadIdx.x == 0) {
        int4 b = w[0];
        for (int k = 1; k < 4; ++k) {
            b.x = min(b.x, w[k].x); b.y = min(b.y, w[k].y);
            b.z = max(b.z, w[k].z); b.w = max(b.w, w[k].w);
        }
        box[blockIdx.x] = b;
    }
}

__device__ __forceinline__ int4 tile_box(const int4 *__restrict__ box, int64_t I, int K,
                                         int64_t n_chunks) {
    int4 b = make_int4(INT_MAX, INT_MAX, INT_MIN, INT_MIN);
    for (int64_t c = I * K; c < min((I + 1) * K, n_chunks); ++c) {
        const int4 q = box[c];
        b.x = min(b.x, q.x); b.y = min(b.y, q.y);
        b.z = max(b.z, q.z); b.w = max(b.w, q.w);
    }
    return b;
}

// a unit is kept if its chunk overlaps the tile itself or the closed boxes meet
__device__ __forceinline__ bool keep_unit(const int4 *__restrict__ box, int4 tb, int64_t I,
                                          int K, int64_t c) {
    if (c < (I + 1) * K) return true;
    const int4 q = box[c];
    return q.x <= tb.z && tb.x <= q.z && q.y <= tb.w && tb.y <= q.w;
}

// one block per row tile: number of kept chunks
__global__ __launch_bounds__(256) void tile_count_kernel(const int4 *__restrict__ box,
                                                         int64_t n_chunks, int K,
                                                         uint32_t *__restrict__ cnt) {
    __shared__ uint32_t red[4];
    const int64_t I = blockIdx.x;
    const int4 tb = tile_box(box, I, K, n_chunks);
    uint32_t k = 0;
    for (int64_t c = I * K + threadIdx.x; c < n_chunks; c += 256)
        k += keep_unit(box, tb, I, K, c) ? 1u : 0u;
    for (int off = 32; off > 0; off >>= 1) k += __shfl_xor(k, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = k;
    __syncthreads();
    if (threadIdx.x == 0) cnt[I] = red[0] + red[1] + red[2] + red[3];
}

// one block per row tile: the kept chunks in increasing order
__global__ __launch_bounds__(256) void tile_fill_kernel(const int4 *__restrict__ box,
                                                        int64_t n_chunks, int K,
                                                        const uint32_t *__restrict__ off,
                                                        int32_t *__restrict__ list) {
    __shared__ uint32_t wsum[4];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int64_t I = blockIdx.x;
    const int4 tb = tile_box(box, I, K, n_chunks);
    int64_t base = off[I];
    for (int64_t c0 = I * K; c0 < n_chunks; c0 += 256) {
        const int64_t c = c0 + tid;
        const bool keep = c < n_chunks && keep_unit(box, tb, I, K, c);
        const unsigned long long m = __builtin_amdgcn_ballot_w64(keep);
        if (lane == 0) wsum[wave] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t before = 0;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        if (keep) list[base + before + (uint32_t)__popcll(m & below)] = (int32_t)c;
        base += wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
    }
}

__global__ void set_count_kernel(unsigned long long *out, unsigned long long v) {
    if (threadIdx.x == 0) *out = v;
}

int blocks_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    return (int)g;
}

#define RB_TRY(expr)                          \
    do {                                      \
        hipError_t _e = (expr);               \
        if (_e != hipSuccess) return _e;      \
    } while (0)

}  // namespace

bool grid_ws_layout(int64_t n_nodes, int64_t n_edges, GridWs *G) {
    if (n_nodes < 0 || n_edges < 0 || n_nodes > (1ll << 31) - 1 || n_edges > (1ll << 30))
        return false;
    const int64_t n = std::max<int64_t>(std::max<int64_t>(n_nodes, n_edges), 1);
    const int64_t nb = (n + kSortTile - 1) / kSortTile;
    const int64_t n_hist = 256 * nb;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = (off + bytes + 255) & ~(size_t)255;
        return o;
    };
    G->params = take(sizeof(GridParams));
    G->keys = take(sizeof(uint32_t) * n);
    G->vals = take(sizeof(int32_t) * n);
    G->keys2 = take(sizeof(uint32_t) * n);
    G->vals2 = take(sizeof(int32_t) * n);
    G->pos = take(sizeof(int2) * n);
    G->hist = take(sizeof(uint32_t) * n_hist);
    G->hist_off = take(sizeof(uint32_t) * (n_hist + 1));
    G->scan_tile = take(sizeof(unsigned long long) * ((n_hist + 2047) / 2048 + 1));
    G->partial = take(sizeof(CrossPartial) * kMaxPartials);
    // pruned edge sweep: records, chunk boxes, per-tile counts and offsets and
    // the unit list, sized for the smallest row tile (256 edges), which has
    // the most units
    const int64_t me = std::max<int64_t>(n_edges, 1);
    G->n_edge_pad = (me + kRecPad - 1) / kRecPad * kRecPad;
    const int64_t n_chunks = G->n_edge_pad / kChunk;
    G->max_units = n_edges <= kMaxPrunedEdges ? sweep_units(me, 1) : 0;
    G->rec = take(sizeof(EdgeRec) * G->n_edge_pad);
    G->box = take(sizeof(int4) * n_chunks);
    G->tile_cnt = take(sizeof(uint32_t) * n_chunks);
    G->tile_off = take(sizeof(uint32_t) * (n_chunks + 1));
    G->list = take(sizeof(int32_t) * std::max<int64_t>(G->max_units, 1));
    G->kacc = take(sizeof(int32_t) * G->n_edge_pad);
    G->scalars = take(sizeof(Scalars));
    G->fwd = take(sizeof(Fwd));
    const int64_t V = std::max<int64_t>(n_nodes, 1);
    G->node_rec = take(V < kGridMinNodes ? sizeof(NodeRec) * ((V + kRecPad - 1) / kRecPad * kRecPad)
                                         : 0);
    G->deg = take(sizeof(uint32_t) * V);
    G->cursor = take(sizeof(uint32_t) * V);
    G->offs = take(sizeof(uint32_t) * (V + 1));
    G->angles = take(sizeof(double) * 2 * me);
    G->nbr = take(sizeof(int32_t) * 2 * me);
    G->dv = take(sizeof(double) * V);
    G->big_list = take(sizeof(int32_t) * V);
    G->n_sort_blocks = nb;
    G->total = off;
    return true;
}

hipError_t launch_radix_sort(uint32_t *keys, int32_t *vals, uint32_t *keys2, int32_t *vals2,
                             int64_t n, uint32_t *hist, uint32_t *hist_off,
                             unsigned long long *scan_tile, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + kSortTile - 1) / kSortTile;
    uint32_t *ki = keys, *ko = keys2;
    int32_t *vi = vals, *vo = vals2;
    for (int shift = 0; shift < 32; shift += 8) {    // four passes: the result ends in keys
        hipLaunchKernelGGL(sort_hist_kernel, dim3((unsigned)nb), dim3(256), 0, st, ki, n, shift,
                           hist, nb);
        RB_TRY(hipGetLastError());
        RB_TRY(launch_scan(hist, 256 * nb, scan_tile, hist_off, st));
        hipLaunchKernelGGL(sort_scatter_kernel, dim3((unsigned)nb), dim3(256), 0, st, ki, vi, n,
                           shift, hist_off, nb, ko, vo);
        RB_TRY(hipGetLastError());
        std::swap(ki, ko);
        std::swap(vi, vo);
    }
    return hipSuccess;
}

hipError_t launch_hub_order(const int32_t *src, const int32_t *dst, int64_t n_nodes,
                            int64_t n_edges, const HubSortBufs &B, hipStream_t st) {
    if (n_edges <= 0) return hipSuccess;
    RB_TRY(launch_degrees(src, dst, n_nodes, n_edges, B.deg, st));
    hipLaunchKernelGGL(hub_key_kernel, dim3(blocks_for(n_edges)), dim3(256), 0, st, src, dst,
                       n_nodes, n_edges, B.deg, B.keys, B.vals);
    RB_TRY(hipGetLastError());
    return launch_radix_sort(B.keys, B.vals, B.keys2, B.vals2, n_edges, B.hist, B.hist_off,
                             B.scan_tile, st);
}

hipError_t launch_grid_bounds(const float *x, const float *y, int64_t n, GridParams *gp,
                              int min_shift, int axis_bits, hipStream_t st) {
    hipLaunchKernelGGL(bounds_init_kernel, dim3(1), dim3(64), 0, st, gp);
    RB_TRY(hipGetLastError());
    if (n > 0) {
        hipLaunchKernelGGL(bounds_kernel, dim3(blocks_for(n)), dim3(256), 0, st, x, y, n, gp);
        RB_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(grid_shift_kernel, dim3(1), dim3(64), 0, st, gp, min_shift, axis_bits);
    return hipGetLastError();
}

hipError_t launch_prune_plan(const float *x, const float *y, int64_t n_nodes,
                             const int32_t *src, const int32_t *dst, int64_t m, int K,
                             const GridWs &G, char *w, hipStream_t st) {
    GridParams *gp = (GridParams *)(w + G.params);
    uint32_t *keys = (uint32_t *)(w + G.keys);
    int32_t *vals = (int32_t *)(w + G.vals);
    EdgeRec *rec = (EdgeRec *)(w + G.rec);
    int4 *box = (int4 *)(w + G.box);
    uint32_t *cnt = (uint32_t *)(w + G.tile_cnt);
    uint32_t *toff = (uint32_t *)(w + G.tile_off);
    int32_t *list = (int32_t *)(w + G.list);
    const SweepLayout lay = sweep_layout(m, K, 0, 0);
    // order: Hilbert index of the box centre on <= 2^14 cells per axis
    RB_TRY(launch_grid_bounds(x, y, n_nodes, gp, 0, 14, st));
    const int32_t *order = nullptr;
    if (m > 0) {
        hipLaunchKernelGGL(edge_key_kernel, dim3(blocks_for(m)), dim3(256), 0, st, x, y, src, dst,
                           n_nodes, m, gp, keys, vals);
        RB_TRY(hipGetLastError());
        RB_TRY(launch_radix_sort(keys, vals, (uint32_t *)(w + G.keys2),
                                 (int32_t *)(w + G.vals2), m, (uint32_t *)(w + G.hist),
                                 (uint32_t *)(w + G.hist_off),
                                 (unsigned long long *)(w + G.scan_tile), st));
        order = vals;
    }
    RB_TRY(launch_edge_prep_ordered(x, y, src, dst, n_nodes, m, G.n_edge_pad, order, rec, st));
    // boxes of every chunk of the padded records (trailing ones are empty)
    hipLaunchKernelGGL(chunk_box_kernel, dim3((unsigned)(G.n_edge_pad / kChunk)), dim3(256), 0,
                       st, rec, box);
    RB_TRY(hipGetLastError());
    hipLaunchKernelGGL(tile_count_kernel, dim3((unsigned)lay.n_row_tiles), dim3(256), 0, st, box,
                       lay.n_chunks, K, cnt);
    RB_TRY(hipGetLastError());
    RB_TRY(launch_scan(cnt, lay.n_row_tiles, (unsigned long long *)(w + G.scan_tile), toff, st));
    hipLaunchKernelGGL(tile_fill_kernel, dim3((unsigned)lay.n_row_tiles), dim3(256), 0, st, box,
                       lay.n_chunks, K, toff, list);
    return hipGetLastError();
}

hipError_t launch_crossing_pruned(const float *x, const float *y, int64_t n_nodes,
                                  const int32_t *src, const int32_t *dst, int64_t m,
                                  double ideal, const GridWs &G, char *w, int variant,
                                  double *out_metric, unsigned long long *out_count,
                                  double *out_dev_sum, hipStream_t st) {
    const int K = cross_variant(variant).rows;
    RB_TRY(launch_prune_plan(x, y, n_nodes, src, dst, m, K, G, w, st));
    const int grid = cross_list_grid(variant);
    CrossPartial *part = (CrossPartial *)(w + G.partial);
    const SweepLayout lay = sweep_layout(m, K, 0, 0);
    RB_TRY(launch_cross_list(variant, (const EdgeRec *)(w + G.rec), (const int32_t *)(w + G.list),
                             (const uint32_t *)(w + G.tile_off), lay.n_row_tiles,
                             lay.n_chunks * kChunk, grid, ideal, part, st));
    return launch_cross_finalize(part, grid, ideal, out_count, nullptr, out_metric, out_dev_sum,
                                 st);
}

hipError_t launch_occlusion_grid(const float *x, const float *y, int64_t n, double T,
                                 const GridWs &G, char *w, unsigned long long *out_count,
                                 hipStream_t st) {
    if (n < 2 || T < 0.0) {
        hipLaunchKernelGGL(set_count_kernel, dim3(1), dim3(64), 0, st, out_count, 0ull);
        return hipGetLastError();
    }
    if (T >= 17592186044416.0) {   // T >= 2^44 exceeds every squared distance: all pairs
        hipLaunchKernelGGL(set_count_kernel, dim3(1), dim3(64), 0, st, out_count,
                           (unsigned long long)n * (unsigned long long)(n - 1) / 2ull);
        return hipGetLastError();
    }
    GridParams *gp = (GridParams *)(w + G.params);
    uint32_t *keys = (uint32_t *)(w + G.keys);
    int32_t *vals = (int32_t *)(w + G.vals);
    // cell side: the smallest power of two whose square exceeds T (so >= d)
    int min_shift = 0;
    while ((double)(1ll << min_shift) * (double)(1ll << min_shift) <= T) ++min_shift;
    RB_TRY(launch_grid_bounds(x, y, n, gp, min_shift, 16, st));
    hipLaunchKernelGGL(node_key_kernel, dim3(blocks_for(n)), dim3(256), 0, st, x, y, n, gp, keys,
                       vals);
    RB_TRY(hipGetLastError());
    RB_TRY(launch_radix_sort(keys, vals, (uint32_t *)(w + G.keys2), (int32_t *)(w + G.vals2), n,
                             (uint32_t *)(w + G.hist), (uint32_t *)(w + G.hist_off),
                             (unsigned long long *)(w + G.scan_tile), st));
    int2 *pos = (int2 *)(w + G.pos);
    hipLaunchKernelGGL(gather_nodes_kernel, dim3(blocks_for(n)), dim3(256), 0, st, x, y, n, vals,
                       pos);
    RB_TRY(hipGetLastError());
    const int blocks = std::min<int>(blocks_for(n), kMaxPartials);
    OcclPartial *part = (OcclPartial *)(w + G.partial);
    hipLaunchKernelGGL(occl_grid_count_kernel, dim3(blocks), dim3(256), 0, st, keys, pos, n,
                       (long long)T, part);
    RB_TRY(hipGetLastError());
    return launch_occl_finalize(part, blocks, out_count, false, st);
}

}  // namespace rb
