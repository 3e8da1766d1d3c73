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
// The sort is a stable least-significant-digit radix sort of (key, value)
// pairs with 8-bit digits written here: per-block digit histograms, one
// exclusive scan over (digit, block), and a scatter that ranks items of equal
// digit by wave ballots, so the order is deterministic.
#include <climits>

#include "rb_device.h"
#include "rb_internal.h"

namespace rb {
namespace {

constexpr int kSortTile = 2048;              // items per block and pass
constexpr int kSortPer = kSortTile / 256;

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
    if ((threadIdx.x & 63) == 0) {
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
    return launch_occl_finalize(part, blocks, out_count, st);
}

}  // namespace rb
