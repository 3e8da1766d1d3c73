// All-pairs node-occlusion sweep (Algorithm 1): count unordered node pairs
// closer than the diameter d = 2r.
//
// Same decomposition as the edge sweep: a row tile of R = 256*K nodes held in
// registers against chunks of 256 nodes staged in LDS, over the upper
// triangle, by a persistent grid taking equal contiguous unit ranges.
// The exact integer test |p_u - p_v|^2 <= T (T = largest integer < d^2) is
// evaluated as  g = x_u x_v + (y_u y_v + q_v) >= h_u  (two fused multiply-adds
// and one compare per pair; see NodeRec).
#include "rb_internal.h"

namespace rb {
namespace {

__device__ __forceinline__ int64_t units_before(int64_t I, int64_t nC, int K) {
    return I * nC - (int64_t)K * I * (I - 1) / 2;
}

template <int K, bool DIAG>
__device__ __forceinline__ uint32_t occl_chunk(const NodeRec *__restrict__ col,
                                               const double (&rX)[K], const double (&rY)[K],
                                               const double (&rH)[K], int64_t row0,
                                               int64_t col0) {
    uint32_t n = 0;
#pragma unroll 2
    for (int j = 0; j < kChunk; ++j) {
        const double cX = col[j].x, cY = col[j].y, cQ = col[j].q;
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const double g = fma(rX[r], cX, fma(rY[r], cY, cQ));
            bool hit = g >= rH[r];
            if (DIAG) hit = hit & (col0 + j > row0 + (int64_t)r * kBlock);
            n += (uint32_t)__popcll(__ballot(hit));
        }
    }
    return n;
}

template <int K>
__global__ __launch_bounds__(kBlock) void occl_sweep_kernel(const NodeRec *__restrict__ rec,
                                                            int64_t nR, int64_t nC,
                                                            int64_t n_units,
                                                            OcclPartial *__restrict__ part) {
    __shared__ NodeRec col[kChunk];
    __shared__ unsigned long long red[kBlock / 64];
    const int tid = threadIdx.x;
    const int64_t G = gridDim.x, b = blockIdx.x;
    const int64_t u_begin = n_units * b / G, u_end = n_units * (b + 1) / G;
    constexpr int64_t R = (int64_t)kBlock * K;

    int64_t lo = 0, hi = nR - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (units_before(mid, nC, K) <= u_begin) lo = mid;
        else hi = mid - 1;
    }
    int64_t I = lo;
    int64_t c = I * K + (u_begin - units_before(I, nC, K));

    double rX[K], rY[K], rH[K];
    int64_t cur_I = -1;
    unsigned long long tot = 0;
    for (int64_t u = u_begin; u < u_end; ++u) {
        if (I != cur_I) {
#pragma unroll
            for (int r = 0; r < K; ++r) {
                const NodeRec v = rec[I * R + (int64_t)r * kBlock + tid];
                rX[r] = v.x; rY[r] = v.y; rH[r] = v.h;
            }
            cur_I = I;
        }
        __syncthreads();
        col[tid] = rec[c * kChunk + tid];
        __syncthreads();
        const int64_t row0 = I * R + tid, col0 = c * kChunk;
        if (c < (I + 1) * K) tot += occl_chunk<K, true>(col, rX, rY, rH, row0, col0);
        else tot += occl_chunk<K, false>(col, rX, rY, rH, row0, col0);
        if (++c == nC) {
            ++I;
            c = I * K;
        }
    }
    const int wave = tid >> 6, lane = tid & 63;
    if (lane == 0) red[wave] = tot;
    __syncthreads();
    if (tid == 0) {
        OcclPartial P;
        P.count = 0;
        P.pad = 0;
        for (int w = 0; w < kBlock / 64; ++w) P.count += red[w];
        part[b] = P;
    }
}

__global__ __launch_bounds__(256) void occl_finalize_kernel(const OcclPartial *__restrict__ part,
                                                            int n_part,
                                                            unsigned long long *out_count) {
    __shared__ unsigned long long s[256];
    const int tid = threadIdx.x;
    unsigned long long c = 0;
    for (int i = tid; i < n_part; i += 256) c += part[i].count;
    s[tid] = c;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (tid < k) s[tid] += s[tid + k];
        __syncthreads();
    }
    if (tid == 0) *out_count = s[0];
}

int g_occl_grid = 0;

}  // namespace

SweepPlan plan_occl(int64_t n_nodes) {
    SweepPlan p{};
    constexpr int K = kOcclRows;
    const int64_t R = (int64_t)kBlock * K;
    const int64_t V = n_nodes > 0 ? n_nodes : 1;
    p.n_row_tiles = (V + R - 1) / R;
    p.n_chunks = (V + kChunk - 1) / kChunk;
    p.n_units = p.n_row_tiles * p.n_chunks - (int64_t)K * p.n_row_tiles * (p.n_row_tiles - 1) / 2;
    if (g_occl_grid == 0) {
        int per_cu = 0;
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, occl_sweep_kernel<K>, kBlock,
                                                           0);
        if (per_cu < 1) per_cu = 1;
        g_occl_grid = per_cu * device_cu_count();
        if (g_occl_grid > kMaxPartials) g_occl_grid = kMaxPartials;
    }
    p.grid = (int)(p.n_units < g_occl_grid ? p.n_units : g_occl_grid);
    return p;
}

hipError_t launch_occl_sweep(const NodeRec *rec, const SweepPlan &p, OcclPartial *part,
                             hipStream_t st) {
    hipLaunchKernelGGL((occl_sweep_kernel<kOcclRows>), dim3(p.grid), dim3(kBlock), 0, st, rec,
                       p.n_row_tiles, p.n_chunks, p.n_units, part);
    return hipGetLastError();
}

hipError_t launch_occl_finalize(const OcclPartial *part, int n_part,
                                unsigned long long *out_count, hipStream_t st) {
    hipLaunchKernelGGL(occl_finalize_kernel, dim3(1), dim3(256), 0, st, part, n_part, out_count);
    return hipGetLastError();
}

}  // namespace rb
