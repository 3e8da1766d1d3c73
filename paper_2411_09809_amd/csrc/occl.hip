// All-pairs node-occlusion sweep (Algorithm 1): count unordered node pairs
// closer than the diameter d = 2r.
//
// Same decomposition as the edge sweep: a row tile of R = 256*K nodes held in
// registers against chunks of 256 nodes staged in LDS, over the upper
// triangle of each layout, one block per equal contiguous range of the unit
// list of all layouts (many more blocks than the chip holds at once).  The exact integer test
// |p_u - p_v|^2 <= T (T = largest integer < d^2) is evaluated as
// g = x_u x_v + (y_u y_v + q_v) >= h_u (see NodeRec).
//
// Occluding pairs are rare in any readable layout, so a chunk is first swept
// keeping only each row's largest g: two fused multiply-adds and one max per
// pair, and no per-pair scalar work (the CU's single scalar unit would
// otherwise bound the sweep).  Only when some row's maximum reaches its h
// is the chunk swept again, counting pairs exactly.
#include "rb_internal.h"

namespace rb {
namespace {

__device__ __forceinline__ int64_t units_before(int64_t I, int64_t nC, int K) {
    return I * nC - (int64_t)K * I * (I - 1) / 2;
}

template <int K, bool DIAG>
__device__ __forceinline__ uint32_t occl_count(const NodeRec *__restrict__ col,
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
            n += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(hit));
        }
    }
    return n;
}

// max of two doubles as one instruction: the compiler's fmax also quiets NaN
// inputs, which costs an extra instruction per pair for the loop-carried
// maximum (no NaN reaches this sweep)
__device__ __forceinline__ double max2(double a, double b) {
    double r;
    __asm__("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

template <int K>
__device__ __forceinline__ uint32_t occl_chunk(const NodeRec *__restrict__ col,
                                               const double (&rX)[K], const double (&rY)[K],
                                               const double (&rH)[K], int64_t row0,
                                               int64_t col0) {
    double gmax[K];
#pragma unroll
    for (int r = 0; r < K; ++r) gmax[r] = -HUGE_VAL;
#pragma unroll 2
    for (int j = 0; j < kChunk; ++j) {
        const double cX = col[j].x, cY = col[j].y, cQ = col[j].q;
#pragma unroll
        for (int r = 0; r < K; ++r)
            gmax[r] = max2(gmax[r], fma(rX[r], cX, fma(rY[r], cY, cQ)));
    }
    bool any = false;
#pragma unroll
    for (int r = 0; r < K; ++r) any |= gmax[r] >= rH[r];
    if (__builtin_expect(__builtin_amdgcn_ballot_w64(any) == 0, 1)) return 0;
    return occl_count<K, false>(col, rX, rY, rH, row0, col0);
}

template <int K, int WAVES, bool BATCH>
__global__ __launch_bounds__(kBlock, WAVES) void occl_sweep_kernel(
    const NodeRec *__restrict__ rec, SweepArgs a, OcclPartial *__restrict__ part) {
    __shared__ NodeRec col[kChunk];
    __shared__ unsigned long long red[kBlock / 64];
    const int tid = threadIdx.x;
    const int64_t G = gridDim.x, b = blockIdx.x;
    const int64_t u_begin = a.unit_base + block_first_unit(a.n_units, G, b);
    const int64_t u_end = a.unit_base + block_first_unit(a.n_units, G, b + 1);
    constexpr int64_t R = (int64_t)kBlock * K;

    int64_t L = 0;
    if (BATCH) {
        int64_t lo = 0, hi = a.n_layouts - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (a.table[mid].unit_off <= u_begin) lo = mid;
            else hi = mid - 1;
        }
        L = lo;
    }
    SweepLayout lay = BATCH ? a.table[L] : a.single;
    const int64_t lu = u_begin - lay.unit_off;
    int64_t lo = 0, hi = lay.n_row_tiles - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (units_before(mid, lay.n_chunks, K) <= lu) lo = mid;
        else hi = mid - 1;
    }
    int64_t I = lo;
    int64_t c = I * K + (lu - units_before(I, lay.n_chunks, K));

    double rX[K], rY[K], rH[K];
    bool rows_loaded = false;
    unsigned long long tot = 0;
    int64_t seg_units = 0;

    auto flush = [&](int64_t slot) {
        const int wave = tid >> 6, lane = tid & 63;
        __syncthreads();
        if (lane == 0) red[wave] = tot;
        __syncthreads();
        if (tid == 0) {
            OcclPartial P;
            P.count = 0;
            P.pad = 0;
            for (int w = 0; w < kBlock / 64; ++w) P.count += red[w];
            part[slot] = P;
        }
        tot = 0;
    };

    for (int64_t u = u_begin; u < u_end; ++u) {
        if (!rows_loaded) {
#pragma unroll
            for (int r = 0; r < K; ++r) {
                const NodeRec v = rec[lay.rec_off + I * R + (int64_t)r * kBlock + tid];
                rX[r] = v.x; rY[r] = v.y; rH[r] = v.h;
            }
            rows_loaded = true;
        }
        __syncthreads();
        col[tid] = rec[lay.rec_off + c * kChunk + tid];
        __syncthreads();
        const int64_t row0 = I * R + tid, col0 = c * kChunk;
        if (c < (I + 1) * K) tot += occl_count<K, true>(col, rX, rY, rH, row0, col0);
        else tot += occl_chunk<K>(col, rX, rY, rH, row0, col0);
        ++seg_units;
        if (++c == lay.n_chunks) {
            ++I;
            c = I * K;
            rows_loaded = false;
            if (BATCH && I == lay.n_row_tiles) {
                flush(b + L);
                seg_units = 0;
                ++L;
                if (L < a.n_layouts) lay = a.table[L];
                I = 0;
                c = 0;
            }
        }
    }
    if (seg_units > 0) flush(BATCH ? b + L : b);
}

// Block i adds slots [i kFoldSpan, (i+1) kFoldSpan) and leaves the total in
// the span's first slot.
__global__ __launch_bounds__(256) void occl_fold_kernel(OcclPartial *__restrict__ part,
                                                        int n_part) {
    __shared__ unsigned long long s[256];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kFoldSpan;
    const int64_t end = std::min<int64_t>(n_part, base + kFoldSpan);
    unsigned long long c = 0;
    for (int64_t i = base + tid; i < end; i += 256) c += part[i].count;
    s[tid] = c;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (tid < k) s[tid] += s[tid + k];
        __syncthreads();
    }
    if (tid == 0) part[base].count = s[0];
}

// Sum of n slots part[0], part[stride], ...
__global__ __launch_bounds__(256) void occl_finalize_kernel(const OcclPartial *__restrict__ part,
                                                            int n, int stride,
                                                            unsigned long long *out_count) {
    __shared__ unsigned long long s[256];
    const int tid = threadIdx.x;
    unsigned long long c = 0;
    for (int i = tid; i < n; i += 256) c += part[(int64_t)i * stride].count;
    s[tid] = c;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (tid < k) s[tid] += s[tid + k];
        __syncthreads();
    }
    if (tid == 0) *out_count = s[0];
}

constexpr SweepVariant kOccl[kOcclVariants] = {{8, 4}, {2, 8}, {4, 6}};

template <int V>
struct OcclV {
    static constexpr int K = kOccl[V].rows, W = kOccl[V].waves;
};

template <int V, bool BATCH>
void launch_v(const NodeRec *rec, const SweepArgs &a, int grid, OcclPartial *part,
              hipStream_t st) {
    hipLaunchKernelGGL((occl_sweep_kernel<OcclV<V>::K, OcclV<V>::W, BATCH>), dim3(grid),
                       dim3(kBlock), 0, st, rec, a, part);
}

}  // namespace

SweepVariant occl_variant(int v) { return kOccl[v]; }

int occl_grid(int) { return kMaxPartials; }

hipError_t launch_occl_sweep(int v, const NodeRec *rec, const SweepArgs &a, int grid,
                             OcclPartial *part, hipStream_t st) {
    const bool batch = a.table != nullptr;
    switch (v) {
        case 0: batch ? launch_v<0, true>(rec, a, grid, part, st) : launch_v<0, false>(rec, a, grid, part, st); break;
        case 1: batch ? launch_v<1, true>(rec, a, grid, part, st) : launch_v<1, false>(rec, a, grid, part, st); break;
        case 2: batch ? launch_v<2, true>(rec, a, grid, part, st) : launch_v<2, false>(rec, a, grid, part, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_occl_finalize(OcclPartial *part, int n_part, unsigned long long *out_count,
                                hipStream_t st) {
    int n = n_part, stride = 1;
    if (n_part > kFoldSpan) {
        n = (n_part + kFoldSpan - 1) / kFoldSpan;
        stride = kFoldSpan;
        hipLaunchKernelGGL(occl_fold_kernel, dim3(n), dim3(256), 0, st, part, n_part);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(occl_finalize_kernel, dim3(1), dim3(256), 0, st, part, n, stride,
                       out_count);
    return hipGetLastError();
}

}  // namespace rb
