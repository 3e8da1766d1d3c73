// All-pairs node-occlusion sweep (Algorithm 1): count unordered node pairs
// closer than the diameter d = 2r.
//
// Same decomposition as the edge sweep: a row tile of R = 256*K nodes held in
// registers (K per thread) against chunks of W nodes staged in LDS, over the upper
// triangle of each layout, one block per equal contiguous range of the unit
// list of all layouts (many more blocks than the chip holds at once).  W is
// 256, or 256/S for the variants that split chunks S ways: a layout of some
// ten thousand nodes has only a few thousand 256-column units, a few per
// block slot, and the last round of blocks would leave most of the chip idle.
//
// The exact integer test |p_u - p_v|^2 <= T (T = largest integer < d^2) is
// evaluated as g = x_u x_v + (y_u y_v + q_v) >= h_u (see NodeRec).
//
// Occluding pairs are rare in any readable layout, so a chunk is first swept
// keeping only each row's largest g: two fused multiply-adds and one max per
// pair, and no per-pair scalar work (the CU's single scalar unit would
// otherwise bound the sweep).  Only when some row's maximum reaches its h
// is the chunk swept again, counting pairs exactly.
#include "rb_internal.h"

namespace rb {
namespace {

// units of the row tiles before tile I: tile i meets chunks i*KS .. nC-1
__device__ __forceinline__ int64_t units_before(int64_t I, int64_t nC, int64_t KS) {
    return I * nC - KS * I * (I - 1) / 2;
}

template <int K, bool DIAG>
__device__ __forceinline__ uint32_t occl_count(const NodeRec *__restrict__ col, int W,
                                               const double (&rX)[K], const double (&rY)[K],
                                               const double (&rH)[K], int64_t row0,
                                               int64_t col0) {
    uint32_t n = 0;
    for (int j0 = 0; j0 < W; j0 += 4) {          // W is a multiple of 4
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int j = j0 + jj;
            const double cX = col[j].x, cY = col[j].y, cQ = col[j].q;
#pragma unroll
            for (int r = 0; r < K; ++r) {
                const double g = fma(rX[r], cX, fma(rY[r], cY, cQ));
                bool hit = g >= rH[r];
                if (DIAG) hit = hit & (col0 + j > row0 + (int64_t)r * kBlock);
                n += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(hit));
            }
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
__device__ __forceinline__ uint32_t occl_chunk(const NodeRec *__restrict__ col, int W,
                                               const double (&rX)[K], const double (&rY)[K],
                                               const double (&rH)[K], int64_t row0,
                                               int64_t col0) {
    double gmax[K];
#pragma unroll
    for (int r = 0; r < K; ++r) gmax[r] = -HUGE_VAL;
    for (int j0 = 0; j0 < W; j0 += 4) {          // W is a multiple of 4
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const double cX = col[j0 + jj].x, cY = col[j0 + jj].y, cQ = col[j0 + jj].q;
#pragma unroll
            for (int r = 0; r < K; ++r)
                gmax[r] = max2(gmax[r], fma(rX[r], cX, fma(rY[r], cY, cQ)));
        }
    }
    bool any = false;
#pragma unroll
    for (int r = 0; r < K; ++r) any |= gmax[r] >= rH[r];
    if (__builtin_expect(__builtin_amdgcn_ballot_w64(any) == 0, 1)) return 0;
    return occl_count<K, false>(col, W, rX, rY, rH, row0, col0);
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
    int W = kChunk >> lay.col_shift;               // columns per unit
    int64_t KS = (int64_t)K << lay.col_shift;      // chunks spanned by a row tile
    const int64_t lu = u_begin - lay.unit_off;
    int64_t lo = 0, hi = lay.n_row_tiles - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (units_before(mid, lay.n_chunks, KS) <= lu) lo = mid;
        else hi = mid - 1;
    }
    int64_t I = lo;
    int64_t c = I * KS + (lu - units_before(I, lay.n_chunks, KS));

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
        if (tid < W) col[tid] = rec[lay.rec_off + c * W + tid];
        __syncthreads();
        const int64_t row0 = I * R + tid, col0 = c * W;
        if (c < (I + 1) * KS) tot += occl_count<K, true>(col, W, rX, rY, rH, row0, col0);
        else tot += occl_chunk<K>(col, W, rX, rY, rH, row0, col0);
        ++seg_units;
        if (++c == lay.n_chunks) {
            ++I;
            c = I * KS;
            rows_loaded = false;
            if (BATCH && I == lay.n_row_tiles) {
                flush(b + L);
                seg_units = 0;
                ++L;
                if (L < a.n_layouts) {
                    lay = a.table[L];
                    W = kChunk >> lay.col_shift;
                    KS = (int64_t)K << lay.col_shift;
                }
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

// rows per thread, waves per SIMD, column split (log2): the split variants
// cut each 256-column chunk into 4 or 8 units, for layouts too small to
// fill the chip with whole chunks
constexpr SweepVariant kOccl[kOcclVariants] = {{8, 5, 0}, {2, 8, 0}, {4, 6, 0}, {4, 6, 2},
                                               {2, 8, 2}, {4, 6, 3}, {2, 8, 3}, {8, 5, 2},
                                               {8, 5, 3}};

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
#define RB_OCASE(V)                                                                       \
    case V:                                                                               \
        if (batch) launch_v<V, true>(rec, a, grid, part, st);                             \
        else launch_v<V, false>(rec, a, grid, part, st);                                  \
        break;
    switch (v) {
        RB_OCASE(0)
        RB_OCASE(1)
        RB_OCASE(2)
        RB_OCASE(3)
        RB_OCASE(4)
        RB_OCASE(5)
        RB_OCASE(6)
        RB_OCASE(7)
        RB_OCASE(8)
        default: return hipErrorInvalidValue;
    }
#undef RB_OCASE
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
