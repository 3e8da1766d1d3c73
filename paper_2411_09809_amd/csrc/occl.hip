// All-pairs node-occlusion sweep (Algorithm 1): count unordered node pairs
// closer than the diameter d = 2r.
//
// Same decomposition as the edge sweep: a row tile of R = 256*K nodes held in
// registers (K per thread) against chunks of W nodes staged in LDS, over the upper
// triangle of each layout (row tiles against their own and later chunks), one
// block per equal contiguous range of the unit list of all layouts (many more
// blocks than the chip holds at once).  W is
// 256, or 256/S for the variants that split chunks S ways: a layout of some
// ten thousand nodes has only a few thousand 256-column units, a few per
// block slot, and the last round of blocks would leave most of the chip idle.
//
// The exact integer test |p_u - p_v|^2 <= T (T = largest integer < d^2) is
// evaluated as g = x_u x_v + (y_u y_v + q_v) >= h_u (see NodeRec).
//
// Occluding pairs are rare in any readable layout, so a chunk is first swept
// with a necessary condition in 32-bit integers, and only when some row of
// the wave meets it is the chunk swept again, counting pairs exactly.  Each
// node has a cell (cx, cy) = floor((p + 2^20) / 32), each coordinate clamped
// to [0, 65535] and packed in one word.  For integer coordinates,
// |cx_u - cx_v| <= floor(|x_u - x_v| / 32) + 1, and an occluding pair has
// |dx| + |dy| <= sqrt(2 T), so its cells satisfy
//     |cx_u - cx_v| + |cy_u - cy_v| <= isqrt(2 T) / 32 + 2 = t
// (the clamp only shrinks cell distances).  One v_sad_u16 gives the cell
// distance of a pair and one v_min3_u32 folds two of them into the row's
// running minimum: 1.5 operations per pair against 3 for the exact test
// (two fused multiply-adds and one max of g), and no per-pair scalar work
// (the CU's single scalar unit would otherwise bound the sweep).  The
// condition holds for 3 times as many pairs as occlude on the 50,000-node
// layout (diameter 64), 17 times on the 1,000,000-node one (diameter 16) and
// about 100 times on small layouts with a diameter far below the 32-unit
// cell; each such pair sends its wave through the exact count of one chunk.
#include "rb_internal.h"

namespace rb {
namespace {

// Ordered pairs (row, column) of a chunk that occlude, counted exactly.
template <int K>
__device__ __forceinline__ uint32_t occl_count(const NodeRec *__restrict__ col, int W,
                                               const double (&rX)[K], const double (&rY)[K],
                                               const double (&rH)[K]) {
    uint32_t n = 0;
    for (int j0 = 0; j0 < W; j0 += 4) {          // W is a multiple of 4
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int j = j0 + jj;
            const double cX = col[j].x, cY = col[j].y, cQ = col[j].q;
#pragma unroll
            for (int r = 0; r < K; ++r) {
                const double g = fma(rX[r], cX, fma(rY[r], cY, cQ));
                n += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(g >= rH[r]));
            }
        }
    }
    return n;
}

// A chunk of the row tile's own diagonal square: every ordered pair, less
// the self pairs of the rows that fall in this chunk.  Over the KS chunks of
// the square this counts each occluding unordered pair of the tile twice: the
// exact integer test is symmetric in the two nodes.  Masking the lower
// triangle instead costs a 64-bit index compare, a select and scalar work per
// pair.  A self pair evaluates to g = x^2 + y^2 + q = n/2 exactly (q = -n/2,
// n = x^2 + y^2, all integers or halves below 2^53), so the pair the count
// took is n >= 2h, decided here from the row's own registers.
// dk: first row of the tile less first column of the chunk (both within the
// tile's own range, so |dk| < R).
template <int K>
__device__ __forceinline__ uint32_t occl_square(const NodeRec *__restrict__ col, int W,
                                                const double (&rX)[K], const double (&rY)[K],
                                                const double (&rH)[K], int dk) {
    uint32_t n = occl_count<K>(col, W, rX, rY, rH);
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const int k = dk + (int)threadIdx.x + r * kBlock;
        const bool self = k >= 0 && k < W && fma(rX[r], rX[r], rY[r] * rY[r]) >= 2.0 * rH[r];
        n -= (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(self));
    }
    return n;
}

// Packed cell of a node; a padding record (q = -2^100) gets (65535, 65535),
// which no row within reach of the filter's limit meets
__device__ __forceinline__ uint32_t node_cell(double x, double y, double q) {
    const double cx = fmin(fmax(floor((x + 1048576.0) * 0.03125), 0.0), 65535.0);
    const double cy = fmin(fmax(floor((y + 1048576.0) * 0.03125), 0.0), 65535.0);
    const uint32_t c = (uint32_t)cx | ((uint32_t)cy << 16);
    return q < -0x1p99 ? 0xffffffffu : c;
}

// t + 1 for the threshold T (an integer in [-1, 2^44]; none occlude when T < 0)
__device__ __forceinline__ uint32_t cell_limit(double T) {
    if (T < 0.0) return 0;
    const uint64_t m = (uint64_t)(2.0 * T);
    uint64_t s = (uint64_t)sqrt((double)m);
    while (s * s > m) --s;
    while ((s + 1) * (s + 1) <= m) ++s;
    return (uint32_t)(s / 32 + 3);
}

// Cell limits beyond this pass every pair (the largest cell distance is
// 2 x 65535): such chunks go straight to the exact count.
constexpr uint32_t kNoCellFilter = 2u * 65535u + 1u;

// min(a, b, c) as one instruction: the compiler rebalances the running
// minimum into two v_min and one v_min3 per four values
__device__ __forceinline__ uint32_t min3u(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    __asm__("v_min3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// Off-diagonal chunk: the cell filter over all K rows of the wave, then the
// exact count if some row has a column within the limit lim1 - 1.
template <int K>
__device__ __forceinline__ uint32_t occl_chunk(const NodeRec *__restrict__ col,
                                               const uint32_t *__restrict__ ccell, int W,
                                               const double (&rX)[K], const double (&rY)[K],
                                               const double (&rH)[K], const uint32_t (&rC)[K],
                                               uint32_t lim1) {
    if (lim1 == 0) return 0;
    if (lim1 <= kNoCellFilter) {
        uint32_t m[K];
#pragma unroll
        for (int r = 0; r < K; ++r) m[r] = 0xffffffffu;
#pragma unroll 2
        for (int j0 = 0; j0 < W; j0 += 4) {          // W is a multiple of 4
            const uint4 c = *reinterpret_cast<const uint4 *>(ccell + j0);
#pragma unroll
            for (int r = 0; r < K; ++r) {
                m[r] = min3u(m[r], __builtin_amdgcn_sad_u16(rC[r], c.x, 0u),
                             __builtin_amdgcn_sad_u16(rC[r], c.y, 0u));
                m[r] = min3u(m[r], __builtin_amdgcn_sad_u16(rC[r], c.z, 0u),
                             __builtin_amdgcn_sad_u16(rC[r], c.w, 0u));
            }
        }
        bool any = false;
#pragma unroll
        for (int r = 0; r < K; ++r) any |= m[r] < lim1;
        if (__builtin_expect(__builtin_amdgcn_ballot_w64(any) == 0, 1)) return 0;
    }
    return occl_count<K>(col, W, rX, rY, rH);
}

// Partial slots hold twice the count: off-diagonal chunks add 2n, the
// diagonal squares their ordered pairs.  The finalize halves the total.
//
// A block starts at raised wave priority and drops it once its rows and first
// column chunk are in: at equal priority the waves already sweeping take
// nearly every issue slot, and a new block's start-up (unit position, loads,
// barriers) stretched to about as long as its sweep.  Each unit's successor
// chunk is fetched into registers while the unit is swept, except in the
// batched 8-row form, whose register budget at 5 waves per SIMD leaves no
// room for it (it would spill).
template <int K, int WAVES, bool BATCH>
__global__ __launch_bounds__(kBlock, WAVES) void occl_sweep_kernel(
    const NodeRec *__restrict__ rec, SweepArgs a, OcclPartial *__restrict__ part) {
    __builtin_amdgcn_s_setprio(3);
    __shared__ NodeRec col[kChunk];
    __shared__ __align__(16) uint32_t ccell[kChunk];
    __shared__ unsigned long long red[kBlock / 64];
    const int tid = threadIdx.x;
    const int64_t G = gridDim.x, b = blockIdx.x;
    // one unit per block (every layout below a few hundred thousand nodes):
    // block b's range is [b, b + 1), with no estimate to correct
    const bool one = a.n_units == G;
    const int64_t u_begin = a.unit_base + (one ? b : first_unit(a.n_units, G, b));
    const int64_t u_end = one ? u_begin + 1 : a.unit_base + first_unit(a.n_units, G, b + 1);
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
    SweepLayout lay = BATCH ? table_entry(a.table, L) : a.single;
    int W = kChunk >> lay.col_shift;               // columns per unit
    int64_t KS = (int64_t)K << lay.col_shift;      // chunks spanned by a row tile
    const int64_t lu = u_begin - lay.unit_off;
    // 32-bit operands when the launch's units all lie below 2^31 (a shard of a
    // huge layout may start far above)
    const bool small = one && !BATCH && a.unit_base + a.n_units <= INT32_MAX;
    int64_t I = small
                    ? tile_of_unit32((int)lu, (int)lay.n_row_tiles, (int)lay.n_chunks, (int)KS)
                    : tile_of_unit(lu, lay.n_row_tiles, lay.n_chunks, KS);
    int64_t c = I * KS + (lu - units_before(I, lay.n_chunks, KS));

    double rX[K], rY[K], rH[K];
    uint32_t rC[K];
    uint32_t lim1 = 0;
    bool rows_loaded = false;
    unsigned long long tot = 0;
    int64_t seg_units = 0;
    constexpr bool PF = !(BATCH && K == 8);
    double nX = 0.0, nY = 0.0, nQ = 0.0;           // this thread's record of the next chunk
    if (PF && u_begin < u_end && tid < W) {
        const NodeRec &v = rec[lay.rec_off + c * W + tid];
        nX = v.x; nY = v.y; nQ = v.q;
    }

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
        if (!PF && tid < W) {
            const NodeRec &v = rec[lay.rec_off + c * W + tid];
            nX = v.x; nY = v.y; nQ = v.q;
        }
        if (!rows_loaded) {
#pragma unroll
            for (int r = 0; r < K; ++r) {
                const NodeRec v = rec[lay.rec_off + I * R + (int64_t)r * kBlock + tid];
                rX[r] = v.x; rY[r] = v.y; rH[r] = v.h;
                rC[r] = node_cell(v.x, v.y, 0.0);
            }
            // the layout's T = n - 2h, from the wave's first row.  Only a tile
            // with off-diagonal units uses it, and such a tile is not the
            // layout's last, so all its rows are nodes (no padding).
            const double T = fma(rX[0], rX[0], rY[0] * rY[0]) - 2.0 * rH[0];
            lim1 = cell_limit(__longlong_as_double(uniform64(__double_as_longlong(T))));
            rows_loaded = true;
        }
        __syncthreads();
        if (tid < W) {
            col[tid].x = nX;
            col[tid].y = nY;
            col[tid].q = nQ;
            ccell[tid] = node_cell(nX, nY, nQ);
        }
        __syncthreads();
        __builtin_amdgcn_s_setprio(0);
        const int Wu = W;
        const bool diag = c < (I + 1) * KS;
        const int dk = (int)(I * R - c * W);       // used only when diag: |dk| < R
        // step to the next unit (possibly of the next layout) and fetch its chunk
        bool layout_done = false;
        if (++c == lay.n_chunks) {
            ++I;
            c = I * KS;
            rows_loaded = false;
            layout_done = BATCH && I == lay.n_row_tiles;
        }
        const int64_t L_unit = L;
        if (layout_done) {
            ++L;
            if (L < a.n_layouts) {
                lay = table_entry(a.table, L);
                W = kChunk >> lay.col_shift;
                KS = (int64_t)K << lay.col_shift;
            }
            I = 0;
            c = 0;
        }
        if (PF && u + 1 < u_end && tid < W) {
            const NodeRec &v = rec[lay.rec_off + c * W + tid];
            nX = v.x; nY = v.y; nQ = v.q;
        }
        if (diag) tot += occl_square<K>(col, Wu, rX, rY, rH, dk);
        else tot += 2 * (unsigned long long)occl_chunk<K>(col, ccell, Wu, rX, rY, rH, rC, lim1);
        ++seg_units;
        if (layout_done) {
            flush(b + L_unit);
            seg_units = 0;
        }
        __builtin_amdgcn_s_setprio(3);
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

// Sum of n slots part[0], part[stride], ..., shifted right by `shift` (1
// for the node sweep's slots, which hold twice the count)
__global__ __launch_bounds__(256) void occl_finalize_kernel(const OcclPartial *__restrict__ part,
                                                            int n, int stride, int shift,
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
    if (tid == 0) *out_count = s[0] >> shift;
}

// rows per thread, waves per SIMD, column split (log2): the split variants
// cut each 256-column chunk into 4 or 8 units, for layouts too small to
// fill the chip with whole chunks
constexpr SweepVariant kOccl[kOcclVariants] = {{8, 5, 0}, {2, 8, 0}, {4, 6, 0}, {4, 6, 2},
                                               {2, 8, 2}, {4, 6, 3}, {2, 8, 3}, {8, 5, 2},
                                               {8, 5, 3}, {4, 8, 0}, {4, 8, 2}, {4, 8, 3}};

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

int occl_grid(int v, int64_t n_units, int64_t n_nodes) {
    int64_t g = std::min<int64_t>(n_units, kMaxPartials);
    if (kOccl[v].col_shift > 0 && n_nodes >= kTwoUnitNodes) g = (g + 1) / 2;
    return (int)g;
}

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
        RB_OCASE(9)
        RB_OCASE(10)
        RB_OCASE(11)
        default: return hipErrorInvalidValue;
    }
#undef RB_OCASE
    return hipGetLastError();
}

hipError_t launch_occl_finalize(OcclPartial *part, int n_part, unsigned long long *out_count,
                                bool doubled, hipStream_t st) {
    int n = n_part, stride = 1;
    if (n_part > kFoldSpan) {
        n = (n_part + kFoldSpan - 1) / kFoldSpan;
        stride = kFoldSpan;
        hipLaunchKernelGGL(occl_fold_kernel, dim3(n), dim3(256), 0, st, part, n_part);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(occl_finalize_kernel, dim3(1), dim3(256), 0, st, part, n, stride,
                       doubled ? 1 : 0, out_count);
    return hipGetLastError();
}

}  // namespace rb
