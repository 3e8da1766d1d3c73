// All-pairs edge-crossing sweep (Algorithm 4) with the crossing-angle term
// of Algorithm 5 fused in.
//
// Work decomposition.  The upper triangle of each layout's |E| x |E| pair
// matrix is cut into units: a row tile of R = 256*K edges (each of the 256
// threads of a block keeps K edge records in registers) against a chunk of
// 256 column edges staged in LDS.  Row tile I meets chunks c >= I*K (the
// first K of them overlap the tile itself and keep only pairs with column
// index > row index).  The units of all layouts form one list, cut into
// equal contiguous ranges, one per block, with many more blocks than the chip
// holds at once (the dispatcher starts each block when a slot frees up, so
// blocks that meet costly units or slower compute units do not hold back the
// end of the launch).  A block keeps its row registers across the
// consecutive units of its range and writes one partial result per layout it
// touches, into slot block + layout, so the final sums run in a fixed order.
//
// Per pair (row edge e, column edge f), all in exact double arithmetic:
//   o1 = L_e(P_f),  o2 = o1 + cross,   o3 = L_f(P_e),  o4 = o3 - cross,
// where L_e(P) = dx_e*P.y - dy_e*P.x - c_e is Algorithm 4's CCW determinant
// of P against e's line, and cross = dx_e*dy_f - dy_e*dx_f.  With
// m = max(o1*o2, o3*o4):
//   m > 0   no crossing (one segment lies strictly on one side of the other's line)
//   m < 0   proper crossing (never a pair of incident edges)
//   m == 0  some end point lies on the other line: the rare path decides
//           (incident pairs are dropped, and when both products are zero the
//           bounding boxes must meet).
// The products are not formed.  Since 4 a b = (a + b)^2 - (a - b)^2, o1 o2 has
// the sign of |2 o1 + cross| - |cross| and o3 o4 that of |2 o3 - cross| -
// |cross|, and with the end-point sums S = P1 + P2 of each edge
//   t1 = 2 o1 + cross = dx_e*S_f.y - dy_e*S_f.x - 2 c_e,
//   t3 = 2 o3 - cross = dx_f*S_e.y - dy_f*S_e.x - 2 c_f,
// two FMAs each.  So m < 0 iff max(|t1|, |t3|) < |cross|, and m == 0 iff that
// maximum equals |cross|: 9 VALU operations per pair for the classification.
// The crossing angle uses the per-edge line angles th in [0, pi):
//   a = pi/2 - | |th_e - th_f| - pi/2 |,  dev = |ideal - a|
// (a = 0 for parallel lines and zero-length edges), on the angles held as
// integers in units of pi / 2^26: |ideal - a| = | | |tq_e - tq_f| - 2^25 |
// - beta | with beta = pi/2 - ideal, three v_sad_u32 (|x - y| + z), the last
// adding into the lane's 32-bit sum under the crossing mask, where the
// double form takes four operations.  The sum is folded into a double every
// 16 columns, before it can overflow.  Each deviation is within 1.5 units
// (7.0e-8) of the same expression on the double angles.
#include "rb_device.h"
#include "rb_internal.h"

namespace rb {
namespace {

constexpr double kHalfPi = 1.5707963267948966192;

// wave-wide count of lanes with p set; the ballot of a compare result is the
// compare's own lane mask, so this costs two scalar instructions
__device__ __forceinline__ uint32_t popc_ballot(bool p) {
    return (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(p));
}

// threadIdx.x rebuilt from the wave's index (a scalar) and the lane id.  One
// volatile asm block, so the compiler recomputes it where it is used instead
// of holding it in a vector register across the sweep (the 4-row angle
// kernels have none to spare).
__device__ __forceinline__ int thread_index(int wave_s) {
    int lane;
    __asm__ volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0"
                     : "=v"(lane));
    return (wave_s << 6) + lane;
}

// An edge as the sweep holds it (rows in registers, columns in LDS): end-point
// sums, direction and 2c (see sweep_form), the integer line angle and the end
// ids.  c2 and tq share one 16-byte LDS read.
struct __align__(16) SweepRec {
    double sx, sy, dx, dy, c2;
    uint32_t tq;
    int32_t pad0;
    int32_t s, t;
    int32_t pad1, pad2;
};
static_assert(sizeof(SweepRec) == 64, "sweep record is 64 bytes");

__device__ __forceinline__ SweepRec sweep_rec(const EdgeRec &r) {
    const EdgeRec e = sweep_form(r);
    SweepRec w;
    w.sx = e.x; w.sy = e.y; w.dx = e.dx; w.dy = e.dy; w.c2 = e.c;
    w.tq = e.tq; w.pad0 = 0;
    w.s = e.s; w.t = e.t;
    w.pad1 = 0; w.pad2 = 0;
    return w;
}

// |x - y| on unsigned 32-bit integers, as one v_sad_u32 (the compiler has
// no builtin for it and emits min, max and a subtraction); absdiff_s takes
// a uniform y from a scalar register
__device__ __forceinline__ uint32_t absdiff(uint32_t x, uint32_t y) {
    uint32_t r;
    __asm__("v_sad_u32 %0, %1, %2, 0" : "=v"(r) : "v"(x), "v"(y));
    return r;
}
__device__ __forceinline__ uint32_t absdiff_s(uint32_t x, uint32_t y_uniform) {
    uint32_t r;
    __asm__("v_sad_u32 %0, %1, %2, 0" : "=v"(r) : "v"(x), "s"(y_uniform));
    return r;
}

// acc += |v - beta| in the lanes of `mask` only (through EXEC, as in
// add_abs_masked)
__device__ __forceinline__ void add_dev_masked(uint32_t &acc, uint32_t v, uint32_t beta,
                                               uint64_t mask) {
    uint64_t saved;
    __asm__("s_and_saveexec_b64 %1, %2\n\t"
            "v_sad_u32 %0, %3, %4, %0\n\t"
            "s_mov_b64 exec, %1"
            : "+v"(acc), "=&s"(saved)
            : "s"(mask), "v"(v), "s"(beta)
            : "scc");
}

template <int K, bool ANGLE, bool DIAG>
__device__ __forceinline__ void sweep_chunk(const SweepRec *__restrict__ col,
                                            const int2 *__restrict__ rid,
                                            const double (&rX)[K], const double (&rY)[K],
                                            const double (&rDX)[K], const double (&rDY)[K],
                                            const double (&rC)[K], const uint32_t (&rTQ)[K],
                                            int wave_s, int diag_off, uint32_t beta,
                                            uint32_t &n_proper, uint32_t &n_touch,
                                            double &acc) {
    const uint32_t ideal_q = kHalfPiQ - beta;          // the deviation of a = 0
    // 16 columns add at most K * 16 deviations of at most 2^25 units: below
    // 2^32 for K <= 4
    static_assert(K <= 4, "the 32-bit angle sum is folded every 16 columns");
    for (int j0 = 0; j0 < kChunk; j0 += 16) {
        uint32_t accq = 0;
#pragma unroll 4
        for (int j = j0; j < j0 + 16; ++j) {
            const double cX = col[j].sx, cY = col[j].sy;
            const double cDX = col[j].dx, cDY = col[j].dy;
            // c2 and tq as one 16-byte read (tq in the low word of the second half)
            const double2 ct = *reinterpret_cast<const double2 *>(&col[j].c2);
            const double cC = ct.x;
            const uint32_t cTQ = ANGLE ? (uint32_t)__double_as_longlong(ct.y) : 0u;
            // the K rows are independent straight-line work; one wave-uniform
            // branch per column takes every row's rare pairs
            uint64_t zm[K];
            uint64_t any_zero = 0;
            const int tid_d = DIAG ? thread_index(wave_s) : 0;   // per column, diagonal units only
#pragma unroll
            for (int r = 0; r < K; ++r) {
                // rows and columns are in sweep form (end-point sums, 2c): t1 =
                // 2 o1 + cr and t3 = 2 o3 - cr directly; the two compares are
                // lane masks (scalar results) used as they are
                const double t1 = fma(rDX[r], cY, fma(-rDY[r], cX, -rC[r]));
                const double t3 = fma(cDX, rY[r], fma(-cDY, rX[r], -cC));
                const double cr = fma(-rDY[r], cDX, rDX[r] * cDY);
                const double t = dev::max_abs(t1, t3);
                uint64_t lt = __builtin_amdgcn_ballot_w64(t < fabs(cr));
                uint64_t le = __builtin_amdgcn_ballot_w64(t <= fabs(cr));
                if (DIAG) {
                    // a diagonal unit keeps column index > row index: with the
                    // tile's first row as origin, diag_off + j > r * 256 + tid
                    const uint64_t tri =
                        __builtin_amdgcn_ballot_w64(diag_off + j > r * kBlock + tid_d);
                    lt &= tri;
                    le &= tri;
                }
                zm[r] = le & ~lt;                              // max of the two products == 0
                const uint64_t pmask = lt;                     // both products < 0
                n_proper += (uint32_t)__popcll(pmask);
                if (ANGLE) {
                    // pi/2 - a = ||tq_e - tq_f| - 2^25|, then += |pi/2 - a - beta|
                    const uint32_t e = absdiff_s(absdiff(rTQ[r], cTQ), kHalfPiQ);
                    add_dev_masked(accq, e, beta, pmask);
                }
                any_zero |= zm[r];
            }
            if (__builtin_expect(any_zero != 0, 0)) {
                // most such pairs share an end id (the incident edges of a hub):
                // the id test comes first and the rest runs only for the others
                double fx = cX, fy = cY, fdx = cDX, fdy = cDY, fc = cC;
                uint32_t ftq = cTQ;
                __asm__ volatile("" : "+v"(fx), "+v"(fy), "+v"(fdx), "+v"(fdy), "+v"(fc), "+v"(ftq));
                // back from sweep form to start point and line constant (exact);
                // after the opaque copy, so none of it is hoisted out of the loop
                fx = 0.5 * (fx - fdx);
                fy = 0.5 * (fy - fdy);
                fc = 0.5 * fc;
                const int2 fid = make_int2(col[j].s, col[j].t);
                const int tid = thread_index(wave_s), lane = tid & 63;
#pragma unroll
                for (int r = 0; r < K; ++r) {
                    bool ok = false;
                    if (((zm[r] >> lane) & 1) && !dev::incident_ids(rid[r * kBlock + tid], fid)) {
                        double ex = rX[r], ey = rY[r], edx = rDX[r], edy = rDY[r], ec = rC[r];
                        __asm__ volatile("" : "+v"(ex), "+v"(ey), "+v"(edx), "+v"(edy), "+v"(ec));
                        ex = 0.5 * (ex - edx);
                        ey = 0.5 * (ey - edy);
                        ec = 0.5 * ec;
                        ok = dev::touching_apart(ex, ey, edx, edy, ec, fx, fy, fdx, fdy, fc);
                        if (ANGLE && ok) {
                            // parallel lines or a zero-length edge: a = 0
                            const double crs = fma(-edy, fdx, edx * fdy);
                            const uint32_t e = absdiff_s(absdiff(rTQ[r], ftq), kHalfPiQ);
                            accq += (crs == 0.0) ? ideal_q : absdiff_s(e, beta);
                        }
                    }
                    n_touch += popc_ballot(ok);
                }
            }
        }
        if (ANGLE) acc = fma((double)accq, kAngleUnit, acc);
    }
}

template <int K, int WAVES, bool ANGLE, bool BATCH>
__global__ __launch_bounds__(kBlock, WAVES) void cross_sweep_kernel(
    const EdgeRec *__restrict__ rec, SweepArgs a, double ideal, CrossPartial *__restrict__ part) {
    __shared__ SweepRec col[kChunk];
    __shared__ int2 rid[kBlock * K];
    __shared__ unsigned long long red_p[kBlock / 64], red_t[kBlock / 64];
    __shared__ double red_d[kBlock / 64];

    // start-up (unit position, row and chunk loads) at raised wave priority,
    // dropped while a unit is swept: at equal priority the waves already
    // sweeping take nearly every issue slot and a new block's start-up
    // stretches out
    __builtin_amdgcn_s_setprio(3);
    const int wave_s = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int64_t G = gridDim.x, b = blockIdx.x;
    const int64_t u_begin = a.unit_base + first_unit(a.n_units, G, b);
    const int64_t u_end = a.unit_base + first_unit(a.n_units, G, b + 1);
    constexpr int64_t R = (int64_t)kBlock * K;
    // pi/2 - ideal in angle units (a scalar)
    const uint32_t beta = __builtin_amdgcn_readfirstlane(quantize_angle(kHalfPi - ideal));

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
    const int64_t lu = u_begin - lay.unit_off;
    int64_t I = tile_of_unit(lu, lay.n_row_tiles, lay.n_chunks, K);
    int64_t c = I * K + (lu - units_before(I, lay.n_chunks, K));

    double rX[K], rY[K], rDX[K], rDY[K], rC[K];
    uint32_t rTQ[K];
    bool rows_loaded = false;
    unsigned long long tot_p = 0, tot_t = 0;
    double acc = 0.0;
    int64_t seg_units = 0;

    auto flush = [&](int64_t slot) {
        if (ANGLE) {
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        }
        const int t = thread_index(wave_s);
        __syncthreads();
        if ((t & 63) == 0) {
            red_p[wave_s] = tot_p;
            red_t[wave_s] = tot_t;
            red_d[wave_s] = acc;
        }
        __syncthreads();
        if (t == 0) {
            CrossPartial P;
            P.proper = 0; P.touch = 0; P.dev = 0.0; P.pad = 0.0;
            for (int w = 0; w < kBlock / 64; ++w) {
                P.proper += red_p[w];
                P.touch += red_t[w];
                P.dev += red_d[w];
            }
            part[slot] = P;
        }
        tot_p = 0; tot_t = 0; acc = 0.0;
    };

    for (int64_t u = u_begin; u < u_end; ++u) {
        __syncthreads();                       // previous chunk and row ids consumed
        if (!rows_loaded) {
            const int tid = thread_index(wave_s);
#pragma unroll
            for (int r = 0; r < K; ++r) {
                const SweepRec e = sweep_rec(edge_row(rec + lay.rec_off,
                                                      I * R + (int64_t)r * kBlock + tid,
                                                      lay.n_chunks * kChunk));
                rX[r] = e.sx; rY[r] = e.sy; rDX[r] = e.dx; rDY[r] = e.dy;
                rC[r] = e.c2; rTQ[r] = e.tq;
                rid[r * kBlock + tid] = make_int2(e.s, e.t);
            }
            rows_loaded = true;
        }
        {
            // the lane's index and staging address are rebuilt each unit: held
            // across the loop they take registers the 3- and 4-row variants
            // do not have
            const int tid = thread_index(wave_s);
            col[tid] = sweep_rec(rec[lay.rec_off + c * kChunk + tid]);
        }
        __syncthreads();
        __builtin_amdgcn_s_setprio(0);
        uint32_t n_p = 0, n_t = 0;
        const int diag_off = (int)(c - I * K) * kChunk;   // used for c < (I + 1) K only
        if (c < (I + 1) * K)
            sweep_chunk<K, ANGLE, true>(col, rid, rX, rY, rDX, rDY, rC, rTQ, wave_s, diag_off,
                                        beta, n_p, n_t, acc);
        else
            sweep_chunk<K, ANGLE, false>(col, rid, rX, rY, rDX, rDY, rC, rTQ, wave_s, diag_off,
                                         beta, n_p, n_t, acc);
        __builtin_amdgcn_s_setprio(3);
        tot_p += n_p;
        tot_t += n_t;
        ++seg_units;
        if (++c == lay.n_chunks) {
            ++I;
            c = I * K;
            rows_loaded = false;
            if (BATCH && I == lay.n_row_tiles) {
                flush(b + L);
                seg_units = 0;
                ++L;
                if (L < a.n_layouts) lay = table_entry(a.table, L);
                I = 0;
                c = 0;
            }
        }
    }
    if (seg_units > 0) flush(BATCH ? b + L : b);
}

// Sum of the partial slots of one layout, in slot order.
// The same sweep over an explicit unit list (the pruned path): tile I meets
// the chunks list[tile_off[I] .. tile_off[I+1]), in increasing order; the
// list's length lives in device memory, so every block writes its partial.
template <int K, int WAVES, bool ANGLE>
__global__ __launch_bounds__(kBlock, WAVES) void cross_list_kernel(
    const EdgeRec *__restrict__ rec, const int32_t *__restrict__ list,
    const uint32_t *__restrict__ tile_off, int64_t n_tiles, int64_t n_rec, double ideal,
    CrossPartial *__restrict__ part) {
    __shared__ SweepRec col[kChunk];
    __shared__ int2 rid[kBlock * K];
    __shared__ unsigned long long red_p[kBlock / 64], red_t[kBlock / 64];
    __shared__ double red_d[kBlock / 64];

    __builtin_amdgcn_s_setprio(3);            // start-up at raised priority, as above
    const int wave_s = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int64_t G = gridDim.x, b = blockIdx.x;
    // the first min(U, G) blocks take one equal range each, so blocks with
    // work are dispatched before the empty ones
    const int64_t U = tile_off[n_tiles];
    const int64_t n_items = std::min<int64_t>(U, G);
    const int64_t u_begin = b < n_items ? first_unit(U, n_items, b) : 0;
    const int64_t u_end = b < n_items ? first_unit(U, n_items, b + 1) : 0;
    constexpr int64_t R = (int64_t)kBlock * K;
    // pi/2 - ideal in angle units (a scalar)
    const uint32_t beta = __builtin_amdgcn_readfirstlane(quantize_angle(kHalfPi - ideal));
    if (u_begin == u_end) {                    // more blocks than kept units
        if (threadIdx.x == 0) {
            CrossPartial P;
            P.proper = 0; P.touch = 0; P.dev = 0.0; P.pad = 0.0;
            part[b] = P;
        }
        return;
    }

    // tile of the first unit: the largest I with tile_off[I] <= u_begin
    int64_t lo = 0, hi = n_tiles - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if ((int64_t)tile_off[mid] <= u_begin) lo = mid;
        else hi = mid - 1;
    }
    int64_t I = lo;

    double rX[K], rY[K], rDX[K], rDY[K], rC[K];
    uint32_t rTQ[K];
    bool rows_loaded = false;
    unsigned long long tot_p = 0, tot_t = 0;
    double acc = 0.0;

    for (int64_t u = u_begin; u < u_end; ++u) {
        while ((int64_t)tile_off[I + 1] <= u) {   // u < U = tile_off[n_tiles]: stops in range
            ++I;
            rows_loaded = false;
        }
        __syncthreads();                       // previous chunk and row ids consumed
        if (!rows_loaded) {
            const int tid = thread_index(wave_s);
#pragma unroll
            for (int r = 0; r < K; ++r) {
                const SweepRec e = sweep_rec(edge_row(rec, I * R + (int64_t)r * kBlock + tid, n_rec));
                rX[r] = e.sx; rY[r] = e.sy; rDX[r] = e.dx; rDY[r] = e.dy;
                rC[r] = e.c2; rTQ[r] = e.tq;
                rid[r * kBlock + tid] = make_int2(e.s, e.t);
            }
            rows_loaded = true;
        }
        const int64_t c = list[u];
        {
            const int tid = thread_index(wave_s);   // rebuilt each unit, as above
            col[tid] = sweep_rec(rec[c * kChunk + tid]);
        }
        __syncthreads();
        __builtin_amdgcn_s_setprio(0);
        uint32_t n_p = 0, n_t = 0;
        const int diag_off = (int)(c - I * K) * kChunk;   // used for c < (I + 1) K only
        if (c < (I + 1) * K)
            sweep_chunk<K, ANGLE, true>(col, rid, rX, rY, rDX, rDY, rC, rTQ, wave_s, diag_off,
                                        beta, n_p, n_t, acc);
        else
            sweep_chunk<K, ANGLE, false>(col, rid, rX, rY, rDX, rDY, rC, rTQ, wave_s, diag_off,
                                         beta, n_p, n_t, acc);
        __builtin_amdgcn_s_setprio(3);
        tot_p += n_p;
        tot_t += n_t;
    }
    if (ANGLE) {
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    }
    const int t = thread_index(wave_s);
    __syncthreads();
    if ((t & 63) == 0) {
        red_p[wave_s] = tot_p;
        red_t[wave_s] = tot_t;
        red_d[wave_s] = acc;
    }
    __syncthreads();
    if (t == 0) {
        CrossPartial P;
        P.proper = 0; P.touch = 0; P.dev = 0.0; P.pad = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) {
            P.proper += red_p[w];
            P.touch += red_t[w];
            P.dev += red_d[w];
        }
        part[b] = P;
    }
}

// Block i adds slots [i kFoldSpan, (i+1) kFoldSpan) in a fixed order and
// leaves the total in the span's first slot.
__global__ __launch_bounds__(256) void cross_fold_kernel(CrossPartial *__restrict__ part,
                                                         int n_part) {
    __shared__ unsigned long long sp[256], st[256];
    __shared__ double sd[256];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kFoldSpan;
    const int64_t end = std::min<int64_t>(n_part, base + kFoldSpan);
    unsigned long long p = 0, t = 0;
    double d = 0.0;
    for (int64_t i = base + tid; i < end; i += 256) {
        p += part[i].proper;
        t += part[i].touch;
        d += part[i].dev;
    }
    sp[tid] = p; st[tid] = t; sd[tid] = d;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            sp[tid] += sp[tid + s];
            st[tid] += st[tid + s];
            sd[tid] += sd[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        part[base].proper = sp[0];
        part[base].touch = st[0];
        part[base].dev = sd[0];
    }
}

// Sum of n slots part[0], part[stride], ..., then the outputs.
__global__ __launch_bounds__(256) void cross_finalize_kernel(
    const CrossPartial *__restrict__ part, int n, int stride, double ideal,
    unsigned long long *out_count, unsigned long long *out_proper, double *out_metric,
    double *out_dev_sum) {
    __shared__ unsigned long long sp[256], st[256];
    __shared__ double sd[256];
    const int tid = threadIdx.x;
    unsigned long long p = 0, t = 0;
    double d = 0.0;
    for (int i = tid; i < n; i += 256) {
        const CrossPartial &q = part[(int64_t)i * stride];
        p += q.proper;
        t += q.touch;
        d += q.dev;
    }
    sp[tid] = p; st[tid] = t; sd[tid] = d;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            sp[tid] += sp[tid + s];
            st[tid] += st[tid + s];
            sd[tid] += sd[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const unsigned long long count = sp[0] + st[0];
        if (out_count) *out_count = count;
        if (out_proper) *out_proper = sp[0];
        const double dev = sd[0] / ideal;
        if (out_dev_sum) *out_dev_sum = dev;
        if (out_metric) *out_metric = count ? 1.0 - dev / (double)count : 1.0;
    }
}

constexpr SweepVariant kCross[kCrossVariants] = {{1, 8, 0}, {2, 7, 0}, {3, 5, 0}, {4, 5, 0}};

template <int V>
struct CrossV {
    static constexpr int K = kCross[V].rows, W = kCross[V].waves;
};

template <int V, bool ANGLE, bool BATCH>
void launch_v(const EdgeRec *rec, const SweepArgs &a, int grid, double ideal, CrossPartial *part,
              hipStream_t st) {
    hipLaunchKernelGGL((cross_sweep_kernel<CrossV<V>::K, CrossV<V>::W, ANGLE, BATCH>),
                       dim3(grid), dim3(kBlock), 0, st, rec, a, ideal, part);
}

}  // namespace

SweepVariant cross_variant(int v) { return kCross[v]; }

int cross_grid(int, bool) { return kMaxPartials; }

int g_list_grid[kCrossVariants];

template <int V>
const void *list_kernel_ptr() {
    return (const void *)cross_list_kernel<CrossV<V>::K, CrossV<V>::W, true>;
}

int cross_list_grid(int v) {
    int &g = g_list_grid[v];
    if (g == 0) {
        const void *k = nullptr;
        switch (v) {
            case 0: k = list_kernel_ptr<0>(); break;
            case 1: k = list_kernel_ptr<1>(); break;
            case 2: k = list_kernel_ptr<2>(); break;
            default: k = list_kernel_ptr<3>(); break;
        }
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kBlock, 0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        g = std::min(per_cu * device_cu_count() * kListBlocksPerSlot, kMaxPartials);
    }
    return g;
}

hipError_t launch_cross_list(int v, const EdgeRec *rec, const int32_t *list,
                             const uint32_t *tile_off, int64_t n_tiles, int64_t n_rec, int grid,
                             double ideal, CrossPartial *part, hipStream_t st) {
#define RB_LCASE(V)                                                                       \
    case V:                                                                               \
        hipLaunchKernelGGL((cross_list_kernel<CrossV<V>::K, CrossV<V>::W, true>), dim3(grid), \
                           dim3(kBlock), 0, st, rec, list, tile_off, n_tiles, n_rec, ideal,   \
                           part);                                                         \
        break;
    switch (v) {
        RB_LCASE(0)
        RB_LCASE(1)
        RB_LCASE(2)
        RB_LCASE(3)
        default: return hipErrorInvalidValue;
    }
#undef RB_LCASE
    return hipGetLastError();
}

hipError_t launch_cross_sweep(int v, bool angle, const EdgeRec *rec, const SweepArgs &a,
                              int grid, double ideal, CrossPartial *part, hipStream_t st) {
    const bool batch = a.table != nullptr;
    if (batch && !variant_offered(angle ? 1 : 0, true, v)) return hipErrorInvalidValue;
#define RB_CASE(V)                                                                  \
    case V:                                                                         \
        if (angle) {                                                                \
            if (batch) launch_v<V, true, true>(rec, a, grid, ideal, part, st);      \
            else launch_v<V, true, false>(rec, a, grid, ideal, part, st);           \
        } else {                                                                    \
            if (batch) launch_v<V, false, true>(rec, a, grid, ideal, part, st);     \
            else launch_v<V, false, false>(rec, a, grid, ideal, part, st);          \
        }                                                                           \
        break;
// the batched form of the excluded variant is never built
#define RB_CASE_SINGLE(V)                                                           \
    case V:                                                                         \
        if (angle) launch_v<V, true, false>(rec, a, grid, ideal, part, st);         \
        else launch_v<V, false, false>(rec, a, grid, ideal, part, st);              \
        break;
    static_assert(kBatchCrossExcluded == 3, "the switch below builds no batched variant 3");
    switch (v) {
        RB_CASE(0)
        RB_CASE(1)
        RB_CASE(2)
        RB_CASE_SINGLE(3)
        default: return hipErrorInvalidValue;
    }
#undef RB_CASE
#undef RB_CASE_SINGLE
    return hipGetLastError();
}

hipError_t launch_cross_finalize(CrossPartial *part, int n_part, double ideal,
                                 unsigned long long *out_count, unsigned long long *out_proper,
                                 double *out_metric, double *out_dev_sum, hipStream_t st) {
    int n = n_part, stride = 1;
    if (n_part > kFoldSpan) {
        n = (n_part + kFoldSpan - 1) / kFoldSpan;
        stride = kFoldSpan;
        hipLaunchKernelGGL(cross_fold_kernel, dim3(n), dim3(256), 0, st, part, n_part);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(cross_finalize_kernel, dim3(1), dim3(256), 0, st, part, n, stride, ideal,
                       out_count, out_proper, out_metric, out_dev_sum);
    return hipGetLastError();
}

}  // namespace rb
