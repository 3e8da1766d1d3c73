// All-pairs edge-crossing sweep (Algorithm 4) with the crossing-angle term
// of Algorithm 5 fused in.
//
// Work decomposition.  The upper triangle of the |E| x |E| pair matrix is cut
// into units: a row tile of R = 256*K edges (each of the 256 threads of a
// block keeps K edge records in registers) against a chunk of 256 column
// edges staged in LDS.  Row tile I meets chunks c >= I*K (the first K of them
// overlap the tile itself and keep only pairs with column index > row index).
// A persistent grid takes equal contiguous ranges of the unit list, so a
// block keeps its row registers across consecutive units and every block
// does the same number of units (+-1).
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
// The crossing angle uses the per-edge line angles th in [0, pi):
//   a = pi/2 - | |th_e - th_f| - pi/2 |,  dev = |ideal - a|
// (a = 0 for parallel lines and zero-length edges).
#include "rb_internal.h"

namespace rb {
namespace {

constexpr double kHalfPi = 1.5707963267948966192;

__device__ __forceinline__ uint32_t popc_ballot(bool p) {
    return (uint32_t)__popcll(__ballot(p));
}

__device__ __forceinline__ int64_t units_before(int64_t I, int64_t nC, int K) {
    return I * nC - (int64_t)K * I * (I - 1) / 2;
}

// Rare path: both products <= 0 and at least one is zero.
__device__ __forceinline__ bool touching_pair(double p12, double p34, double rx, double ry,
                                              double rdx, double rdy, int rs, int rt,
                                              const EdgeRec &f) {
    bool incident = (rs == f.s) | (rs == f.t) | (rt == f.s) | (rt == f.t);
    bool ok = fmin(p12, p34) < 0.0;
    if (!ok) {
        double ax0 = fmin(rx, rx + rdx), ax1 = fmax(rx, rx + rdx);
        double ay0 = fmin(ry, ry + rdy), ay1 = fmax(ry, ry + rdy);
        double bx0 = fmin(f.x, f.x + f.dx), bx1 = fmax(f.x, f.x + f.dx);
        double by0 = fmin(f.y, f.y + f.dy), by1 = fmax(f.y, f.y + f.dy);
        ok = (fmax(ax0, bx0) <= fmin(ax1, bx1)) && (fmax(ay0, by0) <= fmin(ay1, by1));
    }
    return ok & !incident;
}

template <int K, bool ANGLE, bool DIAG>
__device__ __forceinline__ void sweep_chunk(const EdgeRec *__restrict__ col,
                                            const double (&rX)[K], const double (&rY)[K],
                                            const double (&rDX)[K], const double (&rDY)[K],
                                            const double (&rC)[K], const double (&rTH)[K],
                                            const int (&rS)[K], const int (&rT)[K],
                                            int64_t row0, int64_t col0, double ideal,
                                            double angc, uint32_t &n_proper, uint32_t &n_touch,
                                            double &acc) {
#pragma unroll 2
    for (int j = 0; j < kChunk; ++j) {
        const double cX = col[j].x, cY = col[j].y;
        const double cDX = col[j].dx, cDY = col[j].dy;
        const double cC = col[j].c;
        const double cTH = ANGLE ? col[j].th : 0.0;
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const double o1 = fma(-rDY[r], cX, fma(rDX[r], cY, -rC[r]));
            const double o3 = fma(-cDY, rX[r], fma(cDX, rY[r], -cC));
            const double cr = fma(-rDY[r], cDX, rDX[r] * cDY);
            const double p12 = o1 * (o1 + cr);
            const double p34 = o3 * (o3 - cr);
            const double m = fmax(p12, p34);
            const bool in_tri = !DIAG || (col0 + j > row0 + (int64_t)r * kBlock);
            const bool prop = (m < 0.0) & in_tri;
            const bool zero = (m == 0.0) & in_tri;
            n_proper += popc_ballot(prop);
            double v = 0.0;
            if (ANGLE) {
                const double u = fabs(rTH[r] - cTH) - kHalfPi;
                v = angc + fabs(u);
                acc = fma(prop ? 1.0 : 0.0, fabs(v), acc);
            }
            if (__ballot(zero)) {
                bool ok = false;
                if (zero)
                    ok = touching_pair(p12, p34, rX[r], rY[r], rDX[r], rDY[r], rS[r], rT[r],
                                       col[j]);
                n_touch += popc_ballot(ok);
                if (ANGLE && ok) acc += (cr == 0.0) ? ideal : fabs(v);
            }
        }
    }
}

template <int K, bool ANGLE>
__global__ __launch_bounds__(kBlock) void cross_sweep_kernel(
    const EdgeRec *__restrict__ rec, int64_t nR, int64_t nC, int64_t n_units, double ideal,
    CrossPartial *__restrict__ part) {
    __shared__ EdgeRec col[kChunk];
    __shared__ unsigned long long red_p[kBlock / 64], red_t[kBlock / 64];
    __shared__ double red_d[kBlock / 64];

    const int tid = threadIdx.x;
    const int64_t G = gridDim.x, b = blockIdx.x;
    const int64_t u_begin = n_units * b / G, u_end = n_units * (b + 1) / G;
    constexpr int64_t R = (int64_t)kBlock * K;
    const double angc = ideal - kHalfPi;

    // row tile of the first unit: the largest I with units_before(I) <= u_begin
    int64_t lo = 0, hi = nR - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (units_before(mid, nC, K) <= u_begin) lo = mid;
        else hi = mid - 1;
    }
    int64_t I = lo;
    int64_t c = I * K + (u_begin - units_before(I, nC, K));

    double rX[K], rY[K], rDX[K], rDY[K], rC[K], rTH[K];
    int rS[K], rT[K];
    int64_t cur_I = -1;
    unsigned long long tot_p = 0, tot_t = 0;
    double acc = 0.0;

    for (int64_t u = u_begin; u < u_end; ++u) {
        if (I != cur_I) {
#pragma unroll
            for (int r = 0; r < K; ++r) {
                const EdgeRec e = rec[I * R + (int64_t)r * kBlock + tid];
                rX[r] = e.x; rY[r] = e.y; rDX[r] = e.dx; rDY[r] = e.dy;
                rC[r] = e.c; rTH[r] = e.th; rS[r] = e.s; rT[r] = e.t;
            }
            cur_I = I;
        }
        __syncthreads();                       // previous chunk fully consumed
        col[tid] = rec[c * kChunk + tid];
        __syncthreads();
        uint32_t n_p = 0, n_t = 0;
        const int64_t row0 = I * R + tid, col0 = c * kChunk;
        if (c < (I + 1) * K)
            sweep_chunk<K, ANGLE, true>(col, rX, rY, rDX, rDY, rC, rTH, rS, rT, row0, col0,
                                        ideal, angc, n_p, n_t, acc);
        else
            sweep_chunk<K, ANGLE, false>(col, rX, rY, rDX, rDY, rC, rTH, rS, rT, row0, col0,
                                         ideal, angc, n_p, n_t, acc);
        tot_p += n_p;
        tot_t += n_t;
        if (++c == nC) {
            ++I;
            c = I * K;
        }
    }

    // block reduction (fixed order: deterministic)
    if (ANGLE) {
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    }
    const int wave = tid >> 6, lane = tid & 63;
    if (lane == 0) {
        red_p[wave] = tot_p;
        red_t[wave] = tot_t;
        red_d[wave] = acc;
    }
    __syncthreads();
    if (tid == 0) {
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

__global__ __launch_bounds__(256) void cross_finalize_kernel(
    const CrossPartial *__restrict__ part, int n_part, double ideal,
    unsigned long long *out_count, unsigned long long *out_proper, double *out_metric,
    double *out_dev_sum) {
    __shared__ unsigned long long sp[256], st[256];
    __shared__ double sd[256];
    const int tid = threadIdx.x;
    unsigned long long p = 0, t = 0;
    double d = 0.0;
    for (int i = tid; i < n_part; i += 256) {
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
        const unsigned long long count = sp[0] + st[0];
        if (out_count) *out_count = count;
        if (out_proper) *out_proper = sp[0];
        const double dev = sd[0] / ideal;
        if (out_dev_sum) *out_dev_sum = dev;
        if (out_metric) *out_metric = count ? 1.0 - dev / (double)count : 1.0;
    }
}

int g_cross_grid[2] = {0, 0};

}  // namespace

SweepPlan plan_cross(int64_t n_edges, bool angle) {
    SweepPlan p{};
    constexpr int K = kCrossRows;
    const int64_t R = (int64_t)kBlock * K;
    const int64_t E = n_edges > 0 ? n_edges : 1;
    p.n_row_tiles = (E + R - 1) / R;
    p.n_chunks = (E + kChunk - 1) / kChunk;
    p.n_units = p.n_row_tiles * p.n_chunks - (int64_t)K * p.n_row_tiles * (p.n_row_tiles - 1) / 2;
    int &g = g_cross_grid[angle ? 1 : 0];
    if (g == 0) {
        int per_cu = 0;
        if (angle)
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, cross_sweep_kernel<K, true>, kBlock, 0);
        else
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, cross_sweep_kernel<K, false>, kBlock, 0);
        if (per_cu < 1) per_cu = 1;
        g = per_cu * device_cu_count();
        if (g > kMaxPartials) g = kMaxPartials;
    }
    p.grid = (int)(p.n_units < g ? p.n_units : g);
    return p;
}

hipError_t launch_cross_sweep(const EdgeRec *rec, const SweepPlan &p, bool angle, double ideal,
                              CrossPartial *part, hipStream_t st) {
    constexpr int K = kCrossRows;
    if (angle)
        hipLaunchKernelGGL((cross_sweep_kernel<K, true>), dim3(p.grid), dim3(kBlock), 0, st, rec,
                           p.n_row_tiles, p.n_chunks, p.n_units, ideal, part);
    else
        hipLaunchKernelGGL((cross_sweep_kernel<K, false>), dim3(p.grid), dim3(kBlock), 0, st, rec,
                           p.n_row_tiles, p.n_chunks, p.n_units, ideal, part);
    return hipGetLastError();
}

hipError_t launch_cross_finalize(const CrossPartial *part, int n_part, double ideal,
                                 unsigned long long *out_count, unsigned long long *out_proper,
                                 double *out_metric, double *out_dev_sum, hipStream_t st) {
    hipLaunchKernelGGL(cross_finalize_kernel, dim3(1), dim3(256), 0, st, part, n_part, ideal,
                       out_count, out_proper, out_metric, out_dev_sum);
    return hipGetLastError();
}

}  // namespace rb
