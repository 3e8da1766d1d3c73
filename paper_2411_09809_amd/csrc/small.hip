// The O(|E|) and O(sum deg log deg) metrics and the layout validator:
//   edge length variation (Algorithm 3), minimum angle (Algorithm 2),
//   precondition checks.
// Every floating-point reduction runs over a fixed grid and combines block
// partials in a fixed order, so results are bit-reproducible.
#include "rb_device.h"
#include "rb_internal.h"

namespace rb {
namespace {

using dev::block_sum;
using dev::direction_angle;
using dev::dv_of;
using dev::edge_length;
using dev::kTwoPi;
using dev::valid_ids;
constexpr int kRedGrid = 1024;       // blocks of the fixed-grid reductions

// ---------------------------------------------------- edge length variation

__global__ __launch_bounds__(256) void elv_pass_kernel(const float *__restrict__ x,
                                                       const float *__restrict__ y,
                                                       const int32_t *__restrict__ src,
                                                       const int32_t *__restrict__ dst,
                                                       int64_t n_nodes, int64_t n_edges,
                                                       const Scalars *sc, int second,
                                                       double *__restrict__ partial) {
    __shared__ double sh[256];
    const double mu = second ? sc->mean : 0.0;
    double acc = 0.0;
    for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < n_edges; e += (int64_t)gridDim.x * 256) {
        const int32_t s = src[e], t = dst[e];
        if (!valid_ids(s, t, n_nodes)) continue;
        const double l = edge_length(x, y, s, t);
        if (second) {
            const double d = l - mu;
            acc = fma(d, d, acc);
        } else {
            acc += l;
        }
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void elv_reduce_kernel(const double *__restrict__ partial,
                                                         int n_part, int64_t n_edges, int second,
                                                         Scalars *sc, double *out_metric,
                                                         double *out_mean) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n_part; i += 256) acc += partial[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x != 0) return;
    const double N = (double)n_edges;
    if (!second) {
        const double mu = n_edges > 0 ? s / N : 0.0;
        sc->mean = mu;
        if (out_mean) *out_mean = mu;
    } else {
        const double mu = sc->mean;
        double m = 0.0;
        if (n_edges >= 2 && mu > 0.0) m = sqrt(s / (N * mu * mu)) / sqrt(N - 1.0);
        *out_metric = m;
    }
}

// ------------------------------------------------------------ minimum angle

__global__ void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void zero_scalars_kernel(Scalars *sc) {
    if (threadIdx.x == 0) {
        sc->mean = 0.0;
        sc->sum_dv = 0.0;
        sc->n_used = 0;
        sc->big_count = 0;
        sc->ml = 0.0;
        sc->eca = 0.0;
        sc->count = 0;
        sc->flags = 0;
    }
}

__global__ __launch_bounds__(256) void degree_kernel(const int32_t *__restrict__ src,
                                                     const int32_t *__restrict__ dst,
                                                     int64_t n_nodes, int64_t n_edges,
                                                     uint32_t *deg) {
    for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < n_edges; e += (int64_t)gridDim.x * 256) {
        const int32_t s = src[e], t = dst[e];
        if (!valid_ids(s, t, n_nodes)) continue;
        atomicAdd(&deg[s], 1u);
        atomicAdd(&deg[t], 1u);
    }
}

// exclusive scan of deg[0..n) into offs[0..n], in tiles of 2048 elements
constexpr int kScanTile = 2048;

__global__ __launch_bounds__(256) void scan_tile_sums_kernel(const uint32_t *__restrict__ deg,
                                                             int64_t n,
                                                             unsigned long long *tile_sum) {
    __shared__ unsigned long long sh[256];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    unsigned long long s = 0;
    for (int k = 0; k < kScanTile / 256; ++k) {
        const int64_t i = base + (int64_t)k * 256 + threadIdx.x;
        if (i < n) s += deg[i];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void scan_tile_offsets_kernel(unsigned long long *tile_sum,
                                                                int64_t n_tiles) {
    // one block: exclusive scan, 256 tiles at a time with a running carry
    __shared__ unsigned long long sh[256];
    unsigned long long carry = 0;
    for (int64_t base = 0; base < n_tiles; base += 256) {
        const int64_t i = base + threadIdx.x;
        const unsigned long long v = i < n_tiles ? tile_sum[i] : 0ull;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int k = 1; k < 256; k <<= 1) {
            unsigned long long t = threadIdx.x >= k ? sh[threadIdx.x - k] : 0ull;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < n_tiles) tile_sum[i] = carry + sh[threadIdx.x] - v;
        carry += sh[255];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void scan_tile_apply_kernel(const uint32_t *__restrict__ deg,
                                                              int64_t n,
                                                              const unsigned long long *tile_off,
                                                              uint32_t *__restrict__ offs) {
    __shared__ unsigned long long sh[256];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    constexpr int per = kScanTile / 256;
    // each thread scans `per` consecutive elements
    unsigned long long loc[per];
    unsigned long long s = 0;
    for (int k = 0; k < per; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * per + k;
        loc[k] = s;
        s += (i < n) ? deg[i] : 0u;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = 1; k < 256; k <<= 1) {
        unsigned long long t = threadIdx.x >= k ? sh[threadIdx.x - k] : 0ull;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    const unsigned long long before = tile_off[blockIdx.x] + sh[threadIdx.x] - s;
    for (int k = 0; k < per; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * per + k;
        if (i < n) offs[i] = (uint32_t)(before + loc[k]);
        if (i == n - 1) offs[n] = (uint32_t)(before + loc[k] + deg[i]);
    }
}

__global__ __launch_bounds__(256) void fill_angles_kernel(const float *__restrict__ x,
                                                          const float *__restrict__ y,
                                                          const int32_t *__restrict__ src,
                                                          const int32_t *__restrict__ dst,
                                                          int64_t n_nodes, int64_t n_edges,
                                                          const uint32_t *__restrict__ offs,
                                                          uint32_t *cursor,
                                                          double *__restrict__ ang,
                                                          int32_t *__restrict__ nbr) {
    for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < n_edges; e += (int64_t)gridDim.x * 256) {
        const int32_t s = src[e], t = dst[e];
        if (!valid_ids(s, t, n_nodes)) continue;
        const double dx = (double)x[t] - (double)x[s];
        const double dy = (double)y[t] - (double)y[s];
        const uint32_t ps = offs[s] + atomicAdd(&cursor[s], 1u);
        const uint32_t pt = offs[t] + atomicAdd(&cursor[t], 1u);
        // the reverse difference is taken from the coordinates, not negated:
        // a zero-length edge must give +0 (angle 0), never -0 (atan2 -> -pi)
        const double rdx = (double)x[s] - (double)x[t];
        const double rdy = (double)y[s] - (double)y[t];
        ang[ps] = direction_angle(dx, dy);       // at s, towards t
        ang[pt] = direction_angle(rdx, rdy);     // at t, towards s
        if (nbr) {                               // the far end of each half-edge
            nbr[ps] = t;
            nbr[pt] = s;
        }
    }
}

// Nodes of degree <= kSmallDeg: one thread each.  The smallest gap between
// circularly consecutive angles equals the smallest circular distance
// min(|a_i - a_j|, 2 pi - |a_i - a_j|) over all pairs, so no sort is needed.
__global__ __launch_bounds__(256) void min_angle_small_kernel(
    const uint32_t *__restrict__ deg, const uint32_t *__restrict__ offs,
    const double *__restrict__ ang, int64_t n_nodes, double *__restrict__ dv,
    int32_t *__restrict__ big_list, Scalars *sc) {
    for (int64_t v = blockIdx.x * 256 + threadIdx.x; v < n_nodes; v += (int64_t)gridDim.x * 256) {
        const uint32_t d = deg[v];
        if (d == 0) {
            dv[v] = 0.0;
            continue;
        }
        if (d > (uint32_t)kSmallDeg) {
            const unsigned long long slot = atomicAdd(&sc->big_count, 1ull);
            big_list[slot] = (int32_t)v;
            continue;
        }
        const uint32_t o = offs[v];
        double a[kSmallDeg];
#pragma unroll
        for (int i = 0; i < kSmallDeg; ++i) a[i] = (uint32_t)i < d ? ang[o + i] : 0.0;
        double best = kTwoPi;
#pragma unroll
        for (int i = 0; i < kSmallDeg; ++i) {
#pragma unroll
            for (int j = i + 1; j < kSmallDeg; ++j) {
                if ((uint32_t)j < d) {
                    const double g = fabs(a[i] - a[j]);
                    best = fmin(best, fmin(g, kTwoPi - g));
                }
            }
        }
        dv[v] = dv_of(best, d);
    }
}

// Ascending sort of a[0..n) by a bitonic network in which every comparator
// puts the minimum at the lower index; indices >= n act as +infinity and are
// never touched, so n need not be a power of two.
__device__ void block_sort(double *a, uint32_t n) {
    uint32_t P = 1;
    while (P < n) P <<= 1;
    const uint32_t half = P >> 1;
    for (uint32_t k = 2; k <= P; k <<= 1) {
        const uint32_t hk = k >> 1;
        for (uint32_t q = threadIdx.x; q < half; q += blockDim.x) {
            const uint32_t i = (q / hk) * k + (q % hk);
            const uint32_t j = i ^ (k - 1);
            if (j < n) {
                const double u = a[i], w = a[j];
                if (w < u) { a[i] = w; a[j] = u; }
            }
        }
        __syncthreads();
        for (uint32_t s = hk >> 1; s > 0; s >>= 1) {
            for (uint32_t q = threadIdx.x; q < half; q += blockDim.x) {
                const uint32_t i = (q / s) * (2 * s) + (q % s);
                const uint32_t j = i + s;
                if (j < n) {
                    const double u = a[i], w = a[j];
                    if (w < u) { a[i] = w; a[j] = u; }
                }
            }
            __syncthreads();
        }
    }
}

// Nodes of larger degree: one block each; sort (in LDS, or in place in the
// angle array for the largest degrees), then the smallest consecutive gap,
// the wrap-around gap included (GetMinAngle of Algorithm 2).
__global__ __launch_bounds__(256) void min_angle_big_kernel(
    const uint32_t *__restrict__ deg, const uint32_t *__restrict__ offs, double *ang,
    const int32_t *__restrict__ big_list, const Scalars *sc, double *__restrict__ dv) {
    __shared__ double buf[kLdsDeg];
    __shared__ double red[256];
    const unsigned long long n_big = sc->big_count;
    for (unsigned long long k = blockIdx.x; k < n_big; k += gridDim.x) {
        const int32_t v = big_list[k];
        const uint32_t d = deg[v];
        double *seg = ang + offs[v];
        double *a = seg;
        if (d <= (uint32_t)kLdsDeg) {
            for (uint32_t i = threadIdx.x; i < d; i += blockDim.x) buf[i] = seg[i];
            a = buf;
        }
        __syncthreads();
        block_sort(a, d);
        double best = kTwoPi;
        for (uint32_t i = threadIdx.x + 1; i < d; i += blockDim.x) best = fmin(best, a[i] - a[i - 1]);
        if (threadIdx.x == 0) best = fmin(best, (kTwoPi - a[d - 1]) + a[0]);
        red[threadIdx.x] = best;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (threadIdx.x < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
            __syncthreads();
        }
        if (threadIdx.x == 0) dv[v] = dv_of(red[0], d);
        __syncthreads();
    }
}

// ------------------------------------------------ minimum-angle gradient
//
// Term T = w_m (1 - M_a), 1 - M_a = 1 - (1/N) sum_v phi_v deg_v / (2 pi) over
// the N vertices of degree >= 1.  phi_v, the smallest gap between v's sorted
// directions, moves with the two directions p -> q that bound it:
// dT/dphi_v = -w_m deg_v / (2 pi N); a direction of v -> u turns as
// (-dy, dx) / l^2 with u (and the opposite with v).  A vertex contributes only
// if its smallest gap is attained once, is nonzero and both bounding edges
// have nonzero length (the kinks contribute 0).  The gaps are those of the
// sorted sweep of Algorithm 2: from each direction to the next, and from the
// last to the first.

__device__ __forceinline__ void ma_scatter(const float *x, const float *y, int32_t v, int32_t up,
                                           int32_t uq, double c, double *gx, double *gy) {
    const double pdx = (double)x[up] - (double)x[v], pdy = (double)y[up] - (double)y[v];
    const double qdx = (double)x[uq] - (double)x[v], qdy = (double)y[uq] - (double)y[v];
    const double pl2 = fma(pdx, pdx, pdy * pdy), ql2 = fma(qdx, qdx, qdy * qdy);
    if (pl2 == 0.0 || ql2 == 0.0) return;
    // phi = alpha_q - alpha_p
    const double qx = c * -qdy / ql2, qy = c * qdx / ql2;
    const double px = c * -pdy / pl2, py = c * pdx / pl2;
    atomicAdd(&gx[uq], qx);
    atomicAdd(&gy[uq], qy);
    atomicAdd(&gx[up], -px);
    atomicAdd(&gy[up], -py);
    atomicAdd(&gx[v], px - qx);
    atomicAdd(&gy[v], py - qy);
}

// Which gap is smallest, and whether it is attained more than once, is
// decided exactly on the integer directions (the angles only order them:
// distinct integer directions below 2^21 differ in angle by far more than
// the rounding of atan2).  The gap from direction p to the next direction q
// is the angle of the rotation taking p to q: the argument, in [0, 2 pi), of
// z = (p . q, p x q), whose parts are integers below 2^44.  Two arguments are
// compared by the half plane of z and then the sign of the cross product of
// the two z in 128-bit integers.  A zero-length edge points along +x (its
// angle is atan2(0, 0) = 0).
struct GapZ {
    long long dot, cr;
};

__device__ __forceinline__ GapZ gap_z(long long px, long long py, long long qx, long long qy) {
    if (px == 0 && py == 0) px = 1;
    if (qx == 0 && qy == 0) qx = 1;
    return {px * qx + py * qy, px * qy - py * qx};
}

// 0 for an argument in [0, pi), 1 for [pi, 2 pi)
__device__ __forceinline__ int gap_half(GapZ z) {
    return (z.cr > 0 || (z.cr == 0 && z.dot > 0)) ? 0 : 1;
}

// sign of arg(a) - arg(b)
__device__ __forceinline__ int gap_cmp(GapZ a, GapZ b) {
    const int ha = gap_half(a), hb = gap_half(b);
    if (ha != hb) return ha < hb ? -1 : 1;
    const __int128 c = (__int128)a.dot * b.cr - (__int128)a.cr * b.dot;
    return c > 0 ? -1 : (c < 0 ? 1 : 0);
}

__device__ __forceinline__ bool gap_is_zero(GapZ z) { return z.cr == 0 && z.dot > 0; }

// integer direction v -> u (coordinates are integers, |c| <= 2^20)
__device__ __forceinline__ void int_dir(const float *x, const float *y, int32_t v, int32_t u,
                                        long long *dx, long long *dy) {
    *dx = (long long)(x[u] - x[v]);
    *dy = (long long)(y[u] - y[v]);
}

// degree 2 .. kSmallDeg: one thread per vertex.  Directions are taken in
// (angle, slot) order; the gap after direction i runs to its successor in
// that order, the gap after the last direction wraps to the first.
__global__ __launch_bounds__(256) void ma_grad_small_kernel(
    const float *__restrict__ x, const float *__restrict__ y, const uint32_t *__restrict__ deg,
    const uint32_t *__restrict__ offs, const double *__restrict__ ang,
    const int32_t *__restrict__ nbr, int64_t n_nodes, double w_m,
    const unsigned long long *__restrict__ n_used, int32_t *__restrict__ big,
    unsigned long long *big_count, double *gx, double *gy) {
    const unsigned long long N = *n_used;
    if (N == 0) return;
    const double c0 = -w_m / ((double)N * kTwoPi);
    for (int64_t v = blockIdx.x * 256 + threadIdx.x; v < n_nodes; v += (int64_t)gridDim.x * 256) {
        const uint32_t d = deg[v];
        if (d < 2) continue;
        if (d > (uint32_t)kSmallDeg) {
            big[atomicAdd(big_count, 1ull)] = (int32_t)v;
            continue;
        }
        const uint32_t o = offs[v];
        double a[kSmallDeg];
        int32_t ex[kSmallDeg], ey[kSmallDeg];
#pragma unroll
        for (int i = 0; i < kSmallDeg; ++i) {
            a[i] = 0.0;
            ex[i] = 0;
            ey[i] = 0;
            if ((uint32_t)i < d) {
                a[i] = ang[o + i];
                long long dx, dy;
                int_dir(x, y, (int32_t)v, nbr[o + i], &dx, &dy);
                ex[i] = (int32_t)dx;
                ey[i] = (int32_t)dy;
            }
        }
        // first direction in (angle, slot) order
        double alo = a[0];
        int lo = 0;
        int32_t lox = ex[0], loy = ey[0];
#pragma unroll
        for (int i = 1; i < kSmallDeg; ++i) {
            if ((uint32_t)i < d && a[i] < alo) {
                alo = a[i];
                lo = i;
                lox = ex[i];
                loy = ey[i];
            }
        }
        GapZ best = {0, 0};
        int at_p = -1, at_q = -1, ties = 0;
#pragma unroll
        for (int i = 0; i < kSmallDeg; ++i) {
            if ((uint32_t)i >= d) continue;
            int nx = -1;                     // successor of (a_i, i)
            double an = 0.0;
            int32_t nqx = 0, nqy = 0;
#pragma unroll
            for (int j = 0; j < kSmallDeg; ++j) {
                if ((uint32_t)j >= d || j == i) continue;
                const bool after = j > i ? a[j] >= a[i] : a[j] > a[i];
                if (after && (nx < 0 || a[j] < an)) {
                    nx = j;
                    an = a[j];
                    nqx = ex[j];
                    nqy = ey[j];
                }
            }
            if (nx < 0) {                    // the wrap gap to the first direction
                nx = lo;
                nqx = lox;
                nqy = loy;
            }
            const GapZ z = gap_z(ex[i], ey[i], nqx, nqy);
            const int c = at_p < 0 ? -1 : gap_cmp(z, best);
            if (c < 0) {
                best = z;
                at_p = i;
                at_q = nx;
                ties = 1;
            } else if (c == 0) {
                ++ties;
            }
        }
        if (ties != 1 || gap_is_zero(best)) continue;
        ma_scatter(x, y, (int32_t)v, nbr[o + at_p], nbr[o + at_q], c0 * (double)d, gx, gy);
    }
}

// (angle, slot) pairs sorted together by the bitonic network of block_sort
__device__ void block_sort_pairs(double *a, int32_t *p, uint32_t n) {
    uint32_t P = 1;
    while (P < n) P <<= 1;
    const uint32_t half = P >> 1;
    auto cmpx = [&](uint32_t i, uint32_t j) {
        const double u = a[i], w = a[j];
        if (w < u || (w == u && p[j] < p[i])) {
            a[i] = w; a[j] = u;
            const int32_t t = p[i]; p[i] = p[j]; p[j] = t;
        }
    };
    for (uint32_t k = 2; k <= P; k <<= 1) {
        const uint32_t hk = k >> 1;
        for (uint32_t q = threadIdx.x; q < half; q += blockDim.x) {
            const uint32_t i = (q / hk) * k + (q % hk);
            const uint32_t j = i ^ (k - 1);
            if (j < n) cmpx(i, j);
        }
        __syncthreads();
        for (uint32_t s = hk >> 1; s > 0; s >>= 1) {
            for (uint32_t q = threadIdx.x; q < half; q += blockDim.x) {
                const uint32_t i = (q / s) * (2 * s) + (q % s);
                const uint32_t j = i + s;
                if (j < n) cmpx(i, j);
            }
            __syncthreads();
        }
    }
}

// degree > kSmallDeg: one block per vertex; sorts the vertex's (angle,
// neighbour) pairs in LDS, or in place in the arrays beyond kLdsDeg
__global__ __launch_bounds__(256) void ma_grad_big_kernel(
    const float *__restrict__ x, const float *__restrict__ y, const uint32_t *__restrict__ deg,
    const uint32_t *__restrict__ offs, double *ang, int32_t *nbr,
    const int32_t *__restrict__ big, const unsigned long long *big_count, double w_m,
    const unsigned long long *__restrict__ n_used, double *gx, double *gy) {
    __shared__ double sa[kLdsDeg];
    __shared__ int32_t sp[kLdsDeg];
    __shared__ long long rd[256], rc[256];
    __shared__ int32_t ri[256];
    __shared__ uint32_t rt[256];
    const unsigned long long n_big = *big_count, N = *n_used;
    const double c0 = N ? -w_m / ((double)N * kTwoPi) : 0.0;
    for (unsigned long long k = blockIdx.x; k < n_big; k += gridDim.x) {
        const int32_t v = big[k];
        const uint32_t d = deg[v];
        double *a = ang + offs[v];
        int32_t *p = nbr + offs[v];
        if (d <= (uint32_t)kLdsDeg) {
            for (uint32_t i = threadIdx.x; i < d; i += blockDim.x) {
                sa[i] = a[i];
                sp[i] = p[i];
            }
            a = sa;
            p = sp;
        }
        __syncthreads();
        block_sort_pairs(a, p, d);
        // the gap after sorted direction i, as a rotation
        auto gap = [&](uint32_t i) {
            long long px, py, qx, qy;
            int_dir(x, y, v, p[i], &px, &py);
            int_dir(x, y, v, p[i + 1 < d ? i + 1 : 0], &qx, &qy);
            return gap_z(px, py, qx, qy);
        };
        // smallest gap, its first position, and how many gaps attain it
        GapZ best = {0, 0};
        int32_t at = -1;
        for (uint32_t i = threadIdx.x; i < d; i += blockDim.x) {
            const GapZ z = gap(i);
            if (at < 0 || gap_cmp(z, best) < 0) {
                best = z;
                at = (int32_t)i;
            }
        }
        rd[threadIdx.x] = best.dot;
        rc[threadIdx.x] = best.cr;
        ri[threadIdx.x] = at;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (threadIdx.x < s) {
                const int32_t oi = ri[threadIdx.x + s];
                const GapZ o = {rd[threadIdx.x + s], rc[threadIdx.x + s]};
                const GapZ m = {rd[threadIdx.x], rc[threadIdx.x]};
                if (oi >= 0 && (ri[threadIdx.x] < 0 || gap_cmp(o, m) < 0)) {
                    rd[threadIdx.x] = o.dot;
                    rc[threadIdx.x] = o.cr;
                    ri[threadIdx.x] = oi;
                }
            }
            __syncthreads();
        }
        const GapZ phi = {rd[0], rc[0]};
        const int32_t at0 = ri[0];
        uint32_t ties = 0;
        for (uint32_t i = threadIdx.x; i < d; i += blockDim.x) ties += gap_cmp(gap(i), phi) == 0;
        rt[threadIdx.x] = ties;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (threadIdx.x < s) rt[threadIdx.x] += rt[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0 && rt[0] == 1 && !gap_is_zero(phi) && at0 >= 0) {
            const uint32_t q = (uint32_t)at0 + 1 < d ? (uint32_t)at0 + 1 : 0u;
            ma_scatter(x, y, v, p[at0], p[q], c0 * (double)d, gx, gy);
        }
        __syncthreads();
    }
}

// loss += w_m (1 - M_a) over the vertices of degree >= 1
__global__ void ma_loss_kernel(double *out_loss, double w_m, const double *ma,
                               const unsigned long long *n_used) {
    if (threadIdx.x == 0 && *n_used) *out_loss += w_m * (1.0 - *ma);
}

__global__ __launch_bounds__(256) void dv_sum_kernel(const uint32_t *__restrict__ deg,
                                                     const double *__restrict__ dv,
                                                     int64_t n_nodes, double *__restrict__ partial,
                                                     unsigned long long *__restrict__ used) {
    __shared__ double sh[256];
    __shared__ unsigned long long su[256];
    double acc = 0.0;
    unsigned long long u = 0;
    for (int64_t v = blockIdx.x * 256 + threadIdx.x; v < n_nodes; v += (int64_t)gridDim.x * 256) {
        if (deg[v] > 0) {
            acc += dv[v];
            ++u;
        }
    }
    su[threadIdx.x] = u;
    const double s = block_sum(acc, sh);
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) su[threadIdx.x] += su[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = s;
        used[blockIdx.x] = su[0];
    }
}

__global__ __launch_bounds__(256) void dv_final_kernel(const double *__restrict__ partial,
                                                       const unsigned long long *__restrict__ used,
                                                       int n_part, double *out_metric,
                                                       double *out_sum_dv,
                                                       unsigned long long *out_n_used) {
    __shared__ double sh[256];
    __shared__ unsigned long long su[256];
    double acc = 0.0;
    unsigned long long u = 0;
    for (int i = threadIdx.x; i < n_part; i += 256) {
        acc += partial[i];
        u += used[i];
    }
    su[threadIdx.x] = u;
    const double s = block_sum(acc, sh);
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) su[threadIdx.x] += su[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const unsigned long long n = su[0];
        *out_metric = n ? 1.0 - s / (double)n : 1.0;
        if (out_sum_dv) *out_sum_dv = s;
        if (out_n_used) *out_n_used = n;
    }
}

// ---------------------------------------------------------------- validation

__global__ __launch_bounds__(256) void validate_nodes_kernel(const float *__restrict__ x,
                                                             const float *__restrict__ y,
                                                             int64_t n, Scalars *sc) {
    int f = 0;
    for (int64_t v = blockIdx.x * 256 + threadIdx.x; v < n; v += (int64_t)gridDim.x * 256) {
        const float a = x[v], b = y[v];
        if (!(a == floorf(a)) || !(b == floorf(b))) f |= 1;
        else if (fabsf(a) > 1048576.0f || fabsf(b) > 1048576.0f) f |= 2;
    }
    if (f) atomicOr(&sc->flags, f);
}

__device__ __forceinline__ unsigned long long mix64(unsigned long long k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

__global__ __launch_bounds__(256) void validate_edges_kernel(const int32_t *__restrict__ src,
                                                             const int32_t *__restrict__ dst,
                                                             int64_t n_edges, int64_t n_nodes,
                                                             unsigned long long *table,
                                                             int64_t table_size, Scalars *sc) {
    const unsigned long long kEmpty = ~0ull;
    int f = 0;
    for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < n_edges; e += (int64_t)gridDim.x * 256) {
        const int32_t s = src[e], t = dst[e];
        if (s < 0 || t < 0 || s >= n_nodes || t >= n_nodes) {
            f |= 4;
            continue;
        }
        if (s == t) {
            f |= 8;
            continue;
        }
        const unsigned long long lo = (unsigned long long)(s < t ? s : t);
        const unsigned long long hi = (unsigned long long)(s < t ? t : s);
        const unsigned long long key = (lo << 32) | hi;
        unsigned long long h = mix64(key) & (unsigned long long)(table_size - 1);
        // the table has at least twice as many slots as edges: the probe ends
        for (int64_t probe = 0; probe < table_size; ++probe) {
            const unsigned long long prev = atomicCAS(&table[h], kEmpty, key);
            if (prev == kEmpty) break;
            if (prev == key) {
                f |= 16;
                break;
            }
            h = (h + 1) & (unsigned long long)(table_size - 1);
        }
    }
    if (f) atomicOr(&sc->flags, f);
}

__global__ void fill_u64_kernel(unsigned long long *p, int64_t n, unsigned long long v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

int grid_for(int64_t n, int cap = 65536) {
    int64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

#define RB_TRY(expr)                          \
    do {                                      \
        hipError_t _e = (expr);               \
        if (_e != hipSuccess) return _e;      \
    } while (0)
#define RB_LAUNCHED() RB_TRY(hipGetLastError())

}  // namespace

hipError_t launch_elv(const float *x, const float *y, const int32_t *src, const int32_t *dst,
                      int64_t n_nodes, int64_t n_edges, double *partial, Scalars *sc, double *out_metric,
                      double *out_mean, hipStream_t st) {
    const int g = grid_for(n_edges, kRedGrid);
    hipLaunchKernelGGL(elv_pass_kernel, dim3(g), dim3(256), 0, st, x, y, src, dst, n_nodes, n_edges, sc, 0,
                       partial);
    RB_LAUNCHED();
    hipLaunchKernelGGL(elv_reduce_kernel, dim3(1), dim3(256), 0, st, partial, g, n_edges, 0, sc,
                       out_metric, out_mean);
    RB_LAUNCHED();
    hipLaunchKernelGGL(elv_pass_kernel, dim3(g), dim3(256), 0, st, x, y, src, dst, n_nodes, n_edges, sc, 1,
                       partial);
    RB_LAUNCHED();
    hipLaunchKernelGGL(elv_reduce_kernel, dim3(1), dim3(256), 0, st, partial, g, n_edges, 1, sc,
                       out_metric, out_mean);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st) {
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t st) {
    hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_degrees(const int32_t *src, const int32_t *dst, int64_t n_nodes,
                          int64_t n_edges, uint32_t *deg, hipStream_t st) {
    RB_TRY(launch_fill_u32(deg, n_nodes > 0 ? n_nodes : 1, 0u, st));
    if (n_edges > 0) {
        hipLaunchKernelGGL(degree_kernel, dim3(grid_for(n_edges)), dim3(256), 0, st, src, dst,
                           n_nodes, n_edges, deg);
        RB_LAUNCHED();
    }
    return hipSuccess;
}

hipError_t launch_zero_scalars(Scalars *sc, hipStream_t st) {
    hipLaunchKernelGGL(zero_scalars_kernel, dim3(1), dim3(64), 0, st, sc);
    return hipGetLastError();
}

hipError_t launch_scan(const uint32_t *deg, int64_t n, unsigned long long *tile, uint32_t *offs,
                       hipStream_t st) {
    const int64_t n_tiles = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(scan_tile_sums_kernel, dim3((unsigned)n_tiles), dim3(256), 0, st, deg, n,
                       tile);
    RB_LAUNCHED();
    hipLaunchKernelGGL(scan_tile_offsets_kernel, dim3(1), dim3(256), 0, st, tile, n_tiles);
    RB_LAUNCHED();
    hipLaunchKernelGGL(scan_tile_apply_kernel, dim3((unsigned)n_tiles), dim3(256), 0, st, deg, n,
                       tile, offs);
    return hipGetLastError();
}

hipError_t launch_min_angle_nodes(const uint32_t *deg, const uint32_t *offs, double *ang,
                                  int64_t n_nodes, double *dv, int32_t *big, Scalars *sc,
                                  hipStream_t st) {
    if (n_nodes <= 0) return hipSuccess;
    hipLaunchKernelGGL(min_angle_small_kernel, dim3(grid_for(n_nodes)), dim3(256), 0, st, deg,
                       offs, ang, n_nodes, dv, big, sc);
    RB_LAUNCHED();
    hipLaunchKernelGGL(min_angle_big_kernel, dim3(1024), dim3(256), 0, st, deg, offs, ang, big, sc,
                       dv);
    return hipGetLastError();
}

hipError_t launch_min_angle(const float *x, const float *y, int64_t n_nodes, const int32_t *src,
                            const int32_t *dst, int64_t n_edges, const MinAngleBufs &B,
                            double *out_metric, double *out_sum_dv,
                            unsigned long long *out_n_used, hipStream_t st) {
    unsigned long long *used = (unsigned long long *)B.partial + kRedGrid;
    unsigned long long *tile = (unsigned long long *)B.dv;   // dv is written only later

    const int64_t V = n_nodes > 0 ? n_nodes : 1;
    RB_TRY(launch_zero_scalars(B.sc, st));
    RB_TRY(launch_fill_u32(B.cursor, V, 0u, st));
    RB_TRY(launch_degrees(src, dst, n_nodes, n_edges, B.deg, st));
    RB_TRY(launch_scan(B.deg, V, tile, B.offs, st));
    if (n_edges > 0) {
        hipLaunchKernelGGL(fill_angles_kernel, dim3(grid_for(n_edges)), dim3(256), 0, st, x, y,
                           src, dst, n_nodes, n_edges, B.offs, B.cursor, B.ang,
                           (int32_t *)nullptr);
        RB_LAUNCHED();
    }
    RB_TRY(launch_min_angle_nodes(B.deg, B.offs, B.ang, n_nodes, B.dv, B.big, B.sc, st));
    const int g = grid_for(n_nodes, kRedGrid);
    hipLaunchKernelGGL(dv_sum_kernel, dim3(g), dim3(256), 0, st, B.deg, B.dv, n_nodes, B.partial,
                       used);
    RB_LAUNCHED();
    hipLaunchKernelGGL(dv_final_kernel, dim3(1), dim3(256), 0, st, B.partial, used, g, out_metric,
                       out_sum_dv, out_n_used);
    return hipGetLastError();
}

hipError_t launch_min_angle_grad(const float *x, const float *y, int64_t n_nodes,
                                 const int32_t *src, const int32_t *dst, int64_t n_edges,
                                 const MinAngleBufs &B, double w_m, const double *ma,
                                 const unsigned long long *n_used,
                                 unsigned long long *big_count, double *out_loss, double *gx,
                                 double *gy, hipStream_t st) {
    if (out_loss) {
        hipLaunchKernelGGL(ma_loss_kernel, dim3(1), dim3(64), 0, st, out_loss, w_m, ma, n_used);
        RB_LAUNCHED();
    }
    if (n_edges <= 0 || n_nodes <= 0) return hipSuccess;
    // the forward pass left the degrees and offsets; the directions are
    // filled again, now with the far end of every half-edge
    RB_TRY(launch_fill_u32(B.cursor, n_nodes, 0u, st));
    RB_TRY(launch_fill_u64(big_count, 1, 0ull, st));
    hipLaunchKernelGGL(fill_angles_kernel, dim3(grid_for(n_edges)), dim3(256), 0, st, x, y, src,
                       dst, n_nodes, n_edges, B.offs, B.cursor, B.ang, B.nbr);
    RB_LAUNCHED();
    hipLaunchKernelGGL(ma_grad_small_kernel, dim3(grid_for(n_nodes)), dim3(256), 0, st, x, y,
                       B.deg, B.offs, B.ang, B.nbr, n_nodes, w_m, n_used, B.big, big_count, gx,
                       gy);
    RB_LAUNCHED();
    hipLaunchKernelGGL(ma_grad_big_kernel, dim3(1024), dim3(256), 0, st, x, y, B.deg, B.offs,
                       B.ang, B.nbr, B.big, big_count, w_m, n_used, gx, gy);
    return hipGetLastError();
}

hipError_t launch_validate(const float *x, const float *y, int64_t n_nodes, const int32_t *src,
                           const int32_t *dst, int64_t n_edges, const WsLayout &L, char *ws,
                           hipStream_t st) {
    Scalars *sc = (Scalars *)(ws + L.scalars);
    unsigned long long *table = (unsigned long long *)(ws + L.hash);
    hipLaunchKernelGGL(zero_scalars_kernel, dim3(1), dim3(64), 0, st, sc);
    RB_LAUNCHED();
    hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(L.hash_size)), dim3(256), 0, st, table,
                       L.hash_size, ~0ull);
    RB_LAUNCHED();
    if (n_nodes > 0) {
        hipLaunchKernelGGL(validate_nodes_kernel, dim3(grid_for(n_nodes)), dim3(256), 0, st, x, y,
                           n_nodes, sc);
        RB_LAUNCHED();
    }
    if (n_edges > 0) {
        hipLaunchKernelGGL(validate_edges_kernel, dim3(grid_for(n_edges)), dim3(256), 0, st, src,
                           dst, n_edges, n_nodes, table, L.hash_size, sc);
        RB_LAUNCHED();
    }
    return hipSuccess;
}

}  // namespace rb
