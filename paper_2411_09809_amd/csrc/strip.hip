// The strip approximation of the enhanced edge-crossing and crossing-angle
// algorithms (Sections 3.2.2 and 3.2.3).
//
// The plane is cut into strips X_k = x0 + k w (x0 the smallest node
// coordinate, integer width w; the horizontal orientation swaps x and y).
// Within strip k only the edges spanning it take part (x_min <= X_k and
// x_max >= X_{k+1}); a pair counts as crossing when the order of the two
// edges' y values at the left line is strictly reversed at the right line,
// and the crossing angle sums |ideal - a| / ideal over those pairs.
//
// GPU form: every edge is cut into one piece per spanned strip, holding the
// numerator of its y at the left line (y at X is (y1 dx + (X - x1) dy) / dx
// with dx > 0, an integer below 2^44 over an integer below 2^22; at the right
// line the numerator grows by w dy).  A bottom-up merge sort orders the
// pieces by (strip, left y, right y); a second one by (strip, right y) counts,
// for each piece of a right run, the pieces of the left run that precede it
// in left order but follow it in right order: the reversed pairs.  Those are
// also enumerated, for the angle sum, by a separate pass per merge level
// that spreads the pairs evenly over the threads (a piece can have up to a
// run length of partners).  Ratios are compared exactly: the two cross
// products are formed as exact sums of two doubles with an FMA.
#include "rb_device.h"
#include "rb_internal.h"

namespace rb {
namespace {

constexpr double kHalfPi = 1.5707963267948966192;

struct __align__(8) Piece {
    int32_t strip;
    int32_t pad;
    double ln;      // numerator of y at the strip's left line
    double dx, dy;  // direction with dx > 0
    double th;      // line angle in [0, pi)
};
static_assert(sizeof(Piece) == 40, "piece is 40 bytes");

// sign of a/b - c/d for b, d > 0, exactly: compare a d with c b as
// unevaluated sums hi + lo of two doubles
__device__ __forceinline__ int cmp_ratio(double a, double b, double c, double d) {
    const double h1 = a * d, l1 = fma(a, d, -h1);
    const double h2 = c * b, l2 = fma(c, b, -h2);
    if (h1 != h2) return h1 < h2 ? -1 : 1;
    if (l1 != l2) return l1 < l2 ? -1 : 1;
    return 0;
}

struct ByStripLeft {          // (strip, y left, y right)
    double w;
    __device__ bool operator()(const Piece &a, const Piece &b) const {
        if (a.strip != b.strip) return a.strip < b.strip;
        const int c = cmp_ratio(a.ln, a.dx, b.ln, b.dx);
        if (c != 0) return c < 0;
        return cmp_ratio(fma(w, a.dy, a.ln), a.dx, fma(w, b.dy, b.ln), b.dx) < 0;
    }
};

struct ByStripRight {         // (strip, y right)
    double w;
    __device__ bool operator()(const Piece &a, const Piece &b) const {
        if (a.strip != b.strip) return a.strip < b.strip;
        return cmp_ratio(fma(w, a.dy, a.ln), a.dx, fma(w, b.dy, b.ln), b.dx) < 0;
    }
};

template <class Less>
__device__ __forceinline__ int64_t lower_bound(const Piece *p, int64_t lo, int64_t hi,
                                               const Piece &v, const Less &less) {
    while (lo < hi) {            // first element not less than v
        const int64_t mid = (lo + hi) >> 1;
        if (less(p[mid], v)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <class Less>
__device__ __forceinline__ int64_t upper_bound(const Piece *p, int64_t lo, int64_t hi,
                                               const Piece &v, const Less &less) {
    while (lo < hi) {            // first element greater than v
        const int64_t mid = (lo + hi) >> 1;
        if (less(v, p[mid])) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void piece_count_kernel(
    const float *__restrict__ x, const float *__restrict__ y, const int32_t *__restrict__ src,
    const int32_t *__restrict__ dst, int64_t n_nodes, int64_t m, long long w,
    const GridParams *__restrict__ gp, uint32_t *__restrict__ cnt,
    unsigned long long *__restrict__ total) {
    const long long x0 = gp->xmin;
    unsigned long long sum = 0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t s = src[e], t = dst[e];
        uint32_t c = 0;
        if (dev::valid_ids(s, t, n_nodes)) {
            const long long a = (int)x[s], b = (int)x[t];
            const long long lo = min(a, b), hi = max(a, b);
            const long long k0 = (lo - x0 + w - 1) / w, k1 = (hi - x0) / w;
            c = (uint32_t)max(0ll, k1 - k0);          // at most 2^21 strips per edge
        }
        cnt[e] = c;
        sum += c;
    }
    // the exact 64-bit total (the 32-bit offsets are valid only below 2^32)
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
    if ((threadIdx.x & 63) == 0 && sum) atomicAdd(total, sum);
}

// one thread per piece: its edge by binary search over the offsets
__global__ __launch_bounds__(256) void piece_fill_kernel(
    const float *__restrict__ x, const float *__restrict__ y, const int32_t *__restrict__ src,
    const int32_t *__restrict__ dst, int64_t m, long long w, const GridParams *__restrict__ gp,
    const uint32_t *__restrict__ off, int64_t P, Piece *__restrict__ out) {
    const long long x0 = gp->xmin;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P;
         p += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = m - 1;             // the last edge with off[e] <= p
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if ((int64_t)off[mid] <= p) lo = mid;
            else hi = mid - 1;
        }
        const int64_t e = lo;
        const int32_t s = src[e], t = dst[e];
        long long ax = (int)x[s], ay = (int)y[s], bx = (int)x[t], by = (int)y[t];
        if (bx < ax) {
            long long q = ax; ax = bx; bx = q;
            q = ay; ay = by; by = q;
        }
        const long long k = (ax - x0 + w - 1) / w + (p - (int64_t)off[e]);
        const long long X = x0 + k * w;
        Piece q;
        q.strip = (int32_t)k;
        q.pad = 0;
        q.dx = (double)(bx - ax);
        q.dy = (double)(by - ay);
        q.ln = (double)(ay * (bx - ax) + (X - ax) * (by - ay));   // exact: |.| < 2^44
        // line angle in [0, pi) as in the edge records (direction has dx > 0)
        q.th = atan2(q.dy < 0.0 ? -q.dy : q.dy, q.dy < 0.0 ? -q.dx : q.dx);
        out[p] = q;
    }
}

// one pass of the bottom-up merge sort: runs of length L merge pairwise
template <class Less>
__global__ __launch_bounds__(256) void merge_pass_kernel(const Piece *__restrict__ in,
                                                         Piece *__restrict__ out, int64_t P,
                                                         int64_t L, Less less) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < P;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = i / (2 * L) * (2 * L);
        const int64_t mid = min(s + L, P), end = min(s + 2 * L, P);
        const Piece v = in[i];
        int64_t pos;
        if (i < mid) pos = s + (i - s) + (lower_bound(in, mid, end, v, less) - mid);
        else pos = s + (i - mid) + (upper_bound(in, s, mid, v, less) - s);
        out[pos] = v;
    }
}

// merge pass by (strip, right y) that also counts, for each piece of a right
// run, the pieces of its left run after it in right order (the reversed
// pairs): cnt[i] of them, from position first[i] of the input on (0 for
// pieces of left runs).  th[i] receives the line angle of input piece i, a
// dense copy for the enumeration.  Block counts accumulate into part[block].
__global__ __launch_bounds__(256) void count_pass_kernel(const Piece *__restrict__ in,
                                                         Piece *__restrict__ out, int64_t P,
                                                         int64_t L, ByStripRight less,
                                                         uint32_t *__restrict__ cnt,
                                                         uint32_t *__restrict__ first,
                                                         double *__restrict__ th,
                                                         CrossPartial *__restrict__ part) {
    __shared__ unsigned long long rc[4];
    unsigned long long n = 0;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;   // grid covers P
    if (i < P) {
        const int64_t s = i / (2 * L) * (2 * L);
        const int64_t mid = min(s + L, P), end = min(s + 2 * L, P);
        const Piece v = in[i];
        int64_t pos;
        uint32_t c = 0, f = 0;
        if (i < mid) {
            pos = s + (i - s) + (lower_bound(in, mid, end, v, less) - mid);
        } else {
            const int64_t ub = upper_bound(in, s, mid, v, less);
            pos = s + (i - mid) + (ub - s);
            // left pieces after v in right order: same strip, right y greater
            c = (uint32_t)(mid - ub);
            f = (uint32_t)ub;
        }
        cnt[i] = c;
        first[i] = f;
        th[i] = v.th;
        n = c;
        out[pos] = v;
    }
    for (int off = 32; off > 0; off >>= 1) n += __shfl_xor(n, off, 64);
    if ((threadIdx.x & 63) == 0) rc[threadIdx.x >> 6] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
        CrossPartial Q = part[blockIdx.x];
        for (int k = 0; k < 4; ++k) Q.proper += rc[k];
        part[blockIdx.x] = Q;
    }
}

// exclusive prefix sums of cnt[0..P) in 64 bits: tiles of 1024 items
constexpr int kPreTile = 1024;

__global__ __launch_bounds__(256) void pre_tile_kernel(const uint32_t *__restrict__ cnt,
                                                       int64_t P,
                                                       unsigned long long *__restrict__ pre,
                                                       unsigned long long *__restrict__ tsum) {
    __shared__ unsigned long long w[256];
    const int64_t base = (int64_t)blockIdx.x * kPreTile + threadIdx.x * 4;
    unsigned long long v[4], t = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = base + k < P ? cnt[base + k] : 0ull;
        t += v[k];
    }
    w[threadIdx.x] = t;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {          // inclusive scan of the thread sums
        const unsigned long long add = threadIdx.x >= off ? w[threadIdx.x - off] : 0ull;
        __syncthreads();
        w[threadIdx.x] += add;
        __syncthreads();
    }
    unsigned long long run = w[threadIdx.x] - t;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (base + k < P) pre[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 255) tsum[blockIdx.x] = w[255];
}

// one block: exclusive scan of the tile sums in place; the total into *W
__global__ __launch_bounds__(256) void pre_top_kernel(unsigned long long *__restrict__ tsum,
                                                      int64_t nt,
                                                      unsigned long long *__restrict__ W) {
    __shared__ unsigned long long w[256];
    const int64_t per = (nt + 255) / 256, b0 = threadIdx.x * per;
    unsigned long long t = 0;
    for (int64_t k = b0; k < min(b0 + per, nt); ++k) t += tsum[k];
    w[threadIdx.x] = t;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const unsigned long long add = threadIdx.x >= off ? w[threadIdx.x - off] : 0ull;
        __syncthreads();
        w[threadIdx.x] += add;
        __syncthreads();
    }
    unsigned long long run = w[threadIdx.x] - t;
    for (int64_t k = b0; k < min(b0 + per, nt); ++k) {
        const unsigned long long x = tsum[k];
        tsum[k] = run;
        run += x;
    }
    if (threadIdx.x == 255) *W = w[255];
}

// the reversed pairs of one merge level, W of them, in (piece, partner)
// order, spread evenly over the waves: wave w takes pairs [w W / NW,
// (w + 1) W / NW) and walks them 64 at a time, lane l on pair base + l.  The
// window's pieces are looked up among the 64 pieces from the one holding its
// first pair (their prefix sums sit one per lane; a search over them is six
// shuffles), with a binary search over all pieces for pairs beyond those.
// Within a piece the partners' angles are 64 consecutive words.  The angle
// terms add into part[block].dev.
__device__ __forceinline__ int64_t piece_of(const unsigned long long *pre,
                                            const unsigned long long *toff, int64_t P,
                                            unsigned long long q) {
    int64_t lo = 0, hi = P - 1;                 // last piece with prefix <= q
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (toff[mid / kPreTile] + pre[mid] <= q) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void enum_pass_kernel(const double *__restrict__ th_in, int64_t P,
                                                        const uint32_t *__restrict__ first,
                                                        const unsigned long long *__restrict__ pre,
                                                        const unsigned long long *__restrict__ toff,
                                                        const unsigned long long *__restrict__ W,
                                                        double angc,
                                                        CrossPartial *__restrict__ part) {
    __shared__ double rd[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long total = *W;
    const unsigned long long NW = (unsigned long long)gridDim.x * (blockDim.x >> 6);
    const unsigned long long w = (unsigned long long)blockIdx.x * (blockDim.x >> 6) + wave;
    const unsigned long long q0 = (unsigned long long)(((unsigned __int128)total * w) / NW);
    const unsigned long long q1 = (unsigned long long)(((unsigned __int128)total * (w + 1)) / NW);
    double acc = 0.0;
    if (q0 < q1) {
        int64_t i0 = piece_of(pre, toff, P, q0);   // piece of the window's first pair
        for (unsigned long long base = q0; base < q1; base += 64) {
            // prefix sums of pieces i0 .. i0 + 63, one per lane (past the last
            // piece: the total, which no pair reaches)
            const int64_t ci = i0 + lane;
            const unsigned long long cg = ci < P ? toff[ci / kPreTile] + pre[ci] : total;
            const unsigned long long edge = __shfl(cg, 63, 64);   // prefix of piece i0 + 63
            const unsigned long long q = base + lane;
            // every lane takes part in the shuffles (no lane may be masked off)
            int j = 0;                            // last candidate with prefix <= q
#pragma unroll
            for (int step = 32; step > 0; step >>= 1) {
                const unsigned long long g = __shfl(cg, j + step < 64 ? j + step : 63, 64);
                if (j + step < 64 && g <= q) j += step;
            }
            int64_t i = i0 + j;
            if (!(q < edge || i0 + 63 >= P - 1))  // beyond the candidates
                i = q < q1 ? piece_of(pre, toff, P, q) : i0;
            if (q < q1) {
                const unsigned long long k = q - (toff[i / kPreTile] + pre[i]);
                const double u = fabs(th_in[i] - th_in[first[i] + k]) - kHalfPi;
                acc += fabs(angc + fabs(u));
            }
            // the next window starts with lane 63's pair + 1: its piece
            if (base + 64 < q1) {
                const unsigned long long nq = base + 64;
                if (nq < edge) {
                    int j = 0;
#pragma unroll
                    for (int step = 32; step > 0; step >>= 1) {
                        const unsigned long long g =
                            __shfl(cg, j + step < 64 ? j + step : 63, 64);
                        if (j + step < 64 && g <= nq) j += step;
                    }
                    i0 += j;
                } else {
                    i0 = piece_of(pre, toff, P, nq);
                }
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) rd[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        CrossPartial Q = part[blockIdx.x];
        Q.dev += rd[0] + rd[1] + rd[2] + rd[3];
        part[blockIdx.x] = Q;
    }
}

__global__ void zero_partials_kernel(CrossPartial *part, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        CrossPartial Q;
        Q.proper = 0; Q.touch = 0; Q.dev = 0.0; Q.pad = 0.0;
        part[i] = Q;
    }
}

int blocks_for(int64_t n) {
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

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

// workspace: [params, 64-bit piece total | counts | offsets | scan tiles |
// pieces | pieces | partials | per-piece pair counts, first partners and
// prefix sums, line angles | tile sums, pair total]
constexpr size_t kHead = sizeof(GridParams) + sizeof(unsigned long long);

size_t strip_ws_bytes(int64_t m, int64_t P) {
    const int64_t me = std::max<int64_t>(m, 1), pe = std::max<int64_t>(P, 1);
    const int64_t nt = (pe + kPreTile - 1) / kPreTile;
    return round256(kHead) + round256(sizeof(uint32_t) * me) +
           round256(sizeof(uint32_t) * (me + 1)) +
           round256(sizeof(unsigned long long) * (me / 2048 + 2)) +
           2 * round256(sizeof(Piece) * pe) + round256(sizeof(CrossPartial) * ((pe + 255) / 256)) +
           2 * round256(sizeof(uint32_t) * pe) + round256(sizeof(unsigned long long) * pe) +
           round256(sizeof(double) * pe) + round256(sizeof(unsigned long long) * (nt + 1));
}

// piece counts and their offsets; the total lands in off[m]
hipError_t launch_strip_count(const float *x, const float *y, const int32_t *src,
                              const int32_t *dst, int64_t n_nodes, int64_t m, int64_t w,
                              char *ws, hipStream_t st) {
    const int64_t me = std::max<int64_t>(m, 1);
    char *p = ws;
    GridParams *gp = (GridParams *)p;
    unsigned long long *total = (unsigned long long *)(p + sizeof(GridParams));
    p += round256(kHead);
    uint32_t *cnt = (uint32_t *)p; p += round256(sizeof(uint32_t) * me);
    uint32_t *off = (uint32_t *)p; p += round256(sizeof(uint32_t) * (me + 1));
    unsigned long long *tile = (unsigned long long *)p;
    RB_TRY(launch_fill_u64(total, 1, 0ull, st));
    RB_TRY(launch_grid_bounds(x, y, n_nodes, gp, 0, 16, st));
    if (m <= 0) return launch_fill_u32(off, 1, 0u, st);
    hipLaunchKernelGGL(piece_count_kernel, dim3(blocks_for(m)), dim3(256), 0, st, x, y, src, dst,
                       n_nodes, m, (long long)w, gp, cnt, total);
    RB_TRY(hipGetLastError());
    return launch_scan(cnt, m, tile, off, st);
}

const unsigned long long *strip_total_ptr(const char *ws) {
    return (const unsigned long long *)(ws + sizeof(GridParams));
}

hipError_t launch_strip_crossing(const float *x, const float *y, const int32_t *src,
                                 const int32_t *dst, int64_t n_nodes, int64_t m, int64_t w,
                                 int64_t P, double ideal, char *ws, double *out_metric,
                                 unsigned long long *out_count, double *out_dev_sum,
                                 hipStream_t st) {
    const int64_t me = std::max<int64_t>(m, 1), pe = std::max<int64_t>(P, 1);
    char *p = ws;
    GridParams *gp = (GridParams *)p; p += round256(kHead);
    p += round256(sizeof(uint32_t) * me);
    uint32_t *off = (uint32_t *)p; p += round256(sizeof(uint32_t) * (me + 1));
    p += round256(sizeof(unsigned long long) * (me / 2048 + 2));
    Piece *a = (Piece *)p; p += round256(sizeof(Piece) * pe);
    Piece *b = (Piece *)p; p += round256(sizeof(Piece) * pe);
    CrossPartial *part = (CrossPartial *)p;
    const int64_t nb = (pe + 255) / 256;
    p += round256(sizeof(CrossPartial) * nb);
    uint32_t *cnt = (uint32_t *)p; p += round256(sizeof(uint32_t) * pe);
    uint32_t *first = (uint32_t *)p; p += round256(sizeof(uint32_t) * pe);
    unsigned long long *pre = (unsigned long long *)p; p += round256(sizeof(unsigned long long) * pe);
    double *th = (double *)p; p += round256(sizeof(double) * pe);
    const int64_t nt = (pe + kPreTile - 1) / kPreTile;
    unsigned long long *toff = (unsigned long long *)p;
    unsigned long long *W = toff + nt;
    // the pair enumeration: enough threads to spread a level's pairs, at most
    // one block per partial slot
    const int enum_grid = (int)std::min<int64_t>(nb, 8192);
    hipLaunchKernelGGL(zero_partials_kernel, dim3(blocks_for(nb)), dim3(256), 0, st, part, nb);
    RB_TRY(hipGetLastError());
    if (P > 0) {
        hipLaunchKernelGGL(piece_fill_kernel, dim3(blocks_for(P)), dim3(256), 0, st, x, y, src,
                           dst, m, (long long)w, gp, off, P, a);
        RB_TRY(hipGetLastError());
        const ByStripLeft by_left{(double)w};
        for (int64_t L = 1; L < P; L *= 2) {
            hipLaunchKernelGGL(merge_pass_kernel<ByStripLeft>, dim3(blocks_for(P)), dim3(256), 0,
                               st, a, b, P, L, by_left);
            RB_TRY(hipGetLastError());
            std::swap(a, b);
        }
        const ByStripRight by_right{(double)w};
        const double angc = ideal - kHalfPi;
        for (int64_t L = 1; L < P; L *= 2) {
            hipLaunchKernelGGL(count_pass_kernel, dim3((unsigned)nb), dim3(256), 0, st, a, b, P,
                               L, by_right, cnt, first, th, part);
            RB_TRY(hipGetLastError());
            hipLaunchKernelGGL(pre_tile_kernel, dim3((unsigned)nt), dim3(256), 0, st, cnt, P, pre,
                               toff);
            RB_TRY(hipGetLastError());
            hipLaunchKernelGGL(pre_top_kernel, dim3(1), dim3(256), 0, st, toff, nt, W);
            RB_TRY(hipGetLastError());
            // the partners of this level are positions of its input, whose
            // angles the count pass copied into th
            hipLaunchKernelGGL(enum_pass_kernel, dim3(enum_grid), dim3(256), 0, st, th, P, first,
                               pre, toff, W, angc, part);
            RB_TRY(hipGetLastError());
            std::swap(a, b);
        }
    }
    return launch_cross_finalize(part, (int)std::min<int64_t>(nb, INT32_MAX), ideal, out_count,
                                 nullptr, out_metric, out_dev_sum, st);
}

}  // namespace rb
