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
// also enumerated, for the angle sum.  Ratios are compared exactly: the two
// cross products are formed as exact sums of two doubles with an FMA.
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
// run, the pieces of its left run after it in right order (reversed pairs),
// and sums their angle terms; block sums accumulate into part[block]
__global__ __launch_bounds__(256) void count_pass_kernel(const Piece *__restrict__ in,
                                                         Piece *__restrict__ out, int64_t P,
                                                         int64_t L, ByStripRight less,
                                                         double ideal,
                                                         CrossPartial *__restrict__ part) {
    __shared__ unsigned long long rc[4];
    __shared__ double rd[4];
    const double angc = ideal - kHalfPi;
    unsigned long long cnt = 0;
    double acc = 0.0;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;   // grid covers P
    if (i < P) {
        const int64_t s = i / (2 * L) * (2 * L);
        const int64_t mid = min(s + L, P), end = min(s + 2 * L, P);
        const Piece v = in[i];
        int64_t pos;
        if (i < mid) {
            pos = s + (i - s) + (lower_bound(in, mid, end, v, less) - mid);
        } else {
            const int64_t ub = upper_bound(in, s, mid, v, less);
            pos = s + (i - mid) + (ub - s);
            // left pieces after v in right order: same strip, right y greater
            cnt = (unsigned long long)(mid - ub);
            for (int64_t j = ub; j < mid; ++j) {
                const double u = fabs(v.th - in[j].th) - kHalfPi;
                acc += fabs(angc + fabs(u));
            }
        }
        out[pos] = v;
    }
    for (int off = 32; off > 0; off >>= 1) {
        cnt += __shfl_xor(cnt, off, 64);
        acc += __shfl_xor(acc, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        rc[threadIdx.x >> 6] = cnt;
        rd[threadIdx.x >> 6] = acc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        CrossPartial Q = part[blockIdx.x];
        for (int k = 0; k < 4; ++k) {
            Q.proper += rc[k];
            Q.dev += rd[k];
        }
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
// pieces | pieces | partials]
constexpr size_t kHead = sizeof(GridParams) + sizeof(unsigned long long);

size_t strip_ws_bytes(int64_t m, int64_t P) {
    const int64_t me = std::max<int64_t>(m, 1), pe = std::max<int64_t>(P, 1);
    return round256(kHead) + round256(sizeof(uint32_t) * me) +
           round256(sizeof(uint32_t) * (me + 1)) +
           round256(sizeof(unsigned long long) * (me / 2048 + 2)) +
           2 * round256(sizeof(Piece) * pe) + round256(sizeof(CrossPartial) * ((pe + 255) / 256));
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
        for (int64_t L = 1; L < P; L *= 2) {
            hipLaunchKernelGGL(count_pass_kernel, dim3((unsigned)nb), dim3(256), 0, st, a, b, P,
                               L, by_right, ideal, part);
            RB_TRY(hipGetLastError());
            std::swap(a, b);
        }
    }
    return launch_cross_finalize(part, (int)std::min<int64_t>(nb, INT32_MAX), ideal, out_count,
                                 nullptr, out_metric, out_dev_sum, st);
}

}  // namespace rb
