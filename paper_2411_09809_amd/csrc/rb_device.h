// Device helpers shared by the per-layout and batched kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rb {
namespace dev {

constexpr double kTwoPi = 6.283185307179586476925;

// ids out of range violate the preconditions; such edges are skipped so that
// no kernel reads or writes outside its buffers
__device__ __forceinline__ bool valid_ids(int32_t s, int32_t t, int64_t n_nodes) {
    return s >= 0 && t >= 0 && s < n_nodes && t < n_nodes;
}

// Euclidean length of the edge s-t: dx^2 + dy^2 < 2^44 is exact in double
__device__ __forceinline__ double edge_length(const float *x, const float *y, int64_t s,
                                              int64_t t) {
    const double dx = (double)x[t] - (double)x[s];
    const double dy = (double)y[t] - (double)y[s];
    return sqrt(fma(dx, dx, dy * dy));
}

// angle of the direction (dx, dy) with the x axis, in [0, 2 pi)
__device__ __forceinline__ double direction_angle(double dx, double dy) {
    const double a = atan2(dy, dx);
    return a < 0.0 ? a + kTwoPi : a;
}

// d_v = (2 pi/deg - phi_min) / (2 pi/deg)
__device__ __forceinline__ double dv_of(double phi_min, uint32_t deg) {
    const double ideal = kTwoPi / (double)deg;
    return (ideal - phi_min) / ideal;
}

// Rarest case of the crossing test: both orientation products are zero and
// the edges share no end id (collinear pieces, or an end point of each edge
// on the other's line): closed segments then cross iff their bounding boxes
// meet.  Kept out of line: it runs for a handful of pairs per layout.
__device__ __noinline__ inline bool boxes_meet(double rx, double ry, double rdx, double rdy,
                                               double fx, double fy, double fdx, double fdy) {
    const double ax0 = fmin(rx, rx + rdx), ax1 = fmax(rx, rx + rdx);
    const double ay0 = fmin(ry, ry + rdy), ay1 = fmax(ry, ry + rdy);
    const double bx0 = fmin(fx, fx + fdx), bx1 = fmax(fx, fx + fdx);
    const double by0 = fmin(fy, fy + fdy), by1 = fmax(fy, fy + fdy);
    return (fmax(ax0, bx0) <= fmin(ax1, bx1)) && (fmax(ay0, by0) <= fmin(ay1, by1));
}

// acc += |v| in the lanes of `mask` only.  A compare's lane mask selects the
// lanes through EXEC, which takes two scalar instructions instead of a vector
// select of an indicator; EXEC is restored within the block.
__device__ __forceinline__ void add_abs_masked(double &acc, double v, uint64_t mask) {
    uint64_t saved;
    __asm__("s_and_saveexec_b64 %1, %2\n\t"
            "v_add_f64 %0, %0, |%3|\n\t"
            "s_mov_b64 exec, %1"
            : "+v"(acc), "=&s"(saved)
            : "s"(mask), "v"(v)
            : "scc");
}

// max(|a|, |b|) as one instruction (absolute-value operands; the compiler's
// fmax would also quiet NaN inputs, and no NaN reaches the sweeps)
__device__ __forceinline__ double max_abs(double a, double b) {
    double r;
    __asm__("v_max_f64 %0, |%1|, |%2|" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Pairs whose larger orientation product is zero.  Edges that share an end
// id are never crossings (incident edges always have both products zero).
__device__ __forceinline__ bool incident_ids(int2 a, int2 b) {
    return (a.x == b.x) | (a.x == b.y) | (a.y == b.x) | (a.y == b.y);
}

// Decision for a pair of edges that share no end id (row edge P + t D,
// column edge F + s G, with line constants c = D x P) whose larger
// orientation product is zero: a negative product means the segments meet
// at an end point of one of them, and two zero products need the box test.
// Callers pass register copies the compiler cannot see through, which keeps
// this arithmetic out of their common path.
__device__ __forceinline__ bool touching_apart(double rx, double ry, double rdx, double rdy,
                                               double rc, double fx, double fy, double fdx,
                                               double fdy, double fc) {
    const double o1 = fma(-rdy, fx, fma(rdx, fy, -rc));
    const double o3 = fma(-fdy, rx, fma(fdx, ry, -fc));
    const double cr = fma(-rdy, fdx, rdx * fdy);
    const double p12 = o1 * (o1 + cr), p34 = o3 * (o3 - cr);
    bool ok = fmin(p12, p34) < 0.0;
    if (p12 == 0.0 && p34 == 0.0) ok = boxes_meet(rx, ry, rdx, rdy, fx, fy, fdx, fdy);
    return ok;
}

__device__ __forceinline__ bool touching_pair(double rx, double ry, double rdx, double rdy,
                                              double rc, int2 rid, double fx, double fy,
                                              double fdx, double fdy, double fc, int2 fid) {
    return !incident_ids(rid, fid) && touching_apart(rx, ry, rdx, rdy, rc, fx, fy, fdx, fdy, fc);
}

// sum over the block (blockDim.x a power of two <= 1024); sh has blockDim.x slots
__device__ __forceinline__ double block_sum(double v, double *sh) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
        if (tid < s) sh[tid] += sh[tid + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// index of the layout owning item i, given offsets off[0..n] (off[0] = 0,
// nondecreasing, off[n] > i): the largest L with off[L] <= i and
// off[L + 1] > i
__device__ __forceinline__ int64_t owner(const int64_t *off, int64_t n, int64_t i) {
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    while (lo + 1 < n && off[lo + 1] <= i) ++lo;     // skip empty layouts
    return lo;
}

}  // namespace dev
}  // namespace rb
