// Per-edge and per-node records for the all-pairs sweeps (the join of the
// edge list with the node positions that precedes Algorithms 4 and 5, and
// the position table of Algorithm 1), plus the padding records that make
// every tile full.
#include "rb_internal.h"

namespace rb {
namespace {

__global__ __launch_bounds__(256) void edge_prep_kernel(const float *__restrict__ x,
                                                        const float *__restrict__ y,
                                                        const int32_t *__restrict__ src,
                                                        const int32_t *__restrict__ dst,
                                                        int64_t n_nodes, int64_t n_edges,
                                                        int64_t n_pad,
                                                        const int32_t *__restrict__ order,
                                                        EdgeRec *__restrict__ rec) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n_pad;
         e += (int64_t)gridDim.x * blockDim.x) {
        EdgeRec r;
        // record e holds edge order[e] when an order is given (a permutation
        // of the edge ids), else edge e
        const int64_t k = (order && e < n_edges) ? (int64_t)order[e] : e;
        const bool in = e < n_edges && k >= 0 && k < n_edges;
        const int32_t s = in ? src[k] : -1;
        const int32_t t = in ? dst[k] : -1;
        // ids out of range (a precondition violation) become padding edges
        if (s >= 0 && t >= 0 && s < n_nodes && t < n_nodes) {
            const double px = x[s], py = y[s];
            const double dx = (double)x[t] - px, dy = (double)y[t] - py;
            r.x = px;
            r.y = py;
            r.dx = dx;
            r.dy = dy;
            r.c = fma(dx, py, -(dy * px));             // exact: |.| < 2^43
            // line angle in [0, pi): fold the direction into the upper half plane
            const bool flip = (dy < 0.0) | ((dy == 0.0) & (dx < 0.0));
            r.th = atan2(flip ? -dy : dy, flip ? -dx : dx);
            r.s = s;
            r.t = t;
        } else {
            // padding edge: every orientation against it is +1, so it never crosses
            r.x = 0.0; r.y = 0.0; r.dx = 0.0; r.dy = 0.0; r.c = -1.0; r.th = 0.0;
            r.s = -1; r.t = -1;
        }
        r.tq = quantize_angle(r.th);
        r.pad1 = 0;
        rec[e] = r;
    }
}

__global__ __launch_bounds__(256) void node_prep_kernel(const float *__restrict__ x,
                                                        const float *__restrict__ y,
                                                        int64_t n_nodes, int64_t n_pad, double T,
                                                        NodeRec *__restrict__ rec) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n_pad;
         v += (int64_t)gridDim.x * blockDim.x) {
        NodeRec r;
        if (v < n_nodes) {
            const double px = x[v], py = y[v];
            const double n = fma(px, px, py * py);      // exact: < 2^41
            r.x = px;
            r.y = py;
            r.q = -0.5 * n;
            r.h = 0.5 * (n - T);
        } else {
            // padding node: as a row it meets nothing (h huge), as a column
            // nothing meets it (q hugely negative)
            r.x = 0.0; r.y = 0.0; r.q = -0x1p100; r.h = 0x1p100;
        }
        rec[v] = r;
    }
}

int grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (int)g;
}

}  // namespace

hipError_t launch_edge_prep(const float *x, const float *y, const int32_t *src,
                            const int32_t *dst, int64_t n_nodes, int64_t n_edges, int64_t n_pad,
                            EdgeRec *rec, hipStream_t st) {
    return launch_edge_prep_ordered(x, y, src, dst, n_nodes, n_edges, n_pad, nullptr, rec, st);
}

hipError_t launch_edge_prep_ordered(const float *x, const float *y, const int32_t *src,
                                    const int32_t *dst, int64_t n_nodes, int64_t n_edges,
                                    int64_t n_pad, const int32_t *order, EdgeRec *rec,
                                    hipStream_t st) {
    hipLaunchKernelGGL(edge_prep_kernel, dim3(grid_for(n_pad)), dim3(256), 0, st, x, y, src,
                       dst, n_nodes, n_edges, n_pad, order, rec);
    return hipGetLastError();
}

hipError_t launch_node_prep(const float *x, const float *y, int64_t n_nodes, int64_t n_pad,
                            double T, NodeRec *rec, hipStream_t st) {
    hipLaunchKernelGGL(node_prep_kernel, dim3(grid_for(n_pad)), dim3(256), 0, st, x, y, n_nodes,
                       n_pad, T, rec);
    return hipGetLastError();
}

}  // namespace rb
