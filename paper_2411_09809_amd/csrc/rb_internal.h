// Internal declarations of the HIP implementation behind include/rb.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rb {

// ------------------------------------------------------------------ records
//
// Per-edge record written by the edge-preparation kernel: the first end
// point P = (x, y), the direction D = (dx, dy) = Q - P, the line constant
// c = dx*y - dy*x, the line angle th in [0, pi) and the end ids.  With integer
// coordinates |.| <= 2^20 every field but th is an integer below 2^43 in
// magnitude, hence exact in double, and so is every orientation value the
// sweep derives from them (Algorithm 4's CCW).
struct __align__(16) EdgeRec {
    double x, y;
    double dx, dy;
    double c, th;
    int32_t s, t;
    int32_t pad0, pad1;
};
static_assert(sizeof(EdgeRec) == 64, "edge record is 64 bytes");

// Per-node record for the occlusion sweep.  With n = x^2 + y^2 and T the
// largest integer below d^2, the test |p_u - p_v|^2 <= T is rewritten as
//     x_u x_v + y_u y_v + q_v >= h_u,   q = -n/2,  h = (n - T)/2,
// which is exact in double (all terms are multiples of 1/2 below 2^45).
struct __align__(16) NodeRec {
    double x, y, q, h;
};
static_assert(sizeof(NodeRec) == 32, "node record is 32 bytes");

// Partial results of one block of a sweep.
struct __align__(16) CrossPartial {
    unsigned long long proper, touch;   // proper crossings, other closed crossings
    double dev;                         // sum of |ideal - a| (radians)
    double pad;
};
struct __align__(16) OcclPartial {
    unsigned long long count;
    unsigned long long pad;
};

// ------------------------------------------------------------------ tiling
constexpr int kBlock = 256;          // threads per sweep block (4 waves)
constexpr int kChunk = 256;          // column records staged in LDS per unit
constexpr int kCrossRows = 4;        // edge rows held per thread
constexpr int kOcclRows = 16;        // node rows held per thread
constexpr int kEdgePad = kBlock * 8; // edge records padded to a multiple of this
constexpr int kNodePad = kBlock * 16;
constexpr int kMaxPartials = 8192;   // partial slots per sweep
constexpr int kSmallDeg = 16;        // min-angle: thread-per-node up to this degree
constexpr int kLdsDeg = 2048;        // min-angle: block sort in LDS up to this degree

// Layout of the caller's workspace (byte offsets, 256-aligned).
struct WsLayout {
    size_t edge_rec, node_rec, partial, scalars;
    size_t deg, cursor, offs, angles, dv, big_list, hash;
    size_t total;
    int64_t n_edge_pad, n_node_pad, hash_size;
};
bool ws_layout(int64_t n_nodes, int64_t n_edges, WsLayout *L);

// Small device scalars used between kernels of one call.
struct __align__(16) Scalars {
    double mean;            // edge length mean
    double sum_dv;
    unsigned long long n_used;
    unsigned long long big_count;
    int32_t flags;
    int32_t pad[7];
};

// ------------------------------------------------------------------ launches
// Every launcher enqueues on `st` and returns the launch status.
hipError_t launch_edge_prep(const float *x, const float *y, const int32_t *src,
                            const int32_t *dst, int64_t n_nodes, int64_t n_edges, int64_t n_pad,
                            EdgeRec *rec, hipStream_t st);
hipError_t launch_node_prep(const float *x, const float *y, int64_t n_nodes, int64_t n_pad,
                            double T, NodeRec *rec, hipStream_t st);

struct SweepPlan {
    int64_t n_row_tiles, n_chunks, n_units;
    int grid;
};
SweepPlan plan_cross(int64_t n_edges, bool angle);
SweepPlan plan_occl(int64_t n_nodes);

hipError_t launch_cross_sweep(const EdgeRec *rec, const SweepPlan &p, bool angle,
                              double ideal, CrossPartial *part, hipStream_t st);
hipError_t launch_cross_finalize(const CrossPartial *part, int n_part, double ideal,
                                 unsigned long long *out_count, unsigned long long *out_proper,
                                 double *out_metric, double *out_dev_sum, hipStream_t st);
hipError_t launch_occl_sweep(const NodeRec *rec, const SweepPlan &p, OcclPartial *part,
                             hipStream_t st);
hipError_t launch_occl_finalize(const OcclPartial *part, int n_part,
                                unsigned long long *out_count, hipStream_t st);

hipError_t launch_elv(const float *x, const float *y, const int32_t *src, const int32_t *dst,
                      int64_t n_nodes, int64_t n_edges, double *partial, Scalars *sc, double *out_metric,
                      double *out_mean, hipStream_t st);

hipError_t launch_min_angle(const float *x, const float *y, int64_t n_nodes,
                            const int32_t *src, const int32_t *dst, int64_t n_edges,
                            const WsLayout &L, char *ws, double *out_metric,
                            double *out_sum_dv, unsigned long long *out_n_used, hipStream_t st);

hipError_t launch_validate(const float *x, const float *y, int64_t n_nodes,
                           const int32_t *src, const int32_t *dst, int64_t n_edges,
                           const WsLayout &L, char *ws, hipStream_t st);

int device_cu_count();

}  // namespace rb
