// Attainable FP64 FMA issue rate of the device: the ceiling the all-pairs
// sweeps are measured against, taken live by the benchmark.  Every thread
// runs 8 independent FMA chains; with 16 VGPRs a SIMD holds its full wave
// complement, so the rate is set by VALU issue and the clock the chip holds
// under this load.
#include "rb_internal.h"

namespace rb {
namespace {

constexpr int kProbeChains = 8;
constexpr int kProbeBlocksPerCU = 32;

__global__ __launch_bounds__(256) void valu_probe_kernel(double a, double b, int iters,
                                                         double *__restrict__ sink) {
    double x[kProbeChains];
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) x[k] = 1e-3 * threadIdx.x + k;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kProbeChains; ++k) x[k] = fma(x[k], a, b);
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) s += x[k];
    if (s == -1.0) sink[0] = s;           // never true; keeps the chains alive
}

}  // namespace

hipError_t launch_valu_probe(int iters, double *sink, double *out_lane_ops, hipStream_t st) {
    const int grid = device_cu_count() * kProbeBlocksPerCU;
    if (out_lane_ops) *out_lane_ops = (double)grid * 256.0 * iters * kProbeChains;
    hipLaunchKernelGGL(valu_probe_kernel, dim3(grid), dim3(256), 0, st, 0.9999999, 1e-7, iters,
                       sink);
    return hipGetLastError();
}

}  // namespace rb
