// Gradient of a layout-optimisation loss built from two of the metrics:
//     L = w_a (1 - E_ca) + w_l M_l
//       = w_a / (ideal |S|) sum_{(e,f) in S} |ideal - a_ef|  +  w_l M_l,
// with the crossing set S frozen at the current (integer) layout.
//
// Through the line angles th in [0, pi) of the edges (a = pi/2 - ||d| - pi/2|,
// d = th_e - th_f), the derivative of one term is
//     d|ideal - a_ef| / d th_e = - d|ideal - a_ef| / d th_f
//                              = sgn(v) * sgn(dot) * sgn(cross)  in {-1, 0, 1},
// where v = (ideal - pi/2) + ||d| - pi/2| (so sgn(a - ideal) = -sgn(v)),
// cross = d_e x d_f and dot = d_e . d_f.  The branch signs come from the exact
// integer cross and dot products (the folding of directions into [0, pi)
// cancels), so perpendicular (dot = 0) and parallel (cross = 0) pairs give 0,
// the symmetric choice at those kinks.  The backward sweep therefore only
// accumulates integers: k_e = sum_f q_ef per edge (rows in registers,
// columns via wave popcounts and LDS, then integer atomics: exact and
// order-independent).  The k_e depend neither on |S| nor on the loss, so the
// same sweep also accumulates the forward terms of every pair (crossing
// count, sum of |ideal - a|): one pass over the pair triangle gives both.
// A per-edge pass applies the chain rule in double:
//     dL/dD_e = w_a k_e / (ideal |S|) (-dy, dx) / l^2 + w_l dM_l/dl_e (dx, dy) / l,
//     dM_l/dl_e = ((l_e - mu)/(N s mu) - s/(N mu^2)) / sqrt(N - 1)   (s: population
//     spread of the lengths), and scatters +dL/dD_e to the head node and
//     -dL/dD_e to the tail node.
#include <algorithm>

#include "rb_device.h"
#include "rb_internal.h"

namespace rb {
namespace {

constexpr double kHalfPi = 1.5707963267948966192;

// k + [lane in plus] - [lane in minus]: the masks enter as the carry-in and
// borrow-in of one add and one subtract
// (in place, so lanes outside EXEC keep their value)
__device__ __forceinline__ int add_mask_bits(int k, uint64_t plus, uint64_t minus) {
    uint64_t c0, c1;
    __asm__("v_addc_co_u32_e64 %0, %1, 0, %0, %3\n\t"
            "v_subbrev_co_u32_e64 %0, %2, 0, %0, %4"
            : "+v"(k), "=&s"(c0), "=&s"(c1)
            : "s"(plus), "s"(minus));
    return k;
}

template <int K, bool DIAG>
__device__ __forceinline__ void adjoint_chunk(const EdgeRec *__restrict__ col,
                                              const int2 *__restrict__ rid,
                                              int8_t *__restrict__ colk, const double (&rX)[K],
                                              const double (&rY)[K], const double (&rDX)[K],
                                              const double (&rDY)[K], const double (&rC)[K],
                                              const double (&rTH)[K], int (&kr)[K], int tid,
                                              int diag_off, double ideal,
                                              double angc, uint32_t &n_proper,
                                              uint32_t &n_touch, double &acc) {
    const int wave = tid >> 6, lane = tid & 63;
    // the column sums of four consecutive columns, one byte each (little
    // endian, as colk's bytes lie), go to LDS as one 32-bit store
    uint32_t packed = 0;
    // one LDS address per group of four columns, opaque so that the compiler
    // neither rebuilds it per column (one instruction per pair at one row per
    // thread) nor folds it away; the columns load at immediate offsets
    typedef __attribute__((address_space(3))) const EdgeRec lds_rec;
    for (int j0 = 0; j0 < kChunk; j0 += 4) {
    lds_rec *grp = (lds_rec *)(col + j0);
    __asm__ volatile("" : "+v"(grp));
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
        const int j = j0 + jj;
        const double cX = grp[jj].x, cY = grp[jj].y;
        const double cDX = grp[jj].dx, cDY = grp[jj].dy;
        const double cC = grp[jj].c, cTH = grp[jj].th;
        int colsum = 0;
        uint64_t zm[K];
        uint64_t any_zero = 0;
#pragma unroll
        for (int r = 0; r < K; ++r) {
            // rows and columns in sweep form, as in the edge sweep: the signs
            // of o1 (o1 + cr) and o3 (o3 - cr) from max(|t1|, |t3|) against
            // |cr|, with t1 = 2 o1 + cr and t3 = 2 o3 - cr, as lane masks
            const double t1 = fma(rDX[r], cY, fma(-rDY[r], cX, -rC[r]));
            const double t3 = fma(cDX, rY[r], fma(-cDY, rX[r], -cC));
            const double cr = fma(-rDY[r], cDX, rDX[r] * cDY);
            const double t = dev::max_abs(t1, t3);
            uint64_t lt = __builtin_amdgcn_ballot_w64(t < fabs(cr));
            uint64_t le = __builtin_amdgcn_ballot_w64(t <= fabs(cr));
            if (DIAG) {
                // a diagonal unit keeps column index > row index: with the
                // tile's first row as origin, diag_off + j > r * 256 + tid
                const uint64_t tri = __builtin_amdgcn_ballot_w64(diag_off + j > r * kBlock + tid);
                lt &= tri;
                le &= tri;
            }
            zm[r] = le & ~lt;
            const double u = fabs(rTH[r] - cTH) - kHalfPi;
            const double v = angc + fabs(u);
            const double dot = fma(rDX[r], cDX, rDY[r] * cDY);
            const double s = (v * dot) * cr;
            // lane masks of the crossing pairs and of their q = +1 / -1
            const uint64_t cmask = lt;
            const uint64_t pmask = __builtin_amdgcn_ballot_w64(s > 0.0) & cmask;
            const uint64_t nmask = __builtin_amdgcn_ballot_w64(s < 0.0) & cmask;
            colsum += (int)__popcll(pmask) - (int)__popcll(nmask);
            kr[r] = add_mask_bits(kr[r], pmask, nmask);
            // forward terms of the same pair: the count and |ideal - a|
            n_proper += (uint32_t)__popcll(cmask);
            dev::add_abs_masked(acc, v, cmask);
            any_zero |= zm[r];
        }
        if (__builtin_expect(any_zero != 0, 0)) {
            // pairs with an end point on the other edge's line
            double fx = cX, fy = cY, fdx = cDX, fdy = cDY, fc = cC, fth = cTH;
            __asm__ volatile("" : "+v"(fx), "+v"(fy), "+v"(fdx), "+v"(fdy), "+v"(fc), "+v"(fth));
            // back from sweep form to start point and line constant (exact);
            // after the opaque copy, so none of it is hoisted out of the loop
            fx = 0.5 * (fx - fdx);
            fy = 0.5 * (fy - fdy);
            fc = 0.5 * fc;
            const int2 fid = make_int2(col[j].s, col[j].t);
#pragma unroll
            for (int r = 0; r < K; ++r) {
                bool pos = false, neg = false, ok = false;
                // incident pairs (the common case here) are settled by their ids
                if (((zm[r] >> lane) & 1) && !dev::incident_ids(rid[r * kBlock + tid], fid)) {
                    double ex = rX[r], ey = rY[r], edx = rDX[r], edy = rDY[r], ec = rC[r];
                    __asm__ volatile("" : "+v"(ex), "+v"(ey), "+v"(edx), "+v"(edy), "+v"(ec));
                    ex = 0.5 * (ex - edx);
                    ey = 0.5 * (ey - edy);
                    ec = 0.5 * ec;
                    ok = dev::touching_apart(ex, ey, edx, edy, ec, fx, fy, fdx, fdy, fc);
                    if (ok) {
                        const double cr = fma(-edy, fdx, edx * fdy);
                        const double v = angc + fabs(fabs(rTH[r] - fth) - kHalfPi);
                        const double s = (v * fma(edx, fdx, edy * fdy)) * cr;
                        pos = s > 0.0;
                        neg = s < 0.0;
                        // parallel lines or a zero-length edge: a = 0
                        acc += (cr == 0.0) ? ideal : fabs(v);
                    }
                }
                n_touch += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(ok));
                kr[r] += (int)pos - (int)neg;
                colsum += (int)__popcll(__builtin_amdgcn_ballot_w64(pos)) -
                          (int)__popcll(__builtin_amdgcn_ballot_w64(neg));
            }
        }
        packed |= ((uint32_t)colsum & 0xffu) << (8 * (j & 3));     // |colsum| <= 64 K
        if ((j & 3) == 3) {
            if (lane == 0) __builtin_memcpy(&colk[wave * kChunk + j - 3], &packed, 4);
            packed = 0;
        }
    }
    }
}

// LIST: the units come from an explicit list (the pruned plan): tile I meets
// chunks list[tile_off[I] .. tile_off[I+1]); its length is read on the device.
template <int K, int WAVES, bool LIST>
__global__ __launch_bounds__(kBlock, WAVES) void adjoint_sweep_kernel(
    const EdgeRec *__restrict__ rec, SweepLayout lay, int64_t n_units,
    const int32_t *__restrict__ list, const uint32_t *__restrict__ tile_off, int64_t n_tiles,
    double ideal, int *__restrict__ kacc, CrossPartial *__restrict__ part) {
    __shared__ EdgeRec col[kChunk];
    __shared__ int2 rid[kBlock * K];
    // per-wave column sums of q: |sum| <= 64 K fits a byte, which keeps the
    // block's LDS under 20 KB (8 blocks per CU)
    __shared__ __align__(16) int8_t colk[(kBlock / 64) * kChunk];
    __shared__ unsigned long long red_p[kBlock / 64], red_t[kBlock / 64];
    __shared__ double red_d[kBlock / 64];
    // start-up at raised wave priority, dropped while a unit is swept (the
    // waves already sweeping would otherwise take nearly every issue slot)
    __builtin_amdgcn_s_setprio(3);
    const int tid = threadIdx.x;
    const int64_t G = gridDim.x, b = blockIdx.x;
    // with a list, the first min(U, G) blocks take one equal range each, so
    // blocks with work are dispatched before the empty ones
    const int64_t U = LIST ? (int64_t)tile_off[n_tiles] : n_units;
    const int64_t n_items = std::min<int64_t>(U, G);
    const int64_t u_begin = b < n_items ? first_unit(U, n_items, b) : 0;
    const int64_t u_end = b < n_items ? first_unit(U, n_items, b + 1) : 0;
    constexpr int64_t R = (int64_t)kBlock * K;
    const double angc = ideal - kHalfPi;
    if (LIST && u_begin == u_end) {            // more blocks than kept units
        if (tid == 0) {
            CrossPartial P;
            P.proper = 0; P.touch = 0; P.dev = 0.0; P.pad = 0.0;
            part[b] = P;
        }
        return;
    }
    int64_t I;
    if (LIST) {
        int64_t lo = 0, hi = n_tiles - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if ((int64_t)tile_off[mid] <= u_begin) lo = mid;
            else hi = mid - 1;
        }
        I = lo;
    } else {
        I = tile_of_unit(u_begin, lay.n_row_tiles, lay.n_chunks, K);
    }
    int64_t c = LIST ? 0 : I * K + (u_begin - units_before(I, lay.n_chunks, K));
    double rX[K], rY[K], rDX[K], rDY[K], rC[K], rTH[K];
    int kr[K];
    bool rows_loaded = false;
    uint32_t n_p = 0, n_t = 0;
    unsigned long long tot_p = 0, tot_t = 0;
    double acc = 0.0;

    auto flush_rows = [&]() {
#pragma unroll
        for (int r = 0; r < K; ++r) {
            if (kr[r] != 0) atomicAdd(&kacc[I * R + (int64_t)r * kBlock + tid], kr[r]);
        }
    };

    for (int64_t u = u_begin; u < u_end; ++u) {
        if (LIST) {
            while ((int64_t)tile_off[I + 1] <= u) {   // u < tile_off[n_tiles]: stops in range
                if (rows_loaded) flush_rows();
                ++I;
                rows_loaded = false;
            }
            c = list[u];
        }
        __syncthreads();                      // previous chunk, ids and column sums consumed
        if (!rows_loaded) {
#pragma unroll
            for (int r = 0; r < K; ++r) {
                const EdgeRec e = sweep_form(edge_row(rec, I * R + (int64_t)r * kBlock + tid,
                                                      lay.n_chunks * kChunk));
                rX[r] = e.x; rY[r] = e.y; rDX[r] = e.dx; rDY[r] = e.dy;
                rC[r] = e.c; rTH[r] = e.th;
                rid[r * kBlock + tid] = make_int2(e.s, e.t);
                kr[r] = 0;
            }
            rows_loaded = true;
        }
        {
            // the lane's staging address is rebuilt each unit, not held across the sweep
            int lane_rec = tid;
            __asm__ volatile("" : "+v"(lane_rec));
            col[tid] = sweep_form(rec[c * kChunk + lane_rec]);
        }
        __syncthreads();
        __builtin_amdgcn_s_setprio(0);
        const int64_t col0 = c * kChunk;
        const int diag_off = (int)(c - I * K) * kChunk;   // used for c < (I + 1) K only
        if (c < (I + 1) * K)
            adjoint_chunk<K, true>(col, rid, colk, rX, rY, rDX, rDY, rC, rTH, kr, tid, diag_off,
                                   ideal, angc, n_p, n_t, acc);
        else
            adjoint_chunk<K, false>(col, rid, colk, rX, rY, rDX, rDY, rC, rTH, kr, tid, diag_off,
                                    ideal, angc, n_p, n_t, acc);
        __builtin_amdgcn_s_setprio(3);
        tot_p += n_p;
        tot_t += n_t;
        n_p = 0;
        n_t = 0;
        __syncthreads();
        {   // the column edge f of a pair receives -q
            int sum = 0;
            for (int w = 0; w < kBlock / 64; ++w) sum += colk[w * kChunk + tid];
            if (sum != 0) atomicSub(&kacc[col0 + tid], sum);
        }
        if (!LIST && ++c == lay.n_chunks) {
            flush_rows();
            ++I;
            c = I * K;
            rows_loaded = false;
        }
    }
    if (rows_loaded) flush_rows();
    // forward partial of this block: crossing counts and the deviation sum
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    const int wave = tid >> 6, lane = tid & 63;
    __syncthreads();
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

// Chain rule per edge, scattered to the end nodes; thread 0 also writes the loss.
__global__ __launch_bounds__(256) void edge_grad_kernel(
    const EdgeRec *__restrict__ rec, const int *__restrict__ kacc, int64_t n_rec,
    int64_t n_edges, const Scalars *__restrict__ sc, double ideal, double w_a, double w_l,
    double *gx, double *gy, double *out_loss) {
    const unsigned long long S = sc->count;
    const double mu = sc->mean, ml = sc->ml, N = (double)n_edges;
    // population spread of the lengths, from M_l = s / mu / sqrt(N - 1)
    const double spread = (n_edges >= 2) ? ml * mu * sqrt(N - 1.0) : 0.0;
    const double ka = S ? w_a / (ideal * (double)S) : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0 && out_loss)
        *out_loss = (S ? w_a * (1.0 - sc->eca) : 0.0) + w_l * ml;
    // one record per edge (in whatever order the sweep used); padding records
    // and edges with bad ids carry s = t = -1
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n_rec;
         p += (int64_t)gridDim.x * blockDim.x) {
        const EdgeRec r = rec[p];
        if (r.s < 0) continue;
        const double l2 = fma(r.dx, r.dx, r.dy * r.dy);
        if (l2 == 0.0) continue;                        // zero-length edge: no direction
        const double l = sqrt(l2);
        const double gth = ka * (double)kacc[p] / l2;
        double gdx = -gth * r.dy, gdy = gth * r.dx;
        if (spread > 0.0 && mu > 0.0) {
            const double dml = w_l * ((l - mu) / (N * spread * mu) - spread / (N * mu * mu)) /
                               sqrt(N - 1.0);
            gdx = fma(dml, r.dx / l, gdx);
            gdy = fma(dml, r.dy / l, gdy);
        }
        atomicAdd(&gx[r.t], gdx);
        atomicAdd(&gy[r.t], gdy);
        atomicAdd(&gx[r.s], -gdx);
        atomicAdd(&gy[r.s], -gdy);
    }
}

__global__ void fill_f64_kernel(double *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// copy the forward results into the scalar block used by the gradient pass
__global__ void stash_kernel(Scalars *sc, const unsigned long long *count, const double *eca,
                             const double *ml, unsigned long long *out_count) {
    if (threadIdx.x == 0) {
        sc->count = *count;
        sc->eca = *eca;
        sc->ml = *ml;
        if (out_count) *out_count = *count;
    }
}

int grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (int)g;
}

constexpr int kAdjRows = 1, kAdjWaves = 8;
static_assert(64 * kAdjRows <= 127, "per-wave column sums are stored as int8_t");
int g_adj_list_grid = 0;

#define RB_TRY(expr)                          \
    do {                                      \
        hipError_t _e = (expr);               \
        if (_e != hipSuccess) return _e;      \
    } while (0)

}  // namespace

hipError_t launch_loss_grad(const float *x, const float *y, int64_t n_nodes, const int32_t *src,
                            const int32_t *dst, int64_t n_edges, double ideal, double w_a,
                            double w_l, double w_m, double *out_loss, double *gx, double *gy,
                            unsigned long long *out_count, const WsLayout &L, char *w,
                            hipStream_t st) {
    EdgeRec *rec = (EdgeRec *)(w + L.edge_rec);
    Scalars *sc = (Scalars *)(w + L.scalars);
    int *kacc = (int *)(w + L.kacc);
    Fwd *fw = (Fwd *)(w + L.fwd);
    unsigned long long *fw_count = &fw->count;
    double *fw_eca = &fw->eca;
    double *fw_ml = &fw->ml;
    const MinAngleBufs mab = min_angle_bufs(L, w);
    // M_a first: its pass starts by clearing the scalar block
    if (w_m != 0.0)
        RB_TRY(launch_min_angle(x, y, n_nodes, src, dst, n_edges, mab, &fw->ma, &fw->sum_dv,
                                &fw->n_used, st));
    // one sweep gives the forward terms (crossing count, deviation sum) and
    // the integer adjoint counts per edge; M_l and the mean length come from
    // the edge-length pass
    RB_TRY(launch_edge_prep(x, y, src, dst, n_nodes, n_edges, L.n_edge_pad, rec, st));
    RB_TRY(launch_zero_scalars(sc, st));
    RB_TRY(launch_elv(x, y, src, dst, n_nodes, n_edges, (double *)(w + L.partial), sc, fw_ml,
                      nullptr, st));
    RB_TRY(launch_fill_u32((uint32_t *)kacc, L.n_edge_pad, 0u, st));
    const SweepLayout lay = sweep_layout(n_edges, kAdjRows, 0, 0);
    const int64_t U = sweep_units(n_edges, kAdjRows);
    const int grid = (int)std::min<int64_t>(U, kMaxPartials);
    CrossPartial *part = (CrossPartial *)(w + L.partial);
    TimedEvents te = timed_begin(4, st);
    hipLaunchKernelGGL((adjoint_sweep_kernel<kAdjRows, kAdjWaves, false>), dim3(grid),
                       dim3(kBlock), 0, st, rec, lay, U, nullptr, nullptr, (int64_t)0, ideal, kacc,
                       part);
    timed_end(te);
    RB_TRY(hipGetLastError());
    RB_TRY(launch_cross_finalize(part, grid, ideal, fw_count, nullptr, fw_eca, nullptr, st));
    hipLaunchKernelGGL(stash_kernel, dim3(1), dim3(64), 0, st, sc, fw_count, fw_eca, fw_ml,
                       out_count);
    RB_TRY(hipGetLastError());
    // chain rule and scatter
    const int64_t V = n_nodes > 0 ? n_nodes : 1;
    hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_for(V)), dim3(256), 0, st, gx, n_nodes);
    RB_TRY(hipGetLastError());
    hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_for(V)), dim3(256), 0, st, gy, n_nodes);
    RB_TRY(hipGetLastError());
    hipLaunchKernelGGL(edge_grad_kernel, dim3(grid_for(n_edges)), dim3(256), 0, st, rec, kacc,
                       n_edges, n_edges, sc, ideal, w_a, w_l, gx, gy, out_loss);
    RB_TRY(hipGetLastError());
    if (w_m == 0.0) return hipSuccess;
    return launch_min_angle_grad(x, y, n_nodes, src, dst, n_edges, mab, w_m, &fw->ma, &fw->n_used,
                                 &fw->big_count, out_loss, gx, gy, st);
}

hipError_t launch_loss_grad_pruned(const float *x, const float *y, int64_t n_nodes,
                                   const int32_t *src, const int32_t *dst, int64_t n_edges,
                                   double ideal, double w_a, double w_l, double w_m,
                                   double *out_loss, double *gx, double *gy,
                                   unsigned long long *out_count, const GridWs &G, char *w,
                                   hipStream_t st) {
    Fwd *fw = (Fwd *)(w + G.fwd);
    const MinAngleBufs mab = min_angle_bufs(G, w);
    if (w_m != 0.0)
        RB_TRY(launch_min_angle(x, y, n_nodes, src, dst, n_edges, mab, &fw->ma, &fw->sum_dv,
                                &fw->n_used, st));
    // the pruned plan (records in Hilbert order, unit list of 2-row tiles),
    // then the same fused sweep over the kept units only
    RB_TRY(launch_prune_plan(x, y, n_nodes, src, dst, n_edges, kAdjRows, G, w, st));
    const EdgeRec *rec = (const EdgeRec *)(w + G.rec);
    Scalars *sc = (Scalars *)(w + G.scalars);
    int *kacc = (int *)(w + G.kacc);
    unsigned long long *fw_count = &fw->count;
    double *fw_eca = &fw->eca;
    double *fw_ml = &fw->ml;
    RB_TRY(launch_zero_scalars(sc, st));
    RB_TRY(launch_elv(x, y, src, dst, n_nodes, n_edges, (double *)(w + G.partial), sc, fw_ml,
                      nullptr, st));
    RB_TRY(launch_fill_u32((uint32_t *)kacc, G.n_edge_pad, 0u, st));
    if (g_adj_list_grid == 0) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, adjoint_sweep_kernel<kAdjRows, kAdjWaves, true>, kBlock, 0) !=
                hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        g_adj_list_grid = std::min(per_cu * device_cu_count() * kListBlocksPerSlot, kMaxPartials);
    }
    const int grid = g_adj_list_grid;
    const SweepLayout lay = sweep_layout(n_edges, kAdjRows, 0, 0);
    CrossPartial *part = (CrossPartial *)(w + G.partial);
    hipLaunchKernelGGL((adjoint_sweep_kernel<kAdjRows, kAdjWaves, true>), dim3(grid),
                       dim3(kBlock), 0, st, rec, lay, (int64_t)0, (const int32_t *)(w + G.list),
                       (const uint32_t *)(w + G.tile_off), lay.n_row_tiles, ideal, kacc, part);
    RB_TRY(hipGetLastError());
    RB_TRY(launch_cross_finalize(part, grid, ideal, fw_count, nullptr, fw_eca, nullptr, st));
    hipLaunchKernelGGL(stash_kernel, dim3(1), dim3(64), 0, st, sc, fw_count, fw_eca, fw_ml,
                       out_count);
    RB_TRY(hipGetLastError());
    const int64_t V = n_nodes > 0 ? n_nodes : 1;
    hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_for(V)), dim3(256), 0, st, gx, n_nodes);
    RB_TRY(hipGetLastError());
    hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_for(V)), dim3(256), 0, st, gy, n_nodes);
    RB_TRY(hipGetLastError());
    hipLaunchKernelGGL(edge_grad_kernel, dim3(grid_for(G.n_edge_pad)), dim3(256), 0, st, rec,
                       kacc, G.n_edge_pad, n_edges, sc, ideal, w_a, w_l, gx, gy, out_loss);
    RB_TRY(hipGetLastError());
    if (w_m == 0.0) return hipSuccess;
    return launch_min_angle_grad(x, y, n_nodes, src, dst, n_edges, mab, w_m, &fw->ma, &fw->n_used,
                                 &fw->big_count, out_loss, gx, gy, st);
}

}  // namespace rb
