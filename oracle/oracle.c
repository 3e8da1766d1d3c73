/*
 * CPU oracle for the five readability metrics of "Scalable Readability
 * Evaluation for Graph Layouts" (arXiv 2411.09809).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  The product library
 * never links, loads or calls it, and the two share no source.
 *
 * Everything here is the plain definition, written out as nested loops:
 *   - integer predicates in int64 (coordinates are integers with |c| <= 2^20,
 *     so every difference is below 2^21 and every 2x2 determinant below 2^43);
 *   - floating-point metrics in double, with compensated (Neumaier) sums;
 *   - OpenMP only splits the outer loop into independent rows; per-row
 *     results are combined afterwards in row order, so results do not depend
 *     on the thread count.
 *
 * Readings taken where the paper is silent or ambiguous (each one is listed
 * with its reason in the design notes):
 *   R1 occlusion compares the squared distance with the squared diameter
 *      d = 2r, strictly (Algorithm 1), each unordered pair once;
 *   R2 edge pairs that share an endpoint id are not crossings;
 *   R3 closed segments: the paper's two CCW products <= 0, and when both
 *      products are zero the bounding boxes must also meet (collinear pieces
 *      that do not touch are not crossings);
 *   R5 the crossing angle is the acute angle between the two lines,
 *      atan2(|cross|, |dot|), in [0, pi/2];
 *   R6 the deviation is |ideal - a| / ideal (Algorithm 5's absolute value);
 *   R7 with no crossing the crossing-angle metric is 1;
 *   R9 the minimum-angle metric averages d_v over vertices of degree >= 1;
 *   R10 the angle at v is that of the direction v -> u, in [0, 2 pi);
 *   R11 N_e = |E|; with |E| < 2 or zero mean length the variation is 0.
 *
 * Status codes: 0 ok, 1 bad argument, 2 coordinate not an integer in range,
 * 3 edge end out of range.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define COORD_LIMIT 1048576.0 /* 2^20 */

/* ------------------------------------------------------------ helpers */

typedef struct { double s, c; } nsum;   /* Neumaier compensated sum */

static void nsum_add(nsum *a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}
static double nsum_get(const nsum *a) { return a->s + a->c; }

static int to_int_coords(const double *x, const double *y, int64_t n,
                         int64_t **ix, int64_t **iy) {
    *ix = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    *iy = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        double a = x[i], b = y[i];
        if (!(a == floor(a)) || !(b == floor(b)) || fabs(a) > COORD_LIMIT ||
            fabs(b) > COORD_LIMIT) {
            free(*ix); free(*iy);
            return 2;
        }
        (*ix)[i] = (int64_t)a;
        (*iy)[i] = (int64_t)b;
    }
    return 0;
}

static int check_edges(const int32_t *src, const int32_t *dst, int64_t m, int64_t n) {
    for (int64_t e = 0; e < m; ++e)
        if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return 3;
    return 0;
}

/* ------------------------------------------- Algorithm 1: node occlusion */

/* Exact test  dist2 < d*d  for an integer dist2 >= 0 and a double d >= 0.
 * d = M * 2^k with M a 53-bit integer, so d^2 = M^2 * 2^(2k) is compared
 * with dist2 in 128-bit integer arithmetic. */
static int less_than_square(int64_t dist2, double d) {
    if (d <= 0.0) return 0;
    int e;
    double f = frexp(d, &e);                      /* d = f 2^e, f in [0.5,1) */
    unsigned __int128 M = (unsigned __int128)(uint64_t)ldexp(f, 53);
    int k2 = 2 * (e - 53);                        /* d^2 = M^2 2^k2 */
    unsigned __int128 M2 = M * M;                 /* < 2^106 */
    unsigned __int128 D = (unsigned __int128)(uint64_t)dist2;
    if (k2 >= 0) return 1;        /* d >= 2^52: d^2 exceeds every squared distance */
    int s = -k2;
    if (s >= 127) return D == 0 && M2 != 0;
    unsigned __int128 q = M2 >> s;
    unsigned __int128 r = M2 - (q << s);
    return D < q || (D == q && r != 0);
}

int oracle_node_occlusion(const double *x, const double *y, int64_t n,
                          double diameter, uint64_t *out_count) {
    if (n < 0 || !out_count || !(diameter >= 0.0) || isinf(diameter)) return 1;
    int64_t *ix, *iy;
    int st = to_int_coords(x, y, n, &ix, &iy);
    if (st) return st;
    uint64_t total = 0;
    #pragma omp parallel for schedule(dynamic, 64) reduction(+:total)
    for (int64_t v = 0; v < n; ++v) {
        for (int64_t u = v + 1; u < n; ++u) {             /* v < u */
            int64_t dx = ix[v] - ix[u], dy = iy[v] - iy[u];
            if (less_than_square(dx * dx + dy * dy, diameter)) total += 1;
        }
    }
    free(ix); free(iy);
    *out_count = total;
    return 0;
}

/* --------------------------------------------- Algorithm 4: edge crossing */

/* CCW(A,B,C): sign of the cross product CA x AB (the procedure of
 * Algorithm 4). */
static int ccw(int64_t ax, int64_t ay, int64_t bx, int64_t by, int64_t cx, int64_t cy) {
    int64_t cax = ax - cx, cay = ay - cy;
    int64_t abx = bx - ax, aby = by - ay;
    int64_t c = cax * aby - cay * abx;
    return (c > 0) - (c < 0);
}

static int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }
static int64_t max64(int64_t a, int64_t b) { return a > b ? a : b; }

/* Algorithm 4 first joins every edge with the positions of its two end
 * nodes (the table the paper calls D_epos); the pair tests below read that
 * table.  Coordinates are integers with |c| <= 2^20, so they fit in int32. */
typedef struct { int32_t v, u; int32_t x1, y1, x2, y2; } epos_t;

static epos_t *join_positions(const int64_t *ix, const int64_t *iy, const int32_t *src,
                              const int32_t *dst, int64_t m) {
    epos_t *E = (epos_t *)malloc(sizeof(epos_t) * (size_t)(m > 0 ? m : 1));
    for (int64_t e = 0; e < m; ++e) {
        E[e].v = src[e];
        E[e].u = dst[e];
        E[e].x1 = (int32_t)ix[src[e]];
        E[e].y1 = (int32_t)iy[src[e]];
        E[e].x2 = (int32_t)ix[dst[e]];
        E[e].y2 = (int32_t)iy[dst[e]];
    }
    return E;
}

/* Crossing test of two edges a = (v1,u1) and b = (v2,u2).
 * Returns 0 (no crossing), 1 (crossing, segments touch or overlap),
 * 2 (proper crossing: each segment strictly separates the other's ends). */
static int edge_pair_crossing(const epos_t *a, const epos_t *b) {
    /* R2: pairs sharing an endpoint id are incident, not crossing */
    if (a->v == b->v || a->v == b->u || a->u == b->v || a->u == b->u) return 0;
    int c1 = ccw(a->x1, a->y1, a->x2, a->y2, b->x1, b->y1);
    int c2 = ccw(a->x1, a->y1, a->x2, a->y2, b->x2, b->y2);
    int c3 = ccw(b->x1, b->y1, b->x2, b->y2, a->x1, a->y1);
    int c4 = ccw(b->x1, b->y1, b->x2, b->y2, a->x2, a->y2);
    int p12 = c1 * c2, p34 = c3 * c4;
    if (p12 > 0 || p34 > 0) return 0;              /* Algorithm 4's <= 0 test */
    if (p12 < 0 && p34 < 0) return 2;
    if (p12 == 0 && p34 == 0) {                    /* R3: boxes must meet */
        int64_t ax0 = min64(a->x1, a->x2), ax1 = max64(a->x1, a->x2);
        int64_t ay0 = min64(a->y1, a->y2), ay1 = max64(a->y1, a->y2);
        int64_t bx0 = min64(b->x1, b->x2), bx1 = max64(b->x1, b->x2);
        int64_t by0 = min64(b->y1, b->y2), by1 = max64(b->y1, b->y2);
        if (max64(ax0, bx0) > min64(ax1, bx1)) return 0;
        if (max64(ay0, by0) > min64(ay1, by1)) return 0;
    }
    return 1;
}

int oracle_edge_crossing(const double *x, const double *y, int64_t n,
                         const int32_t *src, const int32_t *dst, int64_t m,
                         uint64_t *out_count, uint64_t *out_proper) {
    if (n < 0 || m < 0 || !out_count) return 1;
    if (check_edges(src, dst, m, n)) return 3;
    int64_t *ix, *iy;
    int st = to_int_coords(x, y, n, &ix, &iy);
    if (st) return st;
    epos_t *E = join_positions(ix, iy, src, dst, m);
    uint64_t closed = 0, proper = 0;
    #pragma omp parallel for schedule(dynamic, 16) reduction(+:closed, proper)
    for (int64_t e = 0; e < m; ++e) {
        for (int64_t f = e + 1; f < m; ++f) {          /* each unordered pair once */
            int r = edge_pair_crossing(&E[e], &E[f]);
            closed += (r != 0);
            proper += (r == 2);
        }
    }
    free(E); free(ix); free(iy);
    *out_count = closed;
    if (out_proper) *out_proper = proper;
    return 0;
}

/* ------------------------------------ Algorithm 5: edge crossing angle */

/* Acute angle between the lines of two edges, from exact integer cross and
 * dot products of their direction vectors (R5). */
static double crossing_angle(const epos_t *a, const epos_t *b) {
    int64_t ax = (int64_t)a->x2 - a->x1, ay = (int64_t)a->y2 - a->y1;
    int64_t bx = (int64_t)b->x2 - b->x1, by = (int64_t)b->y2 - b->y1;
    int64_t cr = ax * by - ay * bx;
    int64_t dt = ax * bx + ay * by;
    return atan2(fabs((double)cr), fabs((double)dt));
}

int oracle_crossing_angle(const double *x, const double *y, int64_t n,
                          const int32_t *src, const int32_t *dst, int64_t m,
                          double ideal_angle, double *out_metric,
                          uint64_t *out_count, double *out_dev_sum) {
    if (n < 0 || m < 0 || !out_metric || !(ideal_angle > 0.0)) return 1;
    if (check_edges(src, dst, m, n)) return 3;
    int64_t *ix, *iy;
    int st = to_int_coords(x, y, n, &ix, &iy);
    if (st) return st;
    epos_t *E = join_positions(ix, iy, src, dst, m);
    double *row_sum = (double *)calloc((size_t)(m > 0 ? m : 1), sizeof(double));
    uint64_t count = 0;
    #pragma omp parallel for schedule(dynamic, 16) reduction(+:count)
    for (int64_t e = 0; e < m; ++e) {
        nsum acc = {0.0, 0.0};
        for (int64_t f = e + 1; f < m; ++f) {
            if (!edge_pair_crossing(&E[e], &E[f])) continue;
            double a = crossing_angle(&E[e], &E[f]);
            nsum_add(&acc, fabs(ideal_angle - a) / ideal_angle);      /* R6 */
            count += 1;
        }
        row_sum[e] = nsum_get(&acc);
    }
    nsum tot = {0.0, 0.0};
    for (int64_t e = 0; e < m; ++e) nsum_add(&tot, row_sum[e]);
    double s = nsum_get(&tot);
    free(row_sum); free(E); free(ix); free(iy);
    *out_metric = count ? 1.0 - s / (double)count : 1.0;               /* R7 */
    if (out_count) *out_count = count;
    if (out_dev_sum) *out_dev_sum = s;
    return 0;
}

/* Per-edge view of Algorithms 4 and 5: for each listed edge e, the number of
 * edges crossing it and the sum of |ideal - a| over those crossings (without
 * the division by the ideal angle).  O(|E|) per listed edge. */
int oracle_crossings_of_edges(const double *x, const double *y, int64_t n,
                              const int32_t *src, const int32_t *dst, int64_t m,
                              double ideal_angle, const int64_t *which, int64_t k,
                              uint64_t *out_count, double *out_dev) {
    if (n < 0 || m < 0 || k < 0 || !which || !out_count) return 1;
    if (check_edges(src, dst, m, n)) return 3;
    for (int64_t i = 0; i < k; ++i)
        if (which[i] < 0 || which[i] >= m) return 1;
    int64_t *ix, *iy;
    int st = to_int_coords(x, y, n, &ix, &iy);
    if (st) return st;
    epos_t *E = join_positions(ix, iy, src, dst, m);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < k; ++i) {
        int64_t e = which[i];
        uint64_t c = 0;
        nsum acc = {0.0, 0.0};
        for (int64_t f = 0; f < m; ++f) {
            if (f == e) continue;
            if (!edge_pair_crossing(&E[e], &E[f])) continue;
            c += 1;
            nsum_add(&acc, fabs(ideal_angle - crossing_angle(&E[e], &E[f])));
        }
        out_count[i] = c;
        if (out_dev) out_dev[i] = nsum_get(&acc);
    }
    free(E); free(ix); free(iy);
    return 0;
}

/* ------------------------------------------ Algorithm 2: minimum angle */

static int cmp_double(const void *a, const void *b) {
    double p = *(const double *)a, q = *(const double *)b;
    return (p > q) - (p < q);
}

/* GetMinAngle: sort, then the smallest gap between neighbours, the wrap-around
 * gap 2 pi - a_n + a_1 included. */
static double get_min_angle(double *a, int64_t k) {
    const double two_pi = 2.0 * M_PI;
    qsort(a, (size_t)k, sizeof(double), cmp_double);
    double best = two_pi - a[k - 1] + a[0];
    for (int64_t i = 1; i < k; ++i) {
        double g = a[i] - a[i - 1];
        if (g < best) best = g;
    }
    return best;
}

int oracle_min_angle(const double *x, const double *y, int64_t n,
                     const int32_t *src, const int32_t *dst, int64_t m,
                     double *out_metric, double *out_sum_dv, uint64_t *out_n_used) {
    if (n < 0 || m < 0 || !out_metric) return 1;
    if (check_edges(src, dst, m, n)) return 3;
    int64_t *ix, *iy;
    int st = to_int_coords(x, y, n, &ix, &iy);
    if (st) return st;
    /* the incident edges of every vertex (what aggregateMessages collects) */
    int64_t *deg = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t e = 0; e < m; ++e) { deg[src[e]]++; deg[dst[e]]++; }
    int64_t *start = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t v = 0; v < n; ++v) start[v + 1] = start[v] + deg[v];
    int64_t *fill = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    for (int64_t e = 0; e < m; ++e) {
        int32_t a = src[e], b = dst[e];
        nbr[start[a] + fill[a]++] = b;
        nbr[start[b] + fill[b]++] = a;
    }
    double *dv = (double *)calloc((size_t)n + 1, sizeof(double));
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t v = 0; v < n; ++v) {
        int64_t k = deg[v];
        if (k == 0) continue;
        double *ang = (double *)malloc(sizeof(double) * (size_t)k);
        for (int64_t i = 0; i < k; ++i) {
            int32_t u = nbr[start[v] + i];
            double a = atan2((double)(iy[u] - iy[v]), (double)(ix[u] - ix[v]));
            if (a < 0.0) a += 2.0 * M_PI;                             /* R10 */
            ang[i] = a;
        }
        double ideal = 2.0 * M_PI / (double)k;                        /* phi(v) */
        dv[v] = (ideal - get_min_angle(ang, k)) / ideal;
        free(ang);
    }
    nsum tot = {0.0, 0.0};
    uint64_t used = 0;
    for (int64_t v = 0; v < n; ++v)
        if (deg[v] > 0) { nsum_add(&tot, dv[v]); used++; }
    double s = nsum_get(&tot);
    *out_metric = used ? 1.0 - s / (double)used : 1.0;                /* R9 */
    if (out_sum_dv) *out_sum_dv = s;
    if (out_n_used) *out_n_used = used;
    free(deg); free(start); free(fill); free(nbr); free(dv); free(ix); free(iy);
    return 0;
}

/* ----------------------------------- Algorithm 3: edge length variation */

int oracle_edge_length_variation(const double *x, const double *y, int64_t n,
                                 const int32_t *src, const int32_t *dst, int64_t m,
                                 double *out_metric, double *out_mean) {
    if (n < 0 || m < 0 || !out_metric) return 1;
    if (check_edges(src, dst, m, n)) return 3;
    int64_t *ix, *iy;
    int st = to_int_coords(x, y, n, &ix, &iy);
    if (st) return st;
    double *len = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    nsum s1 = {0.0, 0.0};
    for (int64_t e = 0; e < m; ++e) {
        int64_t dx = ix[dst[e]] - ix[src[e]], dy = iy[dst[e]] - iy[src[e]];
        len[e] = sqrt((double)(dx * dx + dy * dy));
        nsum_add(&s1, len[e]);
    }
    double Ne = (double)m;                                            /* R11 */
    double mu = m ? nsum_get(&s1) / Ne : 0.0;
    nsum s2 = {0.0, 0.0};
    for (int64_t e = 0; e < m; ++e) {
        double d = len[e] - mu;
        nsum_add(&s2, d * d);
    }
    double metric = 0.0;
    if (m >= 2 && mu > 0.0) {
        double la = sqrt(nsum_get(&s2) / (Ne * mu * mu));
        metric = la / sqrt(Ne - 1.0);
    }
    *out_metric = metric;
    if (out_mean) *out_mean = mu;
    free(len); free(ix); free(iy);
    return 0;
}

/* ------------------------------------------------ pairwise test helpers */

/* The crossing and angle tests of one pair of segments with four distinct
 * endpoints (used by the tests to pin the predicate on exhaustive lattices). */
int oracle_segment_pair(const double *p, double ideal_angle, int *out_kind,
                        double *out_angle) {
    double x[4] = {p[0], p[2], p[4], p[6]};
    double y[4] = {p[1], p[3], p[5], p[7]};
    int64_t *ix, *iy;
    int st = to_int_coords(x, y, 4, &ix, &iy);
    if (st) return st;
    const int32_t src[2] = {0, 2}, dst[2] = {1, 3};
    epos_t *E = join_positions(ix, iy, src, dst, 2);
    *out_kind = edge_pair_crossing(&E[0], &E[1]);
    if (out_angle) *out_angle = crossing_angle(&E[0], &E[1]);
    free(E);
    (void)ideal_angle;
    free(ix); free(iy);
    return 0;
}

/* ------------------------------ loss of a layout-optimisation step (adjoint)
 *
 * The paper names layout optimisation as an application (Conclusion) without
 * defining a loss; the reading used here (R14) is
 *     L = w_a (1 - E_ca) + w_l M_l
 *       = w_a / (ideal |S|) sum_{(e,f) in S} |ideal - a_ef|  +  w_l M_l,
 * with the crossing set S frozen (found on the integer layout, then held
 * fixed while the coordinates move), a_ef = atan2(|c|, |g|) the acute line
 * angle from c = d_e x d_f and g = d_e . d_f, and M_l of Algorithm 3.
 * The gradient is the plain chain rule of that expression, with the
 * one-sided kinks (a = ideal, g = 0, c = 0, equal edge lengths, zero-length
 * edges) contributing 0. */

/* S: every crossing pair e < f (Algorithms 4/5 with readings R2, R3), in
 * (e, f) order; written only when cap >= |S|. */
int oracle_crossing_pairs(const double *x, const double *y, int64_t n,
                          const int32_t *src, const int32_t *dst, int64_t m,
                          int64_t *out_pairs, int64_t cap, int64_t *out_n) {
    if (n < 0 || m < 0 || !out_n || cap < 0 || (cap > 0 && !out_pairs)) return 1;
    if (check_edges(src, dst, m, n)) return 3;
    int64_t *ix, *iy;
    int st = to_int_coords(x, y, n, &ix, &iy);
    if (st) return st;
    epos_t *E = join_positions(ix, iy, src, dst, m);
    /* count per row, then fill each row's slice: the pairs come out in
     * (e, f) order whatever the thread count */
    int64_t *row = (int64_t *)calloc((size_t)m + 1, sizeof(int64_t));
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t e = 0; e < m; ++e) {
        int64_t c = 0;
        for (int64_t f = e + 1; f < m; ++f)
            c += edge_pair_crossing(&E[e], &E[f]) != 0;
        row[e + 1] = c;
    }
    for (int64_t e = 0; e < m; ++e) row[e + 1] += row[e];
    const int64_t k = m ? row[m] : 0;
    if (cap >= k && k > 0) {
        #pragma omp parallel for schedule(dynamic, 16)
        for (int64_t e = 0; e < m; ++e) {
            int64_t at = row[e];
            for (int64_t f = e + 1; f < m; ++f)
                if (edge_pair_crossing(&E[e], &E[f])) {
                    out_pairs[2 * at] = e;
                    out_pairs[2 * at + 1] = f;
                    ++at;
                }
        }
    }
    free(row);
    free(E); free(ix); free(iy);
    *out_n = k;
    return 0;
}

static double sgn(double v) { return (v > 0.0) - (v < 0.0); }

/* loss and, when gx/gy are given, its analytic gradient (arrays of n) */
static int loss_impl(const double *x, const double *y, int64_t n, const int32_t *src,
                     const int32_t *dst, int64_t m, const int64_t *pairs, int64_t n_pairs,
                     double ideal, double w_a, double w_l, double *out_loss, double *gx,
                     double *gy) {
    if (n < 0 || m < 0 || n_pairs < 0 || (n_pairs > 0 && !pairs) || !(ideal > 0.0) || !out_loss)
        return 1;
    if (check_edges(src, dst, m, n)) return 3;
    for (int64_t i = 0; i < n_pairs; ++i)
        if (pairs[2 * i] < 0 || pairs[2 * i] >= m || pairs[2 * i + 1] < 0 || pairs[2 * i + 1] >= m)
            return 1;
    if (gx) for (int64_t v = 0; v < n; ++v) { gx[v] = 0.0; gy[v] = 0.0; }
    /* crossing-angle term */
    nsum dev = {0.0, 0.0};
    const double scale = n_pairs ? w_a / (ideal * (double)n_pairs) : 0.0;
    for (int64_t i = 0; i < n_pairs; ++i) {
        const int64_t e = pairs[2 * i], f = pairs[2 * i + 1];
        const double ax = x[dst[e]] - x[src[e]], ay = y[dst[e]] - y[src[e]];
        const double bx = x[dst[f]] - x[src[f]], by = y[dst[f]] - y[src[f]];
        const double c = ax * by - ay * bx, g = ax * bx + ay * by;
        const double a = atan2(fabs(c), fabs(g));
        nsum_add(&dev, fabs(ideal - a));
        if (!gx || c == 0.0) continue;
        /* d|ideal - a|/da = -sgn(ideal - a);  a = atan2(|c|, |g|) */
        const double k = -sgn(ideal - a) * scale;
        const double den = c * c + g * g;
        const double da_dc = sgn(c) * fabs(g) / den, da_dg = -sgn(g) * fabs(c) / den;
        /* c = ax by - ay bx,  g = ax bx + ay by */
        const double dax = da_dc * by + da_dg * bx, day = -da_dc * bx + da_dg * by;
        const double dbx = -da_dc * ay + da_dg * ax, dby = da_dc * ax + da_dg * ay;
        gx[dst[e]] += k * dax; gx[src[e]] -= k * dax;
        gy[dst[e]] += k * day; gy[src[e]] -= k * day;
        gx[dst[f]] += k * dbx; gx[src[f]] -= k * dbx;
        gy[dst[f]] += k * dby; gy[src[f]] -= k * dby;
    }
    double loss = n_pairs ? w_a * nsum_get(&dev) / (ideal * (double)n_pairs) : 0.0;
    /* edge-length-variation term (Algorithm 3) */
    if (m >= 2) {
        double *len = (double *)malloc(sizeof(double) * (size_t)m);
        nsum s1 = {0.0, 0.0};
        for (int64_t e = 0; e < m; ++e) {
            const double dx = x[dst[e]] - x[src[e]], dy = y[dst[e]] - y[src[e]];
            len[e] = sqrt(dx * dx + dy * dy);
            nsum_add(&s1, len[e]);
        }
        const double N = (double)m, mu = nsum_get(&s1) / N;
        nsum s2 = {0.0, 0.0};
        for (int64_t e = 0; e < m; ++e) nsum_add(&s2, (len[e] - mu) * (len[e] - mu));
        if (mu > 0.0) {
            const double sigma = sqrt(nsum_get(&s2) / N);        /* population spread */
            const double ml = sigma / mu / sqrt(N - 1.0);
            loss += w_l * ml;
            if (gx && sigma > 0.0) {
                for (int64_t e = 0; e < m; ++e) {
                    if (len[e] == 0.0) continue;
                    /* dM_l/dl_e = ((l_e - mu)/(N sigma mu) - sigma/(N mu^2)) / sqrt(N - 1) */
                    const double dl = w_l * ((len[e] - mu) / (N * sigma * mu) - sigma / (N * mu * mu)) /
                                      sqrt(N - 1.0);
                    const double dx = x[dst[e]] - x[src[e]], dy = y[dst[e]] - y[src[e]];
                    gx[dst[e]] += dl * dx / len[e]; gx[src[e]] -= dl * dx / len[e];
                    gy[dst[e]] += dl * dy / len[e]; gy[src[e]] -= dl * dy / len[e];
                }
            }
        }
        free(len);
    }
    *out_loss = loss;
    return 0;
}

int oracle_loss(const double *x, const double *y, int64_t n, const int32_t *src,
                const int32_t *dst, int64_t m, const int64_t *pairs, int64_t n_pairs,
                double ideal, double w_a, double w_l, double *out_loss) {
    return loss_impl(x, y, n, src, dst, m, pairs, n_pairs, ideal, w_a, w_l, out_loss, NULL, NULL);
}

int oracle_loss_grad(const double *x, const double *y, int64_t n, const int32_t *src,
                     const int32_t *dst, int64_t m, const int64_t *pairs, int64_t n_pairs,
                     double ideal, double w_a, double w_l, double *out_loss, double *gx,
                     double *gy) {
    if (!gx || !gy) return 1;
    return loss_impl(x, y, n, src, dst, m, pairs, n_pairs, ideal, w_a, w_l, out_loss, gx, gy);
}

/* ------------------------------------------------ row slices of the sweeps
 * The pairs (i, j) with r0 <= i < r1 and i < j (edges for crossings, nodes
 * for occlusion): a slice of Algorithms 4/5 and 1, for checking one shard of
 * a layout too large for the full brute force. */
int oracle_crossing_angle_rows(const double *x, const double *y, int64_t n,
                               const int32_t *src, const int32_t *dst, int64_t m,
                               double ideal_angle, int64_t r0, int64_t r1,
                               uint64_t *out_count, uint64_t *out_proper,
                               double *out_dev_sum) {
    if (n < 0 || m < 0 || r0 < 0 || r1 < r0 || r1 > m || !out_count || !(ideal_angle > 0.0))
        return 1;
    if (check_edges(src, dst, m, n)) return 3;
    int64_t *ix, *iy;
    int st = to_int_coords(x, y, n, &ix, &iy);
    if (st) return st;
    epos_t *E = join_positions(ix, iy, src, dst, m);
    const int64_t k = r1 - r0;
    double *row_sum = (double *)calloc((size_t)(k > 0 ? k : 1), sizeof(double));
    uint64_t count = 0, proper = 0;
    #pragma omp parallel for schedule(dynamic, 4) reduction(+:count, proper)
    for (int64_t e = r0; e < r1; ++e) {
        nsum acc = {0.0, 0.0};
        for (int64_t f = e + 1; f < m; ++f) {
            int r = edge_pair_crossing(&E[e], &E[f]);
            if (!r) continue;
            nsum_add(&acc, fabs(ideal_angle - crossing_angle(&E[e], &E[f])) /
                               ideal_angle);
            count += 1;
            proper += (r == 2);
        }
        row_sum[e - r0] = nsum_get(&acc);
    }
    nsum tot = {0.0, 0.0};
    for (int64_t i = 0; i < k; ++i) nsum_add(&tot, row_sum[i]);
    free(row_sum); free(E); free(ix); free(iy);
    *out_count = count;
    if (out_proper) *out_proper = proper;
    if (out_dev_sum) *out_dev_sum = nsum_get(&tot);
    return 0;
}

int oracle_node_occlusion_rows(const double *x, const double *y, int64_t n, double diameter,
                               int64_t r0, int64_t r1, uint64_t *out_count) {
    if (n < 0 || r0 < 0 || r1 < r0 || r1 > n || !out_count || !(diameter >= 0.0) || isinf(diameter))
        return 1;
    int64_t *ix, *iy;
    int st = to_int_coords(x, y, n, &ix, &iy);
    if (st) return st;
    uint64_t total = 0;
    #pragma omp parallel for schedule(dynamic, 16) reduction(+:total)
    for (int64_t v = r0; v < r1; ++v)
        for (int64_t u = v + 1; u < n; ++u) {
            int64_t dx = ix[v] - ix[u], dy = iy[v] - iy[u];
            if (less_than_square(dx * dx + dy * dy, diameter)) total += 1;
        }
    free(ix); free(iy);
    *out_count = total;
    return 0;
}

/* ------------------------------- Section 3.2.2 / 3.2.3: strip approximation
 *
 * The enhanced edge-crossing and crossing-angle methods cut the plane into
 * strips X_k = x0 + k w (x0 the smallest node coordinate, w an integer width;
 * horizontal != 0 swaps the roles of x and y).  Within strip k they compare
 * only edges that span it (x_min <= X_k and x_max >= X_{k+1}, so vertical
 * edges never take part) and count a pair as crossing when the order of
 * their y values at the two strip lines is reversed; the crossing angle
 * averages |ideal - a| / ideal over those pairs.  Reading taken: reversed
 * means strictly (equal y at either line, e.g. a crossing on a strip line,
 * does not count).  y at X is the rational (y1 dx + (X - x1) dy) / dx with the
 * edge oriented so that dx > 0; orders are compared exactly in 128 bits. */
static int y_order(int64_t X, const int64_t *a, const int64_t *b) {
    /* a, b: {x1, y1, dx, dy} with dx > 0; sign of y_a(X) - y_b(X) */
    __int128 na = (__int128)a[1] * a[2] + (__int128)(X - a[0]) * a[3];
    __int128 nb = (__int128)b[1] * b[2] + (__int128)(X - b[0]) * b[3];
    __int128 l = na * b[2], r = nb * a[2];
    return (l > r) - (l < r);
}

int oracle_enhanced_crossing(const double *x, const double *y, int64_t n,
                             const int32_t *src, const int32_t *dst, int64_t m,
                             int64_t width, int horizontal, double ideal_angle,
                             uint64_t *out_count, double *out_dev_sum) {
    if (n < 0 || m < 0 || width < 1 || !out_count || !(ideal_angle > 0.0)) return 1;
    if (check_edges(src, dst, m, n)) return 3;
    int64_t *ix, *iy;
    int st = to_int_coords(x, y, n, &ix, &iy);
    if (st) return st;
    if (horizontal) { int64_t *t = ix; ix = iy; iy = t; }
    int64_t x0 = 0;
    for (int64_t i = 0; i < n; ++i) if (i == 0 || ix[i] < x0) x0 = ix[i];
    /* edges as {x1, y1, dx, dy} with dx > 0; strips k0 <= k < k1 spanned */
    int64_t *E = (int64_t *)malloc(sizeof(int64_t) * 4 * (size_t)(m > 0 ? m : 1));
    int64_t *k0 = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    int64_t *k1 = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    int64_t kmax = 0;
    for (int64_t e = 0; e < m; ++e) {
        int64_t ax = ix[src[e]], ay = iy[src[e]], bx = ix[dst[e]], by = iy[dst[e]];
        if (bx < ax) { int64_t t = ax; ax = bx; bx = t; t = ay; ay = by; by = t; }
        E[4 * e] = ax; E[4 * e + 1] = ay; E[4 * e + 2] = bx - ax; E[4 * e + 3] = by - ay;
        /* first line at or right of ax, last line at or left of bx */
        k0[e] = (ax - x0 + width - 1) / width;
        k1[e] = (bx - x0) / width;            /* strips k0 .. k1-1 are spanned */
        if (bx == ax) k1[e] = k0[e];
        if (k1[e] > kmax) kmax = k1[e];
    }
    uint64_t count = 0;
    double *strip_sum = (double *)calloc((size_t)(kmax > 0 ? kmax : 1), sizeof(double));
    /* strips are independent: one per iteration, sums combined in strip order */
    #pragma omp parallel for schedule(dynamic, 1) reduction(+:count)
    for (int64_t k = 0; k < kmax; ++k) {
        int64_t *mem = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
        int64_t cnt = 0;
        for (int64_t e = 0; e < m; ++e)
            if (k0[e] <= k && k < k1[e]) mem[cnt++] = e;
        const int64_t XL = x0 + k * width, XR = XL + width;
        nsum acc = {0.0, 0.0};
        for (int64_t i = 0; i < cnt; ++i)
            for (int64_t j = i + 1; j < cnt; ++j) {
                const int64_t *a = E + 4 * mem[i], *b = E + 4 * mem[j];
                if (y_order(XL, a, b) * y_order(XR, a, b) >= 0) continue;
                count += 1;
                /* acute angle between the lines (the exact path's definition) */
                int64_t cr = a[2] * b[3] - a[3] * b[2];
                int64_t dt = a[2] * b[2] + a[3] * b[3];
                double ang = atan2(fabs((double)cr), fabs((double)dt));
                nsum_add(&acc, fabs(ideal_angle - ang) / ideal_angle);
            }
        strip_sum[k] = nsum_get(&acc);
        free(mem);
    }
    nsum tot = {0.0, 0.0};
    for (int64_t k = 0; k < kmax; ++k) nsum_add(&tot, strip_sum[k]);
    free(strip_sum);
    free(E); free(k0); free(k1); free(ix); free(iy);
    *out_count = count;
    if (out_dev_sum) *out_dev_sum = nsum_get(&tot);
    return 0;
}

/* ------------------------------ minimum-angle term of the optimisation loss
 *
 * T = w_m (1 - M_a) at (possibly non-integer) coordinates, with M_a of
 * Algorithm 2 (mean over vertices of degree >= 1, readings R9, R10):
 * 1 - M_a = 1 - (1/N) sum_v phi_v deg_v / (2 pi), phi_v the smallest gap
 * between the sorted directions v -> u of v's edges (2 pi for degree 1).
 * phi_v moves with the two directions that bound that gap, so
 *     dT/d alpha_next = -dT/d alpha_prev = -w_m deg_v / (2 pi N),
 * and a direction alpha of v -> u turns with u as (-dy, dx) / l^2 (and with v
 * as the opposite).  Kinks contribute 0: a smallest gap attained twice, a
 * zero gap (two edges in one direction) or a zero-length edge bounding it.
 * The gradient (if gx, gy are given) is added to gx, gy.
 *
 * Which gap is smallest, and whether it is attained twice, is decided
 * exactly when every coordinate is an integer with |c| <= 2^20 (the domain
 * of the library): the gap from direction p to the next direction q is the
 * angle of the rotation taking p to q, the argument in [0, 2 pi) of
 * z = (p . q, p x q), and two such arguments are compared by the half plane
 * of z and the sign of the 128-bit cross product of the two z (no rounding;
 * gaps that are equal as real numbers, e.g. to (2,1), (1,1), (1,2), tie).
 * A zero-length edge points along +x (R10: atan2(0, 0) = 0).  At other
 * coordinates (the finite-difference pins jitter the layout off the
 * integers, where exact ties do not occur) the gaps are compared as the
 * differences of the sorted double angles. */
typedef struct { double a; int32_t u; int64_t dx, dy; } dir_t;

static int cmp_dir(const void *p, const void *q) {
    double a = ((const dir_t *)p)->a, b = ((const dir_t *)q)->a;
    return (a > b) - (a < b);
}

typedef struct { int64_t dot, cr; } gapz_t;   /* p . q and p x q */

static gapz_t gap_between(const dir_t *p, const dir_t *q) {
    int64_t px = p->dx, py = p->dy, qx = q->dx, qy = q->dy;
    if (px == 0 && py == 0) px = 1;            /* R10: direction 0 */
    if (qx == 0 && qy == 0) qx = 1;
    gapz_t z = {px * qx + py * qy, px * qy - py * qx};
    return z;
}

/* 0 for an argument in [0, pi), 1 for [pi, 2 pi) (z is never 0) */
static int gap_half(gapz_t z) { return (z.cr > 0 || (z.cr == 0 && z.dot > 0)) ? 0 : 1; }

/* sign of arg(a) - arg(b), both in [0, 2 pi) */
static int gap_cmp(gapz_t a, gapz_t b) {
    int ha = gap_half(a), hb = gap_half(b);
    if (ha != hb) return ha < hb ? -1 : 1;
    __int128 c = (__int128)a.dot * b.cr - (__int128)a.cr * b.dot;   /* a x b */
    return c > 0 ? -1 : (c < 0 ? 1 : 0);
}

int oracle_min_angle_term(const double *x, const double *y, int64_t n, const int32_t *src,
                          const int32_t *dst, int64_t m, double w_m, double *out_term,
                          double *gx, double *gy) {
    if (n < 0 || m < 0 || !out_term) return 1;
    if (check_edges(src, dst, m, n)) return 3;
    const double two_pi = 2.0 * M_PI;
    int64_t *deg = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t e = 0; e < m; ++e) { deg[src[e]]++; deg[dst[e]]++; }
    int64_t *start = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t v = 0; v < n; ++v) start[v + 1] = start[v] + deg[v];
    int64_t *fill = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    for (int64_t e = 0; e < m; ++e) {
        nbr[start[src[e]] + fill[src[e]]++] = dst[e];
        nbr[start[dst[e]] + fill[dst[e]]++] = src[e];
    }
    int64_t used = 0;
    for (int64_t v = 0; v < n; ++v) used += deg[v] > 0;
    int64_t *ix = NULL, *iy = NULL;
    const int exact = to_int_coords(x, y, n, &ix, &iy) == 0;   /* integer layout */
    nsum tot = {0.0, 0.0};
    dir_t *dir = (dir_t *)malloc(sizeof(dir_t) * (size_t)(2 * m + 1));
    for (int64_t v = 0; v < n; ++v) {
        const int64_t k = deg[v];
        if (k == 0) continue;
        for (int64_t i = 0; i < k; ++i) {
            const int32_t u = nbr[start[v] + i];
            double a = atan2(y[u] - y[v], x[u] - x[v]);
            if (a < 0.0) a += two_pi;                                  /* R10 */
            dir[i].a = a;
            dir[i].u = u;
            dir[i].dx = exact ? ix[u] - ix[v] : 0;
            dir[i].dy = exact ? iy[u] - iy[v] : 0;
        }
        qsort(dir, (size_t)k, sizeof(dir_t), cmp_dir);
        /* gaps: dir[i] -> dir[i+1], and the wrap dir[k-1] -> dir[0] */
        double phi = two_pi;                             /* the metric's phi_v */
        int64_t at = -1, ties = 0;                       /* the gradient's gap */
        int zero_gap = 0;
        if (k >= 2) {
            double best_g = two_pi;
            gapz_t best_z = {0, 0};
            for (int64_t i = 0; i < k; ++i) {
                const double g = i + 1 < k ? dir[i + 1].a - dir[i].a
                                           : two_pi - dir[k - 1].a + dir[0].a;
                if (g < phi) phi = g;
                int c;
                if (exact) {
                    const gapz_t z = gap_between(&dir[i], &dir[i + 1 < k ? i + 1 : 0]);
                    c = at < 0 ? -1 : gap_cmp(z, best_z);
                    if (c < 0) best_z = z;
                } else {
                    c = (at < 0 || g < best_g) ? -1 : (g == best_g ? 0 : 1);
                }
                if (c < 0) { best_g = g; at = i; ties = 1; }
                else if (c == 0) ties++;
            }
            zero_gap = exact ? (best_z.cr == 0 && best_z.dot > 0) : !(best_g > 0.0);
        }
        nsum_add(&tot, phi * (double)k / two_pi);
        if (!gx || !gy || k < 2 || ties != 1 || zero_gap) continue;
        const double c = -w_m * (double)k / (two_pi * (double)used);   /* dT / d phi_v */
        const dir_t p = dir[at], q = dir[at + 1 < k ? at + 1 : 0];
        const double pdx = x[p.u] - x[v], pdy = y[p.u] - y[v];
        const double qdx = x[q.u] - x[v], qdy = y[q.u] - y[v];
        const double pl2 = pdx * pdx + pdy * pdy, ql2 = qdx * qdx + qdy * qdy;
        if (pl2 == 0.0 || ql2 == 0.0) continue;
        /* phi = alpha_q - alpha_p: +1 through q, -1 through p */
        gx[q.u] += c * -qdy / ql2;  gy[q.u] += c * qdx / ql2;
        gx[v] -= c * -qdy / ql2;    gy[v] -= c * qdx / ql2;
        gx[p.u] -= c * -pdy / pl2;  gy[p.u] -= c * pdx / pl2;
        gx[v] += c * -pdy / pl2;    gy[v] += c * pdx / pl2;
    }
    *out_term = used ? w_m * (1.0 - nsum_get(&tot) / (double)used) : 0.0;
    if (exact) { free(ix); free(iy); }
    free(dir); free(deg); free(start); free(fill); free(nbr);
    return 0;
}
