/* CPU oracle of the readability metrics -- test infrastructure only.
 * Coordinates are passed as doubles holding integers with |c| <= 2^20.
 * All functions return 0 on success (see oracle.c for the other codes). */
#ifndef RB_ORACLE_H
#define RB_ORACLE_H
#include <stdint.h>

int oracle_node_occlusion(const double *x, const double *y, int64_t n,
                          double diameter, uint64_t *out_count);
int oracle_edge_crossing(const double *x, const double *y, int64_t n,
                         const int32_t *src, const int32_t *dst, int64_t m,
                         uint64_t *out_count, uint64_t *out_proper);
int oracle_crossing_angle(const double *x, const double *y, int64_t n,
                          const int32_t *src, const int32_t *dst, int64_t m,
                          double ideal_angle, double *out_metric,
                          uint64_t *out_count, double *out_dev_sum);
int oracle_crossings_of_edges(const double *x, const double *y, int64_t n,
                              const int32_t *src, const int32_t *dst, int64_t m,
                              double ideal_angle, const int64_t *which, int64_t k,
                              uint64_t *out_count, double *out_dev);
int oracle_min_angle(const double *x, const double *y, int64_t n,
                     const int32_t *src, const int32_t *dst, int64_t m,
                     double *out_metric, double *out_sum_dv, uint64_t *out_n_used);
int oracle_edge_length_variation(const double *x, const double *y, int64_t n,
                                 const int32_t *src, const int32_t *dst, int64_t m,
                                 double *out_metric, double *out_mean);
int oracle_segment_pair(const double *p, double ideal_angle, int *out_kind,
                        double *out_angle);
int oracle_crossing_pairs(const double *x, const double *y, int64_t n,
                          const int32_t *src, const int32_t *dst, int64_t m,
                          int64_t *out_pairs, int64_t cap, int64_t *out_n);
int oracle_loss(const double *x, const double *y, int64_t n, const int32_t *src,
                const int32_t *dst, int64_t m, const int64_t *pairs, int64_t n_pairs,
                double ideal, double w_a, double w_l, double *out_loss);
int oracle_loss_grad(const double *x, const double *y, int64_t n, const int32_t *src,
                     const int32_t *dst, int64_t m, const int64_t *pairs, int64_t n_pairs,
                     double ideal, double w_a, double w_l, double *out_loss, double *gx,
                     double *gy);
int oracle_crossing_angle_rows(const double *x, const double *y, int64_t n,
                               const int32_t *src, const int32_t *dst, int64_t m,
                               double ideal_angle, int64_t r0, int64_t r1,
                               uint64_t *out_count, uint64_t *out_proper,
                               double *out_dev_sum);
int oracle_node_occlusion_rows(const double *x, const double *y, int64_t n, double diameter,
                               int64_t r0, int64_t r1, uint64_t *out_count);
int oracle_enhanced_crossing(const double *x, const double *y, int64_t n,
                             const int32_t *src, const int32_t *dst, int64_t m,
                             int64_t width, int horizontal, double ideal_angle,
                             uint64_t *out_count, double *out_dev_sum);
int oracle_min_angle_term(const double *x, const double *y, int64_t n, const int32_t *src,
                          const int32_t *dst, int64_t m, double w_m, double *out_term,
                          double *gx, double *gy);
#endif
