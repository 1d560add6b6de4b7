/*
 * Fermat path oracle -- TEST INFRASTRUCTURE ONLY (tests, the smoke check and
 * the CPU-baseline leg of the benchmark). Plain FP64 CPU reference of the
 * path-length minimisation of Sec. III-B (Eqs. 1-5) and of the
 * implicit-differentiation gradient of Sec. III-D (Eqs. 8-13).
 *
 * Inputs use the C-ABI tables (FP32 object table obj[9][K]: b, a1, a2 with
 * a2 == 0 marking an edge; point table pts[3][Q]; src/dst[N]; order[N] or
 * NULL (= n_max for every path); ids[n_max][N]).
 * Outputs are path-major FP64:
 *   x_out [N][n_max][3]  interaction points (NaN beyond the path's order)
 *   len_out [N]          L(T*) with exact (unsmoothed) segment lengths
 *   t_out [N][n_max][2]  parameters; the padded second parameter of an edge
 *                        is 0
 *   flags [N]            ORACLE_* bits
 *   iters [N]            Newton iterations over all smoothing levels
 * All functions return 0, or -1 on invalid sizes (nothing is written then).
 */
#ifndef FERMAT_ORACLE_H
#define FERMAT_ORACLE_H

#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_NMAX 6

enum {
  ORACLE_COLLAPSED = 1, /* two consecutive points closer than 1e-6 S */
  ORACLE_ILL = 2,       /* Hessian condition number above 1e12 */
  ORACLE_NOCONV = 4,    /* last smoothing level hit its iteration cap */
  ORACLE_INVALID = 8,   /* bad id / order / point index or non-finite input */
  ORACLE_KKT = 16       /* gradient of a collapsed minimiser (constrained form) */
};

/* validity bits of oracle_validate */
enum { ORACLE_EXTENT = 1, ORACLE_SPECULAR = 2, ORACLE_VISIBLE = 4 };

int oracle_solve(int64_t N, int n_max, const float *obj, int64_t K,
                 const float *pts, int64_t Q, const int32_t *src,
                 const int32_t *dst, const uint8_t *order, const int32_t *ids,
                 double S, double *x_out, double *len_out, double *t_out,
                 int32_t *flags, int32_t *iters, int nthreads);

/* Gradient of  sum_i g_len[i] L*_i + sum_{i,j} g_x[i][j] . x*_ij  with respect
 * to TX (g_tx[N][3]), RX (g_rx[N][3]) and each slot's object b (g_b[N][n][3])
 * and basis vectors (g_a[N][n][2][3]), per path (not summed over objects).
 * t_sol is a solution in the t_out layout. status[i] is 0 for a smooth
 * minimiser (the IFT of Sec. III-D), ORACLE_KKT for a minimiser with one
 * interior segment shorter than 1e-6 S whose two objects' directions span
 * space (the IFT on the KKT conditions of the collapse constraint), and
 * ORACLE_COLLAPSED for any other collapse or a singular system (outputs
 * NaN). */
int oracle_grad(int64_t N, int n_max, const float *obj, int64_t K,
                const float *pts, int64_t Q, const int32_t *src,
                const int32_t *dst, const uint8_t *order, const int32_t *ids,
                double S, const double *t_sol, const double *g_len,
                const double *g_x, double *g_tx, double *g_rx, double *g_b,
                double *g_a, int32_t *status, int nthreads);

/* L(T) (Eq. 5) at given parameters t_in [N][n_max][2]. */
int oracle_length(int64_t N, int n_max, const float *obj, int64_t K,
                  const float *pts, int64_t Q, const int32_t *src,
                  const int32_t *dst, const uint8_t *order, const int32_t *ids,
                  const double *t_in, double *len_out);

/* Validity of solved paths on finite objects (see fermat_oracle.c):
 * t_in [N][n_max][2], x_in [N][n_max][3] path-major; flags [N]. */
int oracle_validate(int64_t N, int n_max, const float *obj, int64_t K,
                    const float *pts, int64_t Q, const int32_t *src,
                    const int32_t *dst, const uint8_t *order, const int32_t *ids,
                    double S, const double *t_in, const double *x_in,
                    double tol, uint8_t *flags, int nthreads);

#endif
