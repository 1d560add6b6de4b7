/*
 * Fermat path oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU reference for the shortest-path problem of
 * Sec. III-B (Eqs. 1-5): for every candidate path
 *     x_0 = TX,  x_j = A_j t_j + b_j (j = 1..n),  x_{n+1} = RX,
 *     L(T) = sum_{i=0}^{n} || x_{i+1} - x_i ||,
 * it returns the minimiser T* (Eq. 4), the points X* = A T* + B and L(T*).
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this file; the product path never does.
 *
 * The result has a plain definition (the arg min of a convex function, which
 * Sec. III-B states is strictly convex in parametric space), so the oracle is
 * a generic, obviously-correct minimiser of that definition, not the paper's
 * BFGS iteration:
 *   1. keep only the active parameters of each object: two for a plane, one
 *      for an edge (its zero second basis vector is layout padding, Sec.
 *      III-B, so it is dropped here);
 *   2. replace each segment length ||r|| by sqrt(||r||^2 + eps^2), a smooth
 *      convex majorant that differs from it by at most eps, so that a
 *      minimiser where two consecutive points coincide (the objective is
 *      nonsmooth there, Sec. V) is still reached by Newton's method;
 *   3. damped Newton (exact gradient and Hessian, dense Gaussian elimination,
 *      Armijo backtracking) at eps = 1e-1 S, 1e-2 S, ..., 1e-15 S, each level
 *      warm-started from the previous one.  Since |r| <= sqrt(|r|^2+eps^2)
 *      <= |r| + eps, the length at the smoothed minimiser exceeds the true
 *      minimum by at most (n+1) eps.  Points move by O(eps) at a smooth
 *      minimiser and by O(eps^(2/3)) in the worst case seen (a straight
 *      pass-through exactly at the meeting line of two planes), i.e. about
 *      1e-10 S at the last level.
 *
 * The gradient oracle (oracle_grad) applies the implicit function theorem of
 * Sec. III-D (Eqs. 8-13) with the Hessian and the mixed derivatives of the
 * optimality condition written out in closed form (derivation in the
 * comments of grad_one), in FP64, at a given solution. At a minimiser with
 * one interior zero-length segment it applies the same theorem to the KKT
 * conditions of the length without that segment under the constraint that
 * its two points coincide (grad_one_kkt, a dense solve of the bordered
 * system): an extension of Sec. III-D, which covers smooth minimisers only,
 * pinned by finite differences of the solve above.
 *
 * Inputs are the FP32 tables of the C ABI, widened exactly to FP64.
 * Outputs are path-major FP64 arrays (see fermat_oracle.h).
 */
#include "fermat_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NMAX ORACLE_NMAX
#define MMAX (2 * ORACLE_NMAX)

typedef struct {
  int n;                 /* interactions */
  int m;                 /* active parameters */
  double x0[3], xe[3];   /* x_0 = TX, x_{n+1} = RX */
  double b[NMAX][3];
  double a[NMAX][2][3];  /* a[j][k] = k-th basis vector of object j */
  int d[NMAX];           /* 1 = edge, 2 = plane */
  int cs[MMAX], ck[MMAX];/* active column c -> (slot, basis index) */
} path_t;

/* ---------------------------------------------------------------- gather -- */

static int load_path(path_t *p, int64_t i, int64_t N, int n_max,
                     const float *obj, int64_t K, const float *pts, int64_t Q,
                     const int32_t *src, const int32_t *dst,
                     const uint8_t *order, const int32_t *ids) {
  int n = order ? (int)order[i] : n_max;
  if (n < 1 || n > n_max) return -1;
  int64_t s = src[i], e = dst[i];
  if (s < 0 || s >= Q || e < 0 || e >= Q) return -1;
  p->n = n;
  for (int c = 0; c < 3; ++c) {
    p->x0[c] = (double)pts[c * Q + s];
    p->xe[c] = (double)pts[c * Q + e];
  }
  int m = 0;
  for (int j = 0; j < n; ++j) {
    int64_t k = ids[(int64_t)j * N + i];
    if (k < 0 || k >= K) return -1;
    for (int c = 0; c < 3; ++c) {
      p->b[j][c] = (double)obj[(0 + c) * K + k];
      p->a[j][0][c] = (double)obj[(3 + c) * K + k];
      p->a[j][1][c] = (double)obj[(6 + c) * K + k];
    }
    int edge = p->a[j][1][0] == 0.0 && p->a[j][1][1] == 0.0 &&
               p->a[j][1][2] == 0.0;
    p->d[j] = edge ? 1 : 2;
    for (int k2 = 0; k2 < p->d[j]; ++k2) {
      p->cs[m] = j;
      p->ck[m] = k2;
      ++m;
    }
  }
  p->m = m;
  for (int c = 0; c < 3; ++c)
    if (!isfinite(p->x0[c]) || !isfinite(p->xe[c])) return -1;
  for (int j = 0; j < n; ++j)
    for (int c = 0; c < 3; ++c)
      if (!isfinite(p->b[j][c]) || !isfinite(p->a[j][0][c]) ||
          !isfinite(p->a[j][1][c]))
        return -1;
  return 0;
}

/* --------------------------------------------------------- path algebra -- */

/* X = A T + B for active parameters t[m] (Eq. 3); x[0] = TX, x[n+1] = RX */
static void points(const path_t *p, const double *t, double x[NMAX + 2][3]) {
  memcpy(x[0], p->x0, sizeof p->x0);
  memcpy(x[p->n + 1], p->xe, sizeof p->xe);
  for (int j = 0; j < p->n; ++j) memcpy(x[j + 1], p->b[j], sizeof p->b[j]);
  for (int c = 0; c < p->m; ++c) {
    int j = p->cs[c], k = p->ck[c];
    for (int q = 0; q < 3; ++q) x[j + 1][q] += t[c] * p->a[j][k][q];
  }
}

static double dot3(const double *u, const double *v) {
  return u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
}

/* smoothed length sum_i sqrt(||x_{i+1} - x_i||^2 + eps^2) (Eq. 5 at eps=0) */
static double length_eps(const path_t *p, const double *t, double eps) {
  double x[NMAX + 2][3];
  points(p, t, x);
  double L = 0.0;
  for (int i = 0; i <= p->n; ++i) {
    double r[3] = {x[i + 1][0] - x[i][0], x[i + 1][1] - x[i][1],
                   x[i + 1][2] - x[i][2]};
    L += sqrt(dot3(r, r) + eps * eps);
  }
  return L;
}

/* Gradient and Hessian of the smoothed length in the active parameters.
 * Segment i (x_i -> x_{i+1}), l_i = sqrt(|r_i|^2 + eps^2), v_i = r_i / l_i:
 *   dl_i/dr_i = v_i,  d^2 l_i/dr_i^2 = M_i = (I - r_i r_i^T / l_i^2) / l_i.
 * Point x_j enters r_{j-1} with sign +1 and r_j with sign -1, so
 *   g_c   = a_c . (v_{j-1} - v_j)                       (c on slot j),
 *   H_cd  = sum_i s_ic s_id a_c^T M_i a_d               (c, d touching i).
 * Segment `skip` (if 0..n) is left out of both: the length without it. */
static void grad_hess_skip(const path_t *p, const double *t, double eps,
                           int skip, double *g, double H[MMAX][MMAX]) {
  double x[NMAX + 2][3];
  points(p, t, x);
  int m = p->m, n = p->n;
  double v[NMAX + 1][3], M[NMAX + 1][3][3];
  for (int i = 0; i <= n; ++i) {
    double r[3] = {x[i + 1][0] - x[i][0], x[i + 1][1] - x[i][1],
                   x[i + 1][2] - x[i][2]};
    double l = sqrt(dot3(r, r) + eps * eps);
    if (l < 1e-300) l = 1e-300;
    for (int q = 0; q < 3; ++q) v[i][q] = r[q] / l;
    for (int q = 0; q < 3; ++q)
      for (int w = 0; w < 3; ++w)
        M[i][q][w] = ((q == w ? 1.0 : 0.0) - r[q] * r[w] / (l * l)) / l;
    if (i == skip) {
      for (int q = 0; q < 3; ++q) {
        v[i][q] = 0.0;
        for (int w = 0; w < 3; ++w) M[i][q][w] = 0.0;
      }
    }
  }
  for (int c = 0; c < m; ++c) {
    int j = p->cs[c];
    const double *ac = p->a[j][p->ck[c]];
    /* slot j is point x_{j+1} in the 0..n+1 numbering: segments j and j+1 */
    double dv[3] = {v[j][0] - v[j + 1][0], v[j][1] - v[j + 1][1],
                    v[j][2] - v[j + 1][2]};
    g[c] = dot3(ac, dv);
  }
  for (int c = 0; c < m; ++c)
    for (int d = 0; d < m; ++d) H[c][d] = 0.0;
  for (int i = 0; i <= n; ++i) {
    /* segment i joins point i (slot i-1, sign -1) and point i+1 (slot i, +1) */
    for (int c = 0; c < m; ++c) {
      int jc = p->cs[c];
      double sc;
      if (jc == i) sc = 1.0;           /* point i+1 is slot i  */
      else if (jc == i - 1) sc = -1.0; /* point i   is slot i-1 */
      else continue;
      const double *ac = p->a[jc][p->ck[c]];
      double Ma[3];
      for (int q = 0; q < 3; ++q)
        Ma[q] = M[i][q][0] * ac[0] + M[i][q][1] * ac[1] + M[i][q][2] * ac[2];
      for (int d = 0; d < m; ++d) {
        int jd = p->cs[d];
        double sd;
        if (jd == i) sd = 1.0;
        else if (jd == i - 1) sd = -1.0;
        else continue;
        H[d][c] += sc * sd * dot3(p->a[jd][p->ck[d]], Ma);
      }
    }
  }
}

static void grad_hess(const path_t *p, const double *t, double eps, double *g,
                      double H[MMAX][MMAX]) {
  grad_hess_skip(p, t, eps, -1, g, H);
}

/* Dense Gaussian elimination with partial pivoting: solves A y = rhs for an
 * m x m matrix stored with row stride ld (m <= KMAX). A is overwritten.
 * Returns -1 if a pivot is exactly zero. */
#define KMAX (MMAX + 3)
static int gauss_solve_ld(int m, int ld, double *A, const double *rhs,
                          double *y) {
  double b[KMAX];
  memcpy(b, rhs, sizeof(double) * m);
#define AE(r, c) A[(r) * ld + (c)]
  for (int k = 0; k < m; ++k) {
    int piv = k;
    for (int r = k + 1; r < m; ++r)
      if (fabs(AE(r, k)) > fabs(AE(piv, k))) piv = r;
    if (AE(piv, k) == 0.0) return -1;
    if (piv != k) {
      for (int c = 0; c < m; ++c) {
        double tmp = AE(k, c);
        AE(k, c) = AE(piv, c);
        AE(piv, c) = tmp;
      }
      double tmp = b[k];
      b[k] = b[piv];
      b[piv] = tmp;
    }
    for (int r = k + 1; r < m; ++r) {
      double f = AE(r, k) / AE(k, k);
      for (int c = k; c < m; ++c) AE(r, c) -= f * AE(k, c);
      b[r] -= f * b[k];
    }
  }
  for (int k = m - 1; k >= 0; --k) {
    double s = b[k];
    for (int c = k + 1; c < m; ++c) s -= AE(k, c) * y[c];
    y[k] = s / AE(k, k);
  }
#undef AE
  return 0;
}

static int gauss_solve(int m, double A[MMAX][MMAX], const double *rhs,
                       double *y) {
  return gauss_solve_ld(m, MMAX, &A[0][0], rhs, y);
}

/* Cyclic Jacobi eigenvalues of a symmetric matrix (for the ILL flag). */
static void jacobi_eigs(int m, double A[MMAX][MMAX], double *ev) {
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int r = 0; r < m; ++r)
      for (int c = r + 1; c < m; ++c) off += A[r][c] * A[r][c];
    if (off < 1e-300) break;
    for (int r = 0; r < m; ++r)
      for (int c = r + 1; c < m; ++c) {
        if (A[r][c] == 0.0) continue;
        double th = (A[c][c] - A[r][r]) / (2.0 * A[r][c]);
        double tt = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        double cs = 1.0 / sqrt(tt * tt + 1.0), sn = tt * cs;
        for (int k = 0; k < m; ++k) {
          double akr = A[k][r], akc = A[k][c];
          A[k][r] = cs * akr - sn * akc;
          A[k][c] = sn * akr + cs * akc;
        }
        for (int k = 0; k < m; ++k) {
          double ark = A[r][k], ack = A[c][k];
          A[r][k] = cs * ark - sn * ack;
          A[c][k] = sn * ark + cs * ack;
        }
      }
  }
  for (int k = 0; k < m; ++k) ev[k] = A[k][k];
}

/* Largest point displacement max_j |A_j dt_j| of a parameter step. */
static double max_disp(const path_t *p, const double *dt) {
  double mx = 0.0;
  for (int j = 0; j < p->n; ++j) {
    double w[3] = {0, 0, 0};
    for (int c = 0; c < p->m; ++c)
      if (p->cs[c] == j)
        for (int q = 0; q < 3; ++q) w[q] += dt[c] * p->a[j][p->ck[c]][q];
    double s = sqrt(dot3(w, w));
    if (s > mx) mx = s;
  }
  return mx;
}

/* ------------------------------------------------------------ the solve -- */

static int solve_one(const path_t *p, double S, double *t, int *iters_out) {
  const int m = p->m;
  const double eps_first = 1e-1, eps_last = 1e-15, eps_factor = 0.1;
  const int max_newton = 100;
  const double disp_stop = 1e-13 * S;
  int iters = 0, converged_last = 0;
  for (int c = 0; c < m; ++c) t[c] = 0.0; /* start at x_j = b_j */
  for (double er = eps_first; er >= eps_last * 0.5; er *= eps_factor) {
    const double eps = er * S;
    converged_last = 0;
    for (int it = 0; it < max_newton; ++it) {
      double g[MMAX], H[MMAX][MMAX], dt[MMAX], ng[MMAX];
      grad_hess(p, t, eps, g, H);
      double Hc[MMAX][MMAX];
      memcpy(Hc, H, sizeof Hc);
      for (int r = 0; r < m; ++r) ng[r] = -g[r];
      if (gauss_solve(m, Hc, ng, dt) != 0) {
        /* singular (e.g. a plane given by parallel vectors): regularise */
        double hmax = 0.0;
        for (int r = 0; r < m; ++r)
          for (int c = 0; c < m; ++c)
            if (fabs(H[r][c]) > hmax) hmax = fabs(H[r][c]);
        for (int r = 0; r < m; ++r) H[r][r] += 1e-12 * hmax + 1e-300;
        if (gauss_solve(m, H, ng, dt) != 0) break;
      }
      double slope = 0.0;
      for (int c = 0; c < m; ++c) slope += g[c] * dt[c];
      if (!(slope < 0.0)) { converged_last = 1; break; } /* no descent left */
      if (max_disp(p, dt) < disp_stop) { /* full step below resolution */
        double tn[MMAX];
        for (int c = 0; c < m; ++c) tn[c] = t[c] + dt[c];
        if (length_eps(p, tn, eps) <= length_eps(p, t, eps))
          memcpy(t, tn, sizeof(double) * m);
        ++iters;
        converged_last = 1;
        break;
      }
      double L0 = length_eps(p, t, eps), s = 1.0, tn[MMAX];
      int accepted = 0;
      while (s > 1e-16) {
        for (int c = 0; c < m; ++c) tn[c] = t[c] + s * dt[c];
        double L1 = length_eps(p, tn, eps);
        /* Armijo with an allowance for the rounding of L itself */
        if (L1 <= L0 + 1e-4 * s * slope + 4e-16 * fabs(L0)) { accepted = 1; break; }
        s *= 0.5;
      }
      ++iters;
      if (!accepted) { converged_last = 1; break; } /* stalled at rounding */
      memcpy(t, tn, sizeof(double) * m);
    }
  }
  *iters_out = iters;
  return converged_last;
}

int oracle_solve(int64_t N, int n_max, const float *obj, int64_t K,
                 const float *pts, int64_t Q, const int32_t *src,
                 const int32_t *dst, const uint8_t *order, const int32_t *ids,
                 double S, double *x_out, double *len_out, double *t_out,
                 int32_t *flags, int32_t *iters, int nthreads) {
  if (N < 0 || n_max < 1 || n_max > NMAX || S <= 0.0) return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t i = 0; i < N; ++i) {
    double *xo = x_out + i * n_max * 3, *to = t_out + i * n_max * 2;
    for (int k = 0; k < n_max * 3; ++k) xo[k] = NAN;
    for (int k = 0; k < n_max * 2; ++k) to[k] = NAN;
    len_out[i] = NAN;
    iters[i] = 0;
    path_t p;
    if (load_path(&p, i, N, n_max, obj, K, pts, Q, src, dst, order, ids)) {
      flags[i] = ORACLE_INVALID;
      continue;
    }
    double t[MMAX];
    int it = 0;
    int ok = solve_one(&p, S, t, &it);
    iters[i] = it;
    int32_t f = ok ? 0 : ORACLE_NOCONV;
    double x[NMAX + 2][3];
    points(&p, t, x);
    double minseg = INFINITY;
    for (int k = 0; k <= p.n; ++k) {
      double r[3] = {x[k + 1][0] - x[k][0], x[k + 1][1] - x[k][1],
                     x[k + 1][2] - x[k][2]};
      double l = sqrt(dot3(r, r));
      if (l < minseg) minseg = l;
    }
    if (minseg < 1e-6 * S) f |= ORACLE_COLLAPSED;
    /* conditioning of the unsmoothed Hessian at the solution */
    if (!(f & ORACLE_COLLAPSED)) {
      double g[MMAX], H[MMAX][MMAX], ev[MMAX];
      grad_hess(&p, t, 0.0, g, H);
      jacobi_eigs(p.m, H, ev);
      double lo = INFINITY, hi = 0.0;
      for (int k = 0; k < p.m; ++k) {
        if (fabs(ev[k]) < lo) lo = fabs(ev[k]);
        if (fabs(ev[k]) > hi) hi = fabs(ev[k]);
      }
      if (!(lo > 0.0) || hi / lo > 1e12) f |= ORACLE_ILL;
    }
    flags[i] = f;
    len_out[i] = length_eps(&p, t, 0.0);
    for (int j = 0; j < p.n; ++j)
      for (int q = 0; q < 3; ++q) xo[j * 3 + q] = x[j + 1][q];
    for (int j = 0; j < p.n; ++j) {
      to[j * 2 + 0] = 0.0;
      to[j * 2 + 1] = 0.0;
    }
    for (int c = 0; c < p.m; ++c) to[p.cs[c] * 2 + p.ck[c]] = t[c];
  }
  return 0;
}

/* ---------------------------------------------------- gradient (IFT) ----- */

/* One path. With u_i = r_i/l_i and P_i = (I - u_i u_i^T)/l_i at the solution:
 *
 *  Optimality (Eq. 8):  grad_T L = [A_j^T (u_{j-1} - u_j)]_j = 0.
 *  Hessian H = d grad_T L / dT, block tridiagonal:
 *     H_jj = A_j^T (P_{j-1} + P_j) A_j,  H_{j,j+1} = -A_j^T P_j A_{j+1}.
 *  Upstream cotangents: gl on L*, gx_j on x_j* = A_j t_j* + b_j.
 *  The L* part is the envelope term: d L* / d theta = d L / d theta at T*.
 *  The X* part is direct (dx_j/dtheta at fixed T) plus w^T dT* / dtheta with
 *  w_j = A_j^T gx_j; by Eqs. 9-13 that is -lam^T d(grad_T L)/dtheta with
 *  H lam = w (the paper's u is -lam, its v is w).
 *  lam^T grad_T L = sum_i delta_i . u_i with q_j = A_j lam_j (q_0=q_{n+1}=0),
 *  delta_i = q_{i+1} - q_i; its theta-derivative at fixed (T, lam) gives
 *     through q_j:  lam_j[k] (u_{j-1} - u_j)  on A_j[:,k];
 *     through u_i:  c_i = P_i delta_i on r_i, i.e. c_{j-1} - c_j on x_j,
 *                   -c_0 on TX, +c_n on RX.
 *  Summing up:
 *     g_TX  = -gl u_0 + c_0
 *     g_RX  =  gl u_n - c_n
 *     g_b_j =  gl (u_{j-1} - u_j) + gx_j - (c_{j-1} - c_j)
 *     g_A_j[:,k] = t_j[k] g_b_j - lam_j[k] (u_{j-1} - u_j).
 *  Slots j are numbered 0..n-1 below; point x_{j+1} is slot j.           */
static int grad_one(const path_t *p, const double *t, double gl,
                    const double *gx /* [n][3] */, double *g_tx, double *g_rx,
                    double *g_b, double *g_a /* [n][2][3] */, double S) {
  const int n = p->n, m = p->m;
  double x[NMAX + 2][3];
  points(p, t, x);
  double u[NMAX + 1][3], l[NMAX + 1];
  for (int i = 0; i <= n; ++i) {
    double r[3] = {x[i + 1][0] - x[i][0], x[i + 1][1] - x[i][1],
                   x[i + 1][2] - x[i][2]};
    l[i] = sqrt(dot3(r, r));
    if (!(l[i] > 1e-6 * S)) return -1; /* collapsed: H unbounded, IFT void */
    for (int q = 0; q < 3; ++q) u[i][q] = r[q] / l[i];
  }
  double g[MMAX], H[MMAX][MMAX], w[MMAX], lam[MMAX];
  grad_hess(p, t, 0.0, g, H);
  for (int c = 0; c < m; ++c)
    w[c] = dot3(p->a[p->cs[c]][p->ck[c]], gx + 3 * p->cs[c]);
  if (gauss_solve(m, H, w, lam) != 0) return -1;
  double lamj[NMAX][2] = {{0}};
  for (int c = 0; c < m; ++c) lamj[p->cs[c]][p->ck[c]] = lam[c];
  double tj[NMAX][2] = {{0}};
  for (int c = 0; c < m; ++c) tj[p->cs[c]][p->ck[c]] = t[c];
  /* q_j for points 0..n+1, delta_i and c_i for segments 0..n */
  double qp[NMAX + 2][3] = {{0}}, cseg[NMAX + 1][3];
  for (int j = 0; j < n; ++j)
    for (int q = 0; q < 3; ++q)
      qp[j + 1][q] = lamj[j][0] * p->a[j][0][q] + lamj[j][1] * p->a[j][1][q];
  for (int i = 0; i <= n; ++i) {
    double dl[3] = {qp[i + 1][0] - qp[i][0], qp[i + 1][1] - qp[i][1],
                    qp[i + 1][2] - qp[i][2]};
    double ud = dot3(u[i], dl);
    for (int q = 0; q < 3; ++q) cseg[i][q] = (dl[q] - u[i][q] * ud) / l[i];
  }
  for (int q = 0; q < 3; ++q) {
    g_tx[q] = -gl * u[0][q] + cseg[0][q];
    g_rx[q] = gl * u[n][q] - cseg[n][q];
  }
  for (int j = 0; j < n; ++j) {
    double du[3], gb[3];
    for (int q = 0; q < 3; ++q) {
      du[q] = u[j][q] - u[j + 1][q];
      gb[q] = gl * du[q] + gx[3 * j + q] - (cseg[j][q] - cseg[j + 1][q]);
      g_b[3 * j + q] = gb[q];
    }
    for (int k = 0; k < 2; ++k)
      for (int q = 0; q < 3; ++q)
        g_a[(j * 2 + k) * 3 + q] =
            (k < p->d[j]) ? tj[j][k] * gb[q] - lamj[j][k] * du[q] : 0.0;
  }
  return 0;
}

/* One path at a collapsed minimiser: exactly one segment z shorter than
 * 1e-6 S, an interior one (1 <= z <= n-1, joining slot z-1 = point z and
 * slot z = point z+1). Sec. III-D differentiates smooth minimisers only;
 * this extends it. Near such a minimiser the solution stays collapsed, so it
 * is the minimiser of
 *     L_s(T) = sum_{i != z} l_i   subject to   c(T) = x_z - x_{z+1} = 0,
 * with a multiplier mu: grad L_s + C^T mu = 0 (C = dc/dT, 3 x m). The
 * implicit function theorem applied to these KKT conditions gives:
 *   L* part:  dL* / dtheta = d(L_s + mu . c) / dtheta at fixed (T, mu);
 *   X* part:  [H_s C^T; C 0] [lam; nu] = [w; 0] (H_s the Hessian of L_s)
 *             and the contribution -lam . d(grad L_s + C^T mu)/d theta
 *             - nu . dc/d theta.
 * With w_z = -mu (a subgradient of the zero length: A_{z-1}^T (u_{z-1} -
 * w_z) = 0 and A_z^T (w_z - u_{z+1}) = 0) the closed forms of grad_one
 * hold with u_z replaced by w_z and c_z = 0, plus -nu on g_b of slot z-1
 * and +nu on g_b of slot z (dc/db), which g_A picks up through t g_b.
 * mu is the least-squares solution of C^T mu = -grad L_s (exact at the
 * minimiser); it is unique when the unit directions of the two objects
 * span space: det(sum of their outer products) > 1e-3 is required.
 * Returns -1 where this does not apply. */
static int grad_one_kkt(const path_t *p, const double *t, double gl,
                        const double *gx, double *g_tx, double *g_rx,
                        double *g_b, double *g_a, double S) {
  const int n = p->n, m = p->m;
  double x[NMAX + 2][3];
  points(p, t, x);
  double u[NMAX + 1][3], l[NMAX + 1];
  int z = -1, nz = 0;
  for (int i = 0; i <= n; ++i) {
    double r[3] = {x[i + 1][0] - x[i][0], x[i + 1][1] - x[i][1],
                   x[i + 1][2] - x[i][2]};
    l[i] = sqrt(dot3(r, r));
    if (!(l[i] > 1e-6 * S)) {
      z = i;
      ++nz;
    }
    for (int q = 0; q < 3; ++q) u[i][q] = r[q] / l[i];
  }
  if (nz != 1 || z < 1 || z > n - 1) return -1;
  double N3[3][3] = {{0}};
  for (int j = z - 1; j <= z; ++j)
    for (int k = 0; k < p->d[j]; ++k) {
      const double *a = p->a[j][k];
      double aa = dot3(a, a);
      for (int q = 0; q < 3; ++q)
        for (int r = 0; r < 3; ++r) N3[q][r] += a[q] * a[r] / aa;
    }
  double det = N3[0][0] * (N3[1][1] * N3[2][2] - N3[1][2] * N3[2][1]) -
               N3[0][1] * (N3[1][0] * N3[2][2] - N3[1][2] * N3[2][0]) +
               N3[0][2] * (N3[1][0] * N3[2][1] - N3[1][1] * N3[2][0]);
  if (!(det > 1e-3)) return -1;
  /* grad L_s, H_s and C */
  double gs[MMAX], Hs[MMAX][MMAX], C[3][MMAX];
  grad_hess_skip(p, t, 0.0, z, gs, Hs);
  for (int c = 0; c < m; ++c) {
    int j = p->cs[c];
    double sg = (j == z - 1) ? 1.0 : (j == z ? -1.0 : 0.0);
    for (int q = 0; q < 3; ++q) C[q][c] = sg * p->a[j][p->ck[c]][q];
  }
  /* mu from the normal equations C C^T mu = -C gs */
  double CC[3][3], rc[3], mu[3];
  for (int q = 0; q < 3; ++q) {
    rc[q] = 0.0;
    for (int c = 0; c < m; ++c) rc[q] -= C[q][c] * gs[c];
    for (int r = 0; r < 3; ++r) {
      CC[q][r] = 0.0;
      for (int c = 0; c < m; ++c) CC[q][r] += C[q][c] * C[r][c];
    }
  }
  if (gauss_solve_ld(3, 3, &CC[0][0], rc, mu) != 0) return -1;
  /* the KKT system */
  const int mk = m + 3;
  double Kk[KMAX][KMAX], rk[KMAX], sol[KMAX];
  for (int r = 0; r < mk; ++r)
    for (int c = 0; c < mk; ++c) Kk[r][c] = 0.0;
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < m; ++c) Kk[r][c] = Hs[r][c];
  for (int q = 0; q < 3; ++q)
    for (int c = 0; c < m; ++c) Kk[c][m + q] = Kk[m + q][c] = C[q][c];
  for (int c = 0; c < m; ++c)
    rk[c] = dot3(p->a[p->cs[c]][p->ck[c]], gx + 3 * p->cs[c]);
  for (int q = 0; q < 3; ++q) rk[m + q] = 0.0;
  if (gauss_solve_ld(mk, KMAX, &Kk[0][0], rk, sol) != 0) return -1;
  const double *lam = sol, *nu = sol + m;
  /* the closed forms of grad_one with u_z = -mu and c_z = 0 */
  for (int q = 0; q < 3; ++q) u[z][q] = -mu[q];
  double lamj[NMAX][2] = {{0}}, tj[NMAX][2] = {{0}};
  for (int c = 0; c < m; ++c) {
    lamj[p->cs[c]][p->ck[c]] = lam[c];
    tj[p->cs[c]][p->ck[c]] = t[c];
  }
  double qp[NMAX + 2][3] = {{0}}, cseg[NMAX + 1][3];
  for (int j = 0; j < n; ++j)
    for (int q = 0; q < 3; ++q)
      qp[j + 1][q] = lamj[j][0] * p->a[j][0][q] + lamj[j][1] * p->a[j][1][q];
  for (int i = 0; i <= n; ++i) {
    double dl[3] = {qp[i + 1][0] - qp[i][0], qp[i + 1][1] - qp[i][1],
                    qp[i + 1][2] - qp[i][2]};
    double ud = dot3(u[i], dl);
    for (int q = 0; q < 3; ++q)
      cseg[i][q] = (i == z) ? 0.0 : (dl[q] - u[i][q] * ud) / l[i];
  }
  for (int q = 0; q < 3; ++q) {
    g_tx[q] = -gl * u[0][q] + cseg[0][q];
    g_rx[q] = gl * u[n][q] - cseg[n][q];
  }
  for (int j = 0; j < n; ++j) {
    double du[3], gb[3];
    for (int q = 0; q < 3; ++q) {
      du[q] = u[j][q] - u[j + 1][q];
      gb[q] = gl * du[q] + gx[3 * j + q] - (cseg[j][q] - cseg[j + 1][q]);
      if (j == z - 1) gb[q] -= nu[q];
      if (j == z) gb[q] += nu[q];
      g_b[3 * j + q] = gb[q];
    }
    for (int k = 0; k < 2; ++k)
      for (int q = 0; q < 3; ++q)
        g_a[(j * 2 + k) * 3 + q] =
            (k < p->d[j]) ? tj[j][k] * gb[q] - lamj[j][k] * du[q] : 0.0;
  }
  return 0;
}

int oracle_grad(int64_t N, int n_max, const float *obj, int64_t K,
                const float *pts, int64_t Q, const int32_t *src,
                const int32_t *dst, const uint8_t *order, const int32_t *ids,
                double S, const double *t_sol, const double *g_len,
                const double *g_x, double *g_tx, double *g_rx, double *g_b,
                double *g_a, int32_t *status, int nthreads) {
  if (N < 0 || n_max < 1 || n_max > NMAX || S <= 0.0) return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t i = 0; i < N; ++i) {
    double *gtx = g_tx + 3 * i, *grx = g_rx + 3 * i;
    double *gb = g_b + i * n_max * 3, *ga = g_a + i * n_max * 6;
    for (int q = 0; q < 3; ++q) gtx[q] = grx[q] = NAN;
    for (int k = 0; k < n_max * 3; ++k) gb[k] = NAN;
    for (int k = 0; k < n_max * 6; ++k) ga[k] = NAN;
    path_t p;
    if (load_path(&p, i, N, n_max, obj, K, pts, Q, src, dst, order, ids)) {
      status[i] = ORACLE_INVALID;
      continue;
    }
    double t[MMAX];
    for (int c = 0; c < p.m; ++c)
      t[c] = t_sol[i * n_max * 2 + p.cs[c] * 2 + p.ck[c]];
    status[i] = 0;
    if (grad_one(&p, t, g_len[i], g_x + i * n_max * 3, gtx, grx, gb, ga, S)) {
      /* a collapsed minimiser: the constrained form, where it applies */
      status[i] = ORACLE_KKT;
      if (grad_one_kkt(&p, t, g_len[i], g_x + i * n_max * 3, gtx, grx, gb, ga,
                       S)) {
        status[i] = ORACLE_COLLAPSED;
        for (int q = 0; q < 3; ++q) gtx[q] = grx[q] = NAN;
        for (int k = 0; k < n_max * 3; ++k) gb[k] = NAN;
        for (int k = 0; k < n_max * 6; ++k) ga[k] = NAN;
      }
    }
  }
  return 0;
}

int oracle_length(int64_t N, int n_max, const float *obj, int64_t K,
                  const float *pts, int64_t Q, const int32_t *src,
                  const int32_t *dst, const uint8_t *order, const int32_t *ids,
                  const double *t_in, double *len_out) {
  if (N < 0 || n_max < 1 || n_max > NMAX) return -1;
  for (int64_t i = 0; i < N; ++i) {
    path_t p;
    if (load_path(&p, i, N, n_max, obj, K, pts, Q, src, dst, order, ids)) {
      len_out[i] = NAN;
      continue;
    }
    double t[MMAX];
    for (int c = 0; c < p.m; ++c)
      t[c] = t_in[i * n_max * 2 + p.cs[c] * 2 + p.ck[c]];
    len_out[i] = length_eps(&p, t, 0.0);
  }
  return 0;
}

/* ------------------------------------------------------------- validity -- */
/*
 * Post-processing of solved paths on finite objects (the step after the
 * solve that Sec. III names but does not study). A face is the
 * parallelogram b + s a1 + u a2, s, u in [0, 1]; an edge the segment
 * b + s a1, s in [0, 1]. For tolerance tol (may be negative):
 *   EXTENT   every interaction parameter lies in [-tol, 1 + tol]
 *   SPECULAR at every face, the previous and next points are on the same
 *            side: with d = n.(x_prev - x) / S and n the unit normal,
 *            both d_in, d_out > tol or both < -tol
 *   VISIBLE  no segment crosses a face of the scene other than the faces of
 *            its own end points: a crossing is a point of the segment at
 *            parameter s in (1e-6, 1 - 1e-6) on the face's plane with both
 *            face parameters in [tol, 1 - tol]; segments parallel to a face
 *            do not cross it; edges occlude nothing.
 * Points and parameters are the caller's (x [N][n_max][3], t
 * [N][n_max][2]); flags[i] gets the bits of the tests that pass.
 */
static int crosses_face(const double *p, const double *q, const double *b,
                        const double *u, const double *v, double tol) {
  double d[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
  double w[3] = {b[0] - p[0], b[1] - p[1], b[2] - p[2]};
  /* p + s d = b + al u + be v: Cramer's rule on [d, -u, -v] (s, al, be) = w */
  double m[3][3] = {{d[0], -u[0], -v[0]}, {d[1], -u[1], -v[1]}, {d[2], -u[2], -v[2]}};
  double det = m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) -
               m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
               m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
  double nd = sqrt(dot3(d, d));
  double nu = sqrt(dot3(u, u)), nv = sqrt(dot3(v, v));
  if (fabs(det) <= 1e-12 * nd * nu * nv) return 0;
  double sol[3];
  for (int k = 0; k < 3; ++k) {
    double mk[3][3];
    memcpy(mk, m, sizeof mk);
    for (int r = 0; r < 3; ++r) mk[r][k] = w[r];
    sol[k] = (mk[0][0] * (mk[1][1] * mk[2][2] - mk[1][2] * mk[2][1]) -
              mk[0][1] * (mk[1][0] * mk[2][2] - mk[1][2] * mk[2][0]) +
              mk[0][2] * (mk[1][0] * mk[2][1] - mk[1][1] * mk[2][0])) / det;
  }
  return sol[0] > 1e-6 && sol[0] < 1.0 - 1e-6 && sol[1] >= tol &&
         sol[1] <= 1.0 - tol && sol[2] >= tol && sol[2] <= 1.0 - tol;
}

int oracle_validate(int64_t N, int n_max, const float *obj, int64_t K,
                    const float *pts, int64_t Q, const int32_t *src,
                    const int32_t *dst, const uint8_t *order, const int32_t *ids,
                    double S, const double *t_in, const double *x_in,
                    double tol, uint8_t *flags, int nthreads) {
  if (N < 0 || n_max < 1 || n_max > NMAX || K < 0 || Q < 0 || !(S > 0)) return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    path_t p;
    if (load_path(&p, i, N, n_max, obj, K, pts, Q, src, dst, order, ids)) {
      flags[i] = 0;
      continue;
    }
    const int n = p.n;
    /* points x[0] = TX, x[1..n], x[n+1] = RX */
    double x[NMAX + 2][3];
    memcpy(x[0], p.x0, sizeof p.x0);
    memcpy(x[n + 1], p.xe, sizeof p.xe);
    for (int j = 0; j < n; ++j)
      for (int c = 0; c < 3; ++c) x[j + 1][c] = x_in[(i * n_max + j) * 3 + c];
    int extent = 1, specular = 1, visible = 1;
    for (int j = 0; j < n; ++j) {
      for (int k = 0; k < p.d[j]; ++k) {
        double tk = t_in[(i * n_max + j) * 2 + k];
        if (!(tk >= -tol && tk <= 1.0 + tol)) extent = 0;
      }
      if (p.d[j] == 2) {
        const double *u = p.a[j][0], *v = p.a[j][1];
        double nrm[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2],
                         u[0] * v[1] - u[1] * v[0]};
        double ln = sqrt(dot3(nrm, nrm));
        double din = 0.0, dout = 0.0;
        for (int c = 0; c < 3; ++c) {
          din += nrm[c] * (x[j][c] - x[j + 1][c]);
          dout += nrm[c] * (x[j + 2][c] - x[j + 1][c]);
        }
        din /= ln * S;
        dout /= ln * S;
        if (!((din > tol && dout > tol) || (din < -tol && dout < -tol))) specular = 0;
      }
    }
    for (int s = 0; s <= n && visible; ++s) {
      /* segment s from point s to point s + 1; own faces: slots s-1 and s */
      int64_t own0 = s >= 1 ? ids[(int64_t)(s - 1) * N + i] : -1;
      int64_t own1 = s < n ? ids[(int64_t)s * N + i] : -1;
      for (int64_t f = 0; f < K && visible; ++f) {
        if (f == own0 || f == own1) continue;
        double b[3], u[3], v[3];
        for (int c = 0; c < 3; ++c) {
          b[c] = obj[c * K + f];
          u[c] = obj[(3 + c) * K + f];
          v[c] = obj[(6 + c) * K + f];
        }
        if (v[0] == 0.0 && v[1] == 0.0 && v[2] == 0.0) continue;
        if (crosses_face(x[s], x[s + 1], b, u, v, tol)) visible = 0;
      }
    }
    flags[i] = (uint8_t)((extent ? ORACLE_EXTENT : 0) |
                         (specular ? ORACLE_SPECULAR : 0) |
                         (visible ? ORACLE_VISIBLE : 0));
  }
  return 0;
}
