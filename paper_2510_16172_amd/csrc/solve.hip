// Batched Fermat path solver for gfx950: one path per lane, the whole state
// of a path in VGPRs.
//
// Phase 1 (FP32): BFGS on L(T) (Sec. III-C) with the fixed-point step-size
// iteration of Eq. 6. The iteration is started at the unit step, and a
// step that does not shorten the path falls back to the first fixed-point
// iterate started at 0 (that one minimises a quadratic majorant of L along
// the direction, so it always shortens the path).
// Phase 2 (FP64): damped Newton steps on the length with every segment
// smoothed to sqrt(|r|^2 + eps^2), eps decreasing level by level, using the
// block-tridiagonal Hessian (2x2 blocks, Sec. III-D notes it is the Hessian
// of a convex function). The last full Newton step gives a certificate.
//
// Parametrisation (Sec. III-B, Eq. 3): x_j = b_j + t_j0 a1_j + t_j1 a2_j;
// an edge has a2 = 0 (padding). Slot j = 0..n-1 is interaction j+1;
// segment i = 0..n runs from point i-1 to point i (point -1 = TX,
// point n = RX), so slot j touches segments j (incoming) and j+1.
#include "common.h"
#include "path64.h"

namespace fpt {

template <int NO>
struct Geo32 {
  float tx[3], rx[3];
  float b[NO][3];
  float a[NO][2][3];  // basis vectors scaled to unit length (0 for padding)
};

// 1/|a| as the FP32 phase uses it (0 for the padding of an edge)
__device__ __forceinline__ void basis_inv32(const float* a1, const float* a2,
                                            bool edge, float& i1, float& i2) {
  float n1 = dot3(a1, a1), n2 = dot3(a2, a2);
  i1 = rsq32(n1 > 0.f ? n1 : 1.f);
  i2 = edge ? 0.f : rsq32(n2 > 0.f ? n2 : 1.f);
}

// Gradient of L at T (Sec. III-B Eq. 5): g_j = A_j^T (u_j - u_{j+1}).
// D parameters per slot: 2 (the padded layout; an edge's second parameter
// stays 0), or 1 for a path whose every interaction is an edge (Sec. III-B:
// the padding only serves a uniform layout).
template <int NO, int D = 2>
__device__ __forceinline__ void grad32(const Geo32<NO>& G, const float* T,
                                       float* g, float (*r)[3], float* l2,
                                       float* il) {
  float x[NO][3];
#pragma unroll
  for (int j = 0; j < NO; ++j)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      x[j][c] = D == 2 ? fmaf(T[2 * j + 1], G.a[j][1][c],
                              fmaf(T[2 * j], G.a[j][0][c], G.b[j][c]))
                       : fmaf(T[j], G.a[j][0][c], G.b[j][c]);
  float u[NO + 1][3];
#pragma unroll
  for (int i = 0; i <= NO; ++i) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float nx = (i == NO) ? G.rx[c] : x[i][c];
      float px = (i == 0) ? G.tx[c] : x[i - 1][c];
      r[i][c] = nx - px;
    }
    l2[i] = fmaxf(dot3(r[i], r[i]), 1e-30f);
    il[i] = rsq32(l2[i]);
#pragma unroll
    for (int c = 0; c < 3; ++c) u[i][c] = r[i][c] * il[i];
  }
#pragma unroll
  for (int j = 0; j < NO; ++j) {
    float du[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) du[c] = u[j][c] - u[j + 1][c];
    g[D * j] = dot3(G.a[j][0], du);
    if (D == 2) g[D * j + 1] = dot3(G.a[j][1], du);
  }
}

// packed upper-triangular index of (a, b), a <= b, of an m x m matrix
__host__ __device__ constexpr int pk(int m, int a, int b) {
  return a * m - a * (a - 1) / 2 + (b - a);
}

// y = H x for symmetric packed H
template <int M>
__device__ __forceinline__ void symv(const float* H, const float* x,
                                     float* y) {
#pragma unroll
  for (int a = 0; a < M; ++a) {
    float s = 0.f;
#pragma unroll
    for (int b = 0; b < M; ++b) {
      int ia = a < b ? a : b, ib = a < b ? b : a;
      s = fmaf(H[pk(M, ia, ib)], x[b], s);
    }
    y[a] = s;
  }
}

struct RefineOut {
  bool certified, refined, finite;
};

// Part A.sub of A.nsub equal parts of a launch's range of paths (the parts
// of one order run on separate streams, so that one part's latency-bound
// passes overlap the next part's BFGS).
__device__ __forceinline__ void sub_range(const SolveArgs& A, int64_t& begin,
                                          int64_t& count) {
  if (A.nsub > 1) {
    const int64_t lo = count * A.sub / A.nsub, hi = count * (A.sub + 1) / A.nsub;
    begin += lo;
    count = hi - lo;
  }
}

// ---------------------------------------------------------------- FP64 ----

// Reads path p's geometry in FP64 and the FP32 1/|a| factors that map the
// FP32 phase's unit-vector parameters back to the caller's parametrisation.
template <int NO>
__device__ __forceinline__ void load_geo64(const SolveArgs& A, int64_t p,
                                           Geo64<NO>& D, float (*inv)[2]) {
  load_geo64<NO>(A.obj, A.pts, A.ids, A.src[p], A.dst[p], A.K, A.Q, A.N, p, D);
#pragma unroll
  for (int j = 0; j < NO; ++j) {
    float a1[3], a2[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      a1[c] = (float)D.a(j, 0, c);
      a2[c] = (float)D.a(j, 1, c);
    }
    basis_inv32(a1, a2, D.edge(j), inv[j][0], inv[j][1]);
  }
}

// The same into this lane's LDS column (see GeoLds): the table values as
// they are (FP32), plus the edge flags and 1/|a| factors in registers.
template <int NO>
__device__ __forceinline__ void load_geo_lds(const SolveArgs& A, int64_t p,
                                             float* col, GeoLds<NO>& D,
                                             float (*inv)[2]) {
  int32_t s = A.src[p], e = A.dst[p];
  s = (s >= 0 && s < A.Q) ? s : 0;
  e = (e >= 0 && e < A.Q) ? e : 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    col[c * kBlock] = A.pts[(int64_t)c * A.Q + s];
    col[(3 + c) * kBlock] = A.pts[(int64_t)c * A.Q + e];
  }
#pragma unroll
  for (int j = 0; j < NO; ++j) {
    int32_t k = A.ids[(int64_t)j * A.N + p];
    k = (k >= 0 && k < A.K) ? k : 0;
    float bb[3], a1[3], a2[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      bb[c] = A.obj[(int64_t)c * A.K + k];
      a1[c] = A.obj[(int64_t)(3 + c) * A.K + k];
      a2[c] = A.obj[(int64_t)(6 + c) * A.K + k];
    }
    const bool edge = (a2[0] == 0.f) && (a2[1] == 0.f) && (a2[2] == 0.f);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      col[(6 + 9 * j + c) * kBlock] = bb[c];
      col[(9 + 9 * j + c) * kBlock] = a1[c];
      col[(12 + 9 * j + c) * kBlock] = edge ? 0.f : a2[c];
    }
    D.edge_[j] = edge;
    basis_inv32(a1, a2, edge, inv[j][0], inv[j][1]);
  }
  D.col = col;
}

template <class GEO, class R = typename GEO::real>
__device__ __forceinline__ R max_disp64(const GEO& G, const R* d) {
  constexpr int NO = GEO::kOrder;
  R m = R(0);
#pragma unroll
  for (int j = 0; j < NO; ++j) {
    R w[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      w[c] = d[2 * j] * G.a(j, 0, c) + d[2 * j + 1] * G.a(j, 1, c);
    m = fmax(m, dot3r(w, w));
  }
  return m;  // squared
}

// Newton run on the eps-smoothed length. The full step t + d is taken if it
// does not lengthen the smoothed path beyond the rounding of L itself. Else,
// with majorant = true, the step along d that minimises the quadratic
// majorant of the smoothed length, sum_i |r_i + a D_i|^2 / (2 l_i) (the
// iteration of Eq. 6 started at a = 0, which cannot lengthen the path), is
// tried: one evaluation, where near a collapsed minimiser a backtracking
// search from the (overshooting) Newton step takes many; with majorant =
// false the step is backtracked by factors of 4 (up to 6 times), which
// makes more progress per step on such paths. From two slots on a trial
// evaluates the length only and the segments of the next step are evaluated
// at the point reached; with one slot the accepted trial's segments are
// kept. prev_small / last_small track whether the last two steps were taken
// in full and moved no point by more than sqrt(cert2); contracting whether
// the last step was at most a tenth of the one before (the quadratic
// contraction of Newton's method near its solution; small steps that do
// not contract are a slow walk along a flat valley), or below 1e-4 sqrt(cert2).
// With stop = true the run ends at the first step (its second or later, so
// that both steps are taken at this smoothing) after which these three hold:
// the step conditions of the certificate, as they would stand had nsteps
// been that step count.
struct NewtonTrack {
  bool prev_small = false, last_small = false, refined = false, contracting = false;
  uint32_t n_eval = 0, n_trial = 0, n_solve = 0;  // evaluations, trial lengths, solves
  double last_d2 = INFINITY;  // squared largest displacement of the last step
};

// The (smoothed) length alone at t: a trial of the step. Same arithmetic as
// eval64's length, so an accepted trial and the segments evaluated after it
// agree bit for bit; keeping only the length through the trials keeps one
// set of segments live instead of two (fewer registers, more waves).
template <class GEO, class R = typename GEO::real>
__device__ __forceinline__ R length_at(const GEO& G, const R* t, R eps2) {
  constexpr int NO = GEO::kOrder;
  R x[NO][3];
  points64(G, t, x);
  R L = R(0);
#pragma unroll
  for (int i = 0; i <= NO; ++i) {
    R r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      r[c] = ((i == NO) ? G.rx(c) : x[i][c]) - ((i == 0) ? G.tx(c) : x[i - 1][c]);
    R q = fmax(dot3r(r, r) + eps2, RealTraits<R>::tiny);
    L += q * rsqr(q);
  }
  return L;
}

template <class GEO, class R = typename GEO::real>
__device__ __forceinline__ void newton_run64(const GEO& G, R* t, R eps2, int nsteps,
                                             R cert2, bool majorant, NewtonTrack& k,
                                             bool stop = false) {
  constexpr int NO = GEO::kOrder;
  Seg64<NO, R> cur;
  eval64(G, t, eps2, cur);
  ++k.n_eval;
  for (int st = 0; st < nsteps; ++st) {
    geo_fence();
    R d[2 * NO];
    const R bound = cur.L + RealTraits<R>::rel * fabs(cur.L);
    const bool ok = hess_solve64<true>(G, cur.v, cur.il, (const R*)nullptr, d);
    ++k.n_solve;
    k.prev_small = k.last_small;
    k.last_small = false;
    k.contracting = false;
    if (!ok) {
      k.last_d2 = 0.0;
      continue;
    }
    const R d2 = max_disp64(G, d);
    // majorant step: a = -sum D_i.v_i / sum |D_i|^2 il_i (v_i = r_i il_i),
    // D_i = A_i d_i - A_{i-1} d_{i-1} the change of segment i along d
    R num = R(0), den = R(0);
    {
      R qp[3] = {R(0), R(0), R(0)};
#pragma unroll
      for (int i = 0; i <= NO; ++i) {
        R qn[3], D[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          qn[c] = (i == NO) ? R(0) : fma(d[2 * i + 1], G.a(i, 1, c), d[2 * i] * G.a(i, 0, c));
          D[c] = qn[c] - qp[c];
          qp[c] = qn[c];
        }
        num += dot3r(D, cur.v[i]);
        den = fma(dot3r(D, D), cur.il[i], den);
      }
    }
    const R amm = (den > R(0)) ? -num * rcpr(den) : R(0);
    R s = R(1);
    bool acc = false;
    const int trials = majorant ? 2 : 7;
    for (int h = 0; h < trials; ++h) {
      geo_fence();
      R tn[2 * NO];
#pragma unroll
      for (int q = 0; q < 2 * NO; ++q) tn[q] = fma(s, d[q], t[q]);
      if constexpr (NO <= 1) {
        // (one slot: registers to spare, the trial keeps its segments)
        Seg64<NO, R> nx;
        eval64(G, tn, eps2, nx);
        ++k.n_eval;
        if (nx.L <= bound) {
#pragma unroll
          for (int q = 0; q < 2 * NO; ++q) t[q] = tn[q];
          cur = nx;
          acc = true;
          break;
        }
      } else {
        const R Ln = length_at(G, tn, eps2);
        ++k.n_trial;
        if (Ln <= bound) {
#pragma unroll
          for (int q = 0; q < 2 * NO; ++q) t[q] = tn[q];
          acc = true;
          break;
        }
      }
      if (majorant) {
        // (the majorant step cannot lengthen the path in exact arithmetic,
        // whatever its size)
        if (!(amm > R(0)) || !isfinite(amm) || amm == R(1)) break;
        s = amm;
      } else {
        s *= R(0.25);
      }
    }
    k.last_small = acc && (s == R(1)) && (d2 <= cert2);
    k.contracting = acc && (s == R(1)) &&
                    ((double)d2 <= 1e-2 * k.last_d2 || (double)d2 <= 1e-8 * (double)cert2);
    k.last_d2 = acc ? (double)(d2 * s * s) : 0.0;
    k.refined = k.refined || acc;
    if (stop && st >= 1 && k.prev_small && k.last_small && k.contracting) break;
    // (the segments at t are current unless a length-only trial moved t;
    // after the last step they are not needed: whatever follows evaluates
    // its own)
    if (NO > 1 && acc && st + 1 < nsteps) {
      geo_fence();
      eval64(G, t, eps2, cur);
      ++k.n_eval;
    }
  }
}

// ------------------------------------------------ collapsed minimisers ---
// At many minimisers two consecutive interaction points coincide (e.g. a
// reflection on a face at the edge that bounds it). The length is not
// differentiable there and the smoothed Newton iteration approaches such a
// point slowly, so refine64 does not certify it. The collapse step
// (merge_runs64 below) makes the two points a, b = a + 1 of a short interior
// segment one point on the intersection of their objects (a line, a point,
// or a plane for two coplanar planes), solves the reduced path by the same
// Newton iteration and certificate, and certifies the collapse as optimal if
// some w with |w| < 1 (|w|^2 <= 1 - 1e-6) satisfies the stationarity of both
// original points,
//   A_a^T (u_in - w) = 0,   A_b^T (w - u_out) = 0,
// where u_in, u_out are the unit vectors of the segments entering a and
// leaving b. Such a w is a subgradient of the zero-length segment's length,
// so 0 lies in the subdifferential of L; L is convex in T, so the point is a
// global minimiser (Sec. III-B, Eq. 5 as a sum of norms of affine maps).

__device__ __forceinline__ void cross3d(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// Orthonormal basis of an object's directions; n = unit normal of a plane.
struct Basis64 {
  double q[2][3], n[3];
  bool line;
};

__device__ __forceinline__ Basis64 basis64(const double (*a)[3], bool edge) {
  Basis64 B;
  double i0 = rsq64(dot3d(a[0], a[0]));
#pragma unroll
  for (int c = 0; c < 3; ++c) B.q[0][c] = a[0][c] * i0;
  double pr = dot3d(a[1], B.q[0]);
  double w[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) w[c] = a[1][c] - pr * B.q[0][c];
  double ww = dot3d(w, w);
  B.line = edge || !(ww > 0.0);
  double i1 = B.line ? 0.0 : rsq64(ww);
#pragma unroll
  for (int c = 0; c < 3; ++c) B.q[1][c] = w[c] * i1;
  cross3d(B.q[0], B.q[1], B.n);
  return B;
}

// The intersection of two objects near ymid: point y0 and an orthonormal
// basis e of its directions (dim 0, 1 or 2), and an orthonormal basis of the
// directions orthogonal to both objects (nnul of them: the common normal of
// two coplanar objects). False if they do not meet within tol of each other
// or the meeting point is further than sqrt(far2) from ymid.
struct Virt64 {
  double y0[3], e[2][3], nul[2][3];
  int dim, nnul;
};

__device__ __forceinline__ bool intersect64(const Basis64& U, const double* bu,
                                            const Basis64& V, const double* bv,
                                            const double* ymid, double tol,
                                            double far2, Virt64& X) {
  constexpr double kPar = 1e-12;  // sin^2 of the angle below which: parallel
#pragma unroll
  for (int c = 0; c < 3; ++c) X.e[0][c] = X.e[1][c] = X.nul[0][c] = X.nul[1][c] = 0.0;
  X.dim = -1;
  X.nnul = 0;
  if (!U.line && !V.line) {
    double d[3];
    cross3d(U.n, V.n, d);
    double dd = dot3d(d, d);
    if (dd > kPar) {
      // line: rows n_u, n_v, e of a 3x3 system (Cramer)
      double il = rsq64(dd), e[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) e[c] = d[c] * il;
      double h0 = dot3d(U.n, bu), h1 = dot3d(V.n, bv), h2 = dot3d(e, ymid);
      double c12[3], c20[3], c01[3];
      cross3d(V.n, e, c12);
      cross3d(e, U.n, c20);
      cross3d(U.n, V.n, c01);
      double det = dot3d(U.n, c12);
      double idet = rcp64(det);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        X.y0[c] = (h0 * c12[c] + h1 * c20[c] + h2 * c01[c]) * idet;
        X.e[0][c] = e[c];
      }
      X.dim = 1;
    } else {
      double g[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) g[c] = bv[c] - bu[c];
      if (!(fabs(dot3d(U.n, g)) < tol)) return false;
      double h = dot3d(U.n, ymid) - dot3d(U.n, bu);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        X.y0[c] = ymid[c] - h * U.n[c];
        X.e[0][c] = U.q[0][c];
        X.e[1][c] = U.q[1][c];
        X.nul[0][c] = U.n[c];
      }
      X.dim = 2;
      X.nnul = 1;
    }
  } else if (U.line != V.line) {
    const Basis64& P = U.line ? V : U;
    const Basis64& Lb = U.line ? U : V;
    const double* bp = U.line ? bv : bu;
    const double* bl = U.line ? bu : bv;
    double sn = dot3d(P.n, Lb.q[0]);
    double g[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) g[c] = bp[c] - bl[c];
    if (sn * sn > kPar) {
      double tt = dot3d(P.n, g) * rcp64(sn);
#pragma unroll
      for (int c = 0; c < 3; ++c) X.y0[c] = bl[c] + tt * Lb.q[0][c];
      X.dim = 0;
    } else {
      if (!(fabs(dot3d(P.n, g)) < tol)) return false;
      double m[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) m[c] = ymid[c] - bl[c];
      double tt = dot3d(Lb.q[0], m);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        X.y0[c] = bl[c] + tt * Lb.q[0][c];
        X.e[0][c] = Lb.q[0][c];
        X.nul[0][c] = P.n[c];
      }
      X.dim = 1;
      X.nnul = 1;
    }
  } else {
    double d[3], w0[3];
    cross3d(U.q[0], V.q[0], d);
#pragma unroll
    for (int c = 0; c < 3; ++c) w0[c] = bu[c] - bv[c];
    double dd = dot3d(d, d);
    if (dd > kPar) {
      // closest points of the two lines
      double cab = dot3d(U.q[0], V.q[0]);
      double du = dot3d(U.q[0], w0), dv = dot3d(V.q[0], w0);
      double iden = rcp64(1.0 - cab * cab);
      double su = (cab * dv - du) * iden, sv = (dv - cab * du) * iden;
      double pu[3], pv[3], g[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        pu[c] = bu[c] + su * U.q[0][c];
        pv[c] = bv[c] + sv * V.q[0][c];
        g[c] = pu[c] - pv[c];
      }
      if (!(dot3d(g, g) < tol * tol)) return false;
      double il = rsq64(dd);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        X.y0[c] = 0.5 * (pu[c] + pv[c]);
        X.nul[0][c] = d[c] * il;
      }
      X.dim = 0;
      X.nnul = 1;
    } else {
      double pr = dot3d(w0, U.q[0]), g[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) g[c] = w0[c] - pr * U.q[0][c];
      if (!(dot3d(g, g) < tol * tol)) return false;
      double m[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) m[c] = ymid[c] - bu[c];
      double tt = dot3d(U.q[0], m);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        X.y0[c] = bu[c] + tt * U.q[0][c];
        X.e[0][c] = U.q[0][c];
      }
      X.dim = 1;
      // two unit vectors orthogonal to the common line
      const double* q = U.q[0];
      double h[3] = {fabs(q[0]) < 0.6 ? 1.0 : 0.0, fabs(q[0]) < 0.6 ? 0.0 : 1.0, 0.0};
      double n0[3], n1[3];
      cross3d(q, h, n0);
      double i0 = rsq64(dot3d(n0, n0));
#pragma unroll
      for (int c = 0; c < 3; ++c) n0[c] *= i0;
      cross3d(q, n0, n1);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        X.nul[0][c] = n0[c];
        X.nul[1][c] = n1[c];
      }
      X.nnul = 2;
    }
  }
  // the meeting point must be near the two collapsing points
  double m[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) m[c] = ymid[c] - X.y0[c];
  double pe0 = dot3d(m, X.e[0]), pe1 = dot3d(m, X.e[1]);
  double dist2 = dot3d(m, m) - pe0 * pe0 - pe1 * pe1;
  return isfinite(dist2) && dist2 < far2;
}

// Parameters of point y on an object (caller's basis a, origin b).
__device__ __forceinline__ void coords64(const double (*a)[3], const double* b,
                                         bool edge, const double* y, double* t) {
  double m[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) m[c] = y[c] - b[c];
  double g00 = dot3d(a[0], a[0]), h0 = dot3d(a[0], m);
  if (edge) {
    t[0] = h0 * rcp64(g00);
    t[1] = 0.0;
    return;
  }
  double g01 = dot3d(a[0], a[1]), g11 = dot3d(a[1], a[1]), h1 = dot3d(a[1], m);
  double idet = rcp64(g00 * g11 - g01 * g01);
  t[0] = (g11 * h0 - g01 * h1) * idet;
  t[1] = (g00 * h1 - g01 * h0) * idet;
}

// The objects of slots a and a + 1 (selected without dynamic register
// indexing).
template <class GEO>
__device__ __forceinline__ void pair64(const GEO& G, int a,
                                       double (*aa)[3], double* ba, bool& ea,
                                       double (*ab)[3], double* bb, bool& eb) {
  constexpr int NO = GEO::kOrder;
#pragma unroll
  for (int j = 0; j + 1 < NO; ++j) {
    const bool s = (j == a);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      aa[0][c] = s ? G.a(j, 0, c) : aa[0][c];
      aa[1][c] = s ? G.a(j, 1, c) : aa[1][c];
      ba[c] = s ? G.b(j, c) : ba[c];
      ab[0][c] = s ? G.a(j + 1, 0, c) : ab[0][c];
      ab[1][c] = s ? G.a(j + 1, 1, c) : ab[1][c];
      bb[c] = s ? G.b(j + 1, c) : bb[c];
    }
    ea = s ? G.edge(j) : ea;
    eb = s ? G.edge(j + 1) : eb;
  }
}

// The subgradient test of a collapse between slots a and a + 1 (the two
// points coincide): u_in and u_out are the unit vectors of the segments into
// slot a and out of slot a + 1, nul an orthonormal basis of the directions
// orthogonal to both objects (zero rows beyond their number). The least-norm
// w with P_U w = P_U u_in and P_V w = P_V u_out (P = projector onto an
// object's directions) is w = (P_U + P_V + P_null)^-1 (P_U u_in + P_V u_out);
// it must satisfy both (residual, so that the path is stationary along the
// intersection too) and |w|^2 <= 1 - 1e-6. Then 0 is a subgradient of the
// length there: the point is the global minimiser (L is convex).
template <class GEO>
__device__ __forceinline__ bool subgradient_ok64(const GEO& G, int a, const double* uin,
                                                 const double* uout,
                                                 const double (*nul)[3]) {
  double aa[2][3] = {}, ab[2][3] = {}, ba[3] = {}, bb[3] = {};
  bool ea = false, eb = false;
  pair64(G, a, aa, ba, ea, ab, bb, eb);
  {
    const Basis64 U = basis64(aa, ea), V = basis64(ab, eb);
    double M[3][3], rhs[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      rhs[r] = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c)
        M[r][c] = nul[0][r] * nul[0][c] + nul[1][r] * nul[1][c];
    }
#pragma unroll
    for (int k2 = 0; k2 < 2; ++k2) {
      const double* qu = U.q[k2];
      const double* qv = V.q[k2];
      double pu = dot3d(qu, uin), pv = dot3d(qv, uout);
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        rhs[r] += qu[r] * pu + qv[r] * pv;
#pragma unroll
        for (int c = 0; c < 3; ++c) M[r][c] += qu[r] * qu[c] + qv[r] * qv[c];
      }
    }
    double C0[3], C1[3], C2[3];
    cross3d(M[1], M[2], C0);
    cross3d(M[2], M[0], C1);
    cross3d(M[0], M[1], C2);
    double idet = rcp64(dot3d(M[0], C0));
    double w[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      w[c] = (C0[c] * rhs[0] + C1[c] * rhs[1] + C2[c] * rhs[2]) * idet;
    // consistency (the reduced stationarity) and |w| < 1
    double res = 0.0;
#pragma unroll
    for (int k2 = 0; k2 < 2; ++k2) {
      double dd[3], ee[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        dd[c] = uin[c] - w[c];
        ee[c] = w[c] - uout[c];
      }
      double ru = dot3d(U.q[k2], dd), rv = dot3d(V.q[k2], ee);
      res += ru * ru + rv * rv;
    }
    if (!(res <= 1e-10) || !(dot3d(w, w) <= 1.0 - 1e-6)) return false;
  }
  return true;
}

// Nonsmooth check. At the smoothed optimum v_i = r_i / l_i plays the role of
// the subgradient of |r_i|: a genuine collapse (r_i -> 0) has |v_i| bounded
// away from 1, while a short segment (< 1e-3 S) with |v_i| close to 1 is a
// degenerate configuration in which the length is nearly flat along the
// segment and the smoothing can pull the points together. Such a path is not
// certified. An interior collapse (|v_i| <= 0.98) must also pass the exact
// subgradient test of its two objects: next to a collapse the smoothed
// length is curved like 1 / eps, so Newton steps are tiny there whether or
// not the point is stationary, and small steps alone prove nothing.
// nlast < NO: only segments 0..nlast are checked and nlast is the last one
// (a reduced path whose slots past nlast - 1 are fixed at RX); with
// allow_collapse false any collapse fails the check.
template <class GEO>
__device__ __forceinline__ bool nonsmooth_ok64(const GEO& G,
                                               const double* t, double eps,
                                               double scale, int nlast = GEO::kOrder,
                                               bool allow_collapse = true) {
  constexpr int NO = GEO::kOrder;
  const double short2 = 1e-6 * scale * scale;
  double x[NO][3];
  points64(G, t, x);
  bool ok = true;
  int ncol = 0, a = 0;
#pragma unroll
  for (int i = 0; i <= NO; ++i) {
    if (i > nlast) continue;
    double r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      r[c] = ((i == NO) ? G.rx(c) : x[i][c]) - ((i == 0) ? G.tx(c) : x[i - 1][c]);
    // |v_i|^2 = q / (q + eps^2) > 0.98^2
    double q = dot3d(r, r);
    const bool flat = q > (0.98 * 0.98) * (q + eps * eps);
    if (q < short2 && flat) ok = false;
    if (q < short2 && !flat && (i == 0 || i == nlast)) ok = false;
    if (q < short2 && !flat && i > 0 && i < nlast) {
      ++ncol;
      a = i - 1;
    }
  }
  if (!ok || ncol == 0) return ok;
  if (ncol > 1 || !allow_collapse) return false;
  if constexpr (NO < 2) {
    return false;
  } else {
    // the segments into slot a and out of slot a + 1, the collapse point
    double rin[3] = {0.0, 0.0, 0.0}, rout[3] = {0.0, 0.0, 0.0}, ymid[3] = {0.0, 0.0, 0.0};
    bool fixed = false;
#pragma unroll
    for (int k = 0; k + 1 < NO; ++k) {
      const bool sel = (k == a);
      fixed = fixed || (sel && (G.fixed(k) || G.fixed(k + 1)));
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double p0 = (k == 0) ? G.tx(c) : x[k > 0 ? k - 1 : 0][c];
        const double p3 = (k + 2 == NO) ? G.rx(c) : x[k + 2 < NO ? k + 2 : 0][c];
        rin[c] = sel ? x[k][c] - p0 : rin[c];
        rout[c] = sel ? p3 - x[k + 1][c] : rout[c];
        ymid[c] = sel ? 0.5 * (x[k][c] + x[k + 1][c]) : ymid[c];
      }
    }
    const double li = dot3d(rin, rin), lo = dot3d(rout, rout);
    if (fixed || !(li > 0.0) || !(lo > 0.0)) return false;
    double uin[3], uout[3];
    const double ii = rsq64(li), io = rsq64(lo);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      uin[c] = rin[c] * ii;
      uout[c] = rout[c] * io;
    }
    double aa[2][3] = {}, ab[2][3] = {}, ba[3] = {}, bb[3] = {};
    bool ea = false, eb = false;
    pair64(G, a, aa, ba, ea, ab, bb, eb);
    const Basis64 U = basis64(aa, ea), V = basis64(ab, eb);
    Virt64 X;
    if (!intersect64(U, ba, V, bb, ymid, 1e-6 * scale, 1.44e-2 * scale * scale, X))
      return false;
    return subgradient_ok64(G, a, uin, uout, X.nul);
  }
}

// Damped Newton refinement, level by level (quick: only the last level, with
// quick_steps steps). t is in the caller's parametrisation.
template <class GEO>
__device__ __forceinline__ RefineOut refine64(const GEO& G, double* t,
                                              const SolveArgs& A, bool quick,
                                              uint32_t (&work)[3]) {
  const double cert2 = (double)A.cert_abs * (double)A.cert_abs;
  NewtonTrack k;
  const int lv0 = quick ? A.n_levels - 1 : 0;
  for (int lv = lv0; lv < A.n_levels; ++lv) {
    double eps = (double)A.level_eps[lv] * (double)A.scale;
    // (the quick pass, which every path takes, uses the one-evaluation
    // majorant fallback; the paths left for the full schedule backtrack)
    newton_run64(G, t, eps * eps, quick ? A.quick_steps : A.level_steps[lv],
                 cert2, quick, k, lv == A.n_levels - 1);
  }
  work[0] += k.n_eval;
  work[1] += k.n_trial;
  work[2] += k.n_solve;
  RefineOut o{false, k.refined, true};
  // One small full step is not enough: along a nearly flat valley of the
  // length a Newton step taken from well outside its quadratic region can be
  // short and still leave the point far from the minimiser (the next step
  // then jumps, or the steps stay alike). Two consecutive small full steps
  // are required, the second contracting.
  o.certified = A.n_levels > 0 && k.prev_small && k.last_small && k.contracting;
  if (o.certified)
    o.certified = nonsmooth_ok64(
        G, t, (double)A.level_eps[A.n_levels - 1] * (double)A.scale, (double)A.scale);
  return o;
}

// ------------------------------------------- several collapsed segments ---
// merge_runs64 takes any number of collapses. Every
// interior segment shorter than short_rel * S is taken as collapsed, and
// each run of consecutive collapsed segments (at most two: three coinciding
// points) becomes one point on the intersection of the run's objects, found
// object by object (a plane, a line or a point; the run fails if they do not
// meet). The reduced path has NO minus the number of collapsed segments
// slots. It is held in a Geo64<NO - 1> whose unused trailing slots are
// points fixed at RX: the segments between them have zero length and no free
// parameter (the smoothed length gains a constant), so the Newton iteration,
// its certificate and the smoothness check run on it unchanged. Then every
// run must pass the subgradient test of run_subgradient64.

// An affine flat: origin o and orthonormal directions q (rows beyond dim are
// zero); dim 0 is a point, 1 a line, 2 a plane.
struct Flat64 {
  double o[3], q[2][3];
  int dim;
};

// The flat of slot j's object (j may be a run-time index: the geometry is
// read through the accessors, from LDS for a GeoLds). An edge has a zero
// second vector.
template <class GEO>
__device__ __forceinline__ Flat64 flat_of64(const GEO& G, int j) {
  double a[2][3];
  Flat64 F;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    a[0][c] = G.a(j, 0, c);
    a[1][c] = G.a(j, 1, c);
    F.o[c] = G.b(j, c);
  }
  const bool edge = a[1][0] == 0.0 && a[1][1] == 0.0 && a[1][2] == 0.0;
  const Basis64 B = basis64(a, edge);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    F.q[0][c] = B.q[0][c];
    F.q[1][c] = B.q[1][c];
  }
  F.dim = B.line ? 1 : 2;
  return F;
}

__device__ __forceinline__ Basis64 basis_of_flat(const Flat64& F) {
  Basis64 B;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    B.q[0][c] = F.q[0][c];
    B.q[1][c] = F.q[1][c];
  }
  cross3d(F.q[0], F.q[1], B.n);
  B.line = F.dim == 1;
  return B;
}

// The intersection X of two flats near ymid (see intersect64): false if they
// do not meet within tol, or meet further than sqrt(far2) from ymid. A point
// meets a flat if it lies on it within tol.
__device__ __forceinline__ bool meet64(const Flat64& U, const Flat64& V,
                                       const double* ymid, double tol, double far2,
                                       Flat64& X) {
  if (U.dim == 0 || V.dim == 0) {
    const bool up = U.dim == 0;
    double m[3], po[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      po[c] = up ? U.o[c] : V.o[c];
      m[c] = po[c] - (up ? V.o[c] : U.o[c]);
    }
    double d2 = dot3d(m, m);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      double qk[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) qk[c] = up ? V.q[k][c] : U.q[k][c];
      const double pk = dot3d(m, qk);
      d2 -= pk * pk;
    }
    if (!(d2 < tol * tol)) return false;
    double g[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      X.o[c] = po[c];
      X.q[0][c] = X.q[1][c] = 0.0;
      g[c] = ymid[c] - po[c];
    }
    X.dim = 0;
    return dot3d(g, g) < far2;
  }
  Virt64 W;
  if (!intersect64(basis_of_flat(U), U.o, basis_of_flat(V), V.o, ymid, tol, far2, W))
    return false;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    X.o[c] = W.y0[c];
    X.q[0][c] = W.e[0][c];
    X.q[1][c] = W.e[1][c];
  }
  X.dim = W.dim;
  return true;
}

// The subgradient test of a run of m = 2 or 3 coinciding points whose
// objects have the orthonormal bases Q_i (rows of F[i].q; an edge has one):
// the segments between them have zero length, u_in enters the first point
// and u_out leaves the last. Point i is stationary along its object if
//   Q_i^T (w_i - w_{i+1}) = 0,   w_0 = u_in,  w_m = u_out,
// for subgradients w_1 .. w_{m-1} of the zero-length segments. The least-norm
// solution is w_j = Q_j mu_j - Q_{j-1} mu_{j-1} with M mu = h, where
// M = C C^T of the constraint matrix C is block tridiagonal (I at the two
// ends of the diagonal, 2 I inside, -Q_i^T Q_{i+1} beside it),
// h_0 = -Q_0^T u_in and h_{m-1} = Q_{m-1}^T u_out. M is singular along
// nu_e = (Q_i^T e)_i for every direction e common to all the objects (E, the
// run's flat); adding nu_e nu_e^T for each leaves w unchanged and makes M
// positive definite. The run passes (0 is returned) if the w satisfy every
// equation (the reduced path is stationary along E) and each has
// |w_j|^2 <= 1 - 1e-6: then 0 is a subgradient of L at the point (L is convex
// in T), in the same way as subgradient_ok64 for a single collapse.
// Otherwise bit j - 1 is set for each w_j above that bound (the segment
// would open: moving the points apart shortens the path), and bit 2 if the
// equations are not met.
__device__ __forceinline__ unsigned run_subgradient64(const Flat64 (&F)[3], int m,
                                                      const double* uin, const double* uout,
                                                      const Flat64& E) {
  constexpr int NB = 6;
  double M[NB][NB], h[NB];
  bool act[3][2];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 2; ++k) act[i][k] = i < m && k < F[i].dim;
#pragma unroll
  for (int r = 0; r < NB; ++r) {
    h[r] = 0.0;
#pragma unroll
    for (int c = 0; c < NB; ++c) M[r][c] = 0.0;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double ci = (i == 0 || i == m - 1) ? 1.0 : 2.0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      M[2 * i + k][2 * i + k] = act[i][k] ? ci : 1.0;
      const double pin = dot3d(F[i].q[k], uin), pout = dot3d(F[i].q[k], uout);
      h[2 * i + k] = !act[i][k] ? 0.0 : (i == 0 ? -pin : (i == m - 1 ? pout : 0.0));
    }
    if (i + 1 < 3) {
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int l = 0; l < 2; ++l) {
          const double v = (act[i][k] && act[i + 1][l]) ? -dot3d(F[i].q[k], F[i + 1].q[l]) : 0.0;
          M[2 * i + k][2 * (i + 1) + l] = v;
          M[2 * (i + 1) + l][2 * i + k] = v;
        }
    }
  }
  // deflation along the common directions
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    if (e >= E.dim) continue;
    double nu[NB];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 2; ++k) nu[2 * i + k] = act[i][k] ? dot3d(F[i].q[k], E.q[e]) : 0.0;
#pragma unroll
    for (int r = 0; r < NB; ++r)
#pragma unroll
      for (int c = 0; c < NB; ++c) M[r][c] = fma(nu[r], nu[c], M[r][c]);
  }
  // Cholesky M = L L^T in place (lower triangle), then the two solves
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    double d = M[j][j];
#pragma unroll
    for (int p = 0; p < j; ++p) d -= M[j][p] * M[j][p];
    if (!(d > 1e-12)) return 4u;
    const double il = rsq64(d);
    M[j][j] = d * il;
#pragma unroll
    for (int r = j + 1; r < NB; ++r) {
      double v = M[r][j];
#pragma unroll
      for (int p = 0; p < j; ++p) v -= M[r][p] * M[j][p];
      M[r][j] = v * il;
    }
  }
  double mu[NB];
#pragma unroll
  for (int r = 0; r < NB; ++r) {
    double v = h[r];
#pragma unroll
    for (int p = 0; p < r; ++p) v -= M[r][p] * mu[p];
    mu[r] = v * rcp64(M[r][r]);
  }
#pragma unroll
  for (int r = NB - 1; r >= 0; --r) {
    double v = mu[r];
#pragma unroll
    for (int p = r + 1; p < NB; ++p) v -= M[p][r] * mu[p];
    mu[r] = v * rcp64(M[r][r]);
  }
  // w_j (j = 1, 2; w_0 = u_in, w_m = u_out), Q mu of each point
  double qm[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      qm[i][c] = (act[i][0] ? mu[2 * i] * F[i].q[0][c] : 0.0) +
                 (act[i][1] ? mu[2 * i + 1] * F[i].q[1][c] : 0.0);
  double w[4][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    w[0][c] = uin[c];
    w[1][c] = qm[1][c] - qm[0][c];
    w[2][c] = (m == 2) ? uout[c] : qm[2][c] - qm[1][c];
    w[3][c] = uout[c];
  }
  unsigned open = 0u;
  double res = 0.0;
#pragma unroll
  for (int j = 1; j <= 2; ++j)
    if (j < m && !(dot3d(w[j], w[j]) <= 1.0 - 1e-6)) open |= 1u << (j - 1);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    if (i >= m) continue;
    double dlt[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) dlt[c] = w[i][c] - w[i + 1][c];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const double rk = act[i][k] ? dot3d(F[i].q[k], dlt) : 0.0;
      res = fma(rk, rk, res);
    }
  }
  return open | (res <= 1e-10 ? 0u : 4u);
}

// Collapsed segments are taken as those shorter than kMergeShortQuick * S
// from the quick pass's point, and kMergeShortFull * S from the full
// schedule's output or a reduced solution.
constexpr double kMergeShortQuick = 6e-2, kMergeShortFull = 1e-3;

// Interior segments of the path at t shorter than sqrt(short2): bit i for
// segment i (slots i - 1 and i); *endshort if the first or last one is.
template <class GEO>
__device__ __forceinline__ unsigned short_segments64(const GEO& G, const double* t,
                                                     double short2, bool* endshort) {
  constexpr int NO = GEO::kOrder;
  double x[NO][3];
  points64(G, t, x);
  unsigned z = 0u;
  bool es = false;
#pragma unroll
  for (int i = 0; i <= NO; ++i) {
    double r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      r[c] = ((i == NO) ? G.rx(c) : x[i][c]) - ((i == 0) ? G.tx(c) : x[i - 1][c]);
    const bool sh = dot3d(r, r) < short2;
    if (i == 0 || i == NO)
      es = es || sh;
    else
      z |= sh ? (1u << i) : 0u;
  }
  *endshort = es;
  return z;
}

// Collapsed minimisers with one or more collapses (see above). t (caller's
// parametrisation) is the start point; on success it holds the certified
// minimiser. The collapsed set is found in rounds, as in an active-set
// method: the first merges the segments shorter than short_rel * S and
// solves the reduced path at the last smoothing level. If that is not
// certified, the next round changes the set and solves again after two
// smoothing levels (1e-4 S, 1e-6 S) from the reduced solution mapped back to
// the full path: a segment whose subgradient exceeds norm 1 is taken out (a
// short segment that is not collapsed: it is never merged again), and the
// segments now shorter than kMergeShortFull * S are added (a collapse the
// start point had not yet come near). At most `rounds` rounds. The geometry is read from LDS with run-time slot
// indices inside the loops over reduced slots, so that the intersection and
// the subgradient test are written once.
template <int NO>
__device__ __forceinline__ bool merge_runs64(const GeoLds<NO>& G, double* t,
                                             const SolveArgs& A, double short_rel,
                                             int rounds, uint32_t (&work)[3]) {
  if constexpr (NO < 2) {
    return false;
  } else {
    constexpr int NR = NO - 1;
    const double S = (double)A.scale;
    const double eps = (double)A.level_eps[A.n_levels - 1] * S;
    const double cert2 = (double)A.cert_abs * (double)A.cert_abs;
    bool endshort = false;
    unsigned z = short_segments64(G, t, short_rel * short_rel * S * S, &endshort);
    if (z == 0u || endshort) return false;
    unsigned opened = 0u;  // segments taken out of the set: never merged again
#pragma unroll 1
    for (int round = 0; round < rounds; ++round) {
      // at most three coinciding points in a run
      if (z == 0u || (z & (z >> 1) & (z >> 2)) != 0u) return false;
      const int nr = NO - __popc(z);
      double x[NO][3];
      points64(G, t, x);
      // reduced slot of every slot; first slot and size of every reduced slot
      int rs[NO], first[NR], cnt[NR];
#pragma unroll
      for (int q = 0; q < NR; ++q) first[q] = cnt[q] = 0;
#pragma unroll
      for (int j = 0; j < NO; ++j) {
        rs[j] = j - __popc(z & ((2u << j) - 2u));
#pragma unroll
        for (int q = 0; q < NR; ++q) {
          first[q] = (q == rs[j] && cnt[q] == 0) ? j : first[q];
          cnt[q] += (q == rs[j]) ? 1 : 0;
        }
      }
      // the reduced path: unused slots fixed at RX
      Geo64<NR> R;
      double tr[2 * NR];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        R.tx_[c] = G.tx(c);
        R.rx_[c] = G.rx(c);
      }
#pragma unroll
      for (int q = 0; q < NR; ++q) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          R.b_[q][c] = G.rx(c);
          R.a_[q][0][c] = R.a_[q][1][c] = 0.0;
        }
        R.edge_[q] = R.fixed_[q] = true;
        tr[2 * q] = tr[2 * q + 1] = 0.0;
      }
#pragma unroll 1
      for (int rr = 0; rr < nr; ++rr) {
        int js = 0, m = 0;
#pragma unroll
        for (int q = 0; q < NR; ++q) {
          js = (q == rr) ? first[q] : js;
          m = (q == rr) ? cnt[q] : m;
        }
        double ym[3] = {0.0, 0.0, 0.0}, t0 = 0.0, t1 = 0.0;
#pragma unroll
        for (int j = 0; j < NO; ++j) {
          const bool in = rs[j] == rr;
#pragma unroll
          for (int c = 0; c < 3; ++c) ym[c] += in ? x[j][c] : 0.0;
          t0 = (j == js) ? t[2 * j] : t0;
          t1 = (j == js) ? t[2 * j + 1] : t1;
        }
        const double im = (m == 3) ? (1.0 / 3.0) : (m == 2 ? 0.5 : 1.0);
#pragma unroll
        for (int c = 0; c < 3; ++c) ym[c] *= im;
        double nb[3], na[2][3], n0 = t0, n1 = t1;
        bool ne, nf = false;
        if (m == 1) {
          // the object itself, in the caller's basis
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            nb[c] = G.b(js, c);
            na[0][c] = G.a(js, 0, c);
            na[1][c] = G.a(js, 1, c);
          }
          ne = na[1][0] == 0.0 && na[1][1] == 0.0 && na[1][2] == 0.0;
        } else {
          Flat64 X;
          if (!meet64(flat_of64(G, js), flat_of64(G, js + 1), ym, 1e-6 * S, 1.44e-2 * S * S, X))
            return false;
          if (m == 3) {
            Flat64 X3;
            if (!meet64(X, flat_of64(G, js + 2), ym, 1e-6 * S, 1.44e-2 * S * S, X3))
              return false;
            X = X3;
          }
          double dm[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            nb[c] = X.o[c];
            na[0][c] = X.q[0][c];
            na[1][c] = X.q[1][c];
            dm[c] = ym[c] - X.o[c];
          }
          ne = X.dim < 2;
          nf = X.dim == 0;
          n0 = nf ? 0.0 : dot3d(dm, X.q[0]);
          n1 = ne ? 0.0 : dot3d(dm, X.q[1]);
        }
#pragma unroll
        for (int q = 0; q < NR; ++q) {
          const bool s = q == rr;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            R.b_[q][c] = s ? nb[c] : R.b_[q][c];
            R.a_[q][0][c] = s ? na[0][c] : R.a_[q][0][c];
            R.a_[q][1][c] = s ? (ne ? 0.0 : na[1][c]) : R.a_[q][1][c];
          }
          R.edge_[q] = s ? ne : R.edge_[q];
          R.fixed_[q] = s ? nf : R.fixed_[q];
          tr[2 * q] = s ? n0 : tr[2 * q];
          tr[2 * q + 1] = s ? n1 : tr[2 * q + 1];
        }
      }
      // solve the reduced path (after two smoothing levels in later rounds):
      // the smooth certificate, no collapse left
      if (round > 0) {
        NewtonTrack k0;
        newton_run64(R, tr, 1e-8 * S * S, 3, cert2, false, k0);
        newton_run64(R, tr, 1e-12 * S * S, 3, cert2, false, k0);
        work[0] += k0.n_eval;
        work[1] += k0.n_trial;
        work[2] += k0.n_solve;
      }
      NewtonTrack k;
      newton_run64(R, tr, eps * eps, 8, cert2, false, k, true);
      work[0] += k.n_eval;
      work[1] += k.n_trial;
      work[2] += k.n_solve;
      bool good = k.prev_small && k.last_small && k.contracting &&
                  nonsmooth_ok64(R, tr, eps, S, nr, false);
      unsigned open = 0u;  // collapsed segments whose subgradient is too long
      double xr[NR][3];
      points64(R, tr, xr);
      if (good) {
        // every run: the subgradient test against its own objects
        Seg64<NR> sg;
        eval64(R, tr, 0.0, sg);
        ++work[0];
#pragma unroll 1
        for (int rr = 0; rr < nr; ++rr) {
          int js = 0, m = 0;
#pragma unroll
          for (int q = 0; q < NR; ++q) {
            js = (q == rr) ? first[q] : js;
            m = (q == rr) ? cnt[q] : m;
          }
          if (m < 2) continue;
          double uin[3], uout[3];
          Flat64 E;
          E.dim = 0;
#pragma unroll
          for (int c = 0; c < 3; ++c) uin[c] = uout[c] = E.o[c] = E.q[0][c] = E.q[1][c] = 0.0;
#pragma unroll
          for (int q = 0; q < NR; ++q) {
            const bool s = q == rr;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              uin[c] = s ? sg.v[q][c] : uin[c];
              uout[c] = s ? sg.v[q + 1][c] : uout[c];
              E.q[0][c] = s ? R.a_[q][0][c] : E.q[0][c];
              E.q[1][c] = s ? R.a_[q][1][c] : E.q[1][c];
            }
            E.dim = s ? (R.fixed_[q] ? 0 : (R.edge_[q] ? 1 : 2)) : E.dim;
          }
          Flat64 F[3];
          F[0] = flat_of64(G, js);
          F[1] = flat_of64(G, js + 1);
          if (m == 3) {
            F[2] = flat_of64(G, js + 2);
          } else {
#pragma unroll
            for (int c = 0; c < 3; ++c) F[2].o[c] = F[2].q[0][c] = F[2].q[1][c] = 0.0;
            F[2].dim = 0;
          }
          const unsigned r = run_subgradient64(F, m, uin, uout, E);
          good = good && r == 0u;
          // (w_1, w_2 of the run belong to segments js + 1, js + 2)
          open |= (r & 3u) << (js + 1);
        }
      }
      // back to the caller's parameters of the full path
#pragma unroll
      for (int j = 0; j < NO; ++j) {
        int m = 0;
        double y[3] = {0.0, 0.0, 0.0}, p0 = 0.0, p1 = 0.0;
#pragma unroll
        for (int q = 0; q < NR; ++q) {
          const bool s = q == rs[j];
          m = s ? cnt[q] : m;
          p0 = s ? tr[2 * q] : p0;
          p1 = s ? tr[2 * q + 1] : p1;
#pragma unroll
          for (int c = 0; c < 3; ++c) y[c] = s ? xr[q][c] : y[c];
        }
        if (m >= 2) {
          double aj[2][3], bj[3], tj[2];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            aj[0][c] = G.a(j, 0, c);
            aj[1][c] = G.a(j, 1, c);
            bj[c] = G.b(j, c);
          }
          coords64(aj, bj, G.edge(j), y, tj);
          p0 = tj[0];
          p1 = tj[1];
        }
        t[2 * j] = p0;
        t[2 * j + 1] = p1;
      }
      if (good) return true;
      // segments that open leave the set; a collapse the start point had not
      // come near shows in the reduced solution as a short segment
      opened |= open;
      const unsigned z2 =
          (z | short_segments64(G, t, kMergeShortFull * kMergeShortFull * S * S, &endshort)) &
          ~opened;
      if (endshort || (z2 == z && round > 0)) return false;
      z = z2;
    }
    return false;
  }
}

// Final outputs of path p from the FP64 parameters td (caller's
// parametrisation): points, exact length, parameters, status (collapsed:
// set FPT_ST_COLLAPSED whatever the segment lengths).
template <class GEO>
__device__ __forceinline__ void write_path64(const SolveArgs& A,
                                             const GEO& D,
                                             const double* td, int64_t p,
                                             bool valid, bool certified,
                                             bool refined, bool collapsed = false) {
  constexpr int NO = GEO::kOrder;
  const float qnan = __builtin_nanf("");
  double xs[NO][3];
  points64(D, td, xs);
  double Lx = 0.0, minl2 = INFINITY;
#pragma unroll
  for (int i = 0; i <= NO; ++i) {
    double rr[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      rr[c] = ((i == NO) ? D.rx(c) : xs[i][c]) - ((i == 0) ? D.tx(c) : xs[i - 1][c]);
    double q2 = dot3d(rr, rr);
    minl2 = fmin(minl2, q2);
    Lx += (q2 > 0.0) ? q2 * rsq64(q2) : 0.0;
  }
  bool finite = isfinite(Lx);
#pragma unroll
  for (int k = 0; k < 2 * NO; ++k) finite = finite && isfinite(td[k]);
  uint8_t st = 0;
  if (!valid) {
    st = FPT_ST_INVALID;
  } else {
    double cs = 1e-6 * (double)A.scale;
    if (certified && finite) st |= FPT_ST_CONVERGED;
    if (refined) st |= FPT_ST_REFINED;
    if (minl2 < cs * cs || collapsed) st |= FPT_ST_COLLAPSED;
    if (!finite) st |= FPT_ST_NONFINITE;
  }
  // no implicit gradient: invalid, non-finite, or a collapse it does not
  // cover (single_collapse)
  if ((st & (FPT_ST_NONFINITE | FPT_ST_INVALID)) ||
      ((st & FPT_ST_COLLAPSED) && single_collapse(D, xs, 1e-12 * (double)A.scale * (double)A.scale) < 0))
    st |= FPT_ST_NOGRAD;
#pragma unroll
  for (int j = 0; j < NO; ++j) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
      A.x[(int64_t)(3 * j + c) * A.N + p] = valid ? (float)xs[j][c] : qnan;
    A.t[(int64_t)(2 * j) * A.N + p] = valid ? (float)td[2 * j] : qnan;
    A.t[(int64_t)(2 * j + 1) * A.N + p] = valid ? (float)td[2 * j + 1] : qnan;
  }
  for (int j = NO; j < (A.pad_outputs ? A.n_max : 0); ++j) {
#pragma unroll
    for (int c = 0; c < 3; ++c) A.x[(int64_t)(3 * j + c) * A.N + p] = qnan;
    A.t[(int64_t)(2 * j) * A.N + p] = qnan;
    A.t[(int64_t)(2 * j + 1) * A.N + p] = qnan;
  }
  A.len[p] = valid ? (float)Lx : qnan;
  A.status[p] = st;
}

// ------------------------------------------------------------- kernel -----

// Highest order whose refinement passes keep the FP64 geometry in registers.
constexpr int kRegGeoMax = 2;

// Per-lane FP32 state of the BFGS iteration (D parameters per slot).
template <int NO, int D = 2>
struct State32 {
  static constexpr int M = D * NO;
  static constexpr int HP = M * (M + 1) / 2;
  float T[M], g[M], P[M], H[HP];    // parameters, gradient, direction, H
  float r[NO + 1][3], l2[NO + 1], il[NO + 1];  // segments at T
};

// Gathers path p: endpoints, objects (basis scaled to unit length), and the
// start point (t_init mapped to unit-vector coordinates, or 0). Returns
// false for an invalid path (its state is still finite and harmless).
template <int NO>
__device__ __forceinline__ bool load_path32(const SolveArgs& A, int64_t p,
                                            Geo32<NO>& G, float (*t0)[2]) {
  bool valid = true;
  // (in bucket order, the first phase reads the caller's arrays through the
  // permutation and leaves copies of the indices at slot p)
  const bool gather = A.perm_in != nullptr;
  const int64_t q = gather ? (int64_t)A.perm_in[p] : p;
  const int32_t* __restrict__ srcv = gather ? A.src_in : A.src;
  const int32_t* __restrict__ dstv = gather ? A.dst_in : A.dst;
  const int32_t* __restrict__ idsv = gather ? A.ids_in : A.ids;
  const float* __restrict__ tin = gather ? A.tinit_in : A.t_init;
  int32_t s = srcv[q], e = dstv[q];
  if (gather) {
    A.src_cp[p] = s;
    A.dst_cp[p] = e;
  }
  valid = valid && s >= 0 && s < A.Q && e >= 0 && e < A.Q;
  s = valid ? s : 0;
  e = valid ? e : 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    G.tx[c] = A.pts[(int64_t)c * A.Q + s];
    G.rx[c] = A.pts[(int64_t)c * A.Q + e];
    valid = valid && isfinite(G.tx[c]) && isfinite(G.rx[c]);
  }
#pragma unroll
  for (int j = 0; j < NO; ++j) {
    int32_t k = idsv[(int64_t)j * A.N + q];
    if (gather) A.ids_cp[(int64_t)j * A.N + p] = k;
    bool kok = k >= 0 && k < A.K;
    valid = valid && kok;
    k = kok ? k : 0;
    float bb[3], a1[3], a2[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      bb[c] = A.obj[(int64_t)c * A.K + k];
      a1[c] = A.obj[(int64_t)(3 + c) * A.K + k];
      a2[c] = A.obj[(int64_t)(6 + c) * A.K + k];
      valid = valid && isfinite(bb[c]) && isfinite(a1[c]) && isfinite(a2[c]);
    }
    bool edge = (a2[0] == 0.f) && (a2[1] == 0.f) && (a2[2] == 0.f);
    valid = valid && dot3(a1, a1) > 0.f && (edge || dot3(a2, a2) > 0.f);
    float i1, i2;
    basis_inv32(a1, a2, edge, i1, i2);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      G.b[j][c] = bb[c];
      G.a[j][0][c] = a1[c] * i1;
      G.a[j][1][c] = a2[c] * i2;
    }
    float u0 = 0.f, u1 = 0.f;
    if (tin) {
      // to unit-vector coordinates: that = t * |a|
      u0 = tin[(int64_t)(2 * j) * A.N + q] * rcp32(i1);
      u1 = edge ? 0.f : tin[(int64_t)(2 * j + 1) * A.N + q] * rcp32(i2);
      if (!isfinite(u0)) u0 = 0.f;
      if (!isfinite(u1)) u1 = 0.f;
    }
    t0[j][0] = u0;
    t0[j][1] = u1;
  }
  if (A.order) valid = valid && (int)A.order[p] == NO;
  return valid;
}

template <int M, int HP>
__device__ __forceinline__ void set_identity(float* H) {
#pragma unroll
  for (int a = 0; a < M; ++a)
#pragma unroll
    for (int b = a; b < M; ++b) H[pk(M, a, b)] = (a == b) ? 1.f : 0.f;
}

// T = t0, H = I, gradient and first direction P = -g.
template <int NO, int D = 2>
__device__ __forceinline__ void init_state(const Geo32<NO>& G,
                                           const float (*t0)[2],
                                           State32<NO, D>& S) {
  constexpr int M = State32<NO, D>::M, HP = State32<NO, D>::HP;
#pragma unroll
  for (int j = 0; j < NO; ++j) {
    S.T[D * j] = t0[j][0];
    if (D == 2) S.T[D * j + 1] = t0[j][1];
  }
  set_identity<M, HP>(S.H);
  grad32<NO, D>(G, S.T, S.g, S.r, S.l2, S.il);
#pragma unroll
  for (int k = 0; k < M; ++k) S.P[k] = -S.g[k];
}

// The line-search variant (fpt_opts.line_search): Armijo's sufficient
// decrease constant and the number of halvings before the majorant step.
constexpr float kArmijoC1 = 1e-4f;
constexpr int kArmijoHalvings = 8;

// One BFGS iteration (Sec. III-C): step size by the fixed-point iteration of
// Eq. 6 (from the unit step, with the majorant step from 0 as fallback),
// step, new gradient, inverse-Hessian update. On the first iteration the
// identity is rescaled to (s^T y / y^T y) I before the update (the usual
// choice of the initial inverse Hessian, Nocedal & Wright eq. 6.20): H = I
// is off by the scale of the segment lengths. Returns the squared largest
// point displacement of the step.
template <int NO, int D = 2, int LS = FPT_LS_EQ6>
__device__ __forceinline__ float bfgs_iter(const Geo32<NO>& G, State32<NO, D>& S,
                                           int fp_iters, bool first) {
  constexpr int M = State32<NO, D>::M, HP = State32<NO, D>::HP;
  // direction in point space: q_j = A_j p_j; segment change D_i
  float q[NO][3];
#pragma unroll
  for (int j = 0; j < NO; ++j)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      q[j][c] = D == 2 ? fmaf(S.P[2 * j + 1], G.a[j][1][c], S.P[2 * j] * G.a[j][0][c])
                       : S.P[j] * G.a[j][0][c];
  float dr[NO + 1], dd[NO + 1];
  float num0 = 0.f, den0 = 0.f, phi0 = 0.f;
#pragma unroll
  for (int i = 0; i <= NO; ++i) {
    float Dv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      Dv[c] = ((i == NO) ? 0.f : q[i][c]) - ((i == 0) ? 0.f : q[i - 1][c]);
    dr[i] = dot3(Dv, S.r[i]);
    dd[i] = dot3(Dv, Dv);
    num0 = fmaf(dr[i], S.il[i], num0);
    den0 = fmaf(dd[i], S.il[i], den0);
    phi0 = fmaf(S.l2[i], S.il[i], phi0);
  }
  // Eq. 6 started at alpha = 0: one step is the majorant minimiser
  float a_mm = (den0 > 1e-30f) ? -num0 * rcp32(den0) : 0.f;
  if (!isfinite(a_mm)) a_mm = 0.f;
  float alpha = 1.f;
  if constexpr (LS == FPT_LS_ARMIJO) {
    // backtracking from the unit step: the length along the direction,
    // sum_i |r_i + a D_i|, needs one rsq per segment and trial; its slope at
    // 0 is num0 (= g.P)
    bool ok = false;
#pragma unroll 1
    for (int h = 0; h <= kArmijoHalvings && !ok; ++h) {
      if (h > 0) alpha *= 0.5f;
      float phi = 0.f;
#pragma unroll
      for (int i = 0; i <= NO; ++i) {
        const float rho2 = fmaxf(fmaf(alpha, fmaf(alpha, dd[i], 2.f * dr[i]), S.l2[i]), 1e-30f);
        phi = fmaf(rho2, rsq32(rho2), phi);
      }
      ok = phi <= fmaf(kArmijoC1 * alpha, num0, phi0);
    }
    if (!ok || !isfinite(alpha)) alpha = a_mm;
  } else {
  // Eq. 6 iterated from the unit step
  for (int f = 0; f < fp_iters; ++f) {
    float num = 0.f, den = 0.f;
#pragma unroll
    for (int i = 0; i <= NO; ++i) {
      float rho2 = fmaxf(fmaf(alpha, fmaf(alpha, dd[i], 2.f * dr[i]), S.l2[i]), 1e-30f);
      float ir = rsq32(rho2);
      num = fmaf(dr[i], ir, num);
      den = fmaf(dd[i], ir, den);
    }
    alpha = (den > 1e-30f) ? -num * rcp32(den) : 0.f;
  }
  // keep it only if it shortens the path
  float phi = 0.f;
#pragma unroll
  for (int i = 0; i <= NO; ++i) {
    float rho2 = fmaxf(fmaf(alpha, fmaf(alpha, dd[i], 2.f * dr[i]), S.l2[i]), 1e-30f);
    phi = fmaf(rho2, rsq32(rho2), phi);
  }
  if (!(phi < phi0) || !(alpha > 0.f) || !isfinite(alpha)) alpha = a_mm;
  }
  // step, new gradient
  float s[M], gn[M];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    s[k] = alpha * S.P[k];
    S.T[k] += s[k];
  }
  grad32<NO, D>(G, S.T, gn, S.r, S.l2, S.il);
  // BFGS inverse update (Nocedal & Wright eq. 6.17), with
  // H y = H g' - H g = H g' + P
  float Hg[M], Hy[M], y[M];
  if (first) {
    // H = I still: scale it, and the direction P = -H g with it
    float sy0 = 0.f, yy0 = 0.f;
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const float yk = gn[k] - S.g[k];
      sy0 = fmaf(s[k], yk, sy0);
      yy0 = fmaf(yk, yk, yy0);
    }
    const float gam = (sy0 > 1e-30f && yy0 > 1e-30f) ? sy0 * rcp32(yy0) : 1.f;
#pragma unroll
    for (int a = 0; a < M; ++a) S.H[pk(M, a, a)] *= gam;
#pragma unroll
    for (int k = 0; k < M; ++k) S.P[k] *= gam;
  }
  symv<M>(S.H, gn, Hg);
  float sy = 0.f, yHy = 0.f, ss = 0.f, yy = 0.f;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    y[k] = gn[k] - S.g[k];
    Hy[k] = Hg[k] + S.P[k];
    sy = fmaf(s[k], y[k], sy);
    yHy = fmaf(y[k], Hy[k], yHy);
    ss = fmaf(s[k], s[k], ss);
    yy = fmaf(y[k], y[k], yy);
  }
  bool upd = (sy > 1e-30f) && (sy * sy > 1e-12f * ss * yy) && isfinite(yHy);
  float rho = upd ? rcp32(sy) : 0.f;
  float c1 = rho * fmaf(rho, yHy, 1.f);
  float w[M], v[M];
  float wg = 0.f, sg = 0.f;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    v[k] = -rho * Hy[k];
    w[k] = fmaf(c1, s[k], v[k]);
    wg = fmaf(w[k], gn[k], wg);
    sg = fmaf(s[k], gn[k], sg);
  }
#pragma unroll
  for (int a = 0; a < M; ++a)
#pragma unroll
    for (int b = a; b < M; ++b)
      S.H[pk(M, a, b)] = fmaf(v[a], s[b], fmaf(s[a], w[b], S.H[pk(M, a, b)]));
  float pp = 0.f;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    S.P[k] = -fmaf(v[k], sg, fmaf(s[k], wg, Hg[k]));
    S.g[k] = gn[k];
    pp = fmaf(S.P[k], S.P[k], pp);
  }
  if (!(pp < 1e30f)) {
    // overflow or NaN in the update: restart from the identity
    set_identity<M, HP>(S.H);
#pragma unroll
    for (int k = 0; k < M; ++k) S.P[k] = -S.g[k];
  }
  float m2 = 0.f;
#pragma unroll
  for (int j = 0; j < NO; ++j) m2 = fmaxf(m2, dot3(q[j], q[j]));
  return alpha * alpha * m2;
}

template <int NO>
struct Geo32View {
  static constexpr int kOrder = NO;
  using real = float;
  const Geo32<NO>& g;
  bool edge_[NO];
  __device__ __forceinline__ float tx(int c) const { return g.tx[c]; }
  __device__ __forceinline__ float rx(int c) const { return g.rx[c]; }
  __device__ __forceinline__ float b(int j, int c) const { return g.b[j][c]; }
  __device__ __forceinline__ float a(int j, int k, int c) const { return g.a[j][k][c]; }
  __device__ __forceinline__ bool edge(int j) const { return edge_[j]; }
  __device__ __forceinline__ bool fixed(int) const { return false; }
};

// The end of the FP32 phase: `polish_steps` Newton steps in FP32 on the
// exact block-tridiagonal Hessian of the length (smoothed by 1e-7 S, the
// majorant step when the full one lengthens the path). The first FP64
// refinement step then starts within FP32 precision of the minimiser, so
// that fewer FP64 steps reach the certificate. A step that is not finite is
// dropped.
constexpr float kPolishEps = 1e-7f;

template <int NO>
__device__ __forceinline__ void polish32(const SolveArgs& A, const Geo32<NO>& G,
                                         float* ST) {
  if (A.polish_steps <= 0) return;
  Geo32View<NO> V{G, {}};
  float T[2 * NO];
#pragma unroll
  for (int j = 0; j < NO; ++j)
    V.edge_[j] = G.a[j][1][0] == 0.f && G.a[j][1][1] == 0.f && G.a[j][1][2] == 0.f;
#pragma unroll
  for (int q = 0; q < 2 * NO; ++q) T[q] = ST[q];
  NewtonTrack k;
  const float eps = kPolishEps * A.scale;
  newton_run64(V, T, eps * eps, A.polish_steps, 0.f, true, k);
  bool fin = true;
#pragma unroll
  for (int q = 0; q < 2 * NO; ++q) fin = fin && isfinite(T[q]);
#pragma unroll
  for (int q = 0; q < 2 * NO; ++q) ST[q] = fin ? T[q] : ST[q];
}

// hands a path over to the refinement kernel: unit-vector parameters,
// iteration count, validity
template <int NO>
__device__ __forceinline__ void store_phase1(const SolveArgs& A, int64_t p,
                                             const float* ST, int it, bool valid) {
#pragma unroll
  for (int k = 0; k < 2 * NO; ++k) A.t[(int64_t)k * A.N + p] = ST[k];
  A.iters[p] = (uint16_t)(it > 65535 ? 65535 : it);
  A.status[p] = valid ? 0 : FPT_ST_INVALID;
}

// The BFGS iterations of one path with D parameters per slot and step rule
// LS, from t0; the result in the padded layout (an edge's second parameter 0).
template <int NO, int D, int LS = FPT_LS_EQ6>
__device__ __forceinline__ void bfgs_run(const SolveArgs& A, const Geo32<NO>& G,
                                         const float (*t0)[2], float* T) {
  State32<NO, D> S;
  init_state<NO, D>(G, t0, S);
  for (int it = 0; it < A.n_iter; ++it) bfgs_iter<NO, D, LS>(G, S, A.fp_iters, it == 0);
#pragma unroll
  for (int j = 0; j < NO; ++j) {
    T[2 * j] = S.T[D * j];
    T[2 * j + 1] = D == 2 ? S.T[D * j + 1] : 0.f;
  }
}

// Phase 1, fixed iteration count (Sec. III-C runs every path for the same
// number of iterations so that all lanes finish together). Up to order
// kUnpaddedMax, a wave whose paths all have only edges runs the BFGS on n
// parameters instead of the padded 2n (Sec. III-B): the padded rows of H
// stay exactly 0 in the padded iteration, so both compute the same iterates
// (they agree to FP32 rounding), and the unpadded one skips the padded
// rows' arithmetic. The test is one ballot on the loaded geometry, so it
// costs nothing where such waves are rare (paths in random order) and pays
// where edge-only paths come in runs (candidates enumerated in order of
// their objects, as the enumeration kernel writes them). Putting the
// edge-only paths of each 256 first in a workgroup, by a partition through
// LDS, made every wave pay for a second read of the object indices and
// three barriers, and it was slower on paths in random order. From order 3
// on the unpadded code path would cost the kernel a wave per SIMD.
constexpr int kUnpaddedMax = 2;

// (LS: the step rule. The line-search variant is an instantiation of its
// own, so that its code costs the default kernel no registers. Six slots:
// asked for two waves per SIMD, the kernel spills 28 bytes where it took
// six AGPRs beyond 256 registers and one wave, and runs 24 % faster; five
// slots at three waves would spill 200 bytes and took twice as long.)
template <int NO, int LS = FPT_LS_EQ6>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(NO == 6 ? 2 : 1)))
void bfgs_kernel(
    SolveArgs A, const int32_t* __restrict__ perm,
    const int64_t* __restrict__ bucket) {
  clear_counters(A);
  int64_t begin = 0, count = A.N;
  if (bucket) {
    begin = bucket[NO - 1];
    count = bucket[NO] - begin;
  }
  sub_range(A, begin, count);
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < count;
       idx += stride) {
    const int64_t p = perm ? (int64_t)perm[begin + idx] : begin + idx;
    Geo32<NO> G;
    float t0[NO][2], T[2 * NO];
    bool valid = load_path32<NO>(A, p, G, t0);
    bool unpadded = false;
    if constexpr (NO <= kUnpaddedMax && LS == FPT_LS_EQ6) {
      bool e = true;
#pragma unroll
      for (int j = 0; j < NO; ++j)
        e = e && G.a[j][1][0] == 0.f && G.a[j][1][1] == 0.f && G.a[j][1][2] == 0.f;
      unpadded = __ballot(e) == __ballot(true);
    }
    if (unpadded)
      bfgs_run<NO, 1, LS>(A, G, t0, T);
    else
      bfgs_run<NO, 2, LS>(A, G, t0, T);
    polish32<NO>(A, G, T);
    store_phase1<NO>(A, p, T, A.n_iter, valid);
  }
}

// ---------------------------------------- exact-Hessian Newton, FP32 ----
// A solver variant for the first phase: damped Newton in FP32 on the exact
// Hessian of the smoothed length (the block-tridiagonal solve of path64.h
// over the path's FP32 registers), from the same start as the BFGS
// (unit-length basis, T = 0 or t_init). `n_iter` steps are split evenly over
// four smoothing levels, the remainder going to the last; a step that would
// lengthen the path is replaced by the majorant step along the Newton
// direction. The FP64 refinement that follows is unchanged.
constexpr int kNewton32Levels = 4;
__device__ __forceinline__ float newton32_eps(int lv) {
  return lv == 0 ? 1e-2f : lv == 1 ? 1e-3f : lv == 2 ? 1e-4f : 1e-5f;
}

template <int NO>
__global__ __launch_bounds__(kBlock) void newton32_kernel(
    SolveArgs A, const int32_t* __restrict__ perm,
    const int64_t* __restrict__ bucket) {
  clear_counters(A);
  int64_t begin = 0, count = A.N;
  if (bucket) {
    begin = bucket[NO - 1];
    count = bucket[NO] - begin;
  }
  sub_range(A, begin, count);
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < count;
       idx += stride) {
    const int64_t p = perm ? (int64_t)perm[begin + idx] : begin + idx;
    Geo32<NO> G;
    float t0[NO][2];
    const bool valid = load_path32<NO>(A, p, G, t0);
    Geo32View<NO> V{G, {}};
    float T[2 * NO];
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      V.edge_[j] = G.a[j][1][0] == 0.f && G.a[j][1][1] == 0.f && G.a[j][1][2] == 0.f;
      T[2 * j] = t0[j][0];
      T[2 * j + 1] = V.edge_[j] ? 0.f : t0[j][1];
    }
    NewtonTrack k;
    const int per = A.n_iter / kNewton32Levels;
    for (int lv = 0; lv < kNewton32Levels; ++lv) {
      const int steps = per + (lv == kNewton32Levels - 1 ? A.n_iter - kNewton32Levels * per : 0);
      if (steps == 0) continue;
      const float eps = newton32_eps(lv) * A.scale;
      newton_run64(V, T, eps * eps, steps, 0.f, true, k);
    }
#pragma unroll
    for (int q = 0; q < 2 * NO; ++q) A.t[(int64_t)q * A.N + p] = isfinite(T[q]) ? T[q] : 0.f;
    A.iters[p] = (uint16_t)(A.n_iter > 65535 ? 65535 : A.n_iter);
    A.status[p] = valid ? 0 : FPT_ST_INVALID;
  }
}

// Phase 1 with early exit, in stages. A stage runs every path of its input
// for at most `iters` more iterations, all lanes of a wavefront in lockstep.
// A path leaves once two consecutive steps moved no point by more than
// exit_rtol * scale, or after n_iter iterations in total; the others are
// appended to a compact list for the next stage, together with their BFGS
// state (T, P, packed H, iteration count, streak), so that the next stage
// runs dense wavefronts again. The first stage reads the order bucket, the
// following ones the previous stage's list (its length is read on the
// device); the last stage hands over every path. The state is stored as
// structure-of-arrays over list slots: [field][cap].

template <int NO>
constexpr int stage_fields() {
  return 4 * NO + (2 * NO) * (2 * NO + 1) / 2 + 2;
}

template <int NO>
__global__ __launch_bounds__(kBlock) void bfgs_stage_kernel(
    SolveArgs A, const int32_t* __restrict__ perm,
    const int64_t* __restrict__ bucket, StageArgs St) {
  constexpr int M = 2 * NO, HP = M * (M + 1) / 2;
  // input: the bucket, or the previous list (kRegions regions of St.rcap
  // slots; pre[] = prefix sums of the region lengths)
  __shared__ int64_t pre[kRegions + 1];
  int64_t begin = 0, count = A.N;
  if (St.in_list) {
    if (threadIdx.x == 0) {
      int64_t acc = 0;
      for (int r = 0; r < kRegions; ++r) {
        pre[r] = acc;
        acc += (int64_t)St.in_count[r * kCounterStride];
      }
      pre[kRegions] = acc;
    }
    __syncthreads();
    count = pre[kRegions];
  } else {
    if (bucket) {
      begin = bucket[NO - 1];
      count = bucket[NO] - begin;
    }
    sub_range(A, begin, count);
  }
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < count;
       idx += stride) {
    int64_t slot_in = idx;
    if (St.in_list) {
      int lo = 0, hi = kRegions;  // largest r with pre[r] <= idx
      while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (pre[mid] <= idx) lo = mid; else hi = mid;
      }
      slot_in = (int64_t)lo * St.rcap + (idx - pre[lo]);
    }
    const int64_t p = St.in_list ? (int64_t)St.in_list[slot_in]
                                 : (perm ? (int64_t)perm[begin + idx] : begin + idx);
    Geo32<NO> G;
    float t0[NO][2];
    const bool valid = load_path32<NO>(A, p, G, t0);
    State32<NO> S;
    int it = 0, streak = 0;
    if (!St.in_list) {
      init_state<NO>(G, t0, S);
    } else {
      const float* src = St.state_in + slot_in;
      const int64_t c = St.cap;
#pragma unroll
      for (int k = 0; k < M; ++k) S.T[k] = src[k * c];
#pragma unroll
      for (int k = 0; k < M; ++k) S.P[k] = src[(M + k) * c];
#pragma unroll
      for (int k = 0; k < HP; ++k) S.H[k] = src[(2 * M + k) * c];
      it = __float_as_int(src[(2 * M + HP) * c]);
      streak = __float_as_int(src[(2 * M + HP + 1) * c]);
      grad32<NO>(G, S.T, S.g, S.r, S.l2, S.il);
    }
    bool done = it >= A.n_iter;
    for (int k = 0; k < St.iters; ++k) {
      if (__all(done)) break;
      if (!done) {
        float d2 = bfgs_iter<NO>(G, S, A.fp_iters, it == 0);
        ++it;
        streak = (d2 <= A.exit_d2) ? streak + 1 : 0;
        done = streak >= 2 || it >= A.n_iter;
      }
    }
    const bool fin = done || !St.out_list || !valid;
    if (fin) {
      polish32<NO>(A, G, S.T);
      store_phase1<NO>(A, p, S.T, it, valid);
    }
    const unsigned long long more = __ballot(!fin);
    if (more) {
      // region of this 64-path chunk of the input: chunks are spread over
      // kRegions counters, each on its own cache line
      const int region = (int)((idx >> 6) % kRegions);
      unsigned long long base = 0;
      if (lane == 0)
        base = atomicAdd(St.out_count + region * kCounterStride,
                         (unsigned long long)__popcll(more));
      base = __shfl(base, 0);
      if (!fin) {
        const int64_t slot = (int64_t)region * St.rcap +
                             (int64_t)(base + (unsigned long long)__popcll(more & below));
        St.out_list[slot] = (int32_t)p;
        float* dst = St.state_out + slot;
        const int64_t c = St.cap;
#pragma unroll
        for (int k = 0; k < M; ++k) dst[k * c] = S.T[k];
#pragma unroll
        for (int k = 0; k < M; ++k) dst[(M + k) * c] = S.P[k];
#pragma unroll
        for (int k = 0; k < HP; ++k) dst[(2 * M + k) * c] = S.H[k];
        dst[(2 * M + HP) * c] = __int_as_float(it);
        dst[(2 * M + HP + 1) * c] = __int_as_float(streak);
      }
    }
  }
}

// Work counters of a wave (segment evaluations, trial lengths, Newton
// solves) into counters [3][kWorkSlots]: wave sums, one atomic per counter
// per wave, spread over kWorkSlots slots by workgroup.
__device__ __forceinline__ void add_work(unsigned long long* w, uint32_t (&work)[3],
                                         int lane) {
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) work[q] += __shfl_xor(work[q], off);
  if (lane == 0) {
    const int slot = blockIdx.x % kWorkSlots;
#pragma unroll
    for (int q = 0; q < 3; ++q)
      atomicAdd(w + q * kWorkSlots + slot, (unsigned long long)work[q]);
  }
}

// Phase 2: FP64 refinement of the parameters left by bfgs_kernel in A.t
// (unit-vector coordinates), certificate, and the final outputs.
// With quick_steps > 0 the refinement runs in two passes: the first takes
// quick_steps Newton steps at the last smoothing level for every path of the
// bucket and writes the certified ones; the others are listed (by the same
// region scheme as the early-exit stages: St.out_list) with their point
// left in A.t, and the second pass (St.in_list) runs the full schedule on
// them from there (after merge_kernel for orders >= 2).
// St.in_list == St.out_list == null: one pass with the full schedule.
// QUICK (St.out_list != null) and the full schedule are separate
// instantiations, so that each gets its own register budget.
// (four and five slots: asked for two waves per SIMD, the full schedule at
// four fits 251 VGPRs without spilling where it took 260 registers and one
// wave, and five spills 68 / 132 bytes; each group ran about 2 % faster. At
// six slots the spills of a second wave (228 / 316 bytes) made it 6 %
// slower.)
template <int NO, bool QUICK>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu((NO == 4 || NO == 5) ? 2 : 1))) void refine_kernel(
    SolveArgs A, const int32_t* __restrict__ perm,
    const int64_t* __restrict__ bucket, StageArgs St) {
  __shared__ int64_t pre[kRegions + 1];
  int64_t begin = 0, count = A.N;
  if (St.in_list) {
    if (threadIdx.x == 0) {
      int64_t acc = 0;
      for (int r = 0; r < kRegions; ++r) {
        pre[r] = acc;
        acc += (int64_t)St.in_count[r * kCounterStride];
      }
      pre[kRegions] = acc;
    }
    __syncthreads();
    count = pre[kRegions];
  } else {
    if (bucket) {
      begin = bucket[NO - 1];
      count = bucket[NO] - begin;
    }
    sub_range(A, begin, count);
  }
  constexpr bool quick = QUICK;
  // At low orders the geometry stays in registers as FP64; from kRegGeoMax + 1
  // on it sits in LDS as FP32 (GeoLds), widened on every use, which saves
  // the registers the larger orders are short of.
  constexpr bool reg_geo = NO <= kRegGeoMax;
  using GeoT = typename std::conditional<reg_geo, Geo64<NO>, GeoLds<NO>>::type;
  __shared__ float geo[reg_geo ? 1 : geo_lds_rows(NO) * kBlock];
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  uint32_t work[3] = {0, 0, 0};
  for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < count;
       idx += stride) {
    int64_t p;
    if (St.in_list) {
      int lo = 0, hi = kRegions;
      while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (pre[mid] <= idx) lo = mid; else hi = mid;
      }
      p = St.in_list[(int64_t)lo * St.rcap + (idx - pre[lo])];
    } else {
      p = perm ? (int64_t)perm[begin + idx] : begin + idx;
    }
    const bool valid = (A.status[p] & FPT_ST_INVALID) == 0;
    GeoT D;
    float inv[NO][2];
    if constexpr (reg_geo)
      load_geo64<NO>(A, p, D, inv);
    else
      load_geo_lds<NO>(A, p, geo + threadIdx.x, D, inv);
    double td[2 * NO];
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      float t0 = A.t[(int64_t)(2 * j) * A.N + p];
      float t1 = A.t[(int64_t)(2 * j + 1) * A.N + p];
      td[2 * j] = (double)t0 * (double)inv[j][0];
      td[2 * j + 1] = D.edge(j) ? 0.0 : (double)t1 * (double)inv[j][1];
    }
    RefineOut ro = refine64(D, td, A, quick, work);
    // list the paths this pass does not certify: the quick pass defers
    // them (to the collapse step and the full schedule), the full schedule
    // writes them and hands them to the last collapse step
    const bool listed = St.out_list != nullptr && valid && !ro.certified;
    const unsigned long long more = __ballot(listed);
    if (more) {
      const int region = (int)((idx >> 6) % kRegions);
      unsigned long long base = 0;
      if (lane == 0)
        base = atomicAdd(St.out_count + region * kCounterStride,
                         (unsigned long long)__popcll(more));
      base = __shfl(base, 0);
      if (listed)
        St.out_list[(int64_t)region * St.rcap +
                    (int64_t)(base + (unsigned long long)__popcll(more & below))] = (int32_t)p;
    }
    if (quick && listed) {
      // hand the quick pass's point to the collapse step and the second pass
      // (unit-vector coordinates, as the FP32 phase left them)
#pragma unroll
      for (int j = 0; j < NO; ++j) {
        A.t[(int64_t)(2 * j) * A.N + p] = (float)(td[2 * j] * rcp64((double)inv[j][0]));
        A.t[(int64_t)(2 * j + 1) * A.N + p] =
            D.edge(j) ? 0.f : (float)(td[2 * j + 1] * rcp64((double)inv[j][1]));
      }
      continue;
    }
    write_path64(A, D, td, p, valid, ro.certified, ro.refined);
  }
  if (A.work) add_work(A.work, work, lane);
}

// The collapse step (merge_runs64) on the listed paths (St.in_list). Mode
// 0, between the quick pass and the full schedule: from the quick pass's
// point (unit-vector coordinates), with collapsed segments taken as those
// shorter than kMergeShortQuick; the paths it certifies are written, the
// others listed (St.out_list) for the full schedule. Mode 1, after the full
// schedule: from its written output (caller's parametrisation), where a
// collapse has come much closer, with kMergeShortFull; it overwrites the
// paths it certifies and leaves the others as written. Mode 0 takes one
// round of merge_runs64 (most of its paths have one collapse, and the full
// schedule follows for the others), mode 1 up to three (a fourth certifies a
// few hundredths of a per cent more of the highest orders and lengthens
// their latency-bound tail).

// (three slots: asked for two waves per SIMD, the compiler spills 244 bytes
// where it otherwise takes 48 AGPRs beyond 256 registers and runs one wave;
// the order-3 refinement group took 3-6 % less time. At four to six slots
// the spills that two waves take cost more than the wave gains, up to half
// again at six; at two slots, three waves instead of two also lost.)
template <int NO>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(NO == 3 ? 2 : 1)))
void merge_kernel(SolveArgs A, StageArgs St) {
  __shared__ int64_t pre[kRegions + 1];
  if (threadIdx.x == 0) {
    int64_t acc = 0;
    for (int r = 0; r < kRegions; ++r) {
      pre[r] = acc;
      acc += (int64_t)St.in_count[r * kCounterStride];
    }
    pre[kRegions] = acc;
  }
  __syncthreads();
  const int64_t count = pre[kRegions];
  __shared__ float geo[geo_lds_rows(NO) * kBlock];
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  uint32_t work[3] = {0, 0, 0};
  for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < count;
       idx += stride) {
    int lo = 0, hi = kRegions;
    while (hi - lo > 1) {
      int mid = (lo + hi) >> 1;
      if (pre[mid] <= idx) lo = mid; else hi = mid;
    }
    const int64_t p = St.in_list[(int64_t)lo * St.rcap + (idx - pre[lo])];
    GeoLds<NO> D;
    float inv[NO][2];
    load_geo_lds<NO>(A, p, geo + threadIdx.x, D, inv);
    double td[2 * NO];
    const bool unit = St.mode == 0;
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      float t0 = A.t[(int64_t)(2 * j) * A.N + p];
      float t1 = A.t[(int64_t)(2 * j + 1) * A.N + p];
      td[2 * j] = (double)t0 * (unit ? (double)inv[j][0] : 1.0);
      td[2 * j + 1] = D.edge(j) ? 0.0 : (double)t1 * (unit ? (double)inv[j][1] : 1.0);
    }
    const bool ok =
        merge_runs64<NO>(D, td, A, unit ? kMergeShortQuick : kMergeShortFull, unit ? 1 : 3, work);
    const unsigned long long more = __ballot(!ok && St.out_list != nullptr);
    if (more) {
      const int region = (int)((idx >> 6) % kRegions);
      unsigned long long base = 0;
      if (lane == 0)
        base = atomicAdd(St.out_count + region * kCounterStride,
                         (unsigned long long)__popcll(more));
      base = __shfl(base, 0);
      if (!ok)
        St.out_list[(int64_t)region * St.rcap +
                    (int64_t)(base + (unsigned long long)__popcll(more & below))] = (int32_t)p;
    }
    if (ok) write_path64(A, D, td, p, true, true, true, true);
  }
  if (A.work) add_work(A.work + 3 * kWorkSlots, work, lane);
}

// ------------------------------------------------------ order bucketing ---
// A counting sort of the path indices by order, without global atomics:
// (1) each workgroup counts the orders of its chunk of kSortChunk paths,
// (2) one workgroup turns the per-chunk counts into per-chunk output
//     offsets (bucket of order n first for n = 1..n_max, invalid orders
//     last), (3) each workgroup scatters its chunk in input order.
// Thread t of a chunk owns its 32 consecutive paths (two 16-byte loads).
// bucket[n-1] .. bucket[n] is the range of order n in perm;
// bucket[n_max] .. bucket[n_max+1] holds the paths with an invalid order.

constexpr int kSortPer = kSortChunk / kBlock;  // paths per thread
static_assert(kSortPer == 32, "two 16-byte loads per thread");

// A thread's 32 consecutive bytes of a per-path byte array (two 16-byte
// loads where aligned; zero past the end).
__device__ __forceinline__ void load32_bytes(const uint8_t* __restrict__ a, int64_t base,
                                             int64_t c1, uint8_t (&o)[kSortPer]) {
  if (base + kSortPer <= c1 && (((uintptr_t)(a + base)) & 15) == 0) {
    const uint4 v0 = *reinterpret_cast<const uint4*>(a + base);
    const uint4 v1 = *reinterpret_cast<const uint4*>(a + base + 16);
    const uint32_t w[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
    for (int q = 0; q < kSortPer; ++q) o[q] = (uint8_t)(w[q >> 2] >> (8 * (q & 3)));
  } else {
#pragma unroll
    for (int q = 0; q < kSortPer; ++q) o[q] = (base + q < c1) ? a[base + q] : 0;
  }
}

// Bins of this thread's paths: 1..n_max, 0 for an invalid order, -1 past
// the end of the chunk. With a status array (the backward pass), bin 7
// takes the collapsed minimisers of orders >= 2 that carry a gradient
// (FPT_ST_COLLAPSED without FPT_ST_NOGRAD), which the backward pass
// differentiates in a kernel of their own.
__device__ __forceinline__ void sort_bins(const uint8_t* __restrict__ order,
                                          const uint8_t* __restrict__ status, int64_t base,
                                          int64_t c1, int n_max, int (&bins)[kSortPer]) {
  uint8_t o[kSortPer];
  load32_bytes(order, base, c1, o);
#pragma unroll
  for (int q = 0; q < kSortPer; ++q) {
    const int b = (o[q] >= 1 && o[q] <= n_max) ? (int)o[q] : 0;
    bins[q] = (base + q < c1) ? b : -1;
  }
  if (status) {
    uint8_t st[kSortPer];
    load32_bytes(status, base, c1, st);
#pragma unroll
    for (int q = 0; q < kSortPer; ++q) {
      const bool kkt = (st[q] & FPT_ST_COLLAPSED) && !(st[q] & FPT_ST_NOGRAD);
      bins[q] = (kkt && bins[q] >= 2) ? 7 : bins[q];
    }
  }
}

// A thread's count per bin as eight 6-bit fields of one 64-bit word (at most
// kSortPer = 32 paths per bin): one shift and one add per path.
__device__ __forceinline__ uint64_t bin_unit(int b) {
  return (b >= 0) ? (1ull << (6 * b)) : 0ull;
}
__device__ __forceinline__ uint32_t bin_field(uint64_t packed, int b) {
  return (uint32_t)(packed >> (6 * b)) & 63u;
}

__device__ __forceinline__ void bin_counts(const int (&bins)[kSortPer],
                                           uint32_t (&cnt)[8]) {
  uint64_t packed = 0;
#pragma unroll
  for (int q = 0; q < kSortPer; ++q) packed += bin_unit(bins[q]);
#pragma unroll
  for (int k = 0; k < 8; ++k) cnt[k] = bin_field(packed, k);
}

__global__ __launch_bounds__(kBlock) void bucket_count_kernel(
    const uint8_t* __restrict__ order, const uint8_t* __restrict__ status, int64_t N,
    int n_max, uint32_t* __restrict__ ccount) {
  __shared__ uint32_t wsum[kBlock / 64][8];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * kSortChunk;
  const int64_t c1 = min(N, c0 + (int64_t)kSortChunk);
  int bins[kSortPer];
  sort_bins(order, status, c0 + (int64_t)threadIdx.x * kSortPer, c1, n_max, bins);
  uint32_t cnt[8];
  bin_counts(bins, cnt);
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cnt[k] += __shfl_xor(cnt[k], off);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 8; ++k) wsum[w][k] = cnt[k];
  __syncthreads();
  if (threadIdx.x < 8) {
    uint32_t t = 0;
#pragma unroll
    for (int v = 0; v < kBlock / 64; ++v) t += wsum[v][threadIdx.x];
    ccount[(int64_t)blockIdx.x * 8 + threadIdx.x] = t;
  }
}

// One workgroup: per-chunk offsets (in place over ccount) and bucket bounds.
// Thread t sums a contiguous run of chunks; an exclusive scan over the
// threads gives each run's start: per bin, over the wave by shuffles, then
// over the four waves' totals in LDS (two barriers; counts fit 32 bits, as
// N < 2^31).
__global__ __launch_bounds__(kBlock) void bucket_scan_kernel(
    uint32_t* __restrict__ ccount, int64_t nchunks, int n_max,
    int64_t* __restrict__ bucket) {
  __shared__ uint32_t wtot[kBlock / 64][8];
  __shared__ uint32_t woff[kBlock / 64][8];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t per = (nchunks + kBlock - 1) / kBlock;
  const int64_t c0 = (int64_t)threadIdx.x * per;
  const int64_t c1 = min(nchunks, c0 + per);
  uint32_t sum[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  // (a chunk's 8 counts are 32 aligned bytes: two 16-byte loads, several
  // chunks in flight)
#pragma unroll 4
  for (int64_t c = c0; c < c1; ++c) {
    const uint4 lo = *reinterpret_cast<const uint4*>(ccount + c * 8);
    const uint4 hi = *reinterpret_cast<const uint4*>(ccount + c * 8 + 4);
    sum[0] += lo.x;
    sum[1] += lo.y;
    sum[2] += lo.z;
    sum[3] += lo.w;
    sum[4] += hi.x;
    sum[5] += hi.y;
    sum[6] += hi.z;
    sum[7] += hi.w;
  }
  uint32_t inc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    inc[k] = sum[k];
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t v = __shfl_up(inc[k], d);
      if (lane >= d) inc[k] += v;
    }
  }
  if (lane == 63)
#pragma unroll
    for (int k = 0; k < 8; ++k) wtot[w][k] = inc[k];
  __syncthreads();
  if (threadIdx.x < 8) {
    // bin k: its waves' offsets, and its start among the bins (orders
    // 1..n_max, then invalid orders, then bin 7, which only the backward
    // pass fills)
    const int k = threadIdx.x;
    uint32_t tot[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      tot[b] = 0;
#pragma unroll
      for (int v = 0; v < kBlock / 64; ++v) tot[b] += wtot[v][b];
    }
    uint32_t acc = 0, st = 0;
    for (int n = 1; n <= n_max; ++n) {
      if (n == k) st = acc;
      acc += tot[n];
      if (k == 0) bucket[n] = (int64_t)acc;
    }
    if (k == 0) st = acc;
    acc += tot[0];
    if (k == 0) bucket[n_max + 1] = (int64_t)acc;
    if (k == 7) st = acc;
    acc += tot[7];
    if (k == 0) {
      bucket[0] = 0;
      bucket[n_max + 2] = (int64_t)acc;
    }
    uint32_t o = st;
#pragma unroll
    for (int v = 0; v < kBlock / 64; ++v) {
      woff[v][k] = o;
      o += wtot[v][k];
    }
  }
  __syncthreads();
  uint32_t run[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) run[k] = woff[w][k] + inc[k] - sum[k];
#pragma unroll 4
  for (int64_t c = c0; c < c1; ++c) {
    const uint4 lo = *reinterpret_cast<const uint4*>(ccount + c * 8);
    const uint4 hi = *reinterpret_cast<const uint4*>(ccount + c * 8 + 4);
    const uint32_t v[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    uint32_t o[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      o[k] = run[k];
      run[k] += v[k];
    }
    *reinterpret_cast<uint4*>(ccount + c * 8) = make_uint4(o[0], o[1], o[2], o[3]);
    *reinterpret_cast<uint4*>(ccount + c * 8 + 4) = make_uint4(o[4], o[5], o[6], o[7]);
  }
}

// Scatter: a stable sort of the chunk. Thread t's paths come after those of
// threads < t in each bin: per-bin exclusive scan of the thread counts over
// the wave (shuffles) and the waves (LDS). Each path's place is its thread's
// start in its bin (kept in LDS, one column per thread) plus the running
// count of that bin over the thread's earlier paths (packed as in
// bin_counts). The sorted chunk is staged in LDS (bins one after another,
// skewed by one slot per 32 against bank conflicts) and copied out with
// consecutive threads on consecutive addresses: each bin of the chunk is one
// contiguous run of perm.
__device__ __forceinline__ int sort_skew(int i) { return i + (i >> 5); }

__global__ __launch_bounds__(kBlock) void bucket_scatter_kernel(
    const uint8_t* __restrict__ order, const uint8_t* __restrict__ status, int64_t N, int n_max,
    const uint32_t* __restrict__ coff, int32_t* __restrict__ perm,
    int32_t* __restrict__ inv) {
  __shared__ uint32_t wtot[kBlock / 64][8];
  __shared__ int32_t stage[kSortChunk + kSortChunk / 32];
  __shared__ int32_t toff[8][kBlock];
  __shared__ int32_t lstart[9];
  __shared__ uint32_t gstart[8];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * kSortChunk;
  const int64_t c1 = min(N, c0 + (int64_t)kSortChunk);
  const int64_t base = c0 + (int64_t)threadIdx.x * kSortPer;
  int bins[kSortPer];
  sort_bins(order, status, base, c1, n_max, bins);
  uint32_t cnt[8], incl[8];
  bin_counts(bins, cnt);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    incl[k] = cnt[k];
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t v = __shfl_up(incl[k], d);
      if (lane >= d) incl[k] += v;
    }
  }
  if (lane == 63)
#pragma unroll
    for (int k = 0; k < 8; ++k) wtot[w][k] = incl[k];
  if (threadIdx.x < 8) gstart[threadIdx.x] = coff[(int64_t)blockIdx.x * 8 + threadIdx.x];
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int k = 0; k < 8; ++k) {
      lstart[k] = acc;
      for (int v = 0; v < kBlock / 64; ++v) acc += (int)wtot[v][k];
    }
    lstart[8] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    int off = lstart[k] + (int)(incl[k] - cnt[k]);
    for (int v = 0; v < w; ++v) off += (int)wtot[v][k];
    toff[k][threadIdx.x] = off;
  }
  // (each thread reads back only its own column: no barrier)
  uint64_t run = 0;
  int lp[kSortPer];  // each path's place in the sorted chunk
#pragma unroll
  for (int q = 0; q < kSortPer; ++q) {
    const int b = bins[q];
    lp[q] = -1;
    if (b >= 0) {
      lp[q] = toff[b][threadIdx.x] + (int)bin_field(run, b);
      stage[sort_skew(lp[q])] = (int32_t)(base + q);
      run += bin_unit(b);
    }
  }
  __syncthreads();
  const int total = lstart[8];
  for (int i = threadIdx.x; i < total; i += kBlock) {
    int k = 0;
#pragma unroll
    for (int b = 1; b < 8; ++b) k += (i >= lstart[b]) ? 1 : 0;
    perm[(int64_t)gstart[k] + (i - lstart[k])] = stage[sort_skew(i)];
  }
  if (!inv) return;
  // the inverse permutation (inv[p] = slot of path p), if asked for: staged
  // in LDS (the sorted chunk is out), then written with consecutive threads
  // on consecutive addresses (a thread's own 32 paths would be 32 stores
  // 128 bytes apart across the wave)
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kSortPer; ++q) {
    const int b = bins[q];
    if (b >= 0)
      stage[sort_skew(threadIdx.x * kSortPer + q)] =
          (int32_t)(gstart[b] + (uint32_t)(lp[q] - lstart[b]));
  }
  __syncthreads();
  const int len = (int)(c1 - c0);
  for (int i = threadIdx.x; i < len; i += kBlock) inv[c0 + i] = stage[sort_skew(i)];
}

// Paths with an order outside 1..n_max: NaN outputs, INVALID status (perm
// null: the outputs are in bucket order).
__global__ __launch_bounds__(kBlock) void invalid_kernel(
    SolveArgs A, const int32_t* __restrict__ perm, const int64_t* __restrict__ bucket) {
  int64_t begin = bucket[A.n_max], count = bucket[A.n_max + 1] - begin;
  const float qnan = __builtin_nanf("");
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < count; idx += stride) {
    int64_t p = perm ? (int64_t)perm[begin + idx] : begin + idx;
    for (int j = 0; j < A.n_max; ++j) {
      for (int c = 0; c < 3; ++c) A.x[(int64_t)(3 * j + c) * A.N + p] = qnan;
      A.t[(int64_t)(2 * j) * A.N + p] = qnan;
      A.t[(int64_t)(2 * j + 1) * A.N + p] = qnan;
    }
    A.len[p] = qnan;
    A.status[p] = FPT_ST_INVALID | FPT_ST_NOGRAD;
    A.iters[p] = 0;
  }
}

// ------------------------------------------------------ bucket order -----
// With an order array, the paths of one order are scattered over the
// caller's arrays, and every per-order kernel would read and write them
// through the permutation: a wave's 64 paths then touch many cache lines per
// access (for an order that holds 1/k of the paths, about k times as many as
// contiguous paths). So the solve works in bucket order: the first phase
// reads each path's inputs through the permutation and leaves copies of its
// indices at its bucket slot s (SolveArgs.perm_in), the passes that follow
// read and write slot s contiguously, and unsort_kernel writes the caller's
// arrays in the caller's order at the end, with consecutive threads on
// consecutive paths (the NaN entries beyond a path's order included), from
// the inverse permutation that the bucketing scatter writes.

// Order of bucket slot s: 1..n_max, or n_max + 1 (the invalid orders).
__device__ __forceinline__ int bucket_order(const int64_t* bnd, int n_max, int64_t s) {
  int n = 1;
  while (n <= n_max && s >= bnd[n]) ++n;
  return n;
}

// Outputs in the caller's order from the bucket-order ones (S): path p from
// slot inv[p], entries beyond its order NaN.
template <int NMAX>
__global__ __launch_bounds__(kBlock) void unsort_kernel(
    SolveArgs S, float* __restrict__ x, float* __restrict__ len, float* __restrict__ t,
    uint8_t* __restrict__ status, uint16_t* __restrict__ iters,
    const int32_t* __restrict__ inv, const int64_t* __restrict__ bucket) {
  __shared__ int64_t bnd[FPT_NMAX + 2];
  if (threadIdx.x <= (unsigned)NMAX + 1) bnd[threadIdx.x] = bucket[threadIdx.x];
  __syncthreads();
  const float qnan = __builtin_nanf("");
  const int64_t N = S.N;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < N; p += stride) {
    const int64_t s = inv[p];
    const int n = bucket_order(bnd, NMAX, s);
    float v[5 * NMAX];
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
      const bool in = j < n && n <= NMAX;
#pragma unroll
      for (int c = 0; c < 3; ++c) v[5 * j + c] = in ? S.x[(int64_t)(3 * j + c) * N + s] : qnan;
      v[5 * j + 3] = in ? S.t[(int64_t)(2 * j) * N + s] : qnan;
      v[5 * j + 4] = in ? S.t[(int64_t)(2 * j + 1) * N + s] : qnan;
    }
    const float l = S.len[s];
    const uint8_t st = S.status[s];
    const uint16_t it = S.iters[s];
    // (streaming stores: nothing here is read again by this solve)
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
        __builtin_nontemporal_store(v[5 * j + c], x + (int64_t)(3 * j + c) * N + p);
      __builtin_nontemporal_store(v[5 * j + 3], t + (int64_t)(2 * j) * N + p);
      __builtin_nontemporal_store(v[5 * j + 4], t + (int64_t)(2 * j + 1) * N + p);
    }
    __builtin_nontemporal_store(l, len + p);
    __builtin_nontemporal_store(st, status + p);
    __builtin_nontemporal_store(it, iters + p);
  }
}

// The same with four consecutive paths per thread, so that every row goes
// out as one 16-byte store (status and iters packed into 4 and 8 bytes):
// for N a multiple of 4 and the caller's arrays aligned to match (the
// one-path kernel above takes every other case).
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <int NMAX>
__global__ __launch_bounds__(kBlock) void unsort4_kernel(
    SolveArgs S, float* __restrict__ x, float* __restrict__ len, float* __restrict__ t,
    uint8_t* __restrict__ status, uint16_t* __restrict__ iters,
    const int32_t* __restrict__ inv, const int64_t* __restrict__ bucket) {
  __shared__ int64_t bnd[FPT_NMAX + 2];
  if (threadIdx.x <= (unsigned)NMAX + 1) bnd[threadIdx.x] = bucket[threadIdx.x];
  __syncthreads();
  const float qnan = __builtin_nanf("");
  const int64_t N = S.N, N4 = N / 4;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < N4; q += stride) {
    const int4 iv = reinterpret_cast<const int4*>(inv)[q];
    const int64_t s[4] = {iv.x, iv.y, iv.z, iv.w};
    int n[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      n[k] = bucket_order(bnd, NMAX, s[k]);
      n[k] = n[k] <= NMAX ? n[k] : 0;  // invalid orders: every row NaN
    }
    // (streaming stores: nothing here is read again by this solve)
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
#pragma unroll
      for (int r = 0; r < 5; ++r) {
        const float* src = r < 3 ? S.x + (int64_t)(3 * j + r) * N : S.t + (int64_t)(2 * j + r - 3) * N;
        float* dst = r < 3 ? x + (int64_t)(3 * j + r) * N : t + (int64_t)(2 * j + r - 3) * N;
        f32x4 v;
        v.x = j < n[0] ? src[s[0]] : qnan;
        v.y = j < n[1] ? src[s[1]] : qnan;
        v.z = j < n[2] ? src[s[2]] : qnan;
        v.w = j < n[3] ? src[s[3]] : qnan;
        __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(dst) + q);
      }
    }
    f32x4 l;
    l.x = S.len[s[0]];
    l.y = S.len[s[1]];
    l.z = S.len[s[2]];
    l.w = S.len[s[3]];
    __builtin_nontemporal_store(l, reinterpret_cast<f32x4*>(len) + q);
    uint32_t st = 0u;
    uint64_t it = 0ull;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      st |= (uint32_t)S.status[s[k]] << (8 * k);
      it |= (uint64_t)S.iters[s[k]] << (16 * k);
    }
    __builtin_nontemporal_store(st, reinterpret_cast<uint32_t*>(status) + q);
    __builtin_nontemporal_store(it, reinterpret_cast<uint64_t*>(iters) + q);
  }
}

// ------------------------------------------------------------- launch -----

template <int NO>
static hipError_t launch_phase(int phase, const SolveArgs& A,
                               const int32_t* perm, const int64_t* bucket,
                               const StageArgs* stage, int grid,
                               hipStream_t st) {
  if (phase == 0) {
    if (A.line_search == FPT_LS_ARMIJO)
      hipLaunchKernelGGL((bfgs_kernel<NO, FPT_LS_ARMIJO>), dim3(grid), dim3(kBlock), 0, st, A,
                         perm, bucket);
    else
      hipLaunchKernelGGL(bfgs_kernel<NO>, dim3(grid), dim3(kBlock), 0, st, A, perm, bucket);
  } else if (phase == 4)
    hipLaunchKernelGGL((refine_kernel<NO, true>), dim3(grid), dim3(kBlock), 0, st, A,
                       perm, bucket, *stage);
  else if (phase == 1)
    hipLaunchKernelGGL((refine_kernel<NO, false>), dim3(grid), dim3(kBlock), 0, st, A,
                       perm, bucket, *stage);
  else if (phase == 2)
    hipLaunchKernelGGL(bfgs_stage_kernel<NO>, dim3(grid), dim3(kBlock), 0,
                       st, A, perm, bucket, *stage);
  else if (phase == 5)
    hipLaunchKernelGGL(newton32_kernel<NO>, dim3(grid), dim3(kBlock), 0, st, A, perm,
                       bucket);
  else
    hipLaunchKernelGGL(merge_kernel<NO>, dim3(grid), dim3(kBlock), 0, st, A,
                       *stage);
  return hipGetLastError();
}

// phase 0: bfgs_kernel<order>, 1: refine_kernel<order> with the full
// schedule (listing the paths it does not certify when stage->out_list is
// set), 4: its quick pass, 5: newton32_kernel<order> (the FP32 Newton variant
// of phase 0), 2: bfgs_stage_kernel<order> (one early-exit stage, `stage`
// describes it), 3: merge_kernel<order> (the collapse step, stage->mode)
hipError_t launch_solve(int phase, int order, const SolveArgs& A,
                        const int32_t* perm, const int64_t* bucket,
                        const StageArgs* stage, int grid, hipStream_t st) {
  switch (order) {
    case 1: return launch_phase<1>(phase, A, perm, bucket, stage, grid, st);
    case 2: return launch_phase<2>(phase, A, perm, bucket, stage, grid, st);
    case 3: return launch_phase<3>(phase, A, perm, bucket, stage, grid, st);
    case 4: return launch_phase<4>(phase, A, perm, bucket, stage, grid, st);
    case 5: return launch_phase<5>(phase, A, perm, bucket, stage, grid, st);
    case 6: return launch_phase<6>(phase, A, perm, bucket, stage, grid, st);
  }
  return hipErrorInvalidValue;
}

int stage_fields_for(int order) {
  switch (order) {
    case 1: return stage_fields<1>();
    case 2: return stage_fields<2>();
    case 3: return stage_fields<3>();
    case 4: return stage_fields<4>();
    case 5: return stage_fields<5>();
    case 6: return stage_fields<6>();
  }
  return 0;
}

template <int NO>
static const void* phase_ptr(int phase) {
  return phase == 0 ? (const void*)bfgs_kernel<NO>
         : phase == 1 ? (const void*)refine_kernel<NO, false>
         : phase == 2 ? (const void*)bfgs_stage_kernel<NO>
         : phase == 3 ? (const void*)merge_kernel<NO>
         : phase == 4 ? (const void*)refine_kernel<NO, true>
                      : (const void*)newton32_kernel<NO>;
}

const void* solve_kernel_ptr(int phase, int order) {
  switch (order) {
    case 1: return phase_ptr<1>(phase);
    case 2: return phase_ptr<2>(phase);
    case 3: return phase_ptr<3>(phase);
    case 4: return phase_ptr<4>(phase);
    case 5: return phase_ptr<5>(phase);
    case 6: return phase_ptr<6>(phase);
  }
  return nullptr;
}

hipError_t launch_bucketing(const uint8_t* order, int64_t N, int n_max,
                            uint32_t* ccount, int64_t* bucket, int32_t* perm,
                            hipStream_t st, int32_t* inv, const uint8_t* status) {
  const int64_t nchunks = (N + kSortChunk - 1) / kSortChunk;
  hipLaunchKernelGGL(bucket_count_kernel, dim3((unsigned)nchunks), dim3(kBlock), 0, st,
                     order, status, N, n_max, ccount);
  hipLaunchKernelGGL(bucket_scan_kernel, dim3(1), dim3(kBlock), 0, st, ccount,
                     nchunks, n_max, bucket);
  hipLaunchKernelGGL(bucket_scatter_kernel, dim3((unsigned)nchunks), dim3(kBlock), 0, st,
                     order, status, N, n_max, ccount, perm, inv);
  return hipGetLastError();
}

template <int NMAX>
static void unsort_launch(const SolveArgs& S, const SolveArgs& A, const int32_t* inv,
                          const int64_t* bucket, int grid, hipStream_t st) {
  const auto al = [](const void* p, uintptr_t a) { return (uintptr_t)p % a == 0; };
  if (S.N % 4 == 0 && al(A.x, 16) && al(A.t, 16) && al(A.len, 16) && al(A.status, 4) &&
      al(A.iters, 8) && al(inv, 16))
    hipLaunchKernelGGL(unsort4_kernel<NMAX>, dim3(grid), dim3(kBlock), 0, st, S, A.x, A.len,
                       A.t, A.status, A.iters, inv, bucket);
  else
    hipLaunchKernelGGL(unsort_kernel<NMAX>, dim3(grid), dim3(kBlock), 0, st, S, A.x, A.len,
                       A.t, A.status, A.iters, inv, bucket);
}

hipError_t launch_unsort(const SolveArgs& S, const SolveArgs& A, const int32_t* inv,
                         const int64_t* bucket, int grid, hipStream_t st) {
  switch (S.n_max) {
    case 1: unsort_launch<1>(S, A, inv, bucket, grid, st); break;
    case 2: unsort_launch<2>(S, A, inv, bucket, grid, st); break;
    case 3: unsort_launch<3>(S, A, inv, bucket, grid, st); break;
    case 4: unsort_launch<4>(S, A, inv, bucket, grid, st); break;
    case 5: unsort_launch<5>(S, A, inv, bucket, grid, st); break;
    case 6: unsort_launch<6>(S, A, inv, bucket, grid, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_invalid(const SolveArgs& A, const int32_t* perm,
                          const int64_t* bucket, int grid, hipStream_t st) {
  hipLaunchKernelGGL(invalid_kernel, dim3(grid), dim3(kBlock), 0, st, A, perm,
                     bucket);
  return hipGetLastError();
}

}  // namespace fpt

namespace fpt {

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0ull;
}

// clears small counters with a kernel rather than a memset node, so that the
// sequence can be captured into a HIP graph
hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace fpt
