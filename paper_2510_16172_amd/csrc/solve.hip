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
template <int NO>
__device__ __forceinline__ void grad32(const Geo32<NO>& G, const float* T,
                                       float* g, float (*r)[3], float* l2,
                                       float* il) {
  float x[NO][3];
#pragma unroll
  for (int j = 0; j < NO; ++j)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      x[j][c] = fmaf(T[2 * j + 1], G.a[j][1][c],
                     fmaf(T[2 * j], G.a[j][0][c], G.b[j][c]));
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
    g[2 * j] = dot3(G.a[j][0], du);
    g[2 * j + 1] = dot3(G.a[j][1], du);
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
      a1[c] = (float)D.a[j][0][c];
      a2[c] = (float)D.a[j][1][c];
    }
    basis_inv32(a1, a2, D.edge[j], inv[j][0], inv[j][1]);
  }
}

template <int NO>
__device__ __forceinline__ double max_disp64(const Geo64<NO>& G,
                                             const double* d) {
  double m = 0.0;
#pragma unroll
  for (int j = 0; j < NO; ++j) {
    double w[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      w[c] = d[2 * j] * G.a[j][0][c] + d[2 * j + 1] * G.a[j][1][c];
    m = fmax(m, dot3d(w, w));
  }
  return m;  // squared
}

// Damped Newton refinement, level by level. t is in the caller's
// parametrisation. A trial step s*d (s = 1, 1/4, 1/16, ...) is taken if it
// does not lengthen the smoothed path beyond the rounding of L itself. The
// segments of an accepted trial are those of the next step, so each step
// evaluates the path once per trial.
template <int NO>
__device__ __forceinline__ RefineOut refine64(const Geo64<NO>& G, double* t,
                                              const SolveArgs& A, bool quick,
                                              uint32_t& n_eval, uint32_t& n_solve) {
  RefineOut o{false, false, true};
  // the last two Newton steps: each taken in full and moving no point by more
  // than the certificate radius
  const double cert2 = (double)A.cert_abs * (double)A.cert_abs;
  bool prev_small = false, last_small = false;
  // quick: only the last level, with quick_steps steps
  const int lv0 = quick ? A.n_levels - 1 : 0;
  for (int lv = lv0; lv < A.n_levels; ++lv) {
    double eps = (double)A.level_eps[lv] * (double)A.scale;
    double eps2 = eps * eps;
    const int nsteps = quick ? A.quick_steps : A.level_steps[lv];
    Seg64<NO> cur;
    eval64<NO>(G, t, eps2, cur);
    ++n_eval;
    for (int st = 0; st < nsteps; ++st) {
      double g[2 * NO], d[2 * NO];
      gradient64<NO>(G, cur.v, g);
#pragma unroll
      for (int k = 0; k < 2 * NO; ++k) g[k] = -g[k];
      const double bound = cur.L + 1e-15 * fabs(cur.L);
      const bool ok = hess_solve64<NO>(G, cur.v, cur.il, g, d);
      ++n_solve;
      prev_small = last_small;
      last_small = false;
      if (!ok) continue;
      const double d2 = max_disp64<NO>(G, d);
      double s = 1.0;
      bool acc = false;
      for (int h = 0; h < 7; ++h) {
        double tn[2 * NO];
#pragma unroll
        for (int k = 0; k < 2 * NO; ++k) tn[k] = fma(s, d[k], t[k]);
        Seg64<NO> nx;
        eval64<NO>(G, tn, eps2, nx);
        ++n_eval;
        if (nx.L <= bound) {
#pragma unroll
          for (int k = 0; k < 2 * NO; ++k) t[k] = tn[k];
          cur = nx;
          acc = true;
          break;
        }
        s *= 0.25;
      }
      // (the segments at t are not kept across the trials: recomputed here
      // in the rare case that every trial failed)
      if (!acc) {
        eval64<NO>(G, t, eps2, cur);
        ++n_eval;
      }
      last_small = acc && (s == 1.0) && (d2 <= cert2);
      o.refined = o.refined || acc;
    }
  }
  // One small full step is not enough: along a nearly flat valley of the
  // length a Newton step taken from well outside its quadratic region can be
  // short and still leave the point far from the minimiser (the next step
  // then jumps). Two consecutive small full steps are required.
  o.certified = A.n_levels > 0 && prev_small && last_small;
  if (o.certified) {
    // Nonsmooth check. At the smoothed optimum v_i = r_i / l_i plays the role
    // of the subgradient of |r_i|: a genuine collapse (r_i -> 0) has |v_i|
    // bounded away from 1, while a short segment with |v_i| close to 1 is a
    // degenerate configuration in which the length is nearly flat along the
    // segment and the smoothing can pull the points together. Such a path is
    // not certified.
    const double eps = (double)A.level_eps[A.n_levels - 1] * (double)A.scale;
    const double short2 = 1e-6 * (double)A.scale * (double)A.scale;  // (1e-3 S)^2
    double x[NO][3];
    points64<NO>(G, t, x);
#pragma unroll
    for (int i = 0; i <= NO; ++i) {
      double r[3];
#pragma unroll
      for (int c = 0; c < 3; ++c)
        r[c] = ((i == NO) ? G.rx[c] : x[i][c]) - ((i == 0) ? G.tx[c] : x[i - 1][c]);
      // |v_i|^2 = q / (q + eps^2) > 0.98^2
      double q = dot3d(r, r);
      if (q < short2 && q > (0.98 * 0.98) * (q + eps * eps)) o.certified = false;
    }
  }
  return o;
}

// ------------------------------------------------------------- kernel -----

// Per-lane FP32 state of the BFGS iteration.
template <int NO>
struct State32 {
  static constexpr int M = 2 * NO;
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
  int32_t s = A.src[p], e = A.dst[p];
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
    int32_t k = A.ids[(int64_t)j * A.N + p];
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
    if (A.t_init) {
      // to unit-vector coordinates: that = t * |a|
      u0 = A.t_init[(int64_t)(2 * j) * A.N + p] * rcp32(i1);
      u1 = edge ? 0.f : A.t_init[(int64_t)(2 * j + 1) * A.N + p] * rcp32(i2);
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
template <int NO>
__device__ __forceinline__ void init_state(const Geo32<NO>& G,
                                           const float (*t0)[2],
                                           State32<NO>& S) {
  constexpr int M = State32<NO>::M, HP = State32<NO>::HP;
#pragma unroll
  for (int j = 0; j < NO; ++j) {
    S.T[2 * j] = t0[j][0];
    S.T[2 * j + 1] = t0[j][1];
  }
  set_identity<M, HP>(S.H);
  grad32<NO>(G, S.T, S.g, S.r, S.l2, S.il);
#pragma unroll
  for (int k = 0; k < M; ++k) S.P[k] = -S.g[k];
}

// One BFGS iteration (Sec. III-C): step size by the fixed-point iteration of
// Eq. 6 (from the unit step, with the majorant step from 0 as fallback),
// step, new gradient, inverse-Hessian update. Returns the squared largest
// point displacement of the step.
template <int NO>
__device__ __forceinline__ float bfgs_iter(const Geo32<NO>& G, State32<NO>& S,
                                           int fp_iters) {
  constexpr int M = State32<NO>::M, HP = State32<NO>::HP;
  // direction in point space: q_j = A_j p_j; segment change D_i
  float q[NO][3];
#pragma unroll
  for (int j = 0; j < NO; ++j)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      q[j][c] = fmaf(S.P[2 * j + 1], G.a[j][1][c], S.P[2 * j] * G.a[j][0][c]);
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
  // Eq. 6 iterated from the unit step
  float alpha = 1.f;
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
  // step, new gradient
  float s[M], gn[M];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    s[k] = alpha * S.P[k];
    S.T[k] += s[k];
  }
  grad32<NO>(G, S.T, gn, S.r, S.l2, S.il);
  // BFGS inverse update (Nocedal & Wright eq. 6.17), with
  // H y = H g' - H g = H g' + P
  float Hg[M], Hy[M], y[M];
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

// hands a path over to the refinement kernel: unit-vector parameters,
// iteration count, validity
template <int NO>
__device__ __forceinline__ void store_phase1(const SolveArgs& A, int64_t p,
                                             const State32<NO>& S, int it,
                                             bool valid) {
#pragma unroll
  for (int k = 0; k < 2 * NO; ++k) A.t[(int64_t)k * A.N + p] = S.T[k];
  A.iters[p] = (uint16_t)(it > 65535 ? 65535 : it);
  A.status[p] = valid ? 0 : FPT_ST_INVALID;
}

// Phase 1, fixed iteration count (Sec. III-C runs every path for the same
// number of iterations so that all lanes finish together).
template <int NO>
__global__ __launch_bounds__(kBlock) void bfgs_kernel(
    SolveArgs A, const int32_t* __restrict__ perm,
    const int64_t* __restrict__ bucket) {
  int64_t begin = 0, count = A.N;
  if (bucket) {
    begin = bucket[NO - 1];
    count = bucket[NO] - begin;
  }
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < count;
       idx += stride) {
    const int64_t p = perm ? (int64_t)perm[begin + idx] : idx;
    Geo32<NO> G;
    float t0[NO][2];
    bool valid = load_path32<NO>(A, p, G, t0);
    State32<NO> S;
    init_state<NO>(G, t0, S);
    for (int it = 0; it < A.n_iter; ++it) bfgs_iter<NO>(G, S, A.fp_iters);
    store_phase1<NO>(A, p, S, A.n_iter, valid);
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
  } else if (bucket) {
    begin = bucket[NO - 1];
    count = bucket[NO] - begin;
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
                                 : (perm ? (int64_t)perm[begin + idx] : idx);
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
        float d2 = bfgs_iter<NO>(G, S, A.fp_iters);
        ++it;
        streak = (d2 <= A.exit_d2) ? streak + 1 : 0;
        done = streak >= 2 || it >= A.n_iter;
      }
    }
    const bool fin = done || !St.out_list || !valid;
    if (fin) store_phase1<NO>(A, p, S, it, valid);
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

// Phase 2: FP64 refinement of the parameters left by bfgs_kernel in A.t
// (unit-vector coordinates), certificate, and the final outputs.
// With quick_steps > 0 the refinement runs in two passes: the first takes
// quick_steps Newton steps at the last smoothing level for every path of the
// bucket and hands over the certified ones; the others are listed (by the
// same region scheme as the early-exit stages: St.out_list) and the second
// pass (St.in_list) runs the full schedule on them from the FP32 result.
// St.in_list == St.out_list == null: one pass with the full schedule.
template <int NO>
__global__ __launch_bounds__(kBlock) void refine_kernel(
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
  } else if (bucket) {
    begin = bucket[NO - 1];
    count = bucket[NO] - begin;
  }
  const bool quick = St.out_list != nullptr;
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  const float qnan = __builtin_nanf("");
  uint32_t n_eval = 0, n_solve = 0;
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
      p = perm ? (int64_t)perm[begin + idx] : idx;
    }
    const bool valid = (A.status[p] & FPT_ST_INVALID) == 0;
    Geo64<NO> D;
    float inv[NO][2];
    load_geo64<NO>(A, p, D, inv);
    double td[2 * NO];
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      float t0 = A.t[(int64_t)(2 * j) * A.N + p];
      float t1 = A.t[(int64_t)(2 * j + 1) * A.N + p];
      td[2 * j] = (double)t0 * (double)inv[j][0];
      td[2 * j + 1] = D.edge[j] ? 0.0 : (double)t1 * (double)inv[j][1];
    }
    RefineOut ro = refine64<NO>(D, td, A, quick, n_eval, n_solve);
    // first pass: defer the paths it does not certify
    const bool defer = quick && valid && !ro.certified;
    const unsigned long long more = __ballot(defer);
    if (more) {
      const int region = (int)((idx >> 6) % kRegions);
      unsigned long long base = 0;
      if (lane == 0)
        base = atomicAdd(St.out_count + region * kCounterStride,
                         (unsigned long long)__popcll(more));
      base = __shfl(base, 0);
      if (defer)
        St.out_list[(int64_t)region * St.rcap +
                    (int64_t)(base + (unsigned long long)__popcll(more & below))] = (int32_t)p;
    }
    if (defer) continue;
    double xs[NO][3];
    points64<NO>(D, td, xs);
    double Lx = 0.0, minl2 = INFINITY;
#pragma unroll
    for (int i = 0; i <= NO; ++i) {
      double rr[3];
#pragma unroll
      for (int c = 0; c < 3; ++c)
        rr[c] = ((i == NO) ? D.rx[c] : xs[i][c]) - ((i == 0) ? D.tx[c] : xs[i - 1][c]);
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
      if (ro.certified && finite) st |= FPT_ST_CONVERGED;
      if (ro.refined) st |= FPT_ST_REFINED;
      if (minl2 < cs * cs) st |= FPT_ST_COLLAPSED;
      if (!finite) st |= FPT_ST_NONFINITE;
    }
#pragma unroll
    for (int j = 0; j < NO; ++j) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
        A.x[(int64_t)(3 * j + c) * A.N + p] = valid ? (float)xs[j][c] : qnan;
      A.t[(int64_t)(2 * j) * A.N + p] = valid ? (float)td[2 * j] : qnan;
      A.t[(int64_t)(2 * j + 1) * A.N + p] = valid ? (float)td[2 * j + 1] : qnan;
    }
    for (int j = NO; j < A.n_max; ++j) {
#pragma unroll
      for (int c = 0; c < 3; ++c) A.x[(int64_t)(3 * j + c) * A.N + p] = qnan;
      A.t[(int64_t)(2 * j) * A.N + p] = qnan;
      A.t[(int64_t)(2 * j + 1) * A.N + p] = qnan;
    }
    A.len[p] = valid ? (float)Lx : qnan;
    A.status[p] = st;
  }
  if (A.work) {
    // wave sums, one atomic per wave
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      n_eval += __shfl_xor(n_eval, off);
      n_solve += __shfl_xor(n_solve, off);
    }
    if (lane == 0) {
      atomicAdd(A.work, (unsigned long long)n_eval);
      atomicAdd(A.work + 1, (unsigned long long)n_solve);
    }
  }
}

// ------------------------------------------------------ order bucketing ---
// A counting sort of the path indices by order, without global atomics:
// (1) each workgroup counts the orders of its chunk of kSortChunk paths,
// (2) one workgroup turns the per-chunk counts into per-chunk output
//     offsets (bucket of order n first for n = 1..n_max, invalid orders
//     last), (3) each workgroup scatters its chunk in input order.
// bucket[n-1] .. bucket[n] is the range of order n in perm;
// bucket[n_max] .. bucket[n_max+1] holds the paths with an invalid order.

__device__ __forceinline__ int order_bin(const uint8_t* order, int64_t i,
                                         int64_t N, int n_max) {
  if (i >= N) return -1;
  int o = order[i];
  return (o >= 1 && o <= n_max) ? o : 0;
}

__global__ __launch_bounds__(kBlock) void bucket_count_kernel(
    const uint8_t* __restrict__ order, int64_t N, int n_max,
    uint32_t* __restrict__ ccount) {
  __shared__ unsigned int loc[8];
  if (threadIdx.x < 8) loc[threadIdx.x] = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t c0 = (int64_t)blockIdx.x * kSortChunk;
  const int64_t c1 = min(N, c0 + (int64_t)kSortChunk);
  for (int64_t i0 = c0; i0 < c1; i0 += kBlock) {
    int b = order_bin(order, i0 + threadIdx.x, c1, n_max);
    for (int k = 0; k <= n_max; ++k) {
      unsigned long long m = __ballot(b == k);
      if (lane == 0 && m) atomicAdd(&loc[k], (unsigned int)__popcll(m));
    }
  }
  __syncthreads();
  if (threadIdx.x < 8) ccount[(int64_t)blockIdx.x * 8 + threadIdx.x] = loc[threadIdx.x];
}

// One workgroup: per-chunk offsets (in place over ccount) and bucket bounds.
__global__ __launch_bounds__(kBlock) void bucket_scan_kernel(
    uint32_t* __restrict__ ccount, int64_t nchunks, int n_max,
    int64_t* __restrict__ bucket) {
  __shared__ unsigned long long part[kBlock][8];
  __shared__ unsigned long long start[8];
  const int64_t per = (nchunks + kBlock - 1) / kBlock;
  const int64_t c0 = (int64_t)threadIdx.x * per;
  const int64_t c1 = min(nchunks, c0 + per);
  unsigned long long sum[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t c = c0; c < c1; ++c)
    for (int k = 0; k <= n_max; ++k) sum[k] += ccount[c * 8 + k];
  for (int k = 0; k < 8; ++k) part[threadIdx.x][k] = sum[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    // exclusive scan over threads, per bin; bin totals
    unsigned long long tot[8];
    for (int k = 0; k <= n_max; ++k) {
      unsigned long long acc = 0;
      for (int t = 0; t < kBlock; ++t) {
        unsigned long long v = part[t][k];
        part[t][k] = acc;
        acc += v;
      }
      tot[k] = acc;
    }
    unsigned long long acc = 0;
    bucket[0] = 0;
    for (int n = 1; n <= n_max; ++n) {
      start[n] = acc;
      acc += tot[n];
      bucket[n] = (int64_t)acc;
    }
    start[0] = acc;
    acc += tot[0];
    bucket[n_max + 1] = (int64_t)acc;
  }
  __syncthreads();
  unsigned long long run[8];
  for (int k = 0; k <= n_max; ++k) run[k] = start[k] + part[threadIdx.x][k];
  for (int64_t c = c0; c < c1; ++c)
    for (int k = 0; k <= n_max; ++k) {
      uint32_t v = ccount[c * 8 + k];
      ccount[c * 8 + k] = (uint32_t)run[k];
      run[k] += v;
    }
}

// Scatter: within a chunk, slices of 256 paths in order; inside a slice,
// wavefronts in order and lanes by rank (ballot + popcount): a stable sort.
__global__ __launch_bounds__(kBlock) void bucket_scatter_kernel(
    const uint8_t* __restrict__ order, int64_t N, int n_max,
    const uint32_t* __restrict__ coff, int32_t* __restrict__ perm) {
  __shared__ unsigned int run[8];
  __shared__ unsigned int wcnt[kBlock / 64][8];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  if (threadIdx.x < 8) run[threadIdx.x] = coff[(int64_t)blockIdx.x * 8 + threadIdx.x];
  __syncthreads();
  const int64_t c0 = (int64_t)blockIdx.x * kSortChunk;
  const int64_t c1 = min(N, c0 + (int64_t)kSortChunk);
  for (int64_t i0 = c0; i0 < c1; i0 += kBlock) {
    const int64_t i = i0 + threadIdx.x;
    const int b = order_bin(order, i, c1, n_max);
    unsigned int my_rank = 0;
    for (int k = 0; k <= n_max; ++k) {
      unsigned long long m = __ballot(b == k);
      if (lane == 0) wcnt[w][k] = (unsigned int)__popcll(m);
      if (b == k) my_rank = (unsigned int)__popcll(m & below);
    }
    __syncthreads();
    if (b >= 0) {
      unsigned int off = run[b] + my_rank;
      for (int v = 0; v < w; ++v) off += wcnt[v][b];
      perm[off] = (int32_t)i;
    }
    __syncthreads();
    if (threadIdx.x <= n_max) {
      unsigned int add = 0;
      for (int v = 0; v < kBlock / 64; ++v) add += wcnt[v][threadIdx.x];
      run[threadIdx.x] += add;
    }
    __syncthreads();
  }
}

// Paths with an order outside 1..n_max: NaN outputs, INVALID status.
__global__ __launch_bounds__(kBlock) void invalid_kernel(
    SolveArgs A, const int32_t* __restrict__ perm, const int64_t* __restrict__ bucket) {
  int64_t begin = bucket[A.n_max], count = bucket[A.n_max + 1] - begin;
  const float qnan = __builtin_nanf("");
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < count; idx += stride) {
    int64_t p = perm[begin + idx];
    for (int j = 0; j < A.n_max; ++j) {
      for (int c = 0; c < 3; ++c) A.x[(int64_t)(3 * j + c) * A.N + p] = qnan;
      A.t[(int64_t)(2 * j) * A.N + p] = qnan;
      A.t[(int64_t)(2 * j + 1) * A.N + p] = qnan;
    }
    A.len[p] = qnan;
    A.status[p] = FPT_ST_INVALID;
    A.iters[p] = 0;
  }
}

// ------------------------------------------------------------- launch -----

template <int NO>
static hipError_t launch_phase(int phase, const SolveArgs& A,
                               const int32_t* perm, const int64_t* bucket,
                               const StageArgs* stage, int grid,
                               hipStream_t st) {
  if (phase == 0)
    hipLaunchKernelGGL(bfgs_kernel<NO>, dim3(grid), dim3(kBlock), 0, st, A,
                       perm, bucket);
  else if (phase == 1)
    hipLaunchKernelGGL(refine_kernel<NO>, dim3(grid), dim3(kBlock), 0, st, A,
                       perm, bucket, *stage);
  else
    hipLaunchKernelGGL(bfgs_stage_kernel<NO>, dim3(grid), dim3(kBlock), 0,
                       st, A, perm, bucket, *stage);
  return hipGetLastError();
}

// phase 0: bfgs_kernel<order>, 1: refine_kernel<order>,
// 2: bfgs_stage_kernel<order> (one early-exit stage, `stage` describes it)
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
         : phase == 1 ? (const void*)refine_kernel<NO>
                      : (const void*)bfgs_stage_kernel<NO>;
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
                            hipStream_t st) {
  const int64_t nchunks = (N + kSortChunk - 1) / kSortChunk;
  hipLaunchKernelGGL(bucket_count_kernel, dim3((unsigned)nchunks), dim3(kBlock), 0, st,
                     order, N, n_max, ccount);
  hipLaunchKernelGGL(bucket_scan_kernel, dim3(1), dim3(kBlock), 0, st, ccount,
                     nchunks, n_max, bucket);
  hipLaunchKernelGGL(bucket_scatter_kernel, dim3((unsigned)nchunks), dim3(kBlock), 0, st,
                     order, N, n_max, ccount, perm);
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
