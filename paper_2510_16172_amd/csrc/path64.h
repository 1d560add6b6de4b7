// Algebra of one path (device side): points, smoothed segments, gradient and
// the block-tridiagonal Newton solve. Written over the geometry's scalar type
// (GEO::real): FP64 for the refinement of the solver and the
// implicit-differentiation backward pass, FP32 for the exact-Hessian Newton
// variant of the first phase.
//
// Parametrisation (Sec. III-B, Eq. 3): x_j = b_j + t_j0 a1_j + t_j1 a2_j,
// with a2 = 0 for an edge (padding). Slot j = 0..n-1 is interaction j+1;
// segment i = 0..n runs from point i-1 to point i (point -1 = TX, point n =
// RX): slot j touches segment j (incoming) and segment j+1 (outgoing).
#pragma once

#include "common.h"

namespace fpt {

// The FP64 helpers below take the geometry of one path through accessors,
// so that it can live in registers (Geo64 in FP64, GeoF32 in FP32) or in LDS
// (GeoLds).
template <int NO>
struct Geo64 {
  static constexpr int kOrder = NO;
  using real = double;
  double tx_[3], rx_[3];
  double b_[NO][3];
  double a_[NO][2][3];  // caller's basis vectors (a[j][1] = 0 for an edge)
  bool edge_[NO];   // second parameter masked (padding)
  bool fixed_[NO];  // both parameters masked: a fixed point (reduced paths)
  __device__ __forceinline__ double tx(int c) const { return tx_[c]; }
  __device__ __forceinline__ double rx(int c) const { return rx_[c]; }
  __device__ __forceinline__ double b(int j, int c) const { return b_[j][c]; }
  __device__ __forceinline__ double a(int j, int k, int c) const { return a_[j][k][c]; }
  __device__ __forceinline__ bool edge(int j) const { return edge_[j]; }
  __device__ __forceinline__ bool fixed(int j) const { return fixed_[j]; }
};

// An FP32 value widened to FP64 behind an empty asm, which hides the value
// from the compiler: each use converts again instead of an FP64 copy staying
// live through the kernel (with the conversions merged, FP32 storage saves
// no registers). The gradient kernels gain from it; the refinement kernels,
// which use the geometry in every Newton step, lost 10-30 % to the extra
// conversions, also where it raised their occupancy, and keep FP64 copies.
__device__ __forceinline__ double widen(float v) {
  asm volatile("" : "+v"(v));
  return (double)v;
}

// Geometry of one lane in FP32 registers (the scene's values, exact in
// FP64), widened at each use.
template <int NO>
struct GeoF32 {
  static constexpr int kOrder = NO;
  using real = double;
  float tx_[3], rx_[3], b_[NO][3], a_[NO][2][3];
  bool edge_[NO];
  __device__ __forceinline__ double tx(int c) const { return widen(tx_[c]); }
  __device__ __forceinline__ double rx(int c) const { return widen(rx_[c]); }
  __device__ __forceinline__ double b(int j, int c) const { return widen(b_[j][c]); }
  __device__ __forceinline__ double a(int j, int k, int c) const { return widen(a_[j][k][c]); }
  __device__ __forceinline__ bool edge(int j) const { return edge_[j]; }
  __device__ __forceinline__ bool fixed(int) const { return false; }
};

// Path p's geometry from the tables, indices out of range clamped to 0 (the
// caller has flagged such a path invalid).
template <int NO>
__device__ __forceinline__ void load_geo_f32(const float* __restrict__ obj,
                                             const float* __restrict__ pts,
                                             const int32_t* __restrict__ ids, int32_t s,
                                             int32_t e, int32_t K, int32_t Q, int64_t N,
                                             int64_t p, GeoF32<NO>& D) {
  s = (s >= 0 && s < Q) ? s : 0;
  e = (e >= 0 && e < Q) ? e : 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    D.tx_[c] = pts[(int64_t)c * Q + s];
    D.rx_[c] = pts[(int64_t)c * Q + e];
  }
#pragma unroll
  for (int j = 0; j < NO; ++j) {
    int32_t k = ids[(int64_t)j * N + p];
    k = (k >= 0 && k < K) ? k : 0;
    float a2[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      D.b_[j][c] = obj[(int64_t)c * K + k];
      D.a_[j][0][c] = obj[(int64_t)(3 + c) * K + k];
      a2[c] = obj[(int64_t)(6 + c) * K + k];
    }
    const bool edge = (a2[0] == 0.f) && (a2[1] == 0.f) && (a2[2] == 0.f);
    D.edge_[j] = edge;
#pragma unroll
    for (int c = 0; c < 3; ++c) D.a_[j][1][c] = edge ? 0.f : a2[c];
  }
}

// Geometry of one lane in LDS: the FP32 scene values (exact in FP64, widened
// on use) in one column of a [geo_lds_rows(NO)][kBlock] float array, so that
// the FP64 kernels keep fewer live registers. Rows: TX, RX, then b, a1, a2
// per slot. (FP64 values in LDS would save the widening on each use, but
// double the array, which then limits how many workgroups of the other
// kernels share the CU.)
__host__ __device__ constexpr int geo_lds_rows(int NO) { return 6 + 9 * NO; }

template <int NO>
struct GeoLds {
  static constexpr int kOrder = NO;
  using real = double;
  const float* col;  // this lane's column: &lds[threadIdx.x]
  bool edge_[NO];
  __device__ __forceinline__ double tx(int c) const { return (double)col[c * kBlock]; }
  __device__ __forceinline__ double rx(int c) const { return (double)col[(3 + c) * kBlock]; }
  __device__ __forceinline__ double b(int j, int c) const {
    return (double)col[(6 + 9 * j + c) * kBlock];
  }
  __device__ __forceinline__ double a(int j, int k, int c) const {
    return (double)col[(9 + 9 * j + 3 * k + c) * kBlock];
  }
  __device__ __forceinline__ bool edge(int j) const { return edge_[j]; }
  __device__ __forceinline__ bool fixed(int) const { return false; }
};

// Loads of a GeoLds are not to be hoisted or merged across this point: it
// bounds how long the widened values stay in registers (no instruction).
__device__ __forceinline__ void geo_fence() { asm volatile("" ::: "memory"); }

// Geometry of path p in FP64 (exact widening of the FP32 tables). Indices out
// of range are clamped to 0 (the caller has flagged such a path invalid).
template <int NO>
__device__ __forceinline__ void load_geo64(const float* __restrict__ obj,
                                           const float* __restrict__ pts,
                                           const int32_t* __restrict__ ids,
                                           int32_t s, int32_t e, int32_t K,
                                           int32_t Q, int64_t N, int64_t p,
                                           Geo64<NO>& D) {
  s = (s >= 0 && s < Q) ? s : 0;
  e = (e >= 0 && e < Q) ? e : 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    D.tx_[c] = pts[(int64_t)c * Q + s];
    D.rx_[c] = pts[(int64_t)c * Q + e];
  }
#pragma unroll
  for (int j = 0; j < NO; ++j) {
    int32_t k = ids[(int64_t)j * N + p];
    k = (k >= 0 && k < K) ? k : 0;
    float a2[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      D.b_[j][c] = obj[(int64_t)c * K + k];
      D.a_[j][0][c] = obj[(int64_t)(3 + c) * K + k];
      a2[c] = obj[(int64_t)(6 + c) * K + k];
    }
    bool edge = (a2[0] == 0.f) && (a2[1] == 0.f) && (a2[2] == 0.f);
    D.edge_[j] = edge;
    D.fixed_[j] = false;
#pragma unroll
    for (int c = 0; c < 3; ++c) D.a_[j][1][c] = edge ? 0.0 : (double)a2[c];
  }
}

template <class GEO, class R = typename GEO::real>
__device__ __forceinline__ void points64(const GEO& G, const R* t, R (*x)[3]) {
  constexpr int NO = GEO::kOrder;
#pragma unroll
  for (int j = 0; j < NO; ++j)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      x[j][c] = fma(t[2 * j + 1], G.a(j, 1, c),
                    fma(t[2 * j], G.a(j, 0, c), G.b(j, c)));
}

// Segments at t: v_i = r_i / l_i and il_i = 1 / l_i with
// l_i = sqrt(|r_i|^2 + eps^2) (eps = 0: the exact length of Eq. 5).
template <class GEO, class R = typename GEO::real>
__device__ __forceinline__ void segments64(const GEO& G, const R* t, R eps2, R (*v)[3],
                                           R* il) {
  constexpr int NO = GEO::kOrder;
  R x[NO][3];
  points64(G, t, x);
#pragma unroll
  for (int i = 0; i <= NO; ++i) {
    R r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      r[c] = ((i == NO) ? G.rx(c) : x[i][c]) - ((i == 0) ? G.tx(c) : x[i - 1][c]);
    R q = fmax(dot3r(r, r) + eps2, RealTraits<R>::tiny);
    il[i] = rsqr(q);
#pragma unroll
    for (int c = 0; c < 3; ++c) v[i][c] = r[c] * il[i];
  }
}

// Segments of the (smoothed) length at t and the length itself.
template <int NO, class R = double>
struct Seg64 {
  R v[NO + 1][3], il[NO + 1], L;
};

template <class GEO, class R = typename GEO::real>
__device__ __forceinline__ void eval64(const GEO& G, const R* t, R eps2,
                                       Seg64<GEO::kOrder, R>& s) {
  constexpr int NO = GEO::kOrder;
  R x[NO][3];
  points64(G, t, x);
  s.L = R(0);
#pragma unroll
  for (int i = 0; i <= NO; ++i) {
    R r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      r[c] = ((i == NO) ? G.rx(c) : x[i][c]) - ((i == 0) ? G.tx(c) : x[i - 1][c]);
    R q = fmax(dot3r(r, r) + eps2, RealTraits<R>::tiny);
    s.il[i] = rsqr(q);
#pragma unroll
    for (int c = 0; c < 3; ++c) s.v[i][c] = r[c] * s.il[i];
    s.L += q * s.il[i];
  }
}

// Solves H d = rhs for the Hessian of the (smoothed) length, given the
// segments (v, il) at the current point. H is block tridiagonal with 2x2
// blocks (slot j couples only to j-1 and j+1):
//   D_j = A_j^T (M_j + M_{j+1}) A_j,  E_j = H_{j,j+1} = -A_j^T M_{j+1} A_{j+1},
//   M_i = (I - v_i v_i^T) / l_i  (the Hessian of l_i in r_i),
// and is solved by block-Thomas elimination (forward Schur complements
// S_j = D_j - E_{j-1}^T S_{j-1}^{-1} E_{j-1}, then back substitution).
// The padded parameter of an edge has a zero row and column in H; its
// diagonal is set to 1 and its right-hand side to 0, so its d is 0. A fixed
// slot has both parameters masked that way.
// With kNewton the right-hand side is minus the gradient of the length at
// the same segments (rhs is not read): g_j = A_j^T (v_j - v_{j+1}) is the
// difference of the projections of v_j and v_{j+1} on the object's directions,
// which the diagonal blocks need anyway.
// Returns false if a pivot block is not positive definite or d is not finite.
template <bool kNewton = false, class GEO, class R = typename GEO::real>
__device__ __forceinline__ bool hess_solve64(const GEO& G, const R (*v)[3], const R* il,
                                             const R* rhs, R* d) {
  constexpr int NO = GEO::kOrder;
  // kept for the back substitution d_j = y_j - W_j d_{j+1}:
  // W_j = S_j^{-1} E_j (rows: slot j's parameters) and y_j = S_j^{-1} z_j
  R W[NO][4], y[NO][2];
  R pW[4] = {0, 0, 0, 0}, pE[4] = {0, 0, 0, 0}, py[2] = {0, 0};
  bool ok = true;
#pragma unroll
  for (int j = 0; j < NO; ++j) {
    R a0[3], a1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      a0[c] = G.a(j, 0, c);
      a1[c] = G.a(j, 1, c);
    }
    R pin0 = dot3r(a0, v[j]), pin1 = dot3r(a1, v[j]);
    R pout0 = dot3r(a0, v[j + 1]), pout1 = dot3r(a1, v[j + 1]);
    R G00 = dot3r(a0, a0), G01 = dot3r(a0, a1), G11 = dot3r(a1, a1);
    R D00 = (G00 - pin0 * pin0) * il[j] + (G00 - pout0 * pout0) * il[j + 1];
    R D01 = (G01 - pin0 * pin1) * il[j] + (G01 - pout0 * pout1) * il[j + 1];
    R D11 = (G11 - pin1 * pin1) * il[j] + (G11 - pout1 * pout1) * il[j + 1];
    R rhs0, rhs1;
    if constexpr (kNewton) {
      rhs0 = pout0 - pin0;
      rhs1 = pout1 - pin1;
    } else {
      rhs0 = rhs[2 * j];
      rhs1 = rhs[2 * j + 1];
    }
    if (G.edge(j)) {
      D01 = R(0);
      D11 = R(1);
      rhs1 = R(0);
    }
    if (G.fixed(j)) {
      D00 = R(1);
      D01 = R(0);
      rhs0 = R(0);
    }
    if (j > 0) {
      // S_j = D_j - E_{j-1}^T W_{j-1},  z_j = rhs_j - E_{j-1}^T y_{j-1}
      D00 -= pE[0] * pW[0] + pE[2] * pW[2];
      D01 -= pE[0] * pW[1] + pE[2] * pW[3];
      D11 -= pE[1] * pW[1] + pE[3] * pW[3];
      rhs0 -= pE[0] * py[0] + pE[2] * py[1];
      rhs1 -= pE[1] * py[0] + pE[3] * py[1];
    }
    R det = D00 * D11 - D01 * D01;
    ok = ok && (det > R(0)) && (D00 > R(0)) && isfinite(det);
    R idet = rcpr(det);
    const R S0 = D11 * idet, S1 = -D01 * idet, S2 = D00 * idet;  // S_j^{-1}
    y[j][0] = S0 * rhs0 + S1 * rhs1;
    y[j][1] = S1 * rhs0 + S2 * rhs1;
    R E[4] = {R(0), R(0), R(0), R(0)};
    if (j + 1 < NO) {
      R b0[3], b1[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        b0[c] = G.a(j + 1, 0, c);
        b1[c] = G.a(j + 1, 1, c);
      }
      R qn0 = dot3r(b0, v[j + 1]), qn1 = dot3r(b1, v[j + 1]);
      R il1 = il[j + 1];
      E[0] = -(dot3r(a0, b0) - pout0 * qn0) * il1;
      E[1] = -(dot3r(a0, b1) - pout0 * qn1) * il1;
      E[2] = -(dot3r(a1, b0) - pout1 * qn0) * il1;
      E[3] = -(dot3r(a1, b1) - pout1 * qn1) * il1;
      if (G.edge(j)) E[2] = E[3] = R(0);
      if (G.edge(j + 1)) E[1] = E[3] = R(0);
      if (G.fixed(j)) E[0] = E[1] = R(0);
      if (G.fixed(j + 1)) E[0] = E[2] = R(0);
    }
    W[j][0] = S0 * E[0] + S1 * E[2];
    W[j][1] = S0 * E[1] + S1 * E[3];
    W[j][2] = S1 * E[0] + S2 * E[2];
    W[j][3] = S1 * E[1] + S2 * E[3];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      pW[k] = W[j][k];
      pE[k] = E[k];
    }
    py[0] = y[j][0];
    py[1] = y[j][1];
  }
  R n0 = R(0), n1 = R(0);
#pragma unroll
  for (int j = NO - 1; j >= 0; --j) {
    R d0 = y[j][0] - (W[j][0] * n0 + W[j][1] * n1);
    R d1 = y[j][1] - (W[j][2] * n0 + W[j][3] * n1);
    if (G.edge(j)) d1 = R(0);
    if (G.fixed(j)) d0 = R(0);
    d[2 * j] = d0;
    d[2 * j + 1] = d1;
    n0 = d0;
    n1 = d1;
    ok = ok && isfinite(d0) && isfinite(d1);
  }
  return ok;
}

// The KKT system of a collapsed minimiser, [H C^T; C 0] [lam; nu] = [w; 0],
// for the constraint x_{z-1} = x_z (C v = A_{z-1} v_{z-1} - A_z v_z), with
// segment z left out of H (il[z] = 0, so H splits into two chains at z).
// One block-Thomas forward elimination as in hess_solve64 carries four
// right-hand sides: w and the three columns C^T e_k (nonzero at slots z-1
// and z only). A first back substitution of the three columns accumulates
// the Schur complement S = C H^{-1} C^T and r = C H^{-1} w (r_k =
// (H^{-1} C^T e_k) . w, H being symmetric) without keeping the solutions;
// nu = S^{-1} r. The forward results are linear in the right-hand side, so
// the second back substitution starts from y_w - sum_k nu_k y_k and gives
// lam = H^{-1} (w - C^T nu) directly.
// Returns false if a pivot block is not positive definite, S is singular or
// a value is not finite.
template <class GEO, class R = typename GEO::real>
__device__ __forceinline__ bool kkt_solve64(const GEO& G, const R (*v)[3], const R* il,
                                            const R* w, int z, R* lam, R (&nu)[3]) {
  constexpr int NO = GEO::kOrder;
  R W[NO][4], y[NO][4][2];  // right-hand sides: 0..2 the columns, 3 w
  R pW[4] = {0, 0, 0, 0}, pE[4] = {0, 0, 0, 0};
  R py[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  bool ok = true;
#pragma unroll
  for (int j = 0; j < NO; ++j) {
    R a0[3], a1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      a0[c] = G.a(j, 0, c);
      a1[c] = G.a(j, 1, c);
    }
    R pin0 = dot3r(a0, v[j]), pin1 = dot3r(a1, v[j]);
    R pout0 = dot3r(a0, v[j + 1]), pout1 = dot3r(a1, v[j + 1]);
    R G00 = dot3r(a0, a0), G01 = dot3r(a0, a1), G11 = dot3r(a1, a1);
    R D00 = (G00 - pin0 * pin0) * il[j] + (G00 - pout0 * pout0) * il[j + 1];
    R D01 = (G01 - pin0 * pin1) * il[j] + (G01 - pout0 * pout1) * il[j + 1];
    R D11 = (G11 - pin1 * pin1) * il[j] + (G11 - pout1 * pout1) * il[j + 1];
    const R sg = j == z - 1 ? R(1) : (j == z ? R(-1) : R(0));
    R rh[4][2];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      rh[k][0] = sg * a0[k];
      rh[k][1] = sg * a1[k];
    }
    rh[3][0] = w[2 * j];
    rh[3][1] = w[2 * j + 1];
    if (G.edge(j)) {
      D01 = R(0);
      D11 = R(1);
#pragma unroll
      for (int k = 0; k < 4; ++k) rh[k][1] = R(0);
    }
    if (G.fixed(j)) {
      D00 = R(1);
      D01 = R(0);
#pragma unroll
      for (int k = 0; k < 4; ++k) rh[k][0] = R(0);
    }
    if (j > 0) {
      D00 -= pE[0] * pW[0] + pE[2] * pW[2];
      D01 -= pE[0] * pW[1] + pE[2] * pW[3];
      D11 -= pE[1] * pW[1] + pE[3] * pW[3];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        rh[k][0] -= pE[0] * py[k][0] + pE[2] * py[k][1];
        rh[k][1] -= pE[1] * py[k][0] + pE[3] * py[k][1];
      }
    }
    R det = D00 * D11 - D01 * D01;
    ok = ok && (det > R(0)) && (D00 > R(0)) && isfinite(det);
    R idet = rcpr(det);
    const R S0 = D11 * idet, S1 = -D01 * idet, S2 = D00 * idet;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      y[j][k][0] = S0 * rh[k][0] + S1 * rh[k][1];
      y[j][k][1] = S1 * rh[k][0] + S2 * rh[k][1];
    }
    R E[4] = {R(0), R(0), R(0), R(0)};
    if (j + 1 < NO) {
      R b0[3], b1[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        b0[c] = G.a(j + 1, 0, c);
        b1[c] = G.a(j + 1, 1, c);
      }
      R qn0 = dot3r(b0, v[j + 1]), qn1 = dot3r(b1, v[j + 1]);
      R il1 = il[j + 1];
      E[0] = -(dot3r(a0, b0) - pout0 * qn0) * il1;
      E[1] = -(dot3r(a0, b1) - pout0 * qn1) * il1;
      E[2] = -(dot3r(a1, b0) - pout1 * qn0) * il1;
      E[3] = -(dot3r(a1, b1) - pout1 * qn1) * il1;
      if (G.edge(j)) E[2] = E[3] = R(0);
      if (G.edge(j + 1)) E[1] = E[3] = R(0);
      if (G.fixed(j)) E[0] = E[1] = R(0);
      if (G.fixed(j + 1)) E[0] = E[2] = R(0);
    }
    W[j][0] = S0 * E[0] + S1 * E[2];
    W[j][1] = S0 * E[1] + S1 * E[3];
    W[j][2] = S1 * E[0] + S2 * E[2];
    W[j][3] = S1 * E[1] + S2 * E[3];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      pW[k] = W[j][k];
      pE[k] = E[k];
      py[k][0] = y[j][k][0];
      py[k][1] = y[j][k][1];
    }
  }
  // the three columns: S and r
  R S[3][3], r[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r[k] = R(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) S[c][k] = R(0);
  }
  R n[3][2] = {{0, 0}, {0, 0}, {0, 0}};
#pragma unroll
  for (int j = NO - 1; j >= 0; --j) {
    const R sg = j == z - 1 ? R(1) : (j == z ? R(-1) : R(0));
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      R d0 = y[j][k][0] - (W[j][0] * n[k][0] + W[j][1] * n[k][1]);
      R d1 = y[j][k][1] - (W[j][2] * n[k][0] + W[j][3] * n[k][1]);
      if (G.edge(j)) d1 = R(0);
      if (G.fixed(j)) d0 = R(0);
      n[k][0] = d0;
      n[k][1] = d1;
      r[k] = fma(d0, w[2 * j], fma(d1, w[2 * j + 1], r[k]));
#pragma unroll
      for (int c = 0; c < 3; ++c)
        S[c][k] = fma(sg, fma(d1, G.a(j, 1, c), d0 * G.a(j, 0, c)), S[c][k]);
    }
  }
  // nu = S^{-1} r (adjugate; S is symmetric positive definite)
  {
    const R c00 = S[1][1] * S[2][2] - S[1][2] * S[2][1];
    const R c01 = S[1][2] * S[2][0] - S[1][0] * S[2][2];
    const R c02 = S[1][0] * S[2][1] - S[1][1] * S[2][0];
    const R det = S[0][0] * c00 + S[0][1] * c01 + S[0][2] * c02;
    ok = ok && fabs(det) > R(0) && isfinite(det);
    const R id = rcpr(det);
    const R i01 = (S[0][2] * S[2][1] - S[0][1] * S[2][2]);
    const R i02 = (S[0][1] * S[1][2] - S[0][2] * S[1][1]);
    const R i11 = (S[0][0] * S[2][2] - S[0][2] * S[2][0]);
    const R i12 = (S[0][2] * S[1][0] - S[0][0] * S[1][2]);
    const R i21 = (S[0][1] * S[2][0] - S[0][0] * S[2][1]);
    const R i22 = (S[0][0] * S[1][1] - S[0][1] * S[1][0]);
    nu[0] = (c00 * r[0] + i01 * r[1] + i02 * r[2]) * id;
    nu[1] = (c01 * r[0] + i11 * r[1] + i12 * r[2]) * id;
    nu[2] = (c02 * r[0] + i21 * r[1] + i22 * r[2]) * id;
  }
  // lam = H^{-1} (w - C^T nu): the same back substitution from the
  // combined forward results
  R m0 = R(0), m1 = R(0);
#pragma unroll
  for (int j = NO - 1; j >= 0; --j) {
    const R y0 = y[j][3][0] - (nu[0] * y[j][0][0] + nu[1] * y[j][1][0] + nu[2] * y[j][2][0]);
    const R y1 = y[j][3][1] - (nu[0] * y[j][0][1] + nu[1] * y[j][1][1] + nu[2] * y[j][2][1]);
    R d0 = y0 - (W[j][0] * m0 + W[j][1] * m1);
    R d1 = y1 - (W[j][2] * m0 + W[j][3] * m1);
    if (G.edge(j)) d1 = R(0);
    if (G.fixed(j)) d0 = R(0);
    lam[2 * j] = d0;
    lam[2 * j + 1] = d1;
    m0 = d0;
    m1 = d1;
    ok = ok && isfinite(d0) && isfinite(d1);
  }
  return ok && isfinite(nu[0]) && isfinite(nu[1]) && isfinite(nu[2]);
}

// The collapsed minimisers the implicit gradient covers (Sec. III-D extended
// to a minimiser with one zero-length segment): at the points x, exactly one
// segment shorter than sqrt(cs2), an interior one (between slots z - 1 and
// z), and the two objects' directions span space, so that the subgradient
// of the zero-length segment, and with it the multiplier of the constraint
// x_{z-1} = x_z, is unique. Returns z, or -1 (no gradient: several
// collapses, a point at TX or RX, two edges, or objects whose directions
// lie in one plane).
template <class GEO, class R = typename GEO::real>
__device__ __forceinline__ int single_collapse(const GEO& G, const R (*x)[3], R cs2) {
  constexpr int NO = GEO::kOrder;
  int nz = 0, z = -1;
#pragma unroll
  for (int i = 0; i <= NO; ++i) {
    R r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      r[c] = ((i == NO) ? G.rx(c) : x[i][c]) - ((i == 0) ? G.tx(c) : x[i - 1][c]);
    const bool zi = dot3r(r, r) < cs2;
    nz += zi ? 1 : 0;
    z = zi ? i : z;
  }
  if (nz != 1 || z <= 0 || z >= NO) return -1;
  // N = sum of v v^T / |v|^2 over both objects' directions: rank 3 iff they
  // span space (det 2 sin^2 of the angle between two planes)
  R N[3][3] = {{R(0), R(0), R(0)}, {R(0), R(0), R(0)}, {R(0), R(0), R(0)}};
#pragma unroll
  for (int j = 0; j < NO; ++j) {
    const bool in = j == z - 1 || j == z;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      R v[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) v[c] = G.a(j, k, c);
      const R n2 = dot3r(v, v);
      const R w = (in && n2 > R(0)) ? rcpr(n2) : R(0);
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int e = 0; e < 3; ++e) N[c][e] = fma(w * v[c], v[e], N[c][e]);
    }
  }
  const R det = N[0][0] * (N[1][1] * N[2][2] - N[1][2] * N[2][1]) -
                N[0][1] * (N[1][0] * N[2][2] - N[1][2] * N[2][0]) +
                N[0][2] * (N[1][0] * N[2][1] - N[1][1] * N[2][0]);
  return det > R(1e-3) ? z : -1;
}

}  // namespace fpt
