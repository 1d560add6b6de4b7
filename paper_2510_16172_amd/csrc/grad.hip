// Implicit-differentiation backward pass (Sec. III-D, Eqs. 8-13), one path
// per lane, FP64, at the solution left by fpt_solve.
//
// Loss: sum_i gl_i L*_i + sum_{i,j} gx_ij . x*_ij. With u_i = r_i / l_i,
// P_i = (I - u_i u_i^T) / l_i and the Hessian H = d grad_T L / dT at T*:
//  * the L* part is the envelope term: d L* / d theta = d L / d theta at T*
//    (the optimality condition of Eq. 8 removes the dT*/dtheta term);
//  * the X* part is the direct term (x_j = A_j t_j + b_j at fixed T) plus
//    w^T dT*/dtheta with w_j = A_j^T gx_j. By Eqs. 9-13 the latter equals
//    -lam^T d(grad_T L)/dtheta with H lam = w (H is symmetric; the paper's
//    u is -lam and its v is w). lam^T grad_T L = sum_i delta_i . u_i with
//    q_j = A_j lam_j, delta_i = q_i - q_{i-1} (q = 0 at TX and RX); its
//    derivative at fixed (T, lam) is lam_jk (u_j - u_{j+1}) on a_jk through
//    q_j, and c_i = P_i delta_i on r_i through u_i.
// Per path this gives, for slot j (segments j in, j+1 out):
//    g_TX  = -gl u_0 + c_0,      g_RX = gl u_n - c_n,
//    g_b_j = gl (u_j - u_{j+1}) + gx_j - (c_j - c_{j+1}),
//    g_a_jk = t_jk g_b_j - lam_jk (u_j - u_{j+1}).
// The paper obtains the mixed derivatives by automatic differentiation; here
// they are written out, so the kernel needs no tape and no iteration.
//
// A collapsed minimiser with one zero-length segment z (points z - 1 and z
// coincide; single_collapse) is the minimiser of L without that segment
// under the constraint c = x_{z-1} - x_z = 0, with multiplier mu = -w, w the
// subgradient of the zero-length segment (A_{z-1}^T (u_{z-1} - w) = 0,
// A_z^T (w - u_{z+1}) = 0). There:
//  * the L* part is the envelope term of the Lagrangian: the formulas above
//    with u_z replaced by w;
//  * the X* part solves the KKT system [H_s C^T; C 0] [lam; nu] = [w_T; 0]
//    (H_s the Hessian without segment z, C = dc/dT), by the Schur
//    complement: (C H_s^{-1} C^T) nu = C H_s^{-1} w_T, then
//    lam = H_s^{-1} (w_T - C^T nu); then the formulas above with u_z
//    replaced by w (that is the derivative of C^T mu) and c_z = 0, plus
//    -nu . dc/dtheta: -nu on g_b of slot z - 1 and +nu on g_b of slot z
//    (and t_jk times those on g_a through g_a = t g_b).
#include <hip/hip_runtime.h>

#include "common.h"
#include "path64.h"

namespace fpt {

// 3x3 solve by the adjugate (a symmetric positive definite M in use here);
// false if M is singular.
__device__ __forceinline__ bool solve3(const double (&M)[3][3], const double* b, double* x) {
  const double c00 = M[1][1] * M[2][2] - M[1][2] * M[2][1];
  const double c01 = M[1][2] * M[2][0] - M[1][0] * M[2][2];
  const double c02 = M[1][0] * M[2][1] - M[1][1] * M[2][0];
  const double det = M[0][0] * c00 + M[0][1] * c01 + M[0][2] * c02;
  if (!(fabs(det) > 0.0) || !isfinite(det)) return false;
  const double id = 1.0 / det;
  const double inv[3][3] = {
      {c00 * id, (M[0][2] * M[2][1] - M[0][1] * M[2][2]) * id, (M[0][1] * M[1][2] - M[0][2] * M[1][1]) * id},
      {c01 * id, (M[0][0] * M[2][2] - M[0][2] * M[2][0]) * id, (M[0][2] * M[1][0] - M[0][0] * M[1][2]) * id},
      {c02 * id, (M[0][1] * M[2][0] - M[0][0] * M[2][1]) * id, (M[0][0] * M[1][1] - M[0][1] * M[1][0]) * id}};
#pragma unroll
  for (int r = 0; r < 3; ++r) x[r] = inv[r][0] * b[0] + inv[r][1] * b[1] + inv[r][2] * b[2];
  return isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]);
}

// Accumulation into the workgroup's LDS tables (LDS) or straight into the
// global gradient. The tables are FP64: on gfx950 an LDS FP32 atomic add
// takes about 195 cycles per wave instruction whatever the addresses, an
// FP64 one about 29 (and the partial sums keep FP64 precision until the one
// flush to the FP32 gradient). The mode is a template parameter: chosen at
// run time inside one kernel, the two pointers would merge into one generic
// address and the LDS adds would become flat atomics.
template <bool LDS>
__device__ __forceinline__ void acc_add(double* lds_base, float* glob, int64_t idx,
                                        float v) {
  if (v == 0.f) return;
  if constexpr (LDS)
    atomicAdd(lds_base + idx, (double)v);
  else
    unsafeAtomicAdd(glob + idx, v);
}

// A collapsed minimiser that carries a gradient (the forward pass leaves
// FPT_ST_NOGRAD off only for the collapses single_collapse covers).
__device__ __forceinline__ bool kkt_path(uint8_t st) {
  return (st & FPT_ST_COLLAPSED) && !(st & FPT_ST_NOGRAD);
}

// The workgroup's FP64 tables into the FP32 gradients, once per workgroup.
__device__ __forceinline__ void flush_tables(const GradArgs& A, const double* sh) {
  __syncthreads();
  const double* s_obj = sh;
  const double* s_pts = sh + 9 * (int64_t)A.K;
  for (int64_t i = threadIdx.x; i < 9 * (int64_t)A.K; i += kBlock)
    if (s_obj[i] != 0.0) unsafeAtomicAdd(A.g_obj + i, (float)s_obj[i]);
  for (int64_t i = threadIdx.x; i < 3 * (int64_t)A.Q; i += kBlock)
    if (s_pts[i] != 0.0) unsafeAtomicAdd(A.g_pts + i, (float)s_pts[i]);
}

// One path's per-path inputs (everything but the scene tables), loaded
// ahead of its computation. They and the geometry are held in FP32 registers
// and widened at each use (GeoF32, widen): at three slots the smooth kernel
// needs 145 VGPRs instead of 168 with FP64 copies; at six, 247 instead of
// 256 plus spills, two waves per SIMD instead of one.
template <int NO>
struct PathIn {
  int64_t p;
  int32_t s, e, kid[NO];
  float t[2 * NO], gx[NO][3], gl;
  uint8_t st, ord;
};

template <int NO>
__device__ __forceinline__ void load_in(const GradArgs& A, int64_t p, PathIn<NO>& I) {
  I.p = p;
  I.st = A.status[p];
  I.ord = A.order ? A.order[p] : (uint8_t)NO;
  I.s = A.src[p];
  I.e = A.dst[p];
#pragma unroll
  for (int j = 0; j < NO; ++j) I.kid[j] = A.ids[(int64_t)j * A.N + p];
#pragma unroll
  for (int k = 0; k < 2 * NO; ++k) I.t[k] = A.t[(int64_t)k * A.N + p];
#pragma unroll
  for (int j = 0; j < NO; ++j)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      I.gx[j][c] = A.g_x ? A.g_x[(int64_t)(3 * j + c) * A.N + p] : 0.f;
  I.gl = A.g_len ? A.g_len[p] : 0.f;
}

// The geometry of a path whose inputs are loaded.
template <int NO>
__device__ __forceinline__ void load_geo_in(const GradArgs& A, const PathIn<NO>& I,
                                            GeoF32<NO>& D) {
  const int32_t s = (I.s >= 0 && I.s < A.Q) ? I.s : 0;
  const int32_t e = (I.e >= 0 && I.e < A.Q) ? I.e : 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    D.tx_[c] = A.pts[(int64_t)c * A.Q + s];
    D.rx_[c] = A.pts[(int64_t)c * A.Q + e];
  }
#pragma unroll
  for (int j = 0; j < NO; ++j) {
    const int32_t k = (I.kid[j] >= 0 && I.kid[j] < A.K) ? I.kid[j] : 0;
    float a2[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      D.b_[j][c] = A.obj[(int64_t)c * A.K + k];
      D.a_[j][0][c] = A.obj[(int64_t)(3 + c) * A.K + k];
      a2[c] = A.obj[(int64_t)(6 + c) * A.K + k];
    }
    const bool edge = (a2[0] == 0.f) && (a2[1] == 0.f) && (a2[2] == 0.f);
    D.edge_[j] = edge;
#pragma unroll
    for (int c = 0; c < 3; ++c) D.a_[j][1][c] = edge ? 0.f : a2[c];
  }
}

// One path's gradient: its per-path outputs and its adds to the object and
// point gradients. KKT: the path is a collapsed minimiser (the constrained
// form above); otherwise a smooth one.
template <int NO, bool LDS, bool KKT>
__device__ __forceinline__ void grad_path(const GradArgs& A, const PathIn<NO>& I,
                                          const GeoF32<NO>& G, double* s_obj, double* s_pts) {
  const int64_t p = I.p;
  const uint8_t stp = I.st;
  const int32_t s = I.s, e = I.e;
  // (no gradient: FPT_ST_NOGRAD, or a collapse where the smooth form runs)
  constexpr uint8_t kOff = KKT ? FPT_ST_NOGRAD : (FPT_ST_NOGRAD | FPT_ST_COLLAPSED);
  bool use = (stp & kOff) == 0 && s >= 0 && s < A.Q && e >= 0 && e < A.Q;
  use = use && (int)I.ord == NO;
  int32_t kid[NO];
#pragma unroll
  for (int j = 0; j < NO; ++j) {
    kid[j] = I.kid[j];
    use = use && kid[j] >= 0 && kid[j] < A.K;
  }
  float tf[2 * NO];
#pragma unroll
  for (int k = 0; k < 2 * NO; ++k) {
    tf[k] = I.t[k];
    use = use && isfinite(tf[k]);
  }
#pragma unroll
  for (int j = 0; j < NO; ++j)
    if (G.edge(j)) tf[2 * j + 1] = 0.f;
  double t[2 * NO];
#pragma unroll
  for (int k = 0; k < 2 * NO; ++k) t[k] = (double)tf[k];
  double u[NO + 1][3], il[NO + 1];
  segments64(G, t, 0.0, u, il);
  // a collapsed minimiser (one zero-length interior segment z): w in place
  // of u_z, segment z out of the Hessian
  int z = -1;
  if constexpr (KKT && NO >= 2) {
    if (use) {
      double best = INFINITY;
#pragma unroll
      for (int i = 1; i < NO; ++i) {
        const bool sm = il[i] > 0.0 && 1.0 / il[i] < best;
        best = sm ? 1.0 / il[i] : best;
        z = sm ? i : z;
      }
    }
  }
  const bool col = KKT && z > 0;
  if constexpr (KKT) use = use && col;
  if (col) {
    // w: least squares of A_{z-1}^T w = A_{z-1}^T u_{z-1}, A_z^T w = A_z^T u_{z+1}
    // (consistent at the minimiser; unique as the directions span space)
    double M[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, rb[3] = {0, 0, 0};
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      const bool in = j == z - 1, out = j == z;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        double v[3], uu[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          v[c] = (in || out) ? G.a(j, k, c) : 0.0;
          uu[c] = in ? u[j][c] : u[j + 1][c];
        }
        // (slot z - 1's incoming segment is z - 1 = j; slot z's outgoing
        // one is z + 1 = j + 1)
        const double pv = dot3d(v, uu);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          rb[c] = fma(v[c], pv, rb[c]);
#pragma unroll
          for (int e2 = 0; e2 < 3; ++e2) M[c][e2] = fma(v[c], v[e2], M[c][e2]);
        }
      }
    }
    double w3[3];
    use = use && solve3(M, rb, w3);
#pragma unroll
    for (int i = 0; i <= NO; ++i) {
      const bool zi = i == z;
#pragma unroll
      for (int c = 0; c < 3; ++c) u[i][c] = zi ? w3[c] : u[i][c];
      il[i] = zi ? 0.0 : il[i];
    }
  }
  const double gl = (double)I.gl;
  float gx[NO][3];
  double w[2 * NO];
#pragma unroll
  for (int j = 0; j < NO; ++j) {
#pragma unroll
    for (int c = 0; c < 3; ++c) gx[j][c] = I.gx[j][c];
    w[2 * j] = G.a(j, 0, 0) * widen(gx[j][0]) + G.a(j, 0, 1) * widen(gx[j][1]) + G.a(j, 0, 2) * widen(gx[j][2]);
    w[2 * j + 1] = G.a(j, 1, 0) * widen(gx[j][0]) + G.a(j, 1, 1) * widen(gx[j][1]) + G.a(j, 1, 2) * widen(gx[j][2]);
  }
  // (the solve runs on every lane: no branch around it)
  double lam[2 * NO], nu[3] = {0.0, 0.0, 0.0};
  bool ok;
  if constexpr (KKT)
    ok = kkt_solve64(G, u, il, w, z, lam, nu);
  else
    ok = hess_solve64(G, u, il, w, lam);
  use = use && ok;
  // c_i = P_i delta_i for every segment
  double cseg[NO + 1][3];
#pragma unroll
  for (int i = 0; i <= NO; ++i) {
    double dl[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double qi = (i == NO) ? 0.0
                            : lam[2 * i] * G.a(i, 0, c) + lam[2 * i + 1] * G.a(i, 1, c);
      double qm = (i == 0) ? 0.0
                           : lam[2 * i - 2] * G.a(i - 1, 0, c) +
                                 lam[2 * i - 1] * G.a(i - 1, 1, c);
      dl[c] = qi - qm;
    }
    double ud = dot3d(u[i], dl);
#pragma unroll
    for (int c = 0; c < 3; ++c) cseg[i][c] = (dl[c] - u[i][c] * ud) * il[i];
  }
  const float zf = 0.f;
  // endpoints
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float gtx = use ? (float)(-gl * u[0][c] + cseg[0][c]) : zf;
    float grx = use ? (float)(gl * u[NO][c] - cseg[NO][c]) : zf;
    if (A.g_end) {
      A.g_end[(int64_t)c * A.N + p] = gtx;
      A.g_end[(int64_t)(3 + c) * A.N + p] = grx;
    }
    if (use) {
      acc_add<LDS>(s_pts, A.g_pts, (int64_t)c * A.Q + s, gtx);
      acc_add<LDS>(s_pts, A.g_pts, (int64_t)c * A.Q + e, grx);
    }
  }
  // objects
#pragma unroll
  for (int j = 0; j < NO; ++j) {
    double du[3], gb[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      du[c] = u[j][c] - u[j + 1][c];
      gb[c] = gl * du[c] + widen(gx[j][c]) - (cseg[j][c] - cseg[j + 1][c]);
      // -nu . dc/db: c = x_{z-1} - x_z
      gb[c] += (j == z - 1) ? -nu[c] : ((j == z) ? nu[c] : 0.0);
    }
    float val[9];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      val[c] = (float)gb[c];
      val[3 + c] = (float)(widen(tf[2 * j]) * gb[c] - lam[2 * j] * du[c]);
      val[6 + c] = G.edge(j) ? 0.f
                             : (float)(widen(tf[2 * j + 1]) * gb[c] - lam[2 * j + 1] * du[c]);
    }
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      float vv = use ? val[r] : zf;
      if (A.g_slot) A.g_slot[(int64_t)(9 * j + r) * A.N + p] = vv;
      if (use) acc_add<LDS>(s_obj, A.g_obj, (int64_t)r * A.K + kid[j], vv);
    }
  }
  if (A.g_slot)
    for (int j = NO; j < A.n_max; ++j)
      for (int r = 0; r < 9; ++r) A.g_slot[(int64_t)(9 * j + r) * A.N + p] = zf;
}

// The paths of one order are split between two kernels: grad_kernel takes
// the smooth ones (and those without a gradient, which get zeros),
// grad_kkt_kernel the collapsed minimisers that carry a gradient (about a
// quarter of the paths of a dense scene, spread over all waves). The
// constrained solve would raise the registers of every path, so it has a
// kernel of its own. That kernel gathers its paths first: each workgroup
// scans 4 x 256 entries at a time (of the batch, or of the bucket of
// collapsed paths of a bucketed batch), appends its order's ones to a
// list in LDS (one atomic per wave: ballot and lane count) and runs the list
// in batches of 256, every lane busy; what is left over waits for the next
// scan, and the workgroup's last scan runs the rest. (The smooth kernel
// gains nothing from the same gathering: measured slower than leaving the
// collapsed lanes idle.)
constexpr int kScan = 4 * kBlock;

template <int NO, bool LDS>
__device__ __forceinline__ void run_kkt_list(const GradArgs& A,
                                             const int32_t* __restrict__ perm,
                                             const int64_t* __restrict__ bucket,
                                             int32_t* list, int32_t& n_list, double* sh) {
  const int64_t nsh = 9 * (int64_t)A.K + 3 * (int64_t)A.Q;
  if (LDS)
    for (int64_t i = threadIdx.x; i < nsh; i += kBlock) sh[i] = 0.0;
  double* s_obj = sh;
  double* s_pts = sh + 9 * (int64_t)A.K;
  // (bucketed: the bin of the collapsed minimisers of every order)
  int64_t begin = 0, count = A.N;
  if (bucket) {
    begin = bucket[A.n_max + 1];
    count = bucket[A.n_max + 2] - begin;
  }
  const int lane = threadIdx.x & 63;
  if (threadIdx.x == 0) n_list = 0;
  const int64_t step = (int64_t)gridDim.x * kScan;
  for (int64_t base = (int64_t)blockIdx.x * kScan; base < count; base += step) {
    __syncthreads();  // n_list and the carried entries are in place
#pragma unroll
    for (int r = 0; r < kScan / kBlock; ++r) {
      const int64_t idx = base + r * kBlock + threadIdx.x;
      int64_t p = 0;
      bool take = false;
      if (idx < count) {
        p = perm ? (int64_t)perm[begin + idx] : idx;
        take = kkt_path(A.status[p]) && (!A.order || (int)A.order[p] == NO);
      }
      const uint64_t m = __ballot(take);
      int at = 0;
      if (lane == 0 && m) at = atomicAdd(&n_list, (int)__popcll(m));
      at = __shfl(at, 0);
      if (take)
        list[at + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] =
            (int32_t)p;
    }
    __syncthreads();
    // (uniform: kept in a scalar register, away from the per-path VGPRs)
    const int n = __builtin_amdgcn_readfirstlane(n_list);
    const bool last = base + step >= count;
    const int full = last ? n : n / kBlock * kBlock;
    for (int i = threadIdx.x; i < full; i += kBlock) {
      PathIn<NO> I;
      load_in<NO>(A, list[i], I);
      GeoF32<NO> G;
      load_geo_in<NO>(A, I, G);
      grad_path<NO, LDS, true>(A, I, G, s_obj, s_pts);
    }
    // carry the rest (fewer than 256, at indices >= 256: no overlap)
    const int rest = n - full;
    int32_t keep = 0;
    if (threadIdx.x < rest) keep = list[full + threadIdx.x];
    __syncthreads();
    if (threadIdx.x < rest) list[threadIdx.x] = keep;
    if (threadIdx.x == 0) n_list = rest;
  }
  if (LDS) flush_tables(A, sh);
}

// (three slots: asked for three waves per SIMD, the compiler stays within
// their 168 VGPRs)
template <int NO, bool LDS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(NO == 3 ? 3 : 1)))
void grad_kernel(GradArgs A, const int32_t* __restrict__ perm,
                 const int64_t* __restrict__ bucket) {
  extern __shared__ double sh[];  // [9K] object gradient, then [3Q] points
  const int64_t nsh = 9 * (int64_t)A.K + 3 * (int64_t)A.Q;
  if (LDS) {
    for (int64_t i = threadIdx.x; i < nsh; i += kBlock) sh[i] = 0.0;
    __syncthreads();
  }
  double* s_obj = sh;
  double* s_pts = sh + 9 * (int64_t)A.K;
  int64_t begin = 0, count = A.N;
  if (bucket) {
    begin = bucket[NO - 1];
    count = bucket[NO] - begin;
  }
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if constexpr (NO >= 3 && NO <= 5) {
    // the next path's inputs are loaded while this one is computed (issued
    // after this one's geometry loads: the load counter drains in order).
    // At orders 3-5 the registers they take leave the waves per SIMD as
    // they are; at orders 1, 2 and 6 they would cost a wave and more time
    // than the overlap gains.
    PathIn<NO> nx;
    if (idx < count) load_in<NO>(A, perm ? (int64_t)perm[begin + idx] : idx, nx);
    for (; idx < count; idx += stride) {
      const PathIn<NO> cu = nx;
      GeoF32<NO> G;
      load_geo_in<NO>(A, cu, G);
      const int64_t i2 = idx + stride;
      if (i2 < count) load_in<NO>(A, perm ? (int64_t)perm[begin + i2] : i2, nx);
      if (kkt_path(cu.st)) continue;  // grad_kkt_kernel's
      grad_path<NO, LDS, false>(A, cu, G, s_obj, s_pts);
    }
  } else {
    for (; idx < count; idx += stride) {
      const int64_t p = perm ? (int64_t)perm[begin + idx] : idx;
      if (NO >= 2 && kkt_path(A.status[p])) continue;  // grad_kkt_kernel's
      PathIn<NO> cu;
      load_in<NO>(A, p, cu);
      GeoF32<NO> G;
      load_geo_in<NO>(A, cu, G);
      grad_path<NO, LDS, false>(A, cu, G, s_obj, s_pts);
    }
  }
  if (LDS) flush_tables(A, sh);
}

// (four and five slots: asked for two waves per SIMD, the kernel spills 36
// / 208 bytes where it took AGPRs beyond 256 registers and one wave; the
// pass ran 7 / 4 % faster)
template <int NO, bool LDS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu((NO == 4 || NO == 5) ? 2 : 1)))
void grad_kkt_kernel(
    GradArgs A, const int32_t* __restrict__ perm, const int64_t* __restrict__ bucket) {
  extern __shared__ double sh[];
  __shared__ int32_t list[kScan + kBlock];
  __shared__ int32_t n_list;
  run_kkt_list<NO, LDS>(A, perm, bucket, list, n_list, sh);
}

// Paths whose order is outside 1..n_max: zero per-path outputs.
__global__ __launch_bounds__(kBlock) void grad_invalid_kernel(
    GradArgs A, const int32_t* __restrict__ perm,
    const int64_t* __restrict__ bucket) {
  int64_t begin = bucket[A.n_max], count = bucket[A.n_max + 1] - begin;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < count;
       idx += stride) {
    int64_t p = perm[begin + idx];
    if (A.g_slot)
      for (int r = 0; r < 9 * A.n_max; ++r) A.g_slot[(int64_t)r * A.N + p] = 0.f;
    if (A.g_end)
      for (int r = 0; r < 6; ++r) A.g_end[(int64_t)r * A.N + p] = 0.f;
  }
}

template <int NO>
static hipError_t launch_grad_order(const GradArgs& A, const int32_t* perm,
                                    const int64_t* bucket, int grid, int kkt_grid,
                                    size_t shmem, hipStream_t st) {
  if (A.lds)
    hipLaunchKernelGGL((grad_kernel<NO, true>), dim3(grid), dim3(kBlock), shmem, st, A,
                       perm, bucket);
  else
    hipLaunchKernelGGL((grad_kernel<NO, false>), dim3(grid), dim3(kBlock), shmem, st, A,
                       perm, bucket);
  if constexpr (NO >= 2) {
    if (A.lds)
      hipLaunchKernelGGL((grad_kkt_kernel<NO, true>), dim3(kkt_grid), dim3(kBlock), shmem,
                         st, A, perm, bucket);
    else
      hipLaunchKernelGGL((grad_kkt_kernel<NO, false>), dim3(kkt_grid), dim3(kBlock), shmem,
                         st, A, perm, bucket);
  }
  return hipGetLastError();
}

hipError_t launch_grad(int order, const GradArgs& A, const int32_t* perm,
                       const int64_t* bucket, int grid, int kkt_grid, size_t shmem,
                       hipStream_t st) {
  switch (order) {
    case 1: return launch_grad_order<1>(A, perm, bucket, grid, kkt_grid, shmem, st);
    case 2: return launch_grad_order<2>(A, perm, bucket, grid, kkt_grid, shmem, st);
    case 3: return launch_grad_order<3>(A, perm, bucket, grid, kkt_grid, shmem, st);
    case 4: return launch_grad_order<4>(A, perm, bucket, grid, kkt_grid, shmem, st);
    case 5: return launch_grad_order<5>(A, perm, bucket, grid, kkt_grid, shmem, st);
    case 6: return launch_grad_order<6>(A, perm, bucket, grid, kkt_grid, shmem, st);
  }
  return hipErrorInvalidValue;
}

// The LDS-table kernels of an order (for the occupancy query): the smooth
// one, or (kkt) the collapsed one (nullptr at order 1, which has none).
const void* grad_kernel_ptr(int order, bool kkt) {
  switch (order) {
    case 1: return kkt ? nullptr : (const void*)grad_kernel<1, true>;
    case 2: return kkt ? (const void*)grad_kkt_kernel<2, true> : (const void*)grad_kernel<2, true>;
    case 3: return kkt ? (const void*)grad_kkt_kernel<3, true> : (const void*)grad_kernel<3, true>;
    case 4: return kkt ? (const void*)grad_kkt_kernel<4, true> : (const void*)grad_kernel<4, true>;
    case 5: return kkt ? (const void*)grad_kkt_kernel<5, true> : (const void*)grad_kernel<5, true>;
    case 6: return kkt ? (const void*)grad_kkt_kernel<6, true> : (const void*)grad_kernel<6, true>;
  }
  return nullptr;
}

hipError_t launch_grad_invalid(const GradArgs& A, const int32_t* perm,
                               const int64_t* bucket, int grid, hipStream_t st) {
  hipLaunchKernelGGL(grad_invalid_kernel, dim3(grid), dim3(kBlock), 0, st, A,
                     perm, bucket);
  return hipGetLastError();
}

}  // namespace fpt
