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
#include <hip/hip_runtime.h>

#include "common.h"
#include "path64.h"

namespace fpt {

constexpr uint8_t kSkip = FPT_ST_COLLAPSED | FPT_ST_INVALID | FPT_ST_NONFINITE;

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

// (three slots: the compiler's register choice lands two VGPRs above what
// three waves per SIMD allow; asked for three it fits them without spilling)
template <int NO, bool LDS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(NO == 3 ? 3 : 1)))
void grad_kernel(
    GradArgs A, const int32_t* __restrict__ perm,
    const int64_t* __restrict__ bucket) {
  extern __shared__ double sh[];  // [9K] object gradient, then [3Q] points
  constexpr bool lds = LDS;
  const int64_t nsh = 9 * (int64_t)A.K + 3 * (int64_t)A.Q;
  if (lds) {
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
  for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < count;
       idx += stride) {
    const int64_t p = perm ? (int64_t)perm[begin + idx] : idx;
    const int32_t s = A.src[p], e = A.dst[p];
    bool use = (A.status[p] & kSkip) == 0 && s >= 0 && s < A.Q && e >= 0 &&
               e < A.Q;
    if (A.order) use = use && (int)A.order[p] == NO;
    int32_t kid[NO];
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      kid[j] = A.ids[(int64_t)j * A.N + p];
      use = use && kid[j] >= 0 && kid[j] < A.K;
    }
    Geo64<NO> G;
    load_geo64<NO>(A.obj, A.pts, A.ids, s, e, A.K, A.Q, A.N, p, G);
    double t[2 * NO];
#pragma unroll
    for (int k = 0; k < 2 * NO; ++k) {
      t[k] = (double)A.t[(int64_t)k * A.N + p];
      use = use && isfinite(t[k]);
    }
#pragma unroll
    for (int j = 0; j < NO; ++j)
      if (G.edge(j)) t[2 * j + 1] = 0.0;
    double u[NO + 1][3], il[NO + 1];
    segments64(G, t, 0.0, u, il);
    const double gl = A.g_len ? (double)A.g_len[p] : 0.0;
    double gx[NO][3], w[2 * NO];
#pragma unroll
    for (int j = 0; j < NO; ++j) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
        gx[j][c] = A.g_x ? (double)A.g_x[(int64_t)(3 * j + c) * A.N + p] : 0.0;
      w[2 * j] = G.a(j, 0, 0) * gx[j][0] + G.a(j, 0, 1) * gx[j][1] + G.a(j, 0, 2) * gx[j][2];
      w[2 * j + 1] = G.a(j, 1, 0) * gx[j][0] + G.a(j, 1, 1) * gx[j][1] + G.a(j, 1, 2) * gx[j][2];
    }
    double lam[2 * NO];
    bool ok = hess_solve64(G, u, il, w, lam);
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
    const float z = 0.f;
    // endpoints
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float gtx = use ? (float)(-gl * u[0][c] + cseg[0][c]) : z;
      float grx = use ? (float)(gl * u[NO][c] - cseg[NO][c]) : z;
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
        gb[c] = gl * du[c] + gx[j][c] - (cseg[j][c] - cseg[j + 1][c]);
      }
      float val[9];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        val[c] = (float)gb[c];
        val[3 + c] = (float)(t[2 * j] * gb[c] - lam[2 * j] * du[c]);
        val[6 + c] = G.edge(j) ? 0.f
                               : (float)(t[2 * j + 1] * gb[c] - lam[2 * j + 1] * du[c]);
      }
#pragma unroll
      for (int r = 0; r < 9; ++r) {
        float vv = use ? val[r] : z;
        if (A.g_slot) A.g_slot[(int64_t)(9 * j + r) * A.N + p] = vv;
        if (use) acc_add<LDS>(s_obj, A.g_obj, (int64_t)r * A.K + kid[j], vv);
      }
    }
    if (A.g_slot)
      for (int j = NO; j < A.n_max; ++j)
        for (int r = 0; r < 9; ++r) A.g_slot[(int64_t)(9 * j + r) * A.N + p] = z;
  }
  if (lds) {
    __syncthreads();
    for (int64_t i = threadIdx.x; i < 9 * (int64_t)A.K; i += kBlock)
      if (s_obj[i] != 0.0) unsafeAtomicAdd(A.g_obj + i, (float)s_obj[i]);
    for (int64_t i = threadIdx.x; i < 3 * (int64_t)A.Q; i += kBlock)
      if (s_pts[i] != 0.0) unsafeAtomicAdd(A.g_pts + i, (float)s_pts[i]);
  }
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
                                    const int64_t* bucket, int grid,
                                    size_t shmem, hipStream_t st) {
  if (A.lds)
    hipLaunchKernelGGL((grad_kernel<NO, true>), dim3(grid), dim3(kBlock), shmem, st, A,
                       perm, bucket);
  else
    hipLaunchKernelGGL((grad_kernel<NO, false>), dim3(grid), dim3(kBlock), shmem, st, A,
                       perm, bucket);
  return hipGetLastError();
}

hipError_t launch_grad(int order, const GradArgs& A, const int32_t* perm,
                       const int64_t* bucket, int grid, size_t shmem,
                       hipStream_t st) {
  switch (order) {
    case 1: return launch_grad_order<1>(A, perm, bucket, grid, shmem, st);
    case 2: return launch_grad_order<2>(A, perm, bucket, grid, shmem, st);
    case 3: return launch_grad_order<3>(A, perm, bucket, grid, shmem, st);
    case 4: return launch_grad_order<4>(A, perm, bucket, grid, shmem, st);
    case 5: return launch_grad_order<5>(A, perm, bucket, grid, shmem, st);
    case 6: return launch_grad_order<6>(A, perm, bucket, grid, shmem, st);
  }
  return hipErrorInvalidValue;
}

// The LDS-table kernel of an order (for the occupancy query).
const void* grad_kernel_ptr(int order) {
  switch (order) {
    case 1: return (const void*)grad_kernel<1, true>;
    case 2: return (const void*)grad_kernel<2, true>;
    case 3: return (const void*)grad_kernel<3, true>;
    case 4: return (const void*)grad_kernel<4, true>;
    case 5: return (const void*)grad_kernel<5, true>;
    case 6: return (const void*)grad_kernel<6, true>;
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
