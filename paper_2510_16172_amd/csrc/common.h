// Device-side helpers shared by the solver and the backward kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fpt.h"

namespace fpt {

constexpr int kBlock = 256;  // threads per workgroup: four wave64s
constexpr int kSortChunk = 8192;  // paths per workgroup in the order sort
constexpr int kRegions = 64;      // list regions of an early-exit stage
constexpr int kCounterStride = 16;
constexpr int kWorkSlots = 64;  // u64 counters 128 bytes apart

// Hardware reciprocal square root (v_rsq_f32), about 1 ulp.
__device__ __forceinline__ float rsq32(float x) {
  return __builtin_amdgcn_rsqf(x);
}
// Hardware reciprocal (v_rcp_f32), about 1 ulp.
__device__ __forceinline__ float rcp32(float x) {
  return __builtin_amdgcn_rcpf(x);
}

// FP64 reciprocal square root: the hardware estimate (v_rsq_f64) refined by
// two Newton-Raphson steps y <- y (3 - x y^2) / 2, each of which doubles the
// number of correct bits.
__device__ __forceinline__ double rsq64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

// FP64 reciprocal: hardware estimate refined by two Newton-Raphson steps
// y <- y (2 - x y).
__device__ __forceinline__ double rcp64(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * fma(-x, y, 2.0);
  y = y * fma(-x, y, 2.0);
  return y;
}

__device__ __forceinline__ float dot3(const float* a, const float* b) {
  return fmaf(a[2], b[2], fmaf(a[1], b[1], a[0] * b[0]));
}
__device__ __forceinline__ double dot3d(const double* a, const double* b) {
  return fma(a[2], b[2], fma(a[1], b[1], a[0] * b[0]));
}

// The path algebra of path64.h in either precision: reciprocal (square
// root) and dot product by type, the floor of a squared segment length, and
// the relative slack of a length comparison (a few rounding errors of L).
__device__ __forceinline__ float rsqr(float x) { return rsq32(x); }
__device__ __forceinline__ double rsqr(double x) { return rsq64(x); }
__device__ __forceinline__ float rcpr(float x) { return rcp32(x); }
__device__ __forceinline__ double rcpr(double x) { return rcp64(x); }
__device__ __forceinline__ float dot3r(const float* a, const float* b) { return dot3(a, b); }
__device__ __forceinline__ double dot3r(const double* a, const double* b) { return dot3d(a, b); }
template <class R>
struct RealTraits;
template <>
struct RealTraits<float> {
  static constexpr float tiny = 1e-30f, rel = 4e-7f;
};
template <>
struct RealTraits<double> {
  static constexpr double tiny = 1e-300, rel = 1e-15;
};

// Arguments shared by every launch of one fpt_solve call.
struct SolveArgs {
  const float* obj;
  const float* pts;
  const int32_t* src;
  const int32_t* dst;
  const uint8_t* order;
  const int32_t* ids;
  const float* t_init;
  float* x;
  float* len;
  float* t;
  uint8_t* status;
  uint16_t* iters;
  int64_t N;
  int32_t K, Q, n_max;
  // options
  int32_t n_iter, fp_iters, early_exit, method;
  int32_t polish_steps;  // FP32 Newton steps at the end of the BFGS phase
  int32_t line_search;   // FPT_LS_EQ6 or FPT_LS_ARMIJO (fixed-count BFGS)
  int32_t sub, nsub;     // this launch is part sub of nsub of its range (sub_range)
  float exit_d2;  // (exit_rtol * scale)^2
  float scale;
  int32_t n_levels;
  float level_eps[FPT_MAX_LEVELS];
  int32_t level_steps[FPT_MAX_LEVELS];
  float cert_abs;  // cert_rtol * scale
  int32_t quick_steps;  // > 0: two-pass refinement (see refine_kernel)
  int32_t pad_outputs;  // 1: write NaN to the entries beyond a path's order
                        // (0 in bucket order: the final copy writes them)
  // The first phase of a solve in bucket order (perm_in non-null): path
  // slot p's inputs are read from the caller's arrays at perm_in[p], and its
  // indices are copied to the bucket-order rows src_cp, dst_cp, ids_cp, which
  // the passes that follow read as src, dst, ids.
  const int32_t* perm_in;
  const int32_t* src_in;
  const int32_t* dst_in;
  const int32_t* ids_in;
  const float* tinit_in;
  int32_t* src_cp;
  int32_t* dst_cp;
  int32_t* ids_cp;
  // null, or the work counters of the launch's order (accounting while
  // timing): [4][kWorkSlots] FP64 path evaluations and Newton solves of
  // refine_kernel, then of merge_kernel's reduced paths; a wave adds to
  // slot blockIdx.x % kWorkSlots so that the atomics do not contend
  unsigned long long* work;
  // null, or clear_n counters that workgroup 0 of a first-phase launch
  // zeroes for the refinement passes that follow it on the same stream (in
  // place of a launch of its own)
  unsigned long long* clear;
  int32_t clear_n;
};

__device__ __forceinline__ void clear_counters(const SolveArgs& A) {
  if (A.clear && blockIdx.x == 0)
    for (int i = threadIdx.x; i < A.clear_n; i += kBlock) A.clear[i] = 0ull;
}

// One early-exit stage of the FP32 solver (see bfgs_stage_kernel).
struct StageArgs {
  const int32_t* in_list;               // null in the first stage
  const unsigned long long* in_count;   // kRegions counters, kCounterStride apart
  int32_t* out_list;                    // null in the last stage
  unsigned long long* out_count;
  const float* state_in;
  float* state_out;
  int64_t cap;                          // kRegions * rcap: state field stride
  int64_t rcap;                         // slots per region
  int32_t iters;
  int32_t mode;                         // collapse step: 0 after the quick
                                        // pass, 1 after the full schedule
};

// Arguments of one fpt_grad call.
struct GradArgs {
  const float* obj;
  const float* pts;
  const int32_t* src;
  const int32_t* dst;
  const uint8_t* order;
  const int32_t* ids;
  const float* t;         // forward T* [n_max][2][N] (caller's parametrisation)
  const uint8_t* status;  // forward status [N]
  const float* g_len;     // [N] or null
  const float* g_x;       // [n_max][3][N] or null
  float* g_pts;           // [3][Q] +=
  float* g_obj;           // [9][K] +=
  float* g_slot;          // [n_max][9][N] or null
  float* g_end;           // [6][N] or null
  int64_t N;
  int32_t K, Q, n_max;
  int32_t lds;            // accumulate per workgroup in LDS first
};

// Arguments of one fpt_validate call.
struct ValidateArgs {
  const float* obj;
  const float* pts;
  const int32_t* src;
  const int32_t* dst;
  const int32_t* ids;
  const float* x;         // forward X* [n_max][3][N]
  const float* t;         // forward T* [n_max][2][N] (caller's parametrisation)
  const uint8_t* status;  // forward status [N]
  const float* tab;       // compact face table [K][16] (face_table_kernel)
  const float* nrm;       // normals of every object [3][K] (0 for an edge)
  const int32_t* nfaces;  // number of faces in tab
  uint8_t* flags;         // [N]
  int64_t N;
  int32_t K, Q, n_max;
};

// Candidate enumeration (enumerate.hip)
struct EnumArgs {
  const int32_t* pair_src;
  const int32_t* pair_dst;
  int32_t* src;
  int32_t* dst;
  uint8_t* order;
  int32_t* ids;  // [n_max][count]
  int64_t rank0, count;
  int64_t first[FPT_NMAX + 1];  // first rank of order omin + i; first[omax - omin + 1] = total
  int64_t per_pair[FPT_NMAX + 1];  // sequences per pair of order n (index n)
  int32_t omin, omax, K, no_repeat, n_max;
};

}  // namespace fpt
