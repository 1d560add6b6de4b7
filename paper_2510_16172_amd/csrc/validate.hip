// Validity of solved paths on finite objects: the post-processing step after
// the solve, which Sec. III names (finite objects, obstruction) but does not
// study. The solver treats every object as its infinite plane or line; here
// a face is the parallelogram b + s a1 + u a2 (s, u in [0, 1]) and an edge
// the segment b + s a1 (s in [0, 1]). Per path, one lane, FP32:
//   EXTENT    every interaction parameter lies in [0, 1];
//   SPECULAR  at every face the previous and next points lie strictly on the
//             same side of its plane (else the minimiser passes through);
//   VISIBLE   no segment crosses a face of the scene other than the faces
//             of its own end points (edges occlude nothing).
#include <hip/hip_runtime.h>

#include "common.h"

namespace fpt {

// Compact face table (edges and degenerate faces left out: they occlude
// nothing), rows of [kFaceRows][K] floats for the F faces found:
//   0 c = b.n, 1-3 n = a1 x a2, 4-6 b, 7-9 pa = (a2 x n) / |n|^2,
//   10-12 pb = (n x a1) / |n|^2, 13 |a1| |a2|, 14 the object index.
// A point h of the plane has h - b = al a1 + be a2 with al = (h - b).pa and
// be = (h - b).pb. Also a [K] table of the normals of every object (0 for an
// edge), for the side test of a path's own objects. One workgroup.
constexpr int kFaceRows = 15;

__global__ __launch_bounds__(kBlock) void face_table_kernel(
    const float* __restrict__ obj, int32_t K, float* __restrict__ tab,
    float* __restrict__ nrm, int32_t* __restrict__ nfaces) {
  __shared__ int32_t wsum[kBlock / 64];
  __shared__ int32_t base;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int32_t k0 = 0; k0 < K; k0 += kBlock) {
    const int32_t k = k0 + threadIdx.x;
    float b[3] = {0.f, 0.f, 0.f}, u[3] = {0.f, 0.f, 0.f}, v[3] = {0.f, 0.f, 0.f};
    if (k < K) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        b[c] = obj[(int64_t)c * K + k];
        u[c] = obj[(int64_t)(3 + c) * K + k];
        v[c] = obj[(int64_t)(6 + c) * K + k];
      }
    }
    float n[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2],
                  u[0] * v[1] - u[1] * v[0]};
    const float nn = dot3(n, n);
    const bool face = k < K && nn > 0.f && isfinite(nn) && isfinite(dot3(b, b));
    if (k < K) {
#pragma unroll
      for (int c = 0; c < 3; ++c) nrm[(int64_t)c * K + k] = face ? n[c] : 0.f;
    }
    // rank of this face among the faces of the chunk
    const unsigned long long m = __ballot(face);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (lane == 0) wsum[wave] = __popcll(m);
    __syncthreads();
    int32_t off = base;
    for (int w = 0; w < wave; ++w) off += wsum[w];
    if (face) {
      const int32_t f = off + __popcll(m & below);
      const float inn = 1.f / nn;
      float pa[3] = {(v[1] * n[2] - v[2] * n[1]) * inn, (v[2] * n[0] - v[0] * n[2]) * inn,
                     (v[0] * n[1] - v[1] * n[0]) * inn};
      float pb[3] = {(n[1] * u[2] - n[2] * u[1]) * inn, (n[2] * u[0] - n[0] * u[2]) * inn,
                     (n[0] * u[1] - n[1] * u[0]) * inn};
      tab[f] = dot3(b, n);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        tab[(int64_t)(1 + c) * K + f] = n[c];
        tab[(int64_t)(4 + c) * K + f] = b[c];
        tab[(int64_t)(7 + c) * K + f] = pa[c];
        tab[(int64_t)(10 + c) * K + f] = pb[c];
      }
      tab[(int64_t)13 * K + f] = sqrtf(dot3(u, u)) * sqrtf(dot3(v, v));
      tab[(int64_t)14 * K + f] = __int_as_float(k);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int32_t t = 0;
      for (int w = 0; w < kBlock / 64; ++w) t += wsum[w];
      base += t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *nfaces = base;
}

// Does segment p -> q = p + d cross face f (interior of the segment: its
// parameter in (1e-6, 1 - 1e-6); face parameters in [0, 1])? pn = p.n and
// the side test come first, without a division, since most faces fail it.
// Segments parallel to the face's plane do not cross it.
__device__ __forceinline__ bool crosses(const float* p, const float* q,
                                        const float* d, float dlen,
                                        const float* __restrict__ tab,
                                        int32_t K, int32_t f) {
  const float c = tab[f];
  const float n0 = tab[(int64_t)1 * K + f], n1 = tab[(int64_t)2 * K + f],
              n2 = tab[(int64_t)3 * K + f];
  const float pn = fmaf(p[2], n2, fmaf(p[1], n1, p[0] * n0));
  const float qn = fmaf(q[2], n2, fmaf(q[1], n1, q[0] * n0));
  const float num = c - pn, den = qn - pn;   // s = num / den
  const bool in_s = (den > 0.f) ? (num > 1e-6f * den && num < (1.f - 1e-6f) * den)
                                : (num < 1e-6f * den && num > (1.f - 1e-6f) * den);
  if (!in_s) return false;
  if (!(fabsf(den) > 1e-12f * dlen * tab[(int64_t)13 * K + f])) return false;
  const float s = num / den;
  float al = 0.f, be = 0.f;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float h = fmaf(s, d[k], p[k]) - tab[(int64_t)(4 + k) * K + f];
    al = fmaf(h, tab[(int64_t)(7 + k) * K + f], al);
    be = fmaf(h, tab[(int64_t)(10 + k) * K + f], be);
  }
  return al >= 0.f && al <= 1.f && be >= 0.f && be <= 1.f;
}

// LDS: the face table is first copied into LDS (all lanes read the same
// face at a time: broadcast reads); else it is read from global memory.
template <int NO, bool LDS>
__global__ __launch_bounds__(kBlock) void validate_kernel(
    ValidateArgs A, const int32_t* __restrict__ perm,
    const int64_t* __restrict__ bucket) {
  extern __shared__ float sface[];
  const int32_t F = *A.nfaces;
  const float* tab = A.tab;
  if constexpr (LDS) {
    for (int r = 0; r < kFaceRows; ++r)
      for (int32_t f = threadIdx.x; f < F; f += kBlock)
        sface[(int64_t)r * A.K + f] = A.tab[(int64_t)r * A.K + f];
    __syncthreads();
    tab = sface;
  }
  int64_t begin = 0, count = A.N;
  if (bucket) {
    begin = bucket[NO - 1];
    count = bucket[NO] - begin;
  }
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < count;
       idx += stride) {
    const int64_t p = perm ? (int64_t)perm[begin + idx] : idx;
    const int32_t s0 = A.src[p], e0 = A.dst[p];
    bool ok = (A.status[p] & (FPT_ST_INVALID | FPT_ST_NONFINITE)) == 0 && s0 >= 0 &&
              s0 < A.Q && e0 >= 0 && e0 < A.Q;
    int32_t kid[NO];
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      kid[j] = A.ids[(int64_t)j * A.N + p];
      ok = ok && kid[j] >= 0 && kid[j] < A.K;
      kid[j] = ok ? kid[j] : 0;
    }
    // points: 0 = TX, 1..NO interactions, NO + 1 = RX
    float x[NO + 2][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[0][c] = A.pts[(int64_t)c * A.Q + (ok ? s0 : 0)];
      x[NO + 1][c] = A.pts[(int64_t)c * A.Q + (ok ? e0 : 0)];
    }
    bool extent = true, specular = true;
#pragma unroll
    for (int j = 0; j < NO; ++j) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        x[j + 1][c] = A.x[(int64_t)(3 * j + c) * A.N + p];
        ok = ok && isfinite(x[j + 1][c]);
      }
      float n[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) n[c] = A.nrm[(int64_t)c * A.K + kid[j]];
      const bool face = n[0] != 0.f || n[1] != 0.f || n[2] != 0.f;
      const float t0 = A.t[(int64_t)(2 * j) * A.N + p];
      const float t1 = A.t[(int64_t)(2 * j + 1) * A.N + p];
      extent = extent && t0 >= 0.f && t0 <= 1.f && (!face || (t1 >= 0.f && t1 <= 1.f));
    }
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      float n[3], di[3], dn[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        n[c] = A.nrm[(int64_t)c * A.K + kid[j]];
        di[c] = x[j][c] - x[j + 1][c];
        dn[c] = x[j + 2][c] - x[j + 1][c];
      }
      const bool face = n[0] != 0.f || n[1] != 0.f || n[2] != 0.f;
      const float a = dot3(n, di), b = dot3(n, dn);
      specular = specular && (!face || (a > 0.f && b > 0.f) || (a < 0.f && b < 0.f));
    }
    // occlusion: every segment against every face of the scene (the face
    // loop is the same for all lanes, so its table reads are wave-uniform)
    bool hit = false;
#pragma unroll
    for (int sgi = 0; sgi <= NO; ++sgi) {
      const int32_t own0 = sgi >= 1 ? kid[sgi > 0 ? sgi - 1 : 0] : -1;
      const int32_t own1 = sgi < NO ? kid[sgi < NO ? sgi : 0] : -1;
      float d[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) d[c] = x[sgi + 1][c] - x[sgi][c];
      const float dlen = sqrtf(dot3(d, d));
      for (int32_t f = 0; f < F; ++f) {
        if ((f & 15) == 0 && __all(hit)) break;
        const int32_t k = __float_as_int(tab[(int64_t)14 * A.K + f]);
        if (!hit && k != own0 && k != own1)
          hit = crosses(x[sgi], x[sgi + 1], d, dlen, tab, A.K, f);
      }
    }
    uint8_t fl = 0;
    if (ok) {
      fl = (extent ? FPT_VALID_EXTENT : 0) | (specular ? FPT_VALID_SPECULAR : 0) |
           (hit ? 0 : FPT_VALID_VISIBLE);
    }
    A.flags[p] = fl;
  }
}

// paths with an order outside 1..n_max (the last bucket): no flag
__global__ __launch_bounds__(kBlock) void validate_invalid_kernel(
    ValidateArgs A, const int32_t* __restrict__ perm,
    const int64_t* __restrict__ bucket) {
  const int64_t begin = bucket[A.n_max], end = bucket[A.n_max + 1];
  for (int64_t i = begin + (int64_t)blockIdx.x * kBlock + threadIdx.x; i < end;
       i += (int64_t)gridDim.x * kBlock)
    A.flags[perm[i]] = 0;
}

hipError_t launch_face_table(const float* obj, int32_t K, float* tab, float* nrm,
                             int32_t* nfaces, hipStream_t st) {
  hipLaunchKernelGGL(face_table_kernel, dim3(1), dim3(kBlock), 0, st, obj, K, tab, nrm,
                     nfaces);
  return hipGetLastError();
}

// LDS staging when the table (kFaceRows x K floats) fits in 64 KB
template <int NO>
static hipError_t launch_validate_n(const ValidateArgs& A, const int32_t* perm,
                                    const int64_t* bucket, int grid, hipStream_t st) {
  const size_t bytes = (size_t)kFaceRows * (size_t)A.K * sizeof(float);
  if (bytes <= 64 * 1024)
    hipLaunchKernelGGL((validate_kernel<NO, true>), dim3(grid), dim3(kBlock), bytes, st,
                       A, perm, bucket);
  else
    hipLaunchKernelGGL((validate_kernel<NO, false>), dim3(grid), dim3(kBlock), 0, st, A,
                       perm, bucket);
  return hipGetLastError();
}

hipError_t launch_validate(int order, const ValidateArgs& A, const int32_t* perm,
                           const int64_t* bucket, int grid, hipStream_t st) {
  switch (order) {
    case 1: return launch_validate_n<1>(A, perm, bucket, grid, st);
    case 2: return launch_validate_n<2>(A, perm, bucket, grid, st);
    case 3: return launch_validate_n<3>(A, perm, bucket, grid, st);
    case 4: return launch_validate_n<4>(A, perm, bucket, grid, st);
    case 5: return launch_validate_n<5>(A, perm, bucket, grid, st);
    case 6: return launch_validate_n<6>(A, perm, bucket, grid, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_validate_invalid(const ValidateArgs& A, const int32_t* perm,
                                   const int64_t* bucket, int grid, hipStream_t st) {
  hipLaunchKernelGGL(validate_invalid_kernel, dim3(grid), dim3(kBlock), 0, st, A, perm,
                     bucket);
  return hipGetLastError();
}

}  // namespace fpt
