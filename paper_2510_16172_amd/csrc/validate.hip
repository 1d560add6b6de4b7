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
// nothing): one record of kFaceRec floats per face found,
//   0-2 n = a1 x a2, 3-5 b, 6-8 pa = (a2 x n) / |n|^2,
//   9-11 pb = (n x a1) / |n|^2, 12 |a1| |a2|, 13 the object index, 14-15 0.
// A point h of the plane has h - b = al a1 + be a2 with al = (h - b).pa and
// be = (h - b).pb. Also a [3][K] table of the normals of every object (0 for
// an edge), for the side test of a path's own objects. One workgroup.
constexpr int kFaceRec = 16;

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
      float* r = tab + (int64_t)f * kFaceRec;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        r[c] = n[c];
        r[3 + c] = b[c];
        r[6 + c] = pa[c];
        r[9 + c] = pb[c];
      }
      r[12] = sqrtf(dot3(u, u)) * sqrtf(dot3(v, v));
      r[13] = __int_as_float(k);
      r[14] = 0.f;
      r[15] = 0.f;
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

// Does the segment p -> p + d cross the face of record r (interior of the
// segment: its parameter s in (1e-6, 1 - 1e-6); face parameters in [0, 1])?
// With den = d.n and num = (b - p).n, s = num / den, and al den =
// (p - b).pa den + num d.pa (likewise be), so every bound is tested on the
// products, without a division or a branch. A segment parallel to the
// face's plane (|den| not above 1e-12 |d| |a1| |a2|) does not cross it.
typedef __attribute__((address_space(4))) const float ConstF;  // read-only, scalar loads

__device__ __forceinline__ bool crosses(const float* p, const float* d, float dlen,
                                        ConstF* r) {
  const float h0 = p[0] - r[3], h1 = p[1] - r[4], h2 = p[2] - r[5];
  const float num = -fmaf(h2, r[2], fmaf(h1, r[1], h0 * r[0]));
  const float den = fmaf(d[2], r[2], fmaf(d[1], r[1], d[0] * r[0]));
  const float ha = fmaf(h2, r[8], fmaf(h1, r[7], h0 * r[6]));
  const float da = fmaf(d[2], r[8], fmaf(d[1], r[7], d[0] * r[6]));
  const float hb = fmaf(h2, r[11], fmaf(h1, r[10], h0 * r[9]));
  const float db = fmaf(d[2], r[11], fmaf(d[1], r[10], d[0] * r[9]));
  const float sg = den < 0.f ? -1.f : 1.f;
  const float ad = fabsf(den), ns = num * sg;
  const float as = fmaf(ha, den, num * da) * sg, bs = fmaf(hb, den, num * db) * sg;
  return (ns > 1e-6f * ad) & (ns < (1.f - 1e-6f) * ad) & (as >= 0.f) & (as <= ad) &
         (bs >= 0.f) & (bs <= ad) & (ad > 1e-12f * dlen * r[12]);
}

// Loads the path's object ids and points (0 = TX, 1..NO interactions,
// NO + 1 = RX); false when the path has no valid solution.
template <int NO>
__device__ __forceinline__ bool load_points(const ValidateArgs& A, int64_t p,
                                            int32_t (&kid)[NO], float (&x)[NO + 2][3]) {
  const int32_t s0 = A.src[p], e0 = A.dst[p];
  bool ok = (A.status[p] & (FPT_ST_INVALID | FPT_ST_NONFINITE)) == 0 && s0 >= 0 &&
            s0 < A.Q && e0 >= 0 && e0 < A.Q;
#pragma unroll
  for (int j = 0; j < NO; ++j) {
    kid[j] = A.ids[(int64_t)j * A.N + p];
    ok = ok && kid[j] >= 0 && kid[j] < A.K;
    kid[j] = ok ? kid[j] : 0;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    x[0][c] = A.pts[(int64_t)c * A.Q + (ok ? s0 : 0)];
    x[NO + 1][c] = A.pts[(int64_t)c * A.Q + (ok ? e0 : 0)];
  }
#pragma unroll
  for (int j = 0; j < NO; ++j)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[j + 1][c] = A.x[(int64_t)(3 * j + c) * A.N + p];
      ok = ok && isfinite(x[j + 1][c]);
    }
  return ok;
}

// EXTENT and SPECULAR bits of a loaded path.
template <int NO>
__device__ __forceinline__ uint8_t local_flags(const ValidateArgs& A, int64_t p,
                                               const int32_t (&kid)[NO],
                                               const float (&x)[NO + 2][3]) {
  bool extent = true, specular = true;
#pragma unroll
  for (int j = 0; j < NO; ++j) {
    float n[3], di[3], dn[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      n[c] = A.nrm[(int64_t)c * A.K + kid[j]];
      di[c] = x[j][c] - x[j + 1][c];
      dn[c] = x[j + 2][c] - x[j + 1][c];
    }
    const bool isface = n[0] != 0.f || n[1] != 0.f || n[2] != 0.f;
    const float t0 = A.t[(int64_t)(2 * j) * A.N + p];
    const float t1 = A.t[(int64_t)(2 * j + 1) * A.N + p];
    extent = extent && t0 >= 0.f && t0 <= 1.f && (!isface || (t1 >= 0.f && t1 <= 1.f));
    const float a = dot3(n, di), b = dot3(n, dn);
    specular = specular && (!isface || (a > 0.f && b > 0.f) || (a < 0.f && b < 0.f));
  }
  return (extent ? FPT_VALID_EXTENT : 0) | (specular ? FPT_VALID_SPECULAR : 0);
}

// Occlusion: every segment against every face of the scene except the faces
// of the segment's own end points. The face loop is the same for every lane:
// its records are read with wave-uniform (scalar) loads, once per face for
// all segments of the path. Lanes that are done (hit, or inactive = !live)
// stop the loop early once the whole wave is.
template <int NO>
__device__ __forceinline__ bool occluded(const int32_t (&kid)[NO], const float (&x)[NO + 2][3],
                                         bool live, int32_t F, const float* face) {
  float d[NO + 1][3], dlen[NO + 1];
#pragma unroll
  for (int sgi = 0; sgi <= NO; ++sgi) {
#pragma unroll
    for (int c = 0; c < 3; ++c) d[sgi][c] = x[sgi + 1][c] - x[sgi][c];
    dlen[sgi] = sqrtf(dot3(d[sgi], d[sgi]));
  }
  bool hit = false;
  for (int32_t f = 0; f < F; ++f) {
    if ((f & 15) == 0 && __all(hit || !live)) break;
    ConstF* r = (ConstF*)face + (int64_t)f * kFaceRec;
    const int32_t k = __float_as_int(r[13]);
    bool h = false;
#pragma unroll
    for (int sgi = 0; sgi <= NO; ++sgi) {
      const bool own = (sgi >= 1 && k == kid[sgi >= 1 ? sgi - 1 : 0]) |
                       (sgi < NO && k == kid[sgi < NO ? sgi : 0]);
      h = h | ((!own) & crosses(x[sgi], d[sgi], dlen[sgi], r));
    }
    hit = hit | h;
  }
  return hit;
}

// Occlusion bit of listed path p (it has EXTENT and SPECULAR), for the lanes
// with `live`.
template <int NO>
__device__ __forceinline__ void occlusion_step(const ValidateArgs& A, const float* face,
                                               int32_t F, int64_t p, bool live) {
  int32_t kid[NO];
  float x[NO + 2][3];
  const bool ok = load_points<NO>(A, p, kid, x) && live;
  const bool hit = occluded<NO>(kid, x, ok, F, face);
  if (ok && !hit) A.flags[p] = FPT_VALID_EXTENT | FPT_VALID_SPECULAR | FPT_VALID_VISIBLE;
}

// LAZY = false: all three bits for every path of the bucket.
// LAZY = true: EXTENT and SPECULAR for every path; the paths that have both
// go into a ring of path indices in LDS, and whenever it holds a full
// workgroup's worth (and once at the end) every lane takes one of them
// through the occlusion test. Only listed paths pay for it, in full waves,
// with no global list or counter.
template <int NO, bool LAZY>
__global__ __launch_bounds__(kBlock) void validate_kernel(
    ValidateArgs A, const float* __restrict__ face, const int32_t* __restrict__ perm,
    const int64_t* __restrict__ bucket) {
  constexpr uint32_t kRing = 2 * kBlock;  // holds < kBlock + one batch
  __shared__ int64_t ring[LAZY ? kRing : 1];
  __shared__ uint32_t tail;
  uint32_t head = 0;  // the same in every thread
  if (LAZY && threadIdx.x == 0) tail = 0;
  if (LAZY) __syncthreads();
  const int32_t F = *A.nfaces;
  int64_t begin = 0, count = A.N;
  if (bucket) {
    begin = bucket[NO - 1];
    count = bucket[NO] - begin;
  }
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  // the loop is uniform over the workgroup (barriers inside)
  for (int64_t b0 = (int64_t)blockIdx.x * kBlock; b0 < count; b0 += stride) {
    const int64_t idx = b0 + threadIdx.x;
    const bool live = idx < count;
    const int64_t p = live ? (perm ? (int64_t)perm[begin + idx] : idx) : 0;
    int32_t kid[NO];
    float x[NO + 2][3];
    const bool loaded = load_points<NO>(A, p, kid, x);  // path 0 for a lane past the end
    const bool ok = live && loaded;
    uint8_t fl = ok ? local_flags<NO>(A, p, kid, x) : 0;
    if constexpr (LAZY) {
      const bool want = fl == (FPT_VALID_EXTENT | FPT_VALID_SPECULAR);
      const unsigned long long m = __ballot(want);
      if (m) {
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(&tail, (uint32_t)__popcll(m));
        base = __shfl(base, 0);
        if (want) {
          const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
          ring[(base + __popcll(m & below)) % kRing] = p;
        }
      }
      if (live) A.flags[p] = fl;
      __syncthreads();
      if (tail - head >= kBlock) {
        occlusion_step<NO>(A, face, F, ring[(head + threadIdx.x) % kRing], true);
        head += kBlock;
      }
      __syncthreads();
    } else {
      const bool hit = occluded<NO>(kid, x, ok, F, face);
      if (ok && !hit) fl |= FPT_VALID_VISIBLE;
      if (live) A.flags[p] = fl;
    }
  }
  if constexpr (LAZY) {
    const uint32_t rest = tail - head;
    if ((threadIdx.x & ~63u) < rest) {  // waves with at least one listed path
      const bool live = threadIdx.x < rest;
      occlusion_step<NO>(A, face, F, live ? ring[(head + threadIdx.x) % kRing] : 0, live);
    }
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

template <int NO>
static hipError_t launch_validate_n(const ValidateArgs& A, bool lazy, const int32_t* perm,
                                    const int64_t* bucket, int grid, hipStream_t st) {
  if (lazy)
    hipLaunchKernelGGL((validate_kernel<NO, true>), dim3(grid), dim3(kBlock), 0, st, A,
                       A.tab, perm, bucket);
  else
    hipLaunchKernelGGL((validate_kernel<NO, false>), dim3(grid), dim3(kBlock), 0, st, A,
                       A.tab, perm, bucket);
  return hipGetLastError();
}

hipError_t launch_validate(int order, const ValidateArgs& A, bool lazy, const int32_t* perm,
                           const int64_t* bucket, int grid, hipStream_t st) {
  switch (order) {
    case 1: return launch_validate_n<1>(A, lazy, perm, bucket, grid, st);
    case 2: return launch_validate_n<2>(A, lazy, perm, bucket, grid, st);
    case 3: return launch_validate_n<3>(A, lazy, perm, bucket, grid, st);
    case 4: return launch_validate_n<4>(A, lazy, perm, bucket, grid, st);
    case 5: return launch_validate_n<5>(A, lazy, perm, bucket, grid, st);
    case 6: return launch_validate_n<6>(A, lazy, perm, bucket, grid, st);
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
