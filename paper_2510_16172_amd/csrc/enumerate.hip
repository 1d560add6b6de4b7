// Candidate enumeration on the device (Sec. III, problem statement: the
// candidates with n interactions are every ordered sequence of n objects,
// for n = 1..n_max, per TX/RX pair). Candidates are ranked by order, then
// pair, then object sequence in lexicographic order; with no_repeat a
// sequence never names the same object twice in a row.
//
// Rank -> candidate, one path per thread: the order from the per-order first
// ranks, then pair = q / M_n and the sequence's index s = q mod M_n. With
// no_repeat the allowed sequences in lexicographic order are the numbers of
// a mixed radix (K, K-1, .., K-1): digit d_0 is the first object, and each
// later digit d_j in 0..K-2 names the d_j-th object other than k_{j-1}, that
// is k_j = d_j + (d_j >= k_{j-1}). Without no_repeat the radix is K
// throughout and k_j = d_j.
#include <hip/hip_runtime.h>

#include "common.h"

namespace fpt {

// q / b and q mod b, on 32 bits when q fits (the common case)
__device__ __forceinline__ uint64_t divmod(uint64_t q, uint32_t b, uint32_t& rem) {
  if ((q >> 32) == 0) {
    const uint32_t q32 = (uint32_t)q;
    const uint32_t d = q32 / b;
    rem = q32 - d * b;
    return d;
  }
  const uint64_t d = q / b;
  rem = (uint32_t)(q - d * b);
  return d;
}

__global__ __launch_bounds__(kBlock) void enumerate_kernel(EnumArgs A) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  const uint32_t base = A.no_repeat ? (uint32_t)(A.K - 1) : (uint32_t)A.K;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < A.count; i += stride) {
    const int64_t r = A.rank0 + i;
    int n = A.omin;
    while (n < A.omax && r >= A.first[n - A.omin + 1]) ++n;
    const uint64_t q = (uint64_t)(r - A.first[n - A.omin]);
    const uint64_t M = (uint64_t)A.per_pair[n];
    const uint64_t pair = q / M;
    uint64_t s = q - pair * M;
    int32_t k[FPT_NMAX];
#pragma unroll
    for (int j = FPT_NMAX - 1; j >= 1; --j) {
      k[j] = -1;
      if (j < n) {
        uint32_t d;
        s = divmod(s, base, d);
        k[j] = (int32_t)d;
      }
    }
    k[0] = (int32_t)s;
    if (A.no_repeat) {
#pragma unroll
      for (int j = 1; j < FPT_NMAX; ++j)
        if (j < n) k[j] += (k[j] >= k[j - 1]) ? 1 : 0;
    }
    A.src[i] = A.pair_src[pair];
    A.dst[i] = A.pair_dst[pair];
    A.order[i] = (uint8_t)n;
#pragma unroll
    for (int j = 0; j < FPT_NMAX; ++j)
      if (j < A.n_max) A.ids[(int64_t)j * A.count + i] = k[j];
  }
}

hipError_t launch_enumerate(const EnumArgs& A, int grid, hipStream_t st) {
  hipLaunchKernelGGL(enumerate_kernel, dim3(grid), dim3(kBlock), 0, st, A);
  return hipGetLastError();
}

}  // namespace fpt
