// Learned initialiser: an MLP 66 -> 256 -> 256 -> 256 -> 8 (ReLU) that maps
// the geometry of an order-4 path to starting parameters for the solver
// (the paper names better initial candidates as future work, Sec. V).
// BF16 operands, FP32 accumulation on the MFMA units (v_mfma_f32_16x16x32_bf16),
// FP32 master weights and Adam.
//
// Every product is written as an "NT" GEMM, C[m][n] = sum_k A[m][k] B[n][k],
// with both operands contiguous in k, so that each lane reads its MFMA
// fragment (8 consecutive bf16) with one 16-byte load. The forward pass
// therefore also stores each activation transposed, and the weights are kept
// in bf16 both as [out][in] and as [in][out].
#include <hip/hip_runtime.h>

#include "common.h"
#include "mlp_host.h"

namespace fpt {

typedef bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// layer sizes (padded): input 66 -> 96, output 8 -> 64
constexpr int kIn = 66, kInP = 96, kHid = 256, kOut = 8, kOutP = 64;

// offsets (in floats) of the FP32 parameters inside the state buffer
constexpr int64_t oW1 = 0;                              // [256][96]
constexpr int64_t oB1 = oW1 + (int64_t)kHid * kInP;     // [256]
constexpr int64_t oW2 = oB1 + kHid;                     // [256][256]
constexpr int64_t oB2 = oW2 + (int64_t)kHid * kHid;
constexpr int64_t oW3 = oB2 + kHid;                     // [256][256]
constexpr int64_t oB3 = oW3 + (int64_t)kHid * kHid;
constexpr int64_t oW4 = oB3 + kHid;                     // [64][256]
constexpr int64_t oB4 = oW4 + (int64_t)kOutP * kHid;    // [64]
static_assert(kParams == oB4 + kOutP, "padded parameter count");

enum GemmEpi {
  EPI_BIAS_RELU = 0,  // relu(acc + bias) -> bf16 C (and C^T)
  EPI_BIAS_F32 = 1,   // acc + bias -> fp32 Cf
  EPI_RELU_MASK = 2,  // acc * (mask > 0) -> bf16 C (and C^T)
  EPI_ATOMIC_F32 = 3  // Cf += acc (split-K partial sums)
};

struct GemmArgs {
  const bf16* A;
  int lda;  // A[m * lda + k]
  const bf16* B;
  int ldb;  // B[n * ldb + k]
  int M, N, K, k_chunk;
  int epi;
  const float* bias;
  const bf16* mask;
  int ldm;
  bf16* C;
  int ldc;
  bf16* CT;
  int ldct;
  float* Cf;
  int ldcf;
};

__device__ __forceinline__ bf16x8 load8(const bf16* p) {
  return *reinterpret_cast<const bf16x8*>(p);
}

// 256 threads = 4 wavefronts; a workgroup computes a 64 x 64 tile of C, each
// wavefront a 32 x 32 quarter as 2 x 2 MFMA 16 x 16 tiles. blockIdx.z is the
// split-K chunk. M, N must be multiples of 16, K of 32, lda/ldb of 8.
__global__ __launch_bounds__(256) void gemm_nt_kernel(GemmArgs g) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 64 + (w >> 1) * 32;
  const int n0 = blockIdx.x * 64 + (w & 1) * 32;
  const int kb = blockIdx.z * g.k_chunk;
  const int ke = min(g.K, kb + g.k_chunk);
  const int li = lane & 15, lk = (lane >> 4) * 8;
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  bool mv[2], nv[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    mv[t] = (m0 + 16 * t) < g.M;
    nv[t] = (n0 + 16 * t) < g.N;
  }
  const bf16x8 zero8 = {};
  for (int k = kb; k < ke; k += 32) {
    bf16x8 fa[2], fb[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      fa[t] = mv[t] ? load8(g.A + (int64_t)(m0 + 16 * t + li) * g.lda + k + lk) : zero8;
      fb[t] = nv[t] ? load8(g.B + (int64_t)(n0 + 16 * t + li) * g.ldb + k + lk) : zero8;
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
  }
  // lane holds rows 4*(lane/16) + r, column lane % 16 of each 16 x 16 tile
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      if (!mv[a] || !nv[b]) continue;
      const int n = n0 + 16 * b + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + 16 * a + (lane >> 4) * 4 + r;
        float v = acc[a][b][r];
        switch (g.epi) {
          case EPI_BIAS_RELU: {
            v = fmaxf(v + g.bias[n], 0.f);
            bf16 hv = (bf16)v;
            g.C[(int64_t)m * g.ldc + n] = hv;
            if (g.CT) g.CT[(int64_t)n * g.ldct + m] = hv;
            break;
          }
          case EPI_BIAS_F32:
            g.Cf[(int64_t)m * g.ldcf + n] = v + (g.bias ? g.bias[n] : 0.f);
            break;
          case EPI_RELU_MASK: {
            bool on = (float)g.mask[(int64_t)m * g.ldm + n] > 0.f;
            bf16 hv = (bf16)(on ? v : 0.f);
            g.C[(int64_t)m * g.ldc + n] = hv;
            if (g.CT) g.CT[(int64_t)n * g.ldct + m] = hv;
            break;
          }
          default:
            unsafeAtomicAdd(g.Cf + (int64_t)m * g.ldcf + n, v);
        }
      }
    }
}

// ----------------------------------------------------------- features ----


// Input features of path p, all lengths divided by the scene size S:
// TX, RX, and per interaction b, the unit basis a1/|a1|, a2/|a2| (0 for an
// edge), b - TX and b - RX: 6 + 4 * 15 = 66 values, zero-padded to 96.
// Target: the solver's parameters in unit-vector coordinates, / S, masked
// where the path is not certified or the parameter is an edge's padding.
// The 96 (padded) features of path i, and its unit-basis norms |a| of each
// slot (for the target and for mapping the output back).
__device__ __forceinline__ void mlp_features(
    const float* __restrict__ obj, const float* __restrict__ pts,
    const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
    const int32_t* __restrict__ ids, int64_t N, int32_t K, int32_t Q,
    float inv_scale, int64_t i, float* f, float (*nrm)[2], bool* edge) {
#pragma unroll
  for (int k = 0; k < kInP; ++k) f[k] = 0.f;
  int32_t s = src[i], e = dst[i];
  s = (s >= 0 && s < Q) ? s : 0;
  e = (e >= 0 && e < Q) ? e : 0;
  float tx[3], rx[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    tx[c] = pts[(int64_t)c * Q + s];
    rx[c] = pts[(int64_t)c * Q + e];
    f[c] = tx[c] * inv_scale;
    f[3 + c] = rx[c] * inv_scale;
  }
#pragma unroll
  for (int j = 0; j < kMlpOrder; ++j) {
    int32_t k = ids[(int64_t)j * N + i];
    k = (k >= 0 && k < K) ? k : 0;
    float bb[3], a1[3], a2[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      bb[c] = obj[(int64_t)c * K + k];
      a1[c] = obj[(int64_t)(3 + c) * K + k];
      a2[c] = obj[(int64_t)(6 + c) * K + k];
    }
    edge[j] = (a2[0] == 0.f) && (a2[1] == 0.f) && (a2[2] == 0.f);
    float n1 = dot3(a1, a1), n2 = dot3(a2, a2);
    float i1 = rsq32(n1 > 0.f ? n1 : 1.f);
    float i2 = edge[j] ? 0.f : rsq32(n2 > 0.f ? n2 : 1.f);
    nrm[j][0] = n1 * i1;
    nrm[j][1] = n2 * i2;
    const int o = 6 + 15 * j;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      f[o + c] = bb[c] * inv_scale;
      f[o + 3 + c] = a1[c] * i1;
      f[o + 6 + c] = a2[c] * i2;
      f[o + 9 + c] = (bb[c] - tx[c]) * inv_scale;
      f[o + 12 + c] = (bb[c] - rx[c]) * inv_scale;
    }
  }
}

__global__ __launch_bounds__(kBlock) void mlp_prep_kernel(MlpPrepArgs A) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;  // batch row
  if (r >= A.count) return;
  const int64_t i = A.base + r;  // path
  float f[kInP], nrm[kMlpOrder][2];
  bool edge[kMlpOrder];
  mlp_features(A.obj, A.pts, A.src, A.dst, A.ids, A.N, A.K, A.Q, A.inv_scale, i, f,
               nrm, edge);
  bool cert = A.status ? (A.status[i] & FPT_ST_CONVERGED) != 0 : false;
  if (A.Y) {
#pragma unroll
    for (int j = 0; j < kMlpOrder; ++j) {
      float t0 = A.t[(int64_t)(2 * j) * A.N + i];
      float t1 = A.t[(int64_t)(2 * j + 1) * A.N + i];
      // unit-vector coordinates: that = t * |a|
      float y0 = t0 * nrm[j][0] * A.inv_scale;
      float y1 = edge[j] ? 0.f : t1 * nrm[j][1] * A.inv_scale;
      bool ok0 = cert && isfinite(y0), ok1 = cert && !edge[j] && isfinite(y1);
      A.Y[r * kOut + 2 * j] = ok0 ? y0 : 0.f;
      A.Y[r * kOut + 2 * j + 1] = ok1 ? y1 : 0.f;
      A.Ym[r * kOut + 2 * j] = ok0 ? 1.f : 0.f;
      A.Ym[r * kOut + 2 * j + 1] = ok1 ? 1.f : 0.f;
    }
  }
#pragma unroll
  for (int k = 0; k < kInP; ++k) {
    bf16 v = (bf16)f[k];
    A.X[r * kInP + k] = v;
    if (A.XT) A.XT[(int64_t)k * A.count + r] = v;
  }
}

// ------------------------------------------------------ fused inference ----
// One workgroup of 16 wavefronts per tile of kTM = 256 paths computes the
// features, the three hidden layers and the output layer, with the
// activations in LDS, and writes t_init: no activation goes through HBM. A
// layer's products stay in the accumulators until every wave has read the
// layer's input, so one LDS buffer holds the input features and then each
// hidden activation in turn. The hidden layers' weights (bf16, L2-resident)
// pass through LDS in chunks of kKC input columns: the workgroup copies a
// chunk with one coalesced 16-byte load per thread, the load of the next
// chunk in flight while the MFMAs use this one, and every wave reads its
// fragments from LDS. (Read from global memory as fragments, each weight
// went through the L1 once for every wave that needed it, and that traffic
// bounded the kernel.) Wave w computes rows 64 (w / 4) .. + 63 and output
// columns 64 (w % 4) .. + 63 of each hidden layer (4 x 4 tiles of 16 x 16).
constexpr int kTM = 256, kLdH = kHid + 8;  // +8: fewer LDS bank conflicts
constexpr int kKC = 32, kLdW = kKC + 8;    // weight chunk [kHid][kKC], padded rows
constexpr int kInferThreads = 1024;
static_assert(kHid * kKC / 8 == kInferThreads, "one 16-byte copy per thread per chunk");

struct MlpInferArgs {
  const float* obj;
  const float* pts;
  const int32_t* src;
  const int32_t* dst;
  const int32_t* ids;
  const float* w32;  // biases (fp32 master copy)
  const bf16* wb;    // bf16 weights [out][in]
  int64_t N;
  int32_t K, Q;
  float scale, inv_scale;
  float* t_init;     // [4][2][N]
};

__device__ __forceinline__ bf16x8 load8s(const bf16* p) {
  return *reinterpret_cast<const bf16x8*>(p);
}

__global__ __launch_bounds__(kInferThreads) void mlp_infer_kernel(MlpInferArgs A) {
  __shared__ __align__(16) bf16 sH[kTM * kLdH];  // features, then H1, H2, H3
  __shared__ __align__(16) bf16 sW[kHid * kLdW];  // a weight chunk
  float* sY = reinterpret_cast<float*>(sW);       // after the hidden layers: outputs
  static_assert(kTM * kOut * sizeof(float) <= kHid * kLdW * sizeof(bf16), "sY fits in sW");
  const int64_t row0 = (int64_t)blockIdx.x * kTM;
  // threads < kTM: scale / |a| per output (unit-vector coordinates / S to the
  // caller's parametrisation; 0 for an edge's padding)
  float osc[kOut];
  if (threadIdx.x < kTM) {
    const int64_t i = row0 + threadIdx.x;
    float f[kInP], nrm[kMlpOrder][2];
    bool edge[kMlpOrder];
    if (i < A.N) {
      mlp_features(A.obj, A.pts, A.src, A.dst, A.ids, A.N, A.K, A.Q, A.inv_scale, i,
                   f, nrm, edge);
    } else {
#pragma unroll
      for (int k = 0; k < kInP; ++k) f[k] = 0.f;
#pragma unroll
      for (int j = 0; j < kMlpOrder; ++j) {
        nrm[j][0] = nrm[j][1] = 1.f;
        edge[j] = false;
      }
    }
#pragma unroll
    for (int k = 0; k < kInP; ++k) sH[threadIdx.x * kLdH + k] = (bf16)f[k];
#pragma unroll
    for (int j = 0; j < kMlpOrder; ++j) {
      osc[2 * j] = nrm[j][0] > 0.f ? A.scale / nrm[j][0] : 0.f;
      osc[2 * j + 1] = (edge[j] || !(nrm[j][1] > 0.f)) ? 0.f : A.scale / nrm[j][1];
    }
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = (lane >> 4) * 8;
  const int mr = 64 * (w >> 2), nc = 64 * (w & 3);
  // this thread's share of a weight chunk: row cn, columns ck .. ck + 7
  const int cn = threadIdx.x >> 2, ck = 8 * (threadIdx.x & 3);
#pragma unroll 1
  for (int layer = 0; layer < 3; ++layer) {
    const int K = layer == 0 ? kInP : kHid;
    const bf16* W = A.wb + (layer == 0 ? oW1 : layer == 1 ? oW2 : oW3);
    const float* bias = A.w32 + (layer == 0 ? oB1 : layer == 1 ? oB2 : oB3);
    f32x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    bf16x8 nxt = load8(W + (int64_t)cn * K + ck);
    for (int k = 0; k < K; k += kKC) {
      // every wave is done with the previous chunk (and, at k = 0, the
      // layer's input is complete in sH)
      __syncthreads();
      *reinterpret_cast<bf16x8*>(sW + cn * kLdW + ck) = nxt;
      if (k + kKC < K) nxt = load8(W + (int64_t)cn * K + k + kKC + ck);
      __syncthreads();
      bf16x8 fa[4], fb[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) fb[b] = load8s(sW + (nc + 16 * b + li) * kLdW + lk);
#pragma unroll
      for (int a = 0; a < 4; ++a) fa[a] = load8s(sH + (mr + 16 * a + li) * kLdH + k + lk);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();  // every wave has read this layer's input
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int n = nc + 16 * b + li;
      const float bn = bias[n];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = mr + 16 * a + (lane >> 4) * 4 + r;
          sH[m * kLdH + n] = (bf16)fmaxf(acc[a][b][r] + bn, 0.f);
        }
    }
  }
  __syncthreads();  // H3 complete; sW free for the outputs
  // output layer: wave w takes rows 16 w .. 16 w + 15, the first 16 outputs
  // (their 8 KB of weights are read as fragments: L1-resident)
  {
    const bf16* W4 = A.wb + oW4;
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < kHid; k += 32) {
      bf16x8 fa = load8s(sH + (16 * w + li) * kLdH + k + lk);
      bf16x8 fb = load8(W4 + (int64_t)li * kHid + k + lk);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb, acc, 0, 0, 0);
    }
    if (li < kOut) {
      const float b4 = A.w32[oB4 + li];
#pragma unroll
      for (int r = 0; r < 4; ++r)
        sY[(16 * w + (lane >> 4) * 4 + r) * kOut + li] = acc[r] + b4;
    }
  }
  __syncthreads();
  if (threadIdx.x < kTM) {
    const int64_t i = row0 + threadIdx.x;
    if (i < A.N) {
#pragma unroll
      for (int q = 0; q < kOut; ++q)
        A.t_init[(int64_t)q * A.N + i] = osc[q] > 0.f ? sY[threadIdx.x * kOut + q] * osc[q] : 0.f;
    }
  }
}

hipError_t launch_mlp_infer(const fpt_scene* sc, const fpt_paths* pa, const float* w32,
                            const bf16* wb, float scale, float* t_init, hipStream_t st) {
  MlpInferArgs A;
  A.obj = sc->obj;
  A.pts = sc->pts;
  A.src = pa->src;
  A.dst = pa->dst;
  A.ids = pa->ids;
  A.w32 = w32;
  A.wb = wb;
  A.N = pa->N;
  A.K = sc->K;
  A.Q = sc->Q;
  A.scale = scale;
  A.inv_scale = 1.f / scale;
  A.t_init = t_init;
  hipLaunchKernelGGL(mlp_infer_kernel, dim3((unsigned)((pa->N + kTM - 1) / kTM)),
                     dim3(kInferThreads), 0, st, A);
  return hipGetLastError();
}

// ------------------------------------------------------- loss, Adam ------

// Masked mean squared error over the 8 outputs; dY = 2 (y - t) m / (8 B),
// written as bf16 [B][64] and transposed [64][B]; loss accumulated into
// *loss (sum of squared errors / (8 B)).
__global__ __launch_bounds__(kBlock) void mlp_loss_kernel(
    const float* __restrict__ Yp, const float* __restrict__ Y,
    const float* __restrict__ Ym, int64_t B, bf16* __restrict__ dY,
    bf16* __restrict__ dYT, float* __restrict__ loss) {
  __shared__ float red[kBlock];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  float acc = 0.f;
  if (i < B) {
    const float sc = 1.f / (float)(kOut * B);
    for (int o = 0; o < kOutP; ++o) {
      float d = 0.f;
      if (o < kOut) {
        float e = (Yp[i * kOutP + o] - Y[i * kOut + o]) * Ym[i * kOut + o];
        acc += e * e;
        d = 2.f * e * sc;
      }
      bf16 v = (bf16)d;
      dY[i * kOutP + o] = v;
      dYT[(int64_t)o * B + i] = v;
    }
    acc *= 1.f / (float)(kOut * B);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) unsafeAtomicAdd(loss, red[0]);
}

// db[n] = sum_k dYT[n][k] (bias gradients), one workgroup per row
__global__ __launch_bounds__(kBlock) void rowsum_kernel(
    const bf16* __restrict__ XT, int64_t ld, int64_t K, float* __restrict__ out) {
  __shared__ float red[kBlock];
  const int64_t row = blockIdx.x;
  float acc = 0.f;
  for (int64_t k = threadIdx.x; k < K; k += kBlock) acc += (float)XT[row * ld + k];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[row] = red[0];
}

__global__ __launch_bounds__(kBlock) void fill_f32_kernel(float* p, int64_t n, float v) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) p[i] = v;
}

// Which entries of the padded parameter vector are real weights (the padding
// of W1's input columns, W4's / b4's output rows stays exactly 0).
__device__ __forceinline__ bool param_live(int64_t i) {
  if (i < oB1) return (i % kInP) < kIn;
  if (i >= oW4 && i < oB4) return (i - oW4) / kHid < kOut;
  if (i >= oB4) return (i - oB4) < kOut;
  return true;
}

// Adam (Kingma & Ba) on the FP32 master weights, then the bf16 copies:
// [out][in] for the forward pass and [in][out] for the input gradients.

__global__ __launch_bounds__(kBlock) void adam_kernel(AdamArgs A) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < kParams; i += stride) {
    float w = A.w[i];
    if (A.grad && param_live(i)) {
      float g = A.grad[i];
      float m = A.b1 * A.m[i] + (1.f - A.b1) * g;
      float v = A.b2 * A.v[i] + (1.f - A.b2) * g * g;
      A.m[i] = m;
      A.v[i] = v;
      float mh = m / A.bc1, vh = v / A.bc2;
      w -= A.lr * mh / (sqrtf(vh) + A.eps);
      A.w[i] = w;
    }
    bf16 wb = (bf16)w;
    A.wb[i] = wb;
    // transposed copies of the weight matrices used for input gradients
    if (i >= oW2 && i < oB2) {
      int64_t r = (i - oW2) / kHid, c = (i - oW2) % kHid;
      A.wbT[oW2 + c * kHid + r] = wb;
    } else if (i >= oW3 && i < oB3) {
      int64_t r = (i - oW3) / kHid, c = (i - oW3) % kHid;
      A.wbT[oW3 + c * kHid + r] = wb;
    } else if (i >= oW4 && i < oB4) {
      int64_t r = (i - oW4) / kHid, c = (i - oW4) % kHid;  // W4 [64][256]
      A.wbT[oW4 + c * kOutP + r] = wb;                     // W4^T [256][64]
    }
  }
}

// He-normal initialisation from a counter-based hash (splitmix64 of
// seed + index, Box-Muller); biases 0; padding 0.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__global__ __launch_bounds__(kBlock) void mlp_init_kernel(float* w, float* m, float* v, uint64_t seed) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < kParams; i += stride) {
    float val = 0.f;
    int fan_in = 0;
    if (i < oB1) fan_in = kIn;
    else if ((i >= oW2 && i < oB2) || (i >= oW3 && i < oB3) || (i >= oW4 && i < oB4)) fan_in = kHid;
    if (fan_in && param_live(i)) {
      uint64_t h1 = splitmix64(seed * 0x100000001B3ull + 2 * (uint64_t)i);
      uint64_t h2 = splitmix64(seed * 0x100000001B3ull + 2 * (uint64_t)i + 1);
      float u1 = ((h1 >> 40) + 1) * (1.0f / 16777217.0f);
      float u2 = (h2 >> 40) * (1.0f / 16777216.0f);
      float z = sqrtf(-2.f * logf(u1)) * cosf(6.2831853f * u2);
      val = z * sqrtf(2.f / (float)fan_in);
    }
    w[i] = val;
    m[i] = 0.f;
    v[i] = 0.f;
  }
}

// ------------------------------------------------------------- host ------


static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

static hipError_t gemm(const GemmArgs& g, int splits, hipStream_t st) {
  dim3 grid(cdiv(g.N, 64), cdiv(g.M, 64), splits);
  hipLaunchKernelGGL(gemm_nt_kernel, grid, dim3(256), 0, st, g);
  return hipGetLastError();
}

static GemmArgs gargs(const bf16* A, int lda, const bf16* B, int ldb, int M, int N, int K) {
  GemmArgs g;
  memset(&g, 0, sizeof(g));
  g.A = A;
  g.lda = lda;
  g.B = B;
  g.ldb = ldb;
  g.M = M;
  g.N = N;
  g.K = K;
  g.k_chunk = K;
  return g;
}

// forward pass on a prepared batch X [Bn][96]: H1..H3 (+ transposes when
// `train`), output Yp [Bn][64] fp32
hipError_t mlp_forward(const float* w32, const bf16* wb, const MlpWork& W,
                       int64_t Bn, bool train, hipStream_t st) {
  hipError_t e;
  const int M = (int)Bn;
  GemmArgs g = gargs(W.X, kInP, wb + oW1, kInP, M, kHid, kInP);
  g.epi = EPI_BIAS_RELU; g.bias = w32 + oB1; g.C = W.H1; g.ldc = kHid;
  g.CT = train ? W.H1T : nullptr; g.ldct = M;
  if ((e = gemm(g, 1, st)) != hipSuccess) return e;
  g = gargs(W.H1, kHid, wb + oW2, kHid, M, kHid, kHid);
  g.epi = EPI_BIAS_RELU; g.bias = w32 + oB2; g.C = W.H2; g.ldc = kHid;
  g.CT = train ? W.H2T : nullptr; g.ldct = M;
  if ((e = gemm(g, 1, st)) != hipSuccess) return e;
  g = gargs(W.H2, kHid, wb + oW3, kHid, M, kHid, kHid);
  g.epi = EPI_BIAS_RELU; g.bias = w32 + oB3; g.C = W.H3; g.ldc = kHid;
  g.CT = train ? W.H3T : nullptr; g.ldct = M;
  if ((e = gemm(g, 1, st)) != hipSuccess) return e;
  g = gargs(W.H3, kHid, wb + oW4, kHid, M, kOutP, kHid);
  g.epi = EPI_BIAS_F32; g.bias = w32 + oB4; g.Cf = W.Yp; g.ldcf = kOutP;
  return gemm(g, 1, st);
}

// backward pass from the loss gradient dY (already in W.dY / W.dYT):
// parameter gradients into grad (fp32, zeroed here first)
hipError_t mlp_backward(const bf16* wbT, const MlpWork& W, int64_t Bn,
                        float* grad, hipStream_t st) {
  hipError_t e;
  const int M = (int)Bn;
  hipLaunchKernelGGL(fill_f32_kernel, dim3(256), dim3(kBlock), 0, st, grad, kParams, 0.f);
  const int kc = 1024;  // split-K chunk for the weight gradients
  const int splits = cdiv(M, kc);
  // layer 4: dW4 [64][256] = dY^T H3, db4
  GemmArgs g = gargs(W.dYT, M, W.H3T, M, kOutP, kHid, M);
  g.k_chunk = kc; g.epi = EPI_ATOMIC_F32; g.Cf = grad + oW4; g.ldcf = kHid;
  if ((e = gemm(g, splits, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(rowsum_kernel, dim3(kOutP), dim3(kBlock), 0, st, W.dYT, (int64_t)M, (int64_t)M, grad + oB4);
  // dH3 = (dY W4) * (H3 > 0)
  g = gargs(W.dY, kOutP, wbT + oW4, kOutP, M, kHid, kOutP);
  g.epi = EPI_RELU_MASK; g.mask = W.H3; g.ldm = kHid; g.C = W.dH; g.ldc = kHid; g.CT = W.dHT; g.ldct = M;
  if ((e = gemm(g, 1, st)) != hipSuccess) return e;
  // layer 3: dW3 = dH3^T H2, db3
  g = gargs(W.dHT, M, W.H2T, M, kHid, kHid, M);
  g.k_chunk = kc; g.epi = EPI_ATOMIC_F32; g.Cf = grad + oW3; g.ldcf = kHid;
  if ((e = gemm(g, splits, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(rowsum_kernel, dim3(kHid), dim3(kBlock), 0, st, W.dHT, (int64_t)M, (int64_t)M, grad + oB3);
  // dH2 = (dH3 W3) * (H2 > 0)
  g = gargs(W.dH, kHid, wbT + oW3, kHid, M, kHid, kHid);
  g.epi = EPI_RELU_MASK; g.mask = W.H2; g.ldm = kHid; g.C = W.dH2; g.ldc = kHid; g.CT = W.dH2T; g.ldct = M;
  if ((e = gemm(g, 1, st)) != hipSuccess) return e;
  // layer 2: dW2 = dH2^T H1, db2
  g = gargs(W.dH2T, M, W.H1T, M, kHid, kHid, M);
  g.k_chunk = kc; g.epi = EPI_ATOMIC_F32; g.Cf = grad + oW2; g.ldcf = kHid;
  if ((e = gemm(g, splits, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(rowsum_kernel, dim3(kHid), dim3(kBlock), 0, st, W.dH2T, (int64_t)M, (int64_t)M, grad + oB2);
  // dH1 = (dH2 W2) * (H1 > 0)   (reuses dH / dHT)
  g = gargs(W.dH2, kHid, wbT + oW2, kHid, M, kHid, kHid);
  g.epi = EPI_RELU_MASK; g.mask = W.H1; g.ldm = kHid; g.C = W.dH; g.ldc = kHid; g.CT = W.dHT; g.ldct = M;
  if ((e = gemm(g, 1, st)) != hipSuccess) return e;
  // layer 1: dW1 [256][96] = dH1^T X, db1
  g = gargs(W.dHT, M, W.XT, M, kHid, kInP, M);
  g.k_chunk = kc; g.epi = EPI_ATOMIC_F32; g.Cf = grad + oW1; g.ldcf = kInP;
  if ((e = gemm(g, splits, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(rowsum_kernel, dim3(kHid), dim3(kBlock), 0, st, W.dHT, (int64_t)M, (int64_t)M, grad + oB1);
  return hipGetLastError();
}

hipError_t launch_mlp_prep(const MlpPrepArgs& A, hipStream_t st) {
  hipLaunchKernelGGL(mlp_prep_kernel, dim3(cdiv(A.count, kBlock)), dim3(kBlock), 0, st, A);
  return hipGetLastError();
}

hipError_t launch_mlp_loss(const MlpWork& W, int64_t Bn, float* loss, hipStream_t st) {
  hipLaunchKernelGGL(mlp_loss_kernel, dim3(cdiv(Bn, kBlock)), dim3(kBlock), 0, st,
                     W.Yp, W.Y, W.Ym, Bn, W.dY, W.dYT, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(const AdamArgs& A, hipStream_t st) {
  hipLaunchKernelGGL(adam_kernel, dim3(cdiv(kParams, kBlock)), dim3(kBlock), 0, st, A);
  return hipGetLastError();
}

hipError_t launch_mlp_init(float* w, float* m, float* v, uint64_t seed, hipStream_t st) {
  hipLaunchKernelGGL(mlp_init_kernel, dim3(cdiv(kParams, kBlock)), dim3(kBlock), 0, st, w, m, v, seed);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t st) {
  hipLaunchKernelGGL(fill_f32_kernel, dim3(256), dim3(kBlock), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace fpt
