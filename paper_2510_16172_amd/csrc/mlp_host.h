// Host-side glue of the learned initialiser (shared by mlp.hip and api.hip).
#pragma once

#include <string.h>

#include "common.h"

namespace fpt {

typedef __bf16 bf16;
constexpr int kMlpOrder = 4;
constexpr int64_t kParams = 172864;  // padded parameter count (see mlp.hip)

struct MlpWork {
  bf16 *X, *XT, *H1, *H1T, *H2, *H2T, *H3, *H3T, *dY, *dYT, *dH, *dHT, *dH2, *dH2T;
  float *Yp, *Y, *Ym;
  int64_t cap;
};

struct MlpPrepArgs {
  const float* obj;
  const float* pts;
  const int32_t* src;
  const int32_t* dst;
  const int32_t* ids;
  const float* t;
  const uint8_t* status;
  int64_t N;
  int64_t base, count;
  int32_t K, Q;
  float inv_scale;
  bf16* X;
  bf16* XT;
  float* Y;
  float* Ym;
};

struct AdamArgs {
  float* w;
  float* m;
  float* v;
  const float* grad;
  float lr, b1, b2, eps, bc1, bc2;
  bf16* wb;
  bf16* wbT;
};

// state buffer: w, m, v, grad (fp32, kParams each), then wb, wbT (bf16)
struct MlpState {
  float *w, *m, *v, *grad;
  bf16 *wb, *wbT;
};

inline MlpState mlp_state(float* base) {
  MlpState S;
  S.w = base;
  S.m = base + kParams;
  S.v = base + 2 * kParams;
  S.grad = base + 3 * kParams;
  S.wb = reinterpret_cast<bf16*>(base + 4 * kParams);
  S.wbT = S.wb + kParams;
  return S;
}

inline AdamArgs adam_args(const MlpState& S, const float* grad, float lr, int step) {
  AdamArgs A;
  A.w = S.w;
  A.m = S.m;
  A.v = S.v;
  A.grad = grad;
  A.lr = lr;
  A.b1 = 0.9f;
  A.b2 = 0.999f;
  A.eps = 1e-8f;
  double t = step < 1 ? 1.0 : (double)step;
  A.bc1 = (float)(1.0 - pow(0.9, t));
  A.bc2 = (float)(1.0 - pow(0.999, t));
  A.wb = S.wb;
  A.wbT = S.wbT;
  return A;
}

// bf16 / f32 elements per batch row of the workspace
inline size_t mlp_work_bf16_per_row() { return 96 * 2 + 256 * 6 + 64 * 2 + 256 * 4; }
inline size_t mlp_work_f32_per_row() { return 64 + 8 + 8; }

inline void mlp_carve(void* mem, int64_t rows, MlpWork& W) {
  bf16* p = reinterpret_cast<bf16*>(mem);
  auto take = [&](int64_t n) { bf16* q = p; p += n * rows; return q; };
  W.X = take(96); W.XT = take(96);
  W.H1 = take(256); W.H1T = take(256); W.H2 = take(256); W.H2T = take(256);
  W.H3 = take(256); W.H3T = take(256);
  W.dY = take(64); W.dYT = take(64);
  W.dH = take(256); W.dHT = take(256); W.dH2 = take(256); W.dH2T = take(256);
  float* f = reinterpret_cast<float*>(p);
  W.Yp = f; f += 64 * rows;
  W.Y = f; f += 8 * rows;
  W.Ym = f;
  W.cap = rows;
}

inline MlpPrepArgs prep_args(const fpt_scene* sc, const fpt_paths* pa,
                             int64_t base, int64_t count, float scale,
                             const MlpWork& W, bool train) {
  MlpPrepArgs P;
  memset(&P, 0, sizeof(P));
  P.obj = sc->obj;
  P.pts = sc->pts;
  P.src = pa->src;
  P.dst = pa->dst;
  P.ids = pa->ids;
  P.N = pa->N;
  P.base = base;
  P.count = count;
  P.K = sc->K;
  P.Q = sc->Q;
  P.inv_scale = 1.0f / scale;
  P.X = W.X;
  P.XT = train ? W.XT : nullptr;
  P.Y = train ? W.Y : nullptr;
  P.Ym = train ? W.Ym : nullptr;
  return P;
}

hipError_t mlp_forward(const float* w32, const bf16* wb, const MlpWork& W,
                       int64_t Bn, bool train, hipStream_t st);
hipError_t mlp_backward(const bf16* wbT, const MlpWork& W, int64_t Bn,
                        float* grad, hipStream_t st);
hipError_t launch_mlp_prep(const MlpPrepArgs& A, hipStream_t st);
hipError_t launch_mlp_infer(const fpt_scene* sc, const fpt_paths* pa, const float* w32,
                            const bf16* wb, float scale, float* t_init, hipStream_t st);
hipError_t launch_mlp_loss(const MlpWork& W, int64_t Bn, float* loss, hipStream_t st);
hipError_t launch_mlp_adam(const AdamArgs& A, hipStream_t st);
hipError_t launch_mlp_init(float* w, float* m, float* v, uint64_t seed, hipStream_t st);
}  // namespace fpt
