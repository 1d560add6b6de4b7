// Host side of the C ABI declared in include/fpt.h: argument checks, the
// handle and its workspace, and the launches of the solver and gradient
// kernels on the caller's stream.
#include <string.h>

#include <string>

#include "common.h"

namespace fpt {
hipError_t launch_solve(int phase, int order, const SolveArgs& A,
                        const int32_t* perm, const int64_t* bucket,
                        unsigned long long* work, int grid, hipStream_t st);
const void* solve_kernel_ptr(int phase, int order);
hipError_t launch_bucketing(const uint8_t* order, int64_t N, int n_max,
                            unsigned long long* counts,
                            unsigned long long* cursor, int64_t* bucket,
                            int32_t* perm, int grid, hipStream_t st);
hipError_t launch_invalid(const SolveArgs& A, const int32_t* perm,
                          const int64_t* bucket, int grid, hipStream_t st);
hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t st);
hipError_t launch_grad(int order, const GradArgs& A, const int32_t* perm,
                       const int64_t* bucket, int grid, size_t shmem,
                       hipStream_t st);
const void* grad_kernel_ptr(int order);
hipError_t launch_grad_invalid(const GradArgs& A, const int32_t* perm,
                               const int64_t* bucket, int grid, hipStream_t st);
}  // namespace fpt

struct fpt_handle {
  int device;
  int num_cu;
  int occ[3][FPT_NMAX + 1];  // resident workgroups per CU, per phase/order
  // optional per-kernel timing
  static constexpr int kRing = 32;
  bool timing = false;
  hipEvent_t ev[FPT_TIMERS][kRing][2] = {};
  int nrec[FPT_TIMERS] = {};  // launches recorded since the last read
  // workspace
  int32_t* perm = nullptr;
  int64_t perm_cap = 0;
  unsigned long long* counts = nullptr;  // [8]
  unsigned long long* cursor = nullptr;  // [8]
  int64_t* bucket = nullptr;             // [8]
  unsigned long long* work = nullptr;    // [8] refill cursors per order
};

static thread_local std::string g_err;

static fpt_status fail(fpt_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

static fpt_status hip_fail(hipError_t e, const char* what) {
  return fail(FPT_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

extern "C" const char* fpt_last_error(void) { return g_err.c_str(); }

extern "C" void fpt_default_opts(fpt_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->iters = 64;
  o->fp_iters = 1;
  o->early_exit = 0;
  o->exit_rtol = 1e-6f;
  o->scale = 1.0f;
  o->n_levels = 4;
  o->level_eps[0] = 1e-3f;
  o->level_eps[1] = 1e-5f;
  o->level_eps[2] = 1e-7f;
  o->level_eps[3] = 1e-9f;
  o->level_steps[0] = 2;
  o->level_steps[1] = 2;
  o->level_steps[2] = 2;
  o->level_steps[3] = 3;
  o->cert_rtol = 1e-5f;
  o->refill_min = 8;
  o->refill_every = 4;
}

// Keeps the caller's current device and switches to the handle's for the
// duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(dev) == hipSuccess)
      ok = true;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

extern "C" fpt_status fpt_create(int device, fpt_handle** out) {
  if (!out) return fail(FPT_EINVAL, "fpt_create: out is NULL");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0)
    return fail(FPT_EUNSUPPORTED, "fpt_create: no HIP device");
  if (device < 0 || device >= ndev)
    return fail(FPT_EINVAL, "fpt_create: device index out of range");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(FPT_EUNSUPPORTED,
                std::string("fpt_create: built for gfx950, device is ") +
                    prop.gcnArchName);
  DeviceGuard g(device);
  if (!g.ok) return fail(FPT_EHIP, "fpt_create: hipSetDevice failed");
  fpt_handle* h = new fpt_handle();
  h->device = device;
  h->num_cu = prop.multiProcessorCount;
  for (int ph = 0; ph < 3; ++ph)
    for (int n = 1; n <= FPT_NMAX; ++n) {
      int occ = 0;
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &occ, fpt::solve_kernel_ptr(ph, n), fpt::kBlock, 0);
      if (e != hipSuccess || occ < 1) occ = 1;
      h->occ[ph][n] = occ;
    }
  void* p = nullptr;
  e = hipMalloc(&p, 4 * 8 * sizeof(unsigned long long));
  if (e != hipSuccess) {
    delete h;
    return fail(FPT_ENOMEM, "fpt_create: workspace allocation failed");
  }
  h->counts = (unsigned long long*)p;
  h->cursor = h->counts + 8;
  h->bucket = (int64_t*)(h->counts + 16);
  h->work = h->counts + 24;
  *out = h;
  return FPT_OK;
}

extern "C" fpt_status fpt_destroy(fpt_handle* h) {
  if (!h) return FPT_OK;
  DeviceGuard g(h->device);
  (void)hipDeviceSynchronize();
  if (h->perm) (void)hipFree(h->perm);
  if (h->counts) (void)hipFree(h->counts);
  for (int i = 0; i < FPT_TIMERS; ++i)
    for (int r = 0; r < fpt_handle::kRing; ++r)
      for (int k = 0; k < 2; ++k)
        if (h->ev[i][r][k]) (void)hipEventDestroy(h->ev[i][r][k]);
  delete h;
  return FPT_OK;
}

static bool aligned(const void* p, size_t a) {
  return ((uintptr_t)p % a) == 0;
}

static fpt_status check_common(const fpt_scene* sc, const fpt_paths* pa,
                               const char* fn) {
  std::string f(fn);
  if (!sc || !pa) return fail(FPT_EINVAL, f + ": scene or paths is NULL");
  if (pa->N < 0) return fail(FPT_EINVAL, f + ": N < 0");
  if (pa->N > (int64_t)INT32_MAX)
    return fail(FPT_EINVAL, f + ": N above 2^31-1 is not supported");
  if (pa->n_max < 1 || pa->n_max > FPT_NMAX)
    return fail(FPT_EINVAL, f + ": n_max outside 1..6");
  if (sc->K < 1 || sc->Q < 1)
    return fail(FPT_EINVAL, f + ": K and Q must be >= 1");
  if (pa->N == 0) return FPT_OK;
  if (!sc->obj || !sc->pts || !pa->src || !pa->dst || !pa->ids)
    return fail(FPT_EINVAL, f + ": a required pointer is NULL");
  if (!aligned(sc->obj, 4) || !aligned(sc->pts, 4) || !aligned(pa->src, 4) ||
      !aligned(pa->dst, 4) || !aligned(pa->ids, 4) ||
      (pa->t_init && !aligned(pa->t_init, 4)))
    return fail(FPT_EINVAL, f + ": misaligned pointer");
  return FPT_OK;
}

static fpt_status check_opts(const fpt_opts* o) {
  if (!o) return fail(FPT_EINVAL, "fpt_solve: opts is NULL");
  if (o->iters < 0 || o->iters > 65535)
    return fail(FPT_EINVAL, "fpt_solve: iters outside 0..65535");
  if (o->fp_iters < 0 || o->fp_iters > 1024)
    return fail(FPT_EINVAL, "fpt_solve: fp_iters outside 0..1024");
  if (!(o->scale > 0.f) || !(o->scale < 1e30f))
    return fail(FPT_EINVAL, "fpt_solve: scale must be positive and finite");
  if (o->n_levels < 0 || o->n_levels > FPT_MAX_LEVELS)
    return fail(FPT_EINVAL, "fpt_solve: n_levels outside 0..8");
  for (int i = 0; i < o->n_levels; ++i) {
    if (!(o->level_eps[i] >= 0.f) || o->level_steps[i] < 0 ||
        o->level_steps[i] > 64)
      return fail(FPT_EINVAL, "fpt_solve: bad refinement level");
  }
  if (!(o->cert_rtol >= 0.f) || !(o->exit_rtol >= 0.f))
    return fail(FPT_EINVAL, "fpt_solve: negative tolerance");
  if (o->early_exit &&
      (o->refill_min < 1 || o->refill_min > 64 || o->refill_every < 1))
    return fail(FPT_EINVAL, "fpt_solve: refill_min outside 1..64 or refill_every < 1");
  return FPT_OK;
}

static fpt_status ensure_perm(fpt_handle* h, int64_t N) {
  if (h->perm_cap >= N) return FPT_OK;
  if (h->perm) {
    (void)hipFree(h->perm);
    h->perm = nullptr;
    h->perm_cap = 0;
  }
  void* p = nullptr;
  int64_t cap = N < 1024 ? 1024 : N;
  if (hipMalloc(&p, (size_t)cap * sizeof(int32_t)) != hipSuccess)
    return fail(FPT_ENOMEM, "workspace allocation failed");
  h->perm = (int32_t*)p;
  h->perm_cap = cap;
  return FPT_OK;
}

// Event pair around the launches of one timer slot (no-op unless enabled).
// Each call records into the next entry of a ring per slot, so that timing
// adds no host synchronisation between calls.
struct SlotTimer {
  fpt_handle* h;
  int slot, r;
  hipStream_t st;
  SlotTimer(fpt_handle* h_, int slot_, hipStream_t st_)
      : h(h_), slot(slot_), r(0), st(st_) {
    if (h->timing) {
      r = h->nrec[slot] % fpt_handle::kRing;
      (void)hipEventRecord(h->ev[slot][r][0], st);
    }
  }
  ~SlotTimer() {
    if (h->timing) {
      (void)hipEventRecord(h->ev[slot][r][1], st);
      h->nrec[slot] += 1;
    }
  }
};

extern "C" fpt_status fpt_set_timing(fpt_handle* h, int enable) {
  if (!h) return fail(FPT_EINVAL, "fpt_set_timing: handle is NULL");
  DeviceGuard g(h->device);
  if (enable && !h->ev[0][0][0]) {
    for (int i = 0; i < FPT_TIMERS; ++i)
      for (int r = 0; r < fpt_handle::kRing; ++r)
        for (int k = 0; k < 2; ++k) {
          hipError_t e = hipEventCreate(&h->ev[i][r][k]);
          if (e != hipSuccess)
            return hip_fail(e, "fpt_set_timing: hipEventCreate");
        }
  }
  h->timing = enable != 0;
  for (int i = 0; i < FPT_TIMERS; ++i) h->nrec[i] = 0;
  return FPT_OK;
}

extern "C" fpt_status fpt_kernel_times(fpt_handle* h, float* ms) {
  if (!h || !ms) return fail(FPT_EINVAL, "fpt_kernel_times: NULL argument");
  DeviceGuard g(h->device);
  for (int i = 0; i < FPT_TIMERS; ++i) {
    ms[i] = -1.f;
    int n = h->nrec[i] < fpt_handle::kRing ? h->nrec[i] : fpt_handle::kRing;
    if (n == 0) continue;
    double sum = 0.0;
    for (int r = 0; r < n; ++r) {
      hipError_t e = hipEventSynchronize(h->ev[i][r][1]);
      if (e != hipSuccess)
        return hip_fail(e, "fpt_kernel_times: hipEventSynchronize");
      float t = 0.f;
      e = hipEventElapsedTime(&t, h->ev[i][r][0], h->ev[i][r][1]);
      if (e != hipSuccess)
        return hip_fail(e, "fpt_kernel_times: hipEventElapsedTime");
      sum += t;
    }
    ms[i] = (float)(sum / n);
    h->nrec[i] = 0;
  }
  return FPT_OK;
}

extern "C" fpt_status fpt_solve(fpt_handle* h, const fpt_scene* sc,
                                const fpt_paths* pa, const fpt_opts* o,
                                const fpt_out* out, void* stream) {
  if (!h) return fail(FPT_EINVAL, "fpt_solve: handle is NULL");
  fpt_status s = check_common(sc, pa, "fpt_solve");
  if (s != FPT_OK) return s;
  s = check_opts(o);
  if (s != FPT_OK) return s;
  if (!out) return fail(FPT_EINVAL, "fpt_solve: out is NULL");
  if (pa->N == 0) return FPT_OK;
  if (!out->x || !out->len || !out->t || !out->status || !out->iters)
    return fail(FPT_EINVAL, "fpt_solve: an output pointer is NULL");
  if (!aligned(out->x, 4) || !aligned(out->len, 4) || !aligned(out->t, 4) ||
      !aligned(out->iters, 2))
    return fail(FPT_EINVAL, "fpt_solve: misaligned output pointer");
  DeviceGuard g(h->device);
  if (!g.ok) return fail(FPT_EHIP, "fpt_solve: hipSetDevice failed");
  hipStream_t st = (hipStream_t)stream;

  fpt::SolveArgs A;
  memset(&A, 0, sizeof(A));
  A.obj = sc->obj;
  A.pts = sc->pts;
  A.src = pa->src;
  A.dst = pa->dst;
  A.order = pa->order;
  A.ids = pa->ids;
  A.t_init = pa->t_init;
  A.x = out->x;
  A.len = out->len;
  A.t = out->t;
  A.status = out->status;
  A.iters = out->iters;
  A.N = pa->N;
  A.K = sc->K;
  A.Q = sc->Q;
  A.n_max = pa->n_max;
  A.n_iter = o->iters;
  A.fp_iters = o->fp_iters;
  A.early_exit = o->early_exit ? 1 : 0;
  A.refill_min = o->refill_min;
  A.refill_every = o->refill_every;
  float ed = o->exit_rtol * o->scale;
  A.exit_d2 = ed * ed;
  A.scale = o->scale;
  A.n_levels = o->n_levels;
  for (int i = 0; i < FPT_MAX_LEVELS; ++i) {
    A.level_eps[i] = o->level_eps[i];
    A.level_steps[i] = o->level_steps[i];
  }
  A.cert_abs = o->cert_rtol * o->scale;

  hipError_t e;
  const int p1 = A.early_exit ? 2 : 0;  // phase-1 kernel variant
  int64_t cap = (pa->N + fpt::kBlock - 1) / fpt::kBlock;
  auto persistent = [&](int ph, int n) -> int {
    int64_t g = (int64_t)h->num_cu * h->occ[ph][n];
    return (int)(g < cap ? g : cap);
  };
  if (A.early_exit) {
    e = fpt::launch_zero_u64(h->work, 8, st);
    if (e != hipSuccess) return hip_fail(e, "fpt_solve: launch");
  }
  if (!pa->order) {
    for (int ph : {p1, 1}) {
      SlotTimer tm(h, (ph == 1 ? FPT_T_REFINE : FPT_T_BFGS) + pa->n_max - 1, st);
      int grid = (ph == 2) ? persistent(2, pa->n_max) : (int)cap;
      e = fpt::launch_solve(ph, pa->n_max, A, nullptr, nullptr, h->work, grid, st);
      if (e != hipSuccess) return hip_fail(e, "fpt_solve: launch");
    }
    return FPT_OK;
  }
  s = ensure_perm(h, pa->N);
  if (s != FPT_OK) return s;
  int sgrid = h->num_cu * 4;
  {
    SlotTimer tm(h, FPT_T_BUCKET, st);
    e = fpt::launch_zero_u64(h->counts, 8, st);
    if (e != hipSuccess) return hip_fail(e, "fpt_solve: launch");
    e = fpt::launch_bucketing(pa->order, pa->N, pa->n_max, h->counts,
                              h->cursor, h->bucket, h->perm, sgrid, st);
    if (e != hipSuccess) return hip_fail(e, "fpt_solve: bucketing launch");
  }
  for (int n = 1; n <= pa->n_max; ++n) {
    for (int ph : {p1, 1}) {
      // persistent: one resident set of workgroups strides over the bucket,
      // whose size is only known on the device
      SlotTimer tm(h, (ph == 1 ? FPT_T_REFINE : FPT_T_BFGS) + n - 1, st);
      e = fpt::launch_solve(ph, n, A, h->perm, h->bucket, h->work,
                            persistent(ph, n), st);
      if (e != hipSuccess) return hip_fail(e, "fpt_solve: launch");
    }
  }
  e = fpt::launch_invalid(A, h->perm, h->bucket, sgrid, st);
  if (e != hipSuccess) return hip_fail(e, "fpt_solve: launch");
  return FPT_OK;
}

// LDS budget of the per-workgroup accumulation of the scene gradient
static const size_t kGradLdsMax = 48 * 1024;

extern "C" fpt_status fpt_grad(fpt_handle* h, const fpt_scene* sc,
                               const fpt_paths* pa, const fpt_out* fwd,
                               const float* g_len, const float* g_x,
                               float* g_pts, float* g_obj, float* g_slot,
                               float* g_end, void* stream) {
  if (!h) return fail(FPT_EINVAL, "fpt_grad: handle is NULL");
  fpt_status s = check_common(sc, pa, "fpt_grad");
  if (s != FPT_OK) return s;
  if (!fwd) return fail(FPT_EINVAL, "fpt_grad: fwd is NULL");
  if (pa->N == 0) return FPT_OK;
  if (!fwd->t || !fwd->status)
    return fail(FPT_EINVAL, "fpt_grad: fwd.t and fwd.status are required");
  if (!g_pts || !g_obj)
    return fail(FPT_EINVAL, "fpt_grad: g_pts and g_obj are required");
  if (!aligned(fwd->t, 4) || !aligned(g_pts, 4) || !aligned(g_obj, 4) ||
      (g_len && !aligned(g_len, 4)) || (g_x && !aligned(g_x, 4)) ||
      (g_slot && !aligned(g_slot, 4)) || (g_end && !aligned(g_end, 4)))
    return fail(FPT_EINVAL, "fpt_grad: misaligned pointer");
  DeviceGuard g(h->device);
  if (!g.ok) return fail(FPT_EHIP, "fpt_grad: hipSetDevice failed");
  hipStream_t st = (hipStream_t)stream;

  fpt::GradArgs A;
  memset(&A, 0, sizeof(A));
  A.obj = sc->obj;
  A.pts = sc->pts;
  A.src = pa->src;
  A.dst = pa->dst;
  A.order = pa->order;
  A.ids = pa->ids;
  A.t = fwd->t;
  A.status = fwd->status;
  A.g_len = g_len;
  A.g_x = g_x;
  A.g_pts = g_pts;
  A.g_obj = g_obj;
  A.g_slot = g_slot;
  A.g_end = g_end;
  A.N = pa->N;
  A.K = sc->K;
  A.Q = sc->Q;
  A.n_max = pa->n_max;
  size_t shmem = (9 * (size_t)sc->K + 3 * (size_t)sc->Q) * sizeof(float);
  A.lds = shmem <= kGradLdsMax ? 1 : 0;
  if (!A.lds) shmem = 0;
  int64_t cap = (pa->N + fpt::kBlock - 1) / fpt::kBlock;
  auto grid_for = [&](int n) -> int {
    if (!A.lds) return (int)cap;  // one path per thread
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &occ, fpt::grad_kernel_ptr(n), fpt::kBlock, shmem) != hipSuccess ||
        occ < 1)
      occ = 1;
    int64_t gsz = (int64_t)h->num_cu * occ;
    return (int)(gsz < cap ? gsz : cap);
  };
  hipError_t e;
  if (!pa->order) {
    SlotTimer tm(h, FPT_T_GRAD, st);
    e = fpt::launch_grad(pa->n_max, A, nullptr, nullptr, grid_for(pa->n_max),
                         shmem, st);
    if (e != hipSuccess) return hip_fail(e, "fpt_grad: launch");
    return FPT_OK;
  }
  s = ensure_perm(h, pa->N);
  if (s != FPT_OK) return s;
  int sgrid = h->num_cu * 4;
  {
    SlotTimer tm(h, FPT_T_BUCKET, st);
    e = fpt::launch_zero_u64(h->counts, 8, st);
    if (e != hipSuccess) return hip_fail(e, "fpt_grad: launch");
    e = fpt::launch_bucketing(pa->order, pa->N, pa->n_max, h->counts,
                              h->cursor, h->bucket, h->perm, sgrid, st);
    if (e != hipSuccess) return hip_fail(e, "fpt_grad: bucketing launch");
  }
  {
    SlotTimer tm(h, FPT_T_GRAD, st);
    for (int n = 1; n <= pa->n_max; ++n) {
      // persistent grid: the bucket size is only known on the device
      int grid = A.lds ? grid_for(n) : (int)(cap < (int64_t)h->num_cu * 8 ? cap : (int64_t)h->num_cu * 8);
      e = fpt::launch_grad(n, A, h->perm, h->bucket, grid, shmem, st);
      if (e != hipSuccess) return hip_fail(e, "fpt_grad: launch");
    }
    e = fpt::launch_grad_invalid(A, h->perm, h->bucket, sgrid, st);
    if (e != hipSuccess) return hip_fail(e, "fpt_grad: launch");
  }
  return FPT_OK;
}
