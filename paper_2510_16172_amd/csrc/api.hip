// Host side of the C ABI declared in include/fpt.h: argument checks, the
// handle and its workspace, and the launches of the solver and gradient
// kernels on the caller's stream.
#include <string.h>

#include <string>

#include "common.h"

namespace fpt {
hipError_t launch_solve(int order, const SolveArgs& A, const int32_t* perm,
                        const int64_t* bucket, int grid, hipStream_t st);
const void* solve_kernel_ptr(int order);
hipError_t launch_bucketing(const uint8_t* order, int64_t N, int n_max,
                            unsigned long long* counts,
                            unsigned long long* cursor, int64_t* bucket,
                            int32_t* perm, int grid, hipStream_t st);
hipError_t launch_invalid(const SolveArgs& A, const int32_t* perm,
                          const int64_t* bucket, int grid, hipStream_t st);
hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t st);
}  // namespace fpt

struct fpt_handle {
  int device;
  int num_cu;
  int occ[FPT_NMAX + 1];  // resident workgroups per CU of solve_kernel<n>
  // workspace
  int32_t* perm = nullptr;
  int64_t perm_cap = 0;
  unsigned long long* counts = nullptr;  // [8]
  unsigned long long* cursor = nullptr;  // [8]
  int64_t* bucket = nullptr;             // [8]
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
  for (int n = 1; n <= FPT_NMAX; ++n) {
    int occ = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &occ, fpt::solve_kernel_ptr(n), fpt::kBlock, 0);
    if (e != hipSuccess || occ < 1) occ = 1;
    h->occ[n] = occ;
  }
  void* p = nullptr;
  e = hipMalloc(&p, 3 * 8 * sizeof(unsigned long long));
  if (e != hipSuccess) {
    delete h;
    return fail(FPT_ENOMEM, "fpt_create: workspace allocation failed");
  }
  h->counts = (unsigned long long*)p;
  h->cursor = h->counts + 8;
  h->bucket = (int64_t*)(h->counts + 16);
  *out = h;
  return FPT_OK;
}

extern "C" fpt_status fpt_destroy(fpt_handle* h) {
  if (!h) return FPT_OK;
  DeviceGuard g(h->device);
  (void)hipDeviceSynchronize();
  if (h->perm) (void)hipFree(h->perm);
  if (h->counts) (void)hipFree(h->counts);
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
  if (!pa->order) {
    int64_t grid = (pa->N + fpt::kBlock - 1) / fpt::kBlock;
    e = fpt::launch_solve(pa->n_max, A, nullptr, nullptr, (int)grid, st);
    if (e != hipSuccess) return hip_fail(e, "fpt_solve: launch");
    return FPT_OK;
  }
  s = ensure_perm(h, pa->N);
  if (s != FPT_OK) return s;
  int sgrid = h->num_cu * 4;
  e = fpt::launch_zero_u64(h->counts, 8, st);
  if (e != hipSuccess) return hip_fail(e, "fpt_solve: launch");
  e = fpt::launch_bucketing(pa->order, pa->N, pa->n_max, h->counts, h->cursor,
                            h->bucket, h->perm, sgrid, st);
  if (e != hipSuccess) return hip_fail(e, "fpt_solve: bucketing launch");
  for (int n = 1; n <= pa->n_max; ++n) {
    // persistent: one resident wave of workgroups per bucket; each workgroup
    // strides over the bucket, whose size is read on the device
    int grid = h->num_cu * h->occ[n];
    int64_t cap = (pa->N + fpt::kBlock - 1) / fpt::kBlock;
    if (grid > cap) grid = (int)cap;
    e = fpt::launch_solve(n, A, h->perm, h->bucket, grid, st);
    if (e != hipSuccess) return hip_fail(e, "fpt_solve: launch");
  }
  e = fpt::launch_invalid(A, h->perm, h->bucket, sgrid, st);
  if (e != hipSuccess) return hip_fail(e, "fpt_solve: launch");
  return FPT_OK;
}
