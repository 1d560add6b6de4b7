// Host side of the C ABI declared in include/fpt.h: argument checks, the
// handle and its workspace, and the launches of the solver and gradient
// kernels on the caller's stream.
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace fpt {
hipError_t launch_solve(int phase, int order, const SolveArgs& A,
                        const int32_t* perm, const int64_t* bucket,
                        const StageArgs* stage, int grid, hipStream_t st);
int stage_fields_for(int order);
const void* solve_kernel_ptr(int phase, int order);
// bucket[n-1] .. bucket[n]: order n; bucket[n_max] .. bucket[n_max+1]:
// invalid orders; with status, bucket[n_max+1] .. bucket[n_max+2]: the
// collapsed minimisers with a gradient (orders >= 2, any order)
hipError_t launch_bucketing(const uint8_t* order, int64_t N, int n_max,
                            uint32_t* ccount, int64_t* bucket, int32_t* perm,
                            hipStream_t st, int32_t* inv = nullptr,
                            const uint8_t* status = nullptr);
hipError_t launch_invalid(const SolveArgs& A, const int32_t* perm,
                          const int64_t* bucket, int grid, hipStream_t st);
hipError_t launch_unsort(const SolveArgs& S, const SolveArgs& A, const int32_t* inv,
                         const int64_t* bucket, int grid, hipStream_t st);
hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t st);
hipError_t launch_grad(int order, const GradArgs& A, const int32_t* perm,
                       const int64_t* bucket, int grid, int kkt_grid, size_t shmem,
                       hipStream_t st);
const void* grad_kernel_ptr(int order, bool kkt);
hipError_t launch_face_table(const float* obj, int32_t K, float* tab, float* nrm,
                             int32_t* nfaces, hipStream_t st);
hipError_t launch_validate(int order, const ValidateArgs& A, bool lazy, const int32_t* perm,
                           const int64_t* bucket, int grid, hipStream_t st);
hipError_t launch_enumerate(const EnumArgs& A, int grid, hipStream_t st);
hipError_t launch_validate_invalid(const ValidateArgs& A, const int32_t* perm,
                                   const int64_t* bucket, int grid, hipStream_t st);
hipError_t launch_grad_invalid(const GradArgs& A, const int32_t* perm,
                               const int64_t* bucket, int grid, hipStream_t st);
}  // namespace fpt
#include "mlp_host.h"


// Units of work that can run on their own stream: an order, or one of up to
// kMaxSplit parts of an order's paths (unit_of).
static const int kMaxSplit = 4;
static const int kUnits = FPT_NMAX * kMaxSplit;
static int unit_of(int n, int part) { return (n - 1) * kMaxSplit + part + 1; }

struct fpt_handle {
  int device;
  int num_cu;
  int occ[6][FPT_NMAX + 1];  // resident workgroups per CU, per phase/order
  // optional per-kernel timing
  static constexpr int kRing = 32;
  bool timing = false;
  hipEvent_t ev[FPT_TIMERS][kRing][2] = {};
  int nrec[FPT_TIMERS] = {};  // launches recorded since the last read
  unsigned long long* work = nullptr;  // [FPT_NMAX][4][kWorkSlots] counters
  float* faces = nullptr;  // validity tables: faces [K][16], normals [3][K], counts
  int64_t faces_cap = 0;
  // workspace
  int32_t* perm = nullptr;
  uint32_t* ccount = nullptr;  // per-chunk order counts / offsets
  int64_t perm_cap = 0;
  unsigned long long* counts = nullptr;  // [8]
  unsigned long long* cursor = nullptr;  // [8]
  int64_t* bucket = nullptr;             // [8]
  // path lists between the stages of the solve (early-exit BFGS stages,
  // refinement passes): per list set (one per order when the orders run on
  // their own streams, else set 0) two ping-pong index lists and four
  // counter blocks (kRegions counters kCounterStride apart, one block per
  // stage, all cleared by one launch); the early-exit BFGS states (set 0)
  unsigned long long* scount = nullptr;  // [kUnits + 1][4][kRegions * kCounterStride]
  int32_t* slist[kUnits + 1][2] = {};
  float* sstate[2] = {nullptr, nullptr};
  int64_t list_cap[kUnits + 1] = {};  // rcap the lists of a set were sized for
  int64_t stage_state_cap = 0, state_rcap = 0;
  // one stream per unit (an order, or a part of one; default priority) with
  // fork / join events
  hipStream_t ostream[kUnits + 1] = {};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[kUnits + 1] = {};
  // per-order launch configuration (autotuner)
  fpt_launch_cfg cfg[FPT_NMAX + 1] = {};
  // learned-initialiser activations (grown on demand)
  fpt::MlpWork mlp = {};
  void* mlp_mem = nullptr;
  // the solve in bucket order (an order array given): the paths' indices
  // and start points in bucket order, the inverse permutation, and the
  // outputs in bucket order (one allocation, see sorted_layout)
  void* sorted_mem = nullptr;
  size_t sorted_bytes = 0;
  // captured graphs that record this handle's solve workspace: while any
  // exists, the workspace is neither grown nor freed
  int live_graphs = 0;
  // this device's copy of the allocation-free solve's scratch array
  unsigned char* scratch = nullptr;
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

static fpt_status scratch_address(int device, unsigned char** out);

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
  o->stage_iters[0] = 16;
  o->stage_iters[1] = 16;
  o->stage_iters[2] = 32;
  o->stage_iters[3] = 0;
  o->quick_steps = 2;
  o->quick_passes = 2;
  o->concurrent_orders = 0;
  o->method = FPT_METHOD_BFGS;
  o->polish_steps = 1;
  o->split = 0;
  o->line_search = FPT_LS_EQ6;
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
  for (int ph = 0; ph < 6; ++ph)
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
  e = hipMalloc(&p, (size_t)(kUnits + 1) * 4 * fpt::kRegions * fpt::kCounterStride *
                       sizeof(unsigned long long));
  if (e != hipSuccess) {
    (void)hipFree(h->counts);
    delete h;
    return fail(FPT_ENOMEM, "fpt_create: workspace allocation failed");
  }
  h->scount = (unsigned long long*)p;
  {
    fpt_status ss = scratch_address(device, &h->scratch);
    if (ss != FPT_OK) {
      (void)hipFree(h->counts);
      (void)hipFree(h->scount);
      delete h;
      return ss;
    }
  }
  *out = h;
  return FPT_OK;
}

extern "C" fpt_status fpt_destroy(fpt_handle* h) {
  if (!h) return FPT_OK;
  if (h->live_graphs > 0)
    return fail(FPT_EINVAL, "fpt_destroy: captured graphs still use this handle");
  DeviceGuard g(h->device);
  (void)hipDeviceSynchronize();
  if (h->perm) (void)hipFree(h->perm);
  if (h->ccount) (void)hipFree(h->ccount);
  if (h->counts) (void)hipFree(h->counts);
  if (h->work) (void)hipFree(h->work);
  if (h->faces) (void)hipFree(h->faces);
  if (h->scount) (void)hipFree(h->scount);
  if (h->mlp_mem) (void)hipFree(h->mlp_mem);
  if (h->sorted_mem) (void)hipFree(h->sorted_mem);
  for (int k = 0; k < 2; ++k)
    if (h->sstate[k]) (void)hipFree(h->sstate[k]);
  for (int w = 0; w <= kUnits; ++w)
    for (int k = 0; k < 2; ++k)
      if (h->slist[w][k]) (void)hipFree(h->slist[w][k]);
  for (int w = 0; w <= kUnits; ++w) {
    if (h->ostream[w]) (void)hipStreamDestroy(h->ostream[w]);
    if (h->ev_join[w]) (void)hipEventDestroy(h->ev_join[w]);
  }
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
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
  if (o->quick_steps < 0 || o->quick_steps > 64)
    return fail(FPT_EINVAL, "fpt_solve: quick_steps outside 0..64");
  if (o->quick_passes < 1 || o->quick_passes > 2)
    return fail(FPT_EINVAL, "fpt_solve: quick_passes outside 1..2");
  if (o->method != FPT_METHOD_BFGS && o->method != FPT_METHOD_NEWTON32)
    return fail(FPT_EINVAL, "fpt_solve: unknown method");
  if (o->polish_steps < 0 || o->polish_steps > 8)
    return fail(FPT_EINVAL, "fpt_solve: polish_steps outside 0..8");
  if (o->line_search != FPT_LS_EQ6 && o->line_search != FPT_LS_ARMIJO)
    return fail(FPT_EINVAL, "fpt_solve: unknown line_search");
  if (o->split < 0 || o->split > kMaxSplit)
    return fail(FPT_EINVAL, "fpt_solve: split outside 0..4");
  if (o->early_exit) {
    if (o->stage_iters[0] < 1)
      return fail(FPT_EINVAL, "fpt_solve: early exit needs stage_iters[0] >= 1");
    for (int k = 0; k < FPT_MAX_STAGES; ++k)
      if (o->stage_iters[k] < 0 || o->stage_iters[k] > 65535)
        return fail(FPT_EINVAL, "fpt_solve: stage_iters outside 0..65535");
  }
  return FPT_OK;
}

// A captured graph holds the addresses of the solve workspace: growing it
// (which frees the old buffers) would leave the graph writing freed memory.
static fpt_status refuse_growth(const fpt_handle*) {
  return fail(FPT_EINVAL,
              "the handle's workspace must grow, but a captured graph records it: "
              "destroy the graphs first (or capture with the largest size first)");
}

static fpt_status ensure_perm(fpt_handle* h, int64_t N) {
  if (h->perm_cap >= N) return FPT_OK;
  if (h->perm && h->live_graphs > 0) return refuse_growth(h);
  if (h->perm) (void)hipFree(h->perm);
  if (h->ccount) (void)hipFree(h->ccount);
  h->perm = nullptr;
  h->ccount = nullptr;
  h->perm_cap = 0;
  void* p = nullptr;
  int64_t cap = N < 1024 ? 1024 : N;
  if (hipMalloc(&p, (size_t)cap * sizeof(int32_t)) != hipSuccess)
    return fail(FPT_ENOMEM, "workspace allocation failed");
  h->perm = (int32_t*)p;
  int64_t nchunks = (cap + fpt::kSortChunk - 1) / fpt::kSortChunk;
  if (hipMalloc(&p, (size_t)nchunks * 8 * sizeof(uint32_t)) != hipSuccess)
    return fail(FPT_ENOMEM, "workspace allocation failed");
  h->ccount = (uint32_t*)p;
  h->perm_cap = cap;
  return FPT_OK;
}

// Lists and states of the early-exit stages. A list has kRegions regions
// of rcap slots; a stage's input chunk of 64 paths appends to one region, so
// rcap = 64 (ceil(N / 4096) + 1) holds every path. The state is sized for
// the largest order.
static int64_t stage_rcap(int64_t N) {
  return 64 * ((N + 64 * fpt::kRegions - 1) / (64 * fpt::kRegions) + 1);
}

// Lists of set w for N paths; the early-exit states (set 0) for order
// n_state (0: none).
static fpt_status ensure_lists(fpt_handle* h, int64_t N, int w) {
  const int64_t rcap = stage_rcap(N);
  if (h->list_cap[w] >= rcap) return FPT_OK;
  if (h->slist[w][0] && h->live_graphs > 0) return refuse_growth(h);
  for (int k = 0; k < 2; ++k) {
    if (h->slist[w][k]) (void)hipFree(h->slist[w][k]);
    h->slist[w][k] = nullptr;
  }
  h->list_cap[w] = 0;
  for (int k = 0; k < 2; ++k) {
    void* p = nullptr;
    if (hipMalloc(&p, (size_t)rcap * fpt::kRegions * sizeof(int32_t)) != hipSuccess)
      return fail(FPT_ENOMEM, "path-list workspace allocation failed");
    h->slist[w][k] = (int32_t*)p;
  }
  h->list_cap[w] = rcap;
  return FPT_OK;
}

static fpt_status ensure_states(fpt_handle* h, int64_t N, int n_state) {
  const int64_t rcap = stage_rcap(N);
  const int64_t need = n_state > 0 ? (int64_t)fpt::stage_fields_for(n_state) * rcap * fpt::kRegions : 0;
  if (h->stage_state_cap >= need && h->state_rcap >= rcap) return FPT_OK;
  if (h->sstate[0] && h->live_graphs > 0) return refuse_growth(h);
  for (int k = 0; k < 2; ++k) {
    if (h->sstate[k]) (void)hipFree(h->sstate[k]);
    h->sstate[k] = nullptr;
  }
  h->stage_state_cap = h->state_rcap = 0;
  for (int k = 0; k < 2; ++k) {
    void* p = nullptr;
    if (hipMalloc(&p, (size_t)need * sizeof(float)) != hipSuccess)
      return fail(FPT_ENOMEM, "early-exit workspace allocation failed");
    h->sstate[k] = (float*)p;
  }
  h->stage_state_cap = need;
  h->state_rcap = rcap;
  return FPT_OK;
}

// Buffers of the solve in bucket order for N paths of at most n_max
// interactions, each 256-byte aligned: outputs x [n_max][3][N],
// t [n_max][2][N], len [N], iters [N], status [N]; the copied indices
// src, dst [N], ids [n_max][N]; the inverse permutation inv [N].
struct SortedLayout {
  size_t x, t, len, iters, status, src, dst, ids, inv, total;
};

static SortedLayout sorted_layout(int64_t N, int n_max) {
  SortedLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  const size_t n = (size_t)N;
  L.x = take(n * 3 * n_max * sizeof(float));
  L.t = take(n * 2 * n_max * sizeof(float));
  L.len = take(n * sizeof(float));
  L.iters = take(n * sizeof(uint16_t));
  L.status = take(n);
  L.src = take(n * sizeof(int32_t));
  L.dst = take(n * sizeof(int32_t));
  L.ids = take(n * n_max * sizeof(int32_t));
  L.inv = take(n * sizeof(int32_t));
  L.total = off;
  return L;
}

static fpt_status ensure_sorted(fpt_handle* h, int64_t N, int n_max) {
  const size_t need = sorted_layout(N, n_max).total;
  if (h->sorted_bytes >= need) return FPT_OK;
  if (h->sorted_mem && h->live_graphs > 0) return refuse_growth(h);
  if (h->sorted_mem) (void)hipFree(h->sorted_mem);
  h->sorted_mem = nullptr;
  h->sorted_bytes = 0;
  if (hipMalloc(&h->sorted_mem, need) != hipSuccess) {
    h->sorted_mem = nullptr;
    return fail(FPT_ENOMEM, "bucket-order workspace allocation failed");
  }
  h->sorted_bytes = need;
  return FPT_OK;
}

// The stream and join event of unit w (and the fork event), created once.
static fpt_status ensure_stream(fpt_handle* h, int w) {
  if (!h->ev_fork &&
      hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) != hipSuccess)
    return fail(FPT_EHIP, "fpt_solve: event creation failed");
  if (h->ostream[w]) return FPT_OK;
  if (hipStreamCreateWithFlags(&h->ostream[w], hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_join[w], hipEventDisableTiming) != hipSuccess)
    return fail(FPT_EHIP, "fpt_solve: stream creation failed");
  return FPT_OK;
}

// How a call is scheduled: units on their own streams (several orders with
// concurrent_orders, or parts of orders) or everything on the caller's
// stream; and the number of parts per order (split; 0 = 2 parts from 2^21
// paths on). Early exit keeps one part on the caller's stream (its BFGS
// states are shared).
struct SolvePlan {
  bool multi;  // units on their own streams
  bool conc;   // one unit per order and part (else per part: the orders of a
               // part run one after another on its stream)
  int split;
  int n_lo;
  int unit(int n, int part) const { return conc ? unit_of(n, part) : part + 1; }
  // The order issued i-th for a part. With one stream per unit, the orders
  // go from the top down: a high order has few paths, and its passes are
  // latency-bound chains that then run beside the large low orders'
  // ALU-bound work instead of after it. The runtime gives streams to its
  // hardware queues in turn as they are created, and a queue runs its
  // launches in order, so the streams are created in this order too (the
  // first multi-stream call on a handle decides). With parts only, odd
  // parts go from the top down: the short, latency-bound launches of a
  // small order then run beside another part's large order.
  int nth(int i, int part, int n_max) const {
    const bool down = multi && (conc || (part & 1));
    return down ? n_max - i : n_lo + i;
  }
};

static SolvePlan solve_plan(const fpt_paths* pa, const fpt_opts* o, bool any_ee) {
  SolvePlan P;
  P.n_lo = pa->order ? 1 : pa->n_max;
  P.split = o->split > 0 ? o->split : (pa->N >= ((int64_t)1 << 21) ? 2 : 1);
  if (any_ee) P.split = 1;
  P.conc = !any_ee && o->concurrent_orders && P.n_lo < pa->n_max;
  P.multi = !any_ee && (P.conc || P.split > 1);
  return P;
}

// Does any order of this call run the early-exit stages?
static bool uses_early_exit(const fpt_handle* h, const fpt_opts* o, int n_max) {
  for (int n = 1; n <= n_max; ++n) {
    const fpt_launch_cfg& c = h->cfg[n];
    if (c.use_override ? c.early_exit != 0 : o->early_exit != 0) return true;
  }
  return false;
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
  if (enable && !h->work) {
    const size_t bytes = 6 * FPT_NMAX * fpt::kWorkSlots * sizeof(unsigned long long);
    hipError_t e = hipMalloc(&h->work, bytes);
    if (e != hipSuccess) return hip_fail(e, "fpt_set_timing: hipMalloc");
    e = hipMemset(h->work, 0, bytes);
    if (e != hipSuccess) return hip_fail(e, "fpt_set_timing: hipMemset");
  }
  h->timing = enable != 0;
  for (int i = 0; i < FPT_TIMERS; ++i) h->nrec[i] = 0;
  return FPT_OK;
}

extern "C" fpt_status fpt_work_counts(fpt_handle* h, uint64_t* counts) {
  if (!h || !counts) return fail(FPT_EINVAL, "fpt_work_counts: NULL argument");
  DeviceGuard g(h->device);
  for (int i = 0; i < 6 * FPT_NMAX; ++i) counts[i] = 0;
  if (!h->work) return FPT_OK;
  const int nw = 6 * FPT_NMAX * fpt::kWorkSlots;
  std::vector<uint64_t> slots(nw);
  const size_t bytes = nw * sizeof(uint64_t);
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(slots.data(), h->work, bytes, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemset(h->work, 0, bytes);
  if (e != hipSuccess) return hip_fail(e, "fpt_work_counts");
  for (int i = 0; i < 6 * FPT_NMAX; ++i)
    for (int s = 0; s < fpt::kWorkSlots; ++s) counts[i] += slots[i * fpt::kWorkSlots + s];
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

// Workspace of one fpt_solve, allocated before any launch (also before a
// graph capture): order buckets, path lists per list set, early-exit
// states, and the per-order streams.
static fpt_status prepare_solve(fpt_handle* h, const fpt_paths* pa, const fpt_opts* o,
                                bool any_ee, const SolvePlan& P) {
  fpt_status s;
  if (pa->order) {
    s = ensure_perm(h, pa->N);
    if (s != FPT_OK) return s;
    s = ensure_sorted(h, pa->N, pa->n_max);
    if (s != FPT_OK) return s;
  }
  const bool lists = any_ee || (o->n_levels > 0 && o->quick_steps > 0);
  if (!lists) {
    if (P.multi)
      for (int i = 0; i <= pa->n_max - P.n_lo; ++i)
        for (int c = 0; c < P.split; ++c) {
          s = ensure_stream(h, P.unit(P.nth(i, c, pa->n_max), c));
          if (s != FPT_OK) return s;
        }
    return FPT_OK;
  }
  if (P.multi) {
    for (int i = 0; i <= pa->n_max - P.n_lo; ++i)
      for (int c = 0; c < P.split; ++c) {
        const int n = P.nth(i, c, pa->n_max);
        s = ensure_stream(h, P.unit(n, c));
        if (s != FPT_OK) return s;
        s = ensure_lists(h, pa->N, P.unit(n, c));
        if (s != FPT_OK) return s;
      }
  } else {
    s = ensure_lists(h, pa->N, 0);
    if (s != FPT_OK) return s;
  }
  return ensure_states(h, pa->N, any_ee ? pa->n_max : 0);
}

// Checks shared by fpt_solve and fpt_solve_noalloc.
static fpt_status check_solve(const fpt_handle* h, const fpt_scene* sc,
                              const fpt_paths* pa, const fpt_opts* o,
                              const fpt_out* out, const char* fn) {
  const std::string f(fn);
  if (!h) return fail(FPT_EINVAL, f + ": handle is NULL");
  fpt_status s = check_common(sc, pa, fn);
  if (s != FPT_OK) return s;
  s = check_opts(o);
  if (s != FPT_OK) return s;
  if (!out) return fail(FPT_EINVAL, f + ": out is NULL");
  if (pa->N == 0) return FPT_OK;
  if (!out->x || !out->len || !out->t || !out->status || !out->iters)
    return fail(FPT_EINVAL, f + ": an output pointer is NULL");
  if (!aligned(out->x, 4) || !aligned(out->len, 4) || !aligned(out->t, 4) ||
      !aligned(out->iters, 2))
    return fail(FPT_EINVAL, f + ": misaligned output pointer");
  if (uses_early_exit(h, o, pa->n_max) && o->method != FPT_METHOD_BFGS)
    return fail(FPT_EINVAL, f + ": early exit is a BFGS schedule");
  return FPT_OK;
}

// Device buffers one solve works in: the order sort (perm, per-chunk counts,
// bucket bounds), the path-list counters (four blocks of kRegions counters,
// kCounterStride apart, per list set), the two ping-pong path lists of each
// list set, and the early-exit BFGS states.
struct SolveWs {
  int32_t* perm;
  uint32_t* ccount;
  int64_t* bucket;
  unsigned long long* scount;
  int32_t* slist[kUnits + 1][2];
  float* sstate[2];
  unsigned char* sorted;  // bucket-order buffers (sorted_layout), or null
};

static SolveWs handle_ws(const fpt_handle* h) {
  SolveWs W;
  memset(&W, 0, sizeof(W));
  W.sorted = (unsigned char*)h->sorted_mem;
  W.perm = h->perm;
  W.ccount = h->ccount;
  W.bucket = h->bucket;
  W.scount = h->scount;
  for (int w = 0; w <= kUnits; ++w)
    for (int k = 0; k < 2; ++k) W.slist[w][k] = h->slist[w][k];
  W.sstate[0] = h->sstate[0];
  W.sstate[1] = h->sstate[1];
  return W;
}

// The launches of one solve on stream st, with the plan P (which units run
// on streams of their own; their streams exist) in the workspace W (sized
// for pa->N).
static fpt_status solve_run(fpt_handle* h, const fpt_scene* sc, const fpt_paths* pa,
                            const fpt_opts* o, const fpt_out* out, hipStream_t st,
                            const SolvePlan& P, const SolveWs& W) {
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
  A.method = o->method;
  A.polish_steps = o->polish_steps;
  A.line_search = o->line_search;
  float ed = o->exit_rtol * o->scale;
  A.exit_d2 = ed * ed;
  A.scale = o->scale;
  A.n_levels = o->n_levels;
  for (int i = 0; i < FPT_MAX_LEVELS; ++i) {
    A.level_eps[i] = o->level_eps[i];
    A.level_steps[i] = o->level_steps[i];
  }
  A.cert_abs = o->cert_rtol * o->scale;
  A.quick_steps = o->n_levels > 0 ? o->quick_steps : 0;
  A.pad_outputs = 1;

  hipError_t e;
  int64_t cap = (pa->N + fpt::kBlock - 1) / fpt::kBlock;
  auto persistent = [&](int ph, int n, int wg_per_cu) -> int {
    int64_t g = (int64_t)h->num_cu * (wg_per_cu > 0 ? wg_per_cu : h->occ[ph][n]);
    return (int)(g < cap ? g : cap);
  };
  const int n_lo = P.n_lo;
  const int32_t* perm = nullptr;
  const int64_t* bucket = nullptr;
  // with a bucket-order workspace the per-order kernels see the paths in
  // bucket order (As, perm null); the caller's arrays are written at the end
  fpt::SolveArgs As = A, Af = A;
  const bool sorted = pa->order && W.sorted;
  const SortedLayout SL = sorted_layout(pa->N, pa->n_max);
  if (pa->order) {
    SlotTimer tm(h, FPT_T_BUCKET, st);
    e = fpt::launch_bucketing(pa->order, pa->N, pa->n_max, W.ccount, W.bucket, W.perm, st,
                              sorted ? (int32_t*)(W.sorted + SL.inv) : nullptr);
    if (e != hipSuccess) return hip_fail(e, "fpt_solve: bucketing launch");
    perm = W.perm;
    bucket = W.bucket;
    if (sorted) {
      unsigned char* b = W.sorted;
      As.x = (float*)(b + SL.x);
      As.len = (float*)(b + SL.len);
      As.t = (float*)(b + SL.t);
      As.iters = (uint16_t*)(b + SL.iters);
      As.status = b + SL.status;
      As.src = (const int32_t*)(b + SL.src);
      As.dst = (const int32_t*)(b + SL.dst);
      As.ids = (const int32_t*)(b + SL.ids);
      As.t_init = nullptr;
      As.order = nullptr;
      As.pad_outputs = 0;
      // the first phase gathers the inputs through the permutation
      Af = As;
      Af.perm_in = W.perm;
      Af.src_in = pa->src;
      Af.dst_in = pa->dst;
      Af.ids_in = pa->ids;
      Af.tinit_in = pa->t_init;
      Af.src_cp = (int32_t*)(b + SL.src);
      Af.dst_cp = (int32_t*)(b + SL.dst);
      Af.ids_cp = (int32_t*)(b + SL.ids);
      perm = nullptr;
    }
  }
  if (P.multi) {
    e = hipEventRecord(h->ev_fork, st);
    if (e != hipSuccess) return hip_fail(e, "fpt_solve: event record");
  }
  const int nc = fpt::kRegions * fpt::kCounterStride;
  const int64_t rcap = stage_rcap(pa->N);
  for (int i = 0; i <= pa->n_max - n_lo; ++i)
  for (int part = 0; part < P.split; ++part) {
    const int n = P.nth(i, part, pa->n_max);
    const int w = P.multi ? P.unit(n, part) : 0;  // list set and stream
    hipStream_t sn = P.multi ? h->ostream[w] : st;
    if (P.multi) {
      e = hipStreamWaitEvent(sn, h->ev_fork, 0);
      if (e != hipSuccess) return hip_fail(e, "fpt_solve: stream wait");
    }
    unsigned long long* cnt = W.scount + (size_t)w * 4 * nc;  // 4 stage blocks
    const fpt_launch_cfg& c = h->cfg[n];
    const bool ee = c.use_override ? c.early_exit != 0 : A.early_exit != 0;
    const int32_t* stages = (c.use_override && ee) ? c.stage_iters : o->stage_iters;
    fpt::SolveArgs An = As;
    An.sub = part;
    An.nsub = P.split;
    if (c.use_override && c.iters > 0) An.n_iter = c.iters;
    if (c.use_override && c.quick_steps > 0 && A.quick_steps > 0) An.quick_steps = c.quick_steps;
    const int qpasses = (c.use_override && c.quick_passes > 0) ? c.quick_passes : o->quick_passes;
    An.work = (h->timing && h->work) ? h->work + 6 * fpt::kWorkSlots * (n - 1) : nullptr;
    // the first phase (its first stage with early exit) gathers the inputs
    fpt::SolveArgs Anf = An;
    Anf.perm_in = Af.perm_in;
    Anf.src_in = Af.src_in;
    Anf.dst_in = Af.dst_in;
    Anf.ids_in = Af.ids_in;
    Anf.tinit_in = Af.tinit_in;
    Anf.src_cp = Af.src_cp;
    Anf.dst_cp = Af.dst_cp;
    Anf.ids_cp = Af.ids_cp;
    {
      SlotTimer tm(h, FPT_T_BFGS + n - 1, sn);
      if (!ee) {
        // one path per thread over the whole input, or persistent over the
        // bucket (its size is only known on the device)
        // (it also clears the counter blocks of the refinement's lists)
        const int ph = An.method == FPT_METHOD_NEWTON32 ? 5 : 0;
        int grid = bucket ? persistent(ph, n, c.wg_per_cu) : (int)cap;
        fpt::SolveArgs Ab = Anf;
        if (An.quick_steps > 0) {
          Ab.clear = cnt;
          Ab.clear_n = 4 * nc;
        }
        e = fpt::launch_solve(ph, n, Ab, perm, bucket, nullptr, grid, sn);
        if (e != hipSuccess) return hip_fail(e, "fpt_solve: launch");
      } else {
        int ns = 0;
        while (ns < FPT_MAX_STAGES && stages[ns] > 0) ++ns;
        for (int k = 0; k < ns; ++k) {
          fpt::StageArgs S;
          memset(&S, 0, sizeof(S));
          S.rcap = rcap;
          S.cap = rcap * fpt::kRegions;
          S.iters = stages[k];
          if (k > 0) {
            S.in_list = W.slist[w][(k - 1) & 1];
            S.in_count = cnt + ((k - 1) & 1) * nc;
            S.state_in = W.sstate[(k - 1) & 1];
          }
          if (k + 1 < ns) {
            S.out_list = W.slist[w][k & 1];
            S.out_count = cnt + (k & 1) * nc;
            S.state_out = W.sstate[k & 1];
            e = fpt::launch_zero_u64(S.out_count, nc, sn);
            if (e != hipSuccess) return hip_fail(e, "fpt_solve: launch");
          }
          int grid = (k == 0 && !bucket) ? (int)cap : persistent(2, n, c.wg_per_cu);
          e = fpt::launch_solve(2, n, k == 0 ? Anf : An, perm, bucket, &S, grid, sn);
          if (e != hipSuccess) return hip_fail(e, "fpt_solve: launch");
        }
      }
    }
    {
      SlotTimer tm(h, FPT_T_REFINE + n - 1, sn);
      fpt::StageArgs R;
      memset(&R, 0, sizeof(R));
      const int rw = c.refine_wg_per_cu;
      int grid = bucket ? persistent(1, n, rw) : (int)cap;
      if (An.quick_steps > 0) {
        // stage k lists its uncertified paths in list k & 1 with counter
        // block k; the blocks are cleared together first (by the first
        // phase's launch unless it ran in early-exit stages, which use them)
        if (ee) {
          e = fpt::launch_zero_u64(cnt, 4 * nc, sn);
          if (e != hipSuccess) return hip_fail(e, "fpt_solve: launch");
        }
        R.rcap = rcap;
        R.cap = rcap * fpt::kRegions;
        // pass 1: quick steps for all, list the uncertified paths
        R.out_list = W.slist[w][0];
        R.out_count = cnt;
        e = fpt::launch_solve(4, n, An, perm, bucket, &R, bucket ? persistent(4, n, rw) : (int)cap,
                              sn);
        if (e != hipSuccess) return hip_fail(e, "fpt_solve: launch");
        int k = 0;  // the stage whose list is current
        // stage k reads list k & 1 with counter block k, and (unless it is
        // the last) lists what it leaves in list (k + 1) & 1 with block k + 1;
        // at most four blocks: quick pass, second quick pass, collapse step,
        // full schedule
        auto next_stage = [&](int phase, int grid_x, bool last, int mode) -> hipError_t {
          fpt::StageArgs Q;
          memset(&Q, 0, sizeof(Q));
          Q.rcap = R.rcap;
          Q.cap = R.cap;
          Q.in_list = W.slist[w][k & 1];
          Q.in_count = cnt + k * nc;
          if (!last) {
            Q.out_list = W.slist[w][(k + 1) & 1];
            Q.out_count = cnt + (k + 1) * nc;
          }
          Q.mode = mode;
          ++k;
          return fpt::launch_solve(phase, n, An, nullptr, nullptr, &Q, grid_x, sn);
        };
        if (qpasses > 1) {
          // second quick pass on the paths the first did not certify
          e = next_stage(4, persistent(4, n, rw), false, 0);
          if (e != hipSuccess) return hip_fail(e, "fpt_solve: launch");
        }
        if (n >= 2) {
          // collapsed minimisers from the quick pass's point: merge attempt on
          // the list, the rest listed again for the full schedule
          e = next_stage(3, persistent(3, n, rw), false, 0);
          if (e != hipSuccess) return hip_fail(e, "fpt_solve: launch");
        }
        // the full schedule on the list; with n >= 2 it lists the paths it
        // leaves uncertified for a last collapse step from its own output,
        // where a collapse has come close enough to be told from a short
        // segment
        e = next_stage(1, persistent(1, n, rw), n < 2, 0);
        if (e != hipSuccess) return hip_fail(e, "fpt_solve: launch");
        if (n >= 2) e = next_stage(3, persistent(3, n, rw), true, 1);
      } else {
        e = fpt::launch_solve(1, n, An, perm, bucket, &R, grid, sn);
      }
      if (e != hipSuccess) return hip_fail(e, "fpt_solve: launch");
    }
    if (P.multi) {
      e = hipEventRecord(h->ev_join[w], sn);
      if (e != hipSuccess) return hip_fail(e, "fpt_solve: event record");
      e = hipStreamWaitEvent(st, h->ev_join[w], 0);
      if (e != hipSuccess) return hip_fail(e, "fpt_solve: stream wait");
    }
  }
  if (pa->order) {
    e = fpt::launch_invalid(As, perm, W.bucket, h->num_cu * 4, st);
    if (e != hipSuccess) return hip_fail(e, "fpt_solve: launch");
    if (sorted) {
      SlotTimer tm(h, FPT_T_UNSORT, st);
      e = fpt::launch_unsort(As, A, (const int32_t*)(W.sorted + SL.inv), W.bucket,
                             h->num_cu * 8, st);
      if (e != hipSuccess) return hip_fail(e, "fpt_solve: launch");
    }
  }
  return FPT_OK;
}


extern "C" fpt_status fpt_solve(fpt_handle* h, const fpt_scene* sc,
                                const fpt_paths* pa, const fpt_opts* o,
                                const fpt_out* out, void* stream) {
  fpt_status s = check_solve(h, sc, pa, o, out, "fpt_solve");
  if (s != FPT_OK || pa->N == 0) return s;
  DeviceGuard g(h->device);
  if (!g.ok) return fail(FPT_EHIP, "fpt_solve: hipSetDevice failed");
  const bool any_ee = uses_early_exit(h, o, pa->n_max);
  // The orders, and parts of one order's paths, are independent: each unit
  // can run on its own stream with its own path lists, so that the small
  // orders and the latency-bound tails of each unit's passes (collapse step,
  // full schedule) overlap other units' work.
  const SolvePlan P = solve_plan(pa, o, any_ee);
  s = prepare_solve(h, pa, o, any_ee, P);
  if (s != FPT_OK) return s;
  return solve_run(h, sc, pa, o, out, (hipStream_t)stream, P, handle_ws(h));
}

// ------------------------------------------------ allocation-free solve ----
// fpt_solve_noalloc works in a fixed array of device memory, `scratch`, in
// place of the handle's growing workspace: the order sort, one list set's
// counters and its two path lists, sized for kNoAllocPaths paths. Each GPU
// holds its own copy for the life of the process. In host code the array's
// name is not a device address: fpt_create looks up this device's copy once
// (hipGetSymbolAddress) and every use goes through that address.
static const int64_t kNoAllocPaths = (int64_t)1 << 20;
static const size_t kNaPermOff = 0;
static const size_t kNaCcountOff = kNaPermOff + (size_t)kNoAllocPaths * sizeof(int32_t);
static const size_t kNaBucketOff =
    kNaCcountOff + (size_t)(kNoAllocPaths / fpt::kSortChunk) * 8 * sizeof(uint32_t);
static const size_t kNaCountOff = kNaBucketOff + 256;
static const size_t kNaCountBytes =
    (size_t)4 * fpt::kRegions * fpt::kCounterStride * sizeof(unsigned long long);
static const size_t kNaListOff = kNaCountOff + kNaCountBytes;
static const size_t kNaListBytes =
    (size_t)64 * (kNoAllocPaths / (64 * fpt::kRegions) + 1) * fpt::kRegions * sizeof(int32_t);
static const size_t kNoAllocBytes = kNaListOff + 2 * kNaListBytes;
static_assert(kNoAllocPaths % fpt::kSortChunk == 0, "whole sort chunks");
static_assert(kNaListBytes % 256 == 0 && kNaCountBytes % 256 == 0, "aligned parts");

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// This device's address of `scratch`, looked up once per device (the
// caller's device is current).
static std::mutex g_scratch_mu;
static unsigned char* g_scratch_dev[64] = {};

static fpt_status scratch_address(int device, unsigned char** out) {
  *out = nullptr;
  if (device < 0 || device >= 64)
    return fail(FPT_EUNSUPPORTED, "fpt_create: device index above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "fpt_create: hipGetSymbolAddress(scratch)");
    if (!p) return fail(FPT_EHIP, "fpt_create: no device address for scratch");
    g_scratch_dev[device] = (unsigned char*)p;
  }
  *out = g_scratch_dev[device];
  return FPT_OK;
}

extern "C" int64_t fpt_noalloc_max_paths(void) { return kNoAllocPaths; }

extern "C" fpt_status fpt_solve_noalloc(fpt_handle* h, const fpt_scene* sc,
                                        const fpt_paths* pa, const fpt_opts* o,
                                        const fpt_out* out, void* stream) {
  fpt_status s = check_solve(h, sc, pa, o, out, "fpt_solve_noalloc");
  if (s != FPT_OK || pa->N == 0) return s;
  if (pa->N > kNoAllocPaths)
    return fail(FPT_EINVAL, "fpt_solve_noalloc: N above fpt_noalloc_max_paths() (2^20)");
  if (uses_early_exit(h, o, pa->n_max))
    return fail(FPT_EINVAL, "fpt_solve_noalloc: early exit needs the handle's workspace");
  if (!h->scratch) return fail(FPT_EHIP, "fpt_solve_noalloc: scratch address unknown");
  DeviceGuard g(h->device);
  if (!g.ok) return fail(FPT_EHIP, "fpt_solve_noalloc: hipSetDevice failed");
  // every unit on the caller's stream, one list set (the results do not
  // depend on the split or on concurrent orders)
  SolvePlan P = solve_plan(pa, o, false);
  P.multi = false;
  P.conc = false;
  P.split = 1;
  SolveWs W;
  memset(&W, 0, sizeof(W));
  unsigned char* base = h->scratch;
  W.perm = (int32_t*)(base + kNaPermOff);
  W.ccount = (uint32_t*)(base + kNaCcountOff);
  W.bucket = (int64_t*)(base + kNaBucketOff);
  W.scount = (unsigned long long*)(base + kNaCountOff);
  W.slist[0][0] = (int32_t*)(base + kNaListOff);
  W.slist[0][1] = (int32_t*)(base + kNaListOff + kNaListBytes);
  return solve_run(h, sc, pa, o, out, (hipStream_t)stream, P, W);
}

// LDS budget of the per-workgroup accumulation of the scene gradient (FP64
// tables: 25.6 KB for the 313-object canyon)
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
  size_t shmem = (9 * (size_t)sc->K + 3 * (size_t)sc->Q) * sizeof(double);
  A.lds = shmem <= kGradLdsMax ? 1 : 0;
  if (!A.lds) shmem = 0;
  int64_t cap = (pa->N + fpt::kBlock - 1) / fpt::kBlock;
  // the collapsed-path kernel takes 1024 entries per workgroup and pass
  const int64_t kkt_cap = (pa->N + 1023) / 1024;
  auto grid_for = [&](int n, bool kkt) -> int {
    const int64_t c = kkt ? kkt_cap : cap;
    if (!A.lds) return (int)c;  // one pass over the paths
    const void* fn = fpt::grad_kernel_ptr(n, kkt);
    if (!fn) return 1;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, fpt::kBlock, shmem) !=
            hipSuccess ||
        occ < 1)
      occ = 1;
    // (the collapsed-path kernel: at most two workgroups per CU. It sees a
    // fraction of the paths, and every workgroup clears and flushes its own
    // tables; at order 2, three per CU took 37 us against 31 with two)
    if (kkt && occ > 2) occ = 2;
    int64_t gsz = (int64_t)h->num_cu * occ;
    return (int)(gsz < c ? gsz : c);
  };
  hipError_t e;
  if (!pa->order) {
    SlotTimer tm(h, FPT_T_GRAD, st);
    e = fpt::launch_grad(pa->n_max, A, nullptr, nullptr, grid_for(pa->n_max, false),
                         grid_for(pa->n_max, true), shmem, st);
    if (e != hipSuccess) return hip_fail(e, "fpt_grad: launch");
    return FPT_OK;
  }
  s = ensure_perm(h, pa->N);
  if (s != FPT_OK) return s;
  int sgrid = h->num_cu * 4;
  {
    SlotTimer tm(h, FPT_T_BUCKET, st);
    e = fpt::launch_bucketing(pa->order, pa->N, pa->n_max, h->ccount,
                              h->bucket, h->perm, st, nullptr, fwd->status);
    if (e != hipSuccess) return hip_fail(e, "fpt_grad: bucketing launch");
  }
  {
    SlotTimer tm(h, FPT_T_GRAD, st);
    for (int n = 1; n <= pa->n_max; ++n) {
      // persistent grid: the bucket size is only known on the device
      int grid = A.lds ? grid_for(n, false) : (int)(cap < (int64_t)h->num_cu * 8 ? cap : (int64_t)h->num_cu * 8);
      int kgrid = A.lds ? grid_for(n, true) : (int)(kkt_cap < (int64_t)h->num_cu * 8 ? kkt_cap : (int64_t)h->num_cu * 8);
      e = fpt::launch_grad(n, A, h->perm, h->bucket, grid, kgrid, shmem, st);
      if (e != hipSuccess) return hip_fail(e, "fpt_grad: launch");
    }
    e = fpt::launch_grad_invalid(A, h->perm, h->bucket, sgrid, st);
    if (e != hipSuccess) return hip_fail(e, "fpt_grad: launch");
  }
  return FPT_OK;
}

// ---------------------------------------------------------- enumeration ----

static const int64_t kEnumLimit = (int64_t)1 << 62;

// Candidates per pair of every order of the spec, and the first rank of
// every order; false on a total above kEnumLimit.
static bool enum_layout(const fpt_enum_spec* sp, int64_t per_pair[FPT_NMAX + 1],
                        int64_t first[FPT_NMAX + 1]) {
  const int64_t radix = sp->no_repeat ? sp->K - 1 : sp->K;
  int64_t m = sp->K, acc = 0;
  for (int n = 1; n <= sp->order_max; ++n) {
    if (n > 1) {
      if (radix != 0 && m > kEnumLimit / radix) return false;
      m *= radix;
    }
    per_pair[n] = m;
    if (n >= sp->order_min) {
      first[n - sp->order_min] = acc;
      if (m != 0 && sp->P > (kEnumLimit - acc) / m) return false;
      acc += (int64_t)sp->P * m;
    }
  }
  first[sp->order_max - sp->order_min + 1] = acc;
  return true;
}

static fpt_status check_enum_spec(const fpt_enum_spec* sp, const char* who) {
  if (!sp) return fail(FPT_EINVAL, std::string(who) + ": spec is NULL");
  if (sp->P < 1 || sp->K < 1)
    return fail(FPT_EINVAL, std::string(who) + ": P and K must be >= 1");
  if (sp->order_min < 1 || sp->order_min > sp->order_max || sp->order_max > FPT_NMAX)
    return fail(FPT_EINVAL, std::string(who) + ": need 1 <= order_min <= order_max <= 6");
  if (sp->no_repeat != 0 && sp->no_repeat != 1)
    return fail(FPT_EINVAL, std::string(who) + ": no_repeat must be 0 or 1");
  return FPT_OK;
}

extern "C" fpt_status fpt_enum_count(const fpt_enum_spec* sp, int64_t* total) {
  fpt_status s = check_enum_spec(sp, "fpt_enum_count");
  if (s != FPT_OK) return s;
  if (!total) return fail(FPT_EINVAL, "fpt_enum_count: total is NULL");
  int64_t per_pair[FPT_NMAX + 1], first[FPT_NMAX + 1];
  if (!enum_layout(sp, per_pair, first))
    return fail(FPT_EINVAL, "fpt_enum_count: more than 2^62 candidates");
  *total = first[sp->order_max - sp->order_min + 1];
  return FPT_OK;
}

extern "C" fpt_status fpt_enumerate(fpt_handle* h, const fpt_enum_spec* sp, int64_t rank0,
                                    int64_t count, int32_t* src, int32_t* dst,
                                    uint8_t* order, int32_t* ids, int32_t n_max,
                                    void* stream) {
  if (!h) return fail(FPT_EINVAL, "fpt_enumerate: handle is NULL");
  fpt_status s = check_enum_spec(sp, "fpt_enumerate");
  if (s != FPT_OK) return s;
  if (n_max < sp->order_max || n_max > FPT_NMAX)
    return fail(FPT_EINVAL, "fpt_enumerate: n_max must be in order_max..6");
  fpt::EnumArgs A;
  memset(&A, 0, sizeof(A));
  if (!enum_layout(sp, A.per_pair, A.first))
    return fail(FPT_EINVAL, "fpt_enumerate: more than 2^62 candidates");
  const int64_t total = A.first[sp->order_max - sp->order_min + 1];
  if (rank0 < 0 || count < 0 || rank0 > total || count > total - rank0)
    return fail(FPT_EINVAL, "fpt_enumerate: ranks outside the candidate set");
  if (count == 0) return FPT_OK;
  if (!sp->pair_src || !sp->pair_dst || !src || !dst || !order || !ids)
    return fail(FPT_EINVAL, "fpt_enumerate: NULL pointer");
  if (!aligned(sp->pair_src, 4) || !aligned(sp->pair_dst, 4) || !aligned(src, 4) ||
      !aligned(dst, 4) || !aligned(ids, 4))
    return fail(FPT_EINVAL, "fpt_enumerate: misaligned pointer");
  DeviceGuard g(h->device);
  if (!g.ok) return fail(FPT_EHIP, "fpt_enumerate: hipSetDevice failed");
  A.pair_src = sp->pair_src;
  A.pair_dst = sp->pair_dst;
  A.src = src;
  A.dst = dst;
  A.order = order;
  A.ids = ids;
  A.rank0 = rank0;
  A.count = count;
  A.omin = sp->order_min;
  A.omax = sp->order_max;
  A.K = sp->K;
  A.no_repeat = sp->no_repeat;
  A.n_max = n_max;
  const int64_t blocks = (count + fpt::kBlock - 1) / fpt::kBlock;
  const int64_t cap = (int64_t)h->num_cu * 8;
  hipError_t e = fpt::launch_enumerate(A, (int)(blocks < cap ? blocks : cap),
                                       (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "fpt_enumerate: launch");
  return FPT_OK;
}

// ------------------------------------------------------------ validity ----

extern "C" fpt_status fpt_validate(fpt_handle* h, const fpt_scene* sc,
                                   const fpt_paths* pa, const fpt_out* fwd,
                                   uint8_t* flags, int32_t mode, void* stream) {
  if (!h) return fail(FPT_EINVAL, "fpt_validate: handle is NULL");
  fpt_status s = check_common(sc, pa, "fpt_validate");
  if (s != FPT_OK) return s;
  if (!fwd || !flags) return fail(FPT_EINVAL, "fpt_validate: fwd and flags are required");
  if (mode != FPT_VALIDATE_ALL && mode != FPT_VALIDATE_LAZY)
    return fail(FPT_EINVAL, "fpt_validate: unknown mode");
  const bool lazy = mode == FPT_VALIDATE_LAZY;
  if (pa->N == 0) return FPT_OK;
  if (!fwd->x || !fwd->t || !fwd->status)
    return fail(FPT_EINVAL, "fpt_validate: fwd.x, fwd.t and fwd.status are required");
  if (!aligned(fwd->x, 4) || !aligned(fwd->t, 4))
    return fail(FPT_EINVAL, "fpt_validate: misaligned pointer");
  DeviceGuard g(h->device);
  if (!g.ok) return fail(FPT_EHIP, "fpt_validate: hipSetDevice failed");
  hipStream_t st = (hipStream_t)stream;
  const int64_t kk = sc->K > 0 ? sc->K : 1;
  const int64_t need = 19 * kk + 64;
  if (h->faces_cap < need) {
    if (h->faces) (void)hipFree(h->faces);
    h->faces = nullptr;
    h->faces_cap = 0;
    void* p = nullptr;
    if (hipMalloc(&p, (size_t)need * sizeof(float)) != hipSuccess)
      return fail(FPT_ENOMEM, "fpt_validate: face table allocation failed");
    h->faces = (float*)p;
    h->faces_cap = need;
  }
  fpt::ValidateArgs A;
  memset(&A, 0, sizeof(A));
  A.obj = sc->obj;
  A.pts = sc->pts;
  A.src = pa->src;
  A.dst = pa->dst;
  A.ids = pa->ids;
  A.x = fwd->x;
  A.t = fwd->t;
  A.status = fwd->status;
  A.tab = h->faces;
  A.nrm = h->faces + 16 * kk;
  A.nfaces = (const int32_t*)(h->faces + 19 * kk);
  A.flags = flags;
  A.N = pa->N;
  A.K = sc->K;
  A.Q = sc->Q;
  A.n_max = pa->n_max;
  hipError_t e;
  SlotTimer tm(h, FPT_T_VALIDATE, st);
  e = fpt::launch_face_table(sc->obj, sc->K, h->faces, h->faces + 16 * kk,
                             (int32_t*)(h->faces + 19 * kk), st);
  if (e != hipSuccess) return hip_fail(e, "fpt_validate: launch");
  const int64_t cap = (pa->N + fpt::kBlock - 1) / fpt::kBlock;
  const int64_t pg = (int64_t)h->num_cu * 8;
  const int grid = (int)(cap < pg ? cap : pg);
  if (!pa->order) {
    e = fpt::launch_validate(pa->n_max, A, lazy, nullptr, nullptr, grid, st);
    if (e != hipSuccess) return hip_fail(e, "fpt_validate: launch");
    return FPT_OK;
  }
  s = ensure_perm(h, pa->N);
  if (s != FPT_OK) return s;
  e = fpt::launch_bucketing(pa->order, pa->N, pa->n_max, h->ccount, h->bucket, h->perm, st);
  if (e != hipSuccess) return hip_fail(e, "fpt_validate: bucketing launch");
  for (int n = 1; n <= pa->n_max; ++n) {
    e = fpt::launch_validate(n, A, lazy, h->perm, h->bucket, grid, st);
    if (e != hipSuccess) return hip_fail(e, "fpt_validate: launch");
  }
  e = fpt::launch_validate_invalid(A, h->perm, h->bucket, h->num_cu * 4, st);
  if (e != hipSuccess) return hip_fail(e, "fpt_validate: launch");
  return FPT_OK;
}

// ------------------------------------------------- learned initialiser ----

static const int64_t kMlpTrainMax = 65536;   // rows per training step

static fpt_status ensure_mlp(fpt_handle* h, int64_t rows) {
  if (h->mlp.cap >= rows) return FPT_OK;
  if (h->mlp_mem) {
    (void)hipFree(h->mlp_mem);
    h->mlp_mem = nullptr;
    h->mlp = fpt::MlpWork{};
  }
  size_t b16 = fpt::mlp_work_bf16_per_row() * (size_t)rows;
  size_t f32 = fpt::mlp_work_f32_per_row() * (size_t)rows;
  void* p = nullptr;
  if (hipMalloc(&p, b16 * 2 + f32 * 4 + 256) != hipSuccess)
    return fail(FPT_ENOMEM, "learned-initialiser workspace allocation failed");
  h->mlp_mem = p;
  fpt::mlp_carve(p, rows, h->mlp);
  return FPT_OK;
}

static fpt_status check_mlp_paths(const fpt_scene* sc, const fpt_paths* pa,
                                  const char* fn) {
  fpt_status s = check_common(sc, pa, fn);
  if (s != FPT_OK) return s;
  if (pa->n_max != fpt::kMlpOrder)
    return fail(FPT_EINVAL, std::string(fn) + ": the initialiser is for order-4 paths (n_max = 4)");
  return FPT_OK;
}

extern "C" int64_t fpt_mlp_state_floats(void) { return 5 * fpt::kParams; }

extern "C" fpt_status fpt_mlp_init(fpt_handle* h, float* state, uint64_t seed,
                                   void* stream) {
  if (!h || !state) return fail(FPT_EINVAL, "fpt_mlp_init: NULL argument");
  if (!aligned(state, 16)) return fail(FPT_EINVAL, "fpt_mlp_init: state not 16-byte aligned");
  DeviceGuard g(h->device);
  hipStream_t st = (hipStream_t)stream;
  fpt::MlpState S = fpt::mlp_state(state);
  hipError_t e = fpt::launch_mlp_init(S.w, S.m, S.v, seed, st);
  if (e != hipSuccess) return hip_fail(e, "fpt_mlp_init: launch");
  fpt::AdamArgs A = fpt::adam_args(S, nullptr, 0.f, 1);
  e = fpt::launch_mlp_adam(A, st);
  if (e != hipSuccess) return hip_fail(e, "fpt_mlp_init: launch");
  return FPT_OK;
}

extern "C" fpt_status fpt_mlp_train_step(fpt_handle* h, float* state,
                                         const fpt_scene* sc,
                                         const fpt_paths* pa,
                                         const fpt_out* target, float scale,
                                         float lr, int32_t step, float* loss,
                                         void* stream) {
  if (!h || !state || !target || !loss)
    return fail(FPT_EINVAL, "fpt_mlp_train_step: NULL argument");
  fpt_status s = check_mlp_paths(sc, pa, "fpt_mlp_train_step");
  if (s != FPT_OK) return s;
  if (pa->N < 64 || pa->N % 64 != 0 || pa->N > kMlpTrainMax)
    return fail(FPT_EINVAL, "fpt_mlp_train_step: batch must be a multiple of 64 in 64..65536");
  if (!target->t || !target->status)
    return fail(FPT_EINVAL, "fpt_mlp_train_step: target.t and target.status are required");
  if (!(scale > 0.f) || !(lr > 0.f) || step < 1)
    return fail(FPT_EINVAL, "fpt_mlp_train_step: scale, lr must be > 0 and step >= 1");
  if (!aligned(state, 16)) return fail(FPT_EINVAL, "fpt_mlp_train_step: state not 16-byte aligned");
  DeviceGuard g(h->device);
  hipStream_t st = (hipStream_t)stream;
  s = ensure_mlp(h, pa->N);
  if (s != FPT_OK) return s;
  fpt::MlpState S = fpt::mlp_state(state);
  fpt::MlpPrepArgs P = fpt::prep_args(sc, pa, 0, pa->N, scale, h->mlp, true);
  P.t = target->t;
  P.status = target->status;
  hipError_t e = fpt::launch_mlp_prep(P, st);
  if (e == hipSuccess) e = fpt::mlp_forward(S.w, S.wb, h->mlp, pa->N, true, st);
  if (e == hipSuccess) e = fpt::launch_mlp_loss(h->mlp, pa->N, loss, st);
  if (e == hipSuccess) e = fpt::mlp_backward(S.wbT, h->mlp, pa->N, S.grad, st);
  if (e == hipSuccess) {
    fpt::AdamArgs A = fpt::adam_args(S, S.grad, lr, step);
    e = fpt::launch_mlp_adam(A, st);
  }
  if (e != hipSuccess) return hip_fail(e, "fpt_mlp_train_step: launch");
  return FPT_OK;
}

extern "C" fpt_status fpt_mlp_infer(fpt_handle* h, const float* state,
                                    const fpt_scene* sc, const fpt_paths* pa,
                                    float scale, float* t_init, void* stream) {
  if (!h || !state || !t_init) return fail(FPT_EINVAL, "fpt_mlp_infer: NULL argument");
  fpt_status s = check_mlp_paths(sc, pa, "fpt_mlp_infer");
  if (s != FPT_OK) return s;
  if (!(scale > 0.f)) return fail(FPT_EINVAL, "fpt_mlp_infer: scale must be > 0");
  if (!aligned(state, 16) || !aligned(t_init, 4))
    return fail(FPT_EINVAL, "fpt_mlp_infer: misaligned pointer");
  if (pa->N == 0) return FPT_OK;
  DeviceGuard g(h->device);
  hipStream_t st = (hipStream_t)stream;
  fpt::MlpState S = fpt::mlp_state(const_cast<float*>(state));
  SlotTimer tm(h, FPT_T_MLP, st);
  // one fused kernel (features, layers, output): no workspace
  hipError_t e = fpt::launch_mlp_infer(sc, pa, S.w, S.wb, scale, t_init, st);
  if (e != hipSuccess) return hip_fail(e, "fpt_mlp_infer: launch");
  return FPT_OK;
}

// ------------------------------------------------ launch configuration ----

extern "C" fpt_status fpt_set_launch(fpt_handle* h, int order,
                                     const fpt_launch_cfg* cfg) {
  if (!h) return fail(FPT_EINVAL, "fpt_set_launch: handle is NULL");
  if (order < 1 || order > FPT_NMAX)
    return fail(FPT_EINVAL, "fpt_set_launch: order outside 1..6");
  if (!cfg) {
    h->cfg[order] = fpt_launch_cfg{};
    return FPT_OK;
  }
  if (cfg->wg_per_cu < 0 || cfg->wg_per_cu > 32 || cfg->refine_wg_per_cu < 0 ||
      cfg->refine_wg_per_cu > 32)
    return fail(FPT_EINVAL, "fpt_set_launch: wg_per_cu / refine_wg_per_cu outside 0..32");
  if (cfg->use_override && (cfg->iters < 0 || cfg->iters > 65535))
    return fail(FPT_EINVAL, "fpt_set_launch: iters outside 0..65535");
  if (cfg->use_override && (cfg->quick_steps < 0 || cfg->quick_steps > 64 ||
                            cfg->quick_passes < 0 || cfg->quick_passes > 2))
    return fail(FPT_EINVAL, "fpt_set_launch: quick_steps / quick_passes out of range");
  if (cfg->use_override && cfg->early_exit) {
    if (cfg->stage_iters[0] < 1)
      return fail(FPT_EINVAL, "fpt_set_launch: early exit needs stage_iters[0] >= 1");
    for (int k = 0; k < FPT_MAX_STAGES; ++k)
      if (cfg->stage_iters[k] < 0 || cfg->stage_iters[k] > 65535)
        return fail(FPT_EINVAL, "fpt_set_launch: stage_iters outside 0..65535");
  }
  h->cfg[order] = *cfg;
  return FPT_OK;
}

// -------------------------------------------------------- graph capture ----

struct fpt_graph {
  int device;
  fpt_handle* h = nullptr;  // whose workspace the graph records
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" fpt_status fpt_graph_capture(fpt_handle* h, const fpt_scene* sc,
                                        const fpt_paths* pa,
                                        const fpt_opts* o, const fpt_out* out,
                                        void* stream, fpt_graph** g) {
  if (!h || !g) return fail(FPT_EINVAL, "fpt_graph_capture: NULL argument");
  *g = nullptr;
  if (!stream) return fail(FPT_EINVAL, "fpt_graph_capture: needs a non-default stream");
  fpt_status s = check_common(sc, pa, "fpt_graph_capture");
  if (s != FPT_OK) return s;
  s = check_opts(o);
  if (s != FPT_OK) return s;
  if (h->timing) return fail(FPT_EINVAL, "fpt_graph_capture: disable timing first");
  DeviceGuard dg(h->device);
  hipStream_t st = (hipStream_t)stream;
  // no allocation inside the capture
  {
    const bool any_ee = uses_early_exit(h, o, pa->n_max);
    s = prepare_solve(h, pa, o, any_ee, solve_plan(pa, o, any_ee));
    if (s != FPT_OK) return s;
  }
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return hip_fail(e, "fpt_graph_capture: begin");
  fpt_status rs = fpt_solve(h, sc, pa, o, out, stream);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(st, &graph);
  if (rs != FPT_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rs;
  }
  if (e != hipSuccess) return hip_fail(e, "fpt_graph_capture: end");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return hip_fail(e, "fpt_graph_capture: instantiate");
  }
  fpt_graph* G = new fpt_graph();
  G->device = h->device;
  G->h = h;
  h->live_graphs += 1;
  G->graph = graph;
  G->exec = exec;
  *g = G;
  return FPT_OK;
}

extern "C" fpt_status fpt_graph_launch(fpt_graph* g, void* stream) {
  if (!g) return fail(FPT_EINVAL, "fpt_graph_launch: graph is NULL");
  DeviceGuard dg(g->device);
  hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "fpt_graph_launch");
  return FPT_OK;
}

extern "C" fpt_status fpt_graph_destroy(fpt_graph* g) {
  if (!g) return FPT_OK;
  DeviceGuard dg(g->device);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->h) g->h->live_graphs -= 1;
  delete g;
  return FPT_OK;
}
