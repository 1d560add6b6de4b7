/*
 * fpt.h - C ABI of the MI355X (gfx950) Fermat path solver.
 *
 * The library minimises the total length of many independent candidate ray
 * paths (Sec. III-B, Eqs. 1-5):
 *     x_0 = TX,  x_j = A_j t_j + b_j  (j = 1..n),  x_{n+1} = RX,
 *     L(T) = sum_{i=0}^{n} || x_{i+1} - x_i ||,   T* = arg min_T L(T).
 * A_j holds the two basis vectors of object j: a plane (reflection, d = 2),
 * or an edge (diffraction, d = 1) padded to d = 2 with a zero second vector,
 * so that every path of order n has one fixed layout (Sec. III-B).
 * The solve is the paper's BFGS with the fixed-point step-size iteration of
 * Eq. 6 (Sec. III-C) in FP32, followed by FP64 Newton refinement steps on the
 * block-tridiagonal Hessian. The gradient is the implicit-differentiation
 * vector-Jacobian product of Sec. III-D (Eqs. 8-13).
 *
 * Memory: every pointer passed to fpt_solve / fpt_grad is a DEVICE pointer
 * owned by the caller; the library never frees it. All arrays are
 * structure-of-arrays with the path index fastest (coalesced):
 *   obj   float [9][K]      rows b(3), a1(3), a2(3); a2 == 0 (all three
 *                           components exactly 0) marks an edge
 *   pts   float [3][Q]      endpoint table
 *   src, dst int32 [N]      x_0 = pts[:, src[i]], x_{n+1} = pts[:, dst[i]]
 *   order uint8 [N]         interactions of path i, 1..n_max; NULL means
 *                           every path has order n_max
 *   ids   int32 [n_max][N]  object of interaction j of path i (entries
 *                           beyond the path's order are ignored)
 *   t_init float [n_max][2][N] or NULL (start at T = 0, i.e. x_j = b_j)
 * Outputs (written for every path):
 *   x      float  [n_max][3][N]   interaction points X*
 *   len    float  [N]             L(T*)
 *   t      float  [n_max][2][N]   T* in the caller's parametrisation (the
 *                                 padded parameter of an edge is 0)
 *   status uint8  [N]             FPT_ST_* bits
 *   iters  uint16 [N]             BFGS iterations run
 * Entries beyond a path's order are written as NaN (x, t).
 * t_init may be the same memory as the output t (a warm start from an
 * earlier solve's result); no other input may overlap an output.
 *
 * Errors: a whole-call error (null or misaligned pointer, n_max outside
 * 1..FPT_NMAX, N < 0, K/Q out of range, bad options) returns a negative
 * fpt_status and launches nothing; fpt_last_error() describes it. A problem
 * of a single path (order outside 1..n_max, an id or point index out of
 * range, non-finite input) is not a call error: that path gets
 * FPT_ST_INVALID and NaN outputs.
 *
 * Execution: asynchronous on the caller's HIP stream (hipStream_t passed as
 * void*; NULL = the legacy default stream). Input buffers must stay valid
 * until the stream has passed the call. The handle owns a device workspace
 * that grows on demand (hipMalloc) and is freed by fpt_destroy; calls that
 * share a handle must be ordered on one stream.
 */
#ifndef FPT_H
#define FPT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { FPT_NMAX = 6, FPT_MAX_LEVELS = 8, FPT_MAX_STAGES = 4 };

typedef enum {
  FPT_OK = 0,
  FPT_EINVAL = -1,      /* bad argument; nothing launched */
  FPT_EUNSUPPORTED = -2,/* no gfx950 device, or feature not built */
  FPT_EHIP = -3,        /* a HIP runtime call failed */
  FPT_ENOMEM = -4       /* workspace allocation failed */
} fpt_status;

/* per-path status bits */
enum {
  FPT_ST_CONVERGED = 1, /* FP64 Newton certificate: the last two Newton steps
                           were taken in full and each moved no point by
                           more than cert_rtol * scale; no short segment
                           with a near-unit smoothed direction remains. Or,
                           for a minimiser where two consecutive interaction
                           points coincide (with FPT_ST_COLLAPSED): the path
                           with the two merged on the intersection of their
                           objects passed that certificate, and a subgradient
                           of the zero-length segment of norm below 1
                           (squared norm <= 1 - 1e-6)
                           satisfies the stationarity of both points */
  FPT_ST_REFINED = 2,   /* at least one FP64 refinement step was accepted */
  FPT_ST_COLLAPSED = 4, /* two consecutive points closer than 1e-6 * scale */
  FPT_ST_NONFINITE = 8, /* the solve produced a non-finite value */
  FPT_ST_INVALID = 16,  /* bad order / id / point index, or non-finite input */
  FPT_ST_NOGRAD = 32    /* fpt_grad gives this path no gradient (zero): set
                           with FPT_ST_NONFINITE or FPT_ST_INVALID, and with
                           FPT_ST_COLLAPSED unless the collapse is one
                           interior zero-length segment whose two objects'
                           unit directions span space (the determinant of
                           the sum of their outer products above 1e-3) */
};

typedef struct fpt_handle fpt_handle;

typedef struct {
  int32_t K;          /* objects */
  const float* obj;   /* [9][K] device */
  int32_t Q;          /* points */
  const float* pts;   /* [3][Q] device */
} fpt_scene;

typedef struct {
  int64_t N;              /* paths (0 is allowed: nothing is launched) */
  int32_t n_max;          /* 1..FPT_NMAX */
  const int32_t* src;     /* [N] */
  const int32_t* dst;     /* [N] */
  const uint8_t* order;   /* [N] or NULL */
  const int32_t* ids;     /* [n_max][N] */
  const float* t_init;    /* [n_max][2][N] or NULL */
} fpt_paths;

typedef struct {
  int32_t iters;        /* BFGS iterations (Sec. III-C runs a fixed count) */
  int32_t fp_iters;     /* fixed-point iterations of Eq. 6 per BFGS step */
  int32_t early_exit;   /* 0: every path runs exactly `iters` iterations.
                           1: a path stops after two consecutive steps that
                           move no point by more than exit_rtol * scale (or
                           after `iters` in total); the solver runs in stages
                           of stage_iters[k] iterations, and the paths still
                           running after a stage are compacted (with their
                           BFGS state) for the next one */
  float exit_rtol;
  float scale;          /* scene size S (> 0): unit of every tolerance */
  int32_t n_levels;     /* FP64 refinement levels, 0..FPT_MAX_LEVELS */
  float level_eps[FPT_MAX_LEVELS];  /* smoothing eps / scale of each level
                                       (0 = exact length) */
  int32_t level_steps[FPT_MAX_LEVELS]; /* Newton steps at each level */
  float cert_rtol;      /* certificate threshold / scale */
  int32_t stage_iters[FPT_MAX_STAGES]; /* early exit: iterations per stage,
                           0-terminated; the last stage hands over every
                           path that is still running */
  int32_t quick_steps;  /* > 0: refinement in two passes; first quick_steps
                           Newton steps at the last level for every path,
                           then the full schedule for the paths that pass
                           did not certify (the certificate needs two steps,
                           so 1 certifies nothing in the first pass).
                           0: the full schedule for all */
  int32_t quick_passes; /* 1 or 2: with 2, the paths the first quick pass
                           does not certify get a second quick pass of
                           quick_steps more steps (compacted) before the
                           rest of the pipeline */
  int32_t concurrent_orders; /* 1: with several orders (and no early exit),
                           each order's kernels run on a stream of their own
                           (forked from and joined back into hip_stream);
                           0: one after the other on hip_stream */
  int32_t method;       /* first phase: FPT_METHOD_BFGS, the paper's FP32 BFGS
                           with the Eq. 6 step (Sec. III-C); or
                           FPT_METHOD_NEWTON32, a solver variant: damped
                           Newton in FP32 on the exact block-tridiagonal
                           Hessian of the smoothed length, `iters` steps split
                           evenly over eps / scale = 1e-2, 1e-3, 1e-4, 1e-5,
                           majorant step when the full step lengthens the
                           path (no early exit). The FP64 refinement, the
                           certificate and the outputs are the same */
  int32_t polish_steps; /* 0..8: FP32 Newton steps on the exact Hessian of the
                           length (smoothed by 1e-7 scale) at the end of the
                           BFGS phase, before the FP64 refinement; they start
                           it within FP32 precision of the minimiser, so that
                           fewer FP64 steps reach the certificate */
  int32_t split;        /* 0..4: each order's paths are solved in `split`
                           equal parts, each on its own stream (forked from
                           and joined back into hip_stream), so that one
                           part's latency-bound passes overlap another's;
                           the results are the same. 0: 2 parts from 2^21
                           paths on, else 1. Early exit uses 1 */
  int32_t line_search;  /* step size of the BFGS (method FPT_METHOD_BFGS, fixed
                           iteration count): FPT_LS_EQ6, the fixed-point
                           iteration of Eq. 6 (Sec. III-C, the paper's); or
                           FPT_LS_ARMIJO, a solver variant (Sec. V names
                           better line searches): backtracking from the unit
                           step, halved until L(T + a P) <= L(T) + 1e-4 a g.P,
                           at most 8 times, else the majorant step of Eq. 6
                           from 0. Early exit uses FPT_LS_EQ6 */
} fpt_opts;

enum { FPT_METHOD_BFGS = 0, FPT_METHOD_NEWTON32 = 1 };
enum { FPT_LS_EQ6 = 0, FPT_LS_ARMIJO = 1 };

/* Defaults: the BFGS method, 64 iterations, 1 fixed-point iteration, 1
 * polish step, no early exit (exit_rtol = 1e-6, stages of 16, 16 and 32
 * iterations), refinement levels eps/S = 1e-3, 1e-5, 1e-7 (2 steps each) and
 * 1e-9 (3 steps) after a quick pass of 2 steps at 1e-9 (twice: quick_passes
 * = 2), cert_rtol = 1e-5, scale = 1, orders one after another, split 0
 * (automatic), the Eq. 6 step (line_search = FPT_LS_EQ6). */
void fpt_default_opts(fpt_opts* opts);

typedef struct {
  float* x;         /* [n_max][3][N] */
  float* len;       /* [N] */
  float* t;         /* [n_max][2][N] */
  uint8_t* status;  /* [N] */
  uint16_t* iters;  /* [N] */
} fpt_out;

/* Creates a handle bound to HIP device `device` (must be gfx950).
 * *h receives the handle, or NULL on error. */
fpt_status fpt_create(int device, fpt_handle** h);

/* Frees the handle and its workspace (synchronises the device first).
 * FPT_EINVAL (and nothing freed) while a graph captured on the handle
 * (fpt_graph_capture) has not been destroyed. */
fpt_status fpt_destroy(fpt_handle* h);

/* Solves every path (Sec. III-B Eq. 4 by the BFGS / fixed-point method of
 * Sec. III-C, then FP64 refinement). See the layout notes above. With
 * quick_steps > 0, the paths of order >= 2 that the quick pass does not
 * certify and that have exactly one short interior segment are first tried
 * as collapsed minimisers (see FPT_ST_CONVERGED); the rest get the full
 * schedule. */
fpt_status fpt_solve(fpt_handle* h, const fpt_scene* scene,
                     const fpt_paths* paths, const fpt_opts* opts,
                     const fpt_out* out, void* hip_stream);

/* Allocation-free variant of fpt_solve, for callers that cannot allocate
 * device memory during the call (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc). Same arguments, outputs and
 * per-path results as fpt_solve (bit for bit), but it never calls hipMalloc
 * or hipFree: its workspace (the order sort and the refinement's path lists)
 * is a fixed array of device memory that the library holds on each GPU from
 * the first fpt_create on that device until the process ends, sized for
 * fpt_noalloc_max_paths() paths (2^20; about 12.7 MB). Limits: N above that
 * maximum, or early exit in opts or in a launch configuration of the handle,
 * return FPT_EINVAL and launch nothing. Every unit runs on hip_stream (the
 * split and concurrent_orders options do not apply). Every call on one GPU
 * shares that array, and it keeps the last call's contents: calls that
 * overlap on one GPU (on different streams, or from different handles or
 * threads) race and must be ordered by the caller. The kernels clear what
 * must start at zero. */
fpt_status fpt_solve_noalloc(fpt_handle* h, const fpt_scene* scene,
                             const fpt_paths* paths, const fpt_opts* opts,
                             const fpt_out* out, void* hip_stream);
int64_t fpt_noalloc_max_paths(void);

/* Implicit-differentiation backward pass (Sec. III-D, Eqs. 8-13) at the
 * solution `fwd` of fpt_solve, for the loss
 *     sum_i g_len[i] * len[i] + sum_{i,j} g_x[j][:][i] . x[j][:][i].
 * g_len [N] and g_x [n_max][3][N] may each be NULL (= zero).
 * Accumulates (+=, caller zeroes) d loss / d pts into g_pts [3][Q] and
 * d loss / d obj into g_obj [9][K] (rows b, a1, a2; the padded a2 of an
 * edge receives nothing). g_slot [n_max][9][N] (optional, may be NULL)
 * receives the unreduced per-path, per-interaction object gradient; g_end
 * [6][N] (optional) the per-path TX and RX gradients. A collapsed minimiser
 * without FPT_ST_NOGRAD (one interior zero-length segment) is differentiated
 * as the minimiser of the length without that segment under the constraint
 * that its two points coincide (the implicit function theorem of Sec. III-D
 * applied to that problem's KKT conditions; the Hessian of Eq. 12 itself is
 * unbounded there). Paths with FPT_ST_NOGRAD contribute zero. */
fpt_status fpt_grad(fpt_handle* h, const fpt_scene* scene,
                    const fpt_paths* paths, const fpt_out* fwd,
                    const float* g_len, const float* g_x, float* g_pts,
                    float* g_obj, float* g_slot, float* g_end,
                    void* hip_stream);

/* Validity of solved paths on finite objects: the post-processing step
 * after the solve (Sec. III names finite objects and obstruction but leaves
 * them out; the solver treats every object as its infinite plane or line).
 * A face is the parallelogram b + s a1 + u a2 with s, u in [0, 1]; an edge
 * the segment b + s a1 with s in [0, 1]. For every path, flags[i] gets
 *   FPT_VALID_EXTENT    every interaction parameter (fwd->t) in [0, 1];
 *   FPT_VALID_SPECULAR  at every face, the previous and next points lie
 *                       strictly on the same side of its plane (a reflection,
 *                       not a pass-through);
 *   FPT_VALID_VISIBLE   no segment crosses a face of the scene other than
 *                       the faces of its own end points (a crossing: at
 *                       segment parameter in (1e-6, 1 - 1e-6), face
 *                       parameters in [0, 1]; edges occlude nothing).
 * A path is valid when all three are set. Paths with FPT_ST_INVALID or
 * FPT_ST_NONFINITE in fwd->status, or an order outside 1..n_max, get 0.
 * Needs fwd->x, fwd->t, fwd->status (device pointers) and flags [N] (device).
 * mode FPT_VALIDATE_ALL tests every segment of every path against every
 * face: O(N n F) for F faces. mode FPT_VALIDATE_LAZY tests occlusion only for
 * the paths that have EXTENT and SPECULAR (gathered per workgroup first) and
 * leaves FPT_VALID_VISIBLE clear on the others; the set of valid paths (all
 * three bits) is the same in both modes. Uses tables of 19 K + 64 floats in
 * the handle's workspace (hipMalloc on growth). */
enum { FPT_VALID_EXTENT = 1, FPT_VALID_SPECULAR = 2, FPT_VALID_VISIBLE = 4 };
enum { FPT_VALIDATE_ALL = 0, FPT_VALIDATE_LAZY = 1 };
fpt_status fpt_validate(fpt_handle* h, const fpt_scene* scene,
                        const fpt_paths* paths, const fpt_out* fwd,
                        uint8_t* flags, int32_t mode, void* hip_stream);

/* Launch configuration of the kernels of one order (what the autotuner
 * chooses). wg_per_cu: workgroups per compute unit of the persistent
 * first-phase launches (0 = as many as the kernel's register use lets
 * reside at once; more than that oversubscribes the CUs, which then take a
 * new workgroup as one ends); refine_wg_per_cu: the same for the FP64
 * refinement launches (quick passes, collapse steps, full schedule);
 * early_exit / stage_iters / iters / quick_steps / quick_passes (each if
 * > 0) override the corresponding fpt_opts fields for paths of that order
 * when use_override is 1. */
/* Candidate enumeration on the device (Sec. III, problem statement: the
 * candidates with n interactions are every ordered sequence of n objects,
 * for n = 1..n_max, per TX/RX pair). The candidates, in rank order:
 *   for n = order_min .. order_max, for pair p = 0 .. P-1, every sequence
 *   (k_1, .., k_n) of object indices in 0..K-1, in lexicographic order,
 *   leaving out those with k_{j+1} == k_j when no_repeat is 1.
 * Order n has P * M_n candidates, M_n = K (K-1)^(n-1) with no_repeat and
 * K^n without. */
typedef struct {
  const int32_t* pair_src;  /* [P] device: point index (into pts) of pair p's TX */
  const int32_t* pair_dst;  /* [P] device: point index of pair p's RX */
  int32_t P;                /* pairs, >= 1 */
  int32_t K;                /* objects, >= 1 */
  int32_t order_min;        /* 1 .. order_max */
  int32_t order_max;        /* order_min .. FPT_NMAX */
  int32_t no_repeat;        /* 0 or 1 */
} fpt_enum_spec;

/* Number of candidates of `spec` into *total (host arithmetic only; the
 * device pointers are not read). FPT_EINVAL for a bad spec or a total
 * above 2^62. */
fpt_status fpt_enum_count(const fpt_enum_spec* spec, int64_t* total);

/* Writes the candidates of ranks rank0 .. rank0 + count - 1 as paths
 * 0 .. count - 1, in the fpt_paths layout with N = count: src [count],
 * dst [count] (from the pair tables), order [count] (u8), ids [n_max][count]
 * (-1 past the path's order). All device pointers, caller-owned; n_max in
 * order_max .. FPT_NMAX. rank0 < 0, count < 0 or rank0 + count above the
 * total is FPT_EINVAL; count == 0 launches nothing. One kernel on
 * `hip_stream`, no allocation: a caller can stream a candidate set of any
 * size through fixed buffers, chunk by chunk. */
fpt_status fpt_enumerate(fpt_handle* h, const fpt_enum_spec* spec, int64_t rank0,
                         int64_t count, int32_t* src, int32_t* dst, uint8_t* order,
                         int32_t* ids, int32_t n_max, void* hip_stream);

typedef struct {
  int32_t wg_per_cu;
  int32_t use_override;
  int32_t early_exit;
  int32_t stage_iters[FPT_MAX_STAGES];
  int32_t iters;        /* 0..65535; 0 = fpt_opts.iters */
  int32_t quick_steps;  /* 0..64; 0 = fpt_opts.quick_steps */
  int32_t quick_passes; /* 0..2; 0 = fpt_opts.quick_passes */
  int32_t refine_wg_per_cu; /* 0..32 */
} fpt_launch_cfg;

/* Sets (cfg != NULL) or resets to defaults (cfg == NULL) the configuration
 * of order `order` (1..6) on this handle. */
fpt_status fpt_set_launch(fpt_handle* h, int order, const fpt_launch_cfg* cfg);

/* HIP-graph capture of one complete fpt_solve (order bucketing, every
 * per-order launch, refinement) on a non-default stream. The graph records
 * the given pointers and options: replays read and write the same buffers.
 * The handle's workspace is sized before the capture; counters are cleared
 * by kernels inside the graph (no memset nodes), so a replay can follow any
 * other work. fpt_graph_launch replays it on `hip_stream`.
 * The graph also records the handle's workspace. Until it is destroyed, a
 * call on the handle that would grow (and so free) a workspace buffer the
 * graph uses returns FPT_EINVAL and launches nothing, and fpt_destroy is
 * refused; capture the largest problem first, or use one handle per size. */
typedef struct fpt_graph fpt_graph;
fpt_status fpt_graph_capture(fpt_handle* h, const fpt_scene* scene,
                             const fpt_paths* paths, const fpt_opts* opts,
                             const fpt_out* out, void* hip_stream,
                             fpt_graph** g);
fpt_status fpt_graph_launch(fpt_graph* g, void* hip_stream);
fpt_status fpt_graph_destroy(fpt_graph* g);

/* Optional per-kernel timing. While enabled, every kernel (group) that
 * fpt_solve and fpt_grad launch is bracketed by a pair of HIP events recorded
 * on the caller's stream, into a ring of 32 event pairs per slot (no host
 * synchronisation is added). fpt_kernel_times waits for the recorded events
 * and writes, per timer slot, the mean duration in milliseconds over the
 * launches recorded since the previous read (at most the last 32), or -1 if
 * there were none, to ms[FPT_TIMERS]; it then clears the counts. Slots:
 *   FPT_T_BUCKET           order bucketing (count, scan, scatter) and the
 *                          copy of the paths' indices into bucket order
 *   FPT_T_BFGS + n - 1     FP32 BFGS kernel of order n (n = 1..6)
 *   FPT_T_REFINE + n - 1   FP64 refinement kernel of order n
 *   FPT_T_GRAD             implicit-differentiation kernel
 *   FPT_T_REDUCE           per-object gradient reduction
 *   FPT_T_MLP              learned-initialiser inference
 *   FPT_T_VALIDATE         path validity (fpt_validate)
 *   FPT_T_UNSORT           the copy of the outputs from bucket order to the
 *                          caller's order (solves with an order array)
 * Enabling allocates the events (returns FPT_EHIP if that fails). */
enum {
  FPT_T_BUCKET = 0,
  FPT_T_BFGS = 1,
  FPT_T_REFINE = 7,
  FPT_T_GRAD = 13,
  FPT_T_REDUCE = 14,
  FPT_T_MLP = 15,
  FPT_T_VALIDATE = 16,
  FPT_T_UNSORT = 17,
  FPT_TIMERS = 18
};
fpt_status fpt_set_timing(fpt_handle* h, int enable);
fpt_status fpt_kernel_times(fpt_handle* h, float* ms);

/* Work done by the FP64 refinement while timing is enabled, for the
 * algorithmic operation count of its kernels: for order n = 1..6,
 *   counts[6(n-1)]     evaluations of the (smoothed) path: points, segment
 *                      lengths and unit vectors, total length;
 *   counts[6(n-1)+1]   trial lengths of a Newton step (points, segment
 *                      lengths, total length: no unit vectors);
 *   counts[6(n-1)+2]   Newton solves (gradient, block-tridiagonal solve);
 * of the refinement passes, and counts[6(n-1)+3 .. 6(n-1)+5] the same for
 * the reduced paths of order n-1 solved by the collapse (merge) step. Summed
 * over the launches since the previous read; the counters are then cleared.
 * Synchronises the device. All zero if timing was never enabled. */
fpt_status fpt_work_counts(fpt_handle* h, uint64_t counts[6 * FPT_NMAX]);

/* Learned initialiser (a better initial candidate, which Sec. V names as
 * future work): an MLP 66 -> 256 -> 256 -> 256 -> 8 with ReLU that maps the
 * geometry of an order-4 path to starting parameters for fpt_solve. BF16
 * MFMA products with FP32 accumulation; FP32 master weights and Adam.
 * Inputs, per path, all lengths divided by `scale`: TX, RX, and for each of
 * the 4 interactions b, a1/|a1|, a2/|a2| (0 for an edge), b - TX, b - RX.
 * Outputs: the 8 parameters in unit-basis coordinates divided by `scale`.
 *
 * `state` is a caller-owned device buffer of fpt_mlp_state_floats() floats,
 * 16-byte aligned (weights, Adam moments, gradient, bf16 copies); its layout
 * is private. The handle keeps an activation workspace (hipMalloc on growth).
 * Paths: n_max must be 4; `order` is ignored (every path has order 4). */
int64_t fpt_mlp_state_floats(void);

/* He-normal weights from a counter-based hash of `seed`, zero biases and
 * Adam moments. */
fpt_status fpt_mlp_init(fpt_handle* h, float* state, uint64_t seed,
                        void* hip_stream);

/* One Adam step (lr, step = 1, 2, ... for the bias correction) on a batch of
 * N paths (N a multiple of 64, at most 65536). The target is a solver output
 * on the same paths (`target->t`, `target->status`): the loss is the mean
 * squared error between prediction and T* (unit-basis coordinates / scale)
 * over certified paths and non-padded parameters; *loss (a device float) is
 * incremented by the batch loss. */
fpt_status fpt_mlp_train_step(fpt_handle* h, float* state,
                              const fpt_scene* scene, const fpt_paths* paths,
                              const fpt_out* target, float scale, float lr,
                              int32_t step, float* loss, void* hip_stream);

/* Predicted start t_init [4][2][N] (caller's parametrisation) for every
 * path, to pass as paths->t_init to fpt_solve. */
fpt_status fpt_mlp_infer(fpt_handle* h, const float* state,
                         const fpt_scene* scene, const fpt_paths* paths,
                         float scale, float* t_init, void* hip_stream);

/* Thread-local description of the last non-OK status of this thread. */
const char* fpt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FPT_H */
