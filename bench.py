#!/usr/bin/env python3
"""Throughput of the Fermat path solver on one MI355X.

Headline workload (default): the street canyon (24 boxes, 121 faces + 192
edges, 64 TX/RX pairs), 8,388,608 sampled interaction sequences of orders
1..6 with P(n) proportional to 2^-n, mixed in one call: order bucketing,
per-order persistent launches (orders on streams of their own) and the FP64
refinement, captured as one HIP graph and replayed. The per-order schedule
(BFGS iteration count, quick refinement passes) is chosen by the autotuner on
a sample before timing, or fixed with --schedule. One step = one graph
replay over all paths, inputs resident in HBM. Metric: converged paths per
second, where converged means certified by the kernel's FP64 check (smooth
Newton certificate, or the subgradient test of a collapsed minimiser); the
cpu_baseline leg times the FP64 oracle on the host and checks the GPU
outputs against it.

Legs that follow (each can be switched off): all 6,270,016 order <= 2
sequences (c2) with validity, enumeration and the FP32 Newton variant on
them; solve + implicit gradient on 2^20 order-3 paths with unrolled autodiff
for comparison (fwd_grad); the learned initialiser trained on 2^22 order-4
paths and evaluated on 2^20 others (learned_init).

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32 = 157.3e12      # published FP32 vector peak (counts packed FP32)
PEAK_FP32_UNPACKED = 78.6e12  # 256 CU x 64 lanes x 2 flop x 2.4 GHz
PEAK_FP64 = 78.6e12        # published FP64 vector peak
PEAK_HBM = 8.0e12
PEAK_BF16 = 2.5e15         # dense BF16 MFMA


# ------------------------------------------------- algorithmic counts -----
# The method's own work, independent of how the kernels are written:
#   one BFGS iteration of an order-n path with m parameters: gradient
#   (points, segments, reciprocal square roots, projections), direction
#   P = -H g (2 m^2), the fixed-point step of Eq. 6, the update T += a P and
#   the inverse-Hessian update (5 m^2):  7 m^2 + 85 n + 28 FP32 FLOP
#   (FMA = 2), which is 28 n^2 + 85 n + 28 on the padded layout m = 2 n:
#   141, 310, 535, 816, 1153, 1546 for n = 1..6;
#   one FP64 Newton step of the refinement: about 150 n FLOP;
#   bytes: 9 + 4 n read per path (indices) and 20 n + 7 written.

def f_iter(n: int, m: int | None = None) -> int:
    m = 2 * n if m is None else m
    return 7 * m * m + 85 * n + 28


def newton_step_flops(n: int) -> int:
    return 150 * n


def io_bytes(n: int) -> int:
    return (9 + 4 * n) + (20 * n + 7)


def store_bytes(n: int, n_max: int) -> int:
    """Bytes the store step moves per path of order n when the outputs come
    back from bucket order to the caller's (the unsort kernel): its results
    read at its bucket slot (20n + 7) and its slot index (4), the caller's
    padded rows written (20 n_max + 7: x and t beyond the order are NaN)."""
    return (20 * n + 7) + 4 + (20 * n_max + 7)


# The builder's own term-by-term FLOP model of each kernel, reported beside
# the algorithmic count (it counts the padded layout, the polish step and the
# refinement's evaluations and trial lengths as the kernels execute them).
def bfgs_flops_per_iter(n: int, fp_iters: int, early_exit: bool) -> int:
    """FP32 flops of one iteration of bfgs_kernel<n> (FMA = 2, every other
    arithmetic op and each rsq / rcp = 1; comparisons and selects = 0).
    Counted term by term from the kernel with m = 2n parameters (the padded
    layout) and s = n + 1 segments:
      direction in point space q_j      9n      segment changes D_i  3(n-1)
      dr_i, dd_i                       10s      num0, den0, phi0      6s
      majorant step                     2       fixed-point iteration f(10s+2)
      descent check phi(alpha)          8s      step s, T += s        2m
      new gradient                25n + 12s      H g'                 2m^2 - m
      y, Hy, s.y, y.Hy, s.s, y.y      10m      curvature test, rho, c1  7
      v, w, w.g', s.g'                 7m      packed update H      2m(m+1)
      new direction, |P|^2             6m
    = 16 n^2 + 125 n + 42 + f (10 n + 12)   (+ 5n + 3 with early exit)."""
    f = int(fp_iters)
    v = 16 * n * n + 125 * n + 42 + f * (10 * n + 12)
    if early_exit:
        v += 5 * n + 3
    return v


def bfgs_init_flops(n: int) -> int:
    """Initial gradient (25n + 12(n+1)) and basis normalisation (18n)."""
    return 25 * n + 12 * (n + 1) + 18 * n


def polish_flops(n: int, steps: int) -> int:
    """FP32 flops of the polish Newton steps at the end of bfgs_kernel<n>
    (newton_run64 on the path's FP32 registers): an evaluation at the start
    and one per step (points 12n; per segment difference 3, squared length 5,
    + eps^2 1, hardware rsq 1, unit vector 3, length sum 2), one trial length
    per step (no unit vectors: 12 per segment), and the Newton solve of
    refine_solve_flops with hardware reciprocals (1 flop instead of 7 for
    each of the n pivots and the majorant step)."""
    if steps <= 0:
        return 0
    ev = 12 * n + 15 * (n + 1)
    tr = 12 * n + 12 * (n + 1)
    so = refine_solve_flops(n) - 6 * (n + 1)
    return ev + steps * (ev + tr + so)


def refine_eval_flops(n: int) -> int:
    """FP64 flops of one evaluation of the smoothed path in refine_kernel<n>
    (eval64): points 4 per coordinate (12n), and per segment difference 3,
    squared length 5, + eps^2 1, reciprocal square root 10 (hardware
    estimate 1, 0.5x 1, two Newton-Raphson steps 4 each), unit vector 3,
    length sum 2: 24 per segment. FMA = 2."""
    return 12 * n + 24 * (n + 1)


def refine_trial_flops(n: int) -> int:
    """FP64 flops of one trial length of a Newton step (length_at): as
    refine_eval_flops without the unit vectors, 21 per segment."""
    return 12 * n + 21 * (n + 1)


def refine_solve_flops(n: int) -> int:
    """FP64 flops of one Newton step of refine_kernel<n> besides the path
    evaluations: gradient 2n (differences of the projections the diagonal
    blocks use); block-tridiagonal Hessian assembly and block-Thomas solve
    83 per slot + 74 per coupling (slot pairs): Gram and projection dot
    products 35, diagonal blocks 21, determinant 3, reciprocal 7, inverse 3,
    y = S^-1 z 6 and back substitution 8 per slot; off-diagonal block 42,
    W = S^-1 E 12 and Schur complement 20 per coupling; largest displacement
    14n; bound 2; trial point 4n; majorant step along d: point changes 9n,
    segment changes 3(n+1), two sums 12(n+1), reciprocal and product 8."""
    return (2 * n + 83 * n + 74 * (n - 1) + 14 * n + 2 + 4 * n
            + 9 * n + 15 * (n + 1) + 8)


def refine_final_flops(n: int) -> int:
    """Per path written: points 12n, exact length 20 per segment."""
    return 12 * n + 20 * (n + 1)



def grad_bytes_per_path(n: int) -> int:
    """Algorithmic HBM bytes of the gradient pass of order n per path
    (grad_kernel<n> for smooth minimisers, grad_kkt_kernel<n> for collapsed
    ones): reads T* (8n), status (1), g_len (4), g_x (12n), src/dst (8),
    ids (4n); the scene tables and the reduced gradient stay in cache /
    LDS."""
    return 8 * n + 1 + 4 + 12 * n + 8 + 4 * n


def run_fwd_grad(args, fpt, scenes, torch):
    """1,048,576 order-3 canyon paths: fpt_solve + fpt_grad (implicit
    differentiation), and autodiff through 64 unrolled BFGS iterations on a
    262,144-path subset for comparison."""
    from paper_2510_16172_amd.unrolled_ad import gather_paths, unrolled_bfgs
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 1 << 20, seed=1004, n=3)
    g_len, g_x = scenes.upstream_grads(b.N, b.n_max, seed=1104)
    solver = fpt.Solver(0)
    db = fpt.DeviceBatch(b, with_order=False)
    opts = fpt.Opts(scale=b.S, iters=args.iters, fp_iters=args.fp_iters)
    chosen = {}
    if not args.no_autotune:
        from paper_2510_16172_amd import autotune
        chosen = autotune.tune(solver, b, opts, sample=1 << 20, repeats=3)
    out = solver.alloc_out(db)
    gl = torch.from_numpy(g_len).cuda()
    gx = torch.from_numpy(g_x).cuda()
    g_pts = torch.zeros((3, b.Q), dtype=torch.float32, device="cuda")
    g_obj = torch.zeros((9, b.K), dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream()
    for _ in range(2):
        solver.solve(db, opts, out=out)
        solver.grad(db, out, g_len=gl, g_x=gx, g_pts=g_pts, g_obj=g_obj)
    torch.cuda.synchronize()
    solver.set_timing(True)
    steps = max(3, args.steps // 2)
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    t_f = t_g = 0.0
    for _ in range(steps):
        e0.record(st)
        solver.solve(db, opts, out=out)
        e1.record(st)
        g_pts.zero_()
        g_obj.zero_()
        solver.grad(db, out, g_len=gl, g_x=gx, g_pts=g_pts, g_obj=g_obj)
        e2.record(st)
        torch.cuda.synchronize()
        t_f += e0.elapsed_time(e1)
        t_g += e1.elapsed_time(e2)
    kt = solver.kernel_times()
    solver.set_timing(False)
    t_f /= steps
    t_g /= steps
    cert = int(((out["status"] & fpt.ST_CONVERGED) != 0).sum().item())
    # certified paths that get a gradient (no FPT_ST_NOGRAD: collapsed
    # minimisers get none)
    cert_grad = int((((out["status"] & fpt.ST_CONVERGED) != 0)
                     & ((out["status"] & fpt.ST_NOGRAD) == 0)).sum().item())
    nograd = float(((out["status"] & fpt.ST_NOGRAD) != 0).float().mean().item())
    tg_kernel = kt[fpt.T_GRAD]
    cg = read_counters("grad_kernels_3", "canyon_c4", "grad")
    res = {
        "workload": "street canyon: 1,048,576 sampled order-3 paths, "
                    "upstream gradients N(0,1)",
        "schedule": chosen.get(3) or {"iters": args.iters},
        "ms_fwd": t_f, "ms_grad": t_g, "grad_kernel_ms": tg_kernel,
        "certified_fraction": cert / b.N,
        "no_gradient_fraction": nograd,
        "certified_with_gradient_fraction": cert_grad / b.N,
        "converged_paths_per_s_fwd_grad": cert_grad / ((t_f + t_g) * 1e-3),
        "certified_paths_per_s_fwd_grad_incl_no_gradient": cert / ((t_f + t_g) * 1e-3),
        "grad_roofline": {
            "kernel": "grad_kernel<3> + grad_kkt_kernel<3>", "bound": "hbm",
            "achieved": grad_bytes_per_path(3) * b.N / (tg_kernel * 1e-3) / 1e9,
            "peak": PEAK_HBM / 1e9, "unit": "GB/s",
            "frac": grad_bytes_per_path(3) * b.N / (tg_kernel * 1e-3) / PEAK_HBM,
            "traffic": cg["hbm_bytes_per_launch"] if cg else None},
        # the same pass against the FP64 vector peak, by the committed
        # counter FLOPs (latency-bound FP64: neither peak is reached)
        "grad_roofline_fp64": None if not (cg and cg.get("counter_fp64_flop_per_launch")) else {
            "kernel": "grad_kernel<3> + grad_kkt_kernel<3>", "bound": "alu",
            "achieved": cg["counter_fp64_flop_per_launch"] / (tg_kernel * 1e-3) / 1e12,
            "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
            "frac": cg["counter_fp64_flop_per_launch"] / (tg_kernel * 1e-3) / PEAK_FP64},
    }
    if args.no_autodiff:
        solver.close()
        return res
    # autodiff through unrolled iterations vs implicit, same subset
    M = 1 << 18
    sub = b.subset(np.arange(M))
    pts = torch.from_numpy(sub.pts).cuda().requires_grad_(True)
    obj = torch.from_numpy(sub.obj).cuda().requires_grad_(True)
    src, dst = torch.from_numpy(sub.src).cuda(), torch.from_numpy(sub.dst).cuda()
    ids = torch.from_numpy(sub.ids).cuda()
    wl = gl[:M]
    wx = gx[:, :, :M].permute(2, 0, 1).contiguous()

    def ad_once():
        pts.grad = None
        obj.grad = None
        tx, rx, B, A1, A2 = gather_paths(pts, obj, src, dst, ids)
        X, L = unrolled_bfgs(tx, rx, B, A1, A2, iters=64)
        loss = (wl * L).sum() + (wx * X).sum()
        loss.backward()

    ad_once()
    torch.cuda.synchronize()
    e0.record(st)
    ad_once()
    e1.record(st)
    torch.cuda.synchronize()
    ad_ms = e0.elapsed_time(e1)
    dbs = fpt.DeviceBatch(sub, with_order=False)
    outs = solver.solve(dbs, opts)
    gps = torch.zeros_like(g_pts)
    gos = torch.zeros_like(g_obj)
    solver.grad(dbs, outs, g_len=wl.contiguous(), g_x=gx[:, :, :M].contiguous(),
                g_pts=gps, g_obj=gos)
    torch.cuda.synchronize()
    e0.record(st)
    solver.grad(dbs, outs, g_len=wl.contiguous(), g_x=gx[:, :, :M].contiguous(),
                g_pts=gps, g_obj=gos)
    e1.record(st)
    torch.cuda.synchronize()
    ift_ms = e0.elapsed_time(e1)
    e0.record(st)
    solver.solve(dbs, opts, out=outs)
    e1.record(st)
    torch.cuda.synchronize()
    solve_ms = e0.elapsed_time(e1)
    res["unrolled_ad"] = {"paths": M, "iters": 64,
                          "ms_fwd_plus_backprop": ad_ms,
                          "ms_implicit_grad": ift_ms,
                          "ms_solve_plus_implicit_grad": solve_ms + ift_ms,
                          "speedup_of_implicit_grad": ad_ms / ift_ms,
                          "speedup_of_solve_plus_implicit": ad_ms / (solve_ms + ift_ms)}
    solver.close()
    return res



# The sources each group of kernels is built from (the host code that
# launches them, api.hip, changes no kernel's bytes or arithmetic).
KERNEL_SOURCES = {"solve": ("solve.hip", "path64.h", "common.h"),
                  "grad": ("grad.hip", "path64.h", "common.h"),
                  "mlp": ("mlp.hip", "common.h")}


def source_digest(group: str = "solve") -> str:
    """Digest of the sources of one group of kernels."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[group]:
        with open(os.path.join(ROOT, "paper_2510_16172_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_counters(kernel: str, workload: str, group: str = "solve"):
    """The committed rocprofv3 counter summary of a kernel (group) on a
    workload, or None if there is none for the current sources of its
    kernels."""
    path = os.path.join(ROOT, "profiles", f"{kernel}__{workload}.counters.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_digest") != source_digest(group):
        return None
    return d


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _compare(sub, ref, o, idx):
    """Per-path comparison of GPU outputs `o` (full arrays, paths idx) with
    the oracle on the sub-batch: within 1e-4 S (points), the gate (points for
    a smooth unique minimiser, length within 1e-5 S for a collapsed or
    non-unique one), certified, certified but outside 1e-4 S."""
    j = np.arange(sub.n_max)[None, :]
    ill = (ref["flags"] & 2) != 0
    col = (ref["flags"] & 1) != 0
    x = np.transpose(o["x"][:, :, idx], (2, 0, 1)).astype(np.float64)
    d = np.linalg.norm(x - ref["x"], axis=-1)
    d = np.where(j < sub.order[:, None].astype(np.int64), d, 0.0)
    err = np.where(np.isfinite(d), d, np.inf).max(axis=1) / sub.S
    ok = err <= 1e-4
    dL = np.abs(o["len"][idx].astype(np.float64) - ref["len"]) / sub.S
    gate = np.where(col | ill, np.where(np.isfinite(dL), dL, np.inf) <= 1e-5, ok)
    cert = (o["status"][idx] & 1) != 0
    return ok, gate, cert, cert & ~ok & ~ill


def cpu_baseline(batch, outs, seconds: float, threads: int, seed: int = 7):
    """The FP64 oracle timed on host cores on a seeded random sample of the
    workload (chunks of 2^15 paths until `seconds` have elapsed, or every
    path), and the GPU results `outs` ({name: output}, "" the headline)
    checked against it on that sample, per order."""
    import oracle
    rng = np.random.default_rng(seed)
    perm = rng.permutation(batch.N)
    chunk = 1 << 15
    done, t_used = 0, 0.0
    nmax = batch.n_max
    tally = {k: np.zeros((nmax + 1, 5), np.int64) for k in outs}  # paths, ok, gate, cert, wrong
    while t_used < seconds and done < batch.N:
        idx = np.sort(perm[done:done + chunk])
        sub = batch.subset(idx)
        t0 = time.perf_counter()
        ref = oracle.solve(sub, threads=threads)
        t_used += time.perf_counter() - t0
        done += len(idx)
        for k, o in outs.items():
            ok, gate, cert, wrong = _compare(sub, ref, o, idx)
            for n in range(1, nmax + 1):
                m = sub.order == n
                tally[k][n] += [m.sum(), ok[m].sum(), gate[m].sum(), cert[m].sum(), wrong[m].sum()]
    # one thread, on the first chunk of the same sample
    sub = batch.subset(np.sort(perm[:min(chunk, batch.N)]))
    t0 = time.perf_counter()
    oracle.solve(sub, threads=1)
    t1 = time.perf_counter() - t0
    what = (f"all {done} paths of the workload" if done == batch.N else
            f"{done} seeded random paths of the workload")

    def summ(t):
        tot = t[1:].sum(0)
        return {"within_1e-4": tot[1] / tot[0], "gate": tot[2] / tot[0],
                "certified": tot[3] / tot[0], "certified_but_wrong": int(tot[4]),
                "paths_within_1e-4": int(tot[1]),
                "per_order": {str(n): {"paths": int(t[n, 0]),
                                       "within_1e-4": float(t[n, 1] / max(t[n, 0], 1)),
                                       "gate": float(t[n, 2] / max(t[n, 0], 1)),
                                       "certified": float(t[n, 3] / max(t[n, 0], 1)),
                                       "certified_but_wrong": int(t[n, 4])}
                              for n in range(1, nmax + 1) if t[n, 0] > 0}}
    res = {"value": done / t_used, "unit": "paths/s", "cores": threads,
           "kind": "oracle",
           "sample": f"{what} ({t_used:.1f} s on {threads} threads)",
           "all_paths": done == batch.N,
           "value_1thread": sub.N / t1,
           "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
           "gpu_vs_oracle": summ(tally[""])}
    others = {k: summ(v) for k, v in tally.items() if k}
    if others:
        res["others_vs_oracle"] = others
    return res


def host_threads() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))


# ------------------------------------------------------- solve timing -----

def timed_solve(args, solver, db, opts, torch):
    """One fpt_solve captured as a HIP graph on a side stream: W warm-up
    replays, then K timed replays bracketed by HIP events on that stream.
    Returns (ms per step, per-step ms, outputs on the host)."""
    out = solver.alloc_out(db)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        solver.solve(db, opts, out=out, stream=st)
        st.synchronize()
        graph = solver.capture(db, opts, out, st)
        for _ in range(args.warmup):
            graph.launch(st)
        st.synchronize()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        ev[0].record(st)
        for k in range(args.steps):
            graph.launch(st)
            ev[k + 1].record(st)
        st.synchronize()
        torch.cuda.synchronize()
    graph.close()
    ms = ev[0].elapsed_time(ev[-1]) / args.steps
    per = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    return ms, per, {k: v.cpu().numpy() for k, v in out.items()}


def breakdown(args, solver, db, opts, torch):
    """The same solve with the library's per-kernel HIP-event timers and the
    refinement's work counters on: orders one after another, one part each,
    so that every timer brackets one order's launches alone on the stream
    they run on. Returns (timer ms, work counts per solve)."""
    opts_seq = dataclasses.replace(opts, concurrent_orders=False, split=1)
    out = solver.alloc_out(db)
    solver.solve(db, opts_seq, out=out)
    torch.cuda.synchronize()
    solver.set_timing(True)
    solver.work_counts()  # clear
    for _ in range(args.steps):
        solver.solve(db, opts_seq, out=out)
    kt = solver.kernel_times()
    work = solver.work_counts()
    solver.set_timing(False)
    work = {n: tuple(v / args.steps for v in w) for n, w in work.items()}
    return kt, work


def _same_schedule(counters, schedule, n, keys):
    """Whether the committed counters of order n were taken with the
    schedule `schedule` gives that order (the FLOP counts depend on it; the
    HBM bytes do not: a kernel reads its paths and writes its results once
    whatever its step counts)."""
    if not counters or schedule is None:
        return False
    a = (counters.get("schedule") or {}).get(str(n)) or {}
    b = schedule.get(n) or schedule.get(str(n)) or {}
    return all(a.get(k) == b.get(k) for k in keys)


def order_rooflines(fpt, batch, out_np, kt, work, opts, workload, schedule=None):
    """Roofline of each order's FP32 phase and FP64 refinement group: the
    algorithmic FLOP count per launch (above) over the launch's measured
    time, against the FP32 / FP64 vector peaks; the builder's model and the
    committed counters beside it (their FLOP counts only where this run's
    schedule for the order is the profiled one)."""
    rows = []
    edge = np.all(batch.obj[6:9] == 0, axis=0)
    for n in range(1, batch.n_max + 1):
        sel = batch.order == n
        cnt = int(sel.sum())
        if cnt == 0:
            continue
        it = out_np["iters"][sel].astype(np.int64)
        # active parameters per path: 2 per face, 1 per edge
        m_act = (2 * n - edge[batch.ids[:n][:, sel]].sum(0)).astype(np.int64)
        fl_pad = int(it.sum()) * f_iter(n)
        fl_act = int((it * (7 * m_act * m_act + 85 * n + 28)).sum())
        fl_mod = (int(it.sum()) * bfgs_flops_per_iter(n, opts.fp_iters, False)
                  + cnt * (bfgs_init_flops(n) + polish_flops(n, opts.polish_steps)))
        t_b = kt[fpt.T_BFGS + n - 1] * 1e-3
        name_b = "newton32_kernel" if opts.method == fpt.METHOD_NEWTON32 else "bfgs_kernel"
        cb = read_counters(f"{name_b}_{n}", workload)
        rows.append({
            "kernel": f"{name_b}<{n}>", "order": n, "paths": cnt, "bound": "alu",
            "achieved": fl_pad / t_b / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
            "frac": fl_pad / t_b / PEAK_FP32,
            "frac_of_unpacked_fp32": fl_pad / t_b / PEAK_FP32_UNPACKED,
            "ms": t_b * 1e3, "flops_per_launch": fl_pad,
            "flops_active_dims": fl_act, "flops_builder_model": fl_mod,
            "iterations_per_path": float(it.mean()),
            "traffic": cb["hbm_bytes_per_launch"] if cb else None,
            "counter_fp32_flop_per_launch": cb.get("counter_fp32_flop_per_launch")
            if _same_schedule(cb, schedule, n, ("iters", "early_exit")) else None,
        })
        ev, tr, so, mev, mtr, mso = work[n]
        fl_r = so * newton_step_flops(n) + mso * newton_step_flops(max(n - 1, 1))
        fl_rm = (ev * refine_eval_flops(n) + tr * refine_trial_flops(n)
                 + so * refine_solve_flops(n)
                 + mev * refine_eval_flops(max(n - 1, 1)) + mtr * refine_trial_flops(max(n - 1, 1))
                 + mso * refine_solve_flops(max(n - 1, 1)) + cnt * refine_final_flops(n))
        t_r = kt[fpt.T_REFINE + n - 1] * 1e-3
        cr = read_counters(f"refine_group_{n}", workload)
        rows.append({
            "kernel": f"refinement group of order {n}: refine_kernel<{n}, true> (quick pass), "
                      f"merge_kernel<{n}> (collapse steps), refine_kernel<{n}, false> (full schedule)",
            "order": n, "paths": cnt, "bound": "alu",
            "achieved": fl_r / t_r / 1e12 if t_r > 0 else 0.0, "peak": PEAK_FP64 / 1e12,
            "unit": "TFLOP/s", "frac": fl_r / t_r / PEAK_FP64 if t_r > 0 else 0.0,
            "ms": t_r * 1e3, "flops_per_launch": fl_r, "flops_builder_model": fl_rm,
            "achieved_builder_model": fl_rm / t_r / 1e12 if t_r > 0 else 0.0,
            "newton_solves_per_path": so / cnt, "collapse_step_solves_per_path": mso / cnt,
            "evaluations_per_path": ev / cnt, "trial_lengths_per_path": tr / cnt,
            "traffic": cr["hbm_bytes_per_launch"] if cr else None,
            "counter_fp64_flop_per_launch": cr.get("counter_fp64_flop_per_launch")
            if _same_schedule(cr, schedule, n, ("iters", "early_exit", "quick_steps",
                                                "quick_passes")) else None,
        })
    return rows


def phase_rooflines(rows):
    """The FP32 first phase and the FP64 refinement of every order together:
    algorithmic FLOPs over the summed launch times (orders one after
    another)."""
    out = {}
    for key, pick, peak in (("fp32_first_phase", lambda r: not r["kernel"].startswith("refinement"),
                             PEAK_FP32),
                            ("fp64_refinement", lambda r: r["kernel"].startswith("refinement"),
                             PEAK_FP64)):
        sel = [r for r in rows if r.get("unit") == "TFLOP/s" and pick(r)]
        if not sel:
            continue
        fl = sum(r["flops_per_launch"] for r in sel)
        ms = sum(r["ms"] for r in sel)
        out[key] = {"flops": fl, "ms": ms, "achieved": fl / (ms * 1e-3) / 1e12,
                    "peak": peak / 1e12, "unit": "TFLOP/s", "frac": fl / (ms * 1e-3) / peak}
    return out


def solve_workload(args, fpt, torch, solver, batch, opts, chosen, workload, outs_extra=None):
    db = fpt.DeviceBatch(batch, device="cuda:0")
    ms, per, out_np = timed_solve(args, solver, db, opts, torch)
    kt, work = breakdown(args, solver, db, opts, torch)
    rows = order_rooflines(fpt, batch, out_np, kt, work, opts, workload, chosen)
    st = out_np["status"]
    cert = (st & fpt.ST_CONVERGED) != 0
    per_order = {str(n): {"paths": int((batch.order == n).sum()),
                          "certified": float(cert[batch.order == n].mean())}
                 for n in range(1, batch.n_max + 1) if (batch.order == n).any()}
    kernel_ms = {"bucketing_and_gather": kt[fpt.T_BUCKET], "unsort": kt[fpt.T_UNSORT]}
    for n in range(1, batch.n_max + 1):
        if (batch.order == n).any():
            kernel_ms[f"first_phase_order{n}"] = kt[fpt.T_BFGS + n - 1]
            kernel_ms[f"refine_order{n}"] = kt[fpt.T_REFINE + n - 1]
    phases = phase_rooflines(rows)
    if kt[fpt.T_UNSORT] > 0:
        # the store step in the caller's layout: one launch per solve
        t_u = kt[fpt.T_UNSORT] * 1e-3
        by = sum(int((batch.order == n).sum()) * store_bytes(n, batch.n_max)
                 for n in range(1, batch.n_max + 1))
        cu = read_counters("unsort_kernel", workload)
        rows.append({
            "kernel": f"unsort{'4' if batch.N % 4 == 0 else ''}_kernel<{batch.n_max}>",
            "order": None, "paths": batch.N,
            "bound": "hbm", "achieved": by / t_u / 1e9, "peak": PEAK_HBM / 1e9,
            "unit": "GB/s", "frac": by / t_u / PEAK_HBM, "ms": t_u * 1e3,
            "bytes_per_launch": by,
            "traffic": cu["hbm_bytes_per_launch"] if cu else None})
    # the dominant kernel: the longest single launch (a refinement group is
    # three to five launches: its rows stand beside it)
    single = [r for r in rows if not r["kernel"].startswith("refinement group")]
    dominant = max(single, key=lambda r: r["ms"])
    groups = [r for r in rows if r["kernel"].startswith("refinement group")]
    other = max(groups, key=lambda r: r["ms"]) if groups else None
    del db
    return {
        "ms_per_step": ms, "ms_per_step_median": float(np.median(per)),
        "ms_per_step_min": float(np.min(per)),
        "certified": int(cert.sum()), "certified_fraction": float(cert.mean()),
        "certified_paths_per_s": float(cert.sum() / (ms * 1e-3)),
        "paths_per_s_all": batch.N / (ms * 1e-3),
        "certified_per_order": per_order,
        "schedule": {str(k): v for k, v in chosen.items()},
        "kernel_ms_orders_one_after_another": kernel_ms,
        "kernel_ms_sum": float(sum(v for v in kernel_ms.values() if v > 0)),
        "roofline": dominant, "roofline_other": other, "rooflines": rows,
        "phase_rooflines": phases,
    }, out_np


def tune_or_fix(args, solver, batch, opts, sample, repeats, schedule=None, candidates=None):
    if schedule:
        chosen = {int(k): v for k, v in json.loads(schedule).items()}
        for n, cfg in chosen.items():
            solver.set_launch(n, cfg)
        return chosen, False
    if args.no_autotune:
        return {}, False
    from paper_2510_16172_amd import autotune
    return autotune.tune(solver, batch, opts, sample=sample, repeats=repeats,
                         candidates=candidates), True


# ------------------------------------------------------------ workloads ----

C3_WORKLOAD = ("street canyon: 8,388,608 sampled paths, orders 1..6 with P(n) "
               "proportional to 2^-n (313 objects, 64 TX/RX pairs), one HIP graph per "
               "step, the orders on streams of their own")
C2_WORKLOAD = ("street canyon: all 6,270,016 interaction sequences of order <= 2 "
               "(313 objects, 64 TX/RX pairs), one HIP graph per step")


def run_c3(args, fpt, scenes, torch):
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 1 << 23, seed=1003, n=None, n_max=6)
    solver = fpt.Solver(0)
    opts = fpt.Opts(scale=b.S, iters=args.iters, fp_iters=args.fp_iters,
                    concurrent_orders=not args.sequential,
                    split=1 if args.sequential else args.split)
    chosen, tuned = tune_or_fix(args, solver, b, opts, 1 << 18, 2, args.schedule)
    res, out_np = solve_workload(args, fpt, torch, solver, b, opts, chosen, "canyon_c3")
    res["config"] = {
        "workload": C3_WORKLOAD, "paths": b.N,
        "order_counts": {str(n): int((b.order == n).sum()) for n in range(1, 7)},
        "autotuned": tuned, "fp_iters": opts.fp_iters,
        "refine_levels": list(zip(opts.level_eps, opts.level_steps)),
        "quick_steps": opts.quick_steps, "quick_passes": opts.quick_passes,
        "polish_steps": opts.polish_steps, "concurrent_orders": opts.concurrent_orders,
        "split": opts.split if opts.split > 0 else 2,
    }
    solver.close()
    return res, b, out_np


def run_c2(args, fpt, scenes, torch, post=True, variant=True, check_seconds=0.0):
    """All order <= 2 sequences; then (not in the metric) validity of the
    solved paths, candidate enumeration and the chain enumerate -> solve ->
    validity, and the solver variants of the first phase (FP32 Newton,
    Armijo line search)."""
    scene = scenes.canyon_scene()
    batch = scenes.canyon_all_paths(scene, n_max=2)
    N = batch.N
    solver = fpt.Solver(0)
    opts = fpt.Opts(scale=batch.S, iters=args.iters, fp_iters=args.fp_iters, split=args.split)
    chosen, tuned = tune_or_fix(args, solver, batch, opts, 1 << 20, 3, args.schedule_c2)
    res, out_np = solve_workload(args, fpt, torch, solver, batch, opts, chosen, "canyon_c2")
    res["config"] = {"workload": C2_WORKLOAD, "paths": N, "autotuned": tuned,
                     "split": opts.split if opts.split > 0 else 2}
    outs = {"": out_np}
    stream = torch.cuda.current_stream()
    db = fpt.DeviceBatch(batch, device="cuda:0")
    out = solver.alloc_out(db)
    solver.solve(db, opts, out=out)
    torch.cuda.synchronize()
    if variant:
        from paper_2510_16172_amd import autotune

        def time_variant(opts_v, candidates):
            chosen_v, _ = tune_or_fix(args, solver, batch, opts_v, 1 << 20, 3, None,
                                      candidates=candidates)
            outv = solver.alloc_out(db)
            for _ in range(args.warmup):
                solver.solve(db, opts_v, out=outv, stream=stream)
            torch.cuda.synchronize()
            v0, v1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            v0.record(stream)
            for _ in range(args.steps):
                solver.solve(db, opts_v, out=outv, stream=stream)
            v1.record(stream)
            torch.cuda.synchronize()
            ms_v = v0.elapsed_time(v1) / args.steps
            o = {k: v.cpu().numpy() for k, v in outv.items()}
            cert_v = int(((o["status"] & fpt.ST_CONVERGED) != 0).sum())
            return o, {"schedule": {str(k): v for k, v in chosen_v.items()},
                       "ms_per_step": ms_v, "certified_fraction": cert_v / N,
                       "certified_paths_per_s": cert_v / (ms_v * 1e-3)}

        outs["newton32"], r = time_variant(fpt.Opts(scale=batch.S, method=fpt.METHOD_NEWTON32),
                                           autotune.NEWTON32_CANDIDATES)
        res["variant_newton32"] = {
            "method": "FP32 exact-Hessian Newton first phase (fpt_opts.method = 1)", **r}
        outs["armijo"], r = time_variant(
            fpt.Opts(scale=batch.S, line_search=fpt.LS_ARMIJO),
            [c for c in autotune.DEFAULT_CANDIDATES if not c.get("early_exit")])
        res["variant_armijo"] = {
            "method": "BFGS with Armijo backtracking in place of the Eq. 6 step "
                      "(fpt_opts.line_search = 1)", **r}
        for n in (1, 2):
            solver.set_launch(n, chosen.get(n))
        solver.solve(db, opts, out=out)
        torch.cuda.synchronize()
    if post:
        res.update(post_legs(fpt, torch, solver, scene, batch, db, out, opts, stream))
    if check_seconds > 0:
        res["oracle_check"] = cpu_baseline(batch, outs, check_seconds, host_threads(), seed=8)
        res["oracle_check"].pop("value_1thread", None)
    solver.close()
    return res


def post_legs(fpt, torch, solver, scene, batch, db, out, opts, stream):
    N = batch.N
    v0, v1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    vflags = solver.validate(db, out, stream=stream)
    torch.cuda.synchronize()
    v0.record(stream)
    for _ in range(3):
        solver.validate(db, out, flags=vflags, stream=stream)
    v1.record(stream)
    torch.cuda.synchronize()
    ms_val = v0.elapsed_time(v1) / 3
    vf = vflags.cpu().numpy()
    lflags = solver.validate(db, out, lazy=True, stream=stream)
    torch.cuda.synchronize()
    v0.record(stream)
    for _ in range(3):
        solver.validate(db, out, flags=lflags, lazy=True, stream=stream)
    v1.record(stream)
    torch.cuda.synchronize()
    ms_val_lazy = v0.elapsed_time(v1) / 3
    lazy_same_valid = bool(np.array_equal(lflags.cpu().numpy() == 7, vf == 7))
    st = out["status"].cpu().numpy()
    n_pairs = scene.meta["n_pairs"]
    tps = torch.arange(0, 2 * n_pairs, 2, dtype=torch.int32, device="cuda:0")
    tpd = tps + 1
    eo = solver.enumerate(tps, tpd, scene.K, 1, 2, stream=stream)
    torch.cuda.synchronize()
    enum_same = all(bool(torch.equal(eo[k], getattr(db, k)))
                    for k in ("src", "dst", "order", "ids"))
    v0.record(stream)
    for _ in range(5):
        solver.enumerate(tps, tpd, scene.K, 1, 2, out=eo, stream=stream)
    v1.record(stream)
    torch.cuda.synchronize()
    ms_enum = v0.elapsed_time(v1) / 5
    enum_bytes = 4 + 4 + 1 + 4 * batch.n_max
    dbe = fpt.DeviceBatch.from_tensors(db.obj, db.pts, eo["src"], eo["dst"], eo["ids"],
                                       eo["order"], S=batch.S)
    outc = solver.alloc_out(dbe)
    cflags = solver.validate(dbe, out, lazy=True, stream=stream)
    solver.solve(dbe, opts, out=outc, stream=stream)
    torch.cuda.synchronize()
    v0.record(stream)
    for _ in range(3):
        solver.enumerate(tps, tpd, scene.K, 1, 2, out=eo, stream=stream)
        solver.solve(dbe, opts, out=outc, stream=stream)
        solver.validate(dbe, outc, flags=cflags, lazy=True, stream=stream)
    v1.record(stream)
    torch.cuda.synchronize()
    ms_chain = v0.elapsed_time(v1) / 3
    return {
        "validate": {
            "ms": ms_val, "paths_per_s": N / (ms_val * 1e-3),
            "ms_lazy": ms_val_lazy, "lazy_same_valid_set": lazy_same_valid,
            "extent": float(((vf & fpt.VALID_EXTENT) != 0).mean()),
            "specular": float(((vf & fpt.VALID_SPECULAR) != 0).mean()),
            "visible": float(((vf & fpt.VALID_VISIBLE) != 0).mean()),
            "valid": float((vf == 7).mean()),
            "valid_and_certified": float(((vf == 7) & ((st & fpt.ST_CONVERGED) != 0)).mean()),
        },
        "enumerate": {
            "ms": ms_enum, "candidates_per_s": N / (ms_enum * 1e-3),
            "bytes_per_candidate": enum_bytes,
            "roofline": {"bound": "hbm", "achieved": N * enum_bytes / (ms_enum * 1e-3) / 1e9,
                         "peak": 8000.0, "unit": "GB/s",
                         "frac": N * enum_bytes / (ms_enum * 1e-3) / 1e9 / 8000.0},
            "same_as_host_generator": enum_same,
        },
        "chain": {
            "steps": "enumerate + solve + lazy validity, one stream",
            "ms": ms_chain, "candidates_per_s": N / (ms_chain * 1e-3),
            "valid_paths": int((cflags == 7).sum().item()),
        },
    }


def run_learned(args, fpt, torch):
    from paper_2510_16172_amd import learned_init
    solver = fpt.Solver(0)
    res, _ = learned_init.run(solver, n_train=1 << 22, n_test=1 << 20,
                              epochs=args.mlp_epochs,
                              log=lambda m: print(m, file=sys.stderr, flush=True))
    solver.close()
    ms = (res.get("equal_iterations") or {}).get("ms_inference")
    if ms:
        # 66 -> 256 -> 256 -> 256 -> 8 with FMA = 2: 300,032 FLOP per path
        fl = 300032 * res["paths"]
        cm = read_counters("mlp_infer_kernel", "canyon_c5", "mlp")
        res["infer_roofline"] = {
            "kernel": "mlp_infer_kernel", "bound": "mfma", "paths": res["paths"],
            "achieved": fl / (ms * 1e-3) / 1e12, "peak": PEAK_BF16 / 1e12,
            "unit": "TFLOP/s", "frac": fl / (ms * 1e-3) / PEAK_BF16, "ms": ms,
            "traffic": cm["hbm_bytes_per_launch"] if cm else None}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=("c3", "c2"), default="c3",
                    help="headline: c3 (orders 1..6, 2^23 paths) or c2 (all order <= 2)")
    ap.add_argument("--iters", type=int, default=64,
                    help="BFGS iterations when the schedule is not autotuned")
    ap.add_argument("--fp-iters", type=int, default=1)
    ap.add_argument("--no-autotune", action="store_true",
                    help="use --iters for every order instead of the autotuned schedule")
    ap.add_argument("--schedule", type=str, default=None,
                    help="JSON {order: launch config} for the headline workload instead of "
                         "autotuning (e.g. a previous run's config.schedule)")
    ap.add_argument("--schedule-c2", type=str, default=None,
                    help="the same for the c2 leg")
    ap.add_argument("--split", type=int, default=0,
                    help="parts per order on their own streams (0: automatic)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c2", action="store_true", help="skip the order <= 2 leg")
    ap.add_argument("--no-post", action="store_true",
                    help="skip validity / enumeration / chain on the c2 leg")
    ap.add_argument("--no-variant", action="store_true",
                    help="skip the FP32 Newton variant on the c2 leg")
    ap.add_argument("--no-grad", action="store_true",
                    help="skip the solve + implicit gradient leg")
    ap.add_argument("--no-autodiff", action="store_true",
                    help="fwd_grad leg without the unrolled-autodiff comparison")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip training and evaluating the learned initialiser")
    ap.add_argument("--mlp-epochs", type=int, default=40)
    ap.add_argument("--sequential", action="store_true",
                    help="profiling: the timed steps of the headline run the orders one "
                         "after another in one part (as the kernel breakdown does)")
    ap.add_argument("--legs-only", action="store_true",
                    help="profiling: skip the headline workload, run only the legs")
    ap.add_argument("--copy-calib", action="store_true",
                    help="copy a 256 MiB buffer three times first (for calibrating the "
                         "HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU; --gpus {args.gpus} is not "
              "supported (paths are independent: several GPUs would each "
              "solve a shard of the path list)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2510_16172_amd import fpt, scenes

    if args.copy_calib:
        a = torch.empty(64 << 20, dtype=torch.float32, device="cuda:0")  # 256 MiB
        bb = torch.empty_like(a)
        for _ in range(3):
            bb.copy_(a)
        torch.cuda.synchronize()
        del a, bb
        print("copy calibration: 268435456 bytes read and written per copy",
              file=sys.stderr, flush=True)

    legs = {}
    if args.legs_only:
        if not args.no_grad:
            legs["fwd_grad"] = run_fwd_grad(args, fpt, scenes, torch)
        if not args.no_learned:
            legs["learned_init"] = run_learned(args, fpt, torch)
        print(json.dumps({"legs_only": True, **legs}), flush=True)
        return
    if args.workload == "c3":
        head, batch, out_np = run_c3(args, fpt, scenes, torch)
    else:
        args.schedule_c2 = args.schedule_c2 or args.schedule
        head = run_c2(args, fpt, scenes, torch, post=not args.no_post,
                      variant=not args.no_variant)
        batch, out_np = None, None
    torch.cuda.empty_cache()
    res = {
        "metric": "converged paths/s (fwd, fwd+grad) at <=1e-4 rel error; % FP32 VALU peak",
        "value": head["certified_paths_per_s"],
        "unit": "paths/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "ms_per_step_median": head["ms_per_step_median"],
        "ms_per_step_min": head["ms_per_step_min"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {**head["config"], "schedule": head["schedule"]},
        "certified_fraction": head["certified_fraction"],
        "certified_per_order": head["certified_per_order"],
        "paths_per_s_all": head["paths_per_s_all"],
        "roofline": head["roofline"],
        "roofline_other": head["roofline_other"],
        "rooflines": head["rooflines"],
        "phase_rooflines": head["phase_rooflines"],
        "kernel_ms_orders_one_after_another": head["kernel_ms_orders_one_after_another"],
    }
    for k in ("validate", "enumerate", "chain", "variant_newton32", "variant_armijo"):
        if k in head:
            res[k] = head[k]
    if not args.no_cpu_baseline and batch is not None:
        res["cpu_baseline"] = cpu_baseline(batch, {"": out_np}, args.cpu_seconds,
                                           host_threads())
    del out_np
    if args.workload == "c3" and not args.no_c2:
        legs["c2"] = run_c2(args, fpt, scenes, torch, post=not args.no_post,
                            variant=not args.no_variant,
                            check_seconds=0.0 if args.no_cpu_baseline else 6.0)
        torch.cuda.empty_cache()
    if not args.no_grad:
        legs["fwd_grad"] = run_fwd_grad(args, fpt, scenes, torch)
        torch.cuda.empty_cache()
    if not args.no_learned:
        legs["learned_init"] = run_learned(args, fpt, torch)
        torch.cuda.empty_cache()
    res.update(legs)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
