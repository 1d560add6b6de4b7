#!/usr/bin/env python3
"""Throughput of the Fermat path solver on one MI355X.

Workload: the street canyon (24 boxes, 121 faces + 192 edges, 64 TX/RX
pairs), every interaction sequence of order 1 and 2 with no immediate repeat:
6,270,016 paths, solved in FP32 (BFGS with the fixed-point step of Eq. 6)
plus FP64 refinement. One step = one fpt_solve over all paths, inputs
resident in HBM. The per-order schedule (number of BFGS iterations, or
early exit in stages) is chosen by the autotuner on a sample before timing
(--no-autotune: --iters / --early-exit for every order). Metric: converged
paths per second, where converged means certified by the kernel's FP64
Newton check; the cpu_baseline leg checks every GPU output against the
oracle and reports how many certified paths are outside 1e-4 S.

Prints ONE JSON line (see the keys at the end of main()).
"""
from __future__ import annotations

import argparse
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


def source_digest() -> str:
    h = hashlib.sha256()
    for f in ("solve.hip", "path64.h", "common.h", "api.hip"):
        with open(os.path.join(ROOT, "paper_2510_16172_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if there is none for the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{kernel}__{workload}.counters.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_digest") != source_digest():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(batch, out_np, seconds: float, threads: int, seed: int = 7,
                 others=None):
    """The FP64 oracle timed on host cores on a seeded random sample of the
    workload (chunks of 2^14 paths until `seconds` have elapsed), and the GPU
    result checked against it on that sample (also each of `others`, a
    {name: output} dict of other GPU results on the same workload)."""
    import oracle
    rng = np.random.default_rng(seed)
    perm = rng.permutation(batch.N)
    chunk = 1 << 14
    done, t_used = 0, 0.0
    outs = {"": out_np, **(others or {})}
    tally = {k: [0, 0, 0] for k in outs}  # within 1e-4, certified, certified but wrong
    while t_used < seconds and done < batch.N:
        idx = np.sort(perm[done:done + chunk])
        sub = batch.subset(idx)
        t0 = time.perf_counter()
        ref = oracle.solve(sub, threads=threads)
        t_used += time.perf_counter() - t0
        done += len(idx)
        j = np.arange(sub.n_max)[None, :]
        ill = (ref["flags"] & 2) != 0
        for k, o in outs.items():
            x = np.transpose(o["x"][:, :, idx], (2, 0, 1)).astype(np.float64)
            d = np.linalg.norm(x - ref["x"], axis=-1)
            d = np.where(j < sub.order[:, None].astype(np.int64), d, 0.0)
            err = np.where(np.isfinite(d), d, np.inf).max(axis=1) / sub.S
            ok = err <= 1e-4
            cert = (o["status"][idx] & 1) != 0
            tally[k][0] += int(ok.sum())
            tally[k][1] += int(cert.sum())
            tally[k][2] += int((cert & ~ok & ~ill).sum())
    n_ok, n_cert, n_fp = tally[""]
    # one thread, on the first chunk of the same sample
    sub = batch.subset(np.sort(perm[:min(chunk, batch.N)]))
    t0 = time.perf_counter()
    oracle.solve(sub, threads=1)
    t1 = time.perf_counter() - t0
    what = (f"all {done} paths of the workload" if done == batch.N else
            f"{done} seeded random paths of the workload")
    return {"value": done / t_used, "unit": "paths/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{what} ({t_used:.1f} s on {threads} threads)",
            "value_1thread": sub.N / t1,
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "gpu_within_1e-4_on_sample": n_ok / done,
            "gpu_within_1e-4_paths": n_ok,
            "gpu_certified_on_sample": n_cert / done,
            "gpu_certified_but_wrong_on_sample": n_fp,
            "others": {k: {"gpu_within_1e-4_on_sample": v[0] / done,
                           "gpu_within_1e-4_paths": v[0],
                           "gpu_certified_on_sample": v[1] / done,
                           "gpu_certified_but_wrong_on_sample": v[2]}
                       for k, v in tally.items() if k}}


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def grad_bytes_per_path(n: int) -> int:
    """Algorithmic HBM bytes of grad_kernel<n> per path: reads T* (8n),
    status (1), g_len (4), g_x (12n), src/dst (8), ids (4n); the scene
    tables and the reduced gradient stay in cache / LDS."""
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
    opts = fpt.Opts(scale=b.S, iters=args.iters, fp_iters=args.fp_iters,
                    early_exit=args.early_exit)
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
    tg_kernel = kt[fpt.T_GRAD]
    res = {
        "workload": "street canyon: 1,048,576 sampled order-3 paths, "
                    "upstream gradients N(0,1)",
        "schedule": chosen.get(3) or {"iters": args.iters,
                                      "early_exit": int(args.early_exit)},
        "ms_fwd": t_f, "ms_grad": t_g, "grad_kernel_ms": tg_kernel,
        "certified_fraction": cert / b.N,
        "converged_paths_per_s_fwd_grad": cert / ((t_f + t_g) * 1e-3),
        "grad_roofline": {
            "kernel": "grad_kernel<3>", "bound": "hbm",
            "achieved": grad_bytes_per_path(3) * b.N / (tg_kernel * 1e-3) / 1e9,
            "peak": PEAK_HBM / 1e9, "unit": "GB/s",
            "frac": grad_bytes_per_path(3) * b.N / (tg_kernel * 1e-3) / PEAK_HBM},
    }
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


def run_uneven(args, fpt, scenes, torch):
    """8,388,608 canyon paths, orders 1..6 with P(n) ~ 2^-n, one captured
    HIP graph per step, per-order launch configuration from the autotuner."""
    from paper_2510_16172_amd import autotune
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 1 << 23, seed=1003, n=None, n_max=6)
    solver = fpt.Solver(0)
    # the orders run on streams of their own (their passes overlap)
    opts = fpt.Opts(scale=b.S, iters=64, concurrent_orders=True)
    chosen = autotune.tune(solver, b, opts, sample=1 << 18, repeats=2)
    db = fpt.DeviceBatch(b)
    out = solver.alloc_out(db)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        solver.solve(db, opts, out=out, stream=st)
        st.synchronize()
        graph = solver.capture(db, opts, out, st)
        for _ in range(2):
            graph.launch(st)
        st.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        steps = max(3, args.steps // 2)
        e0.record(st)
        for _ in range(steps):
            graph.launch(st)
        e1.record(st)
        st.synchronize()
    ms = e0.elapsed_time(e1) / steps
    cert = int(((out["status"] & fpt.ST_CONVERGED) != 0).sum().item())
    graph.close()
    solver.close()
    return {"workload": "street canyon: 8,388,608 paths, orders 1..6 with "
                        "P(n) proportional to 2^-n, one HIP graph per step, "
                        "one stream per order inside it",
            "ms_per_step": ms, "certified_fraction": cert / b.N,
            "converged_paths_per_s": cert / (ms * 1e-3),
            "autotuned": {str(k): v for k, v in chosen.items()},
            "order_counts": {str(n): int((b.order == n).sum()) for n in range(1, 7)}}


def run_learned(args, fpt, torch):
    from paper_2510_16172_amd import learned_init
    solver = fpt.Solver(0)
    res, _ = learned_init.run(solver, n_train=1 << 22, n_test=1 << 20,
                              epochs=args.mlp_epochs,
                              log=lambda m: print(m, file=sys.stderr, flush=True))
    solver.close()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--iters", type=int, default=64,
                    help="BFGS iterations when the schedule is not autotuned")
    ap.add_argument("--fp-iters", type=int, default=1)
    ap.add_argument("--early-exit", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use --iters / --early-exit for every order instead "
                         "of the autotuned per-order schedule")
    ap.add_argument("--schedule", type=str, default=None,
                    help="JSON {order: launch config} applied with fpt_set_launch "
                         "instead of autotuning (e.g. a previous run's config.schedule)")
    ap.add_argument("--split", type=int, default=0,
                    help="parts per order on their own streams (0: automatic, "
                         "2 from 2^21 paths on); the instrumented pass uses 1")
    ap.add_argument("--no-variant", action="store_true",
                    help="skip the FP32 Newton solver-variant leg")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-grad", action="store_true",
                    help="skip the forward+gradient leg")
    ap.add_argument("--uneven", action="store_true",
                    help="also run the mixed-order (1..6) graph workload")
    ap.add_argument("--learned", action="store_true",
                    help="also train and evaluate the learned initialiser")
    ap.add_argument("--mlp-epochs", type=int, default=40)
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain device copy of known size (for "
                         "calibrating the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU; --gpus {args.gpus} is not "
              "supported (paths are independent: several GPUs would each "
              "solve a shard of the path list)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2510_16172_amd import fpt, scenes

    scene = scenes.canyon_scene()
    batch = scenes.canyon_all_paths(scene, n_max=2)
    N = batch.N
    solver = fpt.Solver(0)
    db = fpt.DeviceBatch(batch, device="cuda:0")
    opts = fpt.Opts(scale=batch.S, iters=args.iters, fp_iters=args.fp_iters,
                    early_exit=args.early_exit, split=args.split)
    out = solver.alloc_out(db)
    stream = torch.cuda.current_stream()
    chosen = {}
    if args.schedule:
        chosen = {int(k): v for k, v in json.loads(args.schedule).items()}
        for n, cfg in chosen.items():
            solver.set_launch(n, cfg)
    elif not args.no_autotune:
        from paper_2510_16172_amd import autotune
        chosen = autotune.tune(solver, batch, opts, sample=1 << 20, repeats=3)
    orders = sorted(int(v) for v in np.unique(batch.order))

    if args.copy_calib:
        a = torch.empty(64 << 20, dtype=torch.float32, device="cuda:0")  # 256 MiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"copy calibration: {a.numel() * 4} bytes read and written per copy",
              file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        solver.solve(db, opts, out=out, stream=stream)
    torch.cuda.synchronize()
    # the timed steps (no library instrumentation)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for k in range(args.steps):
        solver.solve(db, opts, out=out, stream=stream)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    ms_step = ev[0].elapsed_time(ev[-1]) / args.steps
    per_step = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    # the same steps again with the per-kernel HIP-event timers and the
    # refinement work counters on, for the kernel breakdown and rooflines; in
    # one part per order (split = 1), so that each timer brackets one launch
    # of the order's whole bucket (the parts overlap in the timed steps)
    import dataclasses
    opts_one = dataclasses.replace(opts, split=1)
    solver.set_timing(True)
    solver.work_counts()  # clear
    for k in range(args.steps):
        solver.solve(db, opts_one, out=out, stream=stream)
    kt = solver.kernel_times()
    work = solver.work_counts()
    solver.set_timing(False)

    # post-processing (not part of the metric): validity of the solved paths
    # on the scene's finite objects
    vflags = solver.validate(db, out, stream=stream)
    torch.cuda.synchronize()
    v0, v1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    v0.record(stream)
    for _ in range(3):
        solver.validate(db, out, flags=vflags, stream=stream)
    v1.record(stream)
    torch.cuda.synchronize()
    ms_val = v0.elapsed_time(v1) / 3
    vf = vflags.cpu().numpy()
    # lazy mode: occlusion only for paths that pass the extent and side tests
    lflags = solver.validate(db, out, lazy=True, stream=stream)
    torch.cuda.synchronize()
    v0.record(stream)
    for _ in range(3):
        solver.validate(db, out, flags=lflags, lazy=True, stream=stream)
    v1.record(stream)
    torch.cuda.synchronize()
    ms_val_lazy = v0.elapsed_time(v1) / 3
    lazy_same_valid = bool(np.array_equal(lflags.cpu().numpy() == 7, vf == 7))

    out_np = {k: v.cpu().numpy() for k, v in out.items()}
    st = out_np["status"]
    certified = int(((st & fpt.ST_CONVERGED) != 0).sum())
    value = certified / (ms_step / 1e3)

    # candidate enumeration on the device (the step before the solve), and
    # the chain candidates -> solve -> validity (lazy) on one stream
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
    enum_bytes = 4 + 4 + 1 + 4 * batch.n_max  # src, dst, order, ids written per candidate
    dbe = fpt.DeviceBatch.from_tensors(db.obj, db.pts, eo["src"], eo["dst"], eo["ids"],
                                       eo["order"], S=batch.S)
    cflags = solver.validate(dbe, out, lazy=True, stream=stream)
    torch.cuda.synchronize()
    v0.record(stream)
    for _ in range(3):
        solver.enumerate(tps, tpd, scene.K, 1, 2, out=eo, stream=stream)
        solver.solve(dbe, opts, out=out, stream=stream)
        solver.validate(dbe, out, flags=cflags, lazy=True, stream=stream)
    v1.record(stream)
    torch.cuda.synchronize()
    ms_chain = v0.elapsed_time(v1) / 3
    chain_valid = int((cflags == 7).sum().item())

    # solver variant (not the paper's method, not in `value`): the FP32
    # exact-Hessian Newton first phase, autotuned the same way, same steps
    variant, others = None, {}
    if not args.no_variant:
        from paper_2510_16172_amd import autotune
        opts_n = fpt.Opts(scale=batch.S, method=fpt.METHOD_NEWTON32)
        chosen_n = autotune.tune(solver, batch, opts_n,
                                 candidates=autotune.NEWTON32_CANDIDATES,
                                 sample=1 << 20, repeats=3)
        for _ in range(args.warmup):
            solver.solve(db, opts_n, out=out, stream=stream)
        torch.cuda.synchronize()
        v0.record(stream)
        for _ in range(args.steps):
            solver.solve(db, opts_n, out=out, stream=stream)
        v1.record(stream)
        torch.cuda.synchronize()
        ms_n = v0.elapsed_time(v1) / args.steps
        others["newton32"] = {k: v.cpu().numpy() for k, v in out.items()}
        cert_n = int(((others["newton32"]["status"] & fpt.ST_CONVERGED) != 0).sum())
        variant = {"method": "FP32 exact-Hessian Newton first phase (fpt_opts.method = 1)",
                   "schedule": {str(k): v for k, v in chosen_n.items()},
                   "ms_per_step": ms_n, "certified_fraction": cert_n / N,
                   "certified_paths_per_s": cert_n / (ms_n * 1e-3)}

    # rooflines of the two kernels of the order-2 bucket (99.7 % of the
    # paths): FP32 BFGS and FP64 refinement; the dominant one is `roofline`
    workload = "canyon_order2_all"
    o2 = batch.order == 2
    ee2 = bool(chosen.get(2, {}).get("early_exit", int(args.early_exit)))
    it2 = out_np["iters"][o2].astype(np.int64)
    fl_b = (int(it2.sum()) * bfgs_flops_per_iter(2, args.fp_iters, ee2)
            + int(o2.sum()) * (bfgs_init_flops(2) + polish_flops(2, opts.polish_steps)))
    t_b = kt[fpt.T_BFGS + 1] * 1e-3
    kname_b = "bfgs_stage_kernel<2>" if ee2 else "bfgs_kernel<2>"
    n_eval, n_trial, n_solve, m_eval, m_trial, m_solve = (v / args.steps for v in work[2])
    # refinement passes at order 2, reduced paths of the collapse step at 1
    fl_r = (n_eval * refine_eval_flops(2) + n_trial * refine_trial_flops(2)
            + n_solve * refine_solve_flops(2)
            + m_eval * refine_eval_flops(1) + m_trial * refine_trial_flops(1)
            + m_solve * refine_solve_flops(1)
            + int(o2.sum()) * refine_final_flops(2))
    t_r = kt[fpt.T_REFINE + 1] * 1e-3
    roof_b = {
        "kernel": kname_b + (" (every stage launch)" if ee2 else ""),
        "bound": "alu", "achieved": fl_b / t_b / 1e12, "peak": PEAK_FP32 / 1e12,
        "unit": "TFLOP/s", "frac": fl_b / t_b / PEAK_FP32,
        "frac_of_unpacked_fp32": fl_b / t_b / PEAK_FP32_UNPACKED,
        "flops_per_launch": fl_b, "ms": t_b * 1e3,
        "traffic": read_traffic(kname_b.split("<")[0] + "_2", workload),
    }
    roof_r = {
        "kernel": "refine_kernel<2> (both passes) + merge_kernel<2>",
        "bound": "alu", "achieved": fl_r / t_r / 1e12, "peak": PEAK_FP64 / 1e12,
        "unit": "TFLOP/s", "frac": fl_r / t_r / PEAK_FP64,
        "flops_per_launch": fl_r, "ms": t_r * 1e3,
        "evaluations_per_path": n_eval / int(o2.sum()),
        "trial_lengths_per_path": n_trial / int(o2.sum()),
        "newton_solves_per_path": n_solve / int(o2.sum()),
        "collapse_step_evaluations_per_path": m_eval / int(o2.sum()),
        "collapse_step_trial_lengths_per_path": m_trial / int(o2.sum()),
        "collapse_step_solves_per_path": m_solve / int(o2.sum()),
        "traffic": read_traffic("refine_kernel_2", workload),
    }
    dominant, other = (roof_b, roof_r) if t_b >= t_r else (roof_r, roof_b)
    kernels_ms = {"bucketing": kt[fpt.T_BUCKET]}
    for n in orders:
        kernels_ms[f"bfgs_order{n}"] = kt[fpt.T_BFGS + n - 1]
        kernels_ms[f"refine_order{n}"] = kt[fpt.T_REFINE + n - 1]
    schedule = {str(n): (chosen.get(n) or {"iters": args.iters,
                                           "early_exit": int(args.early_exit)})
                for n in orders}
    res = {
        "metric": "converged paths/s (fwd, fwd+grad) at <=1e-4 rel error",
        "value": value,
        "unit": "paths/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_median": float(np.median(per_step)),
        "ms_per_step_min": float(np.min(per_step)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": "street canyon: all 6,270,016 interaction sequences "
                        "of order <= 2 (313 objects, 64 TX/RX pairs)",
            "paths": N, "fp_iters": args.fp_iters,
            "schedule": schedule,
            "autotuned": not args.no_autotune and not args.schedule,
            "refine_levels": list(zip(opts.level_eps, opts.level_steps)),
            "quick_steps": opts.quick_steps,
            "quick_passes": opts.quick_passes,
            "polish_steps": opts.polish_steps,
            "split": opts.split if opts.split > 0 else (2 if N >= (1 << 21) else 1),
        },
        "certified_fraction": certified / N,
        "paths_per_s_all": N / (ms_step / 1e3),
        "kernel_ms": kernels_ms,
        "roofline": dominant,
        "roofline_other": other,
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
        "variant_newton32": variant,
        "chain": {
            "steps": "enumerate + solve + lazy validity, one stream",
            "ms": ms_chain, "candidates_per_s": N / (ms_chain * 1e-3),
            "valid_paths": chain_valid,
        },
    }
    if not args.no_cpu_baseline:
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
        res["cpu_baseline"] = cpu_baseline(batch, out_np, args.cpu_seconds, threads,
                                           others=others)
        if res["cpu_baseline"]["sample"].startswith("all "):
            # every output checked against the oracle: paths within 1e-4 S per
            # second, certified or not (the certificate is conservative)
            res["paths_within_1e-4_per_s_oracle_checked"] = (
                res["cpu_baseline"]["gpu_within_1e-4_paths"] / (ms_step / 1e3))
    solver.close()
    del db, out
    torch.cuda.empty_cache()
    if not args.no_grad:
        res["fwd_grad"] = run_fwd_grad(args, fpt, scenes, torch)
        torch.cuda.empty_cache()
    if args.uneven:
        res["uneven_orders"] = run_uneven(args, fpt, scenes, torch)
        torch.cuda.empty_cache()
    if args.learned:
        res["learned_init"] = run_learned(args, fpt, torch)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
