"""Learned initialiser: training on solver outputs and evaluation.

The network (fpt_mlp_*) maps the geometry of an order-4 path to starting
parameters; the solver refines them to the same accuracy bar, and paths the
solver does not certify from the learned start are solved again from T = 0
(fallback). The plain solver is therefore both the teacher (its certified
solutions are the training targets) and what decides whether a prediction
was good enough.
"""
from __future__ import annotations

import time

import numpy as np

from . import fpt, scenes


def dedup_against(train: scenes.Batch, test: scenes.Batch) -> scenes.Batch:
    """Drops training paths whose (pair, object sequence) appears in test."""
    def keys(b):
        return np.concatenate([b.src[None, :].astype(np.int64),
                               b.ids.astype(np.int64)], 0).T
    tr, te = keys(train), keys(test)
    allk = np.concatenate([te, tr])
    _, inv = np.unique(allk, axis=0, return_inverse=True)
    inv = inv.ravel()
    in_test = np.zeros(inv.max() + 1, bool)
    in_test[inv[:len(te)]] = True
    keep = ~in_test[inv[len(te):]]
    return train.subset(np.nonzero(keep)[0])


def train(solver, mlp, db: fpt.DeviceBatch, target, scale: float, epochs: int,
          batch: int = 16384, lr: float = 1e-3, seed: int = 0, log=None):
    """Adam epochs over the paths of db against the solver output `target`,
    the step size decaying linearly to 0.1 lr. Returns the mean training
    loss of each epoch."""
    import torch
    N = db.N
    rng = np.random.default_rng(seed)
    losses = []
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(N).astype(np.int64)).cuda()
        loss.zero_()
        nb = 0
        for b0 in range(0, N - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            sub = fpt.DeviceBatch.from_tensors(
                db.obj, db.pts, db.src[idx].contiguous(), db.dst[idx].contiguous(),
                db.ids[:, idx].contiguous(), None, S=scale)
            tgt = {"t": target["t"][:, :, idx].contiguous(),
                   "status": target["status"][idx].contiguous(),
                   "x": target["x"], "len": target["len"], "iters": target["iters"]}
            # decay the step size linearly over the run
            frac = (ep * (N // batch) + nb) / max(1, epochs * (N // batch))
            mlp.train_step(sub, tgt, scale, lr * (1.0 - 0.9 * frac), loss)
            nb += 1
        losses.append(loss.item() / max(nb, 1))
        if log:
            log(f"epoch {ep}: loss {losses[-1]:.4e}")
    return losses


def evaluate(solver, mlp, db: fpt.DeviceBatch, opts, repeats: int = 3):
    """Zero start vs learned start (+ fallback) on db. Returns statistics and
    timings (HIP events on the current stream), the zero-start outputs, and
    the learned-start outputs in which every path the learned start left
    uncertified carries the result of the fallback solve from T = 0."""
    import torch
    st = torch.cuda.current_stream()

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        best = None
        for _ in range(repeats):
            e0.record(st)
            r = fn()
            e1.record(st)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        return r, best

    db.t_init = None
    out0, ms0 = timed(lambda: solver.solve(db, opts))
    tinit = torch.empty((4, 2, db.N), dtype=torch.float32, device="cuda")

    def learned():
        mlp.infer(db, opts.scale, out=tinit)
        db.t_init = tinit
        o = solver.solve(db, opts)
        db.t_init = None
        return o
    out1, ms1 = timed(learned)
    # fallback: paths not certified from the learned start, solved from 0
    cert1 = (out1["status"] & fpt.ST_CONVERGED) != 0
    fb = torch.nonzero(~cert1).flatten()
    ms_fb = 0.0
    n_fb_cert = 0
    if fb.numel() > 0:
        sub = fpt.DeviceBatch.from_tensors(db.obj, db.pts, db.src[fb].contiguous(),
                                           db.dst[fb].contiguous(),
                                           db.ids[:, fb].contiguous(), None, S=db.S)
        outf, ms_fb = timed(lambda: solver.solve(sub, opts))
        n_fb_cert = int(((outf["status"] & fpt.ST_CONVERGED) != 0).sum().item())
    c0 = int(((out0["status"] & fpt.ST_CONVERGED) != 0).sum().item())
    c1 = int(cert1.sum().item())
    it0 = out0["iters"].cpu().numpy().astype(np.int64)
    it1 = out1["iters"].cpu().numpy().astype(np.int64)
    if fb.numel() > 0:
        # the fallback's results replace the learned start's at its paths
        # (path index last in every output array)
        for k in out1:
            out1[k][..., fb] = outf[k]
    N = db.N
    res = {
        "paths": N,
        "zero_init": {"certified": c0 / N, "ms": ms0, "iters_mean": float(it0.mean()),
                      "iters_p50": float(np.median(it0)), "iters_p99": float(np.percentile(it0, 99)),
                      "converged_paths_per_s": c0 / (ms0 * 1e-3)},
        "learned_init": {"certified": c1 / N, "certified_with_fallback": (c1 + n_fb_cert) / N,
                         "ms_infer_plus_solve": ms1, "ms_fallback": ms_fb,
                         "fallback_paths": int(fb.numel()),
                         "iters_mean": float(it1.mean()), "iters_p50": float(np.median(it1)),
                         "iters_p99": float(np.percentile(it1, 99)),
                         "converged_paths_per_s": (c1 + n_fb_cert) / ((ms1 + ms_fb) * 1e-3)},
        "iterations_saved_mean": float(it0.mean() - it1.mean()),
    }
    return res, out0, out1


def compare_fixed(solver, mlp, db: fpt.DeviceBatch, scale: float,
                  iters=(4, 8, 16, 24), repeats: int = 3):
    """Zero vs learned start at equal fixed iteration counts: certified
    fraction, solve time, and certified paths/s with and without the
    network's inference time (HIP events on the current stream)."""
    import torch
    tinit = torch.empty((4, 2, db.N), dtype=torch.float32, device="cuda")

    def timed(fn):
        torch.cuda.synchronize()
        best = None
        for _ in range(repeats):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            r = fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        return r, best

    _, ms_inf = timed(lambda: mlp.infer(db, scale, out=tinit))
    rows = []
    for k in iters:
        o = fpt.Opts(scale=scale, iters=int(k))
        db.t_init = None
        o0, ms0 = timed(lambda: solver.solve(db, o))
        db.t_init = tinit
        o1, ms1 = timed(lambda: solver.solve(db, o))
        db.t_init = None
        c0 = int(((o0["status"] & fpt.ST_CONVERGED) != 0).sum().item())
        c1 = int(((o1["status"] & fpt.ST_CONVERGED) != 0).sum().item())
        rows.append({"iters": int(k),
                     "zero": {"certified": c0 / db.N, "ms": ms0,
                              "converged_paths_per_s": c0 / (ms0 * 1e-3)},
                     "learned": {"certified": c1 / db.N, "ms_solve": ms1,
                                 "converged_paths_per_s_solve_only": c1 / (ms1 * 1e-3),
                                 "converged_paths_per_s_with_inference":
                                     c1 / ((ms1 + ms_inf) * 1e-3)}})
    return {"ms_inference": ms_inf, "fixed_iterations": rows}


def run(solver, n_train: int = 1 << 22, n_test: int = 1 << 20, epochs: int = 40,
        opts_kw=None, log=None, seed: int = 0, lr: float = 2e-3):
    """The full experiment on the street canyon, order-4 paths."""
    import torch
    sc = scenes.canyon_scene()
    t0 = time.perf_counter()
    test = scenes.canyon_sample_paths(sc, n_test, seed=1006 + seed, n=4)
    trainb = dedup_against(scenes.canyon_sample_paths(sc, n_train, seed=1005 + seed, n=4), test)
    opts_kw = dict(opts_kw or {})
    teach = fpt.Opts(scale=sc.S, iters=96)
    dbt = fpt.DeviceBatch(trainb, with_order=False)
    target = solver.solve(dbt, teach)
    torch.cuda.synchronize()
    mlp = fpt.Mlp(solver, seed=seed)
    t1 = time.perf_counter()
    losses = train(solver, mlp, dbt, target, sc.S, epochs, lr=lr, log=log, seed=seed)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    dbe = fpt.DeviceBatch(test, with_order=False)
    opts = fpt.Opts(scale=sc.S, **{**dict(iters=64, early_exit=True), **opts_kw})
    res, _, _ = evaluate(solver, mlp, dbe, opts)
    res["equal_iterations"] = compare_fixed(solver, mlp, dbe, sc.S)
    res.update({"train_paths": trainb.N, "train_certified": float(
        ((target["status"] & fpt.ST_CONVERGED) != 0).float().mean().item()),
        "epochs": epochs, "train_loss": losses, "train_s": t_train,
        "setup_s": time.perf_counter() - t0 - t_train})
    return res, mlp
