"""Autotuner of the per-order launch configuration of the FP32 solver.

For each order present in a workload it times candidate configurations
(the number of fixed BFGS iterations, or per-lane early exit in stages;
the quick FP64 refinement passes) on a sample of that order's paths and keeps
the one with the most certified-converged paths per second of that order's
kernels (BFGS + refinement, timed with the library's HIP-event timers). The
iteration count trades FP32 BFGS time against FP64 refinement time: paths
the BFGS leaves further from the minimiser need more Newton steps. A second
stage then tries the tile settings around the best schedule, one at a time:
workgroups per compute unit of the first phase and of the FP64 refinement
(the resident count, or an oversubscribed grid that the CUs drain as
workgroups end); a setting is kept only where it beats the schedule without
it, and the two winners are tried together. With several orders in the
batch (`whole`), their kernels overlap in one solve, and what is fastest
for an order alone need not be fastest beside the others (an order's
kernels slow the others down, and a latency-bound pass costs little when
other orders fill the GPU): a last stage searches on the complete solve,
one order at a time from the largest bucket down, over the neighbouring
iteration counts, the quick-pass settings and the tile settings, keeping a
change when it raises the certified paths per second of the whole solve
(captured as a HIP graph and replayed), for at most two sweeps. Results are cached in a JSON
file keyed by GPU architecture, a digest of the built library, a digest of
every solver option, the candidate set, the order, and a power-of-two
bucket of the sample size (the last stage is timed anew on every call),
and applied with fpt_set_launch.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

DEFAULT_CANDIDATES = (
    [{"wg_per_cu": 0, "early_exit": 0, "iters": k, "quick_steps": qs, "quick_passes": qp}
     for k in (8, 10, 12, 14, 16, 20, 24, 32, 48)
     for (qs, qp) in ((2, 1), (2, 2), (3, 1))]
    + [{"wg_per_cu": 0, "early_exit": 1, "iters": 64, "stage_iters": s,
        "quick_steps": 2, "quick_passes": 2}
       for s in ([16, 16, 32], [12, 12, 16, 24])]
)


# Tile settings of the second stage, each tried on the best schedule.
TILE_CANDIDATES = ([{"wg_per_cu": w} for w in (8, 16, 32)]
                   + [{"refine_wg_per_cu": w} for w in (4, 8, 16)])


# The FP32 Newton variant of the first phase (fpt_opts.method): its step
# count, with the same quick refinement settings.
NEWTON32_CANDIDATES = [
    {"wg_per_cu": 0, "early_exit": 0, "iters": k, "quick_steps": qs, "quick_passes": qp}
    for k in (4, 6, 8, 10, 12, 16) for (qs, qp) in ((2, 1), (2, 2), (3, 1))]


def default_cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "fpt", "autotune.json")


_LIB_DIGEST = None


def _lib_digest() -> str:
    """Digest of the built library: a rebuild (changed kernels, certificate
    or defaults) invalidates every cached choice."""
    global _LIB_DIGEST
    if _LIB_DIGEST is None:
        from . import fpt
        with open(fpt.LIB_PATH, "rb") as fh:
            _LIB_DIGEST = hashlib.sha1(fh.read()).hexdigest()[:12]
    return _LIB_DIGEST


def _opts_digest(opts) -> str:
    """Digest of every solver option (the C struct's bytes): iteration and
    fixed-point counts, polish steps, refinement levels, tolerances, split."""
    import ctypes
    c = opts.to_c()
    return hashlib.sha1(ctypes.string_at(ctypes.addressof(c), ctypes.sizeof(c))).hexdigest()[:12]


def _key(arch: str, order: int, n: int, opts, candidates, tiles) -> str:
    tag = hashlib.sha1(json.dumps([candidates, tiles], sort_keys=True).encode()).hexdigest()[:8]
    return (f"v6/{arch}/lib{_lib_digest()}/o{_opts_digest(opts)}/c{tag}/order{order}/"
            f"n2^{max(0, int(np.log2(max(n, 1))))}")


TILE_KEYS = ("wg_per_cu", "refine_wg_per_cu")
# smallest relative gain in the whole-solve stage that counts as a win (the
# timing noise of a median of seven solves is below it)
WHOLE_MIN_GAIN = 3e-3


def _neighbours(cfg, candidates):
    """Configurations next to cfg: the fixed iteration counts of the
    candidate set on either side, the other quick-pass settings, the other
    tile settings."""
    out = []
    if not cfg.get("early_exit"):
        its = sorted({c["iters"] for c in candidates if not c.get("early_exit")})
        if cfg.get("iters") in its:
            i = its.index(cfg["iters"])
            out += [{**cfg, "iters": its[j]} for j in (i - 1, i + 1) if 0 <= j < len(its)]
    qset = sorted({(c.get("quick_steps", 2), c.get("quick_passes", 2)) for c in candidates})
    here = (cfg.get("quick_steps", 2), cfg.get("quick_passes", 2))
    out += [{**cfg, "quick_steps": q, "quick_passes": p} for q, p in qset if (q, p) != here]
    for k, vals in (("wg_per_cu", (0, 8, 16)), ("refine_wg_per_cu", (0, 8))):
        out += [{**cfg, k: v} for v in vals if v != cfg.get(k, 0)]
    return out


def _whole_rate(solver, db, opts, out, chosen, repeats):
    """Certified paths per second of the complete solve of db with the
    per-order configurations `chosen`: the solve captured as a HIP graph and
    replayed (as a caller that repeats it would run it), the median of
    `repeats` timed replays."""
    import torch
    from . import fpt
    for n, cfg in chosen.items():
        solver.set_launch(n, cfg)
    st = torch.cuda.Stream()
    ms = []
    with torch.cuda.stream(st):
        solver.solve(db, opts, out=out, stream=st)
        st.synchronize()
        g = solver.capture(db, opts, out, st)
        try:
            g.launch(st)  # warm-up
            for _ in range(repeats):
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(st)
                g.launch(st)
                b.record(st)
                st.synchronize()
                ms.append(a.elapsed_time(b))
        finally:
            g.close()
    cert = int(((out["status"] & fpt.ST_CONVERGED) != 0).sum().item())
    return cert / (float(np.median(ms)) * 1e-3)


def tune(solver, batch, opts, candidates=None, sample=1 << 18, repeats=3,
         cache_path: str | None = None, seed: int = 0, tiles=None, whole=True):
    """Returns {order: cfg} for the orders in `batch` and applies it.
    `tiles`: the second stage's settings (default TILE_CANDIDATES; [] skips
    the stage). `whole`: the last stage on the complete batch when it holds
    several orders."""
    import torch
    from . import fpt
    candidates = candidates or DEFAULT_CANDIDATES
    tiles = TILE_CANDIDATES if tiles is None else list(tiles)
    cache_path = cache_path or default_cache_path()
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    cache = {}
    if os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except Exception:
            cache = {}
    rng = np.random.default_rng(seed)
    chosen = {}
    for n in sorted(set(int(v) for v in np.unique(batch.order))):
        idx = np.nonzero(batch.order == n)[0]
        key = _key(arch, n, len(idx), opts, candidates, tiles)
        if key in cache:
            chosen[n] = cache[key]["cfg"]
            continue
        if len(idx) > sample:
            idx = np.sort(rng.choice(idx, sample, replace=False))
        sub = batch.subset(idx)
        sub = type(sub)(sub.obj, sub.pts, sub.src, sub.dst, sub.order,
                        np.ascontiguousarray(sub.ids[:n]), sub.S, sub.meta)
        db = fpt.DeviceBatch(sub, with_order=False)
        out = solver.alloc_out(db)
        results = []

        def trial(cfg):
            solver.set_launch(n, cfg)
            solver.solve(db, opts, out=out)  # warm-up
            torch.cuda.synchronize()
            solver.set_timing(True)
            for _ in range(repeats):
                solver.solve(db, opts, out=out)
            kt = solver.kernel_times()
            solver.set_timing(False)
            ms = kt[fpt.T_BFGS + n - 1] + kt[fpt.T_REFINE + n - 1]
            cert = int(((out["status"] & fpt.ST_CONVERGED) != 0).sum().item())
            rate = cert / (ms * 1e-3)
            results.append({"cfg": cfg, "ms": ms, "certified": cert, "rate": rate})
            return rate

        best, best_rate = None, -1.0
        for cfg in candidates:
            rate = trial(cfg)
            if rate > best_rate:
                best, best_rate = cfg, rate
        # second stage: tile settings on the best schedule, one at a time,
        # then the winners of the two kinds together
        base, winners = dict(best), {}
        for tile in tiles:
            cfg = {**base, **tile}
            rate = trial(cfg)
            k = next(iter(tile))
            if rate > best_rate and rate > winners.get(k, (None, best_rate))[1]:
                winners[k] = (tile[k], rate)
            if rate > best_rate:
                best, best_rate = cfg, rate
        if len(winners) > 1:
            cfg = {**base, **{k: v for k, (v, _) in winners.items()}}
            rate = trial(cfg)
            if rate > best_rate:
                best, best_rate = cfg, rate
        chosen[n] = best
        cache[key] = {"cfg": best, "rate": best_rate, "trials": results}
    if whole and len(chosen) > 1:
        db = fpt.DeviceBatch(batch)
        out = solver.alloc_out(db)
        reps = max(7, repeats)
        base = _whole_rate(solver, db, opts, out, chosen, reps)
        counts = {n: int((batch.order == n).sum()) for n in chosen}
        for _ in range(2):
            changed = False
            for n in sorted(chosen, key=lambda k: -counts[k]):
                for cfg in _neighbours(chosen[n], candidates):
                    trial = {**chosen, n: cfg}
                    rate = _whole_rate(solver, db, opts, out, trial, reps)
                    if rate > base * (1 + WHOLE_MIN_GAIN):
                        chosen, base, changed = trial, rate, True
            if not changed:
                break
        del db, out
    for n, cfg in chosen.items():
        solver.set_launch(n, cfg)
    try:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        json.dump(cache, open(cache_path, "w"), indent=1)
    except OSError:
        pass
    return chosen
