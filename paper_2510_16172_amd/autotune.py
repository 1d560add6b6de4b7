"""Autotuner of the per-order launch configuration of the FP32 solver.

For each order present in a workload it times candidate configurations
(the number of fixed BFGS iterations, or per-lane early exit in stages;
the quick FP64 refinement passes) on a sample of that order's paths and keeps
the one with the most certified-converged paths per second of that order's
kernels (BFGS + refinement, timed with the library's HIP-event timers). The
iteration count trades FP32 BFGS time against FP64 refinement time: paths
the BFGS leaves further from the minimiser need more Newton steps. Results are
cached in a JSON file keyed by GPU architecture, a digest of the built
library, a digest of every solver option, the candidate set, the order, and
a power-of-two bucket of the sample size, and applied with fpt_set_launch.
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


def _key(arch: str, order: int, n: int, opts, candidates) -> str:
    tag = hashlib.sha1(json.dumps(candidates, sort_keys=True).encode()).hexdigest()[:8]
    return (f"v5/{arch}/lib{_lib_digest()}/o{_opts_digest(opts)}/c{tag}/order{order}/"
            f"n2^{max(0, int(np.log2(max(n, 1))))}")


def tune(solver, batch, opts, candidates=None, sample=1 << 18, repeats=3,
         cache_path: str | None = None, seed: int = 0):
    """Returns {order: cfg} for the orders in `batch` and applies it."""
    import torch
    from . import fpt
    candidates = candidates or DEFAULT_CANDIDATES
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
        key = _key(arch, n, len(idx), opts, candidates)
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
        best, best_rate, results = None, -1.0, []
        for cfg in candidates:
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
            if rate > best_rate:
                best, best_rate = cfg, rate
        chosen[n] = best
        cache[key] = {"cfg": best, "rate": best_rate, "trials": results}
    for n, cfg in chosen.items():
        solver.set_launch(n, cfg)
    try:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        json.dump(cache, open(cache_path, "w"), indent=1)
    except OSError:
        pass
    return chosen
