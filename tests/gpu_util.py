"""Helpers for the GPU parity tests: run the HIP path, compare with the oracle."""
from __future__ import annotations

import numpy as np


def run_gpu(solver, batch, opts, with_order=True, t_init=None):
    import torch
    from paper_2510_16172_amd import fpt
    db = fpt.DeviceBatch(batch, with_order=with_order)
    if t_init is not None:
        db.t_init = torch.from_numpy(np.ascontiguousarray(t_init, np.float32)).cuda()
    out = solver.solve(db, opts)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def point_error(batch, gpu, ref):
    """max_j |x_j(gpu) - x_j(oracle)| / S per path (NaN-safe: inf)."""
    n_max = batch.n_max
    xg = np.transpose(gpu["x"], (2, 0, 1)).astype(np.float64)  # N, n, 3
    diff = np.linalg.norm(xg - ref["x"], axis=-1)
    j = np.arange(n_max)[None, :]
    active = j < batch.order[:, None].astype(np.int64)
    diff = np.where(active, diff, 0.0)
    diff = np.where(np.isfinite(diff), diff, np.inf)
    return diff.max(axis=1) / batch.S


def summary(batch, gpu, ref, rtol=1e-4):
    from paper_2510_16172_amd import fpt
    e = point_error(batch, gpu, ref)
    ok = e <= rtol
    cert = (gpu["status"] & fpt.ST_CONVERGED) != 0
    ill = (ref["flags"] & 2) != 0
    col = (ref["flags"] & 1) != 0
    return dict(err=e, ok=ok, cert=cert, ill=ill, col=col,
                frac_ok=float(ok.mean()), frac_cert=float(cert.mean()),
                false_pos=int((cert & ~ok & ~ill).sum()))
