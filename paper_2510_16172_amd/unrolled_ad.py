"""Baseline for the gradient: reverse-mode autodiff through unrolled solver
iterations (the approach Sec. III-D replaces by implicit differentiation and
Sec. IV-B times against it).

The same FP32 BFGS as the HIP solver (unit-vector basis, identity initial
inverse Hessian rescaled by s^T y / y^T y at the first update, the
fixed-point step of Eq. 6 started at the unit step with the majorant step
from zero as fallback) written with batched PyTorch ops,
so that autograd records every iteration. Used only to time the comparison;
it is not part of the solver.
"""
from __future__ import annotations

import torch


def gather_paths(pts, obj, src, dst, ids):
    """Differentiable per-path geometry: tx, rx [N,3]; B, A1, A2 [N,n,3]."""
    tx = pts[:, src.long()].T
    rx = pts[:, dst.long()].T
    idl = ids.long().T  # N, n
    B = obj[0:3][:, idl].permute(1, 2, 0)
    A1 = obj[3:6][:, idl].permute(1, 2, 0)
    A2 = obj[6:9][:, idl].permute(1, 2, 0)
    return tx, rx, B, A1, A2


def unrolled_bfgs(tx, rx, B, A1, A2, iters: int, fp_iters: int = 1):
    """Returns (X [N,n,3], L [N]) after `iters` recorded BFGS iterations."""
    N, n, _ = B.shape
    m = 2 * n
    n1 = A1.norm(dim=-1, keepdim=True)
    n2 = A2.norm(dim=-1, keepdim=True)
    edge = n2 == 0
    U1 = A1 / n1
    U2 = torch.where(edge, torch.zeros_like(A2), A2 / torch.where(edge, torch.ones_like(n2), n2))
    A = torch.stack([U1, U2], dim=-1)  # N, n, 3, 2

    def points(T):
        X = B + (A * T.view(N, n, 1, 2)).sum(-1)
        return torch.cat([tx[:, None], X, rx[:, None]], dim=1), X

    def grad(T):
        Xf, _ = points(T)
        r = Xf[:, 1:] - Xf[:, :-1]
        l2 = (r * r).sum(-1).clamp_min(1e-30)
        il = torch.rsqrt(l2)
        u = r * il[..., None]
        du = u[:, :-1] - u[:, 1:]
        g = (A * du[..., None]).sum(-2).reshape(N, m)
        return g, r, l2, il

    T = torch.zeros(N, m, device=B.device, dtype=B.dtype)
    H = torch.eye(m, device=B.device, dtype=B.dtype).expand(N, m, m)
    g, r, l2, il = grad(T)
    P = -g
    for it in range(iters):
        q = (A * P.view(N, n, 1, 2)).sum(-1)                       # N, n, 3
        z = torch.zeros_like(q[:, :1])
        D = torch.cat([q, z], 1) - torch.cat([z, q], 1)           # N, n+1, 3
        dr = (D * r).sum(-1)
        dd = (D * D).sum(-1)
        num0 = (dr * il).sum(-1)
        den0 = (dd * il).sum(-1)
        a_mm = torch.where(den0 > 1e-30, -num0 / den0.clamp_min(1e-30), torch.zeros_like(den0))
        alpha = torch.ones_like(a_mm)
        for _f in range(fp_iters):
            rho2 = (l2 + alpha[:, None] * (2 * dr + alpha[:, None] * dd)).clamp_min(1e-30)
            ir = torch.rsqrt(rho2)
            num = (dr * ir).sum(-1)
            den = (dd * ir).sum(-1)
            alpha = torch.where(den > 1e-30, -num / den.clamp_min(1e-30), torch.zeros_like(den))
        rho2 = (l2 + alpha[:, None] * (2 * dr + alpha[:, None] * dd)).clamp_min(1e-30)
        phi = torch.sqrt(rho2).sum(-1)
        phi0 = (l2 * il).sum(-1)
        keep = (phi < phi0) & (alpha > 0) & torch.isfinite(alpha)
        alpha = torch.where(keep, alpha, a_mm)
        s = alpha[:, None] * P
        T = T + s
        gn, r, l2, il = grad(T)
        y = gn - g
        if it == 0:
            sy0 = (s * y).sum(-1)
            yy0 = (y * y).sum(-1)
            gam = torch.where((sy0 > 1e-30) & (yy0 > 1e-30),
                              sy0 / torch.where(yy0 > 1e-30, yy0, torch.ones_like(yy0)),
                              torch.ones_like(sy0))
            H = H * gam[:, None, None]
            P = P * gam[:, None]
        Hg = torch.bmm(H, gn[:, :, None])[..., 0]
        Hy = Hg + P
        sy = (s * y).sum(-1)
        yHy = (y * Hy).sum(-1)
        ss = (s * s).sum(-1)
        yy = (y * y).sum(-1)
        upd = (sy > 1e-30) & (sy * sy > 1e-12 * ss * yy)
        rho = torch.where(upd, 1.0 / torch.where(upd, sy, torch.ones_like(sy)), torch.zeros_like(sy))
        c1 = rho * (1 + rho * yHy)
        v = -rho[:, None] * Hy
        w = c1[:, None] * s + v
        H = H + s[:, :, None] * w[:, None, :] + v[:, :, None] * s[:, None, :]
        wg = (w * gn).sum(-1)
        sg = (s * gn).sum(-1)
        P = -(Hg + s * wg[:, None] + v * sg[:, None])
        g = gn
    Xf, X = points(T)
    r = Xf[:, 1:] - Xf[:, :-1]
    L = torch.sqrt((r * r).sum(-1)).sum(-1)
    return X, L
