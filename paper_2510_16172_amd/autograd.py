"""torch.autograd.Function around fpt_solve / fpt_grad.

Forward: the HIP solver (interaction points X* and lengths L*).
Backward: the implicit-differentiation kernel (Sec. III-D, Eqs. 8-13): one
block-tridiagonal Hessian solve per path, no unrolled iterations. Gradients
flow to the endpoint table ``pts [3][Q]`` and the object table
``obj [9][K]`` (rows b, a1, a2); ids, order, src and dst are not
differentiable. A collapsed minimiser with one interior zero-length
segment is differentiated as the minimiser of the length without that
segment under the constraint that its two points coincide (the implicit
function theorem on that problem's KKT conditions). Paths flagged NOGRAD
(invalid, non-finite, or any other collapse) contribute no gradient.
"""
from __future__ import annotations

import torch

from . import fpt


class FermatPaths(torch.autograd.Function):

    @staticmethod
    def forward(ctx, pts, obj, src, dst, ids, order, solver, opts):
        db = fpt.DeviceBatch.from_tensors(obj.detach(), pts.detach(), src, dst,
                                          ids, order, S=opts.scale)
        out = solver.solve(db, opts)
        ctx.solver = solver
        ctx.db = db
        ctx.out = out
        ctx.mark_non_differentiable(out["status"])
        return out["x"], out["len"], out["status"]

    @staticmethod
    def backward(ctx, g_x, g_len, _g_status):
        db = ctx.db
        g_pts = torch.zeros_like(db.pts)
        g_obj = torch.zeros_like(db.obj)
        g_x = None if g_x is None else g_x.contiguous()
        g_len = None if g_len is None else g_len.contiguous()
        ctx.solver.grad(db, ctx.out, g_len=g_len, g_x=g_x, g_pts=g_pts,
                        g_obj=g_obj)
        return g_pts, g_obj, None, None, None, None, None, None


def fermat_paths(pts, obj, src, dst, ids, order=None, solver=None, opts=None):
    """(x [n_max][3][N], len [N], status [N]) with autograd support."""
    if solver is None:
        solver = fpt.Solver(pts.device.index or 0)
    if opts is None:
        opts = fpt.Opts()
    return FermatPaths.apply(pts, obj, src, dst, ids, order, solver, opts)


def object_grad_to_vertices(g_obj, edge_mask):
    """Chain rule from (b, a1, a2) to the vertices of a face (b = v0,
    a1 = v1 - v0, a2 = v3 - v0) or an edge (b = v0, a1 = v1 - v0).
    Returns g_v0, g_v1, g_v3 ([3][K] each; g_v3 is 0 for edges)."""
    gb, ga1, ga2 = g_obj[0:3], g_obj[3:6], g_obj[6:9]
    ga2 = torch.where(edge_mask[None, :], torch.zeros_like(ga2), ga2)
    return gb - ga1 - ga2, ga1, ga2
