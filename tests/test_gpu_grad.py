"""Parity of the implicit-differentiation backward kernel (fpt_grad, through
the C ABI) with the oracle's IFT gradient and with finite differences of the
oracle's solve (Sec. III-D)."""
import numpy as np
import pytest

import gpu_util
import pins
from paper_2510_16172_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2510_16172_amd import fpt
    s = fpt.Solver(0)
    yield s
    s.close()


def _fwd_grad(solver, b, g_len, g_x, iters=128, with_order=True):
    """GPU forward + backward; per-path (g_slot, g_end) and reduced grads."""
    import torch
    from paper_2510_16172_amd import fpt
    db = fpt.DeviceBatch(b, with_order=with_order)
    out = solver.solve(db, fpt.Opts(scale=b.S, iters=iters))
    gl = torch.from_numpy(np.ascontiguousarray(g_len, np.float32)).cuda()
    gx = torch.from_numpy(np.ascontiguousarray(g_x, np.float32)).cuda()
    g_slot = torch.empty((b.n_max, 9, b.N), dtype=torch.float32, device="cuda")
    g_end = torch.empty((6, b.N), dtype=torch.float32, device="cuda")
    g_pts, g_obj = solver.grad(db, out, g_len=gl, g_x=gx, g_slot=g_slot,
                               g_end=g_end)
    torch.cuda.synchronize()
    o = {k: v.cpu().numpy() for k, v in out.items()}
    return o, g_slot.cpu().numpy(), g_end.cpu().numpy(), g_pts.cpu().numpy(), g_obj.cpu().numpy()


def _compare_per_path(b, o, g_slot, g_end, ref, gref, mask, rtol):
    """GPU per-path gradients vs the oracle's at the oracle's solution, on
    paths in `mask`; tolerance relative to each path's largest entry."""
    n = b.n_max
    gs = np.transpose(g_slot, (2, 0, 1))           # N, n, 9
    ge = g_end.T                                    # N, 6
    want_slot = np.concatenate([gref["g_b"], gref["g_a"].reshape(b.N, n, 6)], -1)
    want_end = np.concatenate([gref["g_tx"], gref["g_rx"]], -1)
    bad = 0
    for i in np.nonzero(mask)[0]:
        k = int(b.order[i])
        w = np.concatenate([want_slot[i, :k].ravel(), want_end[i]])
        g = np.concatenate([gs[i, :k].ravel(), ge[i]])
        scale = 1.0 + np.abs(w).max()
        if not np.all(np.abs(g - w) <= rtol * scale):
            bad += 1
    return bad


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_grad_vs_oracle_canyon(solver, oracle_mod, n):
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 3000, seed=5000 + n, n=n)
    g_len, g_x = scenes.upstream_grads(b.N, b.n_max, seed=5100 + n)
    o, g_slot, g_end, g_pts, g_obj = _fwd_grad(solver, b, g_len, g_x)
    ref = oracle_mod.solve(b, threads=8)
    gref = oracle_mod.grad(b, ref["t"], g_len.astype(np.float64),
                           np.transpose(g_x, (2, 0, 1)).astype(np.float64), threads=8)
    s = gpu_util.summary(b, o, ref)
    from paper_2510_16172_amd import fpt
    col_gpu = (o["status"] & fpt.ST_COLLAPSED) != 0
    # well-posed paths: certified on the GPU, smooth and unique per the oracle
    mask = s["cert"] & ~s["col"] & ~s["ill"] & (gref["status"] == 0) & ~col_gpu
    assert mask.mean() > {1: 0.95, 2: 0.75, 3: 0.6, 4: 0.45, 5: 0.35, 6: 0.25}[n]
    bad = _compare_per_path(b, o, g_slot, g_end, ref, gref, mask, rtol=2e-3)
    print(f"n={n} compared={mask.sum()} bad={bad}", flush=True)
    assert bad <= max(1, int(0.002 * mask.sum()))
    # collapsed minimisers with one interior zero-length segment: the
    # constrained (KKT) gradient, against the oracle's at its solution
    nograd = (o["status"] & fpt.ST_NOGRAD) != 0
    kkt = (s["cert"] & col_gpu & ~nograd & s["col"] & (gref["status"] == oracle_mod.KKT))
    if n >= 2:
        assert kkt.sum() > 0.5 * (col_gpu & s["cert"]).sum()
        bad_k = _compare_per_path(b, o, g_slot, g_end, ref, gref, kkt, rtol=2e-3)
        print(f"n={n} collapsed compared={kkt.sum()} bad={bad_k}", flush=True)
        assert bad_k <= max(1, int(0.002 * kkt.sum()))
    # no gradient: invalid and non-finite paths, and collapses the
    # constrained form does not cover; they contribute exactly zero
    bad_in = (o["status"] & (fpt.ST_INVALID | fpt.ST_NONFINITE)) != 0
    assert np.all(nograd[bad_in])
    assert not np.any(nograd & ~bad_in & ~col_gpu)
    if n == 1:
        np.testing.assert_array_equal(nograd, bad_in | col_gpu)
    assert np.all(g_slot[:, :, nograd] == 0) and np.all(g_end[:, nograd] == 0)


def test_grad_vs_oracle_mixed_orders(solver, oracle_mod):
    """Orders 1-6 in one bucketed batch: the smooth kernels take their
    order's bucket, the collapsed-minimiser kernels the shared bin of
    collapsed paths filtered by order; per path against the oracle."""
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 24000, seed=5050, n=None, n_max=6)
    g_len, g_x = scenes.upstream_grads(b.N, b.n_max, seed=5051)
    o, g_slot, g_end, g_pts, g_obj = _fwd_grad(solver, b, g_len, g_x)
    ref = oracle_mod.solve(b, threads=8)
    gref = oracle_mod.grad(b, ref["t"], g_len.astype(np.float64),
                           np.transpose(g_x, (2, 0, 1)).astype(np.float64), threads=8)
    s = gpu_util.summary(b, o, ref)
    from paper_2510_16172_amd import fpt
    col_gpu = (o["status"] & fpt.ST_COLLAPSED) != 0
    nograd = (o["status"] & fpt.ST_NOGRAD) != 0
    smooth = s["cert"] & ~s["col"] & ~s["ill"] & (gref["status"] == 0) & ~col_gpu
    kkt = s["cert"] & col_gpu & ~nograd & s["col"] & (gref["status"] == oracle_mod.KKT)
    for name, m in (("smooth", smooth), ("collapsed", kkt)):
        for n in range(1 if name == "smooth" else 2, 7):
            mo = m & (b.order == n)
            assert mo.sum() > 20, (name, n, mo.sum())
            bad = _compare_per_path(b, o, g_slot, g_end, ref, gref, mo, rtol=2e-3)
            print(f"{name} n={n} compared={mo.sum()} bad={bad}", flush=True)
            assert bad <= max(1, int(0.002 * mo.sum()))
    assert np.all(g_slot[:, :, nograd] == 0) and np.all(g_end[:, nograd] == 0)


def test_grad_reduction_matches_per_path_sum(solver):
    """g_obj / g_pts equal the sums of the per-path outputs (float atomics:
    to rounding), for the LDS-accumulated canyon tables."""
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 20000, seed=5200, n=None, n_max=4)
    g_len, g_x = scenes.upstream_grads(b.N, b.n_max, seed=5201)
    o, g_slot, g_end, g_pts, g_obj = _fwd_grad(solver, b, g_len, g_x, iters=64)
    want_obj = np.zeros((9, b.K))
    want_pts = np.zeros((3, b.Q))
    for j in range(b.n_max):
        act = b.order > j
        for r in range(9):
            np.add.at(want_obj[r], b.ids[j, act], g_slot[j, r, act].astype(np.float64))
    for c in range(3):
        np.add.at(want_pts[c], b.src, g_end[c].astype(np.float64))
        np.add.at(want_pts[c], b.dst, g_end[3 + c].astype(np.float64))
    sc_obj = 1.0 + np.abs(want_obj).max()
    sc_pts = 1.0 + np.abs(want_pts).max()
    np.testing.assert_allclose(g_obj, want_obj, atol=2e-5 * sc_obj)
    np.testing.assert_allclose(g_pts, want_pts, atol=2e-5 * sc_pts)
    # edges' padded a2 rows receive nothing
    edge = np.all(b.obj[6:9] == 0, axis=0)
    assert np.all(g_obj[6:9, edge] == 0)


def test_grad_global_atomics_path(solver, oracle_mod):
    """Per-path geometry (K = N n objects: too large for the LDS tables) uses
    global atomics; checked against the oracle gradient."""
    b = scenes.random_paths(4000, 3, seed=5300)
    g_len, g_x = scenes.upstream_grads(b.N, b.n_max, seed=5301)
    o, g_slot, g_end, g_pts, g_obj = _fwd_grad(solver, b, g_len, g_x,
                                               with_order=False)
    ref = oracle_mod.solve(b, threads=8)
    gref = oracle_mod.grad(b, ref["t"], g_len.astype(np.float64),
                           np.transpose(g_x, (2, 0, 1)).astype(np.float64), threads=8)
    s = gpu_util.summary(b, o, ref)
    mask = s["cert"] & ~s["col"] & ~s["ill"] & (gref["status"] == 0)
    bad = _compare_per_path(b, o, g_slot, g_end, ref, gref, mask, rtol=2e-3)
    assert bad <= max(1, int(0.002 * mask.sum()))
    # each object belongs to one path: the reduced table is the per-path one
    for j in range(3):
        np.testing.assert_allclose(g_obj[:, b.ids[j]], g_slot[j], atol=1e-6,
                                   rtol=1e-6)


def test_grad_global_atomics_collapsed(solver, oracle_mod):
    """Canyon order-3 paths, each with its own objects (K = 3N: too large
    for the LDS tables), so both gradient kernels add straight into the
    global gradient; smooth and collapsed paths against the oracle, and the
    reduced table equal to the per-path one."""
    sc = scenes.canyon_scene()
    b0 = scenes.canyon_sample_paths(sc, 3000, seed=5310, n=3)
    b = pins.batch_from_paths([pins.path_geometry(b0, i) for i in range(b0.N)], S=b0.S)
    assert 9 * b.K * 8 > 48 * 1024
    g_len, g_x = scenes.upstream_grads(b.N, b.n_max, seed=5311)
    o, g_slot, g_end, g_pts, g_obj = _fwd_grad(solver, b, g_len, g_x)
    ref = oracle_mod.solve(b, threads=8)
    gref = oracle_mod.grad(b, ref["t"], g_len.astype(np.float64),
                           np.transpose(g_x, (2, 0, 1)).astype(np.float64), threads=8)
    s = gpu_util.summary(b, o, ref)
    from paper_2510_16172_amd import fpt
    col_gpu = (o["status"] & fpt.ST_COLLAPSED) != 0
    nograd = (o["status"] & fpt.ST_NOGRAD) != 0
    smooth = s["cert"] & ~s["col"] & ~s["ill"] & (gref["status"] == 0) & ~col_gpu
    kkt = s["cert"] & col_gpu & ~nograd & s["col"] & (gref["status"] == oracle_mod.KKT)
    assert smooth.sum() > 1000 and kkt.sum() > 300
    for m in (smooth, kkt):
        bad = _compare_per_path(b, o, g_slot, g_end, ref, gref, m, rtol=2e-3)
        assert bad <= max(1, int(0.002 * m.sum()))
    for j in range(3):
        np.testing.assert_allclose(g_obj[:, b.ids[j]], g_slot[j], atol=1e-6, rtol=1e-6)
    np.testing.assert_allclose(g_pts[:, b.src], g_end[0:3], atol=1e-6, rtol=1e-6)
    np.testing.assert_allclose(g_pts[:, b.dst], g_end[3:6], atol=1e-6, rtol=1e-6)


def test_grad_corner(solver, oracle_mod):
    """Hand-built collapses: two planes meeting at a line (the constrained
    gradient, against the oracle's) and two crossing edges (no gradient)."""
    import test_oracle_pins as T
    b = pins.batch_from_paths(T.corner_paths(200, seed=98), S=10.0)
    g_len, g_x = scenes.upstream_grads(b.N, b.n_max, seed=5320)
    o, g_slot, g_end, g_pts, g_obj = _fwd_grad(solver, b, g_len, g_x)
    ref = oracle_mod.solve(b, threads=8)
    gref = oracle_mod.grad(b, ref["t"], g_len.astype(np.float64),
                           np.transpose(g_x, (2, 0, 1)).astype(np.float64), threads=8)
    from paper_2510_16172_amd import fpt
    st = o["status"]
    assert st[0] & fpt.ST_COLLAPSED and st[0] & fpt.ST_NOGRAD and st[0] & fpt.ST_CONVERGED
    assert np.all(g_slot[:, :, 0] == 0) and np.all(g_end[:, 0] == 0)
    s = gpu_util.summary(b, o, ref)
    kkt = (s["cert"] & ((st & fpt.ST_COLLAPSED) != 0) & ((st & fpt.ST_NOGRAD) == 0)
           & (gref["status"] == oracle_mod.KKT))
    assert kkt.sum() >= 60
    bad = _compare_per_path(b, o, g_slot, g_end, ref, gref, kkt, rtol=2e-3)
    assert bad == 0


def test_grad_vs_finite_differences(solver, oracle_mod):
    """GPU gradient of sum(gl L + gx . x) vs central differences of the FP64
    oracle's solve (h = 2^-10 m ~ 1e-3 m, Richardson-extrapolated), over all
    inputs of 64 order-3 canyon paths (each path given its own objects)."""
    import pins
    sc = scenes.canyon_scene()
    b0 = scenes.canyon_sample_paths(sc, 2000, seed=5400, n=3)
    ref0 = oracle_mod.solve(b0, threads=8)
    ok0 = np.nonzero(ref0["flags"] == 0)[0]
    paths = [pins.path_geometry(b0, int(i)) for i in ok0[:64]]
    b = pins.batch_from_paths(paths, S=b0.S)
    g_len, g_x = scenes.upstream_grads(b.N, b.n_max, seed=5401)
    o, g_slot, g_end, g_pts, g_obj = _fwd_grad(solver, b, g_len, g_x)
    import test_oracle_pins as T
    gl = g_len.astype(np.float64)
    gx = np.transpose(g_x, (2, 0, 1)).astype(np.float64)
    h = 2.0 ** -10
    d1 = T._fd_grad(oracle_mod, b, gl, gx, h)
    d2 = T._fd_grad(oracle_mod, b, gl, gx, h / 2)
    fd_tx, fd_rx, fd_obj = [(4.0 * y - x) / 3.0 for x, y in zip(d1, d2)]
    from paper_2510_16172_amd import fpt
    cert = (o["status"] & fpt.ST_CONVERGED) != 0
    assert cert.mean() > 0.9
    checked = 0
    for i in np.nonzero(cert)[0]:
        want = np.concatenate([fd_tx[i], fd_rx[i], fd_obj[i].ravel()])
        got = np.concatenate([g_pts[:, b.src[i]], g_pts[:, b.dst[i]],
                              np.stack([g_obj[:, b.ids[j, i]] for j in range(3)]).ravel()])
        edge = [np.all(b.obj[6:9, b.ids[j, i]] == 0) for j in range(3)]
        for j in range(3):
            if edge[j]:
                want[6 + 9 * j + 6: 6 + 9 * j + 9] = 0.0
        scale = 1.0 + np.abs(want).max()
        np.testing.assert_allclose(got, want, atol=2e-3 * scale)
        checked += 1
    assert checked >= 50


@pytest.mark.parametrize("n", [2, 3])
def test_collapsed_grad_vs_finite_differences(solver, oracle_mod, n):
    """Collapsed minimisers (one interior zero-length segment, stable under
    perturbation): the GPU gradient against central differences of the FP64
    oracle's solve, over all inputs of each path."""
    import test_oracle_pins as T
    paths, S = T.stable_single_collapses(oracle_mod, n, 48, seed=5500 + n)
    assert len(paths) >= 24
    b = pins.batch_from_paths(paths, S=S)
    g_len, g_x = scenes.upstream_grads(b.N, b.n_max, seed=5501)
    o, g_slot, g_end, g_pts, g_obj = _fwd_grad(solver, b, g_len, g_x)
    gl = g_len.astype(np.float64)
    gx = np.transpose(g_x, (2, 0, 1)).astype(np.float64)
    h = 2.0 ** -10
    d1 = T._fd_grad(oracle_mod, b, gl, gx, h)
    d2 = T._fd_grad(oracle_mod, b, gl, gx, h / 2)
    fd_tx, fd_rx, fd_obj = [(4.0 * y - x) / 3.0 for x, y in zip(d1, d2)]
    from paper_2510_16172_amd import fpt
    st = o["status"]
    cert = (st & fpt.ST_CONVERGED) != 0
    has = cert & ((st & fpt.ST_COLLAPSED) != 0) & ((st & fpt.ST_NOGRAD) == 0)
    assert has.mean() > 0.8
    for i in np.nonzero(has)[0]:
        want = np.concatenate([fd_tx[i], fd_rx[i], fd_obj[i].ravel()])
        got = np.concatenate([g_pts[:, b.src[i]], g_pts[:, b.dst[i]],
                              np.stack([g_obj[:, b.ids[j, i]] for j in range(n)]).ravel()])
        for j in range(n):
            if np.all(b.obj[6:9, b.ids[j, i]] == 0):
                want[6 + 9 * j + 6: 6 + 9 * j + 9] = 0.0
        scale = 1.0 + np.abs(want).max()
        np.testing.assert_allclose(got, want, atol=2e-3 * scale)


def test_autograd_function(solver, oracle_mod):
    import torch
    from paper_2510_16172_amd import fpt
    from paper_2510_16172_amd.autograd import fermat_paths
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 2000, seed=5500, n=2)
    dev = "cuda"
    pts = torch.from_numpy(b.pts).to(dev).requires_grad_(True)
    obj = torch.from_numpy(b.obj).to(dev).requires_grad_(True)
    src = torch.from_numpy(b.src).to(dev)
    dst = torch.from_numpy(b.dst).to(dev)
    ids = torch.from_numpy(b.ids).to(dev)
    opts = fpt.Opts(scale=b.S, iters=128)
    x, L, st = fermat_paths(pts, obj, src, dst, ids, None, solver, opts)
    g_len, g_x = scenes.upstream_grads(b.N, b.n_max, seed=5501)
    w_len = torch.from_numpy(g_len).to(dev)
    w_x = torch.from_numpy(g_x).to(dev)
    loss = (w_len * L).sum() + (w_x * x).sum()
    loss.backward()
    # same as the direct fpt_grad call
    o, g_slot, g_end, g_pts, g_obj = _fwd_grad(solver, b, g_len, g_x, with_order=False)
    np.testing.assert_allclose(obj.grad.cpu().numpy(), g_obj, rtol=1e-4,
                               atol=1e-4 * (1 + np.abs(g_obj).max()))
    np.testing.assert_allclose(pts.grad.cpu().numpy(), g_pts, rtol=1e-4,
                               atol=1e-4 * (1 + np.abs(g_pts).max()))


def _fd_vertex_grad(oracle_mod, b, gl, gx, h):
    """Central differences of f = sum_i gl_i L*_i + gx_i . x*_i through the
    oracle solve with respect to the vertices of every object: a face is
    b = v0, a1 = v1 - v0, a2 = v3 - v0, an edge b = v0, a1 = v1 - v0. Moving
    v0 moves b and (with the opposite sign) a1 and, for a face, a2; moving
    v1 moves a1; moving v3 moves a2 (faces only). Each path owns its objects,
    so every path is perturbed at once. h = 2^-k is exact on these FP32
    values (all below 2^13 in magnitude). Returns [N][n][3 vertices][3]."""
    N, n = b.N, b.n_max
    edge = np.all(b.obj[6:9] == 0, axis=0)

    def f(obj):
        r = oracle_mod.solve(scenes.Batch(obj, b.pts, b.src, b.dst, b.order,
                                          b.ids, b.S), threads=8)
        return gl * r["len"] + np.einsum("njc,njc->n", gx, r["x"])

    g = np.zeros((N, n, 3, 3))
    for j in range(n):
        k = b.ids[j]
        face = ~edge[k]
        for v in range(3):
            for c in range(3):
                o1, o2 = b.obj.copy(), b.obj.copy()
                for sgn, o in ((1.0, o1), (-1.0, o2)):
                    if v == 0:
                        o[c, k] += sgn * h
                        o[3 + c, k] -= sgn * h
                        o[6 + c, k[face]] -= sgn * h
                    elif v == 1:
                        o[3 + c, k] += sgn * h
                    else:
                        o[6 + c, k[face]] += sgn * h
                d = (f(o1) - f(o2)) / (2.0 * h)
                if v == 2:
                    d = np.where(face, d, 0.0)
                g[:, j, v, c] = d
    return g


def test_vertex_gradients_vs_finite_differences(solver, oracle_mod):
    """d(sum gl L* + gx . X*) / d(face and edge vertices): the GPU's object
    gradient through the vertex chain rule (object_grad_to_vertices) against
    Richardson-extrapolated central differences of the FP64 oracle's solve
    with respect to the vertices themselves, on 64 smooth order-3 canyon
    paths (each path given its own objects)."""
    import torch
    import pins
    from paper_2510_16172_amd import fpt
    from paper_2510_16172_amd.autograd import object_grad_to_vertices
    sc = scenes.canyon_scene()
    b0 = scenes.canyon_sample_paths(sc, 2000, seed=5600, n=3)
    ref0 = oracle_mod.solve(b0, threads=8)
    ok0 = np.nonzero(ref0["flags"] == 0)[0]
    b = pins.batch_from_paths([pins.path_geometry(b0, int(i)) for i in ok0[:64]], S=b0.S)
    assert np.abs(b.obj).max() < 2.0 ** 13
    g_len, g_x = scenes.upstream_grads(b.N, b.n_max, seed=5601)
    o, g_slot, g_end, g_pts, g_obj = _fwd_grad(solver, b, g_len, g_x)
    edge = np.all(b.obj[6:9] == 0, axis=0)
    gv0, gv1, gv3 = (t.cpu().numpy() for t in object_grad_to_vertices(
        torch.from_numpy(g_obj), torch.from_numpy(edge)))
    gl = g_len.astype(np.float64)
    gx = np.transpose(g_x, (2, 0, 1)).astype(np.float64)
    h = 2.0 ** -10
    d1 = _fd_vertex_grad(oracle_mod, b, gl, gx, h)
    d2 = _fd_vertex_grad(oracle_mod, b, gl, gx, h / 2)
    fd = (4.0 * d2 - d1) / 3.0
    cert = (o["status"] & fpt.ST_CONVERGED) != 0
    assert cert.mean() > 0.9
    checked = 0
    for i in np.nonzero(cert)[0]:
        got = np.stack([np.stack([gv0[:, b.ids[j, i]], gv1[:, b.ids[j, i]],
                                  gv3[:, b.ids[j, i]]]) for j in range(3)])
        want = fd[i]
        scale = 1.0 + np.abs(want).max()
        np.testing.assert_allclose(got, want, atol=2e-3 * scale, err_msg=f"path {i}")
        checked += 1
    # faces and edges both appear
    assert edge[b.ids[:, cert]].any() and (~edge[b.ids[:, cert]]).any()
    assert checked >= 50
