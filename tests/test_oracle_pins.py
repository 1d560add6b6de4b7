"""Pins of the FP64 oracle against what the geometry fixes (CPU only).

Each test compares the oracle with something other than itself: hand-worked
minimisers (tests/golden), the image method, the single-edge closed form,
brute-force grid search, optimality conditions and symmetries of the problem
of Sec. III-B, and central finite differences for the gradient of Sec. III-D.
"""
import json
import os

import numpy as np
import pytest

import pins
from paper_2510_16172_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_worked.json")


def _solve(oracle_mod, b):
    r = oracle_mod.solve(b, threads=4)
    assert np.all(r["flags"] & (oracle_mod.INVALID | oracle_mod.NOCONV) == 0)
    return r


def test_golden_hand_worked(oracle_mod):
    cases = json.load(open(GOLDEN))["cases"]
    paths = [(np.array(c["tx"], float), np.array(c["rx"], float),
              [tuple(np.array(v, float) for v in o) for o in c["objects"]])
             for c in cases]
    b = pins.batch_from_paths(paths, S=10.0)
    r = _solve(oracle_mod, b)
    want = {"collapsed pass-through at a corner line",
            "straight through the corner of three planes",
            "ground reflection then a corner line"}
    for i, c in enumerate(cases):
        n = len(c["objects"])
        # smooth minimisers: the smoothing (eps = 1e-15 S at the last level)
        # moves a point by O(eps); where points coincide by O(eps^(2/3)),
        # about 1e-10 S
        atol = 1e-9 * b.S if c["name"] in want else 1e-9
        np.testing.assert_allclose(r["x"][i, :n], np.array(c["x"]), atol=atol,
                                   err_msg=c["name"])
        assert abs(r["len"][i] - c["L"]) < 1e-12, c["name"]
    names = [c["name"] for c in cases]
    collapsed = r["flags"] & oracle_mod.COLLAPSED != 0
    assert {names[i] for i in np.nonzero(collapsed)[0]} == want


def test_single_reflection_image_method(oracle_mod):
    N = 400
    b = scenes.random_paths(N, 1, seed=11, kinds=np.ones((1, N), bool))
    r = _solve(oracle_mod, b)
    n_same = 0
    for i in range(N):
        tx, rx, objs = pins.path_geometry(b, i)
        bb, a1, a2 = objs[0]
        nv = np.cross(a1, a2)
        same_side = np.dot(tx - bb, nv) * np.dot(rx - bb, nv) > 0
        if same_side:
            n_same += 1
            x, L, valid = pins.image_method(tx, rx, objs)
            assert valid
            np.testing.assert_allclose(r["x"][i, 0], x[0], atol=1e-9 * b.S)
            assert abs(r["len"][i] - L) < 1e-12 * b.S
        else:
            # pass-through: the straight segment crosses the plane
            L = np.linalg.norm(rx - tx)
            assert abs(r["len"][i] - L) < 1e-12 * b.S
            s = np.dot(bb - tx, nv) / np.dot(rx - tx, nv)
            np.testing.assert_allclose(r["x"][i, 0], tx + s * (rx - tx),
                                       atol=1e-9 * b.S)
    assert 100 < n_same < 300


@pytest.mark.parametrize("n", [2, 3, 4])
def test_reflection_chains_image_method(oracle_mod, n):
    N = 3000
    b = scenes.random_paths(N, n, seed=20 + n, kinds=np.ones((n, N), bool))
    r = _solve(oracle_mod, b)
    n_valid = 0
    for i in range(N):
        tx, rx, objs = pins.path_geometry(b, i)
        x, L, valid = pins.image_method(tx, rx, objs)
        if not valid:
            continue
        n_valid += 1
        assert abs(r["len"][i] - L) < 1e-11 * b.S
        np.testing.assert_allclose(r["x"][i, :n], x, atol=1e-8 * b.S)
    assert n_valid >= 30


def test_single_edge_closed_form(oracle_mod):
    N = 500
    b = scenes.random_paths(N, 1, seed=31, kinds=np.zeros((1, N), bool))
    r = _solve(oracle_mod, b)
    for i in range(N):
        tx, rx, objs = pins.path_geometry(b, i)
        bb, a1, _ = objs[0]
        t, x, L = pins.edge_closed_form(tx, rx, bb, a1)
        assert abs(r["len"][i] - L) < 1e-12 * b.S
        np.testing.assert_allclose(r["x"][i, 0], x, atol=1e-9 * b.S)
        assert abs(r["t"][i, 0, 0] - t) < 1e-9 * b.S
        assert r["t"][i, 0, 1] == 0.0


def test_brute_force_tiny(oracle_mod):
    b1 = scenes.random_paths(8, 1, seed=41)
    b2 = scenes.random_paths(10, 2, seed=42)
    for b in (b1, b2):
        r = _solve(oracle_mod, b)
        for i in range(b.N):
            tx, rx, objs = pins.path_geometry(b, i)
            t, L = pins.brute_force(tx, rx, objs)
            # the oracle is at least as short, and not measurably shorter
            assert r["len"][i] <= L + 1e-12 * b.S
            assert L - r["len"][i] < 1e-9 * b.S
            xb = pins.path_points(tx, rx, objs, t)[1:-1]
            np.testing.assert_allclose(r["x"][i, :len(objs)], xb,
                                       atol=1e-4 * b.S)


def _check_optimality(oracle_mod, b, r, rng):
    """Stationarity, reflection / Keller-cone laws, subgradients at
    collapsed minimisers, bounds. Returns the number of collapsed paths."""
    probes = 0
    collapsed = 0
    for i in range(b.N):
        tx, rx, objs = pins.path_geometry(b, i)
        n = len(objs)
        xs = np.vstack([tx, r["x"][i, :n], rx])
        u, ell = pins.segment_dirs(xs)
        assert r["len"][i] >= np.linalg.norm(rx - tx) - 1e-12 * b.S
        assert abs(r["len"][i] - ell.sum()) < 1e-12 * b.S
        for j, (bb, a1, a2) in enumerate(objs):
            x = r["x"][i, j]
            tt = r["t"][i, j]
            np.testing.assert_allclose(bb + tt[0] * a1 + tt[1] * a2, x,
                                       atol=1e-12 * b.S)
        if r["flags"][i] & oracle_mod.COLLAPSED:
            # nonsmooth minimiser: 0 must lie in the subdifferential of the
            # convex L (Sec. III-B, Eq. 5), i.e. every zero-length segment has
            # a subgradient w, |w| <= 1, that makes all points stationary
            res, wmax = pins.subgradient_optimality(tx, rx, objs, xs, b.S)
            assert res < 1e-9, (i, res)
            assert 0.0 < wmax <= 1.0 + 1e-9, (i, wmax)
            collapsed += 1
            continue
        for j, (bb, a1, a2) in enumerate(objs):
            du = u[j] - u[j + 1]
            assert abs(np.dot(a1, du)) < 1e-9 * np.linalg.norm(a1)
            if np.any(a2 != 0):
                # law of reflection: equal tangential parts, and the normal
                # parts are equal (pass-through) or opposite (specular)
                assert abs(np.dot(a2, du)) < 1e-9 * np.linalg.norm(a2)
                nv = np.cross(a1, a2)
                nv /= np.linalg.norm(nv)
                assert abs(abs(np.dot(u[j], nv)) - abs(np.dot(u[j + 1], nv))) < 1e-9
            else:
                # Keller cone: equal angles with the edge direction
                e = a1 / np.linalg.norm(a1)
                assert abs(np.dot(u[j], e) - np.dot(u[j + 1], e)) < 1e-9
    # L* <= L(T) for random T near and far from T*
    for scale in (1e-3, 1e-1, 3.0):
        t = r["t"] + scale * rng.standard_normal(r["t"].shape)
        for j in range(b.n_max):
            edge = np.all(b.obj[6:9, np.maximum(b.ids[j], 0)] == 0, axis=0)
            t[edge, j, 1] = 0.0
        L = oracle_mod.length(b, np.nan_to_num(t))
        ok = b.order > 0
        assert np.all(r["len"][ok] <= L[ok] + 1e-12 * b.S)
        probes += ok.sum()
    return collapsed


def test_optimality_random(oracle_mod):
    rng = np.random.default_rng(5)
    for n in (1, 2, 3, 5, 6):
        b = scenes.random_paths(300, n, seed=50 + n)
        r = _solve(oracle_mod, b)
        ncol = _check_optimality(oracle_mod, b, r, rng)
        assert n == 1 or ncol >= 30


def test_optimality_canyon(oracle_mod):
    rng = np.random.default_rng(6)
    sc = scenes.canyon_scene()
    for n in (1, 2, 3, 5, 6):
        b = scenes.canyon_sample_paths(sc, 400, seed=60 + n, n=n)
        r = _solve(oracle_mod, b)
        ncol = _check_optimality(oracle_mod, b, r, rng)
        assert n == 1 or ncol >= 30


def test_reversal_symmetry(oracle_mod):
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 500, seed=71, n=3)
    rev = scenes.Batch(b.obj, b.pts, b.dst.copy(), b.src.copy(), b.order,
                       np.ascontiguousarray(b.ids[::-1]), b.S)
    r = _solve(oracle_mod, b)
    q = _solve(oracle_mod, rev)
    np.testing.assert_allclose(q["len"], r["len"], rtol=0, atol=1e-11 * b.S)
    # points are unique unless the Hessian is singular (ILL: e.g. a face
    # between two of its own edges, where the middle point can slide)
    unique = ((r["flags"] | q["flags"]) & oracle_mod.ILL) == 0
    assert unique.sum() > 0.95 * b.N
    np.testing.assert_allclose(q["x"][unique, ::-1], r["x"][unique],
                               atol=1e-7 * b.S)


def test_rigid_motion_and_reparametrisation(oracle_mod):
    rng = np.random.default_rng(7)
    b = scenes.random_paths(300, 3, seed=72)
    r = _solve(oracle_mod, b)
    # rigid motion x -> R x + c applied to every point and basis vector
    Rm, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    c = rng.uniform(-3, 3, 3)
    obj = b.obj.astype(np.float64)
    pts = b.pts.astype(np.float64)
    obj2 = np.vstack([Rm @ obj[0:3] + c[:, None], Rm @ obj[3:6], Rm @ obj[6:9]])
    edge = np.all(obj[6:9] == 0, axis=0)
    obj2[6:9, edge] = 0.0
    pts2 = Rm @ pts + c[:, None]
    b2 = scenes.Batch(obj2.astype(np.float32), pts2.astype(np.float32),
                      b.src, b.dst, b.order, b.ids, b.S)
    r2 = _solve(oracle_mod, b2)
    # inputs were rounded to FP32 after the motion: compare loosely
    x_mapped = np.einsum("ab,njb->nja", Rm, r["x"]) + c
    np.testing.assert_allclose(r2["x"], x_mapped, atol=1e-4 * b.S)
    np.testing.assert_allclose(r2["len"], r["len"], atol=1e-5 * b.S)
    # reparametrisation: basis a -> a M (M invertible, exact powers of two
    # so that FP32 keeps it exact) and origin b -> b + a1 (t shifts by -1)
    obj3 = obj.copy()
    a1 = obj[3:6].copy()
    a2 = obj[6:9].copy()
    obj3[0:3] = obj[0:3] + a1
    obj3[3:6] = 2.0 * a1
    obj3[6:9] = np.where(edge, 0.0, a2 * 0.5 + a1)
    b3 = scenes.Batch(obj3.astype(np.float32), b.pts, b.src, b.dst, b.order,
                      b.ids, b.S)
    r3 = _solve(oracle_mod, b3)
    np.testing.assert_allclose(r3["x"], r["x"], atol=1e-5 * b.S)
    np.testing.assert_allclose(r3["len"], r["len"], atol=1e-6 * b.S)


def test_edge_scaling_same_point(oracle_mod):
    """An edge is one parameter whatever the length of its direction (the
    padded second parameter stays 0); scaling the direction by 4 divides t
    by 4 and leaves the point unchanged."""
    N = 200
    b = scenes.random_paths(N, 2, seed=73, kinds=np.zeros((2, N), bool))
    r = _solve(oracle_mod, b)
    obj = b.obj.copy()
    obj[3:6] *= 4.0
    r2 = _solve(oracle_mod, scenes.Batch(obj, b.pts, b.src, b.dst, b.order,
                                         b.ids, b.S))
    np.testing.assert_allclose(r2["x"], r["x"], atol=1e-9 * b.S)
    np.testing.assert_allclose(r2["t"] * 4.0, r["t"], atol=1e-9 * b.S)
    assert np.all(r["t"][..., 1] == 0.0)


# ------------------------------------------------------------------ gradient


def _fd_grad(oracle_mod, b, gl, gx, h):
    """Central differences of f = sum_i gl_i L*_i + gx_i . x*_i through the
    oracle solve, one input coordinate at a time for every path at once
    (each path owns its objects and points). The inputs are FP32, so the
    difference quotient divides by the step FP32 actually took."""
    N, n = b.N, b.n_max

    def f(obj, pts):
        r = oracle_mod.solve(scenes.Batch(obj, pts, b.src, b.dst, b.order,
                                          b.ids, b.S), threads=4)
        return gl * r["len"] + np.einsum("njc,njc->n", gx, r["x"])

    g_tx = np.zeros((N, 3))
    g_rx = np.zeros((N, 3))
    g_obj = np.zeros((N, n, 9))
    for which, col, out in (("src", b.src, g_tx), ("dst", b.dst, g_rx)):
        for c in range(3):
            p1, p2 = b.pts.copy(), b.pts.copy()
            p1[c, col] += h
            p2[c, col] -= h
            step = p1[c, col].astype(np.float64) - p2[c, col]
            out[:, c] = (f(b.obj, p1) - f(b.obj, p2)) / step
    for j in range(n):
        for rr in range(9):
            o1, o2 = b.obj.copy(), b.obj.copy()
            o1[rr, b.ids[j]] += h
            o2[rr, b.ids[j]] -= h
            step = o1[rr, b.ids[j]].astype(np.float64) - o2[rr, b.ids[j]]
            g_obj[:, j, rr] = (f(o1, b.pts) - f(o2, b.pts)) / step
    return g_tx, g_rx, g_obj


@pytest.mark.parametrize("n", [1, 2, 3])
def test_gradient_vs_finite_differences(oracle_mod, n):
    N = 64
    b = scenes.random_paths(N, n, seed=80 + n)
    r = _solve(oracle_mod, b)
    rng = np.random.default_rng(81)
    gl = rng.standard_normal(N)
    gx = rng.standard_normal((N, n, 3))
    g = oracle_mod.grad(b, r["t"], gl, gx, threads=4)
    # Richardson extrapolation of central differences at h and h/2: O(h^4)
    h = 2.0 ** -10
    d1 = _fd_grad(oracle_mod, b, gl, gx, h)
    d2 = _fd_grad(oracle_mod, b, gl, gx, h / 2)
    fd_tx, fd_rx, fd_obj = [(4.0 * b2 - b1) / 3.0 for b1, b2 in zip(d1, d2)]
    # only well-separated smooth minimisers (FD across a kink is meaningless)
    seg_min = np.full(N, np.inf)
    for i in range(N):
        tx, rx, objs = pins.path_geometry(b, i)
        xs = np.vstack([tx, r["x"][i, :n], rx])
        seg_min[i] = pins.segment_dirs(xs)[1].min()
    ok = (g["status"] == 0) & (seg_min > 0.05 * b.S) & (r["flags"] == 0)
    assert ok.sum() >= N // 2
    edge = np.stack([np.all(b.obj[6:9, b.ids[j]] == 0, axis=0)
                     for j in range(n)], 1)
    ga = g["g_a"].reshape(N, n, 6)
    for i in np.nonzero(ok)[0]:
        scale = 1.0 + np.abs(fd_obj[i]).max()
        np.testing.assert_allclose(g["g_tx"][i], fd_tx[i], atol=2e-5 * scale)
        np.testing.assert_allclose(g["g_rx"][i], fd_rx[i], atol=2e-5 * scale)
        np.testing.assert_allclose(g["g_b"][i], fd_obj[i, :, 0:3],
                                   atol=2e-5 * scale)
        for j in range(n):
            want = fd_obj[i, j, 3:9].copy()
            if edge[i, j]:
                want[3:] = 0.0  # padded parameter: no gradient
            np.testing.assert_allclose(ga[i, j], want, atol=2e-5 * scale)


def stable_single_collapses(oracle_mod, n, count, seed, wmax=0.9):
    """Canyon paths of order n whose oracle minimiser has exactly one
    zero-length segment, an interior one, with a subgradient of norm below
    wmax (so that the minimiser stays collapsed under small perturbations),
    each returned as its own geometry (tx, rx, objs)."""
    sc = scenes.canyon_scene()
    b0 = scenes.canyon_sample_paths(sc, 4000, seed=seed, n=n)
    r0 = oracle_mod.solve(b0, threads=4)  # (unconverged paths skipped below)
    out = []
    for i in np.nonzero((r0["flags"] & oracle_mod.COLLAPSED) != 0)[0]:
        if r0["flags"][i] & (oracle_mod.NOCONV | oracle_mod.INVALID):
            continue
        tx, rx, objs = pins.path_geometry(b0, int(i))
        xs = np.vstack([tx, r0["x"][i, :n], rx])
        runs, ell = pins.collapse_runs(xs, b0.S)
        if ell[0] < 1e-6 * b0.S or ell[n] < 1e-6 * b0.S:
            continue
        long_runs = [rn for rn in runs if len(rn) > 1]
        if len(long_runs) != 1 or len(long_runs[0]) != 2:
            continue
        a, bb = long_runs[0]
        u = np.diff(xs, axis=0) / ell[:, None]
        _, res, wm = pins.run_subgradient([objs[a], objs[bb]], u[a], u[bb + 1])
        # directions that do not span space (two edges, an edge in a face's
        # plane) leave the multiplier undetermined: not covered
        dirs = [v / np.linalg.norm(v) for k in (a, bb) for v in objs[k][1:]
                if np.any(v != 0)]
        if np.linalg.det(sum(np.outer(v, v) for v in dirs)) <= 1e-3:
            continue
        if wm < wmax and res < 1e-6:
            out.append((tx, rx, objs))
        if len(out) == count:
            break
    return out, b0.S


@pytest.mark.parametrize("n", [2, 3, 4])
def test_collapsed_gradient_vs_finite_differences(oracle_mod, n):
    """The constrained (KKT) gradient at a minimiser with one interior
    zero-length segment against central differences of the oracle's own
    solve (Richardson-extrapolated), over all inputs of each path."""
    paths, S = stable_single_collapses(oracle_mod, n, 24, seed=95 + n)
    assert len(paths) >= 12
    b = pins.batch_from_paths(paths, S=S)
    r = _solve(oracle_mod, b)
    rng = np.random.default_rng(96)
    gl = rng.standard_normal(b.N)
    gx = rng.standard_normal((b.N, n, 3))
    g = oracle_mod.grad(b, r["t"], gl, gx, threads=4)
    kkt = g["status"] == oracle_mod.KKT
    assert kkt.sum() >= len(paths) - 1
    h = 2.0 ** -10
    d1 = _fd_grad(oracle_mod, b, gl, gx, h)
    d2 = _fd_grad(oracle_mod, b, gl, gx, h / 2)
    fd_tx, fd_rx, fd_obj = [(4.0 * b2 - b1) / 3.0 for b1, b2 in zip(d1, d2)]
    edge = np.stack([np.all(b.obj[6:9, b.ids[j]] == 0, axis=0)
                     for j in range(n)], 1)
    ga = g["g_a"].reshape(b.N, n, 6)
    for i in np.nonzero(kkt)[0]:
        scale = 1.0 + np.abs(fd_obj[i]).max()
        np.testing.assert_allclose(g["g_tx"][i], fd_tx[i], atol=1e-7 * scale)
        np.testing.assert_allclose(g["g_rx"][i], fd_rx[i], atol=1e-7 * scale)
        np.testing.assert_allclose(g["g_b"][i], fd_obj[i, :, 0:3],
                                   atol=1e-7 * scale)
        for j in range(n):
            want = fd_obj[i, j, 3:9].copy()
            if edge[i, j]:
                want[3:] = 0.0
            np.testing.assert_allclose(ga[i, j], want, atol=1e-7 * scale)


def corner_paths(n_face, seed):
    """Hand-built collapses: the first path reflects off two edges that cross
    at the origin (x- and y-axis) with TX and RX placed so that both points
    sit at the crossing (subgradient sqrt(2/3) < 1: a collapsed minimiser
    whose objects' directions span only a plane); then n_face paths off the
    planes z = 0 and x = 0 from random TX, RX in the quadrant x, z > 0, of
    which about half collapse onto the planes' meeting line."""
    rng = np.random.default_rng(seed)
    z3 = (0.0, 0.0, 0.0)
    paths = [(np.array([-1.0, -1.0, 1.0]), np.array([1.0, 1.0, 1.0]),
              [(np.array([-5.0, 0, 0]), np.array([10.0, 0, 0]), np.array(z3)),
               (np.array([0, -5.0, 0]), np.array([0, 10.0, 0]), np.array(z3))])]
    for _ in range(n_face):
        tx = rng.uniform([0.2, -3, 0.2], [3, 3, 3])
        rx = rng.uniform([0.2, -3, 0.2], [3, 3, 3])
        paths.append((tx, rx, [
            (np.array([-5.0, -5.0, 0.0]), np.array([10.0, 0, 0]), np.array([0, 10.0, 0])),
            (np.array([0.0, -5.0, -5.0]), np.array([0, 10.0, 0]), np.array([0, 0, 10.0]))]))
    return paths


def test_collapsed_gradient_corner(oracle_mod):
    """Two planes meeting at a line: paths that collapse onto the line get
    the constrained gradient (checked by central differences); two crossing
    edges (directions spanning only a plane) get none."""
    b = pins.batch_from_paths(corner_paths(60, seed=99), S=10.0)
    r = _solve(oracle_mod, b)
    rng = np.random.default_rng(100)
    gl = rng.standard_normal(b.N)
    gx = rng.standard_normal((b.N, 2, 3))
    g = oracle_mod.grad(b, r["t"], gl, gx, threads=4)
    assert r["flags"][0] & oracle_mod.COLLAPSED
    np.testing.assert_allclose(r["x"][0], 0.0, atol=1e-9)
    assert g["status"][0] == oracle_mod.COLLAPSED and np.all(np.isnan(g["g_b"][0]))
    col = np.nonzero((r["flags"][1:] & oracle_mod.COLLAPSED) != 0)[0] + 1
    assert len(col) >= 15
    assert np.all(g["status"][col] == oracle_mod.KKT)
    h = 2.0 ** -10
    d1 = _fd_grad(oracle_mod, b, gl, gx, h)
    d2 = _fd_grad(oracle_mod, b, gl, gx, h / 2)
    fd_tx, fd_rx, fd_obj = [(4.0 * b2 - b1) / 3.0 for b1, b2 in zip(d1, d2)]
    ga = g["g_a"].reshape(b.N, 2, 6)
    for i in col:
        scale = 1.0 + np.abs(fd_obj[i]).max()
        np.testing.assert_allclose(g["g_tx"][i], fd_tx[i], atol=1e-7 * scale)
        np.testing.assert_allclose(g["g_rx"][i], fd_rx[i], atol=1e-7 * scale)
        np.testing.assert_allclose(g["g_b"][i], fd_obj[i, :, 0:3], atol=1e-7 * scale)
        np.testing.assert_allclose(ga[i], fd_obj[i, :, 3:9], atol=1e-7 * scale)


def test_gradient_structure(oracle_mod):
    """A_j^T g_b_j = 0: moving an object within its own span leaves the
    solution unchanged; with g_x = 0 the gradient is the envelope term."""
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 600, seed=90, n=3)
    r = _solve(oracle_mod, b)
    rng = np.random.default_rng(91)
    gl = rng.standard_normal(b.N)
    gx = rng.standard_normal((b.N, 3, 3))
    g = oracle_mod.grad(b, r["t"], gl, gx, threads=4)
    ok = g["status"] == 0
    assert ok.sum() > b.N // 2
    for i in np.nonzero(ok)[0]:
        tx, rx, objs = pins.path_geometry(b, i)
        for j, (bb, a1, a2) in enumerate(objs):
            scale = 1.0 + np.abs(g["g_b"][i, j]).max()
            assert abs(np.dot(a1, g["g_b"][i, j])) < 1e-7 * scale * np.linalg.norm(a1)
            assert abs(np.dot(a2, g["g_b"][i, j])) < 1e-7 * scale * (1 + np.linalg.norm(a2))
    g0 = oracle_mod.grad(b, r["t"], gl, np.zeros_like(gx), threads=4)
    for i in np.nonzero(ok)[0][:100]:
        tx, rx, objs = pins.path_geometry(b, i)
        xs = np.vstack([tx, r["x"][i, :3], rx])
        u, _ = pins.segment_dirs(xs)
        np.testing.assert_allclose(g0["g_tx"][i], -gl[i] * u[0], atol=1e-9)
        np.testing.assert_allclose(g0["g_rx"][i], gl[i] * u[-1], atol=1e-9)


# ------------------------------------------------------------ validity ----
# Post-processing on finite objects (faces are parallelograms b + s a1 + u a2,
# edges segments b + s a1, parameters in [0, 1]).

def _validity_batch(paths, extra_objs, S=10.0):
    """Batch of explicit order-n paths whose object table also holds
    `extra_objs` (occluder candidates that no path uses)."""
    from paper_2510_16172_amd.scenes import Batch
    b = pins.batch_from_paths(paths, S)
    if extra_objs:
        ext = np.array([np.concatenate(o) for o in extra_objs], np.float32).T
        obj = np.concatenate([b.obj, ext], axis=1)
        b = Batch(np.ascontiguousarray(obj), b.pts, b.src, b.dst, b.order, b.ids, b.S)
    return b


def _flags_for(oracle_mod, paths, t_list, extra=(), tol=0.0):
    b = _validity_batch(paths, list(extra))
    n = b.n_max
    t = np.zeros((b.N, n, 2))
    x = np.zeros((b.N, n, 3))
    for i, ((tx, rx, objs), ts) in enumerate(zip(paths, t_list)):
        for j, ((bb, a1, a2), tj) in enumerate(zip(objs, ts)):
            t[i, j] = tj
            x[i, j] = np.asarray(bb) + tj[0] * np.asarray(a1) + tj[1] * np.asarray(a2)
    return oracle_mod.validate(b, t, x, tol=tol)


def test_validity_hand_cases(oracle_mod):
    """Reflection at (1,0,0) of TX (0,0,1) -> RX (2,0,1) on the floor z = 0."""
    E, SP, V = oracle_mod.EXTENT, oracle_mod.SPECULAR, oracle_mod.VISIBLE
    tx, rx = (0.0, 0.0, 1.0), (2.0, 0.0, 1.0)
    floor = ((-1.0, -1.0, 0.0), (4.0, 0.0, 0.0), (0.0, 2.0, 0.0))   # x in [-1,3]
    small = ((-1.0, -1.0, 0.0), (1.0, 0.0, 0.0), (0.0, 2.0, 0.0))   # x in [-1,0]
    wall = ((0.5, -1.0, 0.0), (0.0, 2.0, 0.0), (0.0, 0.0, 2.0))     # x = 0.5
    wall_off = ((0.5, 2.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 2.0))  # y in [2,3]
    edge = ((0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 0.0, 0.0))
    paths = [(tx, rx, [floor]), (tx, rx, [small]), (tx, (2.0, 0.0, -1.0), [floor]),
             (tx, rx, [floor]), (tx, rx, [edge]), (tx, rx, [edge])]
    t_list = [[(0.5, 0.5)], [(2.0, 0.5)], [(0.5, 0.5)], [(0.5, 0.5)],
              [(0.5, 0.0)], [(1.5, 0.0)]]
    f = _flags_for(oracle_mod, paths[:3], t_list[:3])
    assert list(f) == [E | SP | V, SP | V, E | V]
    # the wall at x = 0.5 cuts TX -> (1,0,0) at (0.5, 0, 0.5), inside it
    f = _flags_for(oracle_mod, paths[3:4], t_list[3:4], extra=[wall])
    assert list(f) == [E | SP]
    f = _flags_for(oracle_mod, paths[3:4], t_list[3:4], extra=[wall_off])
    assert list(f) == [E | SP | V]
    # an edge has no side test; its one parameter must lie in [0, 1]
    f = _flags_for(oracle_mod, paths[4:], t_list[4:])
    assert list(f) == [E | SP | V, SP | V]


def test_validity_crossing_vs_linear_solve(oracle_mod):
    """VISIBLE against an independent crossing test: each segment-face pair
    solved with numpy.linalg.solve (LU) instead of Cramer's rule; pairs
    within 1e-7 of a decision boundary are left out."""
    rng = np.random.default_rng(77)
    faces = []
    for _ in range(40):
        b = rng.uniform(-5, 5, 3)
        q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        faces.append((b, q[:, 0] * rng.uniform(1, 4), q[:, 1] * rng.uniform(1, 4)))
    dummy = ((50.0, 50.0, 50.0), (1.0, 0.0, 0.0), (0.0, 0.0, 0.0))  # an edge
    paths, t_list, want, keep = [], [], [], []
    for i in range(400):
        tx = rng.uniform(-6, 6, 3)
        rx = rng.uniform(-6, 6, 3)
        xm = rng.uniform(-6, 6, 3)
        # order-1 path TX -> xm -> RX with xm placed on the dummy edge's line
        obj = ((xm - np.array([0.5, 0, 0])), (1.0, 0.0, 0.0), (0.0, 0.0, 0.0))
        paths.append((tx, rx, [obj]))
        t_list.append([(0.5, 0.0)])
        hit, tie = False, False
        for p, q in ((tx, xm), (xm, rx)):
            for (b, u, v) in faces:
                M = np.stack([q - p, -u, -v], 1)
                if abs(np.linalg.det(M)) <= 1e-12 * np.linalg.norm(q - p) * np.linalg.norm(u) * np.linalg.norm(v):
                    continue
                s, al, be = np.linalg.solve(M, b - p)
                margins = [s - 1e-6, 1 - 1e-6 - s, al, 1 - al, be, 1 - be]
                inside = all(m > 0 for m in margins)
                if min(abs(m) for m in margins) < 1e-7:
                    tie = True
                hit = hit or inside
        want.append(not hit)
        keep.append(not tie)
    b = _validity_batch(paths, faces)
    t = np.array([[tl[0]] for tl in t_list])
    x = np.array([[p[2][0][0] + 0.5 * np.asarray(p[2][0][1])] for p in paths])
    f = oracle_mod.validate(b, t, x)
    got = (f & oracle_mod.VISIBLE) != 0
    keep = np.array(keep)
    assert keep.sum() > 390 and 0.2 < np.mean(want) < 0.9
    np.testing.assert_array_equal(got[keep], np.array(want)[keep])


def test_subgradient_pin_catches_displaced_collapse(oracle_mod):
    """The subgradient check above is sharp: moving a run of coinciding
    points together along a direction they share (a collapse that is no
    longer stationary) or opening the zero-length segment fails it."""
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 400, seed=63, n=3)
    r = _solve(oracle_mod, b)
    moved = opened = 0
    for i in np.nonzero(r["flags"] & oracle_mod.COLLAPSED)[0]:
        tx, rx, objs = pins.path_geometry(b, i)
        xs = np.vstack([tx, r["x"][i, :3], rx])
        runs, _ = pins.collapse_runs(xs, b.S)
        run = next((q for q in runs if len(q) == 2), None)
        if run is None:
            continue
        Qa = pins._span_basis(*objs[run[0]][1:])
        Qb = pins._span_basis(*objs[run[1]][1:])
        # a direction in both objects (their meeting line), if any
        M = Qa @ Qa.T + Qb @ Qb.T
        ev, V = np.linalg.eigh(M)
        if ev[-1] > 2.0 - 1e-9:
            e = V[:, -1]
            ys = xs.copy()
            for k in run:
                ys[k + 1] += 1e-3 * b.S * e
            res, _ = pins.subgradient_optimality(tx, rx, objs, ys, b.S)
            assert res > 1e-5
            moved += 1
        # open the collapse: the first point moves within its own object
        ys = xs.copy()
        ys[run[0] + 1] += 1e-3 * b.S * Qa[:, 0]
        res, _ = pins.subgradient_optimality(tx, rx, objs, ys, b.S)
        assert res > 1e-5
        opened += 1
    assert moved >= 10 and opened >= 30
