"""Fermat path oracle: TEST INFRASTRUCTURE ONLY.

Plain FP64 CPU reference for the path-length minimisation of Sec. III-B
(Eqs. 1-5) and the implicit-differentiation gradient of Sec. III-D
(Eqs. 8-13), in ``fermat_oracle.c``. Only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark may import this package; the product
path (the HIP library and its binding) never does, and the two share no code.

The oracle's own pins (image method, single-edge closed form, brute force,
invariants, finite differences) live in ``tests/``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfermat_oracle.so")
SOURCES = [os.path.join(HERE, "fermat_oracle.c")]

COLLAPSED, ILL, NOCONV, INVALID, KKT = 1, 2, 4, 8, 16
EXTENT, SPECULAR, VISIBLE = 1, 2, 4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, strict IEEE: no fast-math)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11",
           "-fno-fast-math", "-ffp-contract=off", "-Wall", "-Wextra",
           "-o", tmp] + SOURCES + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        I64, I32, D = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        lib.oracle_solve.argtypes = [I64, I32, P, I64, P, I64, P, P, P, P, D,
                                     P, P, P, P, P, I32]
        lib.oracle_solve.restype = I32
        lib.oracle_grad.argtypes = [I64, I32, P, I64, P, I64, P, P, P, P, D,
                                    P, P, P, P, P, P, P, P, I32]
        lib.oracle_grad.restype = I32
        lib.oracle_length.argtypes = [I64, I32, P, I64, P, I64, P, P, P, P, P,
                                      P]
        lib.oracle_length.restype = I32
        lib.oracle_validate.argtypes = [I64, I32, P, I64, P, I64, P, P, P, P,
                                        D, P, P, D, P, I32]
        lib.oracle_validate.restype = I32
        _lib = lib
    return _lib


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data


def _tables(b):
    obj, po = _c(b.obj, np.float32)
    pts, pp = _c(b.pts, np.float32)
    src, ps = _c(b.src, np.int32)
    dst, pd = _c(b.dst, np.int32)
    order, pn = _c(b.order, np.uint8)
    ids, pi = _c(b.ids, np.int32)
    keep = (obj, pts, src, dst, order, ids)
    return keep, (po, obj.shape[1], pp, pts.shape[1], ps, pd, pn, pi)


def solve(b, threads: int = 0):
    """Solve every path of a :class:`scenes.Batch`. Returns a dict with
    ``x [N][n_max][3]``, ``len [N]``, ``t [N][n_max][2]`` (float64),
    ``flags [N]`` and ``iters [N]`` (int32)."""
    lib = _load()
    N, n_max = b.N, b.n_max
    x = np.empty((N, n_max, 3))
    ln = np.empty(N)
    t = np.empty((N, n_max, 2))
    fl = np.empty(N, np.int32)
    it = np.empty(N, np.int32)
    keep, (po, K, pp, Q, ps, pd, pn, pi) = _tables(b)
    rc = lib.oracle_solve(N, n_max, po, K, pp, Q, ps, pd, pn, pi, float(b.S),
                          x.ctypes.data, ln.ctypes.data, t.ctypes.data,
                          fl.ctypes.data, it.ctypes.data, int(threads))
    if rc != 0:
        raise ValueError("oracle_solve rejected the sizes")
    del keep
    return dict(x=x, len=ln, t=t, flags=fl, iters=it)


def grad(b, t_sol, g_len, g_x, threads: int = 0):
    """IFT gradient at solution ``t_sol [N][n_max][2]``.

    ``g_len [N]`` and ``g_x [N][n_max][3]`` are the upstream cotangents.
    Returns per-path ``g_tx, g_rx [N][3]``, ``g_b [N][n_max][3]``,
    ``g_a [N][n_max][2][3]`` and ``status [N]``: 0 at a smooth minimiser,
    KKT at a minimiser with one interior zero-length segment (the IFT on the
    collapse constraint's KKT conditions), COLLAPSED where neither applies
    (outputs NaN)."""
    lib = _load()
    N, n_max = b.N, b.n_max
    t_sol = np.ascontiguousarray(t_sol, np.float64)
    g_len = np.ascontiguousarray(g_len, np.float64)
    g_x = np.ascontiguousarray(g_x, np.float64)
    assert t_sol.shape == (N, n_max, 2) and g_len.shape == (N,)
    assert g_x.shape == (N, n_max, 3)
    g_tx = np.empty((N, 3))
    g_rx = np.empty((N, 3))
    g_b = np.empty((N, n_max, 3))
    g_a = np.empty((N, n_max, 2, 3))
    st = np.empty(N, np.int32)
    keep, (po, K, pp, Q, ps, pd, pn, pi) = _tables(b)
    rc = lib.oracle_grad(N, n_max, po, K, pp, Q, ps, pd, pn, pi, float(b.S),
                         t_sol.ctypes.data, g_len.ctypes.data,
                         g_x.ctypes.data, g_tx.ctypes.data, g_rx.ctypes.data,
                         g_b.ctypes.data, g_a.ctypes.data, st.ctypes.data,
                         int(threads))
    if rc != 0:
        raise ValueError("oracle_grad rejected the sizes")
    del keep
    return dict(g_tx=g_tx, g_rx=g_rx, g_b=g_b, g_a=g_a, status=st)


def length(b, t):
    """L(T) (Eq. 5) in FP64 at parameters ``t [N][n_max][2]``."""
    lib = _load()
    t = np.ascontiguousarray(t, np.float64)
    assert t.shape == (b.N, b.n_max, 2)
    out = np.empty(b.N)
    keep, (po, K, pp, Q, ps, pd, pn, pi) = _tables(b)
    rc = lib.oracle_length(b.N, b.n_max, po, K, pp, Q, ps, pd, pn, pi,
                           t.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_length rejected the sizes")
    del keep
    return out


def validate(b, t, x, tol: float = 0.0, threads: int = 0):
    """Validity bits (EXTENT, SPECULAR, VISIBLE) of solved paths on the finite
    objects of the scene, for parameters ``t [N][n_max][2]`` and points
    ``x [N][n_max][3]``; ``tol`` widens (> 0) or narrows the tests (see
    ``fermat_oracle.c``)."""
    lib = _load()
    t = np.ascontiguousarray(t, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    assert t.shape == (b.N, b.n_max, 2) and x.shape == (b.N, b.n_max, 3)
    out = np.empty(b.N, np.uint8)
    keep, (po, K, pp, Q, ps, pd, pn, pi) = _tables(b)
    rc = lib.oracle_validate(b.N, b.n_max, po, K, pp, Q, ps, pd, pn, pi,
                             float(b.S), t.ctypes.data, x.ctypes.data,
                             float(tol), out.ctypes.data, int(threads))
    if rc != 0:
        raise ValueError("oracle_validate rejected the sizes")
    del keep
    return out
