"""Parity of the line-search variant of the BFGS (fpt_opts.line_search =
LS_ARMIJO: backtracking from the unit step in place of the fixed-point step
of Eq. 6; a solver variant, not the paper's step) with the FP64 oracle,
through the C ABI, at the bar of the BFGS tests: no certified path more
than 1e-4 S from the oracle's minimiser, no path shorter than the minimum,
the per-path gate on at least 99 % of the paths of every order."""
import numpy as np
import pytest

import gpu_util
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


def _opts(S, **kw):
    from paper_2510_16172_amd import fpt
    return fpt.Opts(scale=S, line_search=fpt.LS_ARMIJO, **kw)


def _check(b, g, ref, min_gate=0.99):
    from paper_2510_16172_amd import fpt
    s = gpu_util.summary(b, g, ref)
    print(f"N={b.N} gate={s['frac_gate']:.4f} ok={s['frac_ok']:.4f} "
          f"cert={s['frac_cert']:.4f} falsepos={s['false_pos']}", flush=True)
    assert s["false_pos"] == 0
    assert np.all(g["len"].astype(np.float64) >= ref["len"] - 1e-6 * b.S)
    assert s["frac_gate"] >= min_gate
    assert np.all((g["status"] & (fpt.ST_INVALID | fpt.ST_NONFINITE)) == 0)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_armijo_canyon_each_order(solver, oracle_mod, n):
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 5000, seed=8300 + n, n=n)
    ref = oracle_mod.solve(b, threads=8)
    g = gpu_util.run_gpu(solver, b, _opts(b.S, iters=16), with_order=False)
    _check(b, g, ref)


def test_armijo_random_order2_64_iterations(solver, oracle_mod):
    b = scenes.random_paths(2000, 2, seed=8400)
    ref = oracle_mod.solve(b, threads=8)
    g = gpu_util.run_gpu(solver, b, _opts(b.S, iters=64), with_order=False)
    _check(b, g, ref)


def _start_length(b):
    """L at T = 0 (every point at its object's origin), FP64."""
    tx = b.pts[:, b.src].T.astype(np.float64)
    rx = b.pts[:, b.dst].T.astype(np.float64)
    P = [tx] + [b.obj[0:3, b.ids[j]].T.astype(np.float64) for j in range(b.n_max)] + [rx]
    return sum(np.linalg.norm(P[i + 1] - P[i], axis=1) for i in range(len(P) - 1))


@pytest.mark.parametrize("n", [1, 3, 6])
def test_armijo_steps_never_lengthen(solver, n):
    """Every accepted step shortens the path (Armijo's condition, else the
    majorant step, which cannot lengthen it): without the FP64 refinement,
    the FP32 phase's end point is no longer than its start, for every path."""
    sc = scenes.canyon_sample_paths(scenes.canyon_scene(), 4000, seed=8500 + n, n=n)
    g = gpu_util.run_gpu(solver, sc, _opts(sc.S, iters=6, level_eps=[], level_steps=[],
                                           polish_steps=0), with_order=False)
    L0 = _start_length(sc)
    assert np.all(np.isfinite(g["len"]))
    assert np.all(g["len"].astype(np.float64) <= L0 * (1 + 1e-6) + 1e-6 * sc.S)
    assert np.mean(g["len"] < L0 * (1 - 1e-3)) > 0.9


def test_armijo_bucketed_equals_uniform(solver):
    """Mixed orders through the order buckets give the same bits as each
    order alone, as for the Eq. 6 step."""
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 6000, seed=8600, n=None, n_max=4)
    opts = _opts(b.S, iters=12)
    g = gpu_util.run_gpu(solver, b, opts)
    for n in range(1, 5):
        idx = np.nonzero(b.order == n)[0]
        sub = b.subset(idx)
        sub = scenes.Batch(sub.obj, sub.pts, sub.src, sub.dst, sub.order,
                           np.ascontiguousarray(sub.ids[:n]), sub.S)
        gu = gpu_util.run_gpu(solver, sub, opts, with_order=False)
        np.testing.assert_array_equal(gu["x"], g["x"][:n, :, idx])
        np.testing.assert_array_equal(gu["status"], g["status"][idx])
