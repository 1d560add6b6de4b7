"""Parity of the FP32 exact-Hessian Newton variant of the first phase
(fpt_opts.method = METHOD_NEWTON32, a solver variant, not the paper's BFGS)
with the FP64 oracle, through the C ABI. The bar is the solver's: no path
it certifies is more than 1e-4 S from the oracle's minimiser, no path is
shorter than the minimum, and the fraction within 1e-4 S reaches the level
the variant attains at each order (printed)."""
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
    return fpt.Opts(scale=S, method=fpt.METHOD_NEWTON32, **kw)


def _check(b, g, ref, min_cert, min_gate=0.99):
    """No certified path wrong, no path shorter than the minimum, and the
    per-path gate of the BFGS tests (points for smooth unique minimisers,
    length for collapsed ones) on min_gate of the paths."""
    from paper_2510_16172_amd import fpt
    s = gpu_util.summary(b, g, ref)
    print(f"N={b.N} gate={s['frac_gate']:.4f} ok={s['frac_ok']:.4f} "
          f"cert={s['frac_cert']:.4f} falsepos={s['false_pos']}", flush=True)
    assert s["false_pos"] == 0
    assert np.all(g["len"].astype(np.float64) >= ref["len"] - 1e-6 * b.S)
    assert s["frac_gate"] >= min_gate and s["frac_cert"] >= min_cert
    assert np.all((g["status"] & (fpt.ST_INVALID | fpt.ST_NONFINITE)) == 0)
    return s


# The variant reaches the parity bar of the BFGS with 32 FP32 Newton steps
# (8 per smoothing level); with 8 steps, where its certified paths/s is
# highest, up to 5 % of the order-6 paths end neither certified nor within
# the gate (the FP64 refinement does not recover a start point left at a
# spurious near-collapse).
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_newton32_random_each_order(solver, oracle_mod, n):
    # 2,000 paths: several workgroups and a ragged tail
    b = scenes.random_paths(2000, n, seed=8100 + n)
    ref = oracle_mod.solve(b, threads=8)
    g = gpu_util.run_gpu(solver, b, _opts(b.S, iters=32), with_order=False)
    _check(b, g, ref, min_cert=0.95)
    assert np.all(g["iters"] == 32)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_newton32_canyon_each_order(solver, oracle_mod, n):
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 5000, seed=8200 + n, n=n)
    ref = oracle_mod.solve(b, threads=8)
    g = gpu_util.run_gpu(solver, b, _opts(b.S, iters=32), with_order=False)
    _check(b, g, ref, min_cert=0.95)


def test_newton32_eight_steps_no_certified_path_wrong(solver, oracle_mod):
    """At its fastest setting (8 steps) the variant certifies fewer paths,
    but none of them wrongly, and no path is shorter than the minimum."""
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 5000, seed=8206, n=6)
    ref = oracle_mod.solve(b, threads=8)
    g = gpu_util.run_gpu(solver, b, _opts(b.S, iters=8), with_order=False)
    _check(b, g, ref, min_cert=0.9, min_gate=0.9)


def test_newton32_and_bfgs_agree_where_both_certify(solver):
    """The minimiser is unique (L is convex): where both first phases lead
    to a certificate the points agree within 2e-4 S."""
    from paper_2510_16172_amd import fpt
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 20000, seed=8300, n=3)
    gn = gpu_util.run_gpu(solver, b, _opts(b.S, iters=8), with_order=False)
    gb = gpu_util.run_gpu(solver, b, fpt.Opts(scale=b.S, iters=24), with_order=False)
    both = ((gn["status"] & gb["status"]) & fpt.ST_CONVERGED) != 0
    assert both.mean() > 0.8
    d = np.linalg.norm(gn["x"].astype(np.float64) - gb["x"], axis=1).max(axis=0) / b.S
    assert np.all(d[both] <= 2e-4)


def test_newton32_mixed_orders_bucketed_equals_uniform(solver):
    """Through the order buckets each order gives the same bits as a batch
    of that order alone."""
    from paper_2510_16172_amd import fpt
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 6000, seed=8400, n=None, n_max=4)
    g = gpu_util.run_gpu(solver, b, _opts(b.S, iters=8))
    for n in range(1, 5):
        idx = np.nonzero(b.order == n)[0]
        sub = b.subset(idx)
        sub = type(sub)(sub.obj, sub.pts, sub.src, sub.dst, sub.order,
                        np.ascontiguousarray(sub.ids[:n]), sub.S, sub.meta)
        gu = gpu_util.run_gpu(solver, sub, _opts(b.S, iters=8), with_order=False)
        np.testing.assert_array_equal(g["x"][:n, :, idx], gu["x"])
        np.testing.assert_array_equal(g["status"][idx], gu["status"])
    assert fpt.METHOD_NEWTON32 == 1


def test_newton32_rejects_early_exit(solver):
    from paper_2510_16172_amd import fpt
    b = scenes.random_paths(64, 2, seed=8500)
    with pytest.raises(fpt.FptError):
        gpu_util.run_gpu(solver, b, _opts(b.S, iters=8, early_exit=True), with_order=False)


def test_newton32_two_parts_equal_one(solver):
    """The FP32 Newton first phase with each order's paths in two parts on
    their own streams (the first phase then clears the refinement's list
    counters, and the second part takes the orders from the top down) gives
    the same bits as one part."""
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 30001, seed=8600, n=None, n_max=4)
    one = gpu_util.run_gpu(solver, b, _opts(b.S, iters=8, split=1))
    two = gpu_util.run_gpu(solver, b, _opts(b.S, iters=8, split=2))
    for key in one:
        np.testing.assert_array_equal(two[key], one[key], err_msg=key)
