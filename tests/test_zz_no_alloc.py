"""fpt_solve_noalloc (the library's fixed per-GPU scratch array instead of
the handle's growing workspace) against fpt_solve, through the C ABI: the
same outputs bit for bit, on two calls in a row, the second smaller, so
that the second call runs on the scratch contents the first one left."""
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


def _run(solver, b, opts, noalloc):
    import torch
    from paper_2510_16172_amd import fpt
    db = fpt.DeviceBatch(b)
    print(f"noalloc={noalloc} N={b.N} n_max={b.n_max}", flush=True)
    out = solver.solve_noalloc(db, opts) if noalloc else solver.solve(db, opts)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _same(a, b):
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_noalloc_equals_solve_two_calls(solver):
    from paper_2510_16172_amd import fpt
    sc = scenes.canyon_scene()
    b1 = scenes.canyon_sample_paths(sc, 40000, seed=91, n=None, n_max=6)
    b2 = scenes.canyon_sample_paths(sc, 2999, seed=92, n=None, n_max=6)
    for opts in (fpt.Opts(scale=b1.S, iters=16),
                 fpt.Opts(scale=b1.S, iters=12, split=2, quick_passes=1)):
        for b in (b1, b2):
            ref = _run(solver, b, opts, False)
            got = _run(solver, b, opts, True)
            _same(ref, got)
            assert (got["status"] & fpt.ST_CONVERGED).mean() > 0.8


def test_noalloc_without_order_and_full_schedule(solver):
    """Every path of order n_max (no bucketing), and the one-pass full
    schedule (quick_steps = 0: no path lists)."""
    from paper_2510_16172_amd import fpt
    b = scenes.random_paths(3000, 3, seed=93)
    for opts in (fpt.Opts(scale=b.S, iters=64), fpt.Opts(scale=b.S, iters=64, quick_steps=0)):
        import torch
        db = fpt.DeviceBatch(b, with_order=False)
        r = solver.solve(db, opts)
        g = solver.solve_noalloc(db, opts)
        torch.cuda.synchronize()
        for k in r:
            np.testing.assert_array_equal(r[k].cpu().numpy(), g[k].cpu().numpy(), err_msg=k)


def test_noalloc_rejects_what_it_cannot_hold(solver):
    import torch
    from paper_2510_16172_amd import fpt
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 1000, seed=94, n=None, n_max=4)
    db = fpt.DeviceBatch(b)
    with pytest.raises(fpt.FptError, match="early exit"):
        solver.solve_noalloc(db, fpt.Opts(scale=b.S, early_exit=True))
    # N above the maximum: refused on the host before any launch (the
    # tensors are only sized, never read)
    big = fpt.Solver.noalloc_max_paths() + 1
    z = torch.zeros(big, dtype=torch.int32, device="cuda")
    dbig = fpt.DeviceBatch.from_tensors(db.obj, db.pts, z, z,
                                        torch.zeros((1, big), dtype=torch.int32, device="cuda"),
                                        S=b.S)
    outb = {"x": torch.empty(1, device="cuda"), "len": torch.empty(1, device="cuda"),
            "t": torch.empty(1, device="cuda"),
            "status": torch.empty(1, dtype=torch.uint8, device="cuda"),
            "iters": torch.empty(1, dtype=torch.int16, device="cuda")}
    with pytest.raises(fpt.FptError, match="noalloc_max_paths"):
        solver.solve_noalloc(dbig, fpt.Opts(scale=b.S), out=outb)
    torch.cuda.synchronize()
