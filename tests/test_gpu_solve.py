"""Parity of the HIP solver (through the C ABI) with the FP64 oracle.

Tolerance: interaction points within 1e-4 of the scene size S (the accuracy
bar the solver is built for). A path the kernel certifies (FPT_ST_CONVERGED)
must meet it. Every path is held to the per-path gate: points within 1e-4 S
where the oracle's minimiser is unique and smooth, length within 1e-5 S where
it is collapsed (coinciding interaction points) or not unique (ILL); at least
99 % of the paths of every order must pass it, and no path may be shorter
than the minimum.
"""
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
    return fpt.Opts(scale=S, **kw)


def _check_common(b, g, ref, min_gate=0.99, rtol=1e-4):
    s = gpu_util.summary(b, g, ref, rtol)
    col = s["col"]
    print(f"N={b.N} gate={s['frac_gate']:.4f} ok={s['frac_ok']:.4f} "
          f"cert={s['frac_cert']:.4f} falsepos={s['false_pos']} "
          f"collapsed={col.mean():.3f} gate-miss smooth={(~s['gate'] & ~col).mean():.4f} "
          f"collapsed={(~s['gate'] & col).mean():.4f}", flush=True)
    # no certified path is wrong
    assert s["false_pos"] == 0
    # no path is shorter than the minimum (beyond FP32 rounding of L)
    Lg = g["len"].astype(np.float64)
    assert np.all(Lg >= ref["len"] - 1e-6 * b.S)
    # the per-path gate: points (smooth unique minimisers), length
    # (collapsed or non-unique ones)
    assert s["frac_gate"] >= min_gate
    ill = s["ill"]
    if ill.any():
        assert np.all(np.abs(Lg[ill] - ref["len"][ill]) <= 1e-5 * b.S)
    # lengths of converged paths: moving each point by at most e changes
    # every segment by at most 2e, so |dL| <= 2 (n+1) e (+ FP32 rounding)
    ok = s["ok"]
    bound = 2.0 * (b.order[ok].astype(np.float64) + 1) * s["err"][ok] * b.S
    assert np.all(np.abs(Lg[ok] - ref["len"][ok]) <= bound + 2e-6 * b.S)
    # status bits
    from paper_2510_16172_amd import fpt
    assert np.all((g["status"] & fpt.ST_INVALID) == 0)
    assert np.all((g["status"] & fpt.ST_NONFINITE) == 0)
    return s


def test_random_order2_64_iterations(solver, oracle_mod):
    """1,024 random order-2 paths, reflection or diffraction with p = 0.5,
    64 fixed iterations, FP32 + FP64 refinement vs the FP64 oracle."""
    b = scenes.random_paths(1024, 2, seed=1001)
    ref = oracle_mod.solve(b, threads=8)
    g = gpu_util.run_gpu(solver, b, _opts(b.S, iters=64), with_order=False)
    s = _check_common(b, g, ref)
    assert np.all(g["iters"] == 64)
    assert s["frac_cert"] >= 0.8


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_random_each_order(solver, oracle_mod, n):
    # 2,000 paths: several 256-path workgroups and a ragged tail
    b = scenes.random_paths(2000, n, seed=3000 + n)
    ref = oracle_mod.solve(b, threads=8)
    g = gpu_util.run_gpu(solver, b, _opts(b.S, iters=128), with_order=False)
    _check_common(b, g, ref)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_canyon_each_order(solver, oracle_mod, n):
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 3000, seed=4000 + n, n=n)
    ref = oracle_mod.solve(b, threads=8)
    g = gpu_util.run_gpu(solver, b, _opts(b.S, iters=128))
    _check_common(b, g, ref)


def test_mixed_orders_bucketed_equals_uniform(solver):
    """Paths of orders 1..6 in one call (device-side bucketing by order) give
    bit-identical results to the same paths solved order by order."""
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 5000, seed=77, n=None, n_max=6)
    opts = _opts(b.S, iters=48)
    g = gpu_util.run_gpu(solver, b, opts)
    for n in range(1, 7):
        idx = np.nonzero(b.order == n)[0]
        if len(idx) == 0:
            continue
        sub = b.subset(idx)
        sub = scenes.Batch(sub.obj, sub.pts, sub.src, sub.dst, sub.order,
                           np.ascontiguousarray(sub.ids[:n]), sub.S)
        gu = gpu_util.run_gpu(solver, sub, opts, with_order=False)
        np.testing.assert_array_equal(gu["x"], g["x"][:n, :, idx])
        np.testing.assert_array_equal(gu["len"], g["len"][idx])
        np.testing.assert_array_equal(gu["status"], g["status"][idx])
        assert np.all(np.isnan(g["x"][n:, :, idx]))


def test_deterministic(solver):
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 4096, seed=78, n=None, n_max=6)
    opts = _opts(b.S, iters=32)
    g1 = gpu_util.run_gpu(solver, b, opts)
    g2 = gpu_util.run_gpu(solver, b, opts)
    for k in g1:
        np.testing.assert_array_equal(g1[k], g2[k])


def test_invalid_paths_and_edge_cases(solver):
    import torch
    from paper_2510_16172_amd import fpt
    b = scenes.random_paths(300, 3, seed=79)
    order = b.order.copy()
    ids = b.ids.copy()
    src = b.src.copy()
    obj = b.obj.copy()
    order[0] = 0            # order below 1
    order[1] = 7            # order above n_max
    ids[1, 2] = b.K + 5     # id out of range
    ids[0, 3] = -2          # negative id
    src[4] = b.Q            # point index out of range
    obj[0, ids[2, 5]] = np.nan  # non-finite geometry
    obj[3:6, ids[1, 6]] = 0.0   # zero first basis vector
    order[7] = 2            # a valid shorter path inside the n_max=3 batch
    bad = scenes.Batch(obj, b.pts, src, b.dst, order, ids, b.S)
    g = gpu_util.run_gpu(solver, bad, _opts(b.S, iters=64))
    for i in range(7):
        assert g["status"][i] == fpt.ST_INVALID | fpt.ST_NOGRAD, i
        assert np.all(np.isnan(g["x"][:, :, i])) and np.isnan(g["len"][i])
    assert g["status"][7] & fpt.ST_INVALID == 0
    assert np.all(np.isfinite(g["x"][:2, :, 7])) and np.all(np.isnan(g["x"][2, :, 7]))
    assert np.all(g["status"][8:] & fpt.ST_INVALID == 0)
    # N = 0: accepted, nothing launched
    empty = b.subset(np.zeros(0, np.int64))
    db = fpt.DeviceBatch(empty)
    solver.solve(db, _opts(b.S))
    torch.cuda.synchronize()
    # whole-call errors launch nothing and raise
    db = fpt.DeviceBatch(b)
    with pytest.raises(fpt.FptError):
        solver.solve(db, _opts(-1.0))
    with pytest.raises(fpt.FptError):
        solver.solve(db, _opts(b.S, iters=-1))


def test_warm_start_from_oracle(solver, oracle_mod):
    """Starting at the oracle's T*, zero BFGS iterations and the refinement
    keep the solution and certify every smooth path."""
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 2000, seed=80, n=3)
    ref = oracle_mod.solve(b, threads=8)
    t0 = np.transpose(ref["t"], (1, 2, 0))  # n, 2, N
    g = gpu_util.run_gpu(solver, b, _opts(b.S, iters=0), t_init=t0)
    s = gpu_util.summary(b, g, ref)
    smooth = ~s["col"] & ~s["ill"]
    assert s["ok"][smooth].all()
    assert s["cert"][smooth].mean() > 0.99
    assert s["false_pos"] == 0


def test_full_canyon_order2_sampled(solver, oracle_mod):
    """All 6,270,016 sequences of order <= 2 in the canyon (the benchmark
    workload and launch): 8,192 sampled paths against the oracle, and
    properties that hold on every path."""
    import torch
    from paper_2510_16172_amd import fpt
    sc = scenes.canyon_scene()
    b = scenes.canyon_all_paths(sc, n_max=2)
    assert b.N == 6_270_016
    opts = _opts(b.S, iters=64)
    db = fpt.DeviceBatch(b)
    out = solver.solve(db, opts)
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    L = out["len"].cpu().numpy().astype(np.float64)
    assert np.all(st & (fpt.ST_INVALID | fpt.ST_NONFINITE) == 0)
    direct = np.linalg.norm(b.pts[:, b.dst] - b.pts[:, b.src], axis=0)
    assert np.all(L >= direct * (1 - 1e-6))
    cert = (st & fpt.ST_CONVERGED) != 0
    print(f"certified {cert.mean():.4f}", flush=True)
    rng = np.random.default_rng(81)
    idx = np.sort(rng.choice(b.N, 8192, replace=False))
    sub = b.subset(idx)
    ref = oracle_mod.solve(sub, threads=8)
    g = {k: (v.cpu().numpy()[..., idx] if v.dim() > 1 else v.cpu().numpy()[idx])
         for k, v in out.items()}
    _check_common(sub, g, ref)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_early_exit_stages_parity(solver, oracle_mod, n):
    """Early exit in stages: a path stops after two small steps, the others
    are compacted for the next stage; same accuracy bar as fixed counts."""
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 3000, seed=4100 + n, n=n)
    ref = oracle_mod.solve(b, threads=8)
    g = gpu_util.run_gpu(solver, b, _opts(b.S, iters=128, early_exit=True))
    _check_common(b, g, ref)
    it = g["iters"].astype(np.int64)
    assert it.max() <= 128 and it.min() >= 1
    print(f"mean iterations {it.mean():.1f}", flush=True)
    assert it.mean() < 100


def test_early_exit_deterministic_and_mixed(solver):
    """Which list slot holds a path depends on timing, the path's arithmetic
    does not: two runs are bit-identical, also with mixed orders, ragged
    buckets and four stages."""
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 9999, seed=4200, n=None, n_max=6)
    opts = _opts(b.S, iters=96, early_exit=True, stage_iters=[8, 8, 16, 64])
    g1 = gpu_util.run_gpu(solver, b, opts)
    g2 = gpu_util.run_gpu(solver, b, opts)
    for k in g1:
        np.testing.assert_array_equal(g1[k], g2[k])
    from paper_2510_16172_amd import fpt
    assert np.all(g1["status"] & (fpt.ST_INVALID | fpt.ST_NONFINITE) == 0)


def test_graph_capture_replays_match_eager(solver):
    """A captured fpt_solve (bucketing + persistent per-order launches with
    early exit + refinement) replayed several times, with other work and
    synchronisations in between, gives the eager result every time."""
    import torch
    from paper_2510_16172_amd import fpt
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 20000, seed=4300, n=None, n_max=6)
    opts = _opts(b.S, iters=64, early_exit=True)
    db = fpt.DeviceBatch(b)
    eager = solver.solve(db, opts)
    torch.cuda.synchronize()
    eager = {k: v.cpu().numpy() for k, v in eager.items()}
    st = torch.cuda.Stream()
    out = solver.alloc_out(db)
    with torch.cuda.stream(st):
        graph = solver.capture(db, opts, out, st)
    for rep in range(3):
        for v in out.values():
            v.zero_()
        torch.cuda.synchronize()
        graph.launch(st)
        st.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
        for k in eager:
            np.testing.assert_array_equal(got[k], eager[k], err_msg=f"replay {rep} {k}")
        # unrelated eager work between replays
        solver.solve(fpt.DeviceBatch(b.subset(np.arange(100))), opts)
        torch.cuda.synchronize()
    graph.close()


def test_autotuner_choices_keep_parity(solver, oracle_mod, tmp_path):
    from paper_2510_16172_amd import autotune
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 12000, seed=4400, n=None, n_max=3)
    opts = _opts(b.S, iters=64)
    chosen = autotune.tune(solver, b, opts, sample=4096, repeats=2,
                           cache_path=str(tmp_path / "tune.json"))
    assert set(chosen) == {1, 2, 3}
    ref = oracle_mod.solve(b, threads=8)
    g = gpu_util.run_gpu(solver, b, opts)
    _check_common(b, g, ref)
    for n in (1, 2, 3):
        solver.set_launch(n, None)


def test_launch_iters_override_matches_opts(solver):
    """A per-order iteration count set with fpt_set_launch gives the same
    result as the same count in fpt_opts."""
    from paper_2510_16172_amd import fpt
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 20000, seed=4500, n=None, n_max=3)
    want = gpu_util.run_gpu(solver, b, _opts(b.S, iters=12))
    for n in (1, 2, 3):
        solver.set_launch(n, {"iters": 12})
    try:
        got = gpu_util.run_gpu(solver, b, _opts(b.S, iters=64))
    finally:
        for n in (1, 2, 3):
            solver.set_launch(n, None)
    for k in want:
        np.testing.assert_array_equal(got[k], want[k], err_msg=k)
    with pytest.raises(fpt.FptError):
        solver.set_launch(2, {"iters": -1})


def test_refine_work_counts(solver):
    """The refinement's evaluation / Newton-solve counters: every path of an
    order starts one level and takes at least quick_steps solves; nothing is
    counted while timing is off."""
    import torch
    from paper_2510_16172_amd import fpt
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 30000, seed=4600, n=None, n_max=3)
    opts = _opts(b.S, iters=16)
    db = fpt.DeviceBatch(b)
    solver.set_timing(True)
    solver.work_counts()
    out = solver.solve(db, opts)
    torch.cuda.synchronize()
    wc = solver.work_counts()
    solver.kernel_times()
    solver.set_timing(False)
    total_levels = sum(opts.level_steps)
    for n in (1, 2, 3):
        cnt = int((b.order == n).sum())
        ev, tr, so, mev, mtr, mso = wc[n]
        assert so >= opts.quick_steps * cnt
        assert so <= (opts.quick_passes * opts.quick_steps + total_levels) * cnt
        # one evaluation at the start of each Newton run (one run per quick
        # pass and per level of the full schedule) plus one per solve that
        # succeeds but the run's last; one trial at least per such solve, at
        # most 7
        runs = opts.quick_passes + len(opts.level_eps)
        if n == 1:
            # one slot: every trial is a full evaluation
            assert tr == 0 and cnt <= ev <= 7 * so + runs * cnt
        else:
            assert cnt <= ev <= so + runs * cnt
            assert so // 2 <= tr <= 7 * so
        if n == 1:
            assert (mev, mtr, mso) == (0, 0, 0)
        assert mso <= 5 * cnt and mev <= 5 * 10 * cnt and mtr <= 7 * mso
    assert wc[4] == (0,) * 6
    solver.solve(db, opts, out=out)
    torch.cuda.synchronize()
    assert all(v == (0,) * 6 for v in solver.work_counts().values())


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_collapsed_minimisers_certified(solver, oracle_mod, n):
    """Minimisers where consecutive interaction points coincide (the
    oracle's COLLAPSED flag), with one collapse or several, and runs of three
    coinciding points: the collapse step certifies most of them, every
    certified one lies within 1e-4 S of the oracle and carries the
    COLLAPSED status."""
    from paper_2510_16172_amd import fpt
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 6000, seed=4700 + n, n=n)
    ref = oracle_mod.solve(b, threads=8)
    g = gpu_util.run_gpu(solver, b, _opts(b.S, iters=16), with_order=False)
    s = _check_common(b, g, ref)
    col = s["col"] & ~s["ill"]
    cc = s["cert"] & col
    runs, longest = gpu_util.zero_runs(b, ref)
    multi = col & ((runs > 1) | (longest > 1))
    cm = s["cert"] & multi
    print(f"n={n} collapsed={col.sum()} certified={cc.sum()} "
          f"several collapses or a run of three={multi.sum()} certified={cm.sum()}",
          flush=True)
    assert col.sum() > 300
    assert cc.sum() >= 0.95 * col.sum()
    if n >= 4:
        assert multi.sum() > 50
        assert cm.sum() >= 0.9 * multi.sum()
    assert np.all((g["status"][cc] & fpt.ST_COLLAPSED) != 0)


def test_concurrent_orders_equal_sequential(solver):
    """Each order on its own stream gives the same result as the orders one
    after the other (eager and through a captured graph)."""
    import torch
    from paper_2510_16172_amd import fpt
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 30000, seed=4800, n=None, n_max=6)
    want = gpu_util.run_gpu(solver, b, _opts(b.S, iters=16))
    got = gpu_util.run_gpu(solver, b, _opts(b.S, iters=16, concurrent_orders=True))
    for k in want:
        np.testing.assert_array_equal(got[k], want[k], err_msg=k)
    db = fpt.DeviceBatch(b)
    opts = _opts(b.S, iters=16, concurrent_orders=True)
    out = solver.alloc_out(db)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        g = solver.capture(db, opts, out, st)
        for _ in range(2):
            g.launch(st)
            st.synchronize()
            rep = {k: v.cpu().numpy() for k, v in out.items()}
            for k in want:
                np.testing.assert_array_equal(rep[k], want[k], err_msg=k)
    g.close()


def test_warm_start_in_place(solver):
    """t_init may be the output t itself (a warm start from the previous
    solve's result, overwritten in place): the same bits as the same start
    from a separate buffer, one order after another and with concurrent
    orders, and NaN in t beyond each path's order."""
    import torch
    from paper_2510_16172_amd import fpt
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 20000, seed=4900, n=None, n_max=5)
    for conc in (False, True):
        opts = _opts(b.S, iters=8, concurrent_orders=conc)
        db = fpt.DeviceBatch(b)
        out = solver.solve(db, opts)
        db.t_init = out["t"].clone()
        want = {k: v.cpu().numpy() for k, v in solver.solve(db, opts).items()}
        db.t_init = out["t"]
        solver.solve(db, opts, out=out)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
        for k in want:
            np.testing.assert_array_equal(got[k], want[k], err_msg=k)
        for n in range(1, 5):
            assert np.all(np.isnan(got["t"][n:, :, b.order == n]))
            assert np.all(np.isnan(want["x"][n:, :, b.order == n]))


@pytest.mark.parametrize("n", [1, 2])
def test_unpadded_edge_paths_match_padded(solver, oracle_mod, n):
    """Paths whose every interaction is an edge run the BFGS on n parameters
    when a whole wave of them comes together, else in the padded layout; the
    padded rows stay exactly 0, so both compute the same iterates (to FP32
    rounding), and after the FP64 refinement the same bits. Edge-only paths
    alone (every wave unpadded) against the same paths spread one in six
    among face paths (no wave of 64 edge-only paths), and the oracle."""
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 150000, seed=5100 + n, n=n)
    edge = np.all(b.obj[6:9] == 0, axis=0)
    eo = np.all(edge[b.ids[:n]], axis=0)
    face = np.all(~edge[b.ids[:n]], axis=0)
    E = np.nonzero(eo)[0][:3000]
    F = np.nonzero(face)[0][:5 * len(E)]
    assert len(E) == 3000 and len(F) == 5 * len(E)
    mix = np.empty(6 * len(E), np.int64)
    mix[0::6] = E
    for r in range(5):
        mix[r + 1::6] = F[r::5]
    opts = _opts(b.S, iters=10)
    ge = gpu_util.run_gpu(solver, b.subset(E), opts, with_order=False)
    gm = gpu_util.run_gpu(solver, b.subset(mix), opts, with_order=False)
    for k in ge:
        np.testing.assert_array_equal(ge[k], gm[k][..., 0::6], err_msg=k)
    sub = b.subset(E[:1000])
    ref = oracle_mod.solve(sub)
    g1 = {k: v[..., :1000] for k, v in ge.items()}
    _check_common(sub, g1, ref)


def test_bucketing_ragged_unaligned_and_invalid_orders(solver):
    """Order bucketing over a ragged size (three chunks of 8,192 paths and a
    tail) with an order array that starts off 16-byte alignment (the
    per-byte load path) and invalid orders: the same bits as with an aligned
    order array, and the invalid paths flagged."""
    import torch
    from paper_2510_16172_amd import fpt
    sc = scenes.canyon_scene()
    N = 3 * 8192 + 77
    b = scenes.canyon_sample_paths(sc, N, seed=4700, n=None, n_max=4)
    order = b.order.copy()
    order[::97] = 0
    order[5::101] = 9
    bad = (order < 1) | (order > 4)
    db = fpt.DeviceBatch(b)
    big = torch.zeros(N + 16, dtype=torch.uint8, device="cuda")
    big[1:N + 1] = torch.from_numpy(order).cuda()
    un = fpt.DeviceBatch.from_tensors(db.obj, db.pts, db.src, db.dst, db.ids,
                                      big[1:N + 1], S=b.S)
    al = fpt.DeviceBatch.from_tensors(db.obj, db.pts, db.src, db.dst, db.ids,
                                      torch.from_numpy(order).cuda(), S=b.S)
    assert un.order.data_ptr() % 16 == 1
    opts = _opts(b.S, iters=16)
    gu = {k: v.cpu().numpy() for k, v in solver.solve(un, opts).items()}
    ga = {k: v.cpu().numpy() for k, v in solver.solve(al, opts).items()}
    for k in ga:
        np.testing.assert_array_equal(gu[k], ga[k], err_msg=k)
    assert np.all((ga["status"][bad] & fpt.ST_INVALID) != 0)
    assert np.all((ga["status"][~bad] & fpt.ST_INVALID) == 0)
    assert ((ga["status"][~bad] & fpt.ST_CONVERGED) != 0).mean() > 0.85


def test_no_certificate_at_nonstationary_collapse(solver, oracle_mod):
    """Three order-2 canyon paths whose iterates end on the intersection line
    of their two walls, which is not where the minimum is (the oracle's path
    is 6.6e-6 m to 8 cm shorter). The smoothed length is curved like 1 / eps
    there, so the Newton steps are tiny; the certificate must not accept them
    (the exact subgradient test rejects them: |w| > 1). Under the schedules
    that led them there (BFGS with 16 iterations and 3 quick steps; the FP32
    Newton variant with 8 steps and 2 quick steps), no certified path may be
    more than 1e-4 S from the oracle."""
    from paper_2510_16172_amd import fpt
    sc = scenes.canyon_scene()
    full = scenes.canyon_all_paths(sc, n_max=2)
    idx = np.array([1508927, 3696120, 5793027])
    rng = np.random.default_rng(4800)
    idx = np.sort(np.concatenate([idx, rng.choice(np.nonzero(full.order == 2)[0], 509, replace=False)]))
    b = full.subset(idx)
    b = type(b)(b.obj, b.pts, b.src, b.dst, b.order, np.ascontiguousarray(b.ids[:2]), b.S, b.meta)
    ref = oracle_mod.solve(b, threads=8)
    for method, iters, qs in ((fpt.METHOD_BFGS, 16, 3), (fpt.METHOD_NEWTON32, 8, 2)):
        g = gpu_util.run_gpu(solver, b, _opts(b.S, iters=iters, quick_steps=qs, quick_passes=1,
                                              method=method), with_order=False)
        s = gpu_util.summary(b, g, ref)
        print(f"method {method}: cert {s['frac_cert']:.4f} ok {s['frac_ok']:.4f}", flush=True)
        assert s["false_pos"] == 0
        assert s["frac_cert"] > 0.9


@pytest.mark.parametrize("with_order", [True, False])
def test_split_parts_equal_one_part(solver, with_order):
    """Solving each order in 2, 3 or 4 parts on their own streams gives the
    same bits as one part (ragged sizes: the parts differ by one path)."""
    from paper_2510_16172_amd import fpt
    sc = scenes.canyon_scene()
    if with_order:
        b = scenes.canyon_sample_paths(sc, 50001, seed=4900, n=None, n_max=4)
    else:
        b = scenes.canyon_sample_paths(sc, 30001, seed=4901, n=3)
    ref = gpu_util.run_gpu(solver, b, _opts(b.S, iters=10, split=1), with_order=with_order)
    for k in (2, 3, 4):
        g = gpu_util.run_gpu(solver, b, _opts(b.S, iters=10, split=k), with_order=with_order)
        for key in ref:
            np.testing.assert_array_equal(g[key], ref[key], err_msg=f"split {k} {key}")


def test_split_graph_replays_match_eager(solver):
    """A captured solve in 2 parts per order (streams forked and joined
    inside the graph) replays to the same bits as the eager solve."""
    import torch
    from paper_2510_16172_amd import fpt
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 40000, seed=4902, n=None, n_max=3)
    opts = _opts(b.S, iters=10, split=2)
    db = fpt.DeviceBatch(b)
    eager = {k: v.cpu().numpy() for k, v in solver.solve(db, opts).items()}
    out = solver.alloc_out(db)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        g = solver.capture(db, opts, out, st)
    try:
        for _ in range(3):
            for v in out.values():
                v.zero_()
            torch.cuda.synchronize()
            g.launch(st)
            st.synchronize()
            for k in eager:
                np.testing.assert_array_equal(out[k].cpu().numpy(), eager[k], err_msg=k)
    finally:
        g.close()


@pytest.mark.parametrize("polish", [0, 2])
def test_polish_steps_keep_parity(solver, oracle_mod, polish):
    """No FP32 polish step, or two: the certificate and the parity bar hold
    (the polish step only moves where the FP64 refinement starts)."""
    b = scenes.random_paths(2000, 3, seed=5000 + polish)
    ref = oracle_mod.solve(b, threads=8)
    g = gpu_util.run_gpu(solver, b, _opts(b.S, iters=24, polish_steps=polish), with_order=False)
    _check_common(b, g, ref)


@pytest.mark.parametrize("variant", ["one_pass", "no_refinement", "concurrent"])
def test_split_variants_equal_one_part(solver, variant):
    """Parts on their own streams with the refinement as one full pass (no
    lists), with no refinement at all, and together with one stream per
    order: the same bits as one part on the caller's stream."""
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 30001, seed=5100, n=None, n_max=5)
    kw = {"iters": 12}
    if variant == "one_pass":
        kw["quick_steps"] = 0
    elif variant == "no_refinement":
        kw["level_eps"], kw["level_steps"] = [], []
    ref = gpu_util.run_gpu(solver, b, _opts(b.S, split=1, **kw))
    g = gpu_util.run_gpu(solver, b, _opts(b.S, split=2,
                                          concurrent_orders=(variant == "concurrent"), **kw))
    for key in ref:
        if variant == "no_refinement" and key in ("x", "t", "len"):
            # the raw FP32 phase: an edge-only path of order <= 2 may run
            # unpadded in one split and padded in the other (a workgroup's
            # paths differ), the same iterates up to FP32 rounding
            np.testing.assert_allclose(g[key], ref[key], rtol=1e-6, atol=1e-6 * b.S,
                                       err_msg=f"{variant} {key}")
        else:
            np.testing.assert_array_equal(g[key], ref[key], err_msg=f"{variant} {key}")


def test_three_quick_steps_keep_parity(solver, oracle_mod):
    """Three quick steps per path (the run may stop after the second once the
    certificate's step conditions hold): no certified path is wrong and the
    parity bar holds, on the canyon paths with their collapsed minimisers."""
    sc = scenes.canyon_scene()
    b = scenes.canyon_sample_paths(sc, 4000, seed=5200, n=2)
    ref = oracle_mod.solve(b, threads=8)
    g = gpu_util.run_gpu(solver, b, _opts(b.S, iters=12, quick_steps=3, quick_passes=1),
                         with_order=False)
    _check_common(b, g, ref)


def test_graph_keeps_its_workspace():
    """While a captured graph records a handle's workspace, a call that
    would grow (and so free) it is refused, and so is destroying the handle;
    after the graph is destroyed both work, and the replay before that still
    gives the eager result."""
    import torch
    from paper_2510_16172_amd import fpt
    s = fpt.Solver(0)
    sc = scenes.canyon_scene()
    small = scenes.canyon_sample_paths(sc, 5000, seed=4310, n=None, n_max=4)
    big = scenes.canyon_sample_paths(sc, 50000, seed=4311, n=None, n_max=4)
    opts = _opts(small.S, iters=16)
    dbs, dbb = fpt.DeviceBatch(small), fpt.DeviceBatch(big)
    eager = s.solve(dbs, opts)
    torch.cuda.synchronize()
    eager = {k: v.cpu().numpy() for k, v in eager.items()}
    st = torch.cuda.Stream()
    out = s.alloc_out(dbs)
    with torch.cuda.stream(st):
        graph = s.capture(dbs, opts, out, st)
    with pytest.raises(fpt.FptError, match="captured graph"):
        s.solve(dbb, opts)
    with pytest.raises(fpt.FptError, match="captured graphs"):
        s.close()
    # a solve that fits the recorded workspace is fine
    s.solve(fpt.DeviceBatch(small.subset(np.arange(1000))), opts)
    torch.cuda.synchronize()
    graph.launch(st)
    st.synchronize()
    for k in eager:
        np.testing.assert_array_equal(out[k].cpu().numpy(), eager[k], err_msg=k)
    graph.close()
    s.solve(dbb, opts)
    torch.cuda.synchronize()
    s.close()


@pytest.mark.parametrize("case", ["random_order2", "canyon_order3"])
def test_sixty_four_fixed_point_iterations(solver, oracle_mod, case):
    """The paper's "ours-64": 64 fixed-point iterations of Eq. 6 per BFGS
    step (fp_iters = 64) instead of one; the same parity bar."""
    if case == "random_order2":
        b = scenes.random_paths(1024, 2, seed=1001)
        g = gpu_util.run_gpu(solver, b, _opts(b.S, iters=64, fp_iters=64), with_order=False)
    else:
        sc = scenes.canyon_scene()
        b = scenes.canyon_sample_paths(sc, 3000, seed=4903, n=3)
        g = gpu_util.run_gpu(solver, b, _opts(b.S, iters=32, fp_iters=64), with_order=False)
    ref = oracle_mod.solve(b, threads=8)
    s = _check_common(b, g, ref)
    assert s["frac_cert"] >= 0.98
