"""BF16 MFMA kernels of the learned initialiser vs the FP64 numpy reference
(tests/mlp_ref.py), and its training behaviour."""
import numpy as np
import pytest

import gpu_util
import mlp_ref
from paper_2510_16172_amd import scenes

pytestmark = pytest.mark.gpu


def _bf16(a):
    """Round to bfloat16 (nearest even), as the kernels store operands."""
    a = np.asarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def solver():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2510_16172_amd import fpt
    s = fpt.Solver(0)
    yield s
    s.close()


def _batch(N, seed):
    sc = scenes.canyon_scene()
    return scenes.canyon_sample_paths(sc, N, seed=seed, n=4)


def test_infer_matches_reference(solver):
    import torch
    from paper_2510_16172_amd import fpt
    b = _batch(1000, 6000)   # ragged: 1000 is not a multiple of 64
    mlp = fpt.Mlp(solver, seed=3)
    db = fpt.DeviceBatch(b)
    t_init = mlp.infer(db, b.S)
    torch.cuda.synchronize()
    W = mlp_ref.unpack(mlp.weights().cpu().numpy())
    Wb = {k: (_bf16(v) if k.startswith("W") else v) for k, v in W.items()}
    X = _bf16(mlp_ref.features(b, b.S))
    Y, _ = mlp_ref.forward(Wb, X)
    # back to the caller's parametrisation
    want = np.zeros((4, 2, b.N))
    for j in range(4):
        k = b.ids[j]
        n1 = np.linalg.norm(b.obj[3:6, k].astype(np.float64), axis=0)
        n2 = np.linalg.norm(b.obj[6:9, k].astype(np.float64), axis=0)
        want[j, 0] = Y[:, 2 * j] * b.S / n1
        want[j, 1] = np.where(n2 > 0, Y[:, 2 * j + 1] * b.S / np.where(n2 > 0, n2, 1), 0)
    got = t_init.cpu().numpy().astype(np.float64)
    scale = np.abs(want).max()
    # bf16 activations between layers: ~1e-2 relative
    assert np.abs(got - want).max() <= 3e-2 * scale
    assert np.corrcoef(got.ravel(), want.ravel())[0, 1] > 0.9995


def test_train_step_gradient_matches_reference(solver):
    import torch
    from paper_2510_16172_amd import fpt
    b = _batch(1024, 6100)
    db = fpt.DeviceBatch(b, with_order=False)
    out = solver.solve(db, fpt.Opts(scale=b.S, iters=96))
    mlp = fpt.Mlp(solver, seed=4)
    W = mlp_ref.unpack(mlp.weights().cpu().numpy().copy())
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    mlp.train_step(db, out, b.S, lr=1e-3, loss_acc=loss)
    torch.cuda.synchronize()
    g_gpu = mlp_ref.unpack(mlp.grad().cpu().numpy())
    Wb = {k: (_bf16(v) if k.startswith("W") else v) for k, v in W.items()}
    X = _bf16(mlp_ref.features(b, b.S))
    t = out["t"].cpu().numpy().astype(np.float64)
    T, M = mlp_ref.targets(b, t, out["status"].cpu().numpy(), b.S)
    L, g = mlp_ref.loss_and_grad(Wb, X, T, M)
    assert abs(loss.item() - L) <= 2e-2 * L
    for k in g:
        a, w = g_gpu[k].ravel(), g[k].ravel()
        cos = np.dot(a, w) / (np.linalg.norm(a) * np.linalg.norm(w) + 1e-30)
        rel = np.linalg.norm(a - w) / (np.linalg.norm(w) + 1e-30)
        print(f"{k}: cos {cos:.5f} rel {rel:.3e}", flush=True)
        assert cos > 0.995 and rel < 0.1, k
    # element by element against the reference that stores the activations
    # and back-propagated errors in bfloat16 where the kernels do: what is
    # left is FP32 accumulation order and the rare value that rounds to the
    # other bfloat16 neighbour. Bound per element: 2^-9 of (|g| + the
    # tensor's RMS), half the bfloat16 unit roundoff (2^-8).
    Lb, gb = mlp_ref.loss_and_grad_bf16(Wb, X, T, M)
    assert abs(loss.item() - Lb) <= 1e-3 * Lb
    for k in gb:
        a, w = g_gpu[k].ravel(), gb[k].ravel()
        rms = np.sqrt(np.mean(w * w)) + 1e-30
        err = np.abs(a - w) / (np.abs(w) + rms)
        print(f"{k}: max elementwise error {err.max():.2e} (x (|g| + rms))", flush=True)
        assert err.max() <= 2.0 ** -9, k


def test_training_reduces_loss(solver):
    import torch
    from paper_2510_16172_amd import fpt
    b = _batch(16384, 6200)
    db = fpt.DeviceBatch(b, with_order=False)
    out = solver.solve(db, fpt.Opts(scale=b.S, iters=96))
    mlp = fpt.Mlp(solver, seed=5)
    losses = []
    for epoch in range(30):
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        mlp.train_step(db, out, b.S, lr=2e-3, loss_acc=loss)
        losses.append(loss.item())
    print("losses", losses[0], losses[-1], flush=True)
    assert losses[-1] < 0.5 * losses[0]
    assert np.all(np.isfinite(losses))


def test_learned_init_gains_over_zero_start(solver):
    """What the trained network gains: on held-out order-4 canyon paths and
    at the same fixed number of BFGS iterations, the solver started from the
    network's prediction certifies more paths than from T = 0, and needs
    fewer iterations to stop under early exit (the plain solver is the
    teacher and the fallback)."""
    import torch
    from paper_2510_16172_amd import fpt, learned_init
    sc = scenes.canyon_scene()
    test = scenes.canyon_sample_paths(sc, 1 << 16, seed=6300, n=4)
    train = learned_init.dedup_against(
        scenes.canyon_sample_paths(sc, 1 << 19, seed=6301, n=4), test)
    dbt = fpt.DeviceBatch(train, with_order=False)
    target = solver.solve(dbt, fpt.Opts(scale=sc.S, iters=96))
    mlp = fpt.Mlp(solver, seed=1)
    losses = learned_init.train(solver, mlp, dbt, target, sc.S, epochs=24,
                                lr=2e-3, batch=8192)
    assert losses[-1] < 0.5 * losses[0]
    dbe = fpt.DeviceBatch(test, with_order=False)
    t0 = mlp.infer(dbe, sc.S)

    def run(t_init, **kw):
        dbe.t_init = t_init
        out = solver.solve(dbe, fpt.Opts(scale=sc.S, **kw))
        torch.cuda.synchronize()
        dbe.t_init = None
        return {k: v.cpu().numpy() for k, v in out.items()}

    # (with the rescaled initial inverse Hessian the start point matters
    # most over the first few iterations: +1.5 points at 3-4, +0.6 at 8)
    z, l = run(None, iters=4), run(t0, iters=4)
    cz = ((z["status"] & fpt.ST_CONVERGED) != 0).mean()
    cl = ((l["status"] & fpt.ST_CONVERGED) != 0).mean()
    print(f"certified at 4 iterations: zero {cz:.4f} learned {cl:.4f}", flush=True)
    assert cl >= cz + 0.008
    ze, le = run(None, iters=64, early_exit=True), run(t0, iters=64, early_exit=True)
    iz, il = ze["iters"].astype(np.float64).mean(), le["iters"].astype(np.float64).mean()
    print(f"mean iterations under early exit: zero {iz:.2f} learned {il:.2f}", flush=True)
    assert il < iz


def test_learned_start_fallback(solver, oracle_mod):
    """learned_init.evaluate: the paths the learned start leaves uncertified
    are solved again from T = 0 and their results replace the learned
    start's. With the fallback, at least as many paths are certified as from
    T = 0 alone, and no certified path of the merged output is wrong against
    the oracle (sampled)."""
    import torch
    from paper_2510_16172_amd import fpt, learned_init
    sc = scenes.canyon_scene()
    test = scenes.canyon_sample_paths(sc, 1 << 15, seed=6400, n=4)
    train = learned_init.dedup_against(
        scenes.canyon_sample_paths(sc, 1 << 17, seed=6401, n=4), test)
    dbt = fpt.DeviceBatch(train, with_order=False)
    target = solver.solve(dbt, fpt.Opts(scale=sc.S, iters=96))
    mlp = fpt.Mlp(solver, seed=2)
    learned_init.train(solver, mlp, dbt, target, sc.S, epochs=4, lr=2e-3, batch=8192)
    dbe = fpt.DeviceBatch(test, with_order=False)
    # few iterations, so that the learned start leaves paths to the fallback
    res, out0, out1 = learned_init.evaluate(solver, mlp, dbe, fpt.Opts(scale=sc.S, iters=4),
                                            repeats=1)
    torch.cuda.synchronize()
    li = res["learned_init"]
    print(res["zero_init"]["certified"], li["certified"], li["certified_with_fallback"],
          li["fallback_paths"], flush=True)
    assert li["fallback_paths"] > 0
    assert li["certified_with_fallback"] >= res["zero_init"]["certified"]
    st1 = out1["status"].cpu().numpy()
    cert1 = (st1 & fpt.ST_CONVERGED) != 0
    assert abs(cert1.mean() - li["certified_with_fallback"]) < 1e-9
    idx = np.sort(np.random.default_rng(6402).choice(test.N, 4096, replace=False))
    sub = test.subset(idx)
    ref = oracle_mod.solve(sub, threads=8)
    g = {k: (v.cpu().numpy()[..., idx] if v.dim() > 1 else v.cpu().numpy()[idx])
         for k, v in out1.items()}
    s = gpu_util.summary(sub, g, ref)
    assert s["false_pos"] == 0
    assert s["frac_gate"] >= 0.97
