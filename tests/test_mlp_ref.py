"""The FP64 MLP reference is pinned by central finite differences of its own
loss (CPU)."""
import numpy as np

import mlp_ref


def test_mlp_reference_gradient_fd():
    rng = np.random.default_rng(0)
    W = {"W1": rng.standard_normal((256, 66)) * 0.1, "b1": rng.standard_normal(256) * 0.1,
         "W2": rng.standard_normal((256, 256)) * 0.06, "b2": rng.standard_normal(256) * 0.1,
         "W3": rng.standard_normal((256, 256)) * 0.06, "b3": rng.standard_normal(256) * 0.1,
         "W4": rng.standard_normal((8, 256)) * 0.06, "b4": rng.standard_normal(8) * 0.1}
    X = rng.standard_normal((32, 66))
    T = rng.standard_normal((32, 8))
    M = (rng.random((32, 8)) < 0.8).astype(float)
    L, g = mlp_ref.loss_and_grad(W, X, T, M)
    h = 1e-6
    for name in W:
        flat = W[name].ravel()
        for idx in rng.choice(flat.size, 6, replace=False):
            old = flat[idx]
            flat[idx] = old + h
            Lp, _ = mlp_ref.loss_and_grad(W, X, T, M)
            flat[idx] = old - h
            Lm, _ = mlp_ref.loss_and_grad(W, X, T, M)
            flat[idx] = old
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - g[name].ravel()[idx]) < 1e-6 * (1 + abs(fd)), name
    assert mlp_ref.PARAMS == 172864
