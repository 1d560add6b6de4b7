"""FP64 numpy reference of the learned initialiser's MLP (66 -> 256 -> 256 ->
256 -> 8, ReLU) and of its features, written from the definitions in
include/fpt.h; used to check the BF16 MFMA kernels. The padded layout of the
library's state buffer (weights [out][in], input padded to 96, output to 64)
is mirrored here only to read the weights."""
from __future__ import annotations

import numpy as np

IN, INP, HID, OUT, OUTP = 66, 96, 256, 8, 64
OFF = {}
_o = 0
for name, shape in (("W1", (HID, INP)), ("b1", (HID,)), ("W2", (HID, HID)),
                    ("b2", (HID,)), ("W3", (HID, HID)), ("b3", (HID,)),
                    ("W4", (OUTP, HID)), ("b4", (OUTP,))):
    OFF[name] = (_o, shape)
    _o += int(np.prod(shape))
PARAMS = _o  # 172864


def unpack(vec):
    """Weights dict (FP64, real sizes) from the first PARAMS floats."""
    d = {}
    for k, (o, shape) in OFF.items():
        d[k] = np.asarray(vec[o:o + int(np.prod(shape))], np.float64).reshape(shape)
    d["W1"] = d["W1"][:, :IN]
    d["W4"] = d["W4"][:OUT]
    d["b4"] = d["b4"][:OUT]
    return d


def features(b, S):
    """[N, 66]: TX, RX, then per interaction b, a1/|a1|, a2/|a2| (0 for an
    edge), b - TX, b - RX; lengths / S."""
    tx = b.pts[:, b.src].T.astype(np.float64)
    rx = b.pts[:, b.dst].T.astype(np.float64)
    cols = [tx / S, rx / S]
    for j in range(4):
        k = b.ids[j]
        bb = b.obj[0:3, k].T.astype(np.float64)
        a1 = b.obj[3:6, k].T.astype(np.float64)
        a2 = b.obj[6:9, k].T.astype(np.float64)
        n2 = np.linalg.norm(a2, axis=1, keepdims=True)
        cols += [bb / S, a1 / np.linalg.norm(a1, axis=1, keepdims=True),
                 np.where(n2 > 0, a2 / np.where(n2 > 0, n2, 1), 0.0),
                 (bb - tx) / S, (bb - rx) / S]
    return np.concatenate(cols, axis=1)


def forward(W, X):
    H1 = np.maximum(X @ W["W1"].T + W["b1"], 0)
    H2 = np.maximum(H1 @ W["W2"].T + W["b2"], 0)
    H3 = np.maximum(H2 @ W["W3"].T + W["b3"], 0)
    Y = H3 @ W["W4"].T + W["b4"]
    return Y, (X, H1, H2, H3)


def loss_and_grad(W, X, T, M):
    """Masked MSE: sum(((Y - T) * M)^2) / (8 B) and its gradient."""
    B = X.shape[0]
    Y, (X, H1, H2, H3) = forward(W, X)
    E = (Y - T) * M
    L = float((E * E).sum() / (OUT * B))
    dY = 2.0 * E / (OUT * B)
    g = {"W4": dY.T @ H3, "b4": dY.sum(0)}
    d3 = (dY @ W["W4"]) * (H3 > 0)
    g["W3"], g["b3"] = d3.T @ H2, d3.sum(0)
    d2 = (d3 @ W["W3"]) * (H2 > 0)
    g["W2"], g["b2"] = d2.T @ H1, d2.sum(0)
    d1 = (d2 @ W["W2"]) * (H1 > 0)
    g["W1"], g["b1"] = d1.T @ X, d1.sum(0)
    return L, g


def targets(b, t, status, S):
    """Unit-basis parameters / S of a solver output t [4][2][N] and the mask
    (certified paths, non-padded parameters)."""
    t = np.asarray(t, np.float64).reshape(4, 2, -1)
    N = b.N
    T = np.zeros((N, OUT))
    M = np.zeros((N, OUT))
    cert = (status & 1) != 0
    for j in range(4):
        k = b.ids[j]
        n1 = np.linalg.norm(b.obj[3:6, k].astype(np.float64), axis=0)
        n2 = np.linalg.norm(b.obj[6:9, k].astype(np.float64), axis=0)
        T[:, 2 * j] = t[j, 0] * n1 / S
        T[:, 2 * j + 1] = np.where(n2 > 0, t[j, 1] * n2 / S, 0.0)
        M[:, 2 * j] = cert & np.isfinite(T[:, 2 * j])
        M[:, 2 * j + 1] = cert & (n2 > 0) & np.isfinite(T[:, 2 * j + 1])
    return np.nan_to_num(T) * M, M


def bf16(a):
    """Round to bfloat16 (nearest even), as the kernels store operands."""
    a = np.asarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def loss_and_grad_bf16(W, X, T, M):
    """loss_and_grad with the training kernels' storage precision: weights,
    inputs, the hidden activations H1..H3, the output error dY and the
    back-propagated dH3..dH1 rounded to bfloat16 where the kernels store
    them (products and sums exact here, FP32 accumulation there). W holds
    the bf16-rounded weights; X the bf16-rounded features."""
    B = X.shape[0]
    H1 = bf16(np.maximum(X @ W["W1"].T + W["b1"], 0))
    H2 = bf16(np.maximum(H1 @ W["W2"].T + W["b2"], 0))
    H3 = bf16(np.maximum(H2 @ W["W3"].T + W["b3"], 0))
    Y = H3 @ W["W4"].T + W["b4"]
    E = (Y - T) * M
    L = float((E * E).sum() / (OUT * B))
    dY = bf16(2.0 * E / (OUT * B))
    g = {"W4": dY.T @ H3, "b4": dY.sum(0)}
    d3 = bf16((dY @ W["W4"]) * (H3 > 0))
    g["W3"], g["b3"] = d3.T @ H2, d3.sum(0)
    d2 = bf16((d3 @ W["W3"]) * (H2 > 0))
    g["W2"], g["b2"] = d2.T @ H1, d2.sum(0)
    d1 = bf16((d2 @ W["W2"]) * (H1 > 0))
    g["W1"], g["b1"] = d1.T @ X, d1.sum(0)
    return L, g
