"""Seeded synthetic workloads for the Fermat path solver.

This module only draws geometry and enumerates interaction sequences. It holds
no step of the path-length minimisation, so the CPU oracle and the HIP path can
both take their inputs from it without sharing any of the method's arithmetic.

Every workload is a :class:`Batch` in the layout the C ABI takes:

* ``obj``   float32 ``[9][K]``  object table, rows ``b(3), a1(3), a2(3)``.
  A point on object k is ``b + t0*a1 + t1*a2`` (the affine parametrisation of
  Sec. III-B, Eq. 3). ``a2 == 0`` exactly marks a straight edge (d = 1); the
  zero second basis vector is the paper's padding of edges to d = 2.
* ``pts``   float32 ``[3][Q]``  endpoint table (TX and RX positions).
* ``src``, ``dst`` int32 ``[N]`` indices into ``pts`` for x_0 and x_{n+1}.
* ``order`` uint8 ``[N]`` number of interactions n of each path.
* ``ids``   int32 ``[n_max][N]`` object of each interaction, -1 beyond order.
* ``S``     scene size: longest side of the bounding box of the points that
  define the scene, the unit of the 1e-4 relative point tolerance.

Workloads (the paper only says its scenes are random, Sec. IV):

* :func:`random_paths` - independent random geometry per path: TX, RX and
  object origins uniform in ``[-10, 10]^3``; each interaction is a plane with
  probability ``p_reflect`` (two orthonormal spanning vectors from the QR
  factor of a 3x3 standard normal matrix), else an edge (unit direction from a
  normalised standard normal vector).
* :func:`canyon_scene` - a street canyon: 24 axis-aligned boxes on a 6x4
  block grid over a 200 m x 200 m ground face, 121 faces + 192 edges, and 64
  TX/RX pairs on the ground outside the footprints at 1.5-30 m height.
* :func:`canyon_all_paths` - every sequence of order 1..n with no immediate
  repeat, for every TX/RX pair.
* :func:`canyon_sample_paths` - sampled sequences (fixed order, or order drawn
  with P(n) proportional to 2^-n).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

N_MAX = 6


@dataclass
class Batch:
    obj: np.ndarray  # float32 [9][K]
    pts: np.ndarray  # float32 [3][Q]
    src: np.ndarray  # int32 [N]
    dst: np.ndarray  # int32 [N]
    order: np.ndarray  # uint8 [N]
    ids: np.ndarray  # int32 [n_max][N]
    S: float
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(self.src.shape[0])

    @property
    def n_max(self) -> int:
        return int(self.ids.shape[0])

    @property
    def K(self) -> int:
        return int(self.obj.shape[1])

    @property
    def Q(self) -> int:
        return int(self.pts.shape[1])

    def subset(self, idx) -> "Batch":
        """Paths ``idx`` over the same object and point tables."""
        idx = np.asarray(idx)
        return Batch(self.obj, self.pts, np.ascontiguousarray(self.src[idx]),
                     np.ascontiguousarray(self.dst[idx]),
                     np.ascontiguousarray(self.order[idx]),
                     np.ascontiguousarray(self.ids[:, idx]), self.S,
                     dict(self.meta))

    def check(self) -> None:
        """Shape and range checks of the layout above (host side only)."""
        assert self.obj.dtype == np.float32 and self.obj.ndim == 2 and self.obj.shape[0] == 9
        assert self.pts.dtype == np.float32 and self.pts.ndim == 2 and self.pts.shape[0] == 3
        for a in (self.src, self.dst):
            assert a.dtype == np.int32 and a.shape == (self.N,)
            if self.N:
                assert a.min() >= 0 and a.max() < self.Q
        assert self.order.dtype == np.uint8 and self.order.shape == (self.N,)
        assert self.ids.dtype == np.int32 and self.ids.shape == (self.n_max, self.N)
        assert 1 <= self.n_max <= N_MAX
        if self.N:
            assert self.order.min() >= 1 and self.order.max() <= self.n_max
            j = np.arange(self.n_max)[:, None]
            active = j < self.order[None, :].astype(np.int64)
            assert np.all(self.ids[active] >= 0) and np.all(self.ids[active] < self.K)
            assert np.all(self.ids[~active] == -1)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _unit_rows(v: np.ndarray) -> np.ndarray:
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def random_paths(N: int, n: int, seed: int, p_reflect: float = 0.5,
                 box: float = 10.0, kinds: np.ndarray | None = None) -> Batch:
    """Independent random geometry per path, K = N*n objects with identity ids.

    ``kinds`` (optional, ``[n][N]`` bool, True = plane) overrides the draw of
    interaction types, e.g. for reflection-only or diffraction-only batches.
    Object of slot j of path i is column ``j*N + i``; TX of path i is point i,
    RX is point ``N + i``.
    """
    rng = _rng(seed)
    tx = rng.uniform(-box, box, (N, 3))
    rx = rng.uniform(-box, box, (N, 3))
    refl = rng.random((n, N)) < p_reflect
    if kinds is not None:
        refl = np.asarray(kinds, dtype=bool).reshape(n, N)
    origin = rng.uniform(-box, box, (n, N, 3))
    gauss = rng.standard_normal((n, N, 3, 3))
    q, _ = np.linalg.qr(gauss)
    plane_a1 = q[..., :, 0]
    plane_a2 = q[..., :, 1]
    edge_dir = _unit_rows(rng.standard_normal((n, N, 3)))
    a1 = np.where(refl[..., None], plane_a1, edge_dir)
    a2 = np.where(refl[..., None], plane_a2, 0.0)
    K = N * n
    obj = np.empty((9, K), np.float32)
    obj[0:3] = origin.reshape(K, 3).T
    obj[3:6] = a1.reshape(K, 3).T
    obj[6:9] = a2.reshape(K, 3).T
    pts = np.empty((3, 2 * N), np.float32)
    pts[:, :N] = tx.T
    pts[:, N:] = rx.T
    src = np.arange(N, dtype=np.int32)
    dst = np.arange(N, 2 * N, dtype=np.int32)
    ids = (np.arange(n, dtype=np.int32)[:, None] * N
           + np.arange(N, dtype=np.int32)[None, :]).astype(np.int32)
    order = np.full(N, n, np.uint8)
    return Batch(obj, pts, src, dst, order, ids, S=2.0 * box,
                 meta=dict(kind="random", seed=seed, n=n, p_reflect=p_reflect,
                           reflect=refl))


# ----------------------------------------------------------------------------
# Street canyon
# ----------------------------------------------------------------------------

GROUND = 200.0
BLOCKS_X, BLOCKS_Y = 6, 4
STREET = 3.0


def canyon_scene(seed: int = 2025, n_pairs: int = 64) -> Batch:
    """Street canyon: ground face, 24 boxes, 64 TX/RX pairs (no paths yet).

    Boxes sit on a 6 x 4 grid of blocks (x pitch 200/6 m, y pitch 50 m); each
    footprint side is U[5, 30] m clipped so that at least a 3 m street is left
    to the block border, its centre is jittered inside the remaining slack,
    and its height is U[5, 40] m. Faces: 4 walls + roof per box (origin at a
    corner, spanning vectors = the two edge vectors of the face) + the ground.
    Edges: 4 roof edges + 4 vertical edges per box (origin at an endpoint,
    a1 = edge vector, a2 = 0); edges on the ground are left out.
    TX and RX are uniform on the ground outside every footprint, at heights
    U[1.5, 30] m. Scene size S = 200 m (the ground side).
    """
    rng = _rng(seed)
    px, py = GROUND / BLOCKS_X, GROUND / BLOCKS_Y
    boxes = []
    for iy in range(BLOCKS_Y):
        for ix in range(BLOCKS_X):
            cx0 = -GROUND / 2 + px * (ix + 0.5)
            cy0 = -GROUND / 2 + py * (iy + 0.5)
            sx = min(rng.uniform(5.0, 30.0), px - 2 * STREET)
            sy = min(rng.uniform(5.0, 30.0), py - 2 * STREET)
            jx = (px - 2 * STREET - sx) / 2
            jy = (py - 2 * STREET - sy) / 2
            cx = cx0 + rng.uniform(-jx, jx)
            cy = cy0 + rng.uniform(-jy, jy)
            h = rng.uniform(5.0, 40.0)
            boxes.append((cx - sx / 2, cy - sy / 2, cx + sx / 2, cy + sy / 2, h))
    faces_b, faces_a1, faces_a2 = [], [], []
    edges_b, edges_a1 = [], []
    half = GROUND / 2
    faces_b.append((-half, -half, 0.0))
    faces_a1.append((GROUND, 0.0, 0.0))
    faces_a2.append((0.0, GROUND, 0.0))
    for (x0, y0, x1, y1, h) in boxes:
        c = [(x0, y0), (x1, y0), (x1, y1), (x0, y1)]
        for k in range(4):  # walls, counter-clockwise seen from above
            (ax, ay), (bx, by) = c[k], c[(k + 1) % 4]
            faces_b.append((ax, ay, 0.0))
            faces_a1.append((bx - ax, by - ay, 0.0))
            faces_a2.append((0.0, 0.0, h))
        faces_b.append((x0, y0, h))  # roof
        faces_a1.append((x1 - x0, 0.0, 0.0))
        faces_a2.append((0.0, y1 - y0, 0.0))
        for k in range(4):  # roof edges
            (ax, ay), (bx, by) = c[k], c[(k + 1) % 4]
            edges_b.append((ax, ay, h))
            edges_a1.append((bx - ax, by - ay, 0.0))
        for k in range(4):  # vertical edges
            ax, ay = c[k]
            edges_b.append((ax, ay, 0.0))
            edges_a1.append((0.0, 0.0, h))
    nf, ne = len(faces_b), len(edges_b)
    K = nf + ne
    obj = np.zeros((9, K), np.float32)
    obj[0:3, :nf] = np.array(faces_b).T
    obj[3:6, :nf] = np.array(faces_a1).T
    obj[6:9, :nf] = np.array(faces_a2).T
    obj[0:3, nf:] = np.array(edges_b).T
    obj[3:6, nf:] = np.array(edges_a1).T

    def inside_any(x, y):
        for (x0, y0, x1, y1, _) in boxes:
            if x0 <= x <= x1 and y0 <= y <= y1:
                return True
        return False

    P = []
    while len(P) < 2 * n_pairs:
        x, y = rng.uniform(-half, half, 2)
        if inside_any(x, y):
            continue
        P.append((x, y, rng.uniform(1.5, 30.0)))
    pts = np.array(P, np.float32).T.copy()  # pair k: TX = 2k, RX = 2k+1
    empty_i = np.zeros(0, np.int32)
    return Batch(obj, pts, empty_i, empty_i, np.zeros(0, np.uint8),
                 np.zeros((1, 0), np.int32), S=GROUND,
                 meta=dict(kind="canyon", seed=seed, n_faces=nf, n_edges=ne,
                           boxes=np.array(boxes), n_pairs=n_pairs))


def _with_paths(scene: Batch, pair: np.ndarray, order: np.ndarray,
                ids: np.ndarray, **meta) -> Batch:
    b = Batch(scene.obj, scene.pts, (2 * pair).astype(np.int32),
              (2 * pair + 1).astype(np.int32), order.astype(np.uint8),
              ids.astype(np.int32), scene.S, dict(scene.meta))
    b.meta.update(meta)
    return b


def canyon_all_paths(scene: Batch, n_max: int = 2) -> Batch:
    """All sequences of order 1..n_max without an immediate repeat, per pair.

    Paths are grouped by order, then by pair, then by the object sequence in
    lexicographic order. For K = 313, 64 pairs and n_max = 2 this is
    64 * (313 + 313*312) = 6,270,016 paths.
    """
    K = scene.K
    P = scene.meta["n_pairs"]
    pairs, orders, idss = [], [], []
    for n in range(1, n_max + 1):
        # all sequences of length n over K with no immediate repeat
        seq = np.arange(K, dtype=np.int32)[:, None]
        for _ in range(n - 1):
            nxt = np.arange(K, dtype=np.int32)
            a = np.repeat(seq, K, axis=0)
            b = np.tile(nxt, seq.shape[0])
            keep = a[:, -1] != b
            seq = np.concatenate([a[keep], b[keep, None]], axis=1)
        M = seq.shape[0]
        pairs.append(np.repeat(np.arange(P, dtype=np.int32), M))
        orders.append(np.full(P * M, n, np.uint8))
        full = np.full((n_max, P * M), -1, np.int32)
        full[:n] = np.tile(seq, (P, 1)).T
        idss.append(full)
    return _with_paths(scene, np.concatenate(pairs), np.concatenate(orders),
                       np.concatenate(idss, axis=1), paths="all", n_max=n_max)


def _sample_sequences(rng, K: int, order: np.ndarray, n_max: int) -> np.ndarray:
    N = order.shape[0]
    ids = np.full((n_max, N), -1, np.int32)
    prev = rng.integers(0, K, N)
    ids[0] = prev
    for j in range(1, n_max):
        # uniform over the K-1 objects different from the previous one
        nxt = rng.integers(0, K - 1, N)
        nxt = nxt + (nxt >= prev)
        ids[j] = nxt
        prev = nxt
    j = np.arange(n_max)[:, None]
    ids[j >= order[None, :].astype(np.int64)] = -1
    return ids


def canyon_sample_paths(scene: Batch, N: int, seed: int, n: int | None = None,
                        n_max: int = N_MAX) -> Batch:
    """N sampled paths: pair uniform over the pairs, objects uniform with no
    immediate repeat. Order is ``n`` for every path, or, when ``n`` is None,
    drawn on {1..n_max} with P(n) proportional to 2^-n."""
    rng = _rng(seed)
    P = scene.meta["n_pairs"]
    pair = rng.integers(0, P, N).astype(np.int32)
    if n is None:
        w = 0.5 ** np.arange(1, n_max + 1)
        order = rng.choice(np.arange(1, n_max + 1), size=N, p=w / w.sum())
    else:
        n_max = n
        order = np.full(N, n)
    order = order.astype(np.uint8)
    ids = _sample_sequences(rng, scene.K, order, n_max)
    return _with_paths(scene, pair, order, ids, paths="sample", seed=seed)


def upstream_grads(N: int, n_max: int, seed: int):
    """Upstream cotangents g_L [N] and g_X [n_max][3][N], i.i.d. N(0, 1)."""
    rng = _rng(seed)
    g_len = rng.standard_normal(N).astype(np.float32)
    g_x = rng.standard_normal((n_max, 3, N)).astype(np.float32)
    return g_len, g_x


def enumerate_face_vertices(scene: Batch):
    """Vertex form of every object: faces b = v0, a1 = v1 - v0, a2 = v3 - v0;
    edges b = v0, a1 = v1 - v0. Returns (V [3][n_vert] float64, map) where
    ``map[k] = (i0, i1, i3)`` (i3 = -1 for an edge)."""
    K = scene.K
    V, m = [], []
    for k in range(K):
        b = scene.obj[0:3, k].astype(np.float64)
        a1 = scene.obj[3:6, k].astype(np.float64)
        a2 = scene.obj[6:9, k].astype(np.float64)
        i0 = len(V)
        V.append(b)
        V.append(b + a1)
        if np.any(a2 != 0):
            V.append(b + a2)
            m.append((i0, i0 + 1, i0 + 2))
        else:
            m.append((i0, i0 + 1, -1))
    return np.array(V).T, np.array(m, np.int64)
