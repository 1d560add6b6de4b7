"""ctypes binding of libfpt.so (the C ABI in include/fpt.h).

Argument marshalling only: every step of the solve and of the gradient runs
in the HIP kernels of the library. PyTorch provides device memory and the
stream (``torch.cuda.current_stream()``). There is no CPU fallback: if the
library is missing or no gfx950 device is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfpt.so")

FPT_NMAX = 6
FPT_MAX_LEVELS = 8

ST_CONVERGED, ST_REFINED, ST_COLLAPSED, ST_NONFINITE, ST_INVALID, ST_NOGRAD = (
    1, 2, 4, 8, 16, 32)

_P = ctypes.c_void_p


class _Scene(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("obj", _P), ("Q", ctypes.c_int32),
                ("pts", _P)]


class _Paths(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("n_max", ctypes.c_int32),
                ("src", _P), ("dst", _P), ("order", _P), ("ids", _P),
                ("t_init", _P)]


class _Opts(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("fp_iters", ctypes.c_int32),
                ("early_exit", ctypes.c_int32), ("exit_rtol", ctypes.c_float),
                ("scale", ctypes.c_float), ("n_levels", ctypes.c_int32),
                ("level_eps", ctypes.c_float * FPT_MAX_LEVELS),
                ("level_steps", ctypes.c_int32 * FPT_MAX_LEVELS),
                ("cert_rtol", ctypes.c_float),
                ("stage_iters", ctypes.c_int32 * 4),
                ("quick_steps", ctypes.c_int32), ("quick_passes", ctypes.c_int32),
                ("concurrent_orders", ctypes.c_int32), ("method", ctypes.c_int32),
                ("polish_steps", ctypes.c_int32), ("split", ctypes.c_int32),
                ("line_search", ctypes.c_int32)]


class _LaunchCfg(ctypes.Structure):
    _fields_ = [("wg_per_cu", ctypes.c_int32), ("use_override", ctypes.c_int32),
                ("early_exit", ctypes.c_int32), ("stage_iters", ctypes.c_int32 * 4),
                ("iters", ctypes.c_int32), ("quick_steps", ctypes.c_int32),
                ("quick_passes", ctypes.c_int32), ("refine_wg_per_cu", ctypes.c_int32)]


class _EnumSpec(ctypes.Structure):
    _fields_ = [("pair_src", _P), ("pair_dst", _P), ("P", ctypes.c_int32),
                ("K", ctypes.c_int32), ("order_min", ctypes.c_int32),
                ("order_max", ctypes.c_int32), ("no_repeat", ctypes.c_int32)]


class _Out(ctypes.Structure):
    _fields_ = [("x", _P), ("len", _P), ("t", _P), ("status", _P),
                ("iters", _P)]


EXPORTED = ["fpt_default_opts", "fpt_create", "fpt_destroy", "fpt_solve",
            "fpt_grad", "fpt_last_error", "fpt_set_timing", "fpt_kernel_times",
            "fpt_mlp_state_floats", "fpt_mlp_init", "fpt_mlp_train_step",
            "fpt_mlp_infer", "fpt_set_launch", "fpt_graph_capture",
            "fpt_graph_launch", "fpt_graph_destroy", "fpt_validate",
            "fpt_work_counts", "fpt_enum_count", "fpt_enumerate",
            "fpt_solve_noalloc", "fpt_noalloc_max_paths"]

# timer slots of fpt_kernel_times
T_BUCKET, T_BFGS, T_REFINE, T_GRAD, T_REDUCE, T_MLP, T_VALIDATE, T_UNSORT, TIMERS = (
    0, 1, 7, 13, 14, 15, 16, 17, 18)
VALID_EXTENT, VALID_SPECULAR, VALID_VISIBLE = 1, 2, 4
VALIDATE_ALL, VALIDATE_LAZY = 0, 1
METHOD_BFGS, METHOD_NEWTON32 = 0, 1
LS_EQ6, LS_ARMIJO = 0, 1
MLP_PARAMS = 172864  # padded parameter count: state[0:MLP_PARAMS] = weights

_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libfpt.so and declares the signatures. Raises if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with `python -m "
            "paper_2510_16172_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    lib.fpt_default_opts.argtypes = [ctypes.POINTER(_Opts)]
    lib.fpt_default_opts.restype = None
    lib.fpt_create.argtypes = [ctypes.c_int, ctypes.POINTER(_P)]
    lib.fpt_create.restype = ctypes.c_int
    lib.fpt_destroy.argtypes = [_P]
    lib.fpt_destroy.restype = ctypes.c_int
    lib.fpt_solve.argtypes = [_P, ctypes.POINTER(_Scene),
                              ctypes.POINTER(_Paths), ctypes.POINTER(_Opts),
                              ctypes.POINTER(_Out), _P]
    lib.fpt_solve.restype = ctypes.c_int
    lib.fpt_solve_noalloc.argtypes = lib.fpt_solve.argtypes
    lib.fpt_solve_noalloc.restype = ctypes.c_int
    lib.fpt_noalloc_max_paths.argtypes = []
    lib.fpt_noalloc_max_paths.restype = ctypes.c_int64
    lib.fpt_grad.argtypes = [_P, ctypes.POINTER(_Scene),
                             ctypes.POINTER(_Paths), ctypes.POINTER(_Out),
                             _P, _P, _P, _P, _P, _P, _P]
    lib.fpt_grad.restype = ctypes.c_int
    lib.fpt_set_timing.argtypes = [_P, ctypes.c_int]
    lib.fpt_set_timing.restype = ctypes.c_int
    lib.fpt_kernel_times.argtypes = [_P, ctypes.POINTER(ctypes.c_float)]
    lib.fpt_kernel_times.restype = ctypes.c_int
    lib.fpt_mlp_state_floats.argtypes = []
    lib.fpt_mlp_state_floats.restype = ctypes.c_int64
    lib.fpt_mlp_init.argtypes = [_P, _P, ctypes.c_uint64, _P]
    lib.fpt_mlp_init.restype = ctypes.c_int
    lib.fpt_mlp_train_step.argtypes = [_P, _P, ctypes.POINTER(_Scene),
                                       ctypes.POINTER(_Paths),
                                       ctypes.POINTER(_Out), ctypes.c_float,
                                       ctypes.c_float, ctypes.c_int32, _P, _P]
    lib.fpt_mlp_train_step.restype = ctypes.c_int
    lib.fpt_mlp_infer.argtypes = [_P, _P, ctypes.POINTER(_Scene),
                                  ctypes.POINTER(_Paths), ctypes.c_float, _P, _P]
    lib.fpt_mlp_infer.restype = ctypes.c_int
    lib.fpt_set_launch.argtypes = [_P, ctypes.c_int, ctypes.POINTER(_LaunchCfg)]
    lib.fpt_set_launch.restype = ctypes.c_int
    lib.fpt_graph_capture.argtypes = [_P, ctypes.POINTER(_Scene),
                                      ctypes.POINTER(_Paths), ctypes.POINTER(_Opts),
                                      ctypes.POINTER(_Out), _P, ctypes.POINTER(_P)]
    lib.fpt_graph_capture.restype = ctypes.c_int
    lib.fpt_graph_launch.argtypes = [_P, _P]
    lib.fpt_graph_launch.restype = ctypes.c_int
    lib.fpt_graph_destroy.argtypes = [_P]
    lib.fpt_graph_destroy.restype = ctypes.c_int
    lib.fpt_validate.argtypes = [_P, ctypes.POINTER(_Scene), ctypes.POINTER(_Paths),
                                 ctypes.POINTER(_Out), _P, ctypes.c_int32, _P]
    lib.fpt_validate.restype = ctypes.c_int
    lib.fpt_enum_count.argtypes = [ctypes.POINTER(_EnumSpec), ctypes.POINTER(ctypes.c_int64)]
    lib.fpt_enum_count.restype = ctypes.c_int
    lib.fpt_enumerate.argtypes = [_P, ctypes.POINTER(_EnumSpec), ctypes.c_int64,
                                  ctypes.c_int64, _P, _P, _P, _P, ctypes.c_int32, _P]
    lib.fpt_enumerate.restype = ctypes.c_int
    lib.fpt_work_counts.argtypes = [_P, ctypes.POINTER(ctypes.c_uint64)]
    lib.fpt_work_counts.restype = ctypes.c_int
    lib.fpt_last_error.argtypes = []
    lib.fpt_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


class FptError(RuntimeError):
    pass


def _check(rc: int, what: str):
    if rc != 0:
        msg = load_library().fpt_last_error().decode()
        raise FptError(f"{what} failed ({rc}): {msg}")


@dataclass
class Opts:
    """Mirror of fpt_opts (defaults of fpt_default_opts)."""
    iters: int = 64
    fp_iters: int = 1
    early_exit: bool = False
    exit_rtol: float = 1e-6
    scale: float = 1.0
    level_eps: list = field(default_factory=lambda: [1e-3, 1e-5, 1e-7, 1e-9])
    level_steps: list = field(default_factory=lambda: [2, 2, 2, 3])
    cert_rtol: float = 1e-5
    stage_iters: list = field(default_factory=lambda: [16, 16, 32])
    quick_steps: int = 2
    quick_passes: int = 2
    concurrent_orders: bool = False
    method: int = 0  # METHOD_BFGS (the paper's) or METHOD_NEWTON32 (variant)
    polish_steps: int = 1
    split: int = 0  # parts per order on their own streams (0: automatic)
    line_search: int = 0  # LS_EQ6 (the paper's Eq. 6 step) or LS_ARMIJO (variant)

    def to_c(self) -> _Opts:
        o = _Opts()
        load_library().fpt_default_opts(ctypes.byref(o))
        o.iters = int(self.iters)
        o.fp_iters = int(self.fp_iters)
        o.early_exit = 1 if self.early_exit else 0
        o.exit_rtol = float(self.exit_rtol)
        o.scale = float(self.scale)
        if len(self.level_eps) != len(self.level_steps):
            raise ValueError("level_eps and level_steps differ in length")
        if len(self.level_eps) > FPT_MAX_LEVELS:
            raise ValueError("at most 8 refinement levels")
        o.n_levels = len(self.level_eps)
        for i in range(FPT_MAX_LEVELS):
            o.level_eps[i] = float(self.level_eps[i]) if i < o.n_levels else 0.0
            o.level_steps[i] = int(self.level_steps[i]) if i < o.n_levels else 0
        o.cert_rtol = float(self.cert_rtol)
        if len(self.stage_iters) > 4:
            raise ValueError("at most 4 early-exit stages")
        for i in range(4):
            o.stage_iters[i] = int(self.stage_iters[i]) if i < len(self.stage_iters) else 0
        o.quick_steps = int(self.quick_steps)
        o.quick_passes = int(self.quick_passes)
        o.concurrent_orders = 1 if self.concurrent_orders else 0
        o.method = int(self.method)
        o.polish_steps = int(self.polish_steps)
        o.split = int(self.split)
        o.line_search = int(self.line_search)
        return o


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _enum_spec(P, K, order_min, order_max, no_repeat=True, pair_src=None, pair_dst=None):
    return _EnumSpec(pair_src.data_ptr() if pair_src is not None else None,
                     pair_dst.data_ptr() if pair_dst is not None else None,
                     int(P), int(K), int(order_min), int(order_max), 1 if no_repeat else 0)


def enum_count(P: int, K: int, order_min: int, order_max: int, no_repeat: bool = True) -> int:
    """fpt_enum_count: number of candidates (every ordered sequence of
    order_min..order_max objects per pair; no immediate repeat if asked)."""
    sp = _enum_spec(P, K, order_min, order_max, no_repeat)
    total = ctypes.c_int64()
    _check(load_library().fpt_enum_count(ctypes.byref(sp), ctypes.byref(total)),
           "fpt_enum_count")
    return int(total.value)


class DeviceBatch:
    """A scenes.Batch copied to the GPU as torch tensors (the C-ABI layout)."""

    def __init__(self, batch, device="cuda", with_order=True):
        import torch
        self.batch = batch
        self.N, self.n_max, self.K, self.Q = batch.N, batch.n_max, batch.K, batch.Q
        self.S = float(batch.S)
        dev = torch.device(device)
        self.obj = torch.from_numpy(np.ascontiguousarray(batch.obj)).to(dev)
        self.pts = torch.from_numpy(np.ascontiguousarray(batch.pts)).to(dev)
        self.src = torch.from_numpy(np.ascontiguousarray(batch.src)).to(dev)
        self.dst = torch.from_numpy(np.ascontiguousarray(batch.dst)).to(dev)
        self.ids = torch.from_numpy(np.ascontiguousarray(batch.ids)).to(dev)
        self.order = (torch.from_numpy(np.ascontiguousarray(batch.order)).to(dev)
                      if with_order else None)
        self.t_init = None

    @classmethod
    def from_tensors(cls, obj, pts, src, dst, ids, order=None, S=1.0,
                     t_init=None):
        """Wraps existing device tensors (no copy)."""
        self = cls.__new__(cls)
        self.batch = None
        self.obj, self.pts, self.src, self.dst = obj, pts, src, dst
        self.ids, self.order, self.t_init = ids, order, t_init
        self.N = int(src.shape[0])
        self.n_max = int(ids.shape[0])
        self.K = int(obj.shape[1])
        self.Q = int(pts.shape[1])
        self.S = float(S)
        for name, tns, dt in (("obj", obj, "float32"), ("pts", pts, "float32"),
                              ("src", src, "int32"), ("dst", dst, "int32"),
                              ("ids", ids, "int32")):
            if str(tns.dtype) != "torch." + dt or not tns.is_contiguous():
                raise ValueError(f"{name} must be a contiguous {dt} tensor")
        if order is not None and (str(order.dtype) != "torch.uint8"
                                  or not order.is_contiguous()):
            raise ValueError("order must be a contiguous uint8 tensor")
        return self

    def c_scene(self) -> _Scene:
        return _Scene(self.K, _ptr(self.obj), self.Q, _ptr(self.pts))

    def c_paths(self) -> _Paths:
        return _Paths(self.N, self.n_max, _ptr(self.src), _ptr(self.dst),
                      _ptr(self.order), _ptr(self.ids), _ptr(self.t_init))


class Solver:
    """Handle on one gfx950 device (fpt_create / fpt_destroy)."""

    def __init__(self, device: int = 0):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.fpt_create(int(device), ctypes.byref(h)), "fpt_create")
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            _check(load_library().fpt_destroy(self._h), "fpt_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_timing(self, enable: bool = True):
        _check(load_library().fpt_set_timing(self._h, 1 if enable else 0),
               "fpt_set_timing")

    def kernel_times(self):
        """Mean ms per timer slot since the last read (-1 = unused)."""
        ms = (ctypes.c_float * TIMERS)()
        _check(load_library().fpt_kernel_times(self._h, ms), "fpt_kernel_times")
        return [float(v) for v in ms]

    def validate(self, db: DeviceBatch, out, flags=None, lazy=False, stream=None):
        """fpt_validate: uint8 [N] validity bits (VALID_*) of the solved
        paths `out` on the scene's finite objects. lazy: occlusion is tested
        only for paths with VALID_EXTENT and VALID_SPECULAR (VALIDATE_LAZY)."""
        import torch
        if flags is None:
            flags = torch.empty(db.N, dtype=torch.uint8, device="cuda")
        sc, pa, ou = db.c_scene(), db.c_paths(), self.c_out(out)
        _check(load_library().fpt_validate(
            self._h, ctypes.byref(sc), ctypes.byref(pa), ctypes.byref(ou),
            _ptr(flags), ctypes.c_int32(VALIDATE_LAZY if lazy else VALIDATE_ALL),
            _stream_ptr(stream)), "fpt_validate")
        return flags

    def enumerate(self, pair_src, pair_dst, K: int, order_min: int, order_max: int,
                  no_repeat: bool = True, rank0: int = 0, count: int | None = None,
                  n_max: int | None = None, out=None, stream=None):
        """fpt_enumerate: candidates of ranks rank0 .. rank0 + count - 1 as
        device tensors {src, dst, order, ids} in the fpt_paths layout.
        pair_src / pair_dst: int32 [P] device tensors of point indices."""
        import torch
        P = int(pair_src.shape[0])
        if int(pair_dst.shape[0]) != P:
            raise ValueError("pair_src and pair_dst differ in length")
        for name, t in (("pair_src", pair_src), ("pair_dst", pair_dst)):
            if t.dtype != torch.int32 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError(f"{name} must be a contiguous int32 device tensor")
        if count is None:
            count = enum_count(P, K, order_min, order_max, no_repeat) - int(rank0)
        n_max = int(order_max if n_max is None else n_max)
        if out is None:
            dev = pair_src.device
            out = {"src": torch.empty(count, dtype=torch.int32, device=dev),
                   "dst": torch.empty(count, dtype=torch.int32, device=dev),
                   "order": torch.empty(count, dtype=torch.uint8, device=dev),
                   "ids": torch.empty((n_max, count), dtype=torch.int32, device=dev)}
        sp = _enum_spec(P, K, order_min, order_max, no_repeat, pair_src, pair_dst)
        _check(load_library().fpt_enumerate(
            self._h, ctypes.byref(sp), ctypes.c_int64(int(rank0)), ctypes.c_int64(int(count)),
            _ptr(out["src"]), _ptr(out["dst"]), _ptr(out["order"]), _ptr(out["ids"]),
            ctypes.c_int32(n_max), _stream_ptr(stream)), "fpt_enumerate")
        return out

    def work_counts(self):
        """{order: (path evaluations, trial lengths, Newton solves, reduced-path
        evaluations, reduced-path trial lengths, reduced-path Newton solves)}
        of the FP64 refinement and collapse step since the previous read
        (counted while timing is enabled)."""
        c = (ctypes.c_uint64 * 36)()
        _check(load_library().fpt_work_counts(self._h, c), "fpt_work_counts")
        return {n: tuple(int(c[6 * (n - 1) + k]) for k in range(6)) for n in range(1, 7)}

    def set_launch(self, order: int, cfg: dict | None):
        """Per-order launch configuration (see fpt_launch_cfg); None resets."""
        lib = load_library()
        if cfg is None:
            _check(lib.fpt_set_launch(self._h, int(order), None), "fpt_set_launch")
            return
        c = _LaunchCfg()
        c.wg_per_cu = int(cfg.get("wg_per_cu", 0))
        c.refine_wg_per_cu = int(cfg.get("refine_wg_per_cu", 0))
        c.use_override = 1 if any(k in cfg for k in (
            "early_exit", "iters", "quick_steps", "quick_passes")) else 0
        c.early_exit = int(cfg.get("early_exit", 0))
        c.iters = int(cfg.get("iters", 0))
        c.quick_steps = int(cfg.get("quick_steps", 0))
        c.quick_passes = int(cfg.get("quick_passes", 0))
        st = list(cfg.get("stage_iters", [16, 16, 32]))
        for i in range(4):
            c.stage_iters[i] = int(st[i]) if i < len(st) else 0
        _check(lib.fpt_set_launch(self._h, int(order), ctypes.byref(c)), "fpt_set_launch")

    def capture(self, db: DeviceBatch, opts, out, stream):
        """HIP graph of one fpt_solve on `stream` (a torch.cuda.Stream that
        is not the default stream); returns a Graph."""
        sc, pa, oc, ou = db.c_scene(), db.c_paths(), opts.to_c(), self.c_out(out)
        g = ctypes.c_void_p()
        _check(load_library().fpt_graph_capture(
            self._h, ctypes.byref(sc), ctypes.byref(pa), ctypes.byref(oc),
            ctypes.byref(ou), _stream_ptr(stream), ctypes.byref(g)),
            "fpt_graph_capture")
        return Graph(g, keep=(self, db, opts, out))

    def alloc_out(self, db: DeviceBatch):
        import torch
        dev = db.obj.device
        N, n = db.N, db.n_max
        return dict(
            x=torch.empty((n, 3, N), dtype=torch.float32, device=dev),
            len=torch.empty((N,), dtype=torch.float32, device=dev),
            t=torch.empty((n, 2, N), dtype=torch.float32, device=dev),
            status=torch.empty((N,), dtype=torch.uint8, device=dev),
            iters=torch.empty((N,), dtype=torch.int16, device=dev),
        )

    @staticmethod
    def c_out(out) -> _Out:
        return _Out(_ptr(out["x"]), _ptr(out["len"]), _ptr(out["t"]),
                    _ptr(out["status"]), _ptr(out["iters"]))

    def solve(self, db: DeviceBatch, opts: Opts | None = None, out=None,
              stream=None):
        """fpt_solve on db; returns the output tensors (async on stream)."""
        if opts is None:
            opts = Opts(scale=db.S)
        if out is None:
            out = self.alloc_out(db)
        sc, pa, oc, ou = db.c_scene(), db.c_paths(), opts.to_c(), self.c_out(out)
        _check(load_library().fpt_solve(self._h, ctypes.byref(sc),
                                        ctypes.byref(pa), ctypes.byref(oc),
                                        ctypes.byref(ou), _stream_ptr(stream)),
               "fpt_solve")
        return out

    def solve_noalloc(self, db: DeviceBatch, opts: Opts | None = None, out=None,
                      stream=None):
        """fpt_solve_noalloc: fpt_solve in the library's fixed per-GPU
        scratch memory (no device allocation by the library; at most
        noalloc_max_paths() paths, no early exit, every unit on `stream`).
        `out` is allocated here by torch if it is not given."""
        if opts is None:
            opts = Opts(scale=db.S)
        if out is None:
            out = self.alloc_out(db)
        sc, pa, oc, ou = db.c_scene(), db.c_paths(), opts.to_c(), self.c_out(out)
        _check(load_library().fpt_solve_noalloc(self._h, ctypes.byref(sc),
                                                ctypes.byref(pa), ctypes.byref(oc),
                                                ctypes.byref(ou), _stream_ptr(stream)),
               "fpt_solve_noalloc")
        return out

    @staticmethod
    def noalloc_max_paths() -> int:
        return int(load_library().fpt_noalloc_max_paths())

    def grad(self, db: DeviceBatch, fwd, g_len=None, g_x=None, g_pts=None,
             g_obj=None, g_slot=None, g_end=None, stream=None):
        """fpt_grad: accumulates into g_pts [3][Q] and g_obj [9][K]."""
        import torch
        dev = db.obj.device
        if g_pts is None:
            g_pts = torch.zeros((3, db.Q), dtype=torch.float32, device=dev)
        if g_obj is None:
            g_obj = torch.zeros((9, db.K), dtype=torch.float32, device=dev)
        sc, pa, ou = db.c_scene(), db.c_paths(), self.c_out(fwd)
        _check(load_library().fpt_grad(
            self._h, ctypes.byref(sc), ctypes.byref(pa), ctypes.byref(ou),
            _ptr(g_len), _ptr(g_x), _ptr(g_pts), _ptr(g_obj), _ptr(g_slot),
            _ptr(g_end), _stream_ptr(stream)), "fpt_grad")
        return g_pts, g_obj


class Mlp:
    """Learned initialiser state on the device (fpt_mlp_*)."""

    def __init__(self, solver: Solver, seed: int = 0, stream=None):
        import torch
        lib = load_library()
        self.solver = solver
        n = int(lib.fpt_mlp_state_floats())
        self.state = torch.empty(n, dtype=torch.float32, device="cuda")
        _check(lib.fpt_mlp_init(solver._h, _ptr(self.state), int(seed),
                                _stream_ptr(stream)), "fpt_mlp_init")
        self.step = 0

    def weights(self):
        return self.state[:MLP_PARAMS]

    def grad(self):
        return self.state[3 * MLP_PARAMS:4 * MLP_PARAMS]

    def train_step(self, db: DeviceBatch, target, scale: float, lr: float,
                   loss_acc, stream=None):
        """One Adam step on the batch db (order 4) against solver output
        `target`; adds the batch loss to the device scalar loss_acc."""
        self.step += 1
        sc, pa, ou = db.c_scene(), db.c_paths(), Solver.c_out(target)
        _check(load_library().fpt_mlp_train_step(
            self.solver._h, _ptr(self.state), ctypes.byref(sc), ctypes.byref(pa),
            ctypes.byref(ou), float(scale), float(lr), int(self.step),
            _ptr(loss_acc), _stream_ptr(stream)), "fpt_mlp_train_step")

    def infer(self, db: DeviceBatch, scale: float, out=None, stream=None):
        """t_init [4][2][N] for db's paths."""
        import torch
        if out is None:
            out = torch.empty((4, 2, db.N), dtype=torch.float32, device="cuda")
        sc, pa = db.c_scene(), db.c_paths()
        _check(load_library().fpt_mlp_infer(
            self.solver._h, _ptr(self.state), ctypes.byref(sc), ctypes.byref(pa),
            float(scale), _ptr(out), _stream_ptr(stream)), "fpt_mlp_infer")
        return out


class Graph:
    """A captured fpt_solve (fpt_graph_*)."""

    def __init__(self, handle, keep):
        self._g = handle
        # the solver whose workspace the graph records (destroyed after the
        # graph), and the buffers the graph reads and writes
        self._keep = keep

    def launch(self, stream=None):
        _check(load_library().fpt_graph_launch(self._g, _stream_ptr(stream)),
               "fpt_graph_launch")

    def close(self):
        if getattr(self, "_g", None):
            load_library().fpt_graph_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
