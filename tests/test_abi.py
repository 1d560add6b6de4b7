"""The C ABI: every function declared in include/*.h is exported by
libfpt.so and loads without a GPU (no compute calls here)."""
import ctypes
import glob
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"\b(fpt_\w+)\s*\(", src):
            names.add(m.group(1))
    return names


def test_library_exports_declared_symbols():
    from paper_2510_16172_amd import fpt
    lib = fpt.load_library()
    declared = _declared()
    assert {"fpt_solve", "fpt_grad", "fpt_create", "fpt_destroy",
            "fpt_default_opts", "fpt_last_error"} <= declared
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert set(fpt.EXPORTED) <= declared


def test_default_opts_and_struct_layout():
    from paper_2510_16172_amd import fpt
    lib = fpt.load_library()
    o = fpt._Opts()
    lib.fpt_default_opts(ctypes.byref(o))
    assert o.iters == 64 and o.fp_iters == 1 and o.n_levels == 4
    assert abs(o.level_eps[3] - 1e-9) < 1e-15 and o.level_steps[3] == 3
    assert abs(o.cert_rtol - 1e-5) < 1e-12
    # mirror of the C struct sizes (natural alignment, LP64)
    assert ctypes.sizeof(fpt._Scene) == 32
    assert ctypes.sizeof(fpt._Paths) == 56
    assert ctypes.sizeof(fpt._Out) == 40
    assert ctypes.sizeof(fpt._LaunchCfg) == 4 * 3 + 16 + 4 + 4 + 4 + 4
    assert ctypes.sizeof(fpt._Opts) == 4 * 6 + 4 * 8 * 2 + 4 + 16 + 4 + 4 + 4 + 4 + 4 + 4 + 4
    assert o.method == fpt.METHOD_BFGS and o.polish_steps == 1 and o.split == 0
    assert o.quick_steps == 2
    assert o.quick_passes == 2
    assert list(o.stage_iters) == [16, 16, 32, 0]


def test_create_without_gpu_fails_cleanly():
    """With no device visible fpt_create reports an error instead of
    crashing (skipped where a GPU is present)."""
    import pytest
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2510_16172_amd import fpt
    lib = fpt.load_library()
    h = ctypes.c_void_p()
    rc = lib.fpt_create(0, ctypes.byref(h))
    assert rc != 0 and not h.value
    assert lib.fpt_last_error()


def test_solve_rejects_bad_arguments_before_launch():
    """Whole-call argument errors return FPT_EINVAL without touching the
    device (a NULL handle is checked first)."""
    from paper_2510_16172_amd import fpt
    lib = fpt.load_library()
    sc, pa = fpt._Scene(), fpt._Paths()
    o = fpt._Opts()
    lib.fpt_default_opts(ctypes.byref(o))
    ou = fpt._Out()
    rc = lib.fpt_solve(None, ctypes.byref(sc), ctypes.byref(pa),
                       ctypes.byref(o), ctypes.byref(ou), None)
    assert rc == -1
    assert b"handle" in lib.fpt_last_error()


def test_enum_count_host_matches_oracle():
    """fpt_enum_count is host arithmetic: it runs without a GPU. Counts
    equal the enumeration oracle's; bad specs and totals above 2^62 are
    rejected."""
    import pytest
    from oracle import candidates as cand
    from paper_2510_16172_amd import fpt
    for P, K, lo, hi, nr in [(64, 313, 1, 2, True), (3, 5, 2, 4, False), (1, 1, 1, 6, True),
                             (7, 2, 1, 6, True), (64, 313, 1, 6, True), (2, 1000, 3, 6, False)]:
        assert fpt.enum_count(P, K, lo, hi, nr) == cand.total(P, K, lo, hi, nr)
    for bad in [(0, 5, 1, 2), (2, 0, 1, 2), (2, 5, 0, 2), (2, 5, 3, 2), (2, 5, 1, 7),
                (1 << 30, 1 << 20, 1, 6)]:
        with pytest.raises(fpt.FptError):
            fpt.enum_count(*bad)
    lib = fpt.load_library()
    sp = fpt._enum_spec(2, 5, 1, 2)
    rc = lib.fpt_enumerate(None, ctypes.byref(sp), 0, 1, None, None, None, None, 2, None)
    assert rc == -1 and b"handle" in lib.fpt_last_error()
