"""The C-ABI library loads on the CPU, exports every entry point that
include/hj.h declares, and rejects invalid arguments before touching a
device (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hj.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hj_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("hj_grid_create", "hj_set_dynamics", "hj_set_scheme", "hj_solve", "hj_step",
                 "hj_solve_batch", "hj_get_info", "hj_grid_destroy", "hj_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2507_11542_amd import hj

    lib = hj.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert "gfx950" in hj.hj_version()


def test_argument_errors_without_device():
    from paper_2507_11542_amd import hj

    lib = hj.lib()
    out = ctypes.c_void_p()
    n = (ctypes.c_int64 * 3)(11, 11, 11)
    lo = (ctypes.c_double * 3)(0, 0, 0)
    hi = (ctypes.c_double * 3)(1, 1, 1)
    bad_hi = (ctypes.c_double * 3)(1, -1, 1)
    assert lib.hj_grid_create(0, n, lo, hi, 0, 0, ctypes.byref(out)) == hj.HJ_E_ARG
    assert lib.hj_grid_create(5, n, lo, hi, 0, 0, ctypes.byref(out)) == hj.HJ_E_ARG
    assert lib.hj_grid_create(3, n, lo, bad_hi, 0, 0, ctypes.byref(out)) == hj.HJ_E_ARG
    assert "lo < hi" in hj.hj_last_error()
    assert lib.hj_grid_create(3, n, lo, hi, 1 << 3, 0, ctypes.byref(out)) == hj.HJ_E_ARG
    assert lib.hj_grid_create(3, n, lo, hi, 0, 7, ctypes.byref(out)) == hj.HJ_E_ARG
    small = (ctypes.c_int64 * 3)(2, 11, 11)
    assert lib.hj_grid_create(3, small, lo, hi, 0, 0, ctypes.byref(out)) == hj.HJ_E_ARG
    huge = (ctypes.c_int64 * 3)(2048, 2048, 1024)
    assert lib.hj_grid_create(3, huge, lo, hi, 0, 0, ctypes.byref(out)) == hj.HJ_E_ARG
    assert lib.hj_set_dynamics(None, 0, None, 0) == hj.HJ_E_ARG
    assert lib.hj_set_scheme(None, 5, 3, 0.8) == hj.HJ_E_ARG
    assert lib.hj_solve(None, None, None, 0.0, 1.0, 0, None) == hj.HJ_E_ARG
    assert lib.hj_solve_noalloc(None, None, None, 0.0, 1.0, 0, None) == hj.HJ_E_ARG
    ts = (ctypes.c_double * 2)(0.5, 1.0)
    assert lib.hj_solve_outputs(None, None, None, 0.0, ts, 2, 0, None) == hj.HJ_E_ARG
    shp = hj.make_shapes([dict(kind="sphere", radius=1.0)])
    assert lib.hj_init_shapes(None, None, ctypes.cast(shp, ctypes.c_void_p), 1,
                              None) == hj.HJ_E_ARG
    assert lib.hj_step(None, None, None, None, 1.0, 0, None, None) == hj.HJ_E_ARG
    assert lib.hj_rhs(None, None, None, None) == hj.HJ_E_ARG
    assert lib.hj_get_info(None, None, None, None) == hj.HJ_E_ARG
    assert lib.hj_set_check(None, hj.HJ_CHECK_FINITE) == hj.HJ_E_ARG
    assert lib.hj_tube_finish(None, None, None, None, 1, -1.0, None) == hj.HJ_E_ARG
    assert lib.hj_solve_mixed(None, None, None, 0.0, 1.0, 1, -1.0, None) == hj.HJ_E_ARG
    assert lib.hj_batch_config(None, 4096, 1024, 1) == hj.HJ_E_ARG
    assert lib.hj_solve_batch(None, 1, None, None, None, None, None, None, None) == hj.HJ_E_ARG
    assert lib.hj_batch_wait(None, None, None, None) == hj.HJ_E_ARG
    assert lib.hj_grid_destroy(None) == hj.HJ_OK
    assert lib.hj_batch_destroy(None) == hj.HJ_OK


def test_no_device_is_reported():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2507_11542_amd import hj

    lib = hj.lib()
    out = ctypes.c_void_p()
    n = (ctypes.c_int64 * 2)(11, 11)
    lo = (ctypes.c_double * 2)(0, 0)
    hi = (ctypes.c_double * 2)(1, 1)
    rc = lib.hj_grid_create(2, n, lo, hi, 0, 0, ctypes.byref(out))
    assert rc in (hj.HJ_E_DEVICE, hj.HJ_E_OOM)
    assert not out.value


def test_injected_allocation_failure(monkeypatch):
    """HJ_FAULT_OOM=1 makes device allocations report HJ_E_OOM (checked before
    any allocator call, so it runs without a device too)."""
    import subprocess
    import sys

    code = ("import ctypes,sys; sys.path.insert(0, %r)\n"
            "from paper_2507_11542_amd import hj\n"
            "lib = hj.lib(); out = ctypes.c_void_p()\n"
            "n = (ctypes.c_int64*2)(11, 11); lo = (ctypes.c_double*2)(0, 0); "
            "hi = (ctypes.c_double*2)(1, 1)\n"
            "rc = lib.hj_grid_create(2, n, lo, hi, 0, 0, ctypes.byref(out))\n"
            "print(rc, hj.hj_last_error())\n" % ROOT)
    env = dict(os.environ, HJ_FAULT_OOM="1", HIP_VISIBLE_DEVICES=os.environ.get(
        "HIP_VISIBLE_DEVICES", ""))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=120)
    rc, msg = r.stdout.strip().split(" ", 1)
    assert int(rc) in (-2, -3)
