"""hj_solve_noalloc (stage buffers in the library's static device scratch)
through the C ABI against hj_solve: bit for bit on two calls in a row, the
second on a smaller grid (the scratch keeps the first call's contents), in
FP64 and FP32; no device memory taken by the call; grids whose stage buffers
exceed the scratch, and GLF, refused before any work."""
import ctypes

import numpy as np
import pytest

from paper_2507_11542_amd import inputs

pytestmark = pytest.mark.gpu


def _scratch_ready(lib, hj, torch, to_dev):
    """One small call first: the static array is brought to the device, and
    its address taken, at the entry point's first call on a device (it then
    stays until the process ends), so later calls can be checked for taking
    no memory."""
    q = inputs.rel_dubins_3d(n=(9, 9, 9), tf=0.05)
    g = hj.Grid.from_problem(q, "fp64")
    d0 = to_dev(q.v0())
    out = torch.empty_like(d0)
    try:
        rc = lib.hj_solve_noalloc(g.handle, ctypes.c_void_p(d0.data_ptr()),
                                  ctypes.c_void_p(out.data_ptr()), 0.0, 0.05, hj.HJ_TUBE,
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert rc == hj.HJ_OK, hj.hj_last_error()
        torch.cuda.synchronize()
    finally:
        g.close()


def _solve_pair(p, prec, lib, hj, torch, to_dev):
    """(hj_solve result, hj_solve_noalloc result) of p on fresh handles; the
    no-alloc handle never runs hj_solve, so it owns no stage buffers."""
    d0 = to_dev(p.v0(), prec)
    ref, out = torch.empty_like(d0), torch.full_like(d0, float("nan"))
    st = torch.cuda.current_stream()
    g = hj.Grid.from_problem(p, prec)
    try:
        g.solve(d0, ref, p.t0, p.tf, p.mode, st)
        torch.cuda.synchronize()
    finally:
        g.close()
    h = hj.Grid.from_problem(p, prec)
    try:
        free0 = torch.cuda.mem_get_info()[0]
        rc = lib.hj_solve_noalloc(h.handle, ctypes.c_void_p(d0.data_ptr()),
                                  ctypes.c_void_p(out.data_ptr()), float(p.t0), float(p.tf),
                                  hj.MODE[p.mode], ctypes.c_void_p(st.cuda_stream))
        assert rc == hj.HJ_OK, hj.hj_last_error()
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        _, _, steps = h.info()
    finally:
        h.close()
    # the stage buffers of this grid would be >= 2 MB; nothing of that size was taken
    assert free1 >= free0 - (1 << 20), (free0, free1)
    return ref.cpu().numpy(), out.cpu().numpy(), steps


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_equals_solve_two_calls(prec):
    import torch

    from gpu_util import to_dev
    from paper_2507_11542_amd import hj

    lib = hj.lib()
    _scratch_ready(lib, hj, torch, to_dev)
    big = inputs.rel_dubins_3d(n=(61, 57, 50), tf=0.4)
    small = inputs.rel_dubins_3d(n=(23, 19, 17), tf=0.3, ve=4.0, we=1.3)
    for p in (big, small):
        print("case", prec, p.n, flush=True)
        ref, got, steps = _solve_pair(p, prec, lib, hj, torch, to_dev)
        assert steps > 0
        assert np.array_equal(ref, got), (prec, p.n, float(np.abs(ref - got).max()))


def test_noalloc_rk2_eno2_double_integrator():
    import torch

    from gpu_util import to_dev
    from paper_2507_11542_amd import hj

    p = inputs.double_integrator_2d(n=201, tf=0.5)
    print("case", p.n, p.scheme, p.order, flush=True)
    _scratch_ready(hj.lib(), hj, torch, to_dev)
    ref, got, _ = _solve_pair(p, "fp64", hj.lib(), hj, torch, to_dev)
    assert np.array_equal(ref, got)


def test_noalloc_refuses_what_does_not_fit():
    import torch

    from gpu_util import to_dev
    from paper_2507_11542_amd import hj

    lib = hj.lib()
    st = torch.cuda.current_stream()
    # 205^3 FP64 nodes: RK3 stage buffers of 138 MB > 128 MiB; nothing enqueued
    p = inputs.rel_dubins_3d(n=205, tf=0.1)
    g = hj.Grid.from_problem(p, "fp64")
    d0 = torch.zeros(p.points, dtype=torch.float64, device="cuda")
    out = torch.empty_like(d0)
    try:
        rc = lib.hj_solve_noalloc(g.handle, ctypes.c_void_p(d0.data_ptr()),
                                  ctypes.c_void_p(out.data_ptr()), 0.0, 0.1, hj.HJ_TUBE,
                                  ctypes.c_void_p(st.cuda_stream))
        assert rc == hj.HJ_E_ARG and "static scratch" in hj.hj_last_error()
    finally:
        g.close()
    # GLF keeps per-stage reduction buffers
    q = inputs.rel_dubins_3d(n=(11, 11, 11), tf=0.1).with_(diss="glf")
    g = hj.Grid.from_problem(q, "fp64")
    d0 = to_dev(q.v0())
    out = torch.empty_like(d0)
    try:
        rc = lib.hj_solve_noalloc(g.handle, ctypes.c_void_p(d0.data_ptr()),
                                  ctypes.c_void_p(out.data_ptr()), 0.0, 0.1, hj.HJ_TUBE,
                                  ctypes.c_void_p(st.cuda_stream))
        assert rc == hj.HJ_E_UNSUPPORTED
    finally:
        g.close()
