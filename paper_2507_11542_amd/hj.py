"""Python binding of libhj (include/hj.h): the same entry points, argument
marshalling only.  Every step of a solve runs in the gfx950 kernels of
libhj.so; there is no CPU fallback: importing this module without the built
library raises.

Device arrays are passed as torch CUDA(HIP) tensors or raw integer device
pointers; streams as torch.cuda.Stream or raw hipStream_t integers.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

_HERE = os.path.dirname(os.path.abspath(__file__))
# HJ_LIB_PATH: another build of the same library (the host-sanitizer tests
# load one); the default is the in-tree build
LIB_PATH = os.environ.get("HJ_LIB_PATH") or os.path.join(_HERE, "libhj.so")

# enum values of include/hj.h
HJ_OK, HJ_E_ARG, HJ_E_OOM, HJ_E_DEVICE, HJ_E_STATE, HJ_E_NUMERIC, HJ_E_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6
HJ_FP64, HJ_FP32 = 0, 1
HJ_SET, HJ_TUBE, HJ_TUBE_VI, HJ_TUBE_OUTPUTS = 0, 1, 2, 3
HJ_UPWIND1, HJ_ENO2, HJ_ENO3, HJ_WENO5 = 1, 2, 3, 5
HJ_RK1, HJ_RK2, HJ_RK3 = 1, 2, 3
HJ_DYN_TRANSLATION, HJ_DYN_BALL, HJ_DYN_DOUBLE_INTEGRATOR, HJ_DYN_REL_DUBINS, \
    HJ_DYN_DUBINS4D, HJ_DYN_ROCKETS = 0, 1, 2, 3, 4, 5

SPACE = {"upwind1": HJ_UPWIND1, "eno2": HJ_ENO2, "eno3": HJ_ENO3, "weno5": HJ_WENO5}
DYN = {"translation": HJ_DYN_TRANSLATION, "ball": HJ_DYN_BALL,
       "double_integrator": HJ_DYN_DOUBLE_INTEGRATOR, "rel_dubins": HJ_DYN_REL_DUBINS,
       "dubins4d": HJ_DYN_DUBINS4D, "rockets": HJ_DYN_ROCKETS}
MODE = {"set": HJ_SET, "tube": HJ_TUBE, "tube_vi": HJ_TUBE_VI, "tube_out": HJ_TUBE_OUTPUTS}
PREC = {"fp64": HJ_FP64, "fp32": HJ_FP32}

SHAPE = {"sphere": 0, "cylinder": 1, "box": 2, "ellipsoid": 3}
HJ_DISS_LF, HJ_DISS_LLF, HJ_DISS_GLF = 0, 1, 2
HJ_CHECK_FINITE = 1
DISSIPATION = {"lf": HJ_DISS_LF, "llf": HJ_DISS_LLF, "glf": HJ_DISS_GLF}
OP = {"union": 0, "intersect": 1, "subtract": 2}


class HjShape(ctypes.Structure):
    """struct hj_shape of include/hj.h"""
    _fields_ = [("kind", ctypes.c_int32), ("op", ctypes.c_int32), ("axes", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("center", ctypes.c_double * 4),
                ("size", ctypes.c_double * 4), ("radius", ctypes.c_double)]


def make_shapes(shape_list) -> "ctypes.Array":
    """hj_shape array from dicts with keys kind, op, axes (axis indices; empty
    = all), center, size, radius (the names of include/hj.h)."""
    arr = (HjShape * len(shape_list))()
    for s, d in zip(arr, shape_list):
        s.kind = SHAPE[d["kind"]]
        s.op = OP[d.get("op", "union")]
        s.axes = sum(1 << a for a in d.get("axes", ()))
        for i, c in enumerate(d.get("center", ())):
            s.center[i] = float(c)
        for i, c in enumerate(d.get("size", ())):
            s.size[i] = float(c)
        s.radius = float(d.get("radius", 0.0))
    return arr


STATUS_NAMES = {HJ_OK: "HJ_OK", HJ_E_ARG: "HJ_E_ARG", HJ_E_OOM: "HJ_E_OOM",
                HJ_E_DEVICE: "HJ_E_DEVICE", HJ_E_STATE: "HJ_E_STATE",
                HJ_E_NUMERIC: "HJ_E_NUMERIC", HJ_E_UNSUPPORTED: "HJ_E_UNSUPPORTED"}


class HJError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhj.so is not built (run paper_2507_11542_amd.build_lib); "
                          "there is no fallback path")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, U, I64 = (ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint32,
                       ctypes.c_int64)
    PD = ctypes.POINTER(ctypes.c_double)
    PI64 = ctypes.POINTER(ctypes.c_int64)
    lib.hj_grid_create.argtypes = [I, PI64, PD, PD, U, I, ctypes.POINTER(P)]
    lib.hj_set_dynamics.argtypes = [P, I, PD, I]
    lib.hj_set_scheme.argtypes = [P, I, I, D]
    lib.hj_solve.argtypes = [P, P, P, D, D, I, P]
    lib.hj_solve_noalloc.argtypes = [P, P, P, D, D, I, P]
    lib.hj_step.argtypes = [P, P, P, PD, D, I, PD, P]
    lib.hj_solve_mixed.argtypes = [P, P, P, D, D, I, D, P]
    lib.hj_tube_finish.argtypes = [P, P, P, P, I, D, P]
    lib.hj_solve_outputs.argtypes = [P, P, P, D, PD, I, I, P]
    lib.hj_set_dissipation.argtypes = [P, I]
    lib.hj_set_check.argtypes = [P, I]
    lib.hj_init_shapes.argtypes = [P, P, P, I, P]
    lib.hj_rhs.argtypes = [P, P, P, P]
    lib.hj_get_schedule.argtypes = [P, D, D, PD, PD, PI64, P]
    lib.hj_get_info.argtypes = [P, PD, PD, PI64]
    lib.hj_grid_destroy.argtypes = [P]
    lib.hj_grid_set_workspace.argtypes = [P, P, P]
    lib.hj_batch_create.argtypes = [ctypes.POINTER(P)]
    lib.hj_batch_config.argtypes = [P, I, I, I]
    lib.hj_solve_batch.argtypes = [P, I, ctypes.POINTER(P), ctypes.POINTER(P),
                                   ctypes.POINTER(P), PD, PD, ctypes.POINTER(I), P]
    lib.hj_step_batch.argtypes = [P, I, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P),
                                  PD, PD, PD, ctypes.POINTER(I), I, ctypes.POINTER(I),
                                  ctypes.POINTER(I), P]
    lib.hj_batch_wait.argtypes = [P, P, PD, PI64]
    lib.hj_batch_destroy.argtypes = [P]
    for name in ("hj_grid_create", "hj_set_dynamics", "hj_set_scheme", "hj_solve",
                 "hj_solve_noalloc", "hj_step",
                 "hj_solve_mixed", "hj_tube_finish", "hj_solve_outputs", "hj_init_shapes",
                 "hj_set_dissipation", "hj_set_check", "hj_rhs", "hj_get_schedule", "hj_get_info", "hj_grid_destroy", "hj_grid_set_workspace",
                 "hj_batch_create",
                 "hj_batch_config", "hj_solve_batch", "hj_step_batch", "hj_batch_wait",
                 "hj_batch_destroy"):
        getattr(lib, name).restype = I
    lib.hj_last_error.argtypes = []
    lib.hj_last_error.restype = ctypes.c_char_p
    lib.hj_version.argtypes = []
    lib.hj_version.restype = ctypes.c_char_p
    return lib


_lib = _load()


def lib() -> ctypes.CDLL:
    return _lib


def hj_last_error() -> str:
    return _lib.hj_last_error().decode()


def hj_version() -> str:
    return _lib.hj_version().decode()


def _check(status: int):
    if status != HJ_OK:
        raise HJError(status, hj_last_error())


def _ptr(x) -> Optional[int]:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _check_array(x, dtype_name: str, numel: int, what: str):
    """A tensor passed as a device array must be a contiguous GPU tensor of
    the element type and node count the call expects (raw integer pointers
    are the caller's responsibility).  Raises ValueError before any library
    call, so a wrong tensor never reaches a kernel."""
    if x is None or isinstance(x, int):
        return
    dt = str(getattr(x, "dtype", ""))
    if not dt.endswith(dtype_name):
        raise ValueError("%s: dtype %s, expected %s" % (what, dt or type(x).__name__, dtype_name))
    if x.numel() != numel:
        raise ValueError("%s: %d elements, expected %d" % (what, x.numel(), numel))
    if not x.is_contiguous():
        raise ValueError("%s: not contiguous" % what)
    if not x.is_cuda:
        raise ValueError("%s: not a GPU tensor" % what)


def _stream(s) -> Optional[int]:
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _darr(vals: Sequence[float]):
    return (ctypes.c_double * max(1, len(vals)))(*vals)


def hj_grid_create(N: Sequence[int], lo: Sequence[float], hi: Sequence[float],
                   periodic_mask: int = 0, prec: int = HJ_FP64) -> ctypes.c_void_p:
    nd = len(N)
    n = (ctypes.c_int64 * nd)(*[int(v) for v in N])
    h = ctypes.c_void_p()
    _check(_lib.hj_grid_create(nd, n, _darr(lo), _darr(hi), int(periodic_mask), int(prec),
                               ctypes.byref(h)))
    return h


def hj_set_dynamics(g, kind: int, params: Sequence[float]):
    _check(_lib.hj_set_dynamics(g, int(kind), _darr(list(params)), len(params)))


def hj_set_scheme(g, space: int = HJ_WENO5, time: int = HJ_RK3, cfl: float = 0.8):
    _check(_lib.hj_set_scheme(g, int(space), int(time), float(cfl)))


def hj_solve(g, V0, V_out, t0: float, tf: float, mode: int = HJ_SET, stream=None):
    _check(_lib.hj_solve(g, _ptr(V0), _ptr(V_out), float(t0), float(tf), int(mode),
                         _stream(stream)))


def hj_solve_noalloc(g, V0, V_out, t0: float, tf: float, mode: int = HJ_SET, stream=None):
    _check(_lib.hj_solve_noalloc(g, _ptr(V0), _ptr(V_out), float(t0), float(tf), int(mode),
                                 _stream(stream)))


def hj_set_dissipation(g, kind: int = HJ_DISS_LF):
    _check(_lib.hj_set_dissipation(g, int(kind)))


def hj_set_check(g, flags: int = HJ_CHECK_FINITE):
    _check(_lib.hj_set_check(g, int(flags)))


def hj_init_shapes(g, V_out, shape_list, stream=None):
    arr = make_shapes(shape_list)
    _check(_lib.hj_init_shapes(g, _ptr(V_out), ctypes.cast(arr, ctypes.c_void_p), len(arr),
                               _stream(stream)))


def hj_solve_outputs(g, V0, V_outs, t0: float, times: Sequence[float], mode: int = HJ_SET,
                     stream=None):
    ts = (ctypes.c_double * len(times))(*[float(t) for t in times])
    _check(_lib.hj_solve_outputs(g, _ptr(V0), _ptr(V_outs), float(t0), ts, len(times),
                                 int(mode), _stream(stream)))


def hj_solve_mixed(g, V0, V_out, t0: float, tf: float, mode: int = HJ_SET, band: float = -1.0,
                   stream=None):
    _check(_lib.hj_solve_mixed(g, _ptr(V0), _ptr(V_out), float(t0), float(tf), int(mode),
                               float(band), _stream(stream)))


def hj_tube_finish(g, V32, V0, V_out, mode: int = HJ_SET, band: float = -1.0, stream=None):
    _check(_lib.hj_tube_finish(g, _ptr(V32), _ptr(V0), _ptr(V_out), int(mode), float(band),
                               _stream(stream)))


def hj_step(g, V, V0, t: float, tf: float, mode: int = HJ_SET, stream=None
            ) -> Tuple[float, float]:
    tt = ctypes.c_double(t)
    dt = ctypes.c_double(0.0)
    _check(_lib.hj_step(g, _ptr(V), _ptr(V0), ctypes.byref(tt), float(tf), int(mode),
                        ctypes.byref(dt), _stream(stream)))
    return tt.value, dt.value


def hj_rhs(g, V, L_out, stream=None):
    _check(_lib.hj_rhs(g, _ptr(V), _ptr(L_out), _stream(stream)))


def hj_get_schedule(g, t0: float, tf: float, ndim: int, stream=None):
    alpha = (ctypes.c_double * 4)()
    dt = ctypes.c_double(0.0)
    steps = ctypes.c_int64(0)
    _check(_lib.hj_get_schedule(g, float(t0), float(tf), alpha, ctypes.byref(dt),
                                ctypes.byref(steps), _stream(stream)))
    return [alpha[k] for k in range(ndim)], dt.value, steps.value


def hj_get_info(g, ndim: int):
    """(alpha, dt, steps of the last solve) of a grid handle."""
    alpha = (ctypes.c_double * 4)()
    dt = ctypes.c_double(0.0)
    steps = ctypes.c_int64(0)
    _check(_lib.hj_get_info(g, alpha, ctypes.byref(dt), ctypes.byref(steps)))
    return [alpha[k] for k in range(ndim)], dt.value, steps.value


def hj_grid_destroy(g):
    _check(_lib.hj_grid_destroy(g))


def hj_grid_set_workspace(g, A, B):
    _check(_lib.hj_grid_set_workspace(g, _ptr(A), _ptr(B)))


def hj_batch_create() -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(_lib.hj_batch_create(ctypes.byref(h)))
    return h


def hj_batch_config(b, tile_nodes: int = 256, workgroups: int = 0, use_graph: bool = True):
    _check(_lib.hj_batch_config(b, int(tile_nodes), int(workgroups), 1 if use_graph else 0))


def hj_solve_batch(b, grids, V0s, Vouts, t0s, tfs, modes, stream=None):
    n = len(grids)
    P = ctypes.c_void_p
    ga = (P * n)(*[g.value if isinstance(g, ctypes.c_void_p) else g for g in grids])
    va = (P * n)(*[_ptr(v) for v in V0s])
    oa = (P * n)(*[_ptr(v) for v in Vouts])
    ta = (ctypes.c_double * n)(*[float(t) for t in t0s])
    fa = (ctypes.c_double * n)(*[float(t) for t in tfs])
    ma = (ctypes.c_int * n)(*[int(m) for m in modes])
    _check(_lib.hj_solve_batch(b, n, ga, va, oa, ta, fa, ma, _stream(stream)))


def hj_step_batch(b, grids, V0s, Vs, t0s, ts, tfs, modes, max_steps, stream=None):
    """Advances each instance in place by up to max_steps steps from ts[i];
    returns (new times, steps taken, finished flags)."""
    n = len(grids)
    P = ctypes.c_void_p
    ga = (P * n)(*[g.value if isinstance(g, ctypes.c_void_p) else g for g in grids])
    va = (P * n)(*[_ptr(v) for v in V0s]) if V0s is not None else None
    oa = (P * n)(*[_ptr(v) for v in Vs])
    t0a = (ctypes.c_double * n)(*[float(t) for t in t0s])
    ta = (ctypes.c_double * n)(*[float(t) for t in ts])
    fa = (ctypes.c_double * n)(*[float(t) for t in tfs])
    ma = (ctypes.c_int * n)(*[int(m) for m in modes])
    taken = (ctypes.c_int * n)()
    done = (ctypes.c_int * n)()
    _check(_lib.hj_step_batch(b, n, ga, va, oa, t0a, ta, fa, ma, int(max_steps), taken, done,
                              _stream(stream)))
    return ([ta[k] for k in range(n)], [taken[k] for k in range(n)],
            [bool(done[k]) for k in range(n)])


def hj_batch_wait(b, n: int, stream=None):
    """Waits for the last batch; returns (final times, work items)."""
    tf = (ctypes.c_double * max(1, n))()
    items = ctypes.c_int64(0)
    _check(_lib.hj_batch_wait(b, _stream(stream), tf, ctypes.byref(items)))
    return [tf[k] for k in range(n)], items.value


def hj_batch_destroy(b):
    _check(_lib.hj_batch_destroy(b))


class Batch:
    """Owning wrapper of one hj_batch_t (marshalling only)."""

    def __init__(self, tile_nodes=256, workgroups=0, use_graph=True):
        self.handle = hj_batch_create()
        self.config(tile_nodes, workgroups, use_graph)

    def config(self, tile_nodes=256, workgroups=0, use_graph=True):
        self.tile_nodes, self.workgroups, self.use_graph = tile_nodes, workgroups, use_graph
        hj_batch_config(self.handle, tile_nodes, workgroups, use_graph)

    @staticmethod
    def _check(grids, *arrays):
        for arr, what in arrays:
            if arr is None:
                continue
            if len(arr) != len(grids):
                raise ValueError("%s: %d arrays for %d grids" % (what, len(arr), len(grids)))
            for i, (g, x) in enumerate(zip(grids, arr)):
                g._check(x, "%s[%d]" % (what, i))

    def solve(self, grids, V0s, Vouts, t0s, tfs, modes, stream=None):
        self._check(grids, (V0s, "V0s"), (Vouts, "Vouts"))
        hj_solve_batch(self.handle, [g.handle for g in grids], V0s, Vouts, t0s, tfs,
                       [MODE[m] if isinstance(m, str) else m for m in modes], stream)

    def step(self, grids, V0s, Vs, t0s, ts, tfs, modes, max_steps, stream=None):
        self._check(grids, (V0s, "V0s"), (Vs, "Vs"))
        return hj_step_batch(self.handle, [g.handle for g in grids], V0s, Vs, t0s, ts, tfs,
                             [MODE[m] if isinstance(m, str) else m for m in modes], max_steps,
                             stream)

    def wait(self, n, stream=None):
        return hj_batch_wait(self.handle, n, stream)

    def close(self):
        if self.handle is not None:
            hj_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Grid:
    """Owning wrapper of one hj_grid_t (marshalling only)."""

    def __init__(self, n, lo, hi, periodic=None, prec="fp64"):
        periodic = periodic or [False] * len(n)
        mask = sum(1 << d for d, p in enumerate(periodic) if p)
        self.n = tuple(int(v) for v in n)
        self.prec = prec
        self.handle = hj_grid_create(self.n, lo, hi, mask, PREC[prec])

    @classmethod
    def from_problem(cls, p, prec="fp64") -> "Grid":
        g = cls(p.n, p.lo, p.hi, p.periodic, prec)
        g.set_dynamics(p.dynamics, p.params)
        g.set_scheme(p.scheme, p.order, p.cfl)
        g.set_dissipation(getattr(p, "diss", "lf"))
        return g

    @property
    def points(self) -> int:
        n = 1
        for v in self.n:
            n *= v
        return n

    def _check(self, x, what, dtype=None, count=1):
        _check_array(x, dtype or ("float64" if self.prec == "fp64" else "float32"),
                     count * self.points, what)

    def set_dynamics(self, name: str, params):
        hj_set_dynamics(self.handle, DYN[name], params)

    def set_scheme(self, space="weno5", order=3, cfl=0.8):
        hj_set_scheme(self.handle, SPACE[space], int(order), cfl)

    def set_dissipation(self, kind="lf"):
        hj_set_dissipation(self.handle, DISSIPATION[kind])

    def set_check(self, finite: bool = True):
        """Scan solve results for NaN/Inf (HJ_E_NUMERIC raises HJError)."""
        hj_set_check(self.handle, HJ_CHECK_FINITE if finite else 0)

    def solve(self, V0, V_out, t0, tf, mode="set", stream=None):
        self._check(V0, "V0")
        self._check(V_out, "V_out")
        hj_solve(self.handle, V0, V_out, t0, tf, MODE[mode], stream)

    def solve_noalloc(self, V0, V_out, t0, tf, mode="set", stream=None):
        """hj_solve with the stage buffers in the library's static scratch."""
        self._check(V0, "V0")
        self._check(V_out, "V_out")
        hj_solve_noalloc(self.handle, V0, V_out, t0, tf, MODE[mode], stream)

    def init_shapes(self, V_out, shape_list, stream=None):
        """V_out <- the implicit surface of shape_list (dicts as in make_shapes)."""
        self._check(V_out, "V_out")
        hj_init_shapes(self.handle, V_out, shape_list, stream)

    def solve_outputs(self, V0, V_outs, t0, times, mode="set", stream=None):
        """V_outs: device array of len(times) * prod(n) elements (for example a
        tensor of shape (len(times),) + n)."""
        self._check(V0, "V0")
        self._check(V_outs, "V_outs", count=len(times))
        hj_solve_outputs(self.handle, V0, V_outs, t0, times, MODE[mode], stream)

    def step(self, V, V0, t, tf, mode="set", stream=None):
        self._check(V, "V")
        self._check(V0, "V0")
        return hj_step(self.handle, V, V0, t, tf, MODE[mode], stream)

    def solve_mixed(self, V0, V_out, t0, tf, mode="set", band=-1.0, stream=None):
        self._check(V0, "V0", "float64")
        self._check(V_out, "V_out", "float64")
        hj_solve_mixed(self.handle, V0, V_out, t0, tf, MODE[mode], band, stream)

    def tube_finish(self, V32, V0, V_out, mode="set", band=-1.0, stream=None):
        self._check(V32, "V32", "float32")
        self._check(V0, "V0", "float64")
        self._check(V_out, "V_out", "float64")
        hj_tube_finish(self.handle, V32, V0, V_out, MODE[mode], band, stream)

    def rhs(self, V, L_out, stream=None):
        self._check(V, "V")
        self._check(L_out, "L_out")
        hj_rhs(self.handle, V, L_out, stream)

    def set_workspace(self, A, B):
        self._check(A, "A")
        self._check(B, "B")
        hj_grid_set_workspace(self.handle, A, B)
        self._workspace = (A, B)  # keep the tensors alive with the grid

    def schedule(self, t0, tf, stream=None):
        return hj_get_schedule(self.handle, t0, tf, len(self.n), stream)

    def info(self):
        """(alpha, dt, RK steps of the last solve)."""
        return hj_get_info(self.handle, len(self.n))

    def close(self):
        if self.handle is not None:
            hj_grid_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
