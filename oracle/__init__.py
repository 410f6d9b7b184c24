"""Plain FP64 CPU oracle for the explicit level-set time step of arXiv 2507.11542.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The product path never imports
this package, and this package imports nothing from the product.

The arithmetic lives in ``hj_oracle.c`` (plain scalar loops, FP64); this module
only marshals numpy arrays through ctypes.  ``build()`` compiles it with gcc.
Functions and the paper passages they follow:

- ``schedule``  alpha, CFL dt and step count          (Sec. 4 CFL condition, Sec. 5 time loop)
- ``derivs``    one-sided derivatives along one axis   (Sec. 3, 3.1, 3.2, 3.3)
- ``rhs_at``    L(V) = -Hhat at chosen nodes          (Sec. 4 Lax-Friedrichs)
- ``steps``     fixed-size TVD-RK steps               (Sec. 5 odeCFL listing)
- ``solve``     full CFL-constrained solve over tspan (Sec. 5, Sec. 6.1 tube)
- ``solve_outputs`` the same through a list of output times (Sec. 6.1, the
                global steps of the rockets game)
- ``shapes``    implicit-surface initial values and their Boolean
                combinations (Sec. 2.2, Fig. 4)
- ``set_dissipation`` Lax-Friedrichs coefficients from the control sets (LF),
                the node's costate box (LLF) or the grid-wide one (GLF) (Sec. 4)

Every function is pinned by a ``-m "not gpu"`` test against closed forms,
invariants, polynomial reproduction, convergence order or brute force; the
values of the relative-Dubins and 4-D Dubins solves away from the front are
"parity unpinned" (no closed form exists; the pins constrain them only through
the shared operators and symmetries).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hj_oracle.c")
_LIB = os.path.join(_HERE, "libhj_oracle.so")
# a test may point the shim at a deliberately mutated build of the oracle
_LIB = os.environ.get("HJ_ORACLE_LIB", _LIB)

SCHEMES = {"upwind1": 1, "eno2": 2, "eno3": 3, "weno5": 5}
DYNAMICS = {"translation": 0, "ball": 1, "double_integrator": 2,
            "rel_dubins": 3, "dubins4d": 4, "rockets": 5}
MODES = {"set": 0, "tube": 1, "tube_vi": 2, "tube_out": 3}
SHAPES = {"sphere": 0, "cylinder": 1, "box": 2, "ellipsoid": 3}
OPS = {"union": 0, "intersect": 1, "subtract": 2}
DISSIPATION = {"lf": 0, "llf": 1, "glf": 2}

_lib = None


def build() -> str:
    """Compile the oracle with gcc (IEEE FP64, no contraction, OpenMP loops)."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-std=c99", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    I = ctypes.c_int
    L = ctypes.c_long
    D = ctypes.c_double
    U = ctypes.c_uint
    lib.orc_schedule.argtypes = [I, P, P, P, U, I, P, I, D, D, D, P, P, P, P]
    lib.orc_schedule.restype = I
    lib.orc_derivs.argtypes = [I, P, P, P, U, I, I, P, P, P]
    lib.orc_derivs.restype = I
    lib.orc_rhs_at.argtypes = [I, P, P, P, U, I, P, I, I, P, P, L, P, P]
    lib.orc_rhs_at.restype = I
    lib.orc_steps.argtypes = [I, P, P, P, U, I, P, I, I, I, P, D, L, P, P, I]
    lib.orc_steps.restype = I
    lib.orc_solve.argtypes = [I, P, P, P, U, I, P, I, I, I, D, P, P, D, D, I, P, P]
    lib.orc_solve.restype = L
    lib.orc_solve_outputs.argtypes = [I, P, P, P, U, I, P, I, I, I, D, P, D, P, L, I, P]
    lib.orc_solve_outputs.restype = L
    lib.orc_shapes.argtypes = [I, P, P, P, U, I, P, P, P, P, P, P, P]
    lib.orc_shapes.restype = I
    lib.orc_box_bound.argtypes = [I, P, P, P, U, I, P, I, L, I, P, P]
    lib.orc_box_bound.restype = D
    lib.orc_set_dissipation.argtypes = [I]
    lib.orc_set_dissipation.restype = I
    lib.orc_set_threads.argtypes = [I]
    lib.orc_set_threads.restype = I
    lib.orc_set_storage_model.argtypes = [I]
    lib.orc_set_storage_model.restype = I
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _grid_args(n, lo, hi, periodic):
    n = np.ascontiguousarray(n, dtype=np.int64)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    mask = 0
    for d, p in enumerate(periodic):
        if p:
            mask |= 1 << d
    return n, lo, hi, mask


def _params(params):
    p = np.zeros(8, dtype=np.float64)
    params = list(params)
    p[: len(params)] = params
    return p, len(params)


def box_bound(n, lo, hi, periodic, dynamics, params, node, axis, blo, bhi) -> float:
    """max over p in the costate box [blo, bhi] of |dH/dp_axis| at one node
    (the LLF/GLF coefficient of Sec. 4)."""
    lib = _load()
    n, lo, hi, mask = _grid_args(n, lo, hi, periodic)
    p, npar = _params(params)
    bl = np.zeros(4)
    bh = np.zeros(4)
    bl[: len(blo)] = blo
    bh[: len(bhi)] = bhi
    return float(lib.orc_box_bound(len(n), _ptr(n), _ptr(lo), _ptr(hi), mask,
                                   DYNAMICS[dynamics], _ptr(p), npar, int(node), int(axis),
                                   _ptr(bl), _ptr(bh)))


def set_dissipation(kind: str = "lf") -> str:
    """Dissipation coefficients of later calls (Sec. 4): "lf" the control-set
    bound (default), "llf" per node over its own costate box, "glf" per node
    over the grid-wide box; returns the previous kind."""
    old = int(_load().orc_set_dissipation(DISSIPATION[kind]))
    return {v: k for k, v in DISSIPATION.items()}[old]


STORAGE_MODEL = {"fp64": 0, "stages": 1, "inputs": 2, "stages+inputs": 3}


def set_storage_model(kind: str = "fp64") -> str:
    """FP32 storage model of ``steps`` (a measurement aid, not the method):
    "stages" rounds every RK stage result (so the state) to single precision
    as it is stored, "inputs" rounds the tables, parameters, cell sizes, alpha
    and the step size to single precision, "stages+inputs" both; the
    arithmetic stays FP64.  "fp64" (the default) is the plain oracle.  Returns
    the previous setting."""
    old = int(_load().orc_set_storage_model(STORAGE_MODEL[kind]))
    return {v: k for k, v in STORAGE_MODEL.items()}[old]


def set_threads(n: int = 0) -> int:
    """Host threads for the node loops (0: all); returns the count in use."""
    return int(_load().orc_set_threads(int(n)))


def schedule(n, lo, hi, periodic, dynamics, params, cfl, t0, tf):
    """alpha per axis, dt, step count and final time of a solve (Sec. 4, Sec. 5)."""
    lib = _load()
    n, lo, hi, mask = _grid_args(n, lo, hi, periodic)
    p, npar = _params(params)
    alpha = np.zeros(4)
    dt = np.zeros(1)
    steps = np.zeros(1, dtype=np.int64)
    tend = np.zeros(1)
    rc = lib.orc_schedule(len(n), _ptr(n), _ptr(lo), _ptr(hi), mask,
                          DYNAMICS[dynamics], _ptr(p), npar, float(cfl), float(t0),
                          float(tf), _ptr(alpha), _ptr(dt), _ptr(steps), _ptr(tend))
    if rc != 0:
        raise ValueError("oracle schedule: bad grid")
    return alpha[: len(n)].copy(), float(dt[0]), int(steps[0]), float(tend[0])


def derivs(v, n, lo, hi, periodic, scheme, axis):
    """(p-, p+) along `axis` at every node (Sec. 3)."""
    lib = _load()
    n, lo, hi, mask = _grid_args(n, lo, hi, periodic)
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert v.size == int(np.prod(n))
    pm = np.empty_like(v)
    pp = np.empty_like(v)
    rc = lib.orc_derivs(len(n), _ptr(n), _ptr(lo), _ptr(hi), mask, SCHEMES[scheme],
                        int(axis), _ptr(v), _ptr(pm), _ptr(pp))
    if rc != 0:
        raise ValueError("oracle derivs: bad grid")
    return pm, pp


def rhs_at(v, n, lo, hi, periodic, dynamics, params, scheme, alpha, nodes):
    """L(V) = -Hhat at the flat node indices `nodes` (Sec. 4)."""
    lib = _load()
    n, lo, hi, mask = _grid_args(n, lo, hi, periodic)
    p, npar = _params(params)
    v = np.ascontiguousarray(v, dtype=np.float64)
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    a = np.zeros(4)
    a[: len(n)] = alpha
    out = np.empty(nodes.size)
    rc = lib.orc_rhs_at(len(n), _ptr(n), _ptr(lo), _ptr(hi), mask, DYNAMICS[dynamics],
                        _ptr(p), npar, SCHEMES[scheme], _ptr(a), _ptr(v), nodes.size,
                        _ptr(nodes), _ptr(out))
    if rc != 0:
        raise ValueError("oracle rhs_at: bad grid")
    return out


def steps(v, v0, n, lo, hi, periodic, dynamics, params, scheme, order, alpha, h,
          nsteps, mode="set"):
    """`nsteps` TVD-RK steps of size h from v (returns a new array; Sec. 5)."""
    lib = _load()
    n, lo, hi, mask = _grid_args(n, lo, hi, periodic)
    p, npar = _params(params)
    out = np.array(v, dtype=np.float64, order="C", copy=True)
    v0 = np.ascontiguousarray(v0 if v0 is not None else v, dtype=np.float64)
    a = np.zeros(4)
    a[: len(n)] = alpha
    rc = lib.orc_steps(len(n), _ptr(n), _ptr(lo), _ptr(hi), mask, DYNAMICS[dynamics],
                       _ptr(p), npar, SCHEMES[scheme], int(order), _ptr(a), float(h),
                       int(nsteps), _ptr(out), _ptr(v0), MODES[mode])
    if rc != 0:
        raise RuntimeError("oracle steps failed")
    return out


def solve(v0, n, lo, hi, periodic, dynamics, params, scheme="weno5", order=3,
          cfl=0.8, t0=0.0, tf=1.0, mode="set"):
    """Full solve over [t0, tf]; returns (V(tf), alpha, dt, steps) (Sec. 5)."""
    lib = _load()
    n, lo, hi, mask = _grid_args(n, lo, hi, periodic)
    p, npar = _params(params)
    v0 = np.ascontiguousarray(v0, dtype=np.float64)
    assert v0.size == int(np.prod(n))
    out = np.empty_like(v0)
    alpha = np.zeros(4)
    dt = np.zeros(1)
    k = lib.orc_solve(len(n), _ptr(n), _ptr(lo), _ptr(hi), mask, DYNAMICS[dynamics],
                      _ptr(p), npar, SCHEMES[scheme], int(order), float(cfl), _ptr(v0),
                      _ptr(out), float(t0), float(tf), MODES[mode], _ptr(alpha), _ptr(dt))
    if k < 0:
        raise RuntimeError("oracle solve failed (%d)" % k)
    return out, alpha[: len(n)].copy(), float(dt[0]), int(k)


def solve_outputs(v0, n, lo, hi, periodic, dynamics, params, times, scheme="weno5",
                  order=3, cfl=0.8, t0=0.0, mode="set"):
    """Solve from V0 at t0 through the ascending output times; returns
    (stack of V at each output time, total step count) (Sec. 5, Sec. 6.1)."""
    lib = _load()
    n, lo, hi, mask = _grid_args(n, lo, hi, periodic)
    p, npar = _params(params)
    v0 = np.ascontiguousarray(v0, dtype=np.float64)
    assert v0.size == int(np.prod(n))
    times = np.ascontiguousarray(times, dtype=np.float64)
    assert times.ndim == 1 and (times.size == 0 or (times[0] >= t0 and
                                                    np.all(np.diff(times) >= 0)))
    outs = np.empty((times.size,) + tuple(int(k) for k in n), dtype=np.float64)
    k = lib.orc_solve_outputs(len(n), _ptr(n), _ptr(lo), _ptr(hi), mask, DYNAMICS[dynamics],
                              _ptr(p), npar, SCHEMES[scheme], int(order), float(cfl),
                              _ptr(v0), float(t0), _ptr(times), int(times.size), MODES[mode],
                              _ptr(outs))
    if k < 0:
        raise RuntimeError("oracle solve failed (%d)" % k)
    return outs, int(k)


def shapes(n, lo, hi, periodic, shape_list):
    """V0 from implicit surfaces (Sec. 2.2).  shape_list: dicts with keys
    kind ("sphere", "cylinder", "box", "ellipsoid"), op ("union",
    "intersect", "subtract"; ignored for the first), axes (axis indices,
    empty = all), center, size (box half-widths / ellipsoid weights) and
    radius."""
    lib = _load()
    n, lo, hi, mask = _grid_args(n, lo, hi, periodic)
    k = len(shape_list)
    kinds = np.array([SHAPES[s["kind"]] for s in shape_list], dtype=np.int32)
    ops = np.array([OPS[s.get("op", "union")] for s in shape_list], dtype=np.int32)
    masks = np.array([sum(1 << a for a in s.get("axes", ())) for s in shape_list],
                     dtype=np.uint32)
    centers = np.zeros((k, 4))
    sizes = np.zeros((k, 4))
    for i, s in enumerate(shape_list):
        c = list(s.get("center", ()))
        z = list(s.get("size", ()))
        centers[i, : len(c)] = c
        sizes[i, : len(z)] = z
    radii = np.array([float(s.get("radius", 0.0)) for s in shape_list])
    out = np.empty(tuple(int(v) for v in n), dtype=np.float64)
    rc = lib.orc_shapes(len(n), _ptr(n), _ptr(lo), _ptr(hi), mask, k, _ptr(kinds), _ptr(ops),
                        _ptr(masks), _ptr(centers), _ptr(sizes), _ptr(radii), _ptr(out))
    if rc != 0:
        raise ValueError("oracle shapes: bad grid or no shapes")
    return out
