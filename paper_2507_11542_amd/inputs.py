"""Seeded synthetic workloads: grids, initial value functions and request mixes.

This module holds no arithmetic of the level-set method itself.  It describes
problems (grid extents, dynamics parameters, horizons) and builds the initial
signed-distance functions V0 on the node coordinates, so that the GPU path and
the CPU oracle can be fed identical inputs.  It imports numpy only.

Workloads (the analytic problems the solver is measured on):

- ``double_integrator_2d``: x1' = x2, x2' = u, |u| <= 1, 101^2 on [-1,1]^2,
  V0 = |x| - 0.5, ENO2 / Lax-Friedrichs / TVD-RK2, CFL 0.8, tube to t = 1.
- ``rel_dubins_3d``: relative Dubins pursuit-evasion, ve = vp = 5,
  |we|,|wp| <= 1, 101^3 on [-6,20]x[-10,10]x[-pi,pi) (psi periodic),
  V0 = sqrt(x^2+y^2) - 5, WENO5 / LF / TVD-RK3, tube to t = 2.8.
- ``rel_dubins_batch``: 64 relative-Dubins tubes with N ~ U{51,61,81,101} and
  speeds / turn bounds drawn from numpy's default_rng(0).
- ``dubins4d``: 4-D Dubins car with speed state, 61^4 on
  [-5,5]^2 x [-pi,pi) x [0,4] (theta periodic), V0 = sqrt(x^2+y^2) - 1,
  WENO5 / LF / TVD-RK3, reachable set to t = 2.
- ``rockets``: the rockets launch game of Dreyfus in relative coordinates
  (x, z, theta), a = 1, g = 32, |u| <= 1, 100^3 on [-64,64]^2 x
  [-pi/2, pi/2] (no periodic axis), V0 = sqrt(x^2+z^2) - 1.5 (the capture
  circle, a cylinder along theta), ENO2 / LF / TVD-RK3, tube as the
  variational inequality over t in [-2.5, 0] with 11 output times.
- ``serving_stream``: Poisson arrivals mixing the three families.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class Problem:
    """One solve request: grid, dynamics, scheme, horizon and V0 recipe."""
    name: str
    n: Tuple[int, ...]
    lo: Tuple[float, ...]
    hi: Tuple[float, ...]
    periodic: Tuple[bool, ...]
    dynamics: str
    params: Tuple[float, ...]
    scheme: str = "weno5"
    order: int = 3
    cfl: float = 0.8
    t0: float = 0.0
    tf: float = 1.0
    mode: str = "tube"
    radius: float = 1.0          # V0 = sqrt(x0^2 + x1^2) - radius
    v0_axes: Tuple[int, ...] = (0, 1)
    diss: str = "lf"             # Lax-Friedrichs coefficients: lf, llf, glf

    @property
    def ndim(self) -> int:
        return len(self.n)

    @property
    def points(self) -> int:
        return int(np.prod(self.n))

    def grid_args(self):
        return self.n, self.lo, self.hi, self.periodic

    def coords(self) -> List[np.ndarray]:
        return node_coords(self.n, self.lo, self.hi, self.periodic)

    def v0(self) -> np.ndarray:
        return sdf_cylinder(self.n, self.lo, self.hi, self.periodic, self.radius,
                            self.v0_axes)

    def shapes(self) -> List[dict]:
        """The same V0 as an implicit-surface recipe (a cylinder over the
        v0 axes), for building it on the device."""
        return [dict(kind="cylinder", axes=tuple(a for a in self.v0_axes if a < self.ndim),
                     radius=self.radius)]

    def with_(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def node_coords(n, lo, hi, periodic) -> List[np.ndarray]:
    """Node coordinates per axis: both ends on a bounded axis, hi excluded on a
    periodic one."""
    xs = []
    for nd, a, b, p in zip(n, lo, hi, periodic):
        h = (b - a) / nd if p else (b - a) / (nd - 1)
        xs.append(a + np.arange(nd, dtype=np.float64) * h)
    return xs


def cell_sizes(n, lo, hi, periodic) -> np.ndarray:
    return np.array([(b - a) / nd if p else (b - a) / (nd - 1)
                     for nd, a, b, p in zip(n, lo, hi, periodic)])


def sdf_cylinder(n, lo, hi, periodic, radius, axes=(0, 1)) -> np.ndarray:
    """Signed distance to {sum over `axes` of x_k^2 <= radius^2}: negative
    inside, C-order array of shape n (float64)."""
    xs = node_coords(n, lo, hi, periodic)
    grids = np.meshgrid(*xs, indexing="ij", sparse=True)
    r2 = 0.0
    for a in axes:
        if a < len(n):
            r2 = r2 + grids[a] ** 2
    out = np.sqrt(r2) - radius
    return np.array(np.broadcast_to(out, tuple(n)), dtype=np.float64, order="C", copy=True)


def sdf_box(n, lo, hi, periodic, center, half, axes) -> np.ndarray:
    """Signed distance to an axis-aligned box (rectangle) over `axes`."""
    xs = node_coords(n, lo, hi, periodic)
    grids = np.meshgrid(*xs, indexing="ij", sparse=True)
    q = [np.abs(grids[a] - c) - h for a, c, h in zip(axes, center, half)]
    outside = 0.0
    inside = -np.inf
    for qa in q:
        outside = outside + np.maximum(qa, 0.0) ** 2
        inside = np.maximum(inside, qa)
    out = np.sqrt(outside) + np.minimum(inside, 0.0)
    return np.array(np.broadcast_to(out, tuple(n)), dtype=np.float64, order="C", copy=True)


def random_field(n, seed=0, amplitude=1.0) -> np.ndarray:
    """Seeded smooth-plus-noise test field (float64, shape n)."""
    rng = np.random.default_rng(seed)
    return amplitude * rng.standard_normal(tuple(n))


# ------------------------------------------------------------------ configs

def double_integrator_2d(n=101, u_max=1.0, tf=1.0, scheme="eno2", order=2) -> Problem:
    return Problem("double_integrator_2d", (n, n), (-1.0, -1.0), (1.0, 1.0),
                   (False, False), "double_integrator", (u_max,), scheme=scheme,
                   order=order, cfl=0.8, tf=tf, mode="tube", radius=0.5)


def rel_dubins_3d(n=101, ve=5.0, vp=5.0, we=1.0, wp=1.0, tf=2.8, scheme="weno5",
                  order=3) -> Problem:
    n3 = (n, n, n) if np.isscalar(n) else tuple(n)
    return Problem("rel_dubins_3d", n3, (-6.0, -10.0, -math.pi),
                   (20.0, 10.0, math.pi), (False, False, True), "rel_dubins",
                   (ve, vp, we, wp), scheme=scheme, order=order, cfl=0.8, tf=tf,
                   mode="tube", radius=5.0)


def dubins4d(n=61, w_max=1.0, a_max=1.0, tf=2.0, scheme="weno5", order=3) -> Problem:
    n4 = (n, n, n, n) if np.isscalar(n) else tuple(n)
    return Problem("dubins4d", n4, (-5.0, -5.0, -math.pi, 0.0),
                   (5.0, 5.0, math.pi, 4.0), (False, False, True, False), "dubins4d",
                   (w_max, a_max), scheme=scheme, order=order, cfl=0.8, tf=tf,
                   mode="set", radius=1.0)


def rockets(n=100, a=1.0, g=32.0, u_max=1.0, t0=-2.5, tf=0.0, scheme="eno2", order=3,
            mode="tube_vi") -> Problem:
    n3 = (n, n, n) if np.isscalar(n) else tuple(n)
    return Problem("rockets", n3, (-64.0, -64.0, -math.pi / 2), (64.0, 64.0, math.pi / 2),
                   (False, False, False), "rockets", (a, g, u_max), scheme=scheme,
                   order=order, cfl=0.8, t0=t0, tf=tf, mode=mode, radius=1.5)


def output_times(t0: float, tf: float, count: int = 11) -> np.ndarray:
    """count equally spaced output times from t0 to tf (both included)."""
    return np.linspace(t0, tf, count)


def rel_dubins_batch(count=64, seed=0, sizes=(51, 61, 81, 101)) -> List[Problem]:
    """Uneven batch of relative-Dubins tubes; draws per instance in the order
    N, ve, vp, we, wp from numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice(sizes))
        ve = float(rng.uniform(3.0, 6.0))
        vp = float(rng.uniform(3.0, 6.0))
        we = float(rng.uniform(0.5, 1.5))
        wp = float(rng.uniform(0.5, 1.5))
        out.append(rel_dubins_3d(n, ve, vp, we, wp))
    return out


@dataclasses.dataclass
class Request:
    arrival: float
    problem: Problem


def serving_stream(count=256, rate=1.0, seed=0,
                   di_sizes=(101, 401), rd_sizes=(51, 121), d4_sizes=(41, 61),
                   horizon=(0.5, 3.0)) -> List[Request]:
    """Poisson arrivals (rate per second) mixing the three families in equal
    thirds; every request uses WENO5 / LF / TVD-RK3."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(count):
        t += float(rng.exponential(1.0 / rate))
        fam = int(rng.integers(0, 3))
        tf = float(rng.uniform(*horizon))
        if fam == 0:
            n = int(rng.integers(di_sizes[0], di_sizes[1] + 1))
            u = float(rng.uniform(0.5, 1.5))
            p = double_integrator_2d(n, u, tf, scheme="weno5", order=3)
        elif fam == 1:
            n = int(rng.integers(rd_sizes[0], rd_sizes[1] + 1))
            ve = float(rng.uniform(3.0, 6.0))
            vp = float(rng.uniform(3.0, 6.0))
            we = float(rng.uniform(0.5, 1.5))
            wp = float(rng.uniform(0.5, 1.5))
            p = rel_dubins_3d(n, ve, vp, we, wp, tf)
        else:
            n = int(rng.integers(d4_sizes[0], d4_sizes[1] + 1))
            w = float(rng.uniform(0.5, 1.5))
            a = float(rng.uniform(0.5, 1.5))
            p = dubins4d(n, w, a, tf)
        out.append(Request(t, p))
    return out


def sample_nodes(shape: Sequence[int], count: int, seed: int = 0) -> np.ndarray:
    """Seeded flat node indices (sorted, unique) for sampled comparisons."""
    total = int(np.prod(shape))
    rng = np.random.default_rng(seed)
    k = min(count, total)
    return np.sort(rng.choice(total, size=k, replace=False)).astype(np.int64)
