"""The oracle's one-sided derivatives against their textbook definitions
evaluated in exact rational arithmetic.

The oracle writes WENO5 on a window of five differences with its constant
fractions as precomputed doubles and one division per weight normalisation,
and ENO2/ENO3 as sums of Newton divided differences with precomputed
reciprocals of Delta x (Sec. 3.2, 3.3).  Here the same quantities are
computed from their definitions with Python fractions, so no rounding and no
arrangement of the arithmetic is shared with the oracle:

- ENO (Sec. 3.2, reading R24): Newton divided differences D1, D2, D3 of the
  node values, the ENO choice by the smaller magnitude (ties to the left
  candidate), and the derivative of the chosen interpolant at the node,
  Q1' + Q2' (+ Q3');
- WENO5 (Sec. 3.3, reading R3): the three third-order candidates, the
  smoothness indicators S1..S3 of Jiang and Peng, alpha_k = gamma_k /
  (S_k + eps)^2 with eps = 1e-6 max_k v_k^2 + 1e-99, omega_k = alpha_k /
  sum alpha, and the weighted candidate; p- from D- v at i-2..i+2, p+ from
  D+ v at i+2..i-2.

The only rounding the exact values skip is the oracle's own: a few units in
the last place of the largest stencil difference (on these fields at most
8e-16 of it, about 4 ulps), held here to 1e-14 of it.  (On adversarial data
the WENO weights could lose more: eps = 1e-6 max v_k^2 keeps the relative
error of each S_k + eps below about 1e3 ulps.)  A wrong coefficient, a
swapped weight, a reversed stencil, a dropped term or another eps moves the
result by far more.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from paper_2507_11542_amd import inputs

N = (29, 31)
LO = (-1.0, -2.0)
HI = (1.5, 2.0)
PER = (False, True)


def _spacing(d):
    return (HI[d] - LO[d]) / (N[d] if PER[d] else N[d] - 1)


def _fields():
    rng = np.random.default_rng(2507)
    x = inputs.node_coords(N, LO, HI, PER)
    gx, gy = np.meshgrid(x[0], x[1], indexing="ij")
    rough = rng.standard_normal(N)
    smooth = np.sin(2.0 * gx) * np.cos(gy) + np.abs(gx - 0.3) - 0.5 * np.abs(gy)
    scaled = 1e3 * rng.standard_normal(N)
    scaled[5:12, :] = 7.0  # flat block: zero differences, ties in the ENO choice
    tiny = 1e-5 * rng.standard_normal(N)
    tiny[:, 10:17] = 0.0  # zero data: eps is the 1e-99 floor
    return {"rough": rough, "smooth": smooth, "scaled": scaled, "tiny": tiny}


def _line(v, node, d):
    """The node's grid line along axis d as exact fractions, with an index map
    that wraps on a periodic axis."""
    idx = list(node)
    vals = []
    for j in range(N[d]):
        idx[d] = j
        vals.append(Fr(float(v[tuple(idx)])))
    if PER[d]:
        return lambda j: vals[j % N[d]]
    return lambda j: vals[j]


def _nodes(d, w):
    """Nodes whose stencil (w either side along d) stays on the grid or wraps."""
    for i in range(N[0]):
        for j in range(N[1]):
            k = (i, j)[d]
            if PER[d] or w <= k <= N[d] - 1 - w:
                yield (i, j)


def _d1(f, dx, k):
    """D1 at the half point k + 1/2."""
    return (f(k + 1) - f(k)) / dx


def _d2(f, dx, k):
    return (_d1(f, dx, k) - _d1(f, dx, k - 1)) / (2 * dx)


def _d3(f, dx, k):
    """D3 at the half point k + 1/2: from D2 at k and k + 1."""
    return (_d2(f, dx, k + 1) - _d2(f, dx, k)) / (3 * dx)


def _eno_exact(f, dx, i, order, minus):
    """Newton-form ENO derivative at node i: k = i - 1 for p-, i for p+."""
    k = i - 1 if minus else i
    q = _d1(f, dx, k)
    if order == 1:
        return q
    if abs(_d2(f, dx, k)) <= abs(_d2(f, dx, k + 1)):
        c, ks = _d2(f, dx, k), k - 1
    else:
        c, ks = _d2(f, dx, k + 1), k
    q += c * (2 * (i - k) - 1) * dx
    if order == 2:
        return q
    a, b = _d3(f, dx, ks), _d3(f, dx, ks + 1)
    cs = a if abs(a) <= abs(b) else b
    m = i - ks
    return q + cs * (3 * m * m - 6 * m + 2) * dx * dx


def _weno_exact(v1, v2, v3, v4, v5):
    """Jiang-Peng HJ-WENO5 on the five differences v1..v5 (Osher-Fedkiw eqs.
    3.28-3.39), exactly."""
    phi1 = v1 / 3 - Fr(7, 6) * v2 + Fr(11, 6) * v3
    phi2 = -v2 / 6 + Fr(5, 6) * v3 + v4 / 3
    phi3 = v3 / 3 + Fr(5, 6) * v4 - v5 / 6
    s1 = Fr(13, 12) * (v1 - 2 * v2 + v3) ** 2 + Fr(1, 4) * (v1 - 4 * v2 + 3 * v3) ** 2
    s2 = Fr(13, 12) * (v2 - 2 * v3 + v4) ** 2 + Fr(1, 4) * (v2 - v4) ** 2
    s3 = Fr(13, 12) * (v3 - 2 * v4 + v5) ** 2 + Fr(1, 4) * (3 * v3 - 4 * v4 + v5) ** 2
    eps = Fr(1e-6) * max(t * t for t in (v1, v2, v3, v4, v5)) + Fr(1e-99)
    a1 = Fr(1, 10) / (s1 + eps) ** 2
    a2 = Fr(6, 10) / (s2 + eps) ** 2
    a3 = Fr(3, 10) / (s3 + eps) ** 2
    return (a1 * phi1 + a2 * phi2 + a3 * phi3) / (a1 + a2 + a3)


def _weno_side(f, dx, i, minus):
    if minus:  # D- v at i-2 .. i+2 = D1 at i-5/2 .. i+3/2
        v = [_d1(f, dx, i + m - 1) for m in (-2, -1, 0, 1, 2)]
    else:  # D+ v at i+2 .. i-2 = D1 at i+5/2 .. i-3/2
        v = [_d1(f, dx, i + m) for m in (2, 1, 0, -1, -2)]
    return _weno_exact(*v), max(abs(t) for t in v)


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("field", ["rough", "smooth", "scaled", "tiny"])
def test_weno5_equals_exact_definition(orc, field, axis):
    v = _fields()[field]
    dx = Fr(_spacing(axis))
    pm, pp = orc.derivs(v, N, LO, HI, PER, "weno5", axis)
    worst = 0.0
    for node in _nodes(axis, 3):
        f = _line(v, node, axis)
        i = node[axis]
        for got, minus in ((pm[node], True), (pp[node], False)):
            want, scale = _weno_side(f, dx, i, minus)
            err = abs(Fr(float(got)) - want)
            if scale == 0:
                assert err == 0, (node, minus)
            else:
                worst = max(worst, float(err / scale))
    assert worst <= 1e-14, worst


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("scheme,order,w", [("upwind1", 1, 1), ("eno2", 2, 2), ("eno3", 3, 3)])
@pytest.mark.parametrize("field", ["rough", "smooth", "scaled"])
def test_eno_equals_exact_definition(orc, field, scheme, order, w, axis):
    v = _fields()[field]
    dx = Fr(_spacing(axis))
    pm, pp = orc.derivs(v, N, LO, HI, PER, scheme, axis)
    worst = 0.0
    for node in _nodes(axis, w):
        f = _line(v, node, axis)
        i = node[axis]
        scale = max(abs(_d1(f, dx, k)) for k in range(i - w, i + w))
        for got, minus in ((pm[node], True), (pp[node], False)):
            err = abs(Fr(float(got)) - _eno_exact(f, dx, i, order, minus))
            if scale == 0:
                assert err == 0, (node, minus)
            else:
                worst = max(worst, float(err / scale))
    assert worst <= 1e-14, worst


def test_exact_weno5_reduces_to_ideal_weights_on_quadratics():
    """Self-check of the exact definition above: on a quadratic V the
    differences v1..v5 lie on a line, the three smoothness indicators are
    equal, so the weights are the ideal (0.1, 0.6, 0.3) and the value is the
    fifth-order upwind combination (2 v1 - 13 v2 + 47 v3 + 27 v4 - 3 v5) / 60,
    which on such data is V' at the node: v3 + (v4 - v3) / 2."""
    for a, b in ((Fr(1), Fr(2)), (Fr(-3, 7), Fr(5, 11)), (Fr(0), Fr(-1, 3))):
        v = [a + b * k for k in range(5)]
        fifth = (2 * v[0] - 13 * v[1] + 47 * v[2] + 27 * v[3] - 3 * v[4]) / 60
        assert _weno_exact(*v) == fifth == v[2] + b / 2
    # one rough substencil: its weight vanishes against the smooth ones
    v = [Fr(50), Fr(0), Fr(1), Fr(2), Fr(3)]
    want = (Fr(6, 10) * (-Fr(0) / 6 + Fr(5, 6) + Fr(2, 3)) + Fr(3, 10) * (Fr(1, 3) + Fr(5, 3) - Fr(1, 2))) / Fr(9, 10)
    assert abs(_weno_exact(*v) - want) < Fr(1, 10**6)
