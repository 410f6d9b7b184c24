"""The oracle's Lax-Friedrichs right-hand side of every compiled dynamics
against the optimal-control value taken by enumeration (Sec. 4 with the
Hamiltonians of Sec. 6.1; sign convention of reading R9).

At sampled nodes of rough data, L = -Hhat = min over the controls (or max
over the evader of min over the pursuer, for the games) of p-bar . f(x, u)
plus sum_d alpha_d (p+_d - p-_d) / 2, with p-bar = (p- + p+) / 2, the
one-sided derivatives from the oracle's derivative routine (pinned against
their definitions elsewhere) and the vector field written out here from the
equations of motion.  The controls are enumerated on a grid of their set
(the optimum of a linear function lies at its ends, which the grid holds),
so a wrong sign, a swapped axis or a dropped term of any Hamiltonian moves
L by a sizeable part of |p| at some node.  Arbitrary alpha values pin the
dissipation sum separately from the schedule.
"""
import math

import numpy as np
import pytest

from paper_2507_11542_amd import inputs


@pytest.fixture
def lf(orc):
    old = orc.set_dissipation("lf")
    yield orc
    orc.set_dissipation(old)


def _rhs_case(orc, p, alpha, fields, seed):
    v = p.v0() + 0.3 * inputs.random_field(p.n, seed=seed)
    d = len(p.n)
    pm, pp = zip(*[orc.derivs(v, *p.grid_args(), p.scheme, k) for k in range(d)])
    pm = np.stack([a.ravel() for a in pm], 1)
    pp = np.stack([a.ravel() for a in pp], 1)
    xs = [a.ravel() for a in np.meshgrid(*p.coords(), indexing="ij")]
    nodes = inputs.sample_nodes(p.n, 40, seed=seed)
    got = orc.rhs_at(v, *p.grid_args(), p.dynamics, p.params, p.scheme, alpha, nodes)
    for k, node in enumerate(nodes):
        x = [a[node] for a in xs]
        pbar = (pm[node] + pp[node]) / 2
        value = fields(x, pbar)
        expect = value + sum(alpha[j] * (pp[node, j] - pm[node, j]) / 2 for j in range(d))
        assert got[k] == pytest.approx(expect, abs=1e-11 * max(1.0, abs(expect))), node


def test_double_integrator_rhs_is_the_control_minimum(lf):
    """x1' = x2, x2' = u, |u| <= umax, the control minimising."""
    p = inputs.double_integrator_2d(n=27, u_max=0.8).with_(n=(27, 25))
    umax = p.params[0]
    us = np.linspace(-umax, umax, 11)

    def value(x, pb):
        return min(pb[0] * x[1] + pb[1] * u for u in us)

    _rhs_case(lf, p, (1.7, 0.8), value, seed=3)


def test_dubins4d_rhs_is_the_control_minimum(lf):
    """x' = v cos th, y' = v sin th, th' = w, v' = a, |w| <= wmax,
    |a| <= amax, the controls minimising."""
    p = inputs.dubins4d(n=(11, 10, 9, 8), w_max=0.7, a_max=1.3)
    wmax, amax = p.params
    ws = np.linspace(-wmax, wmax, 7)
    acc = np.linspace(-amax, amax, 7)

    def value(x, pb):
        _, _, th, v = x
        return min(pb[0] * v * math.cos(th) + pb[1] * v * math.sin(th) + pb[2] * w + pb[3] * a
                   for w in ws for a in acc)

    _rhs_case(lf, p, (4.0, 4.0, 0.7, 1.3), value, seed=4)


def test_rel_dubins_rhs_is_the_game_value(lf):
    """Relative Dubins pursuit-evasion: evader turn rate maximising, pursuer
    turn rate minimising (the LF form of the box tests' game value)."""
    p = inputs.rel_dubins_3d(n=(12, 11, 10), ve=4.0, vp=5.5, we=0.9, wp=1.2, scheme="eno2")
    ve, vp, we, wp = p.params
    ue_s = np.linspace(-we, we, 7)
    up_s = np.linspace(-wp, wp, 7)

    def value(x, pb):
        px, py, psi = x
        return max(min(pb @ np.array([-ve + vp * math.cos(psi) + ue * py,
                                      vp * math.sin(psi) - ue * px, up - ue])
                       for up in up_s) for ue in ue_s)

    _rhs_case(lf, p, (15.0, 12.0, 2.1), value, seed=5)


def test_translation_rhs_is_the_transport(lf):
    """x' = b (no control): L = p-bar . b plus the dissipation (the set of
    states that reach the target moves against b)."""
    n, lo, hi, per = (17, 15, 13), (-1.0, -2.0, 0.0), (1.0, 1.0, 2.0), (False, True, False)
    p = inputs.rel_dubins_3d(n=n).with_(dynamics="translation", params=(0.5, -1.25, 2.0),
                                        lo=lo, hi=hi, periodic=per)
    b = np.array(p.params)

    def value(x, pb):
        return b @ pb

    _rhs_case(lf, p, (0.5, 1.25, 2.0), value, seed=6)
