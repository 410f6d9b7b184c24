"""Pins of the oracle's rockets game (Sec. 6.1), its tube variants (the
min[0,H] variational form; the min with V0 at output times only) and output
times, against the dynamics, closed forms and invariants.

What a plausible mistake would break:
- a sign or a swapped abs argument in the rockets Hamiltonian: the brute-force
  game value over the control sets, and the pure-drift closed form (which also
  fixes the sign of g);
- a wrong per-axis bound: alpha against its closed form over the grid nodes;
- the restricted update taken the wrong way, or per step instead of per
  stage: monotonicity, the forward-Euler identity, the frozen shrinking ball;
- output intervals that do not restart, or a tube taken every step: the
  composition identities and the single-output identity.
"""
import math

import numpy as np
import pytest

from paper_2507_11542_amd import inputs, metrics

PI = math.pi


def _rockets_f(x, th, ue, up, a, g):
    """The game's vector field (the one inside the Hamiltonian's definition):
    xdot = a cos th + ue x, zdot = a sin th + a + up x - g, thdot = up - ue."""
    return (a * np.cos(th) + ue * x, a * np.sin(th) + a + up * x - g,
            up - ue + 0.0 * x)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_rockets_hamiltonian_is_the_game_value(orc, seed):
    """On linear data (p- = p+ = p exactly, no dissipation) L = -H(x, p), and
    -H = max over ue of min over up of p.f, enumerated over the control sets
    (p.f is bilinear in the controls, so the grid's end points are exact)."""
    rng = np.random.default_rng(seed)
    a, g, um = 1.0, 32.0, float(rng.uniform(0.5, 1.5))
    n, lo, hi, per = (9, 8, 7), (-5.0, -4.0, -PI / 2), (6.0, 3.0, PI / 2), (False,) * 3
    c = rng.normal(size=3)
    X, Z, TH = np.meshgrid(*inputs.node_coords(n, lo, hi, per), indexing="ij")
    v = np.ascontiguousarray(c[0] * X + c[1] * Z + c[2] * TH)
    nodes = np.arange(int(np.prod(n)))
    l = orc.rhs_at(v, n, lo, hi, per, "rockets", (a, g, um), "eno2", (3.0, 5.0, 7.0), nodes)
    us = np.linspace(-um, um, 21)
    best = np.full(X.shape, -np.inf)
    for ue in us:
        worst = np.full(X.shape, np.inf)
        for up in us:
            f1, f2, f3 = _rockets_f(X, TH, ue, up, a, g)
            worst = np.minimum(worst, c[0] * f1 + c[1] * f2 + c[2] * f3)
        best = np.maximum(best, worst)
    assert np.abs(l - best.ravel()).max() < 1e-9


def test_rockets_drift_is_a_translation_per_heading(orc):
    """With umax = 0 each theta slice is transported at
    b(th) = (a cos th, a sin th + a - g): V_t = b . grad V, so linear data
    V0 = c.x gives V(t) = V0 + t (c1 b1 + c2 b2) exactly (up to rounding)."""
    a, g = 1.0, 32.0
    n, lo, hi, per = (11, 12, 9), (-6.0, -6.0, -PI / 2), (6.0, 6.0, PI / 2), (False,) * 3
    X, Z, TH = np.meshgrid(*inputs.node_coords(n, lo, hi, per), indexing="ij")
    c = (0.7, -1.3)
    v0 = np.ascontiguousarray(c[0] * X + c[1] * Z)
    T = 0.05
    out, *_ = orc.solve(v0, n, lo, hi, per, "rockets", (a, g, 0.0), "eno2", 3, 0.8, 0.0, T,
                        "set")
    exact = v0 + T * (c[0] * a * np.cos(TH) + c[1] * (a * np.sin(TH) + a - g))
    assert np.abs(out - exact).max() < 1e-11


def test_rockets_alpha_closed_form(orc):
    """alpha = (max a|cos th| + umax max|x|, max|a sin th + a - g| + umax max|x|,
    2 umax) over the grid nodes; with 100 nodes on [-pi/2, pi/2] the node
    nearest th = 0 is pi/198 away, and th = -pi/2 gives |a sin th + a - g| = g."""
    p = inputs.rockets()
    alpha, dt, k, tend = orc.schedule(*p.grid_args(), p.dynamics, p.params, p.cfl, p.t0, p.tf)
    assert alpha[0] == pytest.approx(math.cos(PI / 198) + 64.0, rel=1e-15)
    assert alpha[1] == pytest.approx(96.0, rel=1e-15)
    assert alpha[2] == 2.0
    dx, dth = 128.0 / 99, PI / 99
    assert dt == pytest.approx(0.8 / (alpha[0] / dx + alpha[1] / dx + alpha[2] / dth),
                               rel=1e-14)
    assert k == math.ceil(2.5 / dt - 1e-9) and tend == 0.0


# ------------------------------------------------ variational-inequality tube
def _ball(n=41, s=1.0):
    lo, hi, per = (-4.0, -4.0), (4.0, 4.0), (False, False)
    X, Y = np.meshgrid(*inputs.node_coords((n, n), lo, hi, per), indexing="ij")
    v0 = np.ascontiguousarray(np.sqrt(X ** 2 + Y ** 2) - 1.0)
    return (n, n), lo, hi, per, v0, X, Y


def test_vi_never_increases(orc):
    """Every step of the restricted update is non-increasing at every node up
    to the rounding of the RK3 convex combinations (a few ulp), while the
    plain update rises by far more in places (relative Dubins)."""
    p = inputs.rel_dubins_3d(n=(21, 19, 12), tf=0.3)
    v = p.v0()
    alpha, dt, k, _ = orc.schedule(*p.grid_args(), p.dynamics, p.params, p.cfl, 0.0, 0.3)
    rose = False
    for _ in range(6):
        nxt = orc.steps(v, p.v0(), *p.grid_args(), p.dynamics, p.params, "weno5", 3, alpha,
                        dt, 1, mode="tube_vi")
        free = orc.steps(v, p.v0(), *p.grid_args(), p.dynamics, p.params, "weno5", 3, alpha,
                         dt, 1, mode="set")
        assert np.all(nxt <= v + 4 * np.spacing(np.abs(v)))
        rose = rose or bool(np.any(free > v + 1e-6))
        v = nxt
    assert rose  # the restriction is active somewhere


def test_vi_euler_is_min_of_previous_and_step(orc):
    """For forward Euler, V + h min(L, 0) = min(V, V + h L) at every node."""
    p = inputs.rel_dubins_3d(n=(17, 15, 10), tf=0.2)
    v0 = p.v0()
    alpha, dt, *_ = orc.schedule(*p.grid_args(), p.dynamics, p.params, p.cfl, 0.0, 0.2)
    v = orc.steps(v0, v0, *p.grid_args(), p.dynamics, p.params, "weno5", 3, alpha, dt, 3,
                  mode="set")
    vi = orc.steps(v, v0, *p.grid_args(), p.dynamics, p.params, "weno5", 1, alpha, dt, 1,
                   mode="tube_vi")
    free = orc.steps(v, v0, *p.grid_args(), p.dynamics, p.params, "weno5", 1, alpha, dt, 1,
                     mode="set")
    assert np.array_equal(vi, np.minimum(v, free))


def test_vi_freezes_a_shrinking_convex_ball(orc):
    """BALL with negative speed shrinks the set: L = |s||p| + dissipation >= 0
    on the convex cone V0 = |x| - 1 (p+ >= p- everywhere), so the restricted
    update returns V0 up to the rounding of the RK3 combinations, while the
    free solve moves."""
    n, lo, hi, per, v0, *_ = _ball()
    out, *_ = orc.solve(v0, n, lo, hi, per, "ball", (-1.0,), "eno2", 3, 0.8, 0.0, 0.5,
                        "tube_vi")
    free, *_ = orc.solve(v0, n, lo, hi, per, "ball", (-1.0,), "eno2", 3, 0.8, 0.0, 0.5, "set")
    assert np.abs(out - v0).max() < 1e-12
    assert np.abs(free - v0).max() > 0.3


def test_vi_growing_ball_closed_form(orc):
    """BALL with unit speed grows the disk: V = |x| - 1 - t near the front,
    with the restricted update as with the free one."""
    n, lo, hi, per, v0, X, Y = _ball(n=81)
    T = 0.8
    out, *_ = orc.solve(v0, n, lo, hi, per, "ball", (1.0,), "weno5", 3, 0.8, 0.0, T, "tube_vi")
    exact = np.sqrt(X ** 2 + Y ** 2) - 1.0 - T
    band = np.abs(exact) < 0.3
    assert np.abs(out - exact)[band].max() < 0.02
    assert metrics.hausdorff_cells(out, exact, per) < 0.3


# ------------------------------------------------------------- output times
def test_outputs_compose_like_separate_solves(orc):
    """Outputs at t1 < t2 equal a solve over [t0, t1] followed by a solve over
    [t1, t2] from its result (each interval runs its own loop), bit for bit,
    for the per-step tube and the restricted update; the step counts add."""
    p = inputs.rel_dubins_3d(n=(15, 13, 10))
    v0 = p.v0()
    t1, t2 = 0.13, 0.31
    for mode in ("tube", "tube_vi", "set"):
        outs, k = orc.solve_outputs(v0, *p.grid_args(), p.dynamics, p.params, [t1, t2],
                                    "weno5", 3, 0.8, 0.0, mode)
        a, _, _, k1 = orc.solve(v0, *p.grid_args(), p.dynamics, p.params, "weno5", 3, 0.8,
                                0.0, t1, mode)
        # the second interval restarts from a; the per-step tube compares with V0
        b, k2 = orc.solve_outputs(a, *p.grid_args(), p.dynamics, p.params, [t2 - t1],
                                  "weno5", 3, 0.8, 0.0, "set" if mode == "set" else mode)
        assert np.array_equal(outs[0], a)
        assert k == k1 + k2
        if mode != "tube":  # the tube's V0 is the solve's own V0, not a
            assert np.array_equal(outs[1], b[0])


def test_tube_at_outputs(orc):
    """The tube taken at output times only: one output at tf is min(free, V0);
    an output at t0 is V0; it is never below the per-step tube's result
    pattern at t0 and equals the free solve where that is below V0."""
    p = inputs.rel_dubins_3d(n=(15, 13, 10), tf=0.25)
    v0 = p.v0()
    outs, k = orc.solve_outputs(v0, *p.grid_args(), p.dynamics, p.params, [0.0, 0.25],
                                "weno5", 3, 0.8, 0.0, "tube_out")
    free, _, _, kf = orc.solve(v0, *p.grid_args(), p.dynamics, p.params, "weno5", 3, 0.8, 0.0,
                               0.25, "set")
    assert np.array_equal(outs[0], v0)
    assert np.array_equal(outs[1], np.minimum(free, v0))
    assert k == kf
    one, *_ = orc.solve(v0, *p.grid_args(), p.dynamics, p.params, "weno5", 3, 0.8, 0.0, 0.25,
                        "tube_out")
    assert np.array_equal(one, outs[1])
