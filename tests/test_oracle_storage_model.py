"""Pins of the oracle's FP32 storage model (``oracle.set_storage_model``), the
measurement aid that separates how the FP64 method responds to single
precision storage from how it responds to single precision arithmetic.

- "stages": every RK stage result is rounded to single precision as it is
  stored.  An RK3 step of the model equals the same step recomposed here from
  the oracle's own right-hand sides with a rounding after each stage (Sec. 5,
  the odeCFL3 stages), and an RK1 step equals one plain FP64 step rounded.
- "inputs": tables, parameters, cell sizes, alpha and the step size in single
  precision.  Where all of them are single-precision numbers already the
  model equals the plain oracle bit for bit; where they are not it does not.
- the default is the plain FP64 oracle, and the solve entry points ignore the
  model.
"""
import numpy as np
import pytest

from paper_2507_11542_amd import inputs


def _r32(v):
    return np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)


@pytest.fixture
def model(orc):
    old = orc.set_storage_model("fp64")
    yield orc
    orc.set_storage_model(old)


def _rough_problem():
    p = inputs.rel_dubins_3d(n=(17, 15, 13), tf=0.05).with_(params=(4.3, 5.7, 0.83, 1.21))
    rng = np.random.default_rng(11)
    v = p.v0() + 0.05 * rng.standard_normal(p.n)
    return p, v


def test_stages_model_rk3_step_recomposed(model):
    p, v = _rough_problem()
    v = _r32(v)
    alpha, dt, _, _ = model.schedule(*p.grid_args(), p.dynamics, p.params, p.cfl, 0.0, 1.0)
    args = (*p.grid_args(), p.dynamics, p.params, p.scheme)
    nodes = np.arange(v.size)

    def L(w):
        return model.rhs_at(w, *args, alpha, nodes).reshape(v.shape)

    w1 = _r32(v + dt * L(v))
    w2 = _r32((3.0 * v + (w1 + dt * L(w1))) / 4.0)
    want = _r32((v + 2.0 * (w2 + dt * L(w2))) / 3.0)
    model.set_storage_model("stages")
    got = model.steps(v, None, *args, 3, alpha, dt, 1, mode="set")
    assert np.array_equal(got, want)
    model.set_storage_model("fp64")
    plain = model.steps(v, None, *args, 3, alpha, dt, 1, mode="set")
    assert not np.array_equal(plain, want)
    assert np.array_equal(got, _r32(got))


def test_stages_model_rk1_is_rounded_fp64_step(model):
    p, v = _rough_problem()
    v = _r32(v)
    alpha, dt, _, _ = model.schedule(*p.grid_args(), p.dynamics, p.params, p.cfl, 0.0, 1.0)
    args = (*p.grid_args(), p.dynamics, p.params, p.scheme)
    plain = model.steps(v, None, *args, 1, alpha, dt, 1, mode="set")
    model.set_storage_model("stages")
    got = model.steps(v, None, *args, 1, alpha, dt, 1, mode="set")
    assert np.array_equal(got, _r32(plain))


def test_stages_model_tube_keeps_v0(model):
    """The tube minimum with a single-precision V0 after the rounded last
    stage: every value is a single-precision number and none exceeds V0."""
    p, v = _rough_problem()
    v0 = _r32(p.v0())
    alpha, dt, _, _ = model.schedule(*p.grid_args(), p.dynamics, p.params, p.cfl, 0.0, 1.0)
    model.set_storage_model("stages")
    got = model.steps(v0, v0, *p.grid_args(), p.dynamics, p.params, p.scheme, 3, alpha, dt, 4,
                      mode="tube")
    assert np.array_equal(got, _r32(got))
    assert np.all(got <= v0)


def test_inputs_model_exact_when_everything_is_single(model):
    """Grid [-1, 1] with 9 nodes (dx = 1/4), translation by b = 1.5, alpha 1.5,
    step 1/8: every input is a single-precision number, so rounding them
    changes nothing."""
    n, lo, hi, per = (9,), (-1.0,), (1.0,), (False,)
    x = np.linspace(-1.0, 1.0, 9)
    v = np.sin(3.0 * x) + 0.25 * x * x
    got = {}
    for kind in ("fp64", "inputs"):
        model.set_storage_model(kind)
        got[kind] = model.steps(v, None, n, lo, hi, per, "translation", (1.5,), "weno5", 3,
                                [1.5], 0.125, 3, mode="set")
    assert np.array_equal(got["fp64"], got["inputs"])


def test_inputs_model_rounds_parameters_and_step(model):
    p, v = _rough_problem()
    alpha, dt, _, _ = model.schedule(*p.grid_args(), p.dynamics, p.params, p.cfl, 0.0, 1.0)
    args = (*p.grid_args(), p.dynamics, p.params, p.scheme, 3, alpha, dt, 1)
    plain = model.steps(v, None, *args, mode="set")
    model.set_storage_model("inputs")
    got = model.steps(v, None, *args, mode="set")
    assert not np.array_equal(got, plain)
    # the same as feeding single-precision parameters, alpha and step to the
    # plain oracle, except for the tables and cell sizes, which only the model
    # rounds: the difference is a rounding-sized perturbation of the step
    model.set_storage_model("fp64")
    fed = model.steps(v, None, *p.grid_args(), p.dynamics, tuple(_r32(p.params)), p.scheme, 3,
                      _r32(alpha), float(_r32(dt)), 1, mode="set")
    assert np.abs(got - fed).max() < 1e-5
    assert np.abs(got - plain).max() < 1e-5


def test_solve_ignores_the_model(model):
    p, _ = _rough_problem()
    ref, *_ = model.solve(p.v0(), *p.grid_args(), p.dynamics, p.params, p.scheme, p.order,
                          p.cfl, 0.0, 0.05, "tube")
    model.set_storage_model("stages+inputs")
    got, *_ = model.solve(p.v0(), *p.grid_args(), p.dynamics, p.params, p.scheme, p.order,
                          p.cfl, 0.0, 0.05, "tube")
    assert np.array_equal(ref, got)
