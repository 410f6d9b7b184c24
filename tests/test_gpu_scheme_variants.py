"""The costate-box dissipation variants (local and global Lax-Friedrichs
coefficients) and ENO3 on the GPU against the FP64 oracle: FP64 solves and
single right-hand sides to 1e-12 for every dynamics; batches take LLF and
refuse GLF."""
import numpy as np
import pytest

from paper_2507_11542_amd import inputs

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu(orc):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    orc.set_threads(0)


def _cases():
    out = []
    for diss in ("llf", "glf"):
        out += [
            ("rel_dubins_%s" % diss, inputs.rel_dubins_3d(n=(23, 21, 18), tf=0.3).with_(
                diss=diss)),
            ("rel_dubins_eno3_%s" % diss, inputs.rel_dubins_3d(n=(19, 17, 16), tf=0.2,
                                                              scheme="eno3").with_(diss=diss)),
            ("rockets_vi_%s" % diss, inputs.rockets(n=(25, 23, 21)).with_(diss=diss)),
            ("dubins4d_%s" % diss, inputs.dubins4d(n=(13, 11, 10, 9), tf=0.2).with_(
                diss=diss)),
            ("double_integrator_%s" % diss, inputs.double_integrator_2d(n=61, tf=0.4).with_(
                diss=diss)),
            ("ball_3d_%s" % diss, inputs.Problem("ball", (19, 17, 15), (-2.0,) * 3, (2.0,) * 3,
                                                 (False, False, True), "ball", (1.0,), "weno5",
                                                 3, 0.8, 0.0, 0.3, "tube", radius=0.8,
                                                 diss=diss)),
        ]
    return out


CASES = _cases()


@pytest.mark.parametrize("name,p", CASES, ids=[c[0] for c in CASES])
def test_box_dissipation_solve_matches_oracle(orc, name, p):
    from gpu_util import gpu_solve, oracle_solve

    ref, *_ = oracle_solve(orc, p)
    got = gpu_solve(p, "fp64")
    assert np.abs(got - ref).max() <= TOL64, name


@pytest.mark.parametrize("diss", ["lf", "llf", "glf"])
@pytest.mark.parametrize("scheme", ["eno2", "eno3", "weno5"])
def test_rhs_on_rough_data(orc, diss, scheme):
    from gpu_util import gpu_rhs

    p = inputs.rel_dubins_3d(n=(17, 15, 12), scheme=scheme).with_(diss=diss)
    v = p.v0() + 0.3 * inputs.random_field(p.n, seed=9)
    got, alpha, dt, k = gpu_rhs(p, v)
    old = orc.set_dissipation(diss)
    try:
        ref = orc.rhs_at(v, *p.grid_args(), p.dynamics, p.params, scheme, alpha,
                         np.arange(p.points))
    finally:
        orc.set_dissipation(old)
    assert np.abs(got.ravel() - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


def test_batch_llf_equals_plain_and_glf_is_refused():
    import torch

    from gpu_util import gpu_solve, to_dev
    from paper_2507_11542_amd import hj

    probs = [inputs.rel_dubins_3d(n=(19, 17, 14), tf=0.2).with_(diss="llf"),
             inputs.rel_dubins_3d(n=(15, 17, 12), tf=0.3)]
    grids = [hj.Grid.from_problem(q, "fp64") for q in probs]
    v0s = [to_dev(q.v0()) for q in probs]
    outs = [torch.empty_like(v) for v in v0s]
    b = hj.Batch()
    st = torch.cuda.current_stream()
    try:
        b.solve(grids, v0s, outs, [q.t0 for q in probs], [q.tf for q in probs],
                [q.mode for q in probs], st)
        b.wait(len(probs), st)
        torch.cuda.synchronize()
        for q, o in zip(probs, outs):
            assert np.array_equal(o.cpu().numpy(), gpu_solve(q, "fp64"))
        grids[0].set_dissipation("glf")
        with pytest.raises(hj.HJError) as ei:
            b.solve(grids, v0s, outs, [q.t0 for q in probs], [q.tf for q in probs],
                    [q.mode for q in probs], st)
        assert ei.value.status == hj.HJ_E_UNSUPPORTED
    finally:
        b.close()
        for g in grids:
            g.close()


def test_glf_fp32_zero_set(orc):
    """FP32 with GLF on the 51^3 relative-Dubins tube: zero set within half a
    cell of the FP64 oracle's."""
    from gpu_util import gpu_solve, oracle_solve
    from paper_2507_11542_amd import metrics

    p = inputs.rel_dubins_3d(n=51, tf=1.0).with_(diss="glf")
    ref, *_ = oracle_solve(orc, p)
    got = gpu_solve(p, "fp32")
    assert metrics.hausdorff_cells(got, ref, p.periodic) <= 0.5
