"""Helpers for the GPU tests: run a Problem through libhj on cuda:0."""
import numpy as np


# Bar of an FP32 solve's front band against the FP64 oracle at a long
# horizon, in units of the largest band spread of three FP32-storage
# realizations of the oracle (FP64 arithmetic, single-precision storage, V0
# differing in its last bits).  The scheme amplifies last-bit differences of
# the stored state linearly, and the FP32 kernels perturb each stage result
# by up to 3 ulps (the local-step tests), against at most half an ulp for
# the storage model's rounding; the three realizations' spreads themselves
# differ by up to 90x for one instance, so their largest is a scale of the
# amplification, not an envelope of it.
SPREAD_BAR_FACTOR = 4.0


def torch_dtype(prec):
    import torch

    return torch.float64 if prec == "fp64" else torch.float32


def to_dev(a, prec="fp64"):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype=torch_dtype(prec))


def gpu_solve(p, prec="fp64", v0=None, t0=None, tf=None, mode=None):
    import torch

    from paper_2507_11542_amd import hj

    v0 = p.v0() if v0 is None else v0
    d0 = to_dev(v0, prec)
    out = torch.empty_like(d0)
    g = hj.Grid.from_problem(p, prec)
    try:
        g.solve(d0, out, p.t0 if t0 is None else t0, p.tf if tf is None else tf,
                p.mode if mode is None else mode, torch.cuda.current_stream())
        torch.cuda.synchronize()
    finally:
        g.close()
    return out.cpu().numpy().astype(np.float64)


def gpu_steps(p, v, v0, nsteps, prec="fp64", mode=None):
    """nsteps full steps of hj_step from (v, t0) toward p.tf; returns (V, t)."""
    import torch

    from paper_2507_11542_amd import hj

    dv = to_dev(v, prec)
    d0 = to_dev(v0, prec)
    g = hj.Grid.from_problem(p, prec)
    t = p.t0
    try:
        for _ in range(nsteps):
            t, _ = g.step(dv, d0, t, p.tf, p.mode if mode is None else mode,
                          torch.cuda.current_stream())
        torch.cuda.synchronize()
    finally:
        g.close()
    return dv.cpu().numpy().astype(np.float64), t


def gpu_rhs(p, v, prec="fp64"):
    import torch

    from paper_2507_11542_amd import hj

    dv = to_dev(v, prec)
    out = torch.empty_like(dv)
    g = hj.Grid.from_problem(p, prec)
    try:
        alpha, dt, k = g.schedule(p.t0, p.tf, torch.cuda.current_stream())
        g.rhs(dv, out, torch.cuda.current_stream())
        torch.cuda.synchronize()
    finally:
        g.close()
    return out.cpu().numpy().astype(np.float64), alpha, dt, k


def oracle_solve(orc, p, v0=None):
    v0 = p.v0() if v0 is None else v0
    old = orc.set_dissipation(p.diss)
    try:
        return orc.solve(v0, *p.grid_args(), p.dynamics, p.params, p.scheme, p.order, p.cfl,
                         p.t0, p.tf, p.mode)
    finally:
        orc.set_dissipation(old)
