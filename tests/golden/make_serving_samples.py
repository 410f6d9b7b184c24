"""Writes tests/golden/serving_stream_samples.txt: for the smallest request of
each family in the 96-request serving stream (seed 0: a double integrator, a
relative-Dubins tube and a 4-D Dubins set, WENO5/LF/RK3), the FP64 oracle's
solution at up to 512 seeded front-band nodes (|V| < 3 max(dx), at least 6
cells from a bounded edge) and 256 seeded nodes anywhere, and the oracle's own
spread in that band when its state is rounded to FP32 after every step
(storage) and also multiplied by (1 + 2^-23 z), z seeded normal, first
(noise), as for the relative-Dubins batch.  Calls only the oracle and the
input generators.

    python tests/golden/make_serving_samples.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2507_11542_amd import inputs  # noqa: E402

EDGE_CELLS = 6


def picked(base):
    """Index of the smallest request of each family, in family order."""
    best = {}
    for k, r in enumerate(base):
        p = r.problem
        if p.dynamics not in best or p.points < base[best[p.dynamics]].problem.points:
            best[p.dynamics] = k
    return [best[f] for f in sorted(best)]


def _stepped(p, alpha, dt, perturb):
    """The oracle's time loop one step at a time, perturb applied after each."""
    v0 = p.v0()
    v = perturb(v0.copy())
    t, eps = p.t0, 100.0 * 2.220446049250313e-16
    while p.tf - t >= eps * (p.tf - p.t0):
        h = dt if dt < p.tf - t else p.tf - t
        v = perturb(oracle.steps(v, v0, *p.grid_args(), p.dynamics, p.params, p.scheme,
                                 p.order, alpha, h, 1, mode=p.mode))
        t = t + h
    return v


def main():
    oracle.set_threads(0)
    base = inputs.serving_stream(count=96, rate=1.0, seed=0)
    lines = []
    for k in picked(base):
        p = base[k].problem
        old = oracle.set_dissipation(p.diss)
        try:
            ref, alpha, dt, steps = oracle.solve(p.v0(), *p.grid_args(), p.dynamics, p.params,
                                                 p.scheme, p.order, p.cfl, p.t0, p.tf, p.mode)
        finally:
            oracle.set_dissipation(old)
        dx = inputs.cell_sizes(*p.grid_args())
        keep = np.abs(ref) < 3.0 * float(np.max(dx))
        for d, per in enumerate(p.periodic):
            if not per:
                idx = np.arange(p.n[d])
                near = (idx < EDGE_CELLS) | (idx >= p.n[d] - EDGE_CELLS)
                shape = [1] * ref.ndim
                shape[d] = p.n[d]
                keep &= ~near.reshape(shape)
        spread = {}
        nrng = np.random.default_rng(7100 + k)

        def rounded(v):
            return v.astype(np.float32).astype(np.float64)

        def noisy(v):
            return rounded(v * (1.0 + 2.0 ** -23 * nrng.standard_normal(v.shape)))

        old = oracle.set_dissipation(p.diss)
        try:
            for name, fn in (("storage", rounded), ("noise", noisy)):
                got = _stepped(p, alpha, dt, fn)
                spread[name] = float(np.abs(got - ref)[keep].max())
        finally:
            oracle.set_dissipation(old)
        band = np.flatnonzero(keep)
        rng = np.random.default_rng(5000 + k)
        band = rng.choice(band, size=min(512, band.size), replace=False)
        anywhere = rng.choice(ref.size, size=min(256, ref.size), replace=False)
        lines.append("# request %d %s n %s steps %d band %d storage_spread %.6e "
                     "noise_spread %.6e\n"
                     % (k, p.dynamics, "x".join(map(str, p.n)), steps, band.size,
                        spread["storage"], spread["noise"]))
        lines.extend("%d %d 1 %.17g\n" % (k, i, ref.ravel()[i]) for i in np.sort(band))
        lines.extend("%d %d 0 %.17g\n" % (k, i, ref.ravel()[i]) for i in np.sort(anywhere))
        print(k, p.dynamics, p.n, steps, spread, flush=True)
    path = os.path.join(HERE, "serving_stream_samples.txt")
    with open(path, "w") as f:
        f.write("# FP64 oracle, smallest request of each family of the 96-request serving "
                "stream (seed 0)\n")
        f.write("# columns: request, flat C-order node index, 1 if front band else 0, V(tf)\n")
        f.writelines(lines)
    print("wrote", path)


if __name__ == "__main__":
    main()
