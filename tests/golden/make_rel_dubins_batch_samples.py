"""Writes tests/golden/rel_dubins_batch_samples.txt: for every instance of the
64-instance relative-Dubins batch (rng 0; N ~ U{51, 61, 81, 101}, WENO5/LF/RK3,
CFL 0.8, tube, t = 2.8):

- the FP64 oracle's value at up to 512 seeded front-band nodes (|V| < 3 max(dx),
  at least 6 cells from a bounded edge);
- the oracle's zero set in three psi slices (psi index n/4, n/2, 3n/4): the
  crossing points of the slice's grid edges, in cell units (for the zero-set
  Hausdorff distance);
- how the FP64 method itself responds to single-precision storage, with the
  oracle's FP32 storage model (``oracle.set_storage_model``) from V0 rounded to
  single precision, max over the same band:
    stage spread        every RK stage result rounded as it is stored;
    stage+input spread  the same, with the tables, parameters, cell sizes,
                        alpha and step size in single precision as well.
  Both runs repeat the oracle's time loop step by step (the last step cut to
  land on t = 2.8); the plain run equals the oracle's solve bit for bit.

Calls only the oracle and the input generators.  At about 6 M updates/s on 8
host threads the whole batch takes about 3 hours (three passes of 2.5e10
updates); records are written one instance at a time, so a run can be split
or resumed:

    python tests/golden/make_rel_dubins_batch_samples.py --out DIR [--instances A:B]
    python tests/golden/make_rel_dubins_batch_samples.py --merge DIR
"""
import argparse
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2507_11542_amd import inputs, metrics  # noqa: E402

BAND_CELLS = 3.0
EDGE_CELLS = 6
SAMPLES = 512
GOLDEN = os.path.join(HERE, "rel_dubins_batch_samples.txt")


def slices(n):
    return (n // 4, n // 2, (3 * n) // 4)


def _r32(v):
    return v.astype(np.float32).astype(np.float64)


def _stepped(p, alpha, dt, v0):
    """The oracle's time loop one step at a time from v0 (the model set by
    the caller applies to each step)."""
    v = v0.copy()
    t, eps = p.t0, 100.0 * 2.220446049250313e-16
    while p.tf - t >= eps * (p.tf - p.t0):
        h = dt if dt < p.tf - t else p.tf - t
        v = oracle.steps(v, v0, *p.grid_args(), p.dynamics, p.params, p.scheme, p.order,
                         alpha, h, 1, mode=p.mode)
        t = t + h
    return v


def band_inner(p, ref):
    dx = inputs.cell_sizes(*p.grid_args())
    band = np.abs(ref) < BAND_CELLS * float(np.max(dx))
    edge = np.zeros(ref.shape, dtype=bool)
    for d, per in enumerate(p.periodic):
        if not per:
            idx = np.arange(p.n[d])
            near = (idx < EDGE_CELLS) | (idx >= p.n[d] - EDGE_CELLS)
            shape = [1] * ref.ndim
            shape[d] = p.n[d]
            edge |= near.reshape(shape)
    return band & ~edge


def instance_record(k, p):
    ref, alpha, dt, steps = oracle.solve(p.v0(), *p.grid_args(), p.dynamics, p.params,
                                         p.scheme, p.order, p.cfl, p.t0, p.tf, p.mode)
    assert np.array_equal(_stepped(p, alpha, dt, p.v0()), ref)
    mask = band_inner(p, ref)
    spread = {}
    for name in ("stages", "stages+inputs"):
        old = oracle.set_storage_model(name)
        try:
            got = _stepped(p, alpha, dt, _r32(p.v0()))
        finally:
            oracle.set_storage_model(old)
        spread[name] = float(np.abs(got - ref)[mask].max())
    nodes = np.flatnonzero(mask)
    sel = np.sort(np.random.default_rng(4100 + k).choice(
        nodes, size=min(SAMPLES, nodes.size), replace=False))
    lines = ["# instance %d n %d steps %d stage_spread %.6e stage_input_spread %.6e\n"
             % (k, p.n[0], steps, spread["stages"], spread["stages+inputs"])]
    lines.extend("s %d %d %.17g\n" % (k, i, ref.ravel()[i]) for i in sel)
    for j, s in enumerate(slices(p.n[2])):
        pts = metrics.zero_set_points(ref[:, :, s], (False, False))
        lines.extend("z %d %d %.6f %.6f\n" % (k, j, a, b) for a, b in pts)
    return lines, steps, spread


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", help="directory for the per-instance records")
    ap.add_argument("--instances", default="0:64")
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--merge", help="merge the records of this directory into the golden file")
    args = ap.parse_args()
    probs = inputs.rel_dubins_batch()
    if args.merge:
        with open(GOLDEN, "w") as f:
            f.write("# FP64 oracle, the 64-instance relative-Dubins batch (rng 0), "
                    "WENO5/LF/RK3 cfl 0.8 tube t=2.8\n")
            f.write("# s rows: instance, flat C-order node index, V(2.8) at front-band nodes\n")
            f.write("# z rows: instance, slice (psi index n/4, n/2, 3n/4), zero-set crossing "
                    "point (axis-0, axis-1 index units)\n")
            for k in range(len(probs)):
                with open(os.path.join(args.merge, "inst_%02d.txt" % k)) as g:
                    f.write(g.read())
        print("wrote", GOLDEN)
        return
    os.makedirs(args.out, exist_ok=True)
    oracle.set_threads(args.threads)
    a, b = (int(x) for x in args.instances.split(":"))
    for k in range(a, b):
        path = os.path.join(args.out, "inst_%02d.txt" % k)
        if os.path.exists(path):
            continue
        lines, steps, spread = instance_record(k, probs[k])
        with open(path + ".tmp", "w") as f:
            f.writelines(lines)
        os.replace(path + ".tmp", path)
        print(k, probs[k].n[0], steps, spread, flush=True)


if __name__ == "__main__":
    main()
