"""Writes tests/golden/serving_stream_samples.txt: for the smallest and the
largest request of each family in the 256-request serving stream (seed 0: a
double integrator, a relative-Dubins tube and a 4-D Dubins set per end, all
WENO5/LF/RK3), the FP64 oracle's solution at up to 512 seeded front-band
nodes (|V| < 3 max(dx), at least 6 cells from a bounded edge) and 256 seeded
nodes anywhere, and the storage spreads in that band: how far the FP64 method
itself moves when everything a single-precision solve stores is single
precision (the oracle's FP32 storage model "stages+inputs": every RK stage
result, V0, tables, parameters, cell sizes, alpha and step size) while its
arithmetic stays FP64, in three realizations (V0 rounded; then nudged by -1,
0 or +1 single-precision ulp per node, seeded), as for the relative-Dubins
batch.  A request whose front lies only within 6 cells of the bounded edges
has no band nodes ("none"); its spread is taken over its 256 sampled nodes
instead ("sampled_spread").  Calls only the oracle and the input generators.
About 1.8e10 updates (four passes over the six requests): an hour on 8 build
host threads, about ten minutes on 16 faster cores.

    python tests/golden/make_serving_samples.py [--out DIR] [--merge DIR]
"""
import argparse
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2507_11542_amd import inputs  # noqa: E402

EDGE_CELLS = 6
REQUESTS = 256
GOLDEN = os.path.join(HERE, "serving_stream_samples.txt")


def picked(base):
    """Indices of the smallest and the largest request of each family (family
    order, smallest first)."""
    fam = {}
    for k, r in enumerate(base):
        fam.setdefault(r.problem.dynamics, []).append((r.problem.points, k))
    out = []
    for f in sorted(fam):
        lst = sorted(fam[f])
        out.extend([lst[0][1], lst[-1][1]])
    return out


def _stepped(p, alpha, dt, v0):
    """The oracle's time loop from v0 (the storage model set by the caller
    applies to every step): its full steps of dt in one call and the last,
    cut to land on tf, in another (the same step sizes as the loop)."""
    t, eps = p.t0, 100.0 * 2.220446049250313e-16
    hs = []
    while p.tf - t >= eps * (p.tf - p.t0):
        h = dt if dt < p.tf - t else p.tf - t
        hs.append(h)
        t = t + h
    full = len(hs) if hs and hs[-1] == dt else len(hs) - 1
    v = v0.copy()
    for h, k in ((dt, full), (hs[-1] if hs else dt, len(hs) - full)):
        if k:
            v = oracle.steps(v, v0, *p.grid_args(), p.dynamics, p.params, p.scheme, p.order,
                             alpha, h, k, mode=p.mode)
    return v


REALIZATIONS = 3


def realization_v0(p, k, r):
    """V0 in single precision for realization r of request k: rounded (r = 0),
    then nudged by -1, 0 or +1 ulp per node (r >= 1, seeded)."""
    v = p.v0().astype(np.float32)
    if r:
        z = np.random.default_rng(9500 + 97 * k + r).integers(-1, 2, size=v.shape)
        v = np.where(z > 0, np.nextafter(v, np.float32(np.inf)),
                     np.where(z < 0, np.nextafter(v, np.float32(-np.inf)), v))
    return v.astype(np.float64)


def request_record(k, p):
    dx = inputs.cell_sizes(*p.grid_args())
    old = oracle.set_dissipation(p.diss)
    try:
        ref, alpha, dt, steps = oracle.solve(p.v0(), *p.grid_args(), p.dynamics, p.params,
                                             p.scheme, p.order, p.cfl, p.t0, p.tf, p.mode)
        print("request %d: oracle solve done (%d steps)" % (k, steps), flush=True)
        keep = np.abs(ref) < 3.0 * float(np.max(dx))
        for d, per in enumerate(p.periodic):
            if not per:
                idx = np.arange(p.n[d])
                near = (idx < EDGE_CELLS) | (idx >= p.n[d] - EDGE_CELLS)
                shape = [1] * ref.ndim
                shape[d] = p.n[d]
                keep &= ~near.reshape(shape)
        band = np.flatnonzero(keep)
        rng = np.random.default_rng(5000 + k)
        band = rng.choice(band, size=min(512, band.size), replace=False)
        anywhere = rng.choice(ref.size, size=min(256, ref.size), replace=False)
        # the spread over the band, or over the sampled nodes when there is no band
        where = np.flatnonzero(keep) if keep.any() else anywhere
        spread = []
        for r in range(REALIZATIONS):
            store = oracle.set_storage_model("stages+inputs")
            try:
                got = _stepped(p, alpha, dt, realization_v0(p, k, r))
            finally:
                oracle.set_storage_model(store)
            spread.append(float(np.abs(got.ravel()[where] - ref.ravel()[where]).max()))
            print("request %d: realization %d spread %.3e" % (k, r, spread[-1]), flush=True)
    finally:
        oracle.set_dissipation(old)
    fmt = " ".join("%.6e" % x for x in spread)
    lines = ["# request %d %s n %s steps %d band %d %s\n"
             % (k, p.dynamics, "x".join(map(str, p.n)), steps, band.size,
                ("storage_spread " + fmt) if keep.any()
                else ("storage_spread none sampled_spread " + fmt))]
    lines.extend("%d %d 1 %.17g\n" % (k, i, ref.ravel()[i]) for i in np.sort(band))
    lines.extend("%d %d 0 %.17g\n" % (k, i, ref.ravel()[i]) for i in np.sort(anywhere))
    return lines, steps, spread


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="directory for the per-request records")
    ap.add_argument("--merge", default=None, help="merge the records of these directories "
                    "(comma separated) into the golden file")
    ap.add_argument("--threads", type=int, default=0)
    args = ap.parse_args()
    base = inputs.serving_stream(count=REQUESTS, rate=1.0, seed=0)
    ids = picked(base)
    if args.merge:
        dirs = args.merge.split(",")
        with open(GOLDEN, "w") as f:
            f.write("# FP64 oracle, smallest and largest request of each family of the "
                    "%d-request serving stream (seed 0)\n" % REQUESTS)
            f.write("# columns: request, flat C-order node index, 1 if front band else 0, "
                    "V(tf)\n")
            for k in ids:
                path = next(os.path.join(d, "req_%03d.txt" % k) for d in dirs
                            if os.path.exists(os.path.join(d, "req_%03d.txt" % k)))
                with open(path) as g:
                    f.write(g.read())
        print("wrote", GOLDEN)
        return
    out = args.out or os.path.join(ROOT, "gpurun_out", "serving_gold")
    os.makedirs(out, exist_ok=True)
    oracle.set_threads(args.threads)
    for k in ids:
        path = os.path.join(out, "req_%03d.txt" % k)
        if os.path.exists(path):
            continue
        p = base[k].problem
        lines, steps, spread = request_record(k, p)
        with open(path + ".tmp", "w") as f:
            f.writelines(lines)
        os.replace(path + ".tmp", path)
        print(k, p.dynamics, p.n, steps, spread, flush=True)


if __name__ == "__main__":
    main()
