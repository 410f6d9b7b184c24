"""Writes tests/golden/rockets_100_vi_samples.txt: the FP64 oracle's rockets
game (100^3, ENO2/LF/RK3, CFL 0.8, t in [-2.5, 0], the variational-inequality
tube, 11 output times) at 2048 seeded node indices of the outputs at
t = -1.25 and t = 0.  Calls only the oracle and the input generators.

    python tests/golden/make_rockets_samples.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2507_11542_amd import inputs  # noqa: E402

OUTPUTS = (5, 10)  # indices into the 11 output times


def main():
    oracle.set_threads(0)
    p = inputs.rockets()
    times = inputs.output_times(p.t0, p.tf)
    outs, k = oracle.solve_outputs(p.v0(), *p.grid_args(), p.dynamics, p.params, times,
                                   p.scheme, p.order, p.cfl, p.t0, p.mode)
    idx = inputs.sample_nodes(p.n, 2048, seed=6041)
    path = os.path.join(HERE, "rockets_100_vi_samples.txt")
    with open(path, "w") as f:
        f.write("# FP64 oracle, rockets game 100^3 ENO2/LF/RK3 cfl 0.8, t in [-2.5, 0], "
                "variational-inequality tube, 11 output times; %d steps in all\n" % k)
        f.write("# columns: output index, flat C-order node index, V at that output\n")
        for o in OUTPUTS:
            for i in idx:
                f.write("%d %d %.17g\n" % (o, i, outs[o].ravel()[i]))
    print("wrote", path, k, "steps")


if __name__ == "__main__":
    main()
