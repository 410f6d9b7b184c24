"""Writes tests/golden/dubins4d_61_set_samples.txt: the FP64 oracle's 4-D
Dubins reachable set (61^4 on [-5,5]^2 x [-pi,pi) x [0,4], WENO5/LF/RK3,
CFL 0.8, t = 2) at 4096 seeded node indices.  Calls only the oracle and the
input generators.

    python tests/golden/make_dubins4d_samples.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2507_11542_amd import inputs  # noqa: E402


def main():
    oracle.set_threads(0)
    p = inputs.dubins4d()
    out, alpha, dt, k = oracle.solve(p.v0(), *p.grid_args(), p.dynamics, p.params, p.scheme,
                                     p.order, p.cfl, p.t0, p.tf, p.mode)
    idx = inputs.sample_nodes(p.n, 4096, seed=4461)
    path = os.path.join(HERE, "dubins4d_61_set_samples.txt")
    with open(path, "w") as f:
        f.write("# FP64 oracle, 4-D Dubins set 61^4 WENO5/LF/RK3 cfl 0.8 t=2; "
                "%d steps, dt=%.17g, alpha=%s\n" % (k, dt, [float(a) for a in alpha]))
        f.write("# columns: flat C-order node index, V(2)\n")
        for i in idx:
            f.write("%d %.17g\n" % (i, out.ravel()[i]))
    print("wrote", path, k, "steps")


if __name__ == "__main__":
    main()
