"""Writes the stored expected values under tests/golden/ from the oracle only
(run: python tests/golden/make_golden.py).  Each file names the passage it
follows."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
import spd_problems as P  # noqa: E402


def leja():
    t = O.leja_reference_points(16)
    with open(os.path.join(HERE, "leja_points_16.txt"), "w") as f:
        f.write("# Leja points of [-1, 1] in the order of (2.7): t0 = 1, t1 = -1, then each point\n")
        f.write("# maximizes prod |t - t_m| over [-1, 1]; ties (products equal to 1e-9 relative)\n")
        f.write("# go to the smaller t.  Written by tests/golden/make_golden.py from oracle/basis.py.\n")
        for v in t:
            f.write(f"{v:.17g}\n")


def trace():
    pr = P.make_config("poisson2d_64")
    _, info = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, s_max=10, tol=1e-10, basis="chebyshev")
    with open(os.path.join(HERE, "poisson2d_64_chebyshev_s10.txt"), "w") as f:
        f.write("# Algorithm 5 (Chebyshev basis, sigma = s-bar_0 = f = 10, eps* = 1e-10) on the 2-D\n")
        f.write("# 5-point Poisson 64 x 64 workload (scaled, b = A x*, x* ~ U(-1, 1) seed 101, x0 = 0).\n")
        f.write("# Written by tests/golden/make_golden.py from oracle/sstep.py.\n")
        f.write(f"# outcome {info['outcome'].name} outer {info['outer']} iters {info['iters']} "
                f"relres_true {info['relres_true']:.17g}\n")
        f.write("# k sbar stilde sk relres_updated\n")
        for t in info["trace"]:
            f.write(f"{t['k']} {t['sbar']} {t['stilde']} {t['sk']} {t['relres_updated']:.17g}\n")


if __name__ == "__main__":
    leja()
    trace()
