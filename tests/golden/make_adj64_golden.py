#!/usr/bin/env python3
"""Write the oracle's reference gradient for the 64^3 adjoint configuration.

Configuration: side-heated cavity (hot wall y = 0, cold wall at
T_c = T_m = 0), Ra = 1e4, Pr = 1, Ste = 0.1, front seeded at s0 = 1 with the
linear seed profile, hot-wall temperatures T_h(x, z) = 1 + 0.1 N(0, 1) from
the seeded generator of tests/inputs.py (seed 0), 100 steps from the initial
state.  The FP64 CPU oracle records the run and takes its reverse sweep:
d f_l / d T_h per column.  Values come from oracle/ only; nothing here
touches the GPU path.

Output (text): the liquid fraction at the end and the gradient of every
column ([z][x] order).
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

from inputs import hot_wall_field  # noqa: E402
from oracle import OracleSim  # noqa: E402

N, STEPS = 64, 100
OUT = os.path.join(HERE, "adj64_ra1e4_oracle_grad.txt")


def main():
    sim = OracleSim(N, ra=1e4, pr=1.0, ste=0.1, t_h=1.0, t_c=0.0, t_m=0.0, ma=0.1, s0=1.0,
                    heating=0, flow=1)
    sim.th[:] = hot_wall_field(N, seed=0)
    t0 = time.time()
    sim.record(STEPS)
    fl = sim.liquid_fraction()
    *_, grad = sim.adjoint()
    print(f"{STEPS} steps recorded and reversed in {time.time() - t0:.0f} s; f_l {fl:.12f}")
    with open(OUT, "w") as fh:
        fh.write("# FP64 oracle, 64^3 side-heated convection melting, Ra=1e4 Pr=1 Ste=0.1, "
                 "s0=1 linear seed, Ma=0.1, T_h = hot_wall_field(64, seed=0); "
                 "d f_l / d T_h after 100 steps; written by make_adj64_golden.py\n")
        fh.write(f"# steps {STEPS}\n")
        fh.write(f"fl {fl:.17e}\n")
        for c, v in enumerate(grad.reshape(-1)):
            fh.write(f"g {c} {v:.17e}\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
