#!/usr/bin/env python3
"""Write the oracle reference for the 64^3 convection-melting run.

Configuration: side-heated cavity (hot wall y = 0 at T_h = 1, cold wall at
T_c = T_m = 0), Ra = 1e4, Pr = 1, Ste = 0.1, front seeded at s0 = 1 with the
linear seed profile, 20000 steps.  Values come from the FP64 CPU oracle only
(oracle/); nothing here touches the GPU path.

Output (text): the liquid fraction every 500 steps, the front of every column
at the end, and the temperature at 2048 seeded cell indices plus the full
mid-plane line x = z = 32 at the end.  Output (binary, numpy .npy, FP64): the
whole final temperature field, [z][y][x].
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import OracleSim  # noqa: E402

N, STEPS, EVERY = 64, 20000, 500
OUT = os.path.join(HERE, "conv64_ra1e4_oracle.txt")
OUT_T = os.path.join(HERE, "conv64_ra1e4_oracle_T.npy")


def sample_cells(n, k=2048, seed=12345):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n ** 3, size=k, replace=False))


def main():
    sim = OracleSim(N, ra=1e4, pr=1.0, ste=0.1, t_h=1.0, t_c=0.0, t_m=0.0, ma=0.1, s0=1.0,
                    heating=0, flow=1)
    fl = []
    t0 = time.time()
    for k in range(STEPS // EVERY):
        sim.step(EVERY)
        fl.append((sim.steps, sim.liquid_fraction()))
        print(f"step {sim.steps} fl {fl[-1][1]:.10f} ({time.time() - t0:.0f} s)", flush=True)
    F = sim.fields()
    T = F["T"].reshape(-1)
    cells = sample_cells(N)
    line = F["T"][N // 2, :, N // 2]
    with open(OUT, "w") as fh:
        fh.write("# FP64 oracle, 64^3 side-heated convection melting, Ra=1e4 Pr=1 Ste=0.1, "
                 "s0=1 linear seed, Ma=0.1; written by make_conv64_golden.py\n")
        fh.write(f"# steps {STEPS}\n")
        for st, v in fl:
            fh.write(f"fl {st} {v:.17e}\n")
        for c, v in enumerate(sim.s.reshape(-1)):
            fh.write(f"s {c} {v:.17e}\n")
        for c in cells:
            fh.write(f"T {c} {T[c]:.17e}\n")
        for y, v in enumerate(line):
            fh.write(f"Tline {y} {v:.17e}\n")
    np.save(OUT_T, np.ascontiguousarray(F["T"], dtype=np.float64), allow_pickle=False)
    print("wrote", OUT, OUT_T)


if __name__ == "__main__":
    main()
