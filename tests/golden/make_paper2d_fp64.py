"""Write the FP64 reference of the Sec. 3 acoustic experiment (600 x 600,
ppw = 10, 60000 steps, Ricker point source, one receiver) with the oracle.

    python tests/golden/make_paper2d_fp64.py

Output: paper2d_ppw10_fp64.csv next to this file -- the receiver's p, vx, vy
after every 50th step (rows "step,p,vx,vy", step = number of steps taken)
and the energy every 500 steps (rows "E,step,value").  Calls only the oracle
and the input generators.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle      # noqa: E402
import workloads   # noqa: E402

EVERY_TRACE = 50
EVERY_ENERGY = 500


def main(nsteps=60000):
    w = workloads.paper2d(ppw=10, nsteps=nsteps)
    t0 = time.time()
    f, _, energy, trace = oracle.acoustic2d(
        w.nx, w.ny, w.order, w.dx, w.dt, w.rho, w.kappa, w.fields(),
        nsteps=nsteps, energy_every=EVERY_ENERGY, source=w.source,
        receivers=w.receivers)
    out = os.path.join(HERE, "paper2d_ppw10_fp64.csv")
    with open(out, "w") as fh:
        fh.write("# FP64 oracle, Sec. 3 setup: 600x600, dx=1/125, dt=1e-4, order 4, "
                 "rho=c=1, Ricker 5 Hz point source on p at (200,200) delayed 0.24 s, "
                 "receiver at (400,400); written by make_paper2d_fp64.py\n")
        for n in range(EVERY_TRACE, nsteps + 1, EVERY_TRACE):
            p, vx, vy = trace[n - 1, 0]
            fh.write(f"{n},{p:.17g},{vx:.17g},{vy:.17g}\n")
        for m, e in enumerate(energy):
            fh.write(f"E,{m * EVERY_ENERGY},{e:.17g}\n")
    print(f"wrote {out} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
