"""Write the FP64 reference of the App. A elastic experiment (600 x 600,
free surfaces at the top and bottom rows, periodic in x, 60000 steps, Ricker
source on vy ten cells below the top surface, one receiver) with the oracle.

    python tests/golden/make_elastic2d_fp64.py

Output: elastic2d_app_a_fp64.csv next to this file -- the receiver's five
fields after every 50th step (rows "step,vx,vy,sxx,syy,sxy", step = number
of steps taken) and the energy every 500 steps (rows "E,step,value").  Calls
only the oracle and the input generators.
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle      # noqa: E402
import workloads   # noqa: E402

EVERY_TRACE = 50
EVERY_ENERGY = 500


def main(nsteps=60000):
    w = workloads.paper_elastic2d(nsteps=nsteps)
    t0 = time.time()
    f, _, energy, trace = oracle.elastic2d(
        w.nx, w.ny, w.dx, w.dt, w.rho, w.lam, w.mu, w.fields(), nsteps=nsteps,
        energy_every=EVERY_ENERGY, source=w.source, receivers=w.receivers)
    out = os.path.join(HERE, "elastic2d_app_a_fp64.csv")
    sx, sy, _ = w.source
    rx, ry = w.receivers[0]
    with open(out, "w") as fh:
        fh.write(f"# FP64 oracle, App. A setup: {w.nx}x{w.ny}, dx=1/125, dt=1e-4, "
                 f"free surfaces on rows 0 and {w.ny - 1}, periodic in x, "
                 f"layered medium (workloads.layered_elastic2d), Ricker 5 Hz on vy "
                 f"at ({sx},{sy}+1/2) delayed 0.24 s, receiver at ({rx},{ry}); "
                 f"written by make_elastic2d_fp64.py\n")
        for n in range(EVERY_TRACE, nsteps + 1, EVERY_TRACE):
            row = ",".join(f"{v:.17g}" for v in trace[n - 1, 0])
            fh.write(f"{n},{row}\n")
        for m, e in enumerate(energy):
            fh.write(f"E,{m * EVERY_ENERGY},{e:.17g}\n")
    print(f"wrote {out} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
