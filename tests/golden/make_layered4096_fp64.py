"""Write the FP64 reference energy of the 4096 x 4096 layered benchmark
workload (order 4, 4 layers, CFL 0.4, four Gaussian pulses) with the oracle.

    python tests/golden/make_layered4096_fp64.py [--starts f16,f32,bf16]
                                                 [--steps 10000] [--threads N]

For each storage format in --starts, the initial state is rounded to that
format (as the GPU library rounds it on upload); the FP64 oracle (fp64
storage, fp64 stencil, plain update) then runs from that rounded state and
its energy is written at step 0 and every 1000 steps up to --steps (0: the
starting energy only).  Rows "start,step,energy" are appended to
layered4096_fp64_energy.csv next to this file as they are computed, so an
interrupted run keeps what it finished.  Calls only the oracle and the
input generators.
"""
import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle      # noqa: E402
import workloads   # noqa: E402

OUT = os.path.join(HERE, "layered4096_fp64_energy.csv")
EVERY = 1000


def done_rows():
    rows = set()
    if os.path.exists(OUT):
        for line in open(OUT):
            if not line.startswith("#"):
                f = line.strip().split(",")
                rows.add((f[0], int(f[1])))
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--starts", default="f16,f32,bf16")
    ap.add_argument("--steps", type=int, default=0)
    ap.add_argument("--threads", type=int, default=0)
    args = ap.parse_args()
    w = workloads.layered2d(nsteps=10000)
    have = done_rows()
    if not os.path.exists(OUT):
        with open(OUT, "w") as fh:
            fh.write("# FP64 oracle energy of the 4096x4096 order-4 layered workload "
                     "(workloads.layered2d), started from the initial state rounded to "
                     "<start>; rows start,step,energy; written by "
                     "make_layered4096_fp64.py\n")
    for start in args.starts.split(","):
        steps_done = {n for (st, n) in have if st == start}
        f = {k: oracle.round_to(v, start) for k, v in w.fields().items()}
        if 0 not in steps_done:
            e0 = oracle.acoustic2d_energy(w.nx, w.ny, w.order, w.dx, w.dt, w.rho,
                                          w.kappa, f)
            with open(OUT, "a") as fh:
                fh.write(f"{start},0,{e0:.17g}\n")
        last = max(steps_done, default=0)
        if args.steps == 0 or last >= args.steps:
            continue
        if last > 0:
            raise SystemExit(f"{start}: rows up to step {last} exist; delete them to "
                             "run again from step 0")
        for n0 in range(0, args.steps, EVERY):
            t = time.time()
            f, _, e = oracle.acoustic2d(w.nx, w.ny, w.order, w.dx, w.dt, w.rho, w.kappa,
                                        f, storage="f64", stencil="f64", comp="none",
                                        nsteps=EVERY, energy_every=EVERY,
                                        nthreads=args.threads)
            with open(OUT, "a") as fh:
                fh.write(f"{start},{n0 + EVERY},{e[-1]:.17g}\n")
            print(f"{start} step {n0 + EVERY}: {e[-1]:.17g} ({time.time() - t:.0f} s)",
                  flush=True)


if __name__ == "__main__":
    main()
