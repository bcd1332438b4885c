"""GPU test of the serving loop: requests of mixed physics, size and
precision arrive over time under a small HBM budget (so some must wait);
each served result equals running the request alone, bit for bit."""
import numpy as np
import pytest

import paper_2310_00236_amd as hw
from paper_2310_00236_amd import serve
from helpers import assert_bitexact
import workloads

pytestmark = pytest.mark.gpu


def _request_inputs(kind, size, nsteps, prec, seed):
    storage, comp = ("f32", "none") if prec == "f32" else ("f16", "twosum")
    if kind == "acoustic2d":
        w = workloads.layered2d(size, size, nsteps=nsteps, npulses=1, seed=seed)
        pb = hw.Problem("acoustic2d", size, size, 1, 4, storage, comp, w.dx, w.dt, 0, 0)
        return pb, [w.rho, w.kappa], w.fields()
    w = workloads.smooth3d(size, nsteps=nsteps, seed=seed)
    pb = hw.Problem("elastic3d", size, size, size, 2, storage, comp, w.dx, w.dt, 0, 0)
    return pb, [w.rho, w.lam, w.mu], w.fields()


def test_served_results_equal_solo_runs():
    specs = [("acoustic2d", 200, 120, "f16+comp"), ("elastic3d", 24, 60, "f32"),
             ("acoustic2d", 96, 300, "f32"), ("acoustic2d", 160, 90, "f16+comp"),
             ("elastic3d", 20, 80, "f16+comp"), ("acoustic2d", 128, 200, "f16+comp"),
             ("acoustic2d", 64, 50, "f32"), ("elastic3d", 16, 110, "f16+comp")]
    jobs, inputs = [], []
    for i, (kind, size, steps, prec) in enumerate(specs):
        pb, mat, f = _request_inputs(kind, size, steps, prec, 9000 + i)
        inputs.append((pb, mat, f, steps))
        # six arrive together (they must share the device under the budget),
        # two arrive later and join whatever is still running
        arrival = 0.0 if i < 6 else 0.05 * (i - 5)
        jobs.append(serve.Job(id=i, arrival=arrival, footprint=hw.footprint(pb),
                              nsteps=steps, cells=pb.cells, payload=(pb, mat, f)))
    budget = sorted(j.footprint for j in jobs)[-1] + sorted(j.footprint for j in jobs)[-2]
    summary, done = serve.serve(jobs, budget, chunk_steps=20)
    assert summary["completed"] == len(specs)
    assert summary["max_resident_requests"] >= 2
    assert summary["peak_resident_bytes"] <= budget
    for j in done:
        pb, mat, f, steps = inputs[j.id]
        plan = hw.Plan(pb)
        plan.set_material(mat)
        plan.set_fields(f)
        plan.advance(steps)
        alone = plan.get_fields()
        plan.close()
        assert_bitexact(j.result[0], alone, f"request {j.id}")
