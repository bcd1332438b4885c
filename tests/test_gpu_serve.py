"""GPU test of the serving loop: requests of mixed physics, size and
precision arrive over time under a small HBM budget (so some must wait);
requests of different kernel groups advance on their own streams, so their
launches overlap.  Each served result (fields and compensation terms)
equals the oracle's run of the request, and running the request alone, bit
for bit."""
import numpy as np
import pytest

import oracle
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


def _oracle_run(pb, mat, fields, nsteps):
    """The oracle from the request's initial state rounded to its storage
    format (as the library rounds it on upload)."""
    names = pb.field_names
    f = {k: oracle.round_to(fields[k] if fields.get(k) is not None
                            else np.zeros(pb.shape), pb.storage) for k in names}
    if pb.physics == "acoustic2d":
        return oracle.acoustic2d(pb.nx, pb.ny, pb.order, pb.dx, pb.dt, mat[0], mat[1], f,
                                 storage=pb.storage, stencil="f32", comp=pb.comp,
                                 nsteps=nsteps)
    return oracle.elastic3d(pb.nx, pb.ny, pb.nz, pb.dx, pb.dt, mat[0], mat[1], mat[2], f,
                            storage=pb.storage, stencil="f32", comp=pb.comp,
                            nsteps=nsteps)


def test_served_results_equal_oracle_and_solo_runs():
    specs = [("acoustic2d", 200, 120, "f16+comp"), ("elastic3d", 24, 60, "f32"),
             ("acoustic2d", 96, 300, "f32"), ("acoustic2d", 160, 90, "f16+comp"),
             ("elastic3d", 20, 80, "f16+comp"), ("acoustic2d", 128, 200, "f16+comp"),
             ("acoustic2d", 64, 50, "f32"), ("elastic3d", 16, 110, "f16+comp"),
             ("elastic3d", 18, 70, "f32"), ("acoustic2d", 150, 130, "f32")]
    jobs, inputs = [], []
    for i, (kind, size, steps, prec) in enumerate(specs):
        pb, mat, f = _request_inputs(kind, size, steps, prec, 9000 + i)
        inputs.append((pb, mat, f, steps))
        # six arrive together (they must share the device under the budget),
        # the others arrive later and join whatever is still running
        arrival = 0.0 if i < 6 else 0.05 * (i - 5)
        jobs.append(serve.Job(id=i, arrival=arrival, footprint=hw.footprint(pb),
                              nsteps=steps, cells=pb.cells, payload=(pb, mat, f)))
    fps = sorted(j.footprint for j in jobs)
    budget = fps[-1] + fps[-2]
    summary, done = serve.serve(jobs, budget, chunk_steps=20)
    assert summary["completed"] == len(specs)
    assert summary["max_resident_requests"] >= 2
    assert summary["peak_resident_bytes"] <= budget
    assert summary["p99_queueing_s"] > 0          # the budget made some wait
    for j in done:
        pb, mat, f, steps = inputs[j.id]
        got, _, got_c = j.result
        want, want_c, _ = _oracle_run(pb, mat, f, steps)
        assert_bitexact(got, want, f"request {j.id} vs oracle")
        if pb.comp != "none":
            assert_bitexact(got_c, want_c, f"request {j.id} comps vs oracle")
        plan = hw.Plan(pb)
        plan.set_material(mat)
        plan.set_fields(f)
        plan.advance(steps)
        alone = plan.get_fields()
        plan.close()
        assert_bitexact(got, alone, f"request {j.id} vs solo")


def test_groups_get_their_own_streams():
    """Four kernel groups (2D/3D x fp32/fp16+comp) map to four distinct
    streams; a fifth group shares one of them."""
    ex = serve.GpuExecutor()
    keys = [("acoustic2d", 4, "f32", "none"), ("acoustic2d", 4, "f16", "twosum"),
            ("elastic3d", 2, "f32", "none"), ("elastic3d", 2, "f16", "twosum"),
            ("acoustic2d", 4, "bf16", "twosum")]
    streams = [ex._stream(k) for k in keys]
    assert len({s.cuda_stream for s in streams[:4]}) == 4
    assert streams[4].cuda_stream in {s.cuda_stream for s in streams[:4]}
    assert all(s.priority == 0 for s in streams)
