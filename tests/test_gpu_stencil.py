"""GPU parity of the stencil-precision variants (the all-fp16 step of
Alg. 1 read literally, and App. B's stencil promoted to fp64 with the update
kept in the storage format) against the oracle's modes: fields,
compensation terms and receiver traces bit-identical, with a point source
(its fp32 samples rounded to the storage format inside the step for the
storage-format stencil)."""
import numpy as np
import pytest

import oracle
import paper_2310_00236_amd as hw
import workloads
from helpers import acoustic_fields, assert_bitexact, layered_material

pytestmark = pytest.mark.gpu

NX, NY = 150, 37
SRC = (77, 16)
RECS = [(0, 0), (63, 15), (64, 16), SRC]


@pytest.mark.parametrize("stencil", ["storage", "f64"])
@pytest.mark.parametrize("storage,comp,order", [
    ("f16", "none", 4), ("f16", "twosum", 4), ("f16", "fast2sum", 2),
    ("bf16", "none", 4), ("bf16", "twosum", 4), ("f32", "none", 4),
    ("f32", "twosum", 2)])
def test_stencil_precision_bitexact(storage, comp, order, stencil):
    rho, kappa, c = layered_material(NX, NY, 701)
    dt = 0.4 * hw.cfl_bound("acoustic2d", order) / c
    f = acoustic_fields(NX, NY, 702, storage, vel=0.02)
    t = (np.arange(25) + 0.5) * dt - 0.8
    samples = oracle.round_to(0.8 * workloads.ricker(t, 1.5), "f32")
    nsteps = 40
    pb = hw.Problem("acoustic2d", NX, NY, 1, order, storage, comp, 1.0, dt, 0,
                    nsteps // 10 + 2, src_cap=len(samples), rec_cap=len(RECS),
                    rec_steps=nsteps, stencil=stencil)
    plan = hw.Plan(pb)
    plan.set_material([rho, kappa])
    plan.set_fields(f)
    plan.set_source(SRC[0], SRC[1], samples)
    plan.set_receivers(RECS)
    plan.advance(nsteps, 10)
    g, gc = plan.get_fields(comps=True)
    gt = plan.receiver_trace()
    ge, _ = plan.energy_trace()
    plan.close()
    fr = {k: oracle.round_to(v, storage) for k, v in f.items()}
    w, wc, we, wt = oracle.acoustic2d(
        NX, NY, order, 1.0, dt, rho, kappa, fr, storage=storage,
        stencil=storage if stencil == "storage" else "f64", comp=comp,
        nsteps=nsteps, energy_every=10, source=(SRC[0], SRC[1], samples),
        receivers=RECS)
    assert_bitexact(g, w, f"{stencil} fields")
    if comp != "none":
        assert_bitexact(gc, wc, f"{stencil} comps")
    assert np.array_equal(gt, wt)
    np.testing.assert_allclose(ge, we, rtol=1e-12, atol=0)


def test_stencil_variants_in_a_batch_and_without_source():
    """Plans with different stencil precisions in one batch_advance call are
    launched separately and each matches its oracle mode; no source."""
    rho, kappa, c = layered_material(NX, NY, 711)
    dt = 0.4 * hw.cfl_bound("acoustic2d", 4) / c
    f = acoustic_fields(NX, NY, 712, "f16", vel=0.02)
    plans = []
    for st in ("f32", "storage", "f64"):
        pb = hw.Problem("acoustic2d", NX, NY, 1, 4, "f16", "twosum", 1.0, dt, 0, 0,
                        stencil=st)
        p = hw.Plan(pb)
        p.set_material([rho, kappa])
        p.set_fields(f)
        plans.append(p)
    hw.batch_advance(plans, [30, 35, 40])
    fr = {k: oracle.round_to(v, "f16") for k, v in f.items()}
    for p, st, n in zip(plans, ("f32", "f16", "f64"), (30, 35, 40)):
        w, wc, _ = oracle.acoustic2d(NX, NY, 4, 1.0, dt, rho, kappa, fr, storage="f16",
                                     stencil=st, comp="twosum", nsteps=n)
        g, gc = p.get_fields(comps=True)
        assert_bitexact(g, w, st)
        assert_bitexact(gc, wc, st + " comps")
        p.close()
