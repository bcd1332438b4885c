"""GPU tests of the runtime around the kernels: batched launches, checkpoint
and resume, energy trace bookkeeping, the blocking convenience call."""
import numpy as np
import pytest

import paper_2310_00236_amd as hw
import workloads
from helpers import (acoustic_fields, assert_bitexact, elastic_fields,
                     gpu_acoustic, layered_material, oracle_acoustic,
                     smooth_medium3d)

pytestmark = pytest.mark.gpu


def _acoustic_plan(nx, ny, storage, comp, seed, trace_cap=64, order=4):
    rho, kappa, c = layered_material(nx, ny, seed)
    dt = 0.4 * hw.cfl_bound("acoustic2d", order) / c
    pb = hw.Problem("acoustic2d", nx, ny, 1, order, storage, comp, 1.0, dt, 0,
                    trace_cap)
    plan = hw.Plan(pb)
    plan.set_material([rho, kappa])
    plan.set_fields(acoustic_fields(nx, ny, seed + 1, storage))
    return plan


def _elastic_plan(n, storage, comp, seed, trace_cap=64):
    rho, lam, mu, cp = smooth_medium3d(n, n + 1, n - 1, seed)
    dt = 0.4 * hw.cfl_bound("elastic3d", 2) / cp
    pb = hw.Problem("elastic3d", n, n + 1, n - 1, 2, storage, comp, 1.0, dt, 0,
                    trace_cap)
    plan = hw.Plan(pb)
    plan.set_material([rho, lam, mu])
    plan.set_fields(elastic_fields(n, n + 1, n - 1, seed + 1))
    return plan


@pytest.mark.parametrize("tile", [1, 2])
def test_batch_bit_identical_to_single_runs(tile):
    """Mixed batch: uneven 2D shots of two precisions, 3D shots, uneven step
    counts; every plan ends bit-identical to running it alone, energy traces
    included.  Tile 1 runs the 3D shots through the two-pass kernels, tile 2
    through the fused marching kernel."""
    specs = [("a", 300, 170, "f16", "twosum", 37), ("a", 129, 400, "f16", "twosum", 20),
             ("a", 64, 64, "f32", "none", 45), ("a", 250, 33, "f16", "twosum", 0),
             ("e", 20, "f16", "twosum", 15), ("e", 12, "f32", "none", 9)]

    def make(s, seed):
        if s[0] == "a":
            return _acoustic_plan(s[1], s[2], s[3], s[4], seed)
        return _elastic_plan(s[1], s[2], s[3], seed)

    steps = [s[-1] for s in specs]
    batch = [make(s, 300 + 10 * i) for i, s in enumerate(specs)]
    hw.batch_advance(batch, steps, energy_every=5, tile=tile)
    alone = [make(s, 300 + 10 * i) for i, s in enumerate(specs)]
    for p, n in zip(alone, steps):
        p.advance(n, energy_every=5)
    for pb_, pa, n in zip(batch, alone, steps):
        fb, cb = pb_.get_fields(comps=True)
        fa, ca = pa.get_fields(comps=True)
        assert_bitexact(fb, fa, "batch fields")
        assert_bitexact(cb, ca, "batch comps")
        eb, sb = pb_.energy_trace()
        ea, sa = pa.energy_trace()
        assert np.array_equal(sb, sa) and np.array_equal(eb, ea)
        assert pb_.step == pa.step == n
    for p in batch + alone:
        p.close()


def test_batch_of_many_shots_crosses_launch_limit():
    plans = [_acoustic_plan(40 + i, 30 + (i % 7), "f16", "twosum", 500 + i,
                            order=2) for i in range(70)]
    steps = [3 + (i % 5) for i in range(70)]
    hw.batch_advance(plans, steps)
    for i in (0, 33, 64, 69):
        ref = _acoustic_plan(40 + i, 30 + (i % 7), "f16", "twosum", 500 + i,
                             order=2)
        ref.advance(steps[i])
        assert_bitexact(plans[i].get_fields(), ref.get_fields(), f"shot {i}")
        ref.close()
    for p in plans:
        p.close()


@pytest.mark.parametrize("physics", ["acoustic2d", "elastic3d"])
def test_checkpoint_resume_bit_exact(physics):
    mk = (lambda: _acoustic_plan(90, 50, "f16", "twosum", 700)) \
        if physics == "acoustic2d" else (lambda: _elastic_plan(14, "f16", "twosum", 710))
    straight = mk()
    straight.advance(40)
    want, wantc = straight.get_fields(comps=True)
    half = mk()
    half.advance(17)
    blob = half.export_state()
    half.advance(5)                 # diverge, then restore
    other = mk()
    other.import_state(blob)
    assert other.step == 17
    other.advance(23)
    got, gotc = other.get_fields(comps=True)
    assert_bitexact(got, want, "resumed")
    assert_bitexact(gotc, wantc, "resumed comps")
    for p in (straight, half, other):
        p.close()


@pytest.mark.parametrize("physics,comp", [("acoustic2d", "twosum"),
                                           ("acoustic2d", "twosum8"),
                                           ("elastic3d", "twosum")])
def test_exported_state_does_not_depend_on_the_arena(physics, comp):
    """A state blob holds every field's padded words; after an odd number of
    steps (and after an import) they come from the second field set, whose
    padding no kernel writes.  Two plans whose arenas held different bytes
    must still export identical blobs."""
    import torch
    if physics == "acoustic2d":
        nx, ny, nz = 70, 21, 1          # pitch 128: 58 padding words per row
        rho, kappa, c = layered_material(nx, ny, 720)
        mat = [rho, kappa]
        f = acoustic_fields(nx, ny, 721, "f16")
        order = 4
    else:
        nx, ny, nz = 13, 9, 7
        rho, lam, mu, c = smooth_medium3d(nx, ny, nz, 722)
        mat = [rho, lam, mu]
        f = elastic_fields(nx, ny, nz, 723)
        order = 2
    dt = 0.4 * hw.cfl_bound(physics, order) / c
    pb = hw.Problem(physics, nx, ny, nz, order, "f16", comp, 1.0, dt, 0, 0)
    blobs = []
    for fill in (0x00, 0xA5):
        arena = torch.full((hw.footprint(pb),), fill, dtype=torch.uint8,
                           device="cuda:0")
        p = hw.Plan(pb, arena=arena)
        p.set_material(mat)
        p.set_fields(f)
        p.advance(7)
        first = p.export_state()
        q = hw.Plan(pb, arena=torch.full_like(arena, 0xFF - fill))
        q.set_material(mat)
        q.import_state(first)
        q.advance(5)
        blobs.append((first, q.export_state()))
        p.close()
        q.close()
    same = [a == b for a, b in zip(blobs[0], blobs[1])]
    assert same == [True, True]


def test_energy_trace_bookkeeping():
    plan = _acoustic_plan(50, 40, "f32", "none", 800, trace_cap=8)
    plan.advance(7, energy_every=3)       # steps 0, 3, 6
    plan.advance(5, energy_every=3)       # steps 9, 12 (6 not repeated)
    e, s = plan.energy_trace()
    assert s.tolist() == [0, 3, 6, 9, 12]
    with pytest.raises(hw.HalfwaveError) as ei:
        plan.advance(30, energy_every=3)
    assert ei.value.name == "HW_E_NOMEM"
    assert plan.step == 12                # nothing was launched
    plan.record_energy()
    e2, s2 = plan.energy_trace()
    assert s2.tolist() == [0, 3, 6, 9, 12, 12] and e2[-1] == e2[-2]
    plan.close()


def test_simulate_matches_plan_api():
    nx, ny = 96, 80
    rho, kappa, c = layered_material(nx, ny, 900)
    dt = 0.4 * hw.cfl_bound("acoustic2d", 4) / c
    f = acoustic_fields(nx, ny, 901, "f16")
    pb = hw.Problem("acoustic2d", nx, ny, 1, 4, "f16", "twosum", 1.0, dt, 0, 16)
    out, e = hw.simulate(pb, [rho, kappa], f, 30, energy_every=10)
    g, _, ge = gpu_acoustic(nx, ny, 4, "f16", "twosum", dt, rho, kappa, f, 30,
                            energy_every=10)
    assert_bitexact(out, g, "simulate")
    assert np.array_equal(e, ge)


@pytest.mark.parametrize("physics,storage,comp", [("acoustic2d", "f16", "twosum"),
                                                   ("acoustic2d", "f16", "twosum8"),
                                                   ("elastic3d", "f32", "none")])
def test_tuned_tile_matches_default_shape(physics, storage, comp):
    """Plan.set_tuned_tile() sets the tuning table's shape for the plan and
    returns it; the run is bit-identical to the default shape's."""
    from paper_2310_00236_amd import tuning
    plans = []
    for tuned in (False, True):
        if physics == "acoustic2d":
            p = _acoustic_plan(300, 130, storage, comp, 905)
        else:
            p = _elastic_plan(20, storage, comp, 906)
        if tuned:
            t = p.set_tuned_tile()
            pb = p.pb
            assert t == tuning.best_tile(pb.physics, pb.order, pb.storage, pb.comp,
                                         pb.nx, pb.ny, pb.nz)
            if physics == "acoustic2d":
                assert hw.tiles(physics)[t][2] == 2          # two steps per launch
        p.advance(21, energy_every=7)
        plans.append((p.get_fields(comps=True), p.energy_trace()[0]))
        p.close()
    (g0, c0), e0 = plans[0]
    (g1, c1), e1 = plans[1]
    assert_bitexact(g1, g0, "tuned shape")
    assert_bitexact(c1, c0, "tuned shape comps")
    assert np.array_equal(e1, e0)


@pytest.mark.parametrize("physics,storage,comp", [("acoustic2d", "f16", "twosum8"),
                                                   ("elastic3d", "f16", "twosum"),
                                                   ("elastic3d", "bf16", "none")])
def test_simulate_matches_oracle(physics, storage, comp):
    """hw_simulate (two-step 2D shape, fused 3D shape) against the oracle
    directly, with an odd step count."""
    if physics == "acoustic2d":
        nx, ny, nz = 131, 45, 1
        rho, kappa, c = layered_material(nx, ny, 907)
        dt = 0.4 * hw.cfl_bound(physics, 4) / c
        f = acoustic_fields(nx, ny, 908, storage)
        mat = [rho, kappa]
        pb = hw.Problem(physics, nx, ny, nz, 4, storage, comp, 1.0, dt, 0, 8)
    else:
        nx, ny, nz = 17, 12, 21
        rho, lam, mu, cp = smooth_medium3d(nx, ny, nz, 909)
        dt = 0.4 * hw.cfl_bound(physics, 2) / cp
        f = elastic_fields(nx, ny, nz, 910)
        mat = [rho, lam, mu]
        pb = hw.Problem(physics, nx, ny, nz, 2, storage, comp, 1.0, dt, 0, 8)
    out, e = hw.simulate(pb, mat, f, 23, energy_every=11)
    if physics == "acoustic2d":
        w, _, we = oracle_acoustic(nx, ny, 4, storage, comp, dt, rho, kappa, f, 23,
                                   energy_every=11)[:3]
    else:
        from helpers import oracle_elastic
        w, _, we = oracle_elastic(nx, ny, nz, storage, comp, dt, rho, lam, mu, f, 23,
                                  energy_every=11)[:3]
    assert_bitexact(out, w, "simulate")
    np.testing.assert_allclose(e, we, rtol=1e-12, atol=0)


def test_validation_errors_on_device_plan():
    nx = ny = 16
    rho = np.ones((ny, nx))
    pb = hw.Problem("acoustic2d", nx, ny, 1, 2, "f16", "none", 1.0, 0.8, 0, 4)
    plan = hw.Plan(pb)
    with pytest.raises(hw.HalfwaveError) as ei:
        plan.set_material([rho, rho])           # CFL 0.8 > 1/sqrt(2)
    assert ei.value.name == "HW_E_UNSTABLE"
    with pytest.raises(hw.HalfwaveError) as ei:
        plan.advance(1)
    assert ei.value.name == "HW_E_STATE"
    plan.close()
