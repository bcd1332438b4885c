"""The two-steps-per-launch 2D acoustic kernels (tile kinds 4 and 5,
temporal blocking) against the oracle: bit-identical fields, compensation
terms and energies for every storage format, update and order, on ragged
grids, with odd step counts (a one-step launch finishes them), odd energy
intervals, captured graphs started from either field set, and batches of
plans of uneven size and step count."""
import numpy as np
import pytest

import paper_2310_00236_amd as hw
from helpers import (ST, acoustic_fields, assert_bitexact, gpu_acoustic,
                     layered_material, oracle_acoustic)

pytestmark = pytest.mark.gpu

TWO = [t for t, s in enumerate(hw.tiles("acoustic2d")) if s[3] in (4, 5)]


def _case(nx, ny, order, storage, seed):
    rho, kappa, c = layered_material(nx, ny, seed)
    dt = 0.45 * hw.cfl_bound("acoustic2d", order) / c
    return rho, kappa, dt, acoustic_fields(nx, ny, seed + 1, storage)


@pytest.mark.parametrize("tile", TWO)
@pytest.mark.parametrize("storage", ST)
@pytest.mark.parametrize("comp", ["none", "fast2sum", "twosum"])
@pytest.mark.parametrize("order", [2, 4])
def test_bitexact(tile, storage, comp, order):
    nx, ny = 150, 37
    rho, kappa, dt, f = _case(nx, ny, order, storage, 301)
    g, gc, ge = gpu_acoustic(nx, ny, order, storage, comp, dt, rho, kappa, f, 25,
                             energy_every=5, tile=tile)
    w, wc, we = oracle_acoustic(nx, ny, order, storage, comp, dt, rho, kappa, f, 25,
                                energy_every=5)
    assert_bitexact(g, w, "fields")
    if comp != "none":
        assert_bitexact(gc, wc, "comps")
    np.testing.assert_allclose(ge, we, rtol=1e-12, atol=0)


@pytest.mark.parametrize("tile", TWO)
@pytest.mark.parametrize("shape", [(200, 75), (64, 32), (130, 100), (13, 260)])
def test_graphs_from_either_field_set(tile, shape):
    """One step, then 101 (graph-captured runs of 32 steps = 16 two-step
    launches, from field set 1 after an aligning single step), then 66."""
    nx, ny = shape
    rho, kappa, dt, f = _case(nx, ny, 4, "f16", 311)
    pb = hw.Problem("acoustic2d", nx, ny, 1, 4, "f16", "twosum", 1.0, dt, 0, 0)
    p = hw.Plan(pb)
    p.set_tile(tile)
    p.set_material([rho, kappa])
    p.set_fields(f)
    for n in (1, 101, 66):
        p.advance(n)
    assert p.step == 168
    g, gc = p.get_fields(comps=True)
    p.close()
    w, wc, _ = oracle_acoustic(nx, ny, 4, "f16", "twosum", dt, rho, kappa, f, 168)
    assert_bitexact(g, w, f"{shape}")
    assert_bitexact(gc, wc, f"{shape} comps")


@pytest.mark.parametrize("tile", TWO)
def test_batch_of_uneven_plans(tile):
    """Plans of different sizes and odd and even step counts in one batched
    call on a two-step shape, with energies every 7 steps."""
    sizes = [(150, 37, 41), (64, 64, 70), (97, 130, 9), (300, 20, 66), (5, 9, 33)]
    plans, want = [], []
    for i, (nx, ny, ns) in enumerate(sizes):
        rho, kappa, dt, f = _case(nx, ny, 4, "f16", 320 + i)
        pb = hw.Problem("acoustic2d", nx, ny, 1, 4, "f16", "twosum", 1.0, dt, 0,
                        ns // 7 + 2)
        p = hw.Plan(pb)
        p.set_material([rho, kappa])
        p.set_fields(f)
        plans.append(p)
        want.append(oracle_acoustic(nx, ny, 4, "f16", "twosum", dt, rho, kappa, f, ns,
                                    energy_every=7))
    hw.batch_advance(plans, [s[2] for s in sizes], energy_every=7, tile=tile)
    for p, (w, wc, we), s in zip(plans, want, sizes):
        g, gc = p.get_fields(comps=True)
        e, _ = p.energy_trace()
        assert p.step == s[2]
        assert_bitexact(g, w, f"{s}")
        assert_bitexact(gc, wc, f"{s} comps")
        np.testing.assert_allclose(e, we, rtol=1e-12, atol=0)
        p.close()


def test_forced_plan_on_a_two_step_shape_runs_one_step_shapes():
    """A plan with a point source and receivers given a two-step shape
    steps on shape 0 (its source clock needs every step): bit-identical to
    the oracle's forced run."""
    import oracle
    nx, ny, ns = 70, 40, 19
    rho, kappa, dt, f = _case(nx, ny, 4, "f16", 330)
    samples = np.sin(np.arange(ns) * 0.3)
    pb = hw.Problem("acoustic2d", nx, ny, 1, 4, "f16", "twosum", 1.0, dt, 0, 0,
                    src_cap=ns, rec_cap=2, rec_steps=ns)
    p = hw.Plan(pb)
    p.set_tile(TWO[0])
    p.set_material([rho, kappa])
    p.set_fields(f)
    p.set_source(10, 12, samples)
    p.set_receivers([(3, 4), (69, 39)])
    p.advance(ns)
    g, gc = p.get_fields(comps=True)
    rec = p.receiver_trace()
    p.close()
    fr = {k: oracle.round_to(v, "f16") for k, v in f.items()}
    w, wc, _, wrec = oracle.acoustic2d(nx, ny, 4, 1.0, dt, rho, kappa, fr, storage="f16",
                                       stencil="f32", comp="twosum", nsteps=ns,
                                       source=(10, 12, samples),
                                       receivers=[(3, 4), (69, 39)])
    assert_bitexact(g, w, "forced")
    assert_bitexact(gc, wc, "forced comps")
    assert np.array_equal(rec, wrec)


@pytest.mark.parametrize("tile", TWO)
@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("order", [2, 4])
def test_bitexact_8bit_words(tile, storage, order):
    """8-bit compensation words on the two-step shapes: the value and the
    byte of every cell of the intermediate state stay in registers; fields,
    read-back compensation terms and energies as the oracle's."""
    nx, ny = 150, 37
    rho, kappa, dt, f = _case(nx, ny, order, storage, 341)
    g, gc, ge = gpu_acoustic(nx, ny, order, storage, "twosum8", dt, rho, kappa, f, 25,
                             energy_every=5, tile=tile)
    w, wc, we = oracle_acoustic(nx, ny, order, storage, "twosum8", dt, rho, kappa, f, 25,
                                energy_every=5)
    assert_bitexact(g, w, "fields")
    assert_bitexact(gc, wc, "comps")
    assert any(np.any(wc[k] != 0) for k in wc)
    np.testing.assert_allclose(ge, we, rtol=1e-12, atol=0)
