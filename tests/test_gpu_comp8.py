"""GPU parity of the compensated update with 8-bit compensation words
(HW_COMP_TWOSUM8) against the oracle's mode: fields and compensation terms
(read back as q * ulp(s) / 2^7) bit-identical, over formats, orders, tile
shapes, grid sizes, with a point source and the stencil variants, in
batches, and across checkpoint/resume."""
import numpy as np
import pytest

import oracle
import paper_2310_00236_amd as hw
import workloads
from helpers import acoustic_fields, assert_bitexact, layered_material

pytestmark = pytest.mark.gpu


def _case(nx, ny, order, storage, seed):
    rho, kappa, c = layered_material(nx, ny, seed)
    dt = 0.4 * hw.cfl_bound("acoustic2d", order) / c
    f = acoustic_fields(nx, ny, seed + 1, storage, vel=0.02)
    return rho, kappa, dt, f


def _oracle(nx, ny, order, storage, dt, rho, kappa, f, nsteps, **kw):
    fr = {k: oracle.round_to(v, storage) for k, v in f.items()}
    return oracle.acoustic2d(nx, ny, order, 1.0, dt, rho, kappa, fr, storage=storage,
                             stencil=kw.pop("stencil", "f32"), comp="twosum8",
                             nsteps=nsteps, **kw)


def _plan(nx, ny, order, storage, dt, rho, kappa, f, tile=0, **kw):
    pb = hw.Problem("acoustic2d", nx, ny, 1, order, storage, "twosum8", 1.0, dt, 0,
                    kw.pop("trace_cap", 0), **kw)
    p = hw.Plan(pb)
    p.set_tile(tile)
    p.set_material([rho, kappa])
    p.set_fields(f)
    return p


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("order", [2, 4])
def test_bitexact(storage, order):
    nx, ny = 150, 37
    rho, kappa, dt, f = _case(nx, ny, order, storage, 801)
    p = _plan(nx, ny, order, storage, dt, rho, kappa, f, trace_cap=8)
    p.advance(45, 15)
    g, gc = p.get_fields(comps=True)
    ge, _ = p.energy_trace()
    p.close()
    w, wc, we = _oracle(nx, ny, order, storage, dt, rho, kappa, f, 45, energy_every=15)
    assert_bitexact(g, w, "fields")
    assert_bitexact(gc, wc, "comps")
    np.testing.assert_allclose(ge, we, rtol=1e-12, atol=0)
    assert any(np.any(wc[k] != 0) for k in wc)          # the words are in use


TILE_KINDS = [t for t, s in enumerate(hw.tiles("acoustic2d")) if s[3] != 1]
MARCH_KINDS = [t for t, s in enumerate(hw.tiles("acoustic2d")) if s[3] == 1]


def test_march_shapes_are_refused():
    """8-bit words run on the tile kernels (one and two steps per launch),
    not on the marching kind: a marching shape is refused by
    hw_plan_set_tile, and a batch given one runs the group on shape 0."""
    nx, ny = 65, 17
    rho, kappa, dt, f = _case(nx, ny, 4, "f16", 811)
    pb = hw.Problem("acoustic2d", nx, ny, 1, 4, "f16", "twosum8", 1.0, dt, 0, 0)
    p = hw.Plan(pb)
    for t in MARCH_KINDS:
        with pytest.raises(hw.HalfwaveError) as e:
            p.set_tile(t)
        assert e.value.name == "HW_E_INVAL"
    p.set_material([rho, kappa])
    p.set_fields(f)
    hw.batch_advance([p], [40], tile=MARCH_KINDS[-1])
    g, gc = p.get_fields(comps=True)
    p.close()
    w, wc, _ = _oracle(nx, ny, 4, "f16", dt, rho, kappa, f, 40)
    assert_bitexact(g, w, "batch with a march shape")
    assert_bitexact(gc, wc, "batch with a march shape, comps")


@pytest.mark.parametrize("shape", [(1, 1), (5, 7), (65, 17), (257, 3), (3, 130)])
@pytest.mark.parametrize("tile", TILE_KINDS)
def test_sizes_and_tiles(shape, tile):
    """Every tile shape the 8-bit words run on."""
    nx, ny = shape
    rho, kappa, dt, f = _case(nx, ny, 4, "f16", 811)
    p = _plan(nx, ny, 4, "f16", dt, rho, kappa, f, tile=tile)
    p.advance(40)                                        # graph-captured run
    g, gc = p.get_fields(comps=True)
    p.close()
    w, wc, _ = _oracle(nx, ny, 4, "f16", dt, rho, kappa, f, 40)
    assert_bitexact(g, w, f"{shape} tile {tile}")
    assert_bitexact(gc, wc, f"{shape} tile {tile} comps")


@pytest.mark.parametrize("storage,scale", [("f16", 1100.0), ("bf16", 2.0 ** 116)])
@pytest.mark.parametrize("tile", [0] + [t for t in TILE_KINDS if hw.tiles("acoustic2d")[t][2] == 2])
def test_overflow_matches_oracle(storage, scale, tile):
    """Two steps from pressures large enough that, in a soft medium, many
    sums round past the largest finite value to infinity and infinities of
    opposite sign make NaNs; the 8-bit word of a cell whose sum is not finite
    is 0.
    The GPU has the oracle's infinities, NaN cells, finite values and
    compensation terms bit for bit (only a NaN's sign and payload are left
    open), on the one-step shape and every two-step shape."""
    nx, ny = 70, 40
    rng = np.random.default_rng(112)
    # a soft medium (c = 0.01) at its stable time step: the velocity
    # increments are about 30 times the pressure differences
    rho, kappa = np.ones((ny, nx)), np.full((ny, nx), 1e-4)
    dt = 0.4 * hw.cfl_bound("acoustic2d", 4) / 1e-2
    f = {"p": scale * rng.uniform(-1.0, 1.0, (ny, nx)),
         "vx": np.zeros((ny, nx)), "vy": np.zeros((ny, nx))}
    p = _plan(nx, ny, 4, storage, dt, rho, kappa, f, tile=tile)
    p.advance(2)
    g, gc = p.get_fields(comps=True)
    p.close()
    w, wc, _ = _oracle(nx, ny, 4, storage, dt, rho, kappa, f, 2)[:3]
    for got, want in ((g, w), (gc, wc)):
        for k in want:
            gn, wn = np.isnan(got[k]), np.isnan(want[k])
            assert np.array_equal(gn, wn), k
            assert np.array_equal(got[k][~gn], want[k][~wn]), k
            assert np.array_equal(np.signbit(got[k][~gn]), np.signbit(want[k][~wn])), k
    for k in g:                                          # every case occurs
        assert np.isinf(g[k]).any() and np.isfinite(g[k]).any(), k
        assert np.any(gc[k][np.isfinite(g[k])] != 0), k
    assert np.isnan(g["p"]).any()


@pytest.mark.parametrize("stencil", ["f32", "storage", "f64"])
def test_with_source_receivers_and_stencils(stencil):
    nx, ny = 150, 37
    rho, kappa, dt, f = _case(nx, ny, 4, "f16", 821)
    t = (np.arange(20) + 0.5) * dt - 0.8
    samples = oracle.round_to(0.8 * workloads.ricker(t, 1.5), "f32")
    recs = [(0, 0), (64, 16), (77, 16)]
    p = _plan(nx, ny, 4, "f16", dt, rho, kappa, f, src_cap=20, rec_cap=3, rec_steps=30,
              stencil=stencil)
    p.set_source(77, 16, samples)
    p.set_receivers(recs)
    p.advance(30)
    g, gc = p.get_fields(comps=True)
    gt = p.receiver_trace()
    p.close()
    w, wc, _, wt = _oracle(nx, ny, 4, "f16", dt, rho, kappa, f, 30,
                           stencil="f16" if stencil == "storage" else stencil,
                           source=(77, 16, samples), receivers=recs)
    assert_bitexact(g, w, stencil)
    assert_bitexact(gc, wc, stencil + " comps")
    assert np.array_equal(gt, wt)


def test_batch_and_checkpoint():
    """8-bit-word plans batched with 16-bit-word plans end as when run
    alone; a checkpoint taken mid-run resumes bit-exactly (the blob holds
    the compensation bytes)."""
    nx, ny = 130, 41
    rho, kappa, dt, f = _case(nx, ny, 4, "f16", 831)
    a = _plan(nx, ny, 4, "f16", dt, rho, kappa, f)
    pb16 = hw.Problem("acoustic2d", nx, ny, 1, 4, "f16", "twosum", 1.0, dt, 0, 0)
    b = hw.Plan(pb16)
    b.set_material([rho, kappa])
    b.set_fields(f)
    c = _plan(nx, ny, 4, "f16", dt, rho, kappa, f)
    hw.batch_advance([a, b, c], [37, 37, 20])
    blob = c.export_state()
    d = _plan(nx, ny, 4, "f16", dt, rho, kappa, f)
    d.import_state(blob)
    d.advance(17)
    w, wc, _ = _oracle(nx, ny, 4, "f16", dt, rho, kappa, f, 37)
    for p in (a, d):
        g, gc = p.get_fields(comps=True)
        assert_bitexact(g, w, "fields")
        assert_bitexact(gc, wc, "comps")
    fr = {k: oracle.round_to(v, "f16") for k, v in f.items()}
    w16, _, _ = oracle.acoustic2d(nx, ny, 4, 1.0, dt, rho, kappa, fr, storage="f16",
                                  stencil="f32", comp="twosum", nsteps=37)
    assert_bitexact(b.get_fields(), w16, "16-bit words")
    for p in (a, b, c, d):
        p.close()
