"""GPU parity of the point source and receivers (Sec. 3: the s_p term of
Eq. 1 with a Ricker time profile, receiver time histories) through the C ABI
against the oracle: fields, compensation terms and receiver traces
bit-identical, for every storage format and update, every tile shape, graph
replays, batched launches and checkpoint/resume."""
import numpy as np
import pytest

import oracle
import paper_2310_00236_amd as hw
import workloads
from helpers import acoustic_fields, assert_bitexact, layered_material

pytestmark = pytest.mark.gpu

NX, NY = 150, 37          # several tiles, ragged in x and y
SRC = (77, 16)            # a cell in an interior tile
RECS = [(0, 0), (63, 15), (64, 16), (149, 36), SRC]   # tile corners, edges, source


def _samples(n, dt, f0=1.5):
    t = (np.arange(n) + 0.5) * dt - 1.2 / f0
    return 0.8 * workloads.ricker(t, f0)


def _setup(order, storage, seed=601):
    rho, kappa, c = layered_material(NX, NY, seed)
    dt = 0.4 * hw.cfl_bound("acoustic2d", order) / c
    f = acoustic_fields(NX, NY, seed + 1, storage, vel=0.02)
    return rho, kappa, dt, f


def _gpu(order, storage, comp, rho, kappa, dt, f, nsteps, samples, recs, tile=0,
         energy_every=0, src=SRC):
    ntrace = (nsteps // energy_every + 2) if energy_every else 0
    pb = hw.Problem("acoustic2d", NX, NY, 1, order, storage, comp, 1.0, dt, 0,
                    ntrace, src_cap=len(samples), rec_cap=len(recs),
                    rec_steps=nsteps)
    plan = hw.Plan(pb)
    plan.set_tile(tile)
    plan.set_material([rho, kappa])
    plan.set_fields(f)
    plan.set_source(src[0], src[1], samples)
    plan.set_receivers(recs)
    plan.advance(nsteps, energy_every)
    out, comps = plan.get_fields(comps=True)
    trace = plan.receiver_trace()
    energy = plan.energy_trace()[0] if energy_every else None
    plan.close()
    return out, comps, trace, energy


def _oracle(order, storage, comp, rho, kappa, dt, f, nsteps, samples, recs,
            energy_every=0, src=SRC):
    fr = {k: oracle.round_to(v, storage) for k, v in f.items()}
    return oracle.acoustic2d(NX, NY, order, 1.0, dt, rho, kappa, fr,
                             storage=storage, stencil="f32", comp=comp,
                             nsteps=nsteps, energy_every=energy_every,
                             source=(src[0], src[1], samples), receivers=recs)


def _shape_index(shape):
    return next(i for i, t in enumerate(hw.tiles("acoustic2d")) if tuple(t) == shape)


# tile shapes that advance two steps per launch
TWO_STEP = [i for i, t in enumerate(hw.tiles("acoustic2d")) if t[2] == 2]


@pytest.mark.parametrize("storage,comp,order", [
    ("f32", "none", 4), ("f16", "none", 4), ("f16", "twosum", 4),
    ("f16", "fast2sum", 2), ("bf16", "none", 4), ("bf16", "twosum", 2)])
def test_bitexact_source_and_receivers(storage, comp, order):
    """45 steps in chunks of 15 between energy logs, the source active for
    the first 30."""
    rho, kappa, dt, f = _setup(order, storage)
    samples = _samples(30, dt)
    g, gc, gt, ge = _gpu(order, storage, comp, rho, kappa, dt, f, 45, samples,
                         RECS, energy_every=15)
    w, wc, we, wt = _oracle(order, storage, comp, rho, kappa, dt, f, 45, samples,
                            RECS, energy_every=15)
    assert_bitexact(g, w, "fields")
    if comp != "none":
        assert_bitexact(gc, wc, "comps")
    assert gt.shape == wt.shape == (45, len(RECS), 3)
    assert np.array_equal(gt, wt), np.argwhere(gt != wt)[:5]
    np.testing.assert_allclose(ge, we, rtol=1e-12, atol=0)


@pytest.mark.parametrize("tile", range(len(hw.tiles("acoustic2d"))))
def test_every_tile_shape(tile):
    """Any tile setting: forced plans step with kernel shape 0, or on their
    two-step shape."""
    rho, kappa, dt, f = _setup(4, "f16", 611)
    samples = _samples(20, dt)
    g, gc, gt, _ = _gpu(4, "f16", "twosum", rho, kappa, dt, f, 24, samples, RECS,
                        tile=tile)
    w, wc, _, wt = _oracle(4, "f16", "twosum", rho, kappa, dt, f, 24, samples, RECS)
    assert_bitexact(g, w, f"tile {tile}")
    assert_bitexact(gc, wc, f"tile {tile} comps")
    assert np.array_equal(gt, wt)


@pytest.mark.parametrize("storage,comp,order", [
    ("f32", "none", 4), ("f16", "none", 2), ("f16", "twosum", 4), ("f16", "fast2sum", 4),
    ("bf16", "twosum", 4), ("f16", "twosum8", 4), ("bf16", "twosum8", 2)])
def test_two_step_source_and_receivers(storage, comp, order):
    """Two steps per launch (64 x 24) with the point source and receivers:
    45 steps in chunks of 15 between energy logs (odd chunks end with a
    one-step launch), the source active for the first 30; fields,
    compensation terms, receiver traces and energies as the oracle's."""
    rho, kappa, dt, f = _setup(order, storage, 641)
    samples = _samples(30, dt)
    tile = _shape_index((64, 24, 2, 5))
    g, gc, gt, ge = _gpu(order, storage, comp, rho, kappa, dt, f, 45, samples,
                         RECS, tile=tile, energy_every=15)
    w, wc, we, wt = _oracle(order, storage, comp, rho, kappa, dt, f, 45, samples,
                            RECS, energy_every=15)
    assert_bitexact(g, w, "fields")
    if comp != "none":
        assert_bitexact(gc, wc, "comps")
    assert np.array_equal(gt, wt), np.argwhere(gt != wt)[:5]
    np.testing.assert_allclose(ge, we, rtol=1e-12, atol=0)


@pytest.mark.parametrize("tile", TWO_STEP)
@pytest.mark.parametrize("src", [(63, 23), (64, 24), (66, 15), (0, 36), (149, 0)])
def test_two_step_source_on_tile_edges(tile, src):
    """The source on or next to a tile's edge, where neighbouring workgroups
    recompute its cell's intermediate pressure in their grown regions, and on
    the grid's corners (periodic wrap): 25 steps (the last a one-step
    launch) as the oracle's, receivers around the source included."""
    rho, kappa, dt, f = _setup(4, "f16", 651)
    samples = _samples(21, dt)
    recs = [src, ((src[0] + 1) % NX, src[1]), (src[0], (src[1] + NY - 1) % NY), (0, 0)]
    g, gc, gt, _ = _gpu(4, "f16", "twosum", rho, kappa, dt, f, 25, samples, recs,
                        tile=tile, src=src)
    w, wc, _, wt = _oracle(4, "f16", "twosum", rho, kappa, dt, f, 25, samples, recs,
                           src=src)
    assert_bitexact(g, w, f"tile {tile} source {src}")
    assert_bitexact(gc, wc, f"tile {tile} source {src} comps")
    assert np.array_equal(gt, wt), np.argwhere(gt != wt)[:5]


@pytest.mark.parametrize("tile", [0, _shape_index((64, 24, 2, 5))])
def test_batched_with_and_without_sources(tile):
    """A batch mixing a forced plan, an unforced one and a receivers-only
    one, with uneven step counts, on the one-step shape 0 and on a two-step
    shape: each ends as the oracle says."""
    rho, kappa, dt, f = _setup(4, "f16", 621)
    samples = _samples(25, dt)

    def make(src, recs, nsteps):
        pb = hw.Problem("acoustic2d", NX, NY, 1, 4, "f16", "twosum", 1.0, dt, 0, 0,
                        src_cap=len(samples), rec_cap=len(RECS), rec_steps=60)
        p = hw.Plan(pb)
        p.set_material([rho, kappa])
        p.set_fields(f)
        if src:
            p.set_source(SRC[0], SRC[1], samples)
        if recs:
            p.set_receivers(RECS)
        return p

    specs = [(True, True, 40), (False, False, 35), (False, True, 50)]
    plans = [make(*s) for s in specs]
    hw.batch_advance(plans, [s[2] for s in specs], tile=tile)
    fr = {k: oracle.round_to(v, "f16") for k, v in f.items()}
    for p, (src, recs, n) in zip(plans, specs):
        out = oracle.acoustic2d(NX, NY, 4, 1.0, dt, rho, kappa, fr, storage="f16",
                                stencil="f32", comp="twosum", nsteps=n,
                                source=(SRC[0], SRC[1], samples) if src else None,
                                receivers=RECS if recs else None)
        got, gc = p.get_fields(comps=True)
        assert_bitexact(got, out[0], "fields")
        assert_bitexact(gc, out[1], "comps")
        if recs:
            assert np.array_equal(p.receiver_trace(), out[3])
        p.close()


def test_checkpoint_resume_keeps_the_source_clock():
    """Export after 20 steps, import into a fresh plan with the same source
    and receivers, continue 30 steps: fields and the receiver rows 20..49
    match the uninterrupted run (the source sample index resumes at 20)."""
    rho, kappa, dt, f = _setup(4, "f16", 631)
    samples = _samples(40, dt)

    def plan():
        pb = hw.Problem("acoustic2d", NX, NY, 1, 4, "f16", "twosum", 1.0, dt, 0, 0,
                        src_cap=40, rec_cap=len(RECS), rec_steps=50)
        p = hw.Plan(pb)
        p.set_material([rho, kappa])
        p.set_source(SRC[0], SRC[1], samples)
        p.set_receivers(RECS)
        return p

    a = plan()
    a.set_fields(f)
    a.advance(50)
    b = plan()
    b.set_fields(f)
    b.advance(20)
    blob = b.export_state()
    c = plan()
    c.import_state(blob)
    c.advance(30)
    assert c.step == 50
    fa, ca = a.get_fields(comps=True)
    fc, cc = c.get_fields(comps=True)
    assert_bitexact(fc, fa, "resumed fields")
    assert_bitexact(cc, ca, "resumed comps")
    assert np.array_equal(c.receiver_trace()[20:], a.receiver_trace()[20:])
    for p in (a, b, c):
        p.close()


def test_removing_the_source_and_trace_bounds():
    rho, kappa, dt, f = _setup(4, "f32", 641)
    pb = hw.Problem("acoustic2d", NX, NY, 1, 4, "f32", "none", 1.0, dt, 0, 0,
                    src_cap=10, rec_cap=1, rec_steps=5)
    p = hw.Plan(pb)
    p.set_material([rho, kappa])
    p.set_fields(f)
    p.set_source(SRC[0], SRC[1], np.ones(10))
    p.set_source(0, 0, [])                      # removed again
    p.set_receivers([SRC])
    p.advance(8)                                # more steps than trace rows
    got = p.get_fields()
    fr = {k: oracle.round_to(v, "f32") for k, v in f.items()}
    want, _, _, tr = oracle.acoustic2d(NX, NY, 4, 1.0, dt, rho, kappa, fr,
                                       storage="f32", stencil="f32", nsteps=8,
                                       receivers=[SRC])
    assert_bitexact(got, want, "no source")
    t = p.receiver_trace()
    assert t.shape == (5, 1, 3) and np.array_equal(t, tr[:5])
    p.close()


def test_graph_replays_keep_the_source_clock():
    """80 steps without energy logging run as two captured 32-step graphs
    plus direct launches; the source samples and trace rows must follow the
    device step counter through the replays, with eager work in between."""
    rho, kappa, dt, f = _setup(4, "f16", 651)
    samples = _samples(70, dt)
    pb = hw.Problem("acoustic2d", NX, NY, 1, 4, "f16", "twosum", 1.0, dt, 0, 0,
                    src_cap=70, rec_cap=len(RECS), rec_steps=80)
    p = hw.Plan(pb)
    p.set_material([rho, kappa])
    p.set_fields(f)
    p.set_source(SRC[0], SRC[1], samples)
    p.set_receivers(RECS)
    p.advance(40)
    mid = p.get_fields()                # eager work between the replays
    p.advance(40)
    got, gc = p.get_fields(comps=True)
    trace = p.receiver_trace()
    p.close()
    w, wc, _, wt = _oracle(4, "f16", "twosum", rho, kappa, dt, f, 80, samples, RECS)
    assert_bitexact(got, w, "fields")
    assert_bitexact(gc, wc, "comps")
    assert np.array_equal(trace, wt)
    assert np.array_equal(mid["p"][SRC[1], SRC[0]], wt[39, -1, 0])
