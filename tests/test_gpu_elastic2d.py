"""GPU parity of the 2D elastic system of App. A (Eq. A1: periodic in x,
free surfaces on rows 0 and ny-1, a point source on vy, receivers) through
the C ABI against the oracle: fields, compensation terms and receiver
traces bit-identical for every storage format and update, graph replays,
batched launches (mixed with acoustic plans) and checkpoint/resume; the
energy to 1e-12; the full-size App. A workload checked on sampled cells."""
import numpy as np
import pytest

import oracle
import paper_2310_00236_amd as hw
import workloads
from helpers import assert_bitexact

pytestmark = pytest.mark.gpu

F = oracle.ELASTIC2D_FIELDS
NX, NY = 150, 37          # ragged in both tile directions (64 x 4 tiles)
SRC = (77, 16)
RECS = [(0, 0), (149, 36), (63, 1), (64, 35), (77, 16)]   # surfaces, tile edges


def _medium(seed):
    rho, lam, mu = workloads.layered_elastic2d(NX, NY, seed, swing=0.2)
    cp = np.sqrt((lam + 2 * mu) / rho).max()
    return rho, lam, mu, cp


def _fields(seed, storage, scale=0.05):
    rng = np.random.default_rng(seed)
    f = {k: oracle.round_to(scale * rng.normal(size=(NY, NX)), storage) for k in F}
    f["syy"][0] = 0.0
    f["syy"][-1] = 0.0
    f["vy"][-1] = 0.0
    f["sxy"][-1] = 0.0
    return f


def _samples(n, dt, f0=1.5):
    return 0.8 * workloads.ricker(np.arange(n) * dt - 1.2 / f0, f0)


def _problem(storage, comp, dt, nsrc=0, nrec=0, rec_steps=0, trace_cap=0):
    return hw.Problem("elastic2d", NX, NY, 1, 2, storage, comp, 1.0, dt, 0,
                      trace_cap, src_cap=nsrc, rec_cap=nrec, rec_steps=rec_steps)


def _gpu(storage, comp, rho, lam, mu, dt, f, nsteps, samples=None, recs=None,
         energy_every=0, tile=0):
    ntrace = (nsteps // energy_every + 2) if energy_every else 0
    nsrc = 0 if samples is None else len(samples)
    nrec = 0 if recs is None else len(recs)
    plan = hw.Plan(_problem(storage, comp, dt, nsrc, nrec, nsteps, ntrace))
    plan.set_tile(tile)
    plan.set_material([rho, lam, mu])
    plan.set_fields(f)
    if samples is not None:
        plan.set_source(SRC[0], SRC[1], samples)
    if recs is not None:
        plan.set_receivers(recs)
    plan.advance(nsteps, energy_every)
    out, comps = plan.get_fields(comps=True)
    trace = plan.receiver_trace() if recs is not None else None
    energy = plan.energy_trace()[0] if energy_every else None
    plan.close()
    return out, comps, trace, energy


def _oracle(storage, comp, rho, lam, mu, dt, f, nsteps, samples=None, recs=None,
            energy_every=0):
    return oracle.elastic2d(NX, NY, 1.0, dt, rho, lam, mu, f, storage=storage,
                            stencil="f32", comp=comp, nsteps=nsteps,
                            energy_every=energy_every,
                            source=None if samples is None else (SRC[0], SRC[1], samples),
                            receivers=recs)


@pytest.mark.parametrize("tile", [0, 1])
@pytest.mark.parametrize("storage,comp", [
    ("f32", "none"), ("f16", "none"), ("f16", "twosum"), ("f16", "fast2sum"),
    ("bf16", "none"), ("bf16", "twosum"), ("f32", "twosum")])
def test_bitexact_with_source_and_receivers(storage, comp, tile):
    """45 steps in chunks of 15 between energy logs, the source active for
    the first 30; both kernel shapes (tile 0: one fused pass, tile 1: two
    passes)."""
    rho, lam, mu, cp = _medium(701)
    dt = 0.5 / cp
    f = _fields(702, storage)
    samples = _samples(30, dt)
    g, gc, gt, ge = _gpu(storage, comp, rho, lam, mu, dt, f, 45, samples, RECS, 15,
                         tile)
    w, wc, we, wt = _oracle(storage, comp, rho, lam, mu, dt, f, 45, samples, RECS, 15)
    assert_bitexact(g, w, "fields")
    if comp != "none":
        assert_bitexact(gc, wc, "comps")
    assert gt.shape == wt.shape == (45, len(RECS), 5)
    assert np.array_equal(gt, wt), np.argwhere(gt != wt)[:5]
    np.testing.assert_allclose(ge, we, rtol=1e-12, atol=0)
    # the free surfaces: syy stays zero, the rows outside the body too
    assert not g["syy"][0].any() and not g["syy"][-1].any()
    assert not g["vy"][-1].any() and not g["sxy"][-1].any()


def test_graph_replays_without_forcing():
    """100 steps of an unforced plan: captured 32-step graphs plus direct
    launches, eager work between the replays."""
    rho, lam, mu, cp = _medium(711)
    dt = 0.6 / cp
    f = _fields(712, "f16")
    plan = hw.Plan(_problem("f16", "twosum", dt))
    plan.set_material([rho, lam, mu])
    plan.set_fields(f)
    plan.advance(50)
    mid = plan.get_fields()
    plan.advance(50)
    got, gc = plan.get_fields(comps=True)
    plan.close()
    w, wc, _ = _oracle("f16", "twosum", rho, lam, mu, dt, f, 100)
    assert_bitexact(got, w, "fields")
    assert_bitexact(gc, wc, "comps")
    w50, _, _ = _oracle("f16", "twosum", rho, lam, mu, dt, f, 50)
    assert_bitexact(mid, w50, "after 50")


def test_batch_mixed_with_acoustic_plans():
    """A batch of a forced elastic2d plan, an unforced one and an acoustic
    plan, with uneven step counts (graph-captured runs): each ends as its
    own oracle run says."""
    rho, lam, mu, cp = _medium(721)
    dt = 0.5 / cp
    f = _fields(722, "f16")
    samples = _samples(25, dt)
    a = hw.Plan(_problem("f16", "twosum", dt, len(samples), len(RECS), 90))
    a.set_material([rho, lam, mu])
    a.set_fields(f)
    a.set_source(SRC[0], SRC[1], samples)
    a.set_receivers(RECS)
    b = hw.Plan(_problem("f16", "twosum", dt))
    b.set_material([rho, lam, mu])
    b.set_fields(f)
    kappa = rho * (lam + 2 * mu) / rho
    pa = hw.Problem("acoustic2d", NX, NY, 1, 4, "f16", "twosum", 1.0, 0.3 / cp, 0, 0)
    c = hw.Plan(pa)
    c.set_material([rho, kappa])
    c.set_fields({"p": oracle.round_to(f["sxx"], "f16")})
    hw.batch_advance([a, b, c], [90, 70, 80])
    w, wc, _, wt = _oracle("f16", "twosum", rho, lam, mu, dt, f, 90, samples, RECS)
    got, gc = a.get_fields(comps=True)
    assert_bitexact(got, w, "forced")
    assert_bitexact(gc, wc, "forced comps")
    assert np.array_equal(a.receiver_trace(), wt)
    w, wc, _ = _oracle("f16", "twosum", rho, lam, mu, dt, f, 70)
    got, gc = b.get_fields(comps=True)
    assert_bitexact(got, w, "unforced")
    assert_bitexact(gc, wc, "unforced comps")
    z = np.zeros((NY, NX))
    wa, _, _ = oracle.acoustic2d(NX, NY, 4, 1.0, 0.3 / cp, rho, kappa,
                                 {"vx": z, "vy": z, "p": oracle.round_to(f["sxx"], "f16")},
                                 storage="f16", stencil="f32", comp="twosum", nsteps=80)
    assert_bitexact(c.get_fields(), wa, "acoustic")
    for p in (a, b, c):
        p.close()


def test_checkpoint_resume_keeps_the_source_clock():
    rho, lam, mu, cp = _medium(731)
    dt = 0.5 / cp
    f = _fields(732, "bf16")
    samples = _samples(40, dt)

    def plan():
        p = hw.Plan(_problem("bf16", "twosum", dt, 40, len(RECS), 50))
        p.set_material([rho, lam, mu])
        p.set_source(SRC[0], SRC[1], samples)
        p.set_receivers(RECS)
        return p

    a = plan()
    a.set_fields(f)
    a.advance(50)
    b = plan()
    b.set_fields(f)
    b.advance(21)
    blob = b.export_state()
    c = plan()
    c.import_state(blob)
    c.advance(29)
    assert c.step == 50
    fa, ca = a.get_fields(comps=True)
    fc, cc = c.get_fields(comps=True)
    assert_bitexact(fc, fa, "resumed")
    assert_bitexact(cc, ca, "resumed comps")
    assert np.array_equal(c.receiver_trace()[21:], a.receiver_trace()[21:])
    for p in (a, b, c):
        p.close()


def test_surface_and_source_rules_enforced():
    rho, lam, mu, cp = _medium(741)
    dt = 0.5 / cp
    plan = hw.Plan(_problem("f16", "none", dt, 4, 1, 4))
    plan.set_material([rho, lam, mu])
    f = _fields(742, "f16")
    bad = dict(f, syy=f["syy"].copy())
    bad["syy"][0, 5] = 0.25
    with pytest.raises(hw.HalfwaveError) as ei:
        plan.set_fields(bad)
    assert ei.value.name == "HW_E_INVAL"
    bad = dict(f, sxy=f["sxy"].copy())
    bad["sxy"][-1, 0] = 0.25
    with pytest.raises(hw.HalfwaveError):
        plan.set_fields(bad)
    plan.set_fields(f)
    with pytest.raises(hw.HalfwaveError) as ei:
        plan.set_source(3, NY - 1, [1.0])
    assert ei.value.name == "HW_E_INVAL"
    plan.set_source(3, NY - 2, [1.0])
    plan.close()


def _patch_oracle(state, comps, w, k_step, j, i, m, samples):
    """One step of the oracle on the rows max(0, j-m) .. min(ny-1, j+m) and
    the 2m+1 columns around (i, j) (periodic in x); rows that are not real
    surfaces are cut (their values do not reach the centre in one step)."""
    ny, nx = w.ny, w.nx
    lo, hi = max(0, j - m), min(ny - 1, j + m)
    rows = np.arange(lo, hi + 1)
    cols = np.arange(i - m, i + m + 1) % nx
    idx = np.ix_(rows, cols)
    f = {k: state[k][idx].astype(np.float64).copy() for k in F}
    c = {k: comps[k][idx].astype(np.float64).copy() for k in F}
    for d in (f, c):
        d["syy"][0] = 0.0
        d["syy"][-1] = 0.0
        d["vy"][-1] = 0.0
        d["sxy"][-1] = 0.0
    src = None
    sx, sy, smp = w.source
    if lo <= sy <= hi - 1 and (sx - (i - m)) % nx <= 2 * m and k_step < len(smp):
        src = (int((sx - (i - m)) % nx), int(sy - lo), smp[k_step:k_step + 1])
    o, oc, _ = oracle.elastic2d(2 * m + 1, len(rows), w.dx, w.dt, w.rho[idx],
                                w.lam[idx], w.mu[idx], f, storage="f16",
                                stencil="f32", comp="twosum", comps=c, nsteps=1,
                                source=src)
    return o, oc, j - lo


def test_app_a_full_size_sampled():
    """The App. A workload (600 x 600, fp16 + TwoSum, the source firing) in
    the configuration the benchmark runs: after 400 steps one more step is
    checked on sampled cells -- both surfaces, the source cell, random
    cells -- against the oracle on local patches; and the energy of the
    state against the oracle's energy of the same state."""
    w = workloads.paper_elastic2d(nsteps=401)
    pb = hw.Problem("elastic2d", w.nx, w.ny, 1, 2, "f16", "twosum", w.dx, w.dt, 0, 2,
                    src_cap=len(w.source[2]), rec_cap=1, rec_steps=401)
    plan = hw.Plan(pb)
    plan.set_material([w.rho, w.lam, w.mu])
    plan.set_fields(w.fields())
    plan.set_source(*w.source)
    plan.set_receivers(w.receivers)
    plan.advance(400)
    before, cbefore = plan.get_fields(comps=True)
    plan.record_energy()
    plan.advance(1)
    after, cafter = plan.get_fields(comps=True)
    e_gpu = plan.energy_trace()[0][0]
    plan.close()
    e_orc = oracle.elastic2d_energy(w.nx, w.ny, w.dx, w.dt, w.rho, w.lam, w.mu, before)
    assert e_gpu == pytest.approx(e_orc, rel=1e-12)
    assert e_orc > 0
    rng = np.random.default_rng(17)
    sx, sy, _ = w.source
    pts = [(0, 0), (w.ny - 1, 599), (0, 313), (w.ny - 1, 7), (1, 200), (w.ny - 2, 401),
           (sy, sx), (sy + 1, sx), (sy - 1, sx + 1)]
    pts += [tuple(int(v) for v in rng.integers(0, 600, size=2)) for _ in range(30)]
    m = 4
    for (j, i) in pts:
        o, oc, jc = _patch_oracle(before, cbefore, w, 400, j, i, m, w.source[2])
        for k in F:
            assert after[k][j, i] == o[k][jc, m], (k, j, i)
            assert cafter[k][j, i] == oc[k][jc, m], (k, j, i)


@pytest.mark.parametrize("tile", [0, 1])
@pytest.mark.parametrize("nx,ny", [(1, 3), (5, 3), (64, 4), (65, 5), (3, 130), (129, 9)])
def test_degenerate_and_ragged_grids(nx, ny, tile):
    """The smallest body (one interior row), one column (x wraps onto
    itself), exact and ragged tiles, a tall thin strip: bit-exact against
    the oracle with the source and a receiver."""
    rho, lam, mu = workloads.layered_elastic2d(nx, ny, 750 + nx, swing=0.2)
    cp = np.sqrt((lam + 2 * mu) / rho).max()
    dt = 0.5 / cp
    rng = np.random.default_rng(751)
    f = {k: oracle.round_to(0.05 * rng.normal(size=(ny, nx)), "f16") for k in F}
    f["syy"][0] = f["syy"][-1] = 0.0
    f["vy"][-1] = f["sxy"][-1] = 0.0
    src = (nx // 2, ny // 2 - 1 if ny > 3 else 0)
    samples = _samples(12, dt)
    rec = [(nx - 1, ny - 1), (0, 0)]
    pb = hw.Problem("elastic2d", nx, ny, 1, 2, "f16", "twosum", 1.0, dt, 0, 0,
                    src_cap=12, rec_cap=2, rec_steps=20)
    plan = hw.Plan(pb)
    plan.set_tile(tile)
    plan.set_material([rho, lam, mu])
    plan.set_fields(f)
    plan.set_source(src[0], src[1], samples)
    plan.set_receivers(rec)
    plan.advance(20)
    got, gc = plan.get_fields(comps=True)
    tr = plan.receiver_trace()
    plan.close()
    w, wc, _, wt = oracle.elastic2d(nx, ny, 1.0, dt, rho, lam, mu, f, storage="f16",
                                    stencil="f32", comp="twosum", nsteps=20,
                                    source=(src[0], src[1], samples), receivers=rec)
    assert_bitexact(got, w, f"{nx}x{ny}")
    assert_bitexact(gc, wc, f"{nx}x{ny} comps")
    assert np.array_equal(tr, wt)


def test_power_of_two_field_scale_is_exact():
    """Fields held times 2^4 (the range scaling of Sec. 5): the unscaled
    results, receiver records included, equal the unscaled run bit for bit
    (source samples are given already scaled).  bf16, whose exponent range
    keeps every value of this run normal (in fp16 the compensation terms are
    often subnormal, where a power-of-two scale changes the rounding)."""
    rho, lam, mu, cp = _medium(761)
    dt = 0.5 / cp
    f = _fields(762, "bf16", scale=0.5)
    samples = _samples(20, dt)
    out = []
    for k in (0, 4):
        pb = hw.Problem("elastic2d", NX, NY, 1, 2, "bf16", "twosum", 1.0, dt, k, 0,
                        src_cap=20, rec_cap=len(RECS), rec_steps=30)
        plan = hw.Plan(pb)
        plan.set_material([rho, lam, mu])
        plan.set_fields(f)
        plan.set_source(SRC[0], SRC[1], samples * 2.0 ** k)
        plan.set_receivers(RECS)
        plan.advance(30)
        out.append((plan.get_fields(comps=True), plan.receiver_trace()))
        plan.close()
    (a, ca), ta = out[0]
    (b, cb), tb = out[1]
    assert_bitexact(b, a, "scaled")
    assert_bitexact(cb, ca, "scaled comps")
    assert np.array_equal(tb, ta)


def test_batch_beyond_the_launch_limit():
    """70 small elastic plans of uneven size and step count in one batch (one
    launch pair per plan, counters ticked in groups of 64): each equals its
    solo run."""
    plans, steps, made = [], [], []
    for i in range(70):
        nx, ny = 20 + i % 9, 3 + i % 6
        rho, lam, mu = workloads.layered_elastic2d(nx, ny, 800 + i, swing=0.2)
        dt = 0.5 / np.sqrt((lam + 2 * mu) / rho).max()
        rng = np.random.default_rng(900 + i)
        f = {k: oracle.round_to(0.05 * rng.normal(size=(ny, nx)), "f16") for k in F}
        f["syy"][0] = f["syy"][-1] = 0.0
        f["vy"][-1] = f["sxy"][-1] = 0.0
        pb = hw.Problem("elastic2d", nx, ny, 1, 2, "f16", "twosum", 1.0, dt, 0, 0,
                        src_cap=5, rec_cap=1, rec_steps=12)
        p = hw.Plan(pb)
        p.set_material([rho, lam, mu])
        p.set_fields(f)
        if i % 2:
            p.set_source(0, 0, [0.25, -0.5, 0.125, 0.0, 1.0])
            p.set_receivers([(nx - 1, ny - 1)])
        plans.append(p)
        steps.append(3 + i % 9)
        made.append((pb, [rho, lam, mu], f, i % 2))
    hw.batch_advance(plans, steps)
    for p, n, (pb, mat, f, forced) in zip(plans, steps, made):
        q = hw.Plan(pb)
        q.set_material(mat)
        q.set_fields(f)
        if forced:
            q.set_source(0, 0, [0.25, -0.5, 0.125, 0.0, 1.0])
            q.set_receivers([(pb.nx - 1, pb.ny - 1)])
        q.advance(n)
        assert_bitexact(p.get_fields(), q.get_fields(), "batched")
        if forced:
            assert np.array_equal(p.receiver_trace(), q.receiver_trace())
        q.close()
    for p in plans:
        p.close()
