"""Pins of the oracle's point source and receivers (Sec. 3: the s_p term of
Eq. 1, a point source on the pressure with a Ricker time profile, and the
receiver time histories; the source line of Alg. 1 and 2).

The source is checked against the dense-operator model (a unit vector at
the source point added to the divergence), against an initial condition it
must reproduce bit for bit, against the closed-form energy it injects into a
medium at rest, and for linearity; the receivers against the fields
themselves.  The Ricker generator is checked against its closed-form zeros,
peak and zero mean.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import brute
import workloads

F = ("vx", "vy", "p")


def _medium(nx, ny, seed):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(1.0, 2.5, size=(ny, nx))
    kappa = rng.uniform(1.0, 4.0, size=(ny, nx))
    return rho, kappa


def _rest(nx, ny):
    return {k: np.zeros((ny, nx)) for k in F}


@pytest.mark.parametrize("order,nx,ny,src", [(2, 7, 5, (2, 1)), (4, 7, 5, (6, 4)),
                                             (4, 3, 6, (0, 5))])
def test_source_and_receivers_match_dense_operators(order, nx, ny, src):
    """Forced run from a random state: the oracle against dense operators
    with the source as a unit vector times the sample; the receiver trace
    against the dense model's fields after every step."""
    rho, kappa = _medium(nx, ny, 31)
    rng = np.random.default_rng(32)
    f = {k: rng.normal(size=(ny, nx)) for k in F}
    samples = rng.normal(size=4)           # active for 4 of the 6 steps
    recs = [(0, 0), src, (nx - 1, ny - 1)]
    ops = brute.acoustic2d_operators(nx, ny, order, 1.0, 0.2, rho, kappa)
    vx, vy, p = (f[k].ravel() for k in F)
    want = []
    for n in range(6):
        s = (src[1] * nx + src[0], samples[n]) if n < len(samples) else None
        vx, vy, p = brute.acoustic2d_step(ops, vx, vy, p, source=s)
        want.append([(p[y * nx + x], vx[y * nx + x], vy[y * nx + x])
                     for x, y in recs])
    got, _, _, trace = oracle.acoustic2d(nx, ny, order, 1.0, 0.2, rho, kappa,
                                         f, nsteps=6,
                                         source=(src[0], src[1], samples),
                                         receivers=recs)
    for k, ref in (("vx", vx), ("vy", vy), ("p", p)):
        np.testing.assert_allclose(got[k].ravel(), ref, rtol=0, atol=1e-13)
    np.testing.assert_allclose(trace, np.array(want), rtol=0, atol=1e-13)


@pytest.mark.parametrize("storage,comp", [("f64", "none"), ("f32", "none"),
                                          ("f16", "none"), ("f16", "twosum"),
                                          ("bf16", "fast2sum")])
def test_single_impulse_is_an_initial_condition(storage, comp):
    """From rest, a source active in step 0 only leaves p^1 = RN(kappa s) at
    the source cell and v^{1/2} = 0; the remaining steps are then exactly the
    unforced run from that state (every format, every update)."""
    nx, ny, order = 23, 19, 4
    rho, kappa = _medium(nx, ny, 33)
    s = 0.731
    stencil = "f64" if storage == "f64" else "f32"
    kw = dict(storage=storage, stencil=stencil, comp=comp)
    forced, cf, _ = oracle.acoustic2d(nx, ny, order, 1.0, 0.1, rho, kappa,
                                      _rest(nx, ny), nsteps=9,
                                      source=(5, 7, [s]), **kw)
    start = _rest(nx, ny)
    r = lambda x, fmt: float(np.asarray(oracle.round_to(x, fmt)).ravel()[0])
    k32 = r(kappa[7, 5], "f32")
    s_r = s if storage == "f64" else r(s, "f32")
    inc = k32 * s_r if storage == "f64" else r(k32 * s_r, "f32")
    start["p"][7, 5] = r(inc, storage)
    free, cfree, _ = oracle.acoustic2d(nx, ny, order, 1.0, 0.1, rho, kappa,
                                       start, nsteps=8, **kw)
    for k in F:
        assert np.array_equal(forced[k], free[k]), k
        if comp != "none":
            assert np.array_equal(cf[k], cfree[k]), k


def test_energy_injected_from_rest():
    """E^1 after one source step from rest is dx^2/2 * kappa * s^2 (the
    velocities at n+1/2 are still zero, so only the pressure term counts)."""
    nx, ny = 16, 12
    rho, kappa = _medium(nx, ny, 34)
    dx, s = 0.5, 1.25
    _, _, E = oracle.acoustic2d(nx, ny, 4, dx, 0.05, rho, kappa, _rest(nx, ny),
                                nsteps=1, energy_every=1, source=(3, 9, [s]))
    k = float(np.asarray(oracle.round_to(kappa[9, 3], "f32")).ravel()[0])
    assert E[0] == 0.0
    assert E[1] == pytest.approx(dx * dx / 2 * k * s * s, rel=1e-14)


def test_response_is_linear_in_the_source():
    """In fp64 from rest, doubling every sample doubles every field value
    exactly (all operations are linear; scaling by 2 is exact)."""
    nx, ny = 20, 14
    rho, kappa = _medium(nx, ny, 35)
    rng = np.random.default_rng(36)
    samples = rng.normal(size=12)
    a, _, _ = oracle.acoustic2d(nx, ny, 4, 1.0, 0.1, rho, kappa, _rest(nx, ny),
                                nsteps=15, source=(4, 4, samples))
    b, _, _ = oracle.acoustic2d(nx, ny, 4, 1.0, 0.1, rho, kappa, _rest(nx, ny),
                                nsteps=15, source=(4, 4, 2.0 * samples))
    for k in F:
        assert np.array_equal(2.0 * a[k], b[k]), k


def test_receiver_rows_are_the_fields_after_each_step():
    nx, ny = 11, 9
    rho, kappa = _medium(nx, ny, 37)
    rng = np.random.default_rng(38)
    f = {k: rng.normal(size=(ny, nx)) for k in F}
    recs = [(3, 4), (10, 8), (0, 0)]
    _, _, _, trace = oracle.acoustic2d(nx, ny, 2, 1.0, 0.2, rho, kappa, f,
                                       nsteps=5, storage="f16", stencil="f32",
                                       comp="twosum", receivers=recs)
    for n in range(5):
        g, _, _ = oracle.acoustic2d(nx, ny, 2, 1.0, 0.2, rho, kappa, f,
                                    nsteps=n + 1, storage="f16",
                                    stencil="f32", comp="twosum")
        for r, (x, y) in enumerate(recs):
            assert tuple(trace[n, r]) == (g["p"][y, x], g["vx"][y, x],
                                          g["vy"][y, x])


def test_bad_source_or_receiver_cells_rejected():
    rho, kappa = _medium(5, 4, 39)
    with pytest.raises(ValueError):
        oracle.acoustic2d(5, 4, 2, 1.0, 0.1, rho, kappa, _rest(5, 4), nsteps=1,
                          source=(5, 0, [1.0]))
    with pytest.raises(ValueError):
        oracle.acoustic2d(5, 4, 2, 1.0, 0.1, rho, kappa, _rest(5, 4), nsteps=1,
                          receivers=[(0, 4)])


def test_ricker_closed_forms():
    f0 = 5.0
    assert workloads.ricker(0.0, f0) == 1.0
    tz = 1.0 / (math.pi * f0 * math.sqrt(2.0))          # zeros of (1 - 2a)
    np.testing.assert_allclose(workloads.ricker([-tz, tz], f0), 0.0, atol=1e-15)
    t = np.linspace(-2.0, 2.0, 400001)
    r = workloads.ricker(t, f0)
    assert abs(np.trapezoid(r, t)) < 1e-9             # zero mean
    assert r.min() == pytest.approx(-2.0 * math.exp(-1.5), rel=1e-6)


def test_paper_workload_geometry():
    w = workloads.paper2d(ppw=10, nsteps=60000)
    assert (w.nx, w.ny, w.dx, w.dt) == (600, 600, 1.0 / 125.0, 1e-4)
    assert w.source[:2] == (200, 200) and w.receivers == [(400, 400)]
    s = w.source[2]
    peak = int(np.argmax(s))                          # at t = delay = 0.24 s
    assert abs((peak + 0.5) * w.dt - 0.24) <= w.dt
    assert s.max() == pytest.approx(w.dt / w.dx ** 2, rel=1e-5)   # half-step offset
    assert abs(s[0]) < 2e-5 * s.max() and abs(s[-1]) < 2e-5 * s.max()
    w30 = workloads.paper2d(ppw=30, nsteps=10)
    assert w30.nx == 1800 and w30.dx == pytest.approx(1.0 / 375.0)
