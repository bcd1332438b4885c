"""Pins of the oracle's stencil-precision modes (App. B: the stencil
promoted to fp64 with the update kept in fp16; and the paper-literal
all-fp16 step of Alg. 1 in which the stencil, its weights and the material
are fp16 values too).

Each mode is re-evaluated with numpy's own arithmetic -- float16 arrays
throughout for the all-fp16 step, float64 stencils with float16 updates for
the promoted one (numpy rounds float64 to float16 directly) -- and App. B's
finding is checked on the oracle: promoting the stencil leaves plain fp16's
energy loss in place, compensation removes it.
"""
import numpy as np
import pytest

import oracle
from oracle import closed_forms
import workloads

F = ("vx", "vy", "p")


def _sh(a, dj, di):
    return np.roll(a, (-dj, -di), axis=(0, 1))


def _stencils(order, w1, w2):
    def grad(a, axis):
        dj, di = (1, 0) if axis == 0 else (0, 1)
        a0 = _sh(a, dj, di) - a
        if order == 2:
            return w1 * a0
        return w1 * a0 + w2 * (_sh(a, 2 * dj, 2 * di) - _sh(a, -dj, -di))

    def div(a, axis):
        dj, di = (1, 0) if axis == 0 else (0, 1)
        a0 = a - _sh(a, -dj, -di)
        if order == 2:
            return w1 * a0
        return w1 * a0 + w2 * (_sh(a, dj, di) - _sh(a, -2 * dj, -2 * di))
    return grad, div


def _update16(v, c, y, comp):
    """v, c float16; y the float16 value added (already rounded)."""
    if comp == "none":
        return v + y, c
    s = v + y
    if comp == "fast2sum":
        return s, y - (s - v)
    pa = s - y
    pb = s - pa
    return s, (v - pa) + (y - pb)


def _native_all16(order, dt, rho, kappa, f, comp, nsteps):
    h = np.float16
    w1, w2 = (h(np.float32(w)) for w in closed_forms.stencil_weights(order, dt, 1.0))
    b = (1.0 / rho).astype(np.float32).astype(h)
    k = kappa.astype(np.float32).astype(h)
    grad, div = _stencils(order, w1, w2)
    st = {key: f[key].astype(h) for key in F}
    cp = {key: np.zeros_like(st[key]) for key in F}
    half = h(0.5)
    for _ in range(nsteps):
        bx = half * (b + _sh(b, 0, 1))
        by = half * (b + _sh(b, 1, 0))
        for key, inc in (("vx", bx * grad(st["p"], 1)), ("vy", by * grad(st["p"], 0))):
            y = inc if comp == "none" else inc + cp[key]
            st[key], cp[key] = _update16(st[key], cp[key], y, comp)
        inc = k * (div(st["vx"], 1) + div(st["vy"], 0))
        y = inc if comp == "none" else inc + cp["p"]
        st["p"], cp["p"] = _update16(st["p"], cp["p"], y, comp)
    return ({key: v.astype(np.float64) for key, v in st.items()},
            {key: v.astype(np.float64) for key, v in cp.items()})


def _native_f64_stencil(order, dt, rho, kappa, f, comp, nsteps):
    h = np.float16
    w1, w2 = (float(np.float32(w)) for w in closed_forms.stencil_weights(order, dt, 1.0))
    b = (1.0 / rho).astype(np.float32).astype(np.float64)
    k = kappa.astype(np.float32).astype(np.float64)
    grad, div = _stencils(order, w1, w2)
    st = {key: f[key].astype(h) for key in F}
    cp = {key: np.zeros_like(st[key]) for key in F}
    for _ in range(nsteps):
        bx = 0.5 * (b + _sh(b, 0, 1))
        by = 0.5 * (b + _sh(b, 1, 0))
        P = st["p"].astype(np.float64)
        for key, inc in (("vx", bx * grad(P, 1)), ("vy", by * grad(P, 0))):
            y = inc if comp == "none" else inc + cp[key].astype(np.float64)
            st[key], cp[key] = _update16(st[key], cp[key], y.astype(h), comp)
        d = div(st["vx"].astype(np.float64), 1) + div(st["vy"].astype(np.float64), 0)
        inc = k * d
        y = inc if comp == "none" else inc + cp["p"].astype(np.float64)
        st["p"], cp["p"] = _update16(st["p"], cp["p"], y.astype(h), comp)
    return ({key: v.astype(np.float64) for key, v in st.items()},
            {key: v.astype(np.float64) for key, v in cp.items()})


def _problem():
    nx, ny = 13, 10
    rng = np.random.default_rng(41)
    rho = rng.uniform(1.0, 2.5, size=(ny, nx))
    kappa = rng.uniform(1.0, 6.0, size=(ny, nx))
    f = {"p": oracle.round_to(workloads.gaussian2d(nx, ny, 6, 4, 2.0), "f16"),
         "vx": oracle.round_to(0.05 * rng.normal(size=(ny, nx)), "f16"),
         "vy": oracle.round_to(0.05 * rng.normal(size=(ny, nx)), "f16")}
    return nx, ny, rho, kappa, f


@pytest.mark.parametrize("comp", ["none", "fast2sum", "twosum"])
@pytest.mark.parametrize("order", [2, 4])
def test_all_f16_step_matches_native_f16(comp, order):
    nx, ny, rho, kappa, f = _problem()
    want, wantc = _native_all16(order, 0.25, rho, kappa, f, comp, 10)
    got, gotc, _ = oracle.acoustic2d(nx, ny, order, 1.0, 0.25, rho, kappa, f,
                                     storage="f16", stencil="f16", comp=comp,
                                     nsteps=10)
    for key in F:
        assert np.array_equal(got[key], want[key]), key
        if comp != "none":
            assert np.array_equal(gotc[key], wantc[key]), key


@pytest.mark.parametrize("comp", ["none", "fast2sum", "twosum"])
@pytest.mark.parametrize("order", [2, 4])
def test_f64_stencil_with_f16_update_matches_native(comp, order):
    nx, ny, rho, kappa, f = _problem()
    want, wantc = _native_f64_stencil(order, 0.25, rho, kappa, f, comp, 10)
    got, gotc, _ = oracle.acoustic2d(nx, ny, order, 1.0, 0.25, rho, kappa, f,
                                     storage="f16", stencil="f64", comp=comp,
                                     nsteps=10)
    for key in F:
        assert np.array_equal(got[key], want[key]), key
        if comp != "none":
            assert np.array_equal(gotc[key], wantc[key]), key


def test_energy_uses_fp32_material_in_every_mode():
    """The energy of a state does not depend on the stencil mode."""
    nx, ny, rho, kappa, f = _problem()
    e = [oracle.acoustic2d(nx, ny, 4, 1.0, 0.25, rho, kappa, f, storage="f16",
                           stencil=s, nsteps=0, energy_every=1)[2][0]
         for s in ("f16", "f32", "f64")]
    assert e[0] == e[1] == e[2]


def test_promoting_the_stencil_does_not_cure_plain_fp16():
    """App. B: with the stencil in fp64 and the update in fp16, the plain
    update still loses energy at a small Courant number; the compensated
    update does not.  The all-fp16 step behaves like the fp32-stencil one."""
    n = 32
    w = workloads.small2d(n, nsteps=0, order=4, cfl=0.0125, sigma=3.0)
    f = {k: oracle.round_to(v, "f16") for k, v in w.fields().items()}
    common = dict(nsteps=6000, energy_every=500)
    args = (n, n, 4, 1.0, w.dt, w.rho, w.kappa, f)
    _, _, e64 = oracle.acoustic2d(*args, **common)
    drift = {}
    for st in ("f64", "f32", "f16"):
        for comp in ("none", "fast2sum"):
            _, _, e = oracle.acoustic2d(*args, storage="f16", stencil=st, comp=comp,
                                        **common)
            drift[st, comp] = (e[-1] - e64[0]) / e64[0]
    for st in ("f64", "f32", "f16"):
        assert drift[st, "none"] < -2e-2
        assert abs(drift[st, "fast2sum"]) < 1e-3
