"""Pins of the 3D elastic oracle (velocity-stress form, the 3D extension of
Eq. A1 of App. A, on the staggered layout; compensated update of Sec. 4).

Checked against the exact conservation law, closed-form compressional and
shear standing modes, dense operators assembled from coordinates, and the
same op sequence evaluated with numpy's native fp32/fp16 arithmetic.
"""
import numpy as np
import pytest

import oracle
from oracle import brute, closed_forms
import workloads

NAMES = oracle.ELASTIC_FIELDS


def _medium(nx, ny, nz, seed):
    rng = np.random.default_rng(seed)
    rho = workloads.smooth_field3d(nx, ny, nz, rng, nmodes=6, kmax=2)
    lam = workloads.smooth_field3d(nx, ny, nz, rng, nmodes=6, kmax=2)
    mu = workloads.smooth_field3d(nx, ny, nz, rng, nmodes=6, kmax=2)
    cp = float(np.sqrt((lam + 2 * mu) / rho).max())
    return rho, lam, mu, cp


def test_energy_conserved_fp64_heterogeneous():
    nx, ny, nz = 13, 11, 9
    rho, lam, mu, cp = _medium(nx, ny, nz, 21)
    rng = np.random.default_rng(22)
    f = {k: 0.1 * rng.normal(size=(nz, ny, nx)) for k in NAMES}
    _, _, E = oracle.elastic3d(nx, ny, nz, 1.0, 0.3 / cp, rho, lam, mu, f,
                               nsteps=300, energy_every=10)
    assert E[0] > 0
    assert np.max(np.abs(E - E[0])) / E[0] < 2e-13


@pytest.mark.parametrize("m,rho,lam,mu,dt", [(2, 1.0, 1.0, 1.0, 0.3),
                                             (3, 2.0, 0.5, 1.5, 0.25)])
def test_p_mode_closed_form(m, rho, lam, mu, dt):
    nx, ny, nz = 16, 3, 4
    init = closed_forms.elastic_p_mode_x(nx, ny, nz, 1.0, dt, rho, lam, mu, m, 0)
    want = closed_forms.elastic_p_mode_x(nx, ny, nz, 1.0, dt, rho, lam, mu, m, 250)
    got, _, _ = oracle.elastic3d(nx, ny, nz, 1.0, dt, rho, lam, mu, init,
                                 nsteps=250)
    for k in NAMES:
        assert np.max(np.abs(got[k] - want[k])) < 1e-11, k


@pytest.mark.parametrize("pair", [("y", "x"), ("y", "z")])
def test_s_mode_closed_form(pair):
    nx, ny, nz = (14, 3, 4) if pair[1] == "x" else (3, 4, 14)
    rho, lam, mu, dt = 1.5, 1.0, 0.75, 0.3
    init = closed_forms.elastic_s_mode(nx, ny, nz, 1.0, dt, rho, lam, mu, 2, 0, pair)
    want = closed_forms.elastic_s_mode(nx, ny, nz, 1.0, dt, rho, lam, mu, 2, 250, pair)
    got, _, _ = oracle.elastic3d(nx, ny, nz, 1.0, dt, rho, lam, mu, init,
                                 nsteps=250)
    for k in NAMES:
        assert np.max(np.abs(got[k] - want[k])) < 1e-11, k


def test_dense_operators_adjoint():
    ops = brute.elastic3d_operators(4, 3, 3, 1.0, 0.2, 1.0, 1.0, 1.0)
    # divergence rows of the velocity update are minus the transposed strain
    assert np.array_equal(ops["vx"][0], -ops["exx"].T)
    assert np.array_equal(ops["vy"][1], -ops["eyy"].T)
    assert np.array_equal(ops["vz"][2], -ops["ezz"].T)
    assert np.array_equal(ops["vx"][1], -ops["sxy"][1].T)
    assert np.array_equal(ops["vy"][0], -ops["sxy"][0].T)
    assert np.array_equal(ops["vx"][2], -ops["sxz"][1].T)
    assert np.array_equal(ops["vz"][0], -ops["sxz"][0].T)
    assert np.array_equal(ops["vy"][2], -ops["syz"][1].T)
    assert np.array_equal(ops["vz"][1], -ops["syz"][0].T)


@pytest.mark.parametrize("shape", [(4, 3, 3), (5, 2, 3), (1, 4, 3)])
def test_matches_dense_operators(shape):
    nx, ny, nz = shape
    rng = np.random.default_rng(23)
    rho = rng.uniform(1.0, 3.0, size=(nz, ny, nx))
    lam = rng.uniform(1.0, 3.0, size=(nz, ny, nx))
    mu = rng.uniform(1.0, 3.0, size=(nz, ny, nx))
    f = {k: rng.normal(size=(nz, ny, nx)) for k in NAMES}
    ops = brute.elastic3d_operators(nx, ny, nz, 1.0, 0.15, rho, lam, mu)
    flat = {k: v.ravel() for k, v in f.items()}
    for _ in range(3):
        flat = brute.elastic3d_step(ops, flat)
    got, _, _ = oracle.elastic3d(nx, ny, nz, 1.0, 0.15, rho, lam, mu, f,
                                 nsteps=3)
    for k in NAMES:
        np.testing.assert_allclose(got[k].ravel(), flat[k], rtol=0, atol=1e-13)


# ------------------------------------------------------ precision emulation --

def _native_run(nx, ny, nz, dt, rho, lam, mu, f, comp, nsteps):
    """The elastic op sequence with numpy's fp32 (stencil) and fp16 (storage)
    arithmetic and np.roll neighbours."""
    f32, f16 = np.float32, np.float16
    w = f32(closed_forms.f32(dt))
    b = (1.0 / rho).astype(f32)
    L = lam.astype(f32)
    M = mu.astype(f32)
    st = {k: f[k].astype(f32).astype(f16) for k in NAMES}
    cs = {k: np.zeros((nz, ny, nx), f16) for k in NAMES}
    ax = {"x": 2, "y": 1, "z": 0}

    def at(a, **off):            # value at index + offset, periodic
        out = a
        for name, o in off.items():
            out = np.roll(out, -o, axis=ax[name])
        return out

    def upd(key, inc):
        v, c = st[key], cs[key]
        if comp == "none":
            st[key] = v + inc.astype(f16)
            return
        y = (inc + c.astype(f32)).astype(f16)
        s = v + y
        pa = s - y
        pb = s - pa
        cs[key] = (v - pa) + (y - pb)
        st[key] = s

    for _ in range(nsteps):
        F = {k: st[k].astype(f32) for k in NAMES}
        half = f32(0.5)
        upd("vx", half * (b + at(b, x=1)) * (w * (((at(F["sxx"], x=1) - F["sxx"]) +
              (F["sxy"] - at(F["sxy"], y=-1))) + (F["sxz"] - at(F["sxz"], z=-1)))))
        upd("vy", half * (b + at(b, y=1)) * (w * (((F["sxy"] - at(F["sxy"], x=-1)) +
              (at(F["syy"], y=1) - F["syy"])) + (F["syz"] - at(F["syz"], z=-1)))))
        upd("vz", half * (b + at(b, z=1)) * (w * (((F["sxz"] - at(F["sxz"], x=-1)) +
              (F["syz"] - at(F["syz"], y=-1))) + (at(F["szz"], z=1) - F["szz"]))))
        V = {k: st[k].astype(f32) for k in ("vx", "vy", "vz")}
        ex = w * (V["vx"] - at(V["vx"], x=-1))
        ey = w * (V["vy"] - at(V["vy"], y=-1))
        ez = w * (V["vz"] - at(V["vz"], z=-1))
        l2m = L + f32(2.0) * M
        upd("sxx", l2m * ex + L * (ey + ez))
        upd("syy", l2m * ey + L * (ex + ez))
        upd("szz", l2m * ez + L * (ex + ey))
        q = f32(0.25)
        upd("sxy", (q * ((M + at(M, x=1)) + (at(M, y=1) + at(M, x=1, y=1)))) *
            (w * ((at(V["vy"], x=1) - V["vy"]) + (at(V["vx"], y=1) - V["vx"]))))
        upd("sxz", (q * ((M + at(M, x=1)) + (at(M, z=1) + at(M, x=1, z=1)))) *
            (w * ((at(V["vz"], x=1) - V["vz"]) + (at(V["vx"], z=1) - V["vx"]))))
        upd("syz", (q * ((M + at(M, y=1)) + (at(M, z=1) + at(M, y=1, z=1)))) *
            (w * ((at(V["vz"], y=1) - V["vz"]) + (at(V["vy"], z=1) - V["vy"]))))
    return ({k: v.astype(np.float64) for k, v in st.items()},
            {k: v.astype(np.float64) for k, v in cs.items()})


@pytest.mark.parametrize("comp", ["none", "twosum"])
def test_emulation_matches_native_arithmetic(comp):
    nx, ny, nz = 7, 6, 5
    rng = np.random.default_rng(24)
    rho = rng.uniform(1.0, 3.0, size=(nz, ny, nx))
    lam = rng.uniform(1.0, 3.0, size=(nz, ny, nx))
    mu = rng.uniform(1.0, 3.0, size=(nz, ny, nx))
    g = workloads.gaussian3d(nx, ny, nz, 3, 3, 2, 1.5)
    f = {k: np.zeros((nz, ny, nx)) for k in NAMES}
    for k in ("sxx", "syy", "szz"):
        f[k] = oracle.round_to(g, "f16")
    f["sxy"] = oracle.round_to(0.3 * rng.normal(size=(nz, ny, nx)), "f16")
    dt = 0.15
    want, wantc = _native_run(nx, ny, nz, dt, rho, lam, mu, f, comp, 8)
    got, gotc, _ = oracle.elastic3d(nx, ny, nz, 1.0, dt, rho, lam, mu, f,
                                    storage="f16", stencil="f32", comp=comp,
                                    nsteps=8)
    for k in NAMES:
        assert np.array_equal(got[k], want[k]), k
        if comp != "none":
            assert np.array_equal(gotc[k], wantc[k]), k


def test_fp16_compensated_energy_closer_than_plain():
    """App. A: the compensated fp16 run keeps the energy far closer to the
    fp64 reference than the plain fp16 run does (small Courant number)."""
    n = 10
    rho, lam, mu, cp = _medium(n, n, n, 25)
    g = workloads.gaussian3d(n, n, n, 5, 5, 5, 2.0)
    f = {k: np.zeros((n, n, n)) for k in NAMES}
    for k in ("sxx", "syy", "szz"):
        f[k] = oracle.round_to(g, "f16")
    dt = 0.01 / cp
    args = (n, n, n, 1.0, dt, rho, lam, mu, f)
    common = dict(nsteps=3000, energy_every=375)
    _, _, e64 = oracle.elastic3d(*args, **common)
    _, _, e16 = oracle.elastic3d(*args, storage="f16", stencil="f32", **common)
    _, _, e6 = oracle.elastic3d(*args, storage="f16", stencil="f32",
                                comp="twosum", **common)
    d16 = (e16[-1] - e64[0]) / e64[0]
    d6 = np.max(np.abs(e6 - e64)) / e64[0]
    assert d16 < -3e-3            # plain fp16 loses energy
    assert d6 < 0.02 * abs(d16)
