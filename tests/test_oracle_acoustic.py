"""Pins of the 2D acoustic oracle (Sec. 3, Eq. 1; Sec. 4, Alg. 1 and 2).

Each test checks the oracle against something other than itself: the exact
conservation law of the discrete scheme, closed-form discrete standing modes,
dense operators assembled from coordinates, the same op sequence evaluated
with numpy's native fp32/fp16 arithmetic and np.roll indexing, exact
symmetries, and the paper's qualitative findings on fp16 energy loss.
"""
import numpy as np
import pytest

import oracle
from oracle import brute, closed_forms
import workloads


def _layered(nx, ny, seed):
    rng = np.random.default_rng(seed)
    c_row, rho_row, _ = workloads.layered_profile(ny, 3, rng)
    rho = np.repeat(rho_row[:, None], nx, axis=1)
    kappa = np.repeat((rho_row * c_row ** 2)[:, None], nx, axis=1)
    # break the x-invariance as well
    rho = rho * (1 + 0.25 * np.sin(2 * np.pi * np.arange(nx) / nx))[None, :]
    return rho, kappa, float(np.sqrt(kappa / rho).max())


def _rel_drift(E):
    return float(np.max(np.abs(E - E[0])) / E[0])


@pytest.mark.parametrize("order", [2, 4])
def test_energy_conserved_fp64_heterogeneous(order):
    nx, ny = 45, 38
    rho, kappa, cmax = _layered(nx, ny, 11)
    dt = 0.3 / cmax
    rng = np.random.default_rng(12)
    fields = {"p": workloads.gaussian2d(nx, ny, 20, 17, 3.0),
              "vx": 0.1 * rng.normal(size=(ny, nx)),
              "vy": 0.1 * rng.normal(size=(ny, nx))}
    _, _, E = oracle.acoustic2d(nx, ny, order, 1.0, dt, rho, kappa, fields,
                                nsteps=600, energy_every=10)
    assert E[0] > 0
    assert _rel_drift(E) < 2e-13


def test_energy_changes_when_scheme_is_broken():
    """The conservation check is sensitive: the energy of a state advanced by
    the scheme with a mismatched time step is not conserved."""
    nx, ny = 32, 32
    rho = np.ones((ny, nx))
    f = {"p": workloads.gaussian2d(nx, ny, 16, 16, 3.0),
         "vx": np.zeros((ny, nx)), "vy": np.zeros((ny, nx))}
    f1, _, _ = oracle.acoustic2d(nx, ny, 4, 1.0, 0.3, rho, rho, f, nsteps=50)
    e_ok = oracle.acoustic2d_energy(nx, ny, 4, 1.0, 0.3, rho, rho, f1)
    e_bad = oracle.acoustic2d_energy(nx, ny, 4, 1.0, 0.31, rho, rho, f1)
    e0 = oracle.acoustic2d_energy(nx, ny, 4, 1.0, 0.3, rho, rho, f)
    assert abs(e_ok - e0) / e0 < 1e-14
    assert abs(e_bad - e0) / e0 > 1e-5    # eight orders above roundoff


@pytest.mark.parametrize("order,nx,ny,mx,my,rho,kappa,dt", [
    (2, 24, 16, 2, 1, 1.0, 1.0, 0.5),
    (4, 24, 16, 3, 2, 2.0, 0.5, 0.9),
    (4, 20, 20, 1, 4, 1.0, 1.0, 0.4),
    (2, 10, 14, 5, 3, 1.5, 3.0, 0.3),   # Nyquist in x
])
def test_standing_mode_closed_form(order, nx, ny, mx, my, rho, kappa, dt):
    n_steps = 300
    init = closed_forms.acoustic_standing_mode(nx, ny, order, 1.0, dt, rho,
                                               kappa, mx, my, 0)
    want = closed_forms.acoustic_standing_mode(nx, ny, order, 1.0, dt, rho,
                                               kappa, mx, my, n_steps)
    got, _, _ = oracle.acoustic2d(nx, ny, order, 1.0, dt, rho, kappa, init,
                                  nsteps=n_steps)
    for k in ("vx", "vy", "p"):
        assert np.max(np.abs(got[k] - want[k])) < 1e-11, k


@pytest.mark.parametrize("order", [2, 4])
def test_dense_operators_adjoint(order):
    """The divergence is minus the transpose of the gradient on the periodic
    staggered grid, which is what makes the energy conserved."""
    Gx, Gy, Dx, Dy, *_ = brute.acoustic2d_operators(7, 5, order, 1.0, 0.3,
                                                    1.0, 1.0)
    assert np.array_equal(Dx, -Gx.T)
    assert np.array_equal(Dy, -Gy.T)


@pytest.mark.parametrize("order,nx,ny", [(2, 7, 5), (4, 7, 5), (4, 3, 6),
                                         (4, 1, 5)])
def test_matches_dense_operators(order, nx, ny):
    rng = np.random.default_rng(13)
    rho = rng.uniform(1.0, 2.5, size=(ny, nx))
    kappa = rng.uniform(1.0, 4.0, size=(ny, nx))
    f = {k: rng.normal(size=(ny, nx)) for k in ("vx", "vy", "p")}
    ops = brute.acoustic2d_operators(nx, ny, order, 1.0, 0.2, rho, kappa)
    vx, vy, p = (f[k].ravel() for k in ("vx", "vy", "p"))
    for _ in range(3):
        vx, vy, p = brute.acoustic2d_step(ops, vx, vy, p)
    got, _, _ = oracle.acoustic2d(nx, ny, order, 1.0, 0.2, rho, kappa, f,
                                  nsteps=3)
    for k, ref in (("vx", vx), ("vy", vy), ("p", p)):
        np.testing.assert_allclose(got[k].ravel(), ref, rtol=0, atol=1e-13)


# ------------------------------------------------------ precision emulation --

def _bf16(x32):
    u = np.asarray(x32, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


class _Native:
    """The op sequence evaluated with numpy's own fp32/fp16 arithmetic."""

    def __init__(self, storage):
        self.storage = storage

    def T(self, x32):
        if self.storage == "f16":
            return np.asarray(x32, np.float32).astype(np.float16)
        if self.storage == "bf16":
            return _bf16(x32)
        return np.asarray(x32, np.float32)

    def add(self, a, b):
        if self.storage == "bf16":
            return _bf16(a.astype(np.float32) + b.astype(np.float32))
        return a + b

    def sub(self, a, b):
        if self.storage == "bf16":
            return _bf16(a.astype(np.float32) - b.astype(np.float32))
        return a - b

    def update(self, v, c, inc, comp):
        if comp == "none":
            return self.add(v, self.T(inc)), c
        y = self.T(inc + c.astype(np.float32))
        s = self.add(v, y)
        if comp == "fast2sum":
            z = self.sub(s, v)
            return s, self.sub(y, z)
        pa = self.sub(s, y)
        pb = self.sub(s, pa)
        da = self.sub(v, pa)
        db = self.sub(y, pb)
        return s, self.add(da, db)


def _native_run(nx, ny, order, dt, rho, kappa, f, storage, comp, nsteps):
    f32 = np.float32
    N = _Native(storage)
    w1, w2 = (f32(w) for w in closed_forms.stencil_weights(order, dt, 1.0))
    b = (1.0 / rho).astype(f32)
    k = kappa.astype(f32)
    st = {key: N.T(f[key].astype(f32)) for key in ("vx", "vy", "p")}
    cp = {key: N.T(np.zeros((ny, nx), f32)) for key in st}

    def sh(a, dj, di):           # value at (j + dj, i + di), periodic
        return np.roll(a, (-dj, -di), axis=(0, 1))

    def grad(a, axis):           # forward staggered difference, fp32
        dj, di = (1, 0) if axis == 0 else (0, 1)
        a0 = sh(a, dj, di) - a
        if order == 2:
            return w1 * a0
        a1 = sh(a, 2 * dj, 2 * di) - sh(a, -dj, -di)
        return w1 * a0 + w2 * a1

    def div(a, axis):            # backward staggered difference, fp32
        dj, di = (1, 0) if axis == 0 else (0, 1)
        a0 = a - sh(a, -dj, -di)
        if order == 2:
            return w1 * a0
        a1 = sh(a, dj, di) - sh(a, -2 * dj, -2 * di)
        return w1 * a0 + w2 * a1

    for _ in range(nsteps):
        P = st["p"].astype(f32)
        bx = f32(0.5) * (b + sh(b, 0, 1))
        by = f32(0.5) * (b + sh(b, 1, 0))
        st["vx"], cp["vx"] = N.update(st["vx"], cp["vx"], bx * grad(P, 1), comp)
        st["vy"], cp["vy"] = N.update(st["vy"], cp["vy"], by * grad(P, 0), comp)
        d = div(st["vx"].astype(f32), 1) + div(st["vy"].astype(f32), 0)
        st["p"], cp["p"] = N.update(st["p"], cp["p"], k * d, comp)
    return ({key: v.astype(np.float64) for key, v in st.items()},
            {key: v.astype(np.float64) for key, v in cp.items()})


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("comp", ["none", "fast2sum", "twosum"])
@pytest.mark.parametrize("order", [2, 4])
def test_emulation_matches_native_arithmetic(storage, comp, order):
    nx, ny = 11, 9
    rng = np.random.default_rng(14)
    rho = rng.uniform(1.0, 2.5, size=(ny, nx))
    kappa = rng.uniform(1.0, 6.0, size=(ny, nx))
    f = {"p": oracle.round_to(workloads.gaussian2d(nx, ny, 5, 4, 2.0), storage),
         "vx": np.zeros((ny, nx)), "vy": np.zeros((ny, nx))}
    dt = 0.25
    want, wantc = _native_run(nx, ny, order, dt, rho, kappa, f, storage, comp, 12)
    got, gotc, _ = oracle.acoustic2d(nx, ny, order, 1.0, dt, rho, kappa, f,
                                     storage=storage, stencil="f32", comp=comp,
                                     nsteps=12)
    for key in ("vx", "vy", "p"):
        assert np.array_equal(got[key], want[key]), key
        if comp != "none":
            assert np.array_equal(gotc[key], wantc[key]), key


def test_zero_compensation_equals_plain():
    """With no bits carried over, the compensated update reduces to the plain
    one for a single step (Alg. 2 vs Alg. 1)."""
    w = workloads.small2d(32, nsteps=1)
    f = {k: oracle.round_to(v, "f16") for k, v in w.fields().items()}
    a, _, _ = oracle.acoustic2d(32, 32, 2, 1.0, w.dt, w.rho, w.kappa, f,
                                storage="f16", stencil="f32", nsteps=1)
    for comp in ("fast2sum", "twosum"):
        b, _, _ = oracle.acoustic2d(32, 32, 2, 1.0, w.dt, w.rho, w.kappa, f,
                                    storage="f16", stencil="f32", comp=comp,
                                    nsteps=1)
        for k in a:
            assert np.array_equal(a[k], b[k])


# ------------------------------------------------------------- invariances --

def _run16(w, f, comp, nsteps):
    return oracle.acoustic2d(w.nx, w.ny, w.order, w.dx, w.dt, w.rho, w.kappa,
                             f, storage="f16", stencil="f32", comp=comp,
                             nsteps=nsteps)[0]


def test_uniform_pressure_is_steady():
    w = workloads.small2d(16, nsteps=0)
    f = {"p": np.full((16, 16), 0.37109375), "vx": np.zeros((16, 16)),
         "vy": np.zeros((16, 16))}
    out = _run16(w, f, "twosum", 20)
    assert np.array_equal(out["p"], f["p"])
    assert not out["vx"].any() and not out["vy"].any()


@pytest.mark.parametrize("comp", ["none", "twosum"])
def test_symmetries_bit_exact(comp):
    """The centred pulse on a homogeneous grid keeps its mirror and diagonal
    symmetries bit for bit in fp16 (rounding to nearest is sign symmetric and
    addition commutes).  Under the mirror x -> -x the staggered vx point
    i+1/2 maps to index n-1-i (about the centre) and vx changes sign."""
    n = 32
    w = workloads.small2d(n, nsteps=0, order=4, cfl=0.4, sigma=3.0)
    f = {k: oracle.round_to(v, "f16") for k, v in w.fields().items()}
    out = _run16(w, f, comp, 40)
    c = n // 2
    idx = (2 * c - np.arange(n)) % n          # p mirror about the centre
    vidx = (2 * c - 1 - np.arange(n)) % n     # vx mirror
    p, vx, vy = out["p"], out["vx"], out["vy"]
    assert np.array_equal(p, p[:, idx])
    assert np.array_equal(p, p[idx, :])
    assert np.array_equal(vx, -vx[:, vidx])
    assert np.array_equal(vy, -vy[vidx, :])
    assert np.array_equal(p, p.T)
    assert np.array_equal(vx, vy.T)
    assert np.abs(p).max() > 0.01


def test_translation_invariance_bit_exact():
    w = workloads.small2d(20, nsteps=0, order=4, cfl=0.4, sigma=2.5)
    rng = np.random.default_rng(15)
    f = {"p": oracle.round_to(rng.normal(size=(20, 20)), "f16"),
         "vx": oracle.round_to(0.1 * rng.normal(size=(20, 20)), "f16"),
         "vy": oracle.round_to(0.1 * rng.normal(size=(20, 20)), "f16")}
    a = _run16(w, f, "twosum", 15)
    g = {k: np.roll(v, (3, -7), axis=(0, 1)) for k, v in f.items()}
    b = _run16(w, g, "twosum", 15)
    for k in a:
        assert np.array_equal(np.roll(a[k], (3, -7), axis=(0, 1)), b[k])


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_power_of_two_scaling_bit_exact(storage):
    """Scaling all fields by a power of two scales every rounded result by the
    same power, as long as nothing reaches the subnormal range; f32 and bf16
    share the fp32 exponent range, so these fields stay normal throughout."""
    w = workloads.small2d(16, nsteps=0, order=4, cfl=0.4, sigma=2.0)
    f = {k: oracle.round_to(v, storage) for k, v in w.fields().items()}
    run = lambda g: oracle.acoustic2d(16, 16, 4, 1.0, w.dt, w.rho, w.kappa, g,
                                      storage=storage, stencil="f32",
                                      comp="twosum", nsteps=20)
    a, ca, _ = run(f)
    b, cb, _ = run({k: v * 2.0 ** 40 for k, v in f.items()})
    for k in a:
        assert np.array_equal(a[k] * 2.0 ** 40, b[k])
        assert np.array_equal(ca[k] * 2.0 ** 40, cb[k])


# ----------------------------------------------------- the paper's findings --

def test_fp16_plain_loses_energy_compensation_restores_it():
    """Sec. 3 and Sec. 4: at a small Courant number the per-step increments
    are far below an fp16 ulp of the field, so the plain fp16 update (Alg. 1)
    loses energy, while the compensated update (Alg. 2) conserves it to the
    fp16 level; the 3- and 6-operation sums behave alike; fp32 agrees with
    fp64 far below the fp16 effects."""
    n = 32
    w = workloads.small2d(n, nsteps=0, order=4, cfl=0.0125, sigma=3.0)
    f = {k: oracle.round_to(v, "f16") for k, v in w.fields().items()}
    steps, every = 6000, 500
    common = dict(nsteps=steps, energy_every=every)
    args = (n, n, 4, 1.0, w.dt, w.rho, w.kappa, f)
    _, _, e64 = oracle.acoustic2d(*args, **common)
    _, _, e32 = oracle.acoustic2d(*args, storage="f32", stencil="f32", **common)
    _, _, e16 = oracle.acoustic2d(*args, storage="f16", stencil="f32", **common)
    _, _, e3 = oracle.acoustic2d(*args, storage="f16", stencil="f32",
                                 comp="fast2sum", **common)
    _, _, e6 = oracle.acoustic2d(*args, storage="f16", stencil="f32",
                                 comp="twosum", **common)
    d16 = (e16[-1] - e64[0]) / e64[0]
    d3 = np.max(np.abs(e3 - e64)) / e64[0]
    d6 = np.max(np.abs(e6 - e64)) / e64[0]
    d32 = np.max(np.abs(e32 - e64)) / e64[0]
    assert d16 < -2e-2            # energy loss, not gain
    assert d3 < 5e-4 and d6 < 5e-4
    assert d3 < 0.02 * abs(d16) and d6 < 0.02 * abs(d16)
    assert d32 < 1e-5
