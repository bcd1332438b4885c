"""Pins of the oracle's 2D elastic free-surface system (Eq. A1, App. A:
periodic in x, free surfaces bounding y, a point source on vy).

What fixes it, independently of its code:
  * exact conservation of the discrete energy in fp64 on a heterogeneous
    medium with random fields (a wrong image sign, surface weight, index or
    stencil operand breaks the adjointness the conservation rests on);
  * closed-form standing modes between the two surfaces, compressional
    (syy held at zero on both surfaces) and shear (sxy odd about each
    surface, the surface itself moving);
  * the surface modulus against the textbook plate modulus E / (1 - nu^2)
    written from Young's modulus and Poisson's ratio;
  * the source: one step from rest moves exactly one vy value, by the
    sample itself (the source acts after the division by rho);
  * bit-exact mirror symmetry in x and periodic translation in x in fp16
    with compensation;
  * a numpy float16/float32 re-evaluation of the reduced-precision step.
"""
import numpy as np
import pytest

import oracle
from oracle import closed_forms

F = oracle.ELASTIC2D_FIELDS


def _medium(nx, ny, seed):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(2.03, 2.62, (ny, nx))
    cs = rng.uniform(1.0, 2.0, (ny, nx))
    cp = cs * rng.uniform(1.6, 2.3, (ny, nx))
    mu = rho * cs ** 2
    lam = rho * (cp ** 2 - 2 * cs ** 2)
    return rho, lam, mu, cp.max()


def _fields(nx, ny, seed, scale=0.1, fmt="f64"):
    rng = np.random.default_rng(seed)
    f = {k: oracle.round_to(scale * rng.normal(size=(ny, nx)), fmt) for k in F}
    f["syy"][0] = 0.0
    f["syy"][-1] = 0.0
    f["vy"][-1] = 0.0
    f["sxy"][-1] = 0.0
    return f


@pytest.mark.parametrize("nx,ny", [(24, 17), (9, 3), (40, 6)])
def test_energy_conserved_fp64(nx, ny):
    rho, lam, mu, cmax = _medium(nx, ny, 11 + nx)
    dt = 0.6 * (1 / np.sqrt(2)) / cmax
    f = _fields(nx, ny, 12 + nx)
    _, _, e = oracle.elastic2d(nx, ny, 1.0, dt, rho, lam, mu, f, nsteps=1500,
                               energy_every=50)
    assert e[0] > 0
    assert np.abs(e - e[0]).max() / e[0] < 1e-12


@pytest.mark.parametrize("kind,m,ny", [("p", 1, 21), ("p", 3, 16), ("s", 2, 21),
                                       ("s", 5, 13)])
def test_standing_modes_between_free_surfaces(kind, m, ny):
    nx, dt, rho, lam, mu = 4, 0.35, 2.2, 3.0, 1.7
    f0 = closed_forms.elastic2d_surface_modes(nx, ny, dt, rho, lam, mu, m, 0, kind)
    got, _, _ = oracle.elastic2d(nx, ny, 1.0, dt, rho, lam, mu, f0, nsteps=400)
    want = closed_forms.elastic2d_surface_modes(nx, ny, dt, rho, lam, mu, m, 400,
                                                kind)
    for k in F:
        assert np.abs(got[k] - want[k]).max() < 2e-13, k
    # not a trivially small state: of each (velocity, stress) pair one is
    # near its amplitude at any time
    pair = ("vy", "syy") if kind == "p" else ("vx", "sxy")
    assert max(np.abs(want[k]).max() for k in pair) > 0.5


def test_surface_modulus_is_the_plate_modulus():
    """A pure horizontal strain rate on the surface row: sxx there changes by
    w * E / (1 - nu^2) * (vx[i] - vx[i-1]) (sigma_yy = 0 at a free surface;
    E = mu (3 lam + 2 mu) / (lam + mu), nu = lam / (2 (lam + mu)))."""
    nx, ny = 8, 5
    rho, lam, mu = 2.4, 5.0, 2.0
    young = mu * (3 * lam + 2 * mu) / (lam + mu)
    nu = lam / (2 * (lam + mu))
    plate = closed_forms.f32(young / (1 - nu ** 2))
    f = {k: np.zeros((ny, nx)) for k in F}
    f["vx"][0, 3] = 0.5                 # at rest but for one surface velocity
    w = 0.25
    got, _, _ = oracle.elastic2d(nx, ny, 1.0, w, rho, lam, mu, f, nsteps=1)
    # the velocity step sees no stress, so vx keeps its value
    assert got["vx"][0, 3] == 0.5
    assert got["sxx"][0, 3] == pytest.approx(plate * w * 0.5, rel=1e-15)
    assert got["sxx"][0, 4] == pytest.approx(-plate * w * 0.5, rel=1e-15)
    assert got["syy"][0].tolist() == [0.0] * nx
    # an interior row uses lam + 2 mu and lam instead
    f["vx"][0, 3] = 0.0
    f["vx"][2, 3] = 0.5
    got, _, _ = oracle.elastic2d(nx, ny, 1.0, w, rho, lam, mu, f, nsteps=1)
    assert got["sxx"][2, 3] == closed_forms.f32(lam + 2 * mu) * w * 0.5
    assert got["syy"][2, 3] == closed_forms.f32(lam) * w * 0.5


def test_source_moves_one_vy_value_by_the_sample():
    nx, ny = 10, 7
    rho, lam, mu, _ = _medium(nx, ny, 5)
    f = {k: np.zeros((ny, nx)) for k in F}
    got, _, _, tr = oracle.elastic2d(nx, ny, 1.0, 0.1, rho, lam, mu, f, nsteps=1,
                                     source=(6, 2, [0.375]),
                                     receivers=[(6, 2), (0, 0)])
    assert got["vy"][2, 6] == 0.375
    assert np.count_nonzero(got["vy"]) == 1
    assert np.count_nonzero(got["vx"]) == 0
    assert tr.shape == (1, 2, 5)
    assert tr[0, 0].tolist() == [got[k][2, 6] for k in F]
    # the source on the last vy row (outside the body) is refused
    with pytest.raises(ValueError):
        oracle.elastic2d(nx, ny, 1.0, 0.1, rho, lam, mu, f, nsteps=1,
                         source=(6, ny - 1, [1.0]))


def _mirror(f):
    """x -> -x: cell-centred values map i -> -i, x-staggered ones i -> -i-1
    and change sign when they are odd in x (vx, sxy)."""
    out = {}
    for k, a in f.items():
        if k in ("vx", "sxy"):
            out[k] = -a[:, ::-1]
        else:
            out[k] = np.roll(a[:, ::-1], 1, axis=1)
    return out


def test_mirror_and_translation_bit_exact_fp16_twosum():
    nx, ny = 14, 9
    rho, lam, mu, cmax = _medium(nx, ny, 21)
    # a medium symmetric about i = 0: a[i] == a[-i]
    sym = lambda a: (a + np.roll(a[:, ::-1], 1, axis=1)) / 2
    rho, lam, mu = sym(rho), sym(lam), sym(mu)
    dt = 0.5 / cmax
    f = _fields(nx, ny, 22, fmt="f16")
    kw = dict(storage="f16", stencil="f32", comp="twosum", nsteps=40)
    a, ca, _ = oracle.elastic2d(nx, ny, 1.0, dt, rho, lam, mu, f, **kw)
    b, cb, _ = oracle.elastic2d(nx, ny, 1.0, dt, rho, lam, mu, _mirror(f), **kw)
    ma, mca = _mirror(a), _mirror(ca)
    for k in F:
        assert np.array_equal(b[k], ma[k]), k
        assert np.array_equal(cb[k], mca[k]), k
    # periodic translation along x
    sh = lambda d: {k: np.roll(v, 5, axis=1) for k, v in d.items()}
    rho2, lam2, mu2 = (np.roll(x, 5, axis=1) for x in (rho, lam, mu))
    t, ct, _ = oracle.elastic2d(nx, ny, 1.0, dt, rho2, lam2, mu2, sh(f), **kw)
    for k in F:
        assert np.array_equal(t[k], sh(a)[k]), k
        assert np.array_equal(ct[k], sh(ca)[k]), k


def _numpy_step(f, c, rho, lam, mu, w, comp):
    """One step re-evaluated with numpy's float32 (stencil) and float16
    (storage) arithmetic."""
    h, s32 = np.float16, np.float32
    ny, nx = f["vx"].shape
    W = s32(w)
    b = (1.0 / rho).astype(s32)
    sur = np.zeros((ny, 1), bool)
    sur[0] = sur[-1] = True
    l2m = np.where(sur, 4.0 * mu * (lam + mu) / (lam + 2.0 * mu),
                   lam + 2.0 * mu).astype(s32)
    lm = np.where(sur, 0.0, lam).astype(s32)
    mxy = np.zeros((ny, nx), s32)
    mxy[:-1] = (0.25 * ((mu[:-1] + np.roll(mu[:-1], -1, 1)) +
                        (mu[1:] + np.roll(mu[1:], -1, 1)))).astype(s32)
    R = lambda a, d: np.roll(a, -d, axis=1)      # R(a, 1)[i] = a[i+1]

    def upd(key, inc, mask=None):
        v, cc = f[key], c[key]
        if comp == "none":
            nv, ncc = (v + inc.astype(h)).astype(h), cc
        else:
            y = (inc + cc.astype(s32)).astype(h)
            s = (v + y).astype(h)
            pa = (s - y).astype(h)
            pb = (s - pa).astype(h)
            nv, ncc = s, ((v - pa).astype(h) + (y - pb).astype(h)).astype(h)
        if mask is not None:
            nv = np.where(mask, nv, v)
            ncc = np.where(mask, ncc, cc)
        f[key], c[key] = nv, ncc

    g32 = {k: f[k].astype(s32) for k in F}
    sxy = g32["sxy"]
    lo = np.vstack([-sxy[:1], sxy[:-1]])
    hi = np.vstack([sxy[:-1], -sxy[-2:-1]])
    d1 = R(g32["sxx"], 1) - g32["sxx"]
    incx = (s32(0.5) * (b + R(b, 1))) * (W * (d1 + (hi - lo)))
    syy = g32["syy"]
    d1 = sxy - R(sxy, -1)
    d2 = np.vstack([syy[1:] - syy[:-1], np.zeros((1, nx), s32)])
    by = np.vstack([s32(0.5) * (b[:-1] + b[1:]), np.ones((1, nx), s32)])
    incy = by * (W * (d1 + d2))
    rows = np.ones((ny, 1), bool)
    rows[-1] = False
    upd("vx", incx)
    upd("vy", incy, rows)
    vx, vy = f["vx"].astype(s32), f["vy"].astype(s32)
    ex = W * (vx - R(vx, -1))
    ey = np.vstack([np.zeros((1, nx), s32), W * (vy[1:-1] - vy[:-2]),
                    np.zeros((1, nx), s32)])
    upd("sxx", l2m * ex + lm * ey)
    upd("syy", l2m * ey + lm * ex, ~sur)
    a1 = R(vy, 1) - vy
    a2 = np.vstack([vx[1:] - vx[:-1], np.zeros((1, nx), s32)])
    upd("sxy", mxy * (W * (a1 + a2)), rows)


@pytest.mark.parametrize("comp", ["none", "twosum"])
def test_f16_step_matches_numpy(comp):
    nx, ny = 11, 8
    rho, lam, mu, cmax = _medium(nx, ny, 31)
    w = float(np.float32(0.5 / cmax))
    f0 = _fields(nx, ny, 32, fmt="f16")
    got, gotc, _ = oracle.elastic2d(nx, ny, 1.0, w, rho, lam, mu, f0,
                                    storage="f16", stencil="f32", comp=comp,
                                    nsteps=12)
    f = {k: f0[k].astype(np.float16) for k in F}
    c = {k: np.zeros((ny, nx), np.float16) for k in F}
    with np.errstate(all="ignore"):
        for _ in range(12):
            _numpy_step(f, c, rho, lam, mu, w, comp)
    for k in F:
        assert np.array_equal(got[k], f[k].astype(np.float64)), k
        if comp != "none":
            assert np.array_equal(gotc[k], c[k].astype(np.float64)), k


def test_compensation_keeps_energy_plain_fp16_loses_it():
    """App. A's finding in the small-Courant regime (Courant number 0.005):
    plain fp16 loses energy (about 4% here), the compensated update keeps
    it (a few parts per million)."""
    nx, ny = 32, 16
    rho, lam, mu, cmax = _medium(nx, ny, 41)
    dt = 0.005 / cmax
    f = {k: np.zeros((ny, nx)) for k in F}
    g = np.exp(-((np.arange(nx)[None, :] - 16) ** 2 +
                 (np.arange(ny)[:, None] - 8) ** 2) / 8.0)
    for k in ("sxx", "syy"):
        f[k] = oracle.round_to(g, "f16")
    f["syy"][0] = 0.0
    f["syy"][-1] = 0.0
    args = (nx, ny, 1.0, dt, rho, lam, mu, f)
    kw = dict(nsteps=4000, energy_every=1000)
    _, _, e64 = oracle.elastic2d(*args, **kw)
    _, _, e0 = oracle.elastic2d(*args, storage="f16", stencil="f32", **kw)
    _, _, e6 = oracle.elastic2d(*args, storage="f16", stencil="f32",
                                comp="twosum", **kw)
    assert abs(e64[-1] - e64[0]) / e64[0] < 1e-12
    assert (e0[-1] - e64[0]) / e64[0] < -2e-2
    assert abs(e6[-1] - e64[0]) / e64[0] < 2e-4


def test_bad_arguments_rejected():
    nx, ny = 6, 5
    rho, lam, mu, _ = _medium(nx, ny, 51)
    f = _fields(nx, ny, 52)
    bad = {k: v.copy() for k, v in f.items()}
    bad["syy"][0, 2] = 1.0
    with pytest.raises(ValueError):
        oracle.elastic2d(nx, ny, 1.0, 0.1, rho, lam, mu, bad, nsteps=1)
    bad = {k: v.copy() for k, v in f.items()}
    bad["sxy"][-1, 0] = 1.0
    with pytest.raises(ValueError):
        oracle.elastic2d(nx, ny, 1.0, 0.1, rho, lam, mu, bad, nsteps=1)
    with pytest.raises(ValueError):
        oracle.elastic2d(nx, 2, 1.0, 0.1, rho[:2], lam[:2], mu[:2],
                         {k: np.zeros((2, nx)) for k in F}, nsteps=1)
    with pytest.raises(ValueError):
        oracle.elastic2d(nx, ny, 1.0, 0.1, rho, lam, mu, f, nsteps=1,
                         storage="f16", stencil="f16")
