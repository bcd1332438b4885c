"""Pins of the oracle's 8-bit compensation word (the compensated sum of
Sec. 4 with the compensation term held in 8 bits relative to the last place
of the sum): hand-computed quantisations, the quantisation bound over
exhaustive fp16 sums, the stagnating recursive sum of Sec. 4, the energy in
the small-Courant regime, and the step re-evaluated with numpy float16."""
import math

import numpy as np
import pytest

import oracle
import workloads

Q = oracle.quantize_comp


def _r16(x):
    return float(np.asarray(oracle.round_to(x, "f16")).ravel()[0])


def test_hand_values():
    u = 2.0 ** -10                                   # fp16 spacing at 1.0
    assert Q(3 * 2.0 ** -17, 1.0, "f16") == 3 * 2.0 ** -17    # 3 * u/128
    assert Q(2.0 ** -18, 1.0, "f16") == 0.0                   # q = 1/2 -> 0
    assert Q(3 * 2.0 ** -18, 1.0, "f16") == 2.0 ** -16        # q = 3/2 -> 2
    assert Q(-u / 2, 1.0, "f16") == -u / 2                    # q = -64
    assert Q(u / 2, -1.5, "f16") == u / 2
    assert Q(2.0 ** -12, 1024.0, "f16") == 0.0                # ulp(1024) = 1
    assert Q(2.0 ** -30, 0.0, "f16") == 2.0 ** -30            # ulp = 2^-24, q = 2
    assert Q(2.0 ** -33, 0.0, "f16") == 0.0                   # q = 1/4 -> 0
    assert Q(2.0 ** -31, 2.0 ** -20, "f16") == 2.0 ** -31     # subnormal s
    assert Q(3 * 2.0 ** -14, 1.0, "bf16") == 3 * 2.0 ** -14   # ulp 2^-7, q = 3
    assert Q(3 * 2.0 ** -15, 1.0, "bf16") == 2.0 ** -13       # q = 3/2 -> 2
    assert math.copysign(1.0, Q(-2.0 ** -20, 1.0, "f16")) == 1.0   # +0, never -0
    assert math.copysign(1.0, Q(-0.0, 1.0, "f16")) == 1.0
    assert Q(float("nan"), 1.0, "f16") == 0.0
    assert Q(1.0, float("inf"), "f16") == 0.0


def _ulp16(s):
    s = abs(float(s))
    if s < 2.0 ** -14:
        return 2.0 ** -24
    return 2.0 ** (math.floor(math.log2(s)) - 10)


def test_quantisation_bound_over_fp16_sums():
    """For sums of fp16 values (a, b): the TwoSum error t is within half a
    last place of s, and the 8-bit word keeps it to 1/256 of a last place,
    on the grid of 1/128 of a last place, with |q| <= 64."""
    rng = np.random.default_rng(51)
    a = rng.normal(size=3000) * 10.0 ** rng.integers(-4, 4, size=3000)
    b = rng.normal(size=3000) * 10.0 ** rng.integers(-7, 1, size=3000)
    a = oracle.round_to(a, "f16")
    b = oracle.round_to(b, "f16")
    checked = 0
    for x, y in zip(a, b):
        s, t = oracle.twosum(float(x), float(y), "f16")
        if not (math.isfinite(s) and math.isfinite(t)):
            continue
        u = _ulp16(s)
        assert abs(t) <= u / 2
        tq = Q(t, s, "f16")
        q = tq / u * 128
        assert q == int(q) and abs(q) <= 64
        assert abs(tq - t) <= u / 256
        checked += 1
    assert checked > 2900


def test_recursive_sum_keeps_the_small_increments():
    """Sec. 4's stagnating sum: adding 2^-13 to 1.0 four thousand times in
    fp16.  Plain fp16 never moves (the increment is below half a last
    place); the 6-op sum with a 16-bit word is exact; with the 8-bit word
    the result is within 1/256 of a last place of the exact sum per step and
    in fact exact here (the increment is a multiple of 1/128 of the last
    place of every partial sum)."""
    inc, n = 2.0 ** -13, 4000
    v = 1.0
    for _ in range(n):
        v = _r16(v + inc)
    assert v == 1.0
    exact = 1.0 + n * inc
    for comp in ("twosum", "twosum8"):
        v, c = 1.0, 0.0
        for _ in range(n):
            y = _r16(inc + c)
            s, t = oracle.twosum(v, y, "f16")
            v, c = s, (Q(t, s, "f16") if comp == "twosum8" else t)
        assert abs((v + c) - exact) <= 2.0 ** -10 / 256, comp


def test_energy_kept_in_the_small_courant_regime():
    """The paper-regime pin of the compensated update, repeated with the
    8-bit word: plain fp16 loses > 2% of the energy over 6000 steps at CFL
    0.0125, the 8-bit-word update stays within 1e-3 of fp64."""
    n = 32
    w = workloads.small2d(n, nsteps=0, order=4, cfl=0.0125, sigma=3.0)
    f = {k: oracle.round_to(v, "f16") for k, v in w.fields().items()}
    args = (n, n, 4, 1.0, w.dt, w.rho, w.kappa, f)
    common = dict(nsteps=6000, energy_every=500)
    _, _, e64 = oracle.acoustic2d(*args, **common)
    _, _, e16 = oracle.acoustic2d(*args, storage="f16", stencil="f32", **common)
    _, _, e8 = oracle.acoustic2d(*args, storage="f16", stencil="f32",
                                 comp="twosum8", **common)
    assert (e16[-1] - e64[0]) / e64[0] < -2e-2
    assert np.max(np.abs(e8 - e64)) / e64[0] < 1e-3


def _native_step8(nx, ny, order, dt, rho, kappa, f, nsteps):
    """The fp16 step with the 8-bit compensation word in numpy: float32
    stencil, float16 TwoSum, quantisation by exponent arithmetic."""
    from oracle import closed_forms
    f32, h = np.float32, np.float16
    w1, w2 = (f32(w) for w in closed_forms.stencil_weights(order, dt, 1.0))
    b = (1.0 / rho).astype(f32)
    k = kappa.astype(f32)

    def sh(a, dj, di):
        return np.roll(a, (-dj, -di), axis=(0, 1))

    def grad(a, axis):
        dj, di = (1, 0) if axis == 0 else (0, 1)
        a0 = sh(a, dj, di) - a
        if order == 2:
            return w1 * a0
        return w1 * a0 + w2 * (sh(a, 2 * dj, 2 * di) - sh(a, -dj, -di))

    def div(a, axis):
        dj, di = (1, 0) if axis == 0 else (0, 1)
        a0 = a - sh(a, -dj, -di)
        if order == 2:
            return w1 * a0
        return w1 * a0 + w2 * (sh(a, dj, di) - sh(a, -2 * dj, -2 * di))

    def ulp(s):
        e = np.floor(np.log2(np.maximum(np.abs(s.astype(np.float64)), 2.0 ** -14)))
        return np.exp2(e - 10)

    def upd(v, c, inc):
        y = (inc + c.astype(f32)).astype(h)
        s = v + y
        pa = s - y
        pb = s - pa
        t = (v - pa) + (y - pb)
        u = ulp(s)
        q = np.rint(t.astype(np.float64) / u * 128.0) + 0.0   # ties to even, no -0
        return s, (q * u / 128.0)

    st = {key: f[key].astype(h) for key in ("vx", "vy", "p")}
    cp = {key: np.zeros(st[key].shape) for key in st}
    for _ in range(nsteps):
        P = st["p"].astype(f32)
        bx = f32(0.5) * (b + sh(b, 0, 1))
        by = f32(0.5) * (b + sh(b, 1, 0))
        st["vx"], cp["vx"] = upd(st["vx"], cp["vx"], bx * grad(P, 1))
        st["vy"], cp["vy"] = upd(st["vy"], cp["vy"], by * grad(P, 0))
        d = div(st["vx"].astype(f32), 1) + div(st["vy"].astype(f32), 0)
        st["p"], cp["p"] = upd(st["p"], cp["p"], k * d)
    return {key: v.astype(np.float64) for key, v in st.items()}, cp


@pytest.mark.parametrize("order", [2, 4])
def test_step_matches_native_evaluation(order):
    nx, ny = 12, 9
    rng = np.random.default_rng(52)
    rho = rng.uniform(1.0, 2.5, size=(ny, nx))
    kappa = rng.uniform(1.0, 6.0, size=(ny, nx))
    f = {"p": oracle.round_to(workloads.gaussian2d(nx, ny, 5, 4, 2.0), "f16"),
         "vx": oracle.round_to(0.05 * rng.normal(size=(ny, nx)), "f16"),
         "vy": oracle.round_to(0.05 * rng.normal(size=(ny, nx)), "f16")}
    want, wantc = _native_step8(nx, ny, order, 0.2, rho, kappa, f, 12)
    got, gotc, _ = oracle.acoustic2d(nx, ny, order, 1.0, 0.2, rho, kappa, f,
                                     storage="f16", stencil="f32", comp="twosum8",
                                     nsteps=12)
    for key in ("vx", "vy", "p"):
        assert np.array_equal(got[key], want[key]), key
        assert np.array_equal(gotc[key], wantc[key]), key
