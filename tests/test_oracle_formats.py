"""Pins of the oracle's rounding and compensated sums (Sec. 2 and Sec. 4).

The rounding routine is checked against the paper's Table 1, against numpy's
own IEEE conversions, against a bit-level round-to-nearest-even written here,
and against exact rational arithmetic.  The compensated sums are checked for
exactness over large structured samples, against the same algorithm run with
numpy's native fp16 arithmetic, and on the stagnating recursive sum that
motivates them.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_formats.json")
PARAMS = {"f32": (24, -126, 127), "f16": (11, -14, 15), "bf16": (8, -126, 127)}


def rn(x, fmt):
    return float(oracle.round_to(np.array([x]), fmt)[0])


def _sig(x, digits=5):
    return float(f"{x:.{digits - 1}e}")


@pytest.mark.parametrize("fmt", ["f32", "f16"])
def test_table1_constants(fmt):
    """Unit roundoff, largest, smallest normal and subnormal of Table 1 are
    recovered from the rounding routine's behaviour."""
    ref = json.load(open(GOLDEN))["formats"][fmt]
    p, emin, emax = PARAMS[fmt]
    u = 2.0 ** -p
    # unit roundoff: 1 + u is a tie and rounds to 1; anything above rounds up
    assert rn(1.0 + u, fmt) == 1.0
    assert rn(1.0 + u * (1 + 2 ** -20), fmt) == 1.0 + 2 * u
    assert _sig(u) == ref["unit_roundoff"]
    ulp_top = 2.0 ** (emax - p + 1)
    largest = rn(2.0 ** (emax + 1) - ulp_top + ulp_top / 4, fmt)
    assert largest == 2.0 ** (emax + 1) - ulp_top
    assert rn(largest + ulp_top * 0.499, fmt) == largest
    assert math.isinf(rn(largest + ulp_top / 2, fmt))         # tie -> inf
    assert _sig(largest) == ref["largest"]
    smallest_normal = 2.0 ** emin
    assert rn(smallest_normal, fmt) == smallest_normal
    assert _sig(smallest_normal) == ref["smallest_normal"]
    sub = 2.0 ** (emin - p + 1)
    assert rn(sub * 0.5, fmt) == 0.0                # tie to even (zero)
    assert rn(sub * 0.5000001, fmt) == sub
    assert rn(sub * 1.5, fmt) == 2 * sub            # tie to even
    assert _sig(sub) == ref["smallest_subnormal"]
    assert ref["fraction_bits"] == p


def test_table1_f64_is_identity():
    ref = json.load(open(GOLDEN))["formats"]["f64"]
    assert _sig(2.0 ** -53) == ref["unit_roundoff"]
    x = np.random.default_rng(1).normal(size=1000)
    assert np.array_equal(oracle.round_to(x, "f64"), x)


def _random_doubles(rng, n, lo_exp, hi_exp):
    mant = rng.uniform(1.0, 2.0, size=n)
    exps = rng.integers(lo_exp, hi_exp, size=n)
    sign = rng.choice([-1.0, 1.0], size=n)
    return sign * np.ldexp(mant, exps)


def _ties(rng, n, p, lo_exp, hi_exp):
    """Exact midpoints between neighbouring p-bit numbers."""
    m = rng.integers(2 ** (p - 1), 2 ** p, size=n).astype(np.float64)
    e = rng.integers(lo_exp, hi_exp, size=n)
    return np.ldexp(m + 0.5, e - (p - 1))


def test_f16_matches_numpy_conversion():
    rng = np.random.default_rng(2)
    x = np.concatenate([_random_doubles(rng, 200000, -30, 17),
                        _ties(rng, 20000, 11, -14, 15),
                        _ties(rng, 20000, 11, -24, -14),   # subnormal midpoints
                        np.array([0.0, -0.0, 65504.0, 65519.99, 65520.0, -65520.0])])
    ref = x.astype(np.float16).astype(np.float64)
    got = oracle.round_to(x, "f16")
    assert np.array_equal(np.signbit(got), np.signbit(ref))
    assert np.array_equal(got, ref)


def test_f32_matches_numpy_conversion():
    rng = np.random.default_rng(3)
    x = np.concatenate([_random_doubles(rng, 200000, -160, 128),
                        _ties(rng, 20000, 24, -126, 127)])
    ref = x.astype(np.float32).astype(np.float64)
    with np.errstate(over="ignore"):
        got = oracle.round_to(x, "f32")
    assert np.array_equal(got, ref)


def _bf16_bits_rne(x32: np.ndarray) -> np.ndarray:
    """Round float32 values to bf16 by integer round-to-nearest-even on the
    bit pattern (keep the top 16 bits)."""
    u = x32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def test_bf16_matches_bit_level_rounding():
    rng = np.random.default_rng(4)
    bits = rng.integers(0, 0x7F800000, size=400000, dtype=np.uint32)
    x32 = bits.view(np.float32) * rng.choice(np.float32([-1, 1]), size=bits.size)
    ref = _bf16_bits_rne(x32)
    got = oracle.round_to(x32.astype(np.float64), "bf16")
    assert np.array_equal(got, ref)


def _exact_round(x: float, p: int, emin: int, emax: int) -> float:
    """Nearest p-bit number to x by exact rational comparison, ties to even."""
    q = Fraction(x)
    if q == 0:
        return x
    sign = -1 if q < 0 else 1
    a = abs(q)
    e = math.floor(math.log2(a))
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, emin)
    quantum = Fraction(2) ** (e - p + 1)
    lo = (a / quantum).__floor__()
    rem = a / quantum - lo
    n = lo + (1 if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and lo % 2) else 0)
    r = n * quantum
    if r > (2 - Fraction(2) ** (1 - p)) * Fraction(2) ** emax:
        return sign * math.inf
    return sign * float(r)


@pytest.mark.parametrize("fmt", ["f32", "f16", "bf16"])
def test_rounding_matches_exact_rationals(fmt):
    p, emin, emax = PARAMS[fmt]
    rng = np.random.default_rng(5)
    x = np.concatenate([_random_doubles(rng, 3000, emin - p - 2, emax + 1),
                        _ties(rng, 1000, p, emin - p + 1, emax)])
    got = oracle.round_to(x, fmt)
    for xi, gi in zip(x, got):
        assert gi == _exact_round(float(xi), p, emin, emax), (xi, gi)


# ------------------------------------------------------- compensated sums --

def _all_finite_f16():
    v = np.arange(0, 0x10000, dtype=np.uint16).view(np.float16)
    return v[np.isfinite(v)].astype(np.float64)


def test_twosum_error_free_f16():
    """Code 2 (6 ops) is error free for every ordering: all finite fp16 a
    against a structured sample of b (every 128th bit pattern, both signs)."""
    a = _all_finite_f16()
    b = a[::128]
    assert oracle.eft_check("f16", 6, a, b, require_order=False) == 0


def test_twosum_overflow_edge_f16():
    """At the top of the fp16 range an intermediate of Code 2 can overflow
    even though the sum itself is finite (Sec. 5 warns about range): the
    split is then not finite, and the exactness check skips such pairs."""
    s, t = oracle.twosum(65504.0, -48.0, "f16")
    assert s == 65472.0 and math.isnan(t)
    a = _all_finite_f16()
    assert oracle.eft_check("f16", 6, a[np.abs(a) < 32768], a[::128],
                            require_order=False) == 0


def test_fast2sum_error_free_when_ordered_f16():
    """Code 1 (3 ops) is error free when |a| >= |b| (Sec. 4) ..."""
    a = _all_finite_f16()
    b = a[::97]
    assert oracle.eft_check("f16", 3, a, b, require_order=True) == 0


def test_fast2sum_not_error_free_when_unordered_f16():
    """... and not in general when |a| < |b|."""
    a = _all_finite_f16()[::31]
    b = _all_finite_f16()[::29]
    assert oracle.eft_check("f16", 3, a, b, require_order=False) > 0


@pytest.mark.parametrize("fmt", ["bf16", "f32"])
def test_compensated_sums_error_free_sampled(fmt):
    p, emin, emax = PARAMS[fmt]
    rng = np.random.default_rng(6)
    a = oracle.round_to(_random_doubles(rng, 3000, emin - p + 2, emax - 1), fmt)
    b = oracle.round_to(np.concatenate([
        _random_doubles(rng, 300, emin - p + 2, emax - 1),
        a[:300] * 2.0 ** -7, a[:300] * 3.0]), fmt)
    assert oracle.eft_check(fmt, 6, a, b, require_order=False) == 0
    assert oracle.eft_check(fmt, 3, a, b, require_order=True) == 0


def _sum_6op_numpy(a, b):
    a, b = np.float16(a), np.float16(b)
    s = a + b
    pa = s - b
    pb = s - pa
    da = a - pa
    db = b - pb
    return s, da + db


def _sum_3op_numpy(a, b):
    a, b = np.float16(a), np.float16(b)
    s = a + b
    z = s - a
    return s, b - z


def test_compensated_sums_match_native_f16_arithmetic():
    """Same op sequences evaluated with numpy's native fp16 arithmetic give
    the same bits as the oracle's emulated fp16."""
    rng = np.random.default_rng(7)
    vals = _all_finite_f16()
    a = rng.choice(vals, size=4000)
    b = rng.choice(vals, size=4000)
    with np.errstate(over="ignore", invalid="ignore"):
        for x, y in zip(a, b):
            for mine, theirs in ((oracle.twosum, _sum_6op_numpy),
                                 (oracle.fast2sum, _sum_3op_numpy)):
                s, t = mine(float(x), float(y), "f16")
                s2, t2 = theirs(x, y)
                if not np.isfinite(s2):
                    continue
                assert (s, t) == (float(s2), float(t2)), (x, y)
                assert math.copysign(1, t) == math.copysign(1, float(t2))


def test_recursive_sum_stagnation_and_compensation():
    """The solution update is a recursive sum (Sec. 4).  Adding delta = 2^-12
    repeatedly in fp16 stagnates exactly where delta drops to half an ulp of
    the running sum (at 2^-1, where the ulp is 2^-11 and the tie rounds to
    even); the compensated recursion tracks the exact sum N*delta to within
    an ulp."""
    delta = 2.0 ** -12
    n = 6000
    s_plain = 0.0
    s, c = 0.0, 0.0
    for _ in range(n):
        s_plain = rn(s_plain + delta, "f16")
        y = rn(delta + c, "f16")
        s, c = oracle.twosum(s, y, "f16")
    assert s_plain == 0.5
    exact = n * delta
    assert abs(s - exact) <= 2.0 ** -10      # one ulp at [1, 2)
    assert abs((s + c) - exact) <= 2.0 ** -22


# ------------------------------------------- exhaustive compensated sums --

EFT_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "eft_exhaustive.json")


@pytest.mark.parametrize("fmt,finite", [("f16", 65536 - 2 * 1024), ("bf16", 65536 - 2 * 128)])
def test_compensated_sums_exhaustive_record(fmt, finite):
    """Every pair of finite fp16 values and every pair of finite bf16 values
    (2^32 pairs less the non-finite ones), run by make_eft_exhaustive.py:
    the 6-operation sum (Code 2) is error free on every pair whose
    operations stay finite, the 3-operation sum (Code 1) on every such
    ordered pair |a| >= |b| (Sec. 4), and it fails on some unordered ones.
    Pairs where an operation overflows are counted apart."""
    rec = json.load(open(EFT_GOLDEN))[fmt]
    assert rec["pairs"] == finite * finite
    assert rec["twosum_not_exact"] == 0
    assert rec["fast2sum_ordered_not_exact"] == 0
    assert rec["fast2sum_unordered_not_exact"] > 0
    assert rec["ordered_pairs"] > finite * finite // 2 - finite
    # overflow only near the top of the range: a small share of the pairs
    assert 0 < rec["twosum_overflow"] < 1e-2 * rec["pairs"]
    assert rec["sum_overflow"] <= rec["twosum_overflow"]


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
def test_compensated_sums_exhaustive_slices(fmt):
    """The same check re-run on slices of first operands (every second
    operand): around 1, the subnormals, the largest values (overflow), and
    negative numbers; the slices' counts are consistent with the record."""
    one = 0x3C00 if fmt == "f16" else 0x3F80
    top = 0x7BFF if fmt == "f16" else 0x7F7F
    total = {k: 0 for k in oracle.EFT_COUNTS}
    for lo, hi in [(one - 32, one + 32), (0, 48), (top - 16, top + 1),
                   (0x8000 | one, (0x8000 | one) + 16)]:
        c = oracle.eft_exhaustive(fmt, lo, hi)
        assert c["twosum_not_exact"] == 0 and c["fast2sum_ordered_not_exact"] == 0
        for k in total:
            total[k] += c[k]
    assert total["twosum_overflow"] > 0 and total["fast2sum_unordered_not_exact"] > 0
    rec = json.load(open(EFT_GOLDEN))[fmt]
    assert total["twosum_overflow"] <= rec["twosum_overflow"]
