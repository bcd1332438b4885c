"""The arithmetic identities the GPU kernels' 8-bit compensation encoding
relies on, checked on the CPU for every case they are used in.

For a TwoSum error t of a sum s the word is q = round(t / ulp(s) * 2^7),
ties to even (the word of Sec. 4's cheaper compensation storage, as this
library reads it).  The kernels compute it as
  fp16: x = ldexp(t, 32 - e) in fp16, r = x + 1536 in fp16, q = low byte of r
  bf16: x = ldexp(t, 141 - e) in fp32, r = x + 1.5 * 2^23 in fp32, q = low byte
(e the exponent field of s, at least 1).  Here, for every exponent field and
every value t of the format with |t| <= ulp(s)/2: the fp16 scaling is
exact, and the low byte equals round-half-even of the exact product."""
import numpy as np


def _low_byte(bits):
    return (bits & 0xff).astype(np.uint8).view(np.int8).astype(np.int64)


def test_fp16_encoding_identity():
    allh = np.arange(65536, dtype=np.uint16).view(np.float16)
    fin = allh[np.isfinite(allh)]
    cases = 0
    for field in range(0, 31):
        e = max(field, 1)
        t = fin[np.abs(fin.astype(np.float64)) <= 2.0 ** (e - 26)]   # ulp(s) = 2^(e-25)
        x = np.ldexp(t, 32 - e)
        assert x.dtype == np.float16
        exact = t.astype(np.float64) * 2.0 ** (32 - e)
        assert np.array_equal(x.astype(np.float64), exact), field
        r = (x + np.float16(1536.0)).astype(np.float16)
        q = _low_byte(r.view(np.uint16))
        want = np.rint(exact).astype(np.int64)                       # ties to even
        assert np.array_equal(q, want), field
        assert np.abs(want).max() <= 64
        cases += t.size
    assert cases > 390000


def test_bf16_encoding_identity():
    allb = (np.arange(65536, dtype=np.uint32) << 16).view(np.float32)
    fin = allb[np.isfinite(allb)]
    for field in range(0, 255):
        e = max(field, 1)
        t = fin[np.abs(fin.astype(np.float64)) <= 2.0 ** (e - 135)]  # ulp(s) = 2^(e-134)
        x = np.ldexp(t, 141 - e).astype(np.float32)
        exact = t.astype(np.float64) * 2.0 ** (141 - e)
        r = (x + np.float32(12582912.0)).astype(np.float32)
        q = _low_byte(r.view(np.uint32))
        assert np.array_equal(q, np.rint(exact).astype(np.int64)), field


def _two_sum_error(v, y):
    s = v + y
    pa = s - y
    pb = s - pa
    da = v - pa
    db = y - pb
    return s, da + db


def test_error_of_an_overflowed_sum_is_nan():
    """The kernels test only t for finiteness: the six-operation sum's error
    is NaN whenever s is not finite.  A sum is not finite only if one operand
    is at least 32752 in magnitude or not finite; every fp16 pair with such
    an operand (in either place) is checked."""
    allh = np.arange(65536, dtype=np.uint16).view(np.float16)
    with np.errstate(all="ignore"):
        large = allh[~(np.abs(allh.astype(np.float64)) < 32752.0)]       # includes inf, NaN
        n = 0
        for a in large:
            for v, y in ((np.float16(a), allh), (allh, np.float16(a))):
                s, t = _two_sum_error(v, y)
                bad = ~np.isfinite(s)
                assert np.all(np.isnan(t[bad]))
                n += int(bad.sum())
    assert n > 10 ** 6
