"""Reference oracle for staggered-grid leapfrog wave propagation.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The GPU library never
calls into it, and it shares no code with the GPU library.

The solver lives in ``oracle.c`` (plain C, fp64 evaluation with explicit
rounding after every operation to emulate fp32/fp16/bf16 arithmetic); this
module builds it with gcc, loads it with ctypes and wraps it for numpy.  The
closed-form solutions are in ``closed_forms.py`` and the dense-operator
construction in ``brute.py``.

Formats: 'f64', 'f32', 'f16', 'bf16'.  Compensation: 'none', 'fast2sum'
(Sec. 4, Code 1, three operations), 'twosum' (Sec. 4, Code 2, six operations).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# AddressSanitizer + UndefinedBehaviorSanitizer build of the same source,
# loaded instead when ORACLE_SANITIZE=1 (the process must preload the
# sanitizer runtimes, see sanitizer_env())
_LIB_SAN = os.path.join(_HERE, "liboracle_san.so")
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined"]

FORMATS = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
COMPS = {"none": 0, "fast2sum": 1, "twosum": 2, "twosum8": 3}
ELASTIC_FIELDS = ("vx", "vy", "vz", "sxx", "syy", "szz", "sxy", "sxz", "syz")
ACOUSTIC_FIELDS = ("vx", "vy", "p")
ELASTIC2D_FIELDS = ("vx", "vy", "sxx", "syy", "sxy")

# The compile line is part of the oracle's definition: no contraction of
# a*b+c into fused multiply-adds, no fast-math value changes.
CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-fPIC", "-shared", "-std=c11"]


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile oracle.c into liboracle.so next to it (liboracle_san.so with
    the sanitizers) and return the path."""
    out = _LIB_SAN if sanitize else _LIB
    flags = [f for f in CFLAGS if f != "-O2"] + SAN_FLAGS if sanitize else CFLAGS
    if force or not os.path.exists(out) or \
            os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *flags, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, out)
    return out


def sanitizer_env() -> dict:
    """Environment for a child process that loads the sanitized oracle: the
    ASan and UBSan runtimes preloaded (the Python interpreter itself is not
    instrumented), leak checks off (the interpreter's own allocations)."""
    def rt(name):
        return subprocess.check_output(["gcc", f"-print-file-name={name}"],
                                       text=True).strip()
    env = dict(os.environ)
    env.update({"ORACLE_SANITIZE": "1",
                "LD_PRELOAD": f"{rt('libasan.so')}:{rt('libubsan.so')}",
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
    return env


_lib = None


def lib():
    global _lib
    if _lib is None:
        san = os.environ.get("ORACLE_SANITIZE") == "1"
        L = ctypes.CDLL(build(force=False, sanitize=san))
        D = ctypes.c_double
        Lg = ctypes.c_long
        I = ctypes.c_int
        P = ctypes.POINTER(ctypes.c_double)
        PP = ctypes.POINTER(P)
        L.orc_round.restype = D
        L.orc_round.argtypes = [D, I]
        L.orc_round_array.restype = None
        L.orc_round_array.argtypes = [P, P, Lg, I]
        L.orc_fast2sum.restype = None
        L.orc_fast2sum.argtypes = [D, D, I, P, P]
        L.orc_twosum.restype = None
        L.orc_twosum.argtypes = [D, D, I, P, P]
        L.orc_eft_check.restype = Lg
        L.orc_eft_check.argtypes = [I, I, P, Lg, P, Lg, I]
        L.orc_eft_exhaustive.restype = None
        L.orc_eft_exhaustive.argtypes = [I, Lg, Lg, ctypes.POINTER(ctypes.c_long)]
        L.orc_quantize_comp.restype = D
        L.orc_quantize_comp.argtypes = [D, D, I]
        L.orc_max_threads.restype = I
        L.orc_max_threads.argtypes = []
        L.orc_acoustic2d.restype = I
        PL = ctypes.POINTER(ctypes.c_long)
        L.orc_acoustic2d.argtypes = [Lg, Lg, I, D, D, P, P, P, P, P, P, P, P,
                                     I, I, I, Lg, Lg, P, I,
                                     Lg, Lg, P, Lg, Lg, PL, PL, P]
        L.orc_acoustic2d_energy.restype = D
        L.orc_acoustic2d_energy.argtypes = [Lg, Lg, I, D, D, P, P, P, P, P]
        L.orc_elastic3d.restype = I
        L.orc_elastic3d.argtypes = [Lg, Lg, Lg, D, D, P, P, P, PP, PP,
                                    I, I, I, Lg, Lg, P, I]
        L.orc_elastic3d_energy.restype = D
        L.orc_elastic3d_energy.argtypes = [Lg, Lg, Lg, D, D, P, P, P, PP]
        L.orc_elastic2d.restype = I
        L.orc_elastic2d.argtypes = [Lg, Lg, D, D, P, P, P, PP, PP, I, I, I,
                                    Lg, Lg, P, I, Lg, Lg, P, Lg, Lg, PL, PL, P]
        L.orc_elastic2d_energy.restype = D
        L.orc_elastic2d_energy.argtypes = [Lg, Lg, D, D, P, P, P, PP]
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if a.shape != shape:
        a = np.ascontiguousarray(np.broadcast_to(a, shape), dtype=np.float64)
    return a


def max_threads() -> int:
    return int(lib().orc_max_threads())


# ---------------------------------------------------------------- formats --

def round_to(x, fmt: str) -> np.ndarray:
    """Round each value to the nearest value of `fmt` (ties to even)."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    y = np.empty_like(x)
    lib().orc_round_array(_ptr(x), _ptr(y), x.size, FORMATS[fmt])
    return y


def fast2sum(a: float, b: float, fmt: str):
    s, t = ctypes.c_double(), ctypes.c_double()
    lib().orc_fast2sum(a, b, FORMATS[fmt], ctypes.byref(s), ctypes.byref(t))
    return s.value, t.value


def twosum(a: float, b: float, fmt: str):
    s, t = ctypes.c_double(), ctypes.c_double()
    lib().orc_twosum(a, b, FORMATS[fmt], ctypes.byref(s), ctypes.byref(t))
    return s.value, t.value


def eft_check(fmt: str, which: int, a, b, require_order: bool) -> int:
    """Number of pairs (a_i, b_j) whose compensated sum is not error free."""
    a = _f64(a, np.shape(a))
    b = _f64(b, np.shape(b))
    return int(lib().orc_eft_check(FORMATS[fmt], which, _ptr(a), a.size,
                                   _ptr(b), b.size, int(require_order)))


EFT_COUNTS = ("pairs", "twosum_not_exact", "twosum_overflow", "ordered_pairs",
              "fast2sum_ordered_not_exact", "fast2sum_ordered_overflow",
              "fast2sum_unordered_not_exact", "sum_overflow")


def eft_exhaustive(fmt: str, a_lo: int = 0, a_hi: int = 1 << 16) -> dict:
    """Exactness of both compensated sums over every pair of finite values
    of a 16-bit format ('f16' or 'bf16') whose first operand's bit pattern
    lies in [a_lo, a_hi) (see orc_eft_exhaustive for the counts)."""
    out = (ctypes.c_long * 8)()
    lib().orc_eft_exhaustive(FORMATS[fmt], a_lo, a_hi, out)
    return dict(zip(EFT_COUNTS, list(out)))


# ---------------------------------------------------------------- solvers --

def acoustic2d(nx, ny, order, dx, dt, rho, kappa, fields, *, storage="f64",
               stencil="f64", comp="none", comps=None, nsteps=0,
               energy_every=0, nthreads=0, source=None, receivers=None):
    """Advance the 2D acoustic system (Eq. 1) by nsteps leapfrog steps.

    fields: dict with 'vx', 'vy', 'p' ([ny, nx] arrays holding values of the
    storage format, state (v^{n-1/2}, p^n)); comps: same keys for the
    compensation terms (zeros if None).  rho, kappa at p points.
    source: (ix, iy, samples) -- a point source on the pressure (the s_p
    term of Eq. 1): step n of this call adds samples[n] (rounded to the
    stencil format) to the pressure right-hand side at cell (ix, iy) before
    the division by beta, for n < len(samples).
    receivers: list of (ix, iy) cells; after step n, trace[n, r] holds
    (p^{n+1}, vx^{n+1/2}, vy^{n+1/2}) at cell r.
    Returns (fields, comps, energy) with energy[m] = E at step
    m*energy_every, plus the receiver trace [nsteps, nrec, 3] when receivers
    are given.
    """
    shape = (ny, nx)
    rho = _f64(rho, shape)
    kappa = _f64(kappa, shape)
    f = {k: _f64(fields[k], shape).copy() for k in ACOUSTIC_FIELDS}
    if comp != "none":
        c = {k: (_f64(comps[k], shape).copy() if comps is not None
                 else np.zeros(shape)) for k in ACOUSTIC_FIELDS}
    else:
        c = {k: None for k in ACOUSTIC_FIELDS}
    ne = nsteps // energy_every + 1 if energy_every > 0 else 0
    energy = np.zeros(max(ne, 1))
    sx, sy, samples = (0, 0, np.zeros(1)) if source is None else source
    samples = np.ascontiguousarray(samples, dtype=np.float64)
    nsrc = 0 if source is None else len(samples)
    rec = [] if receivers is None else list(receivers)
    PL = ctypes.POINTER(ctypes.c_long)
    rx = np.ascontiguousarray([r[0] for r in rec] or [0], dtype=np.int64)
    ry = np.ascontiguousarray([r[1] for r in rec] or [0], dtype=np.int64)
    trace = np.zeros((max(nsteps, 1), max(len(rec), 1), 3))
    rc = lib().orc_acoustic2d(nx, ny, order, dx, dt, _ptr(rho), _ptr(kappa),
                              _ptr(f["vx"]), _ptr(f["vy"]), _ptr(f["p"]),
                              _ptr(c["vx"]), _ptr(c["vy"]), _ptr(c["p"]),
                              FORMATS[storage], FORMATS[stencil], COMPS[comp],
                              nsteps, energy_every, _ptr(energy), nthreads,
                              int(sx), int(sy), _ptr(samples), nsrc, len(rec),
                              rx.ctypes.data_as(PL), ry.ctypes.data_as(PL),
                              _ptr(trace))
    if rc != 0:
        raise ValueError("oracle rejected the acoustic2d arguments")
    if receivers is not None:
        return f, c, energy[:ne], trace[:nsteps, :len(rec)]
    return f, c, energy[:ne]


def acoustic2d_energy(nx, ny, order, dx, dt, rho, kappa, fields) -> float:
    shape = (ny, nx)
    rho = _f64(rho, shape)
    kappa = _f64(kappa, shape)
    f = {k: _f64(fields[k], shape) for k in ACOUSTIC_FIELDS}
    return float(lib().orc_acoustic2d_energy(
        nx, ny, order, dx, dt, _ptr(rho), _ptr(kappa), _ptr(f["vx"]),
        _ptr(f["vy"]), _ptr(f["p"])))


def _ptr_array(arrs):
    P = ctypes.POINTER(ctypes.c_double)
    return (P * len(arrs))(*[_ptr(a) for a in arrs])


def elastic3d(nx, ny, nz, dx, dt, rho, lam, mu, fields, *, storage="f64",
              stencil="f64", comp="none", comps=None, nsteps=0,
              energy_every=0, nthreads=0):
    """Advance the 3D velocity-stress system by nsteps leapfrog steps.

    fields: dict keyed by ELASTIC_FIELDS, [nz, ny, nx] arrays; material rho,
    lambda, mu at cell centres.  Returns (fields, comps, energy).
    """
    shape = (nz, ny, nx)
    rho, lam, mu = (_f64(a, shape) for a in (rho, lam, mu))
    f = {k: _f64(fields[k], shape).copy() for k in ELASTIC_FIELDS}
    if comp != "none":
        c = {k: (_f64(comps[k], shape).copy() if comps is not None
                 else np.zeros(shape)) for k in ELASTIC_FIELDS}
        cptr = _ptr_array([c[k] for k in ELASTIC_FIELDS])
    else:
        c = {k: None for k in ELASTIC_FIELDS}
        cptr = None
    fptr = _ptr_array([f[k] for k in ELASTIC_FIELDS])
    ne = nsteps // energy_every + 1 if energy_every > 0 else 0
    energy = np.zeros(max(ne, 1))
    rc = lib().orc_elastic3d(nx, ny, nz, dx, dt, _ptr(rho), _ptr(lam),
                             _ptr(mu), fptr, cptr, FORMATS[storage],
                             FORMATS[stencil], COMPS[comp], nsteps,
                             energy_every, _ptr(energy), nthreads)
    if rc != 0:
        raise ValueError("oracle rejected the elastic3d arguments")
    return f, c, energy[:ne]


def elastic3d_energy(nx, ny, nz, dx, dt, rho, lam, mu, fields) -> float:
    shape = (nz, ny, nx)
    rho, lam, mu = (_f64(a, shape) for a in (rho, lam, mu))
    f = {k: _f64(fields[k], shape) for k in ELASTIC_FIELDS}
    return float(lib().orc_elastic3d_energy(
        nx, ny, nz, dx, dt, _ptr(rho), _ptr(lam), _ptr(mu),
        _ptr_array([f[k] for k in ELASTIC_FIELDS])))


def elastic2d(nx, ny, dx, dt, rho, lam, mu, fields, *, storage="f64",
              stencil="f64", comp="none", comps=None, nsteps=0,
              energy_every=0, nthreads=0, source=None, receivers=None):
    """Advance the 2D velocity-stress system of Eq. (A1), App. A (periodic
    in x, free surfaces on rows 0 and ny-1) by nsteps leapfrog steps.

    fields: dict keyed by ELASTIC2D_FIELDS, [ny, nx] arrays (syy zero on
    both surface rows, vy and sxy zero on row ny-1); material rho, lambda,
    mu at cells.  source: (ix, iy, samples) -- step n of this call adds
    samples[n] (rounded to the stencil format) to vy at (ix, iy + 1/2)
    after the division by rho.  receivers: list of (ix, iy) cells; after
    step n, trace[n, r] holds the five fields there.  Returns (fields,
    comps, energy), plus the trace [nsteps, nrec, 5] when receivers are
    given.
    """
    shape = (ny, nx)
    rho, lam, mu = (_f64(a, shape) for a in (rho, lam, mu))
    f = {k: _f64(fields[k], shape).copy() for k in ELASTIC2D_FIELDS}
    if comp != "none":
        c = {k: (_f64(comps[k], shape).copy() if comps is not None
                 else np.zeros(shape)) for k in ELASTIC2D_FIELDS}
        cptr = _ptr_array([c[k] for k in ELASTIC2D_FIELDS])
    else:
        c = {k: None for k in ELASTIC2D_FIELDS}
        cptr = None
    fptr = _ptr_array([f[k] for k in ELASTIC2D_FIELDS])
    ne = nsteps // energy_every + 1 if energy_every > 0 else 0
    energy = np.zeros(max(ne, 1))
    sx, sy, samples = (0, 0, np.zeros(1)) if source is None else source
    samples = np.ascontiguousarray(samples, dtype=np.float64)
    nsrc = 0 if source is None else len(samples)
    rec = [] if receivers is None else list(receivers)
    PL = ctypes.POINTER(ctypes.c_long)
    rx = np.ascontiguousarray([r[0] for r in rec] or [0], dtype=np.int64)
    ry = np.ascontiguousarray([r[1] for r in rec] or [0], dtype=np.int64)
    nf = len(ELASTIC2D_FIELDS)
    trace = np.zeros((max(nsteps, 1), max(len(rec), 1), nf))
    rc = lib().orc_elastic2d(nx, ny, dx, dt, _ptr(rho), _ptr(lam), _ptr(mu),
                             fptr, cptr, FORMATS[storage], FORMATS[stencil],
                             COMPS[comp], nsteps, energy_every, _ptr(energy),
                             nthreads, int(sx), int(sy), _ptr(samples), nsrc,
                             len(rec), rx.ctypes.data_as(PL),
                             ry.ctypes.data_as(PL), _ptr(trace))
    if rc != 0:
        raise ValueError("oracle rejected the elastic2d arguments")
    if receivers is not None:
        return f, c, energy[:ne], trace[:nsteps, :len(rec)]
    return f, c, energy[:ne]


def elastic2d_energy(nx, ny, dx, dt, rho, lam, mu, fields) -> float:
    shape = (ny, nx)
    rho, lam, mu = (_f64(a, shape) for a in (rho, lam, mu))
    f = {k: _f64(fields[k], shape) for k in ELASTIC2D_FIELDS}
    return float(lib().orc_elastic2d_energy(
        nx, ny, dx, dt, _ptr(rho), _ptr(lam), _ptr(mu),
        _ptr_array([f[k] for k in ELASTIC2D_FIELDS])))


def quantize_comp(t: float, s: float, fmt: str) -> float:
    """The compensation term t of the sum s as an 8-bit word holds it:
    round(t / ulp(s) * 2^7) * ulp(s) / 2^7 (see orc_quantize_comp)."""
    return float(lib().orc_quantize_comp(float(t), float(s), FORMATS[fmt]))
