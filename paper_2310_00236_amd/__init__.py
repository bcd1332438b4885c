"""Python binding of libhalfwave (the C ABI declared in include/halfwave.h).

Staggered-grid leapfrog wave propagation on an MI355X with fp32/fp16/bf16
state and compensated updates (Gao & Harms, "Half precision wave
simulation").  Every step of the computation runs in the library's HIP
kernels; this module only marshals arguments.  PyTorch supplies the device
memory (one uint8 tensor per plan, the arena) and the stream.

There is no fallback: if the library is not built, importing the binding's
entry points raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhalfwave.so")

ACOUSTIC2D, ELASTIC3D, ELASTIC2D = 0, 1, 2
PHYSICS = {"acoustic2d": ACOUSTIC2D, "elastic3d": ELASTIC3D, "elastic2d": ELASTIC2D}
STORAGE = {"f32": 0, "f16": 1, "bf16": 2}
COMP = {"none": 0, "fast2sum": 1, "twosum": 2, "twosum8": 3}
STENCIL = {"f32": 0, "storage": 1, "f64": 2}
ACOUSTIC_FIELDS = ("vx", "vy", "p")
ELASTIC_FIELDS = ("vx", "vy", "vz", "sxx", "syy", "szz", "sxy", "sxz", "syz")
ELASTIC2D_FIELDS = ("vx", "vy", "sxx", "syy", "sxy")
STATUS = {0: "HW_OK", 1: "HW_E_INVAL", 2: "HW_E_UNSTABLE", 3: "HW_E_RANGE",
          4: "HW_E_NOMEM", 5: "HW_E_DEVICE", 6: "HW_E_NONFINITE",
          7: "HW_E_STATE"}
ABI_VERSION = 6
NOALLOC_MAX_BYTES = 64 << 20      # HW_NOALLOC_MAX_BYTES


class HalfwaveError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__(f"{self.name}: {message}")


class _Problem(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_uint32), ("physics", ctypes.c_int32),
                ("order", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("comp", ctypes.c_int32), ("scale_log2", ctypes.c_int32),
                ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("nz", ctypes.c_int64), ("dx", ctypes.c_double),
                ("dt", ctypes.c_double), ("trace_cap", ctypes.c_int64),
                ("src_cap", ctypes.c_int64), ("rec_cap", ctypes.c_int32),
                ("stencil", ctypes.c_int32), ("rec_steps", ctypes.c_int64)]


_lib = None


def lib():
    """The loaded libhalfwave.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is not built; run `python -m paper_2310_00236_amd.build`")
    # torch must be loaded first: its HIP runtime then satisfies the
    # library's libamdhip64 dependency, so device memory and streams from
    # torch and the library's launches live in one runtime.  Loading the
    # library first would bring in a second HIP runtime in this process.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I32, I64, U32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    D = ctypes.c_double
    PD = ctypes.POINTER(ctypes.c_double)
    PPD = ctypes.POINTER(PD)
    PI64 = ctypes.POINTER(ctypes.c_int64)
    PPlan = ctypes.c_void_p
    PProb = ctypes.POINTER(_Problem)
    sig = {
        "hw_abi_version": (U32, []),
        "hw_last_error": (ctypes.c_char_p, []),
        "hw_num_fields": (I32, [I32]),
        "hw_num_materials": (I32, [I32]),
        "hw_footprint": (I32, [PProb, ctypes.POINTER(ctypes.c_size_t)]),
        "hw_cfl_bound": (D, [I32, I32]),
        "hw_plan_create": (I32, [PProb, P, ctypes.c_size_t, ctypes.POINTER(P)]),
        "hw_plan_destroy": (None, [PPlan]),
        "hw_set_material": (I32, [PPlan, PPD, P]),
        "hw_set_fields": (I32, [PPlan, PPD, P]),
        "hw_advance": (I32, [PPlan, I64, I64, P]),
        "hw_record_energy": (I32, [PPlan, P]),
        "hw_energy_trace": (I32, [PPlan, PD, PI64, I64, PI64, P]),
        "hw_get_fields": (I32, [PPlan, PPD, PPD, P]),
        "hw_plan_step": (I64, [PPlan]),
        "hw_state_size": (I32, [PPlan, ctypes.POINTER(ctypes.c_size_t)]),
        "hw_state_export": (I32, [PPlan, P, ctypes.c_size_t, P]),
        "hw_state_import": (I32, [PPlan, P, ctypes.c_size_t, P]),
        "hw_tile_count": (I32, [I32]),
        "hw_tile_info": (I32, [I32, I32, ctypes.POINTER(I32), ctypes.POINTER(I32),
                               ctypes.POINTER(I32), ctypes.POINTER(I32)]),
        "hw_plan_set_tile": (I32, [PPlan, I32]),
        "hw_set_source": (I32, [PPlan, I64, I64, PD, I64, P]),
        "hw_set_receivers": (I32, [PPlan, I32, PI64, PI64, P]),
        "hw_receiver_trace": (I32, [PPlan, PD, I64, PI64, P]),
        "hw_batch_advance": (I32, [ctypes.POINTER(P), I32, PI64, I64, I32, P]),
        "hw_simulate": (I32, [PProb, PPD, PPD, I64, I64, PD, I64, PI64, P,
                              ctypes.c_size_t, P]),
        "hw_simulate_noalloc": (I32, [PProb, PPD, PPD, I64, I64, PD, I64, PI64, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    if L.hw_abi_version() != ABI_VERSION:
        raise RuntimeError("libhalfwave ABI version mismatch")
    _lib = L
    return L


def _check(status: int):
    if status != 0:
        raise HalfwaveError(status, lib().hw_last_error().decode())


def _stream_handle(stream, device):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


def _f64_ptrs(arrays, n, shape, allow_none):
    keep = []
    ptrs = (ctypes.POINTER(ctypes.c_double) * n)()
    for i in range(n):
        a = arrays[i] if i < len(arrays) else None
        if a is None:
            if not allow_none:
                raise ValueError("array %d is missing" % i)
            ptrs[i] = ctypes.POINTER(ctypes.c_double)()
            continue
        a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
        if a.shape != shape:
            a = np.ascontiguousarray(np.broadcast_to(a, shape), dtype=np.float64)
        keep.append(a)
        ptrs[i] = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return ptrs, keep


@dataclass
class Problem:
    """Mirror of hw_problem (see include/halfwave.h)."""
    physics: str                  # 'acoustic2d', 'elastic3d' or 'elastic2d'
    nx: int
    ny: int
    nz: int = 1
    order: int = 2
    storage: str = "f32"          # 'f32', 'f16', 'bf16'
    comp: str = "none"            # 'none', 'fast2sum', 'twosum'
    dx: float = 1.0
    dt: float = 0.5
    scale_log2: int = 0
    trace_cap: int = 0
    src_cap: int = 0              # point-source samples reserved (2D)
    rec_cap: int = 0              # receivers reserved (2D, <= 64)
    rec_steps: int = 0            # receiver trace rows reserved
    stencil: str = "f32"          # stencil precision: 'f32', 'storage', 'f64'

    def c(self) -> _Problem:
        return _Problem(ABI_VERSION,
                        PHYSICS[self.physics],
                        self.order, STORAGE[self.storage], COMP[self.comp],
                        self.scale_log2, self.nx, self.ny, self.nz, self.dx,
                        self.dt, self.trace_cap, self.src_cap, self.rec_cap,
                        STENCIL[self.stencil], self.rec_steps)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx) if self.physics == "elastic3d" else \
            (self.ny, self.nx)

    @property
    def field_names(self):
        return {"acoustic2d": ACOUSTIC_FIELDS, "elastic3d": ELASTIC_FIELDS,
                "elastic2d": ELASTIC2D_FIELDS}[self.physics]

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz


def footprint(pb: Problem) -> int:
    n = ctypes.c_size_t()
    _check(lib().hw_footprint(ctypes.byref(pb.c()), ctypes.byref(n)))
    return n.value


def cfl_bound(physics: str, order: int) -> float:
    return lib().hw_cfl_bound(PHYSICS[physics], order)


def tiles(physics: str):
    """Kernel shapes by index: (tx, ty, tz, kind) as hw_tile_info."""
    ph = PHYSICS[physics]
    out = []
    for t in range(lib().hw_tile_count(ph)):
        v = [ctypes.c_int32() for _ in range(4)]
        _check(lib().hw_tile_info(ph, t, *[ctypes.byref(x) for x in v]))
        out.append(tuple(x.value for x in v))
    return out


def tile_label(shape) -> str:
    tx, ty, tz, kind = shape
    return f"{tx}x{ty}" + (f"x{tz}" if tz > 1 else "") + f"/k{kind}"


class Plan:
    """One simulation resident in a device arena (a torch uint8 tensor)."""

    def __init__(self, pb: Problem, device="cuda:0", arena=None):
        import torch
        self.pb = pb
        self.device = torch.device(device)
        self.bytes = footprint(pb)
        if arena is None:
            arena = torch.empty(self.bytes, dtype=torch.uint8, device=self.device)
        self.arena = arena
        h = ctypes.c_void_p()
        _check(lib().hw_plan_create(ctypes.byref(pb.c()),
                                    ctypes.c_void_p(arena.data_ptr()),
                                    arena.numel() * arena.element_size(),
                                    ctypes.byref(h)))
        self.handle = h

    def _s(self, stream):
        return _stream_handle(stream, self.device)

    def close(self):
        """Wait for the device's work, then destroy the plan (hw_plan_destroy
        must not run while launches of the plan may still be pending, on any
        stream the plan was driven on)."""
        if self.handle:
            import torch
            torch.cuda.synchronize(self.device)
            lib().hw_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_material(self, material: Sequence[np.ndarray], stream=None):
        n = lib().hw_num_materials(self.pb.c().physics)
        ptrs, keep = _f64_ptrs(list(material), n, self.pb.shape, False)
        _check(lib().hw_set_material(self.handle, ptrs, self._s(stream)))
        self._sync(stream)
        del keep

    def set_fields(self, fields, stream=None):
        if isinstance(fields, dict):
            fields = [fields.get(k) for k in self.pb.field_names]
        ptrs, keep = _f64_ptrs(list(fields), len(self.pb.field_names),
                               self.pb.shape, True)
        _check(lib().hw_set_fields(self.handle, ptrs, self._s(stream)))
        self._sync(stream)
        del keep

    def _sync(self, stream):
        import torch
        (stream or torch.cuda.current_stream(self.device)).synchronize()

    def advance(self, nsteps: int, energy_every: int = 0, stream=None):
        _check(lib().hw_advance(self.handle, nsteps, energy_every, self._s(stream)))

    def record_energy(self, stream=None):
        _check(lib().hw_record_energy(self.handle, self._s(stream)))

    def energy_trace(self, stream=None, allow_nonfinite=False):
        n = ctypes.c_int64()
        cap = max(self.pb.trace_cap, 1)
        e = np.zeros(cap)
        s = np.zeros(cap, dtype=np.int64)
        st = lib().hw_energy_trace(
            self.handle, e.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            s.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), cap,
            ctypes.byref(n), self._s(stream))
        if not (allow_nonfinite and st == 6):
            _check(st)
        return e[:n.value].copy(), s[:n.value].copy()

    def get_fields(self, comps=False, stream=None):
        names = self.pb.field_names
        out = {k: np.empty(self.pb.shape) for k in names}
        cout = {k: np.empty(self.pb.shape) for k in names} if comps else None
        P = ctypes.POINTER(ctypes.c_double)
        fp = (P * len(names))(*[out[k].ctypes.data_as(P) for k in names])
        cp = (P * len(names))(*[cout[k].ctypes.data_as(P) for k in names]) \
            if comps else None
        _check(lib().hw_get_fields(self.handle, fp, cp, self._s(stream)))
        return (out, cout) if comps else out

    @property
    def step(self) -> int:
        return lib().hw_plan_step(self.handle)

    def set_tile(self, tile: int):
        _check(lib().hw_plan_set_tile(self.handle, tile))

    def set_tuned_tile(self) -> int:
        """Set the kernel shape the tuning table holds for this plan's
        physics, order, storage, compensation and size, and return it (a
        new plan runs shape 0, the one-step kernel; the tuned 2D shapes
        advance two steps per launch).  Every shape gives the same bits."""
        from . import tuning
        pb = self.pb
        t = tuning.best_tile(pb.physics, pb.order, pb.storage, pb.comp, pb.nx, pb.ny, pb.nz)
        self.set_tile(t)
        return t

    def export_state(self, stream=None) -> bytes:
        n = ctypes.c_size_t()
        _check(lib().hw_state_size(self.handle, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(lib().hw_state_export(self.handle, buf, n.value, self._s(stream)))
        return buf.raw

    def import_state(self, blob: bytes, stream=None):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(lib().hw_state_import(self.handle, buf, len(blob), self._s(stream)))

    def set_source(self, ix: int, iy: int, samples, stream=None):
        """Point source at cell (ix, iy): on the pressure (acoustic), on vy
        at (ix, iy + 1/2) (2D elastic); step n adds samples[n] (see
        hw_set_source).  An empty sample list removes it."""
        a = np.ascontiguousarray(np.asarray(samples, dtype=np.float64).ravel())
        _check(lib().hw_set_source(self.handle, ix, iy,
                                   a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   len(a), self._s(stream)))

    def set_receivers(self, cells, stream=None):
        """Record (p, vx, vy) -- 2D elastic: the five fields -- at the given
        (ix, iy) cells after every step."""
        cells = list(cells)
        ix = np.ascontiguousarray([c[0] for c in cells] or [0], dtype=np.int64)
        iy = np.ascontiguousarray([c[1] for c in cells] or [0], dtype=np.int64)
        P64 = ctypes.POINTER(ctypes.c_int64)
        _check(lib().hw_set_receivers(self.handle, len(cells), ix.ctypes.data_as(P64),
                                      iy.ctypes.data_as(P64), self._s(stream)))
        self._nrec = len(cells)

    def receiver_trace(self, stream=None) -> np.ndarray:
        """[rows, receivers, m] array after each step: (p, vx, vy), m = 3;
        2D elastic: the five fields in field order, m = 5."""
        nrec = getattr(self, "_nrec", 0)
        rows = ctypes.c_int64()
        cap = max(self.pb.rec_steps, 1)
        m = 5 if self.pb.physics == "elastic2d" else 3
        out = np.zeros((cap, max(nrec, 1), m))
        _check(lib().hw_receiver_trace(self.handle,
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       cap, ctypes.byref(rows), self._s(stream)))
        return out[:rows.value, :nrec].copy()


def batch_advance(plans: Sequence[Plan], nsteps, energy_every: int = 0,
                  tile: int = -1, stream=None):
    """Advance many plans together (one launch per step per kernel kind)."""
    n = len(plans)
    if isinstance(nsteps, int):
        nsteps = [nsteps] * n
    hs = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    ns = (ctypes.c_int64 * n)(*nsteps)
    _check(lib().hw_batch_advance(hs, n, ns, energy_every, tile,
                                  _stream_handle(stream, plans[0].device)))


def _simulate_args(pb: Problem, material, fields):
    names = pb.field_names
    if isinstance(fields, dict):
        fields = [fields.get(k) for k in names]
    work = [np.array(np.broadcast_to(np.zeros(pb.shape) if f is None else f,
                                     pb.shape), dtype=np.float64) for f in fields]
    P = ctypes.POINTER(ctypes.c_double)
    fp = (P * len(names))(*[w.ctypes.data_as(P) for w in work])
    mp, keep = _f64_ptrs(list(material), len(material), pb.shape, False)
    cap = max(pb.trace_cap, 1)
    e = np.zeros(cap)
    return names, work, fp, mp, keep, cap, e


def simulate(pb: Problem, material, fields, nsteps: int, energy_every: int = 0,
             device="cuda:0"):
    """Blocking run through hw_simulate; returns (fields, energy)."""
    import torch
    arena = torch.empty(footprint(pb), dtype=torch.uint8, device=device)
    names, work, fp, mp, keep, cap, e = _simulate_args(pb, material, fields)
    n = ctypes.c_int64()
    _check(lib().hw_simulate(ctypes.byref(pb.c()), mp, fp, nsteps, energy_every,
                             e.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), cap,
                             ctypes.byref(n), ctypes.c_void_p(arena.data_ptr()),
                             arena.numel(), _stream_handle(None, torch.device(device))))
    return dict(zip(names, work)), e[:n.value].copy()


def simulate_noalloc(pb: Problem, material, fields, nsteps: int, energy_every: int = 0,
                     device="cuda:0", stream=None):
    """Blocking run through hw_simulate_noalloc (no device allocation: the
    plan lives in the library's static device array of NOALLOC_MAX_BYTES
    per GPU); returns (fields, energy)."""
    import torch
    dev = torch.device(device)
    names, work, fp, mp, keep, cap, e = _simulate_args(pb, material, fields)
    n = ctypes.c_int64()
    with torch.cuda.device(dev):
        _check(lib().hw_simulate_noalloc(ctypes.byref(pb.c()), mp, fp, nsteps,
                                         energy_every,
                                         e.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                         cap, ctypes.byref(n), _stream_handle(stream, dev)))
    return dict(zip(names, work)), e[:n.value].copy()
