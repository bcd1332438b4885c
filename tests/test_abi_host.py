"""Host-side tests of the C ABI (no GPU needed): the library loads, exports
every entry point its header declares, and validates problems, materials and
fields before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2310_00236_amd as hw

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include",
                      "halfwave.h")
FAKE_ARENA = 1 << 20      # aligned non-NULL address, for machines without a GPU


def _gpu_visible():
    # counting devices does not initialise one
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


_GPU = _gpu_visible()
_arenas = []


def _arena_address(nbytes):
    """The arena handed to hw_plan_create.  Without a GPU, an aligned address
    that no call here dereferences: every call either stops at host-side
    validation or fails for want of a device.  Where a GPU is visible, the
    calls that pass validation go on to the device and write the arena, so
    it must be real device memory (kept alive until the session ends)."""
    if not _GPU:
        return FAKE_ARENA
    import torch
    t = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda:0")
    _arenas.append(t)
    return (t.data_ptr() + 255) // 256 * 256


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hw_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 20
    hw.lib()                      # loads torch's HIP runtime first
    L = ctypes.CDLL(hw.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_abi_version_and_counts():
    L = hw.lib()
    assert L.hw_abi_version() == hw.ABI_VERSION
    assert L.hw_num_fields(0) == 3 and L.hw_num_fields(1) == 9
    assert L.hw_num_materials(0) == 2 and L.hw_num_materials(1) == 3
    assert L.hw_num_fields(7) == 0


def test_cfl_bounds():
    assert hw.cfl_bound("acoustic2d", 2) == pytest.approx(2 ** -0.5)
    assert hw.cfl_bound("acoustic2d", 4) == pytest.approx(1 / (2 ** 0.5 * (9 / 8 + 1 / 24)))
    assert hw.cfl_bound("elastic3d", 2) == pytest.approx(3 ** -0.5)
    assert hw.lib().hw_cfl_bound(1, 4) < 0


def test_tiles_listed():
    t2, t3 = hw.tiles("acoustic2d"), hw.tiles("elastic3d")
    assert len(t2) >= 2 and len(t3) >= 2
    assert all(tx % 64 == 0 and ty % 4 == 0 and kind in (0, 1, 3, 4, 5)
               for tx, ty, tz, kind in t2)
    # tz: time steps per launch (2 for the temporally blocked kinds 4 and 5)
    assert all(tz == (2 if kind in (4, 5) else 1) for tx, ty, tz, kind in t2)
    assert all(ty % 8 == 0 for tx, ty, tz, kind in t2 if kind in (3, 5))
    assert any(kind == 4 for *_, kind in t2) and any(kind == 5 for *_, kind in t2)
    assert all((kind == 0 and tx * ty == 256 and tz == 1) or
               (kind == 2 and tx == 64 and (ty + 2) % 4 == 0 and tz >= 1)
               for tx, ty, tz, kind in t3)
    assert any(kind == 2 for *_, kind in t3)


def _pb(**kw):
    base = dict(physics="acoustic2d", nx=32, ny=24, nz=1, order=4, storage="f16",
                comp="twosum", dx=1.0, dt=0.1, scale_log2=0, trace_cap=4)
    base.update(kw)
    return hw.Problem(**base)


@pytest.mark.parametrize("kw", [
    dict(nx=0), dict(ny=-1), dict(nz=2), dict(order=3), dict(order=6),
    dict(physics="elastic3d", nz=4, order=4), dict(dt=0.0), dict(dx=-1.0),
    dict(dt=float("nan")), dict(trace_cap=-1), dict(scale_log2=61),
    dict(src_cap=-1), dict(rec_cap=65), dict(rec_cap=-1), dict(rec_steps=-2),
    dict(physics="elastic3d", nz=4, order=2, src_cap=8),
    dict(physics="elastic3d", nz=4, order=2, rec_cap=1, rec_steps=4),
    dict(physics="elastic3d", nz=4, order=2, stencil="f64"),
    dict(comp="twosum8", storage="f32"),
    dict(physics="elastic3d", nz=4, order=2, comp="twosum8"),
])
def test_invalid_problems(kw):
    with pytest.raises(hw.HalfwaveError) as ei:
        hw.footprint(_pb(**kw))
    assert ei.value.name == "HW_E_INVAL"


def test_invalid_enums_and_abi():
    for field, val in (("storage", 7), ("comp", 4), ("physics", 3),
                       ("abi_version", 99), ("stencil", 3), ("stencil", -1)):
        c = _pb().c()
        setattr(c, field, val)
        n = ctypes.c_size_t()
        assert hw.lib().hw_footprint(ctypes.byref(c), ctypes.byref(n)) == 1


def test_footprint_grows_with_precision_and_compensation():
    f16 = hw.footprint(_pb(storage="f16", comp="none"))
    f16c8 = hw.footprint(_pb(storage="f16", comp="twosum8"))
    f16c = hw.footprint(_pb(storage="f16", comp="twosum"))
    f32 = hw.footprint(_pb(storage="f32", comp="none"))
    assert f16 < f16c8 < f16c and f16 < f32


def _plan(pb, arena_bytes=None):
    h = ctypes.c_void_p()
    n = hw.footprint(pb) if arena_bytes is None else arena_bytes
    st = hw.lib().hw_plan_create(ctypes.byref(pb.c()), ctypes.c_void_p(_arena_address(n)),
                                 n, ctypes.byref(h))
    return st, h


def test_plan_create_checks_arena():
    pb = _pb()
    st, _ = _plan(pb, hw.footprint(pb) - 1)
    assert st == 4                                   # HW_E_NOMEM
    h = ctypes.c_void_p()
    st = hw.lib().hw_plan_create(ctypes.byref(pb.c()),
                                 ctypes.c_void_p(_arena_address(hw.footprint(pb)) + 8),
                                 hw.footprint(pb), ctypes.byref(h))
    assert st == 1 and not h.value                   # misaligned: INVAL
    st, h = _plan(pb)
    assert st == 0 and h.value
    hw.lib().hw_plan_destroy(h)


def _set(fn, h, arrays):
    P = ctypes.POINTER(ctypes.c_double)
    keep = [np.ascontiguousarray(a, dtype=np.float64) if a is not None else None
            for a in arrays]
    ptrs = (P * len(keep))(*[a.ctypes.data_as(P) if a is not None else P()
                             for a in keep])
    return fn(h, ptrs, None)


@pytest.mark.parametrize("mat,status", [
    ("rho0", 1), ("kappa_neg", 1), ("nan", 1), ("unstable", 2)])
def test_material_validation_before_device(mat, status):
    pb = _pb(dt=0.2)
    st, h = _plan(pb)
    rho = np.ones((24, 32))
    kappa = np.ones((24, 32))
    if mat == "rho0":
        rho[3, 4] = 0.0
    elif mat == "kappa_neg":
        kappa[5, 5] = -1.0
    elif mat == "nan":
        kappa[0, 0] = np.nan
    elif mat == "unstable":
        kappa[10, 10] = 20.0        # c = 4.5 at one cell: CFL 0.9 > 0.606
    assert _set(hw.lib().hw_set_material, h, [rho, kappa]) == status
    hw.lib().hw_plan_destroy(h)


def test_elastic_material_validation():
    pb = _pb(physics="elastic3d", nx=8, ny=6, nz=5, order=2, dt=0.1)
    st, h = _plan(pb)
    one = np.ones((5, 6, 8))
    mu = one.copy()
    mu[1, 1, 1] = 0.0
    assert _set(hw.lib().hw_set_material, h, [one, one, mu]) == 1
    lam = one.copy()
    lam[2, 2, 2] = -0.7             # 3 lambda + 2 mu < 0
    assert _set(hw.lib().hw_set_material, h, [one, lam, one]) == 1
    assert _set(hw.lib().hw_set_material, h, [one, one, 40 * one]) == 2
    hw.lib().hw_plan_destroy(h)


@pytest.mark.parametrize("storage,value,scale,status", [
    ("f16", 65504.0, 0, None), ("f16", 65505.0, 0, 3), ("f16", np.inf, 0, 3),
    ("f16", np.nan, 0, 3), ("f16", 1100.0, 6, 3), ("f16", 1000.0, 6, None), ("bf16", 1e38, 0, None),
    ("bf16", 3.4e38, 0, 3), ("f32", 1e39, 0, 3)])
def test_field_range_validation(storage, value, scale, status):
    pb = _pb(storage=storage, scale_log2=scale)
    st, h = _plan(pb)
    p = np.zeros((24, 32))
    p[1, 2] = value
    got = _set(hw.lib().hw_set_fields, h, [None, None, p])
    if status is None:
        assert got != 3             # passes validation (then needs a device)
    else:
        assert got == status
        assert b"does not fit" in hw.lib().hw_last_error()
    hw.lib().hw_plan_destroy(h)


def test_advance_before_upload_is_state_error():
    st, h = _plan(_pb())
    assert hw.lib().hw_advance(h, 1, 0, None) == 7
    assert hw.lib().hw_plan_step(h) == 0
    hw.lib().hw_plan_destroy(h)


def test_footprint_reserves_source_and_receivers():
    base = hw.footprint(_pb())
    assert hw.footprint(_pb(src_cap=1000)) >= base + 4000
    assert hw.footprint(_pb(rec_cap=3, rec_steps=100)) >= base + 3 * 100 * 3 * 8


def test_source_and_receiver_validation_before_device():
    """Every argument check of hw_set_source / hw_set_receivers runs before
    any HIP call, so a plan on a placeholder arena exercises them all."""
    P = ctypes.POINTER(ctypes.c_double)
    P64 = ctypes.POINTER(ctypes.c_int64)
    st, h = _plan(_pb(src_cap=4, rec_cap=2, rec_steps=10))
    assert st == 0
    L = hw.lib()
    s5 = np.ones(5)
    assert L.hw_set_source(h, 1, 1, s5.ctypes.data_as(P), 5, None) == 4   # > src_cap
    assert L.hw_set_source(h, 32, 1, s5.ctypes.data_as(P), 4, None) == 1  # x outside
    assert L.hw_set_source(h, 0, -1, s5.ctypes.data_as(P), 4, None) == 1
    bad = np.array([1.0, np.inf, 0.0, 0.0])
    assert L.hw_set_source(h, 0, 0, bad.ctypes.data_as(P), 4, None) == 3  # RANGE
    big = np.array([1e39, 0.0, 0.0, 0.0])                                  # fp32 overflow
    assert L.hw_set_source(h, 0, 0, big.ctypes.data_as(P), 4, None) == 3
    ix = np.array([0, 5, 7], dtype=np.int64)
    iy = np.array([0, 23, 24], dtype=np.int64)
    assert L.hw_set_receivers(h, 3, ix.ctypes.data_as(P64), iy.ctypes.data_as(P64), None) == 4
    assert L.hw_set_receivers(h, 2, ix[1:].ctypes.data_as(P64), iy[1:].ctypes.data_as(P64),
                              None) == 1                                  # y = 24 outside
    L.hw_plan_destroy(h)
    st, h = _plan(_pb(physics="elastic3d", nz=4, order=2))
    assert st == 0
    assert L.hw_set_source(h, 0, 0, s5.ctypes.data_as(P), 1, None) == 1
    assert L.hw_set_receivers(h, 1, ix.ctypes.data_as(P64), iy.ctypes.data_as(P64), None) == 1
    L.hw_plan_destroy(h)


def test_elastic2d_problem_rules():
    """The 2D elastic system (App. A, free surfaces): order 2, nz = 1,
    ny >= 3, the fp32 stencil, 16-bit compensation words; sources and
    receivers allowed, with five values per receiver and trace row."""
    L = hw.lib()
    assert L.hw_num_fields(2) == 5 and L.hw_num_materials(2) == 3
    assert hw.cfl_bound("elastic2d", 2) == pytest.approx(2 ** -0.5)
    assert L.hw_cfl_bound(2, 4) < 0
    assert hw.tiles("elastic2d") == [(64, 4, 1, 1), (64, 4, 1, 0)]
    e2 = dict(physics="elastic2d", order=2)
    for kw in (dict(order=4), dict(nz=2), dict(ny=2), dict(stencil="f64"),
               dict(stencil="storage"), dict(comp="twosum8")):
        with pytest.raises(hw.HalfwaveError) as ei:
            hw.footprint(_pb(**{**e2, **kw}))
        assert ei.value.name == "HW_E_INVAL", kw
    base = hw.footprint(_pb(**e2))
    assert hw.footprint(_pb(**e2, rec_cap=3, rec_steps=100)) >= base + 3 * 100 * 5 * 8
    assert hw.footprint(_pb(**e2, storage="f32", comp="none")) < \
        hw.footprint(_pb(**e2, storage="f32", comp="twosum"))


def test_elastic2d_host_validation_before_device():
    P = ctypes.POINTER(ctypes.c_double)
    L = hw.lib()
    pb = _pb(physics="elastic2d", order=2, nx=12, ny=7, dt=0.1, src_cap=4,
             rec_cap=1, rec_steps=4)
    st, h = _plan(pb)
    assert st == 0
    one = np.ones((7, 12))
    lam = one.copy()
    lam[3, 4] = -1.5                # lambda + mu < 0
    assert _set(L.hw_set_material, h, [one, lam, one]) == 1
    mu = one.copy()
    mu[0, 0] = 0.0
    assert _set(L.hw_set_material, h, [one, one, mu]) == 1
    assert _set(L.hw_set_material, h, [one, one, 40 * one]) == 2       # unstable
    z = np.zeros((7, 12))
    syy = z.copy()
    syy[6, 3] = 0.5                 # syy on the bottom surface
    assert _set(L.hw_set_fields, h, [None, None, None, syy, None]) == 1
    vy = z.copy()
    vy[6, 0] = 0.5                  # vy outside the body
    assert _set(L.hw_set_fields, h, [None, vy, None, None, None]) == 1
    assert b"elastic2d" in L.hw_last_error()
    s1 = np.ones(1)
    assert L.hw_set_source(h, 3, 6, s1.ctypes.data_as(P), 1, None) == 1  # row ny-1
    L.hw_plan_destroy(h)


def test_noalloc_refuses_before_the_device():
    # invalid problems and problems beyond the static array fail on the host,
    # before any HIP call (no GPU here)
    L = hw.lib()
    P = ctypes.POINTER(ctypes.c_double)
    one = np.ones(4)
    mat = (P * 3)(*[one.ctypes.data_as(P)] * 3)
    fld = (P * 9)(*[one.ctypes.data_as(P)] * 9)
    n = ctypes.c_int64()
    big = hw.Problem("acoustic2d", 2048, 2048, 1, 4, "f16", "twosum", 1.0, 0.3, 0, 1)
    assert hw.footprint(big) > hw.NOALLOC_MAX_BYTES
    st = L.hw_simulate_noalloc(ctypes.byref(big.c()), mat, fld, 1, 0, None, 0,
                               ctypes.byref(n), None)
    assert hw.STATUS[st] == "HW_E_NOMEM"
    assert "at most" in L.hw_last_error().decode()
    bad = hw.Problem("acoustic2d", 8, 8, 1, 3, "f16", "twosum", 1.0, 0.3, 0, 1)
    st = L.hw_simulate_noalloc(ctypes.byref(bad.c()), mat, fld, 1, 0, None, 0,
                               ctypes.byref(n), None)
    assert hw.STATUS[st] == "HW_E_INVAL"
    st = L.hw_simulate_noalloc(ctypes.byref(bad.c()), mat, None, 1, 0, None, 0,
                               ctypes.byref(n), None)
    assert hw.STATUS[st] == "HW_E_INVAL"
