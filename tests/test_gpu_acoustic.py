"""GPU parity of the 2D acoustic path (through the C ABI) against the oracle.

Bit-exact against the oracle's op-by-op emulation of every storage format
and compensation mode, on grids that span several tiles with ragged tails,
on tiny grids where the stencil wraps several times, for every compiled tile
shape; within the stated tolerances against the FP64 reference (relative
energy drift and relative L2 field error) on the small homogeneous workload.
"""
import numpy as np
import pytest

import oracle
import paper_2310_00236_amd as hw
import workloads
from helpers import (ST, acoustic_fields, assert_bitexact, gpu_acoustic,
                     layered_material, oracle_acoustic, rel_drift, rel_l2)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage", ST)
@pytest.mark.parametrize("comp", ["none", "fast2sum", "twosum"])
@pytest.mark.parametrize("order", [2, 4])
def test_bitexact_vs_emulation(storage, comp, order):
    nx, ny = 150, 37           # 3 x 3 tiles of 64 x 16 with ragged tails
    rho, kappa, c = layered_material(nx, ny, 101)
    dt = 0.45 * hw.cfl_bound("acoustic2d", order) / c
    f = acoustic_fields(nx, ny, 102, storage)
    g, gc, ge = gpu_acoustic(nx, ny, order, storage, comp, dt, rho, kappa, f, 25,
                             energy_every=5)
    w, wc, we = oracle_acoustic(nx, ny, order, storage, comp, dt, rho, kappa, f,
                                25, energy_every=5)
    assert_bitexact(g, w, "fields")
    if comp != "none":
        assert_bitexact(gc, wc, "comps")
    # the energy is an fp64 sum over cells in another order
    np.testing.assert_allclose(ge, we, rtol=1e-12, atol=0)


@pytest.mark.parametrize("shape", [(1, 1), (1, 5), (4, 4), (5, 7), (7, 3),
                                   (64, 16), (65, 17), (257, 3), (3, 130)])
@pytest.mark.parametrize("tile", range(len(hw.tiles("acoustic2d"))))
def test_bitexact_sizes_and_tiles(shape, tile):
    nx, ny = shape
    rho, kappa, c = layered_material(nx, ny, 103)
    dt = 0.4 * hw.cfl_bound("acoustic2d", 4) / c
    f = acoustic_fields(nx, ny, 104, "f16")
    g, gc, _ = gpu_acoustic(nx, ny, 4, "f16", "twosum", dt, rho, kappa, f, 9,
                            tile=tile)
    w, wc, _ = oracle_acoustic(nx, ny, 4, "f16", "twosum", dt, rho, kappa, f, 9)
    assert_bitexact(g, w, f"{shape} tile {tile}")
    assert_bitexact(gc, wc, f"{shape} tile {tile} comps")


def test_small_homogeneous_workload_parity():
    """128x128, order 2, CFL 0.5, centred Gaussian, 1000 steps, energy every
    step: bit-exact against the emulation for fp16 plain and compensated, and
    within tolerance of the FP64 reference started from the same rounded
    initial state (so only the time stepping's roundoff is measured)."""
    w = workloads.small2d()
    f = w.fields()
    args = (w.nx, w.ny, w.order)
    refs = {}
    for storage in ("f32", "f16", "bf16"):
        fr = {k: oracle.round_to(v, storage) for k, v in f.items()}
        refs[storage] = oracle_acoustic(*args, "f64", "none", w.dt, w.rho,
                                        w.kappa, fr, w.nsteps, energy_every=1)
    results = {}
    for storage, comp in (("f32", "none"), ("f16", "none"), ("f16", "twosum"),
                          ("f16", "fast2sum"), ("bf16", "twosum")):
        g, _, ge = gpu_acoustic(*args, storage, comp, w.dt, w.rho, w.kappa, f,
                                w.nsteps, energy_every=1)
        results[(storage, comp)] = (g, ge)
        if storage == "f16":
            o, _, _ = oracle_acoustic(*args, storage, comp, w.dt, w.rho, w.kappa,
                                      f, w.nsteps)
            assert_bitexact(g, o, f"{storage}+{comp}")
    g32, e32 = results[("f32", "none")]
    assert rel_drift(e32, refs["f32"][2]) <= 1e-5
    assert rel_l2(g32, refs["f32"][0]) <= 1e-4
    for comp in ("twosum", "fast2sum"):
        g16c, e16c = results[("f16", comp)]
        assert rel_drift(e16c, refs["f16"][2]) <= 1e-3
        assert rel_l2(g16c, refs["f16"][0]) <= 5e-2


def test_compensation_fixes_energy_loss_small_cfl():
    """At a small Courant number plain fp16 loses energy and the compensated
    update does not (Sec. 3, Sec. 4), on the GPU."""
    n = 96
    w = workloads.small2d(n, nsteps=4000, order=4, cfl=0.0125, sigma=6.0)
    f = w.fields()
    _, _, e64 = oracle_acoustic(n, n, 4, "f64", "none", w.dt, w.rho, w.kappa,
                                {k: oracle.round_to(v, "f16") for k, v in f.items()},
                                w.nsteps, energy_every=500)
    _, _, e16 = gpu_acoustic(n, n, 4, "f16", "none", w.dt, w.rho, w.kappa, f,
                             w.nsteps, energy_every=500)
    _, _, e6 = gpu_acoustic(n, n, 4, "f16", "twosum", w.dt, w.rho, w.kappa, f,
                            w.nsteps, energy_every=500)
    loss = (e16[-1] - e64[0]) / e64[0]
    assert loss < -1e-2
    assert rel_drift(e6, e64) < 0.05 * abs(loss)


def test_symmetry_bit_exact_on_gpu():
    n = 128
    w = workloads.small2d(n, nsteps=300)
    g, _, _ = gpu_acoustic(n, n, 2, "f16", "none", w.dt, w.rho, w.kappa,
                           w.fields(), w.nsteps)
    c = n // 2
    idx = (2 * c - np.arange(n)) % n
    vidx = (2 * c - 1 - np.arange(n)) % n
    assert np.array_equal(g["p"], g["p"][:, idx])
    assert np.array_equal(g["p"], g["p"].T)
    assert np.array_equal(g["vx"], -g["vx"][:, vidx])
    assert np.array_equal(g["vx"], g["vy"].T)


def test_power_of_two_field_scale_is_exact():
    """Holding the fields scaled by 2^k (Sec. 5, range) gives the same
    results as the emulation run on scaled inputs, returned unscaled."""
    nx, ny = 70, 40
    rho, kappa, c = layered_material(nx, ny, 105)
    dt = 0.4 * hw.cfl_bound("acoustic2d", 4) / c
    f = {k: v * 1e-3 for k, v in acoustic_fields(nx, ny, 106, "f16").items()}
    g, gc, _ = gpu_acoustic(nx, ny, 4, "f16", "twosum", dt, rho, kappa, f, 30,
                            scale_log2=10)
    fs = {k: v * 1024.0 for k, v in f.items()}
    w, wc, _ = oracle_acoustic(nx, ny, 4, "f16", "twosum", dt, rho, kappa, fs, 30)
    assert_bitexact(g, {k: v / 1024.0 for k, v in w.items()}, "scaled")
    assert_bitexact(gc, {k: v / 1024.0 for k, v in wc.items()}, "scaled comps")


@pytest.mark.parametrize("comp", ["none", "twosum"])
def test_bf16_subnormal_range_bitexact(comp):
    """bf16 has fp32's exponent range, so fields scaled to about 2^-120 put
    part of the values and all compensation terms among the bf16 subnormals
    (spacing 2^-133) and part of the fp32 stencil among the fp32 subnormals:
    the rounding to bf16 keeps them, bit for bit as in the oracle."""
    nx, ny = 70, 40
    rho, kappa, c = layered_material(nx, ny, 107)
    dt = 0.4 * hw.cfl_bound("acoustic2d", 4) / c
    f = {k: v * 2.0 ** -120 for k, v in acoustic_fields(nx, ny, 108, "bf16").items()}
    g, gc, _ = gpu_acoustic(nx, ny, 4, "bf16", comp, dt, rho, kappa, f, 20)
    w, wc, _ = oracle_acoustic(nx, ny, 4, "bf16", comp, dt, rho, kappa, f, 20)
    assert_bitexact(g, w, "bf16 subnormal range")
    if comp != "none":
        assert_bitexact(gc, wc, "bf16 subnormal range comps")
    tiny = lambda a: np.any((a != 0) & (np.abs(a) < 2.0 ** -126))
    for k in g:                                          # the range is exercised
        assert tiny(g[k]) and np.any(np.abs(g[k]) >= 2.0 ** -126), k
        assert comp == "none" or tiny(gc[k]), k


@pytest.mark.parametrize("comp", ["none", "twosum"])
def test_bf16_overflow_matches_oracle(comp):
    """Fields near the top of the bf16 range, one step: some pressure
    differences overflow fp32, some pressure sums are finite in fp32 but round
    past the largest finite bf16 to infinity, and infinities of opposite sign
    meet to make NaNs.  The GPU has
    the oracle's infinities and NaN cells and its finite values bit for bit
    (only the sign and payload of a NaN are left open)."""
    nx, ny = 70, 40
    rng = np.random.default_rng(109)
    ones = np.ones((ny, nx))
    dt = 0.4 * hw.cfl_bound("acoustic2d", 4)
    f = {"p": 2.0 ** 127 * rng.uniform(-1.5, 1.5, (ny, nx)),
         "vx": np.zeros((ny, nx)), "vy": np.zeros((ny, nx))}
    g, gc, _ = gpu_acoustic(nx, ny, 4, "bf16", comp, dt, ones, ones, f, 1)
    w, wc, _ = oracle_acoustic(nx, ny, 4, "bf16", comp, dt, ones, ones, f, 1)
    pairs = [(g, w)] + ([(gc, wc)] if comp != "none" else [])
    for got, want in pairs:
        for k in want:
            gn, wn = np.isnan(got[k]), np.isnan(want[k])
            assert np.array_equal(gn, wn), k
            assert np.array_equal(got[k][~gn], want[k][~wn]), k
            assert np.array_equal(np.signbit(got[k][~gn]), np.signbit(want[k][~wn])), k
    for k in g:
        assert np.isinf(g[k]).any() and np.isfinite(g[k]).any(), k


@pytest.mark.parametrize("storage,comp", [("f16", "twosum"), ("f32", "none"),
                                          ("f16", "none"), ("bf16", "none"),
                                          ("f16", "twosum8")])
def test_full_grid_two_steps_at_full_size(storage, comp):
    """4096x4096 layered workload, order 4, every variant the benchmark
    times, each in its tuned tile shape: after 200 steps, the next two
    steps of the whole grid are compared cell by cell (fields and
    compensation terms, signed zeros included) with the oracle started from
    the GPU's state, and the energies of the three states with the oracle's
    (fp64 both, relative 1e-12).  Every tile of the launch, the XCD band
    renumbering and the last, partial band are covered."""
    from paper_2310_00236_amd import tuning
    w = workloads.layered2d(nsteps=200)
    pb = hw.Problem("acoustic2d", w.nx, w.ny, 1, 4, storage, comp, w.dx,
                    w.dt, 0, 4)
    plan = hw.Plan(pb)
    plan.set_tile(tuning.best_tile("acoustic2d", 4, storage, comp, w.nx, w.ny))
    plan.set_material([w.rho, w.kappa])
    plan.set_fields(w.fields())
    plan.advance(w.nsteps)
    before, cb = plan.get_fields(comps=True)
    plan.advance(2, energy_every=1)
    after, ca = plan.get_fields(comps=True)
    energy, steps = plan.energy_trace()
    plan.close()
    assert list(steps) == [200, 201, 202]
    o, oc, oe = oracle.acoustic2d(w.nx, w.ny, 4, w.dx, w.dt, w.rho, w.kappa, before,
                                  storage=storage, stencil="f32", comp=comp,
                                  comps=cb if comp != "none" else None, nsteps=2,
                                  energy_every=1)
    for k in after:
        bad = np.flatnonzero((after[k] != o[k]) |
                             (np.signbit(after[k]) != np.signbit(o[k])))
        assert bad.size == 0, (k, bad.size, np.unravel_index(bad[0], after[k].shape))
        if comp != "none":
            bad = np.flatnonzero((ca[k] != oc[k]) | (np.signbit(ca[k]) != np.signbit(oc[k])))
            assert bad.size == 0, ("comp", k, bad.size)
    np.testing.assert_allclose(energy, oe, rtol=1e-12, atol=0)


def test_overflow_is_reported():
    """A state at the top of the fp16 range (Table 1) overflows in one step;
    the energy becomes non-finite and the sticky status reports it."""
    nx = ny = 32
    rho = np.ones((ny, nx))
    p = np.full((ny, nx), 65504.0)
    p[16, 16] = -65504.0
    pb = hw.Problem("acoustic2d", nx, ny, 1, 2, "f16", "none", 1.0, 0.5, 0, 8)
    plan = hw.Plan(pb)
    plan.set_material([rho, rho])
    plan.set_fields({"p": p})
    plan.advance(2, energy_every=1)
    with pytest.raises(hw.HalfwaveError) as ei:
        plan.energy_trace()
    assert ei.value.name == "HW_E_NONFINITE"
    e, _ = plan.energy_trace(allow_nonfinite=True)
    assert np.isfinite(e[0]) and not np.isfinite(e[-1])
    plan.close()
