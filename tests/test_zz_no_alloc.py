"""hw_simulate_noalloc (the entry point that allocates no device memory)
against hw_simulate (which runs in a caller-provided arena): bit-identical
fields and energies, on two calls in a row, the second on a smaller
problem, and on a third call of another physics; problems beyond the
static array's size are refused."""
import numpy as np
import pytest

import paper_2310_00236_amd as hw
import helpers

pytestmark = pytest.mark.gpu


def _same(a, b):
    return all(np.array_equal(a[k], b[k]) and
               np.array_equal(np.signbit(a[k]), np.signbit(b[k])) for k in b)


def _acoustic(nx, ny, storage, comp, nsteps, every, seed):
    rho, kappa, c = helpers.layered_material(nx, ny, seed)
    dt = 0.4 * hw.cfl_bound("acoustic2d", 4) / c
    f = helpers.acoustic_fields(nx, ny, seed + 1, storage)
    pb = hw.Problem("acoustic2d", nx, ny, 1, 4, storage, comp, 1.0, dt, 0,
                    nsteps // every + 2)
    return pb, [rho, kappa], f


def _check(pb, mat, f, nsteps, every):
    want, we = hw.simulate(pb, mat, f, nsteps, every)
    got, ge = hw.simulate_noalloc(pb, mat, f, nsteps, every)
    assert _same(got, want)
    assert np.array_equal(ge, we) and len(ge) == nsteps // every + 1


def test_noalloc_matches_arena_run_twice_then_smaller():
    # 70 steps: hw_simulate replays captured graphs, the static-array run
    # launches every step directly
    pb, mat, f = _acoustic(150, 37, "f16", "twosum", 70, 10, 11)
    _check(pb, mat, f, 70, 10)
    pb, mat, f = _acoustic(150, 37, "f16", "twosum", 70, 10, 11)
    _check(pb, mat, f, 70, 10)
    pb2, mat2, f2 = _acoustic(67, 19, "bf16", "fast2sum", 25, 5, 21)
    _check(pb2, mat2, f2, 25, 5)


def test_noalloc_elastic3d_after_acoustic():
    pb, mat, f = _acoustic(96, 40, "f32", "none", 12, 4, 31)
    _check(pb, mat, f, 12, 4)
    n = 14
    rho, lam, mu, c = helpers.smooth_medium3d(n, n + 1, n - 1, 5)
    dt = 0.3 * hw.cfl_bound("elastic3d", 2) / c
    pb3 = hw.Problem("elastic3d", n, n + 1, n - 1, 2, "f16", "twosum", 1.0, dt, 0, 4)
    rng = np.random.default_rng(6)
    f3 = {k: 0.1 * rng.normal(size=pb3.shape) for k in pb3.field_names}
    _check(pb3, [rho, lam, mu], f3, 9, 3)


def test_noalloc_refuses_problems_beyond_the_array():
    n = 2048                      # fp16 + comp: far above 64 MiB
    rho = np.ones((n, n))
    pb = hw.Problem("acoustic2d", n, n, 1, 4, "f16", "twosum", 1.0, 0.3, 0, 1)
    assert hw.footprint(pb) > hw.NOALLOC_MAX_BYTES
    with pytest.raises(hw.HalfwaveError) as e:
        hw.simulate_noalloc(pb, [rho, rho], {}, 1)
    assert e.value.name == "HW_E_NOMEM"
    # and the array still serves a valid call afterwards
    pb, mat, f = _acoustic(33, 17, "f16", "twosum", 6, 3, 41)
    _check(pb, mat, f, 6, 3)
