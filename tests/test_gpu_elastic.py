"""GPU parity of the 3D elastic path (through the C ABI) against the oracle."""
import numpy as np
import pytest

import oracle
import paper_2310_00236_amd as hw
from helpers import (ST, assert_bitexact, elastic_fields, gpu_elastic,
                     oracle_elastic, rel_drift, rel_l2, smooth_medium3d)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("tile", [0, 2])
@pytest.mark.parametrize("storage", ST)
@pytest.mark.parametrize("comp", ["none", "fast2sum", "twosum"])
def test_bitexact_vs_emulation(storage, comp, tile):
    nx, ny, nz = 70, 11, 7        # ragged in x and y for every tile shape
    rho, lam, mu, cp = smooth_medium3d(nx, ny, nz, 201)
    dt = 0.4 * hw.cfl_bound("elastic3d", 2) / cp
    f = elastic_fields(nx, ny, nz, 202)
    g, gc, ge = gpu_elastic(nx, ny, nz, storage, comp, dt, rho, lam, mu, f, 12,
                            energy_every=4, tile=tile)
    w, wc, we = oracle_elastic(nx, ny, nz, storage, comp, dt, rho, lam, mu, f,
                               12, energy_every=4)
    assert_bitexact(g, w, "fields")
    if comp != "none":
        assert_bitexact(gc, wc, "comps")
    np.testing.assert_allclose(ge, we, rtol=1e-12, atol=0)


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 3, 1), (5, 4, 3), (33, 9, 2),
                                   (130, 13, 9), (9, 7, 130)])
@pytest.mark.parametrize("tile", range(len(hw.tiles("elastic3d"))))
def test_bitexact_sizes_and_tiles(shape, tile):
    nx, ny, nz = shape
    rho, lam, mu, cp = smooth_medium3d(nx, ny, nz, 203)
    dt = 0.4 * hw.cfl_bound("elastic3d", 2) / cp
    f = elastic_fields(nx, ny, nz, 204)
    g, gc, _ = gpu_elastic(nx, ny, nz, "f16", "twosum", dt, rho, lam, mu, f, 6,
                           tile=tile)
    w, wc, _ = oracle_elastic(nx, ny, nz, "f16", "twosum", dt, rho, lam, mu, f, 6)
    assert_bitexact(g, w, f"{shape} tile {tile}")
    assert_bitexact(gc, wc, f"{shape} tile {tile} comps")


def test_fp64_tolerances():
    """32^3 smooth medium, CFL 0.3, explosive source, 300 steps: fp32 and
    fp16+TwoSum against the FP64 reference from the same rounded start."""
    n = 32
    rho, lam, mu, cp = smooth_medium3d(n, n, n, 205)
    dt = 0.3 / cp
    f = elastic_fields(n, n, n, 206, vel=0.0)
    f16 = {k: oracle.round_to(v, "f16") for k, v in f.items()}
    ref, _, e64 = oracle_elastic(n, n, n, "f64", "none", dt, rho, lam, mu, f16,
                                 300, energy_every=10)
    g32, _, e32 = gpu_elastic(n, n, n, "f32", "none", dt, rho, lam, mu, f16, 300,
                              energy_every=10)
    g16, _, e16 = gpu_elastic(n, n, n, "f16", "twosum", dt, rho, lam, mu, f16,
                              300, energy_every=10)
    assert rel_drift(e32, e64) <= 1e-5
    assert rel_l2(g32, ref) <= 1e-4
    assert rel_drift(e16, e64) <= 1e-3
    assert rel_l2(g16, ref) <= 5e-2
