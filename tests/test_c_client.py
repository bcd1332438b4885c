"""The C ABI used from plain C: tests/c_client/halfwave_run (built by the
build step) reads a problem, material and fields from a file, drives
libhalfwave through halfwave.h alone -- no Python, no torch, the arena from
hipMalloc -- and writes the results.  On the GPU its fields, compensation
terms and energies must be the oracle's, bit for bit (energies to 1e-12);
on any machine it must report invalid problems through hw_last_error before
touching the device."""
import os
import subprocess
import sys

import numpy as np
import pytest

import paper_2310_00236_amd as hw
from helpers import (acoustic_fields, assert_bitexact, elastic_fields,
                     layered_material, oracle_acoustic, oracle_elastic,
                     smooth_medium3d)

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_client", "halfwave_run")


def _write_input(path, pb, nsteps, every, tile, material, fields):
    head = np.array([hw.PHYSICS[pb.physics], pb.order, hw.STORAGE[pb.storage],
                     hw.COMP[pb.comp], pb.nx, pb.ny, pb.nz, nsteps, every, tile,
                     pb.trace_cap], dtype="<i8")
    with open(path, "wb") as f:
        f.write(head.tobytes())
        f.write(np.array([pb.dx, pb.dt], dtype="<f8").tobytes())
        for a in material:
            f.write(np.ascontiguousarray(a, dtype="<f8").tobytes())
        for k in pb.field_names:
            a = fields.get(k)
            a = np.zeros(pb.shape) if a is None else a
            f.write(np.ascontiguousarray(a, dtype="<f8").tobytes())


def _read_output(path, pb):
    n = int(np.prod(pb.shape))
    raw = open(path, "rb").read()
    names = pb.field_names
    vals = np.frombuffer(raw, dtype="<f8", count=2 * len(names) * n)
    f = {k: vals[i * n:(i + 1) * n].reshape(pb.shape) for i, k in enumerate(names)}
    c = {k: vals[(len(names) + i) * n:(len(names) + i + 1) * n].reshape(pb.shape)
         for i, k in enumerate(names)}
    off = 8 * 2 * len(names) * n
    ne = int(np.frombuffer(raw[off:off + 8], dtype="<i8")[0])
    e = np.frombuffer(raw[off + 8:], dtype="<f8", count=ne)
    return f, c, e


def _run(tmp_path, pb, nsteps, every, tile, material, fields):
    assert os.path.exists(EXE), "the C client is not built (tests/c_client/build.py)"
    inp, out = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    _write_input(inp, pb, nsteps, every, tile, material, fields)
    return subprocess.run([EXE, inp, out], capture_output=True, text=True, timeout=120), out


def test_client_reports_invalid_problems(tmp_path):
    """Runs anywhere: an invalid order is refused by hw_footprint, on the
    host, with hw_last_error's message; a missing argument is a usage
    error."""
    nx, ny = 16, 8
    pb = hw.Problem("acoustic2d", nx, ny, 1, 3, "f16", "twosum", 1.0, 0.1, 0, 0)
    r, _ = _run(tmp_path, pb, 1, 0, -1, [np.ones((ny, nx))] * 2, {})
    assert r.returncode == 1, r.stderr
    assert "hw_footprint" in r.stderr and "status 1" in r.stderr
    u = subprocess.run([EXE], capture_output=True, text=True, timeout=60)
    assert u.returncode == 2 and "usage" in u.stderr


TWO_STEP = [t for t, s in enumerate(hw.tiles("acoustic2d")) if s[2] == 2]


@pytest.mark.gpu
@pytest.mark.parametrize("storage,comp,tile", [("f16", "twosum", TWO_STEP[-1]),
                                               ("f16", "twosum8", TWO_STEP[0]),
                                               ("f32", "none", -1),
                                               ("bf16", "fast2sum", 0)])
def test_client_acoustic_matches_oracle(tmp_path, storage, comp, tile):
    nx, ny, nsteps, every = 150, 37, 25, 5
    print(f"C client: acoustic2d {nx}x{ny} {storage}+{comp} tile {tile}", flush=True)
    rho, kappa, c = layered_material(nx, ny, 951)
    dt = 0.4 * hw.cfl_bound("acoustic2d", 4) / c
    f = acoustic_fields(nx, ny, 952, storage)
    pb = hw.Problem("acoustic2d", nx, ny, 1, 4, storage, comp, 1.0, dt, 0, 8)
    r, out = _run(tmp_path, pb, nsteps, every, tile, [rho, kappa], f)
    assert r.returncode == 0, r.stderr
    g, gc, ge = _read_output(out, pb)
    w, wc, we = oracle_acoustic(nx, ny, 4, storage, comp, dt, rho, kappa, f, nsteps,
                                energy_every=every)[:3]
    assert_bitexact(g, w, "C client fields")
    if comp != "none":
        assert_bitexact(gc, wc, "C client comps")
    assert len(ge) == nsteps // every + 1
    np.testing.assert_allclose(ge, we, rtol=1e-12, atol=0)


@pytest.mark.gpu
def test_client_elastic3d_matches_oracle(tmp_path):
    n, nsteps = 14, 9
    print(f"C client: elastic3d {n}^3 f16+twosum", flush=True)
    rho, lam, mu, cp = smooth_medium3d(n, n + 1, n - 1, 953)
    dt = 0.4 * hw.cfl_bound("elastic3d", 2) / cp
    f = elastic_fields(n, n + 1, n - 1, 954)
    pb = hw.Problem("elastic3d", n, n + 1, n - 1, 2, "f16", "twosum", 1.0, dt, 0, 4)
    r, out = _run(tmp_path, pb, nsteps, 3, -1, [rho, lam, mu], f)
    assert r.returncode == 0, r.stderr
    g, gc, ge = _read_output(out, pb)
    w, wc, we = oracle_elastic(n, n + 1, n - 1, "f16", "twosum", dt, rho, lam, mu, f,
                               nsteps, energy_every=3)[:3]
    assert_bitexact(g, w, "C client 3D fields")
    assert_bitexact(gc, wc, "C client 3D comps")
    np.testing.assert_allclose(ge, we, rtol=1e-12, atol=0)
