"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a child
process loads the sanitized build of oracle.c and drives every entry point
(all formats and compensations, sources, receivers, energies, the
compensated-sum checks) on small grids with ragged sizes; any invalid
memory access or undefined behaviour aborts it."""
import os
import subprocess
import sys

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import numpy as np, oracle, workloads
assert oracle.lib()._name.endswith("liboracle_san.so"), oracle.lib()._name
rng = np.random.default_rng(3)
for fmt in ("f64", "f32", "f16", "bf16"):
    for comp in ("none", "fast2sum", "twosum") + (("twosum8",) if fmt in ("f16", "bf16") else ()):
        for order in (2, 4):
            for nx, ny in ((1, 1), (5, 3), (9, 7)):
                rho = rng.uniform(1, 2, (ny, nx)); kap = rng.uniform(1, 2, (ny, nx))
                f = {k: oracle.round_to(0.1 * rng.normal(size=(ny, nx)), fmt) for k in oracle.ACOUSTIC_FIELDS}
                st = "f64" if fmt == "f64" else "f32"
                oracle.acoustic2d(nx, ny, order, 1.0, 0.1, rho, kap, f, storage=fmt, stencil=st,
                                  comp=comp, nsteps=3, energy_every=1,
                                  source=(nx // 2, ny // 2, [0.1, -0.2]), receivers=[(0, 0), (nx - 1, ny - 1)])
                oracle.acoustic2d_energy(nx, ny, order, 1.0, 0.1, rho, kap, f)
        for sten in (fmt, "f64"):
            if fmt != "f64":
                oracle.acoustic2d(6, 5, 4, 1.0, 0.1, np.ones((5, 6)), np.ones((5, 6)),
                                  {k: np.zeros((5, 6)) for k in oracle.ACOUSTIC_FIELDS},
                                  storage=fmt, stencil=sten, comp=comp, nsteps=2)
    for comp in ("none", "twosum"):
        n = (3, 4, 5)
        m = [rng.uniform(1, 2, n[::-1]) for _ in range(3)]
        f = {k: oracle.round_to(0.1 * rng.normal(size=n[::-1]), fmt) for k in oracle.ELASTIC_FIELDS}
        oracle.elastic3d(*n, 1.0, 0.05, *m, f, storage=fmt, stencil="f32" if fmt != "f64" else "f64",
                         comp=comp, nsteps=2, energy_every=1)
        oracle.elastic3d_energy(*n, 1.0, 0.05, *m, f)
        nx, ny = 7, 4
        m2 = [rng.uniform(1, 2, (ny, nx)) for _ in range(3)]
        f2 = {k: np.zeros((ny, nx)) for k in oracle.ELASTIC2D_FIELDS}
        f2["sxx"] = oracle.round_to(0.1 * rng.normal(size=(ny, nx)), fmt)
        oracle.elastic2d(nx, ny, 1.0, 0.05, *m2, f2, storage=fmt, stencil="f32" if fmt != "f64" else "f64",
                         comp=comp, nsteps=2, energy_every=1, source=(3, 1, [0.5]), receivers=[(0, 0), (6, 3)])
        oracle.elastic2d_energy(nx, ny, 1.0, 0.05, *m2, f2)
for fmt in ("f16", "bf16"):
    c = oracle.eft_exhaustive(fmt, 0x3c00, 0x3c08)
    assert c["twosum_not_exact"] == 0
a = oracle.round_to(rng.normal(size=50), "f16")
assert oracle.eft_check("f16", 6, a, a, False) == 0
oracle.quantize_comp(1e-4, 1.0, "f16")
print("SANITIZED-OK")
"""


def test_oracle_under_sanitizers():
    oracle.build(force=False, sanitize=True)
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, env=oracle.sanitizer_env(),
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "SANITIZED-OK" in r.stdout, r.stderr[-4000:]
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
