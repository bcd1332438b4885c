"""Shared helpers of the GPU parity tests: run the same seeded problem through
the C ABI (via the Python binding) and through the CPU oracle."""
import numpy as np

import oracle
import paper_2310_00236_amd as hw
import workloads

ST = ("f32", "f16", "bf16")


def layered_material(nx, ny, seed, nlayers=3):
    rng = np.random.default_rng(seed)
    c_row, rho_row, _ = workloads.layered_profile(ny, nlayers, rng)
    rho = np.repeat(rho_row[:, None], nx, axis=1)
    rho = rho * (1 + 0.2 * np.sin(2 * np.pi * np.arange(nx) / nx))[None, :]
    kappa = np.repeat((rho_row * c_row ** 2)[:, None], nx, axis=1)
    c_eff = float(np.sqrt(kappa.max() / rho.min()))
    return rho, kappa, c_eff


def acoustic_fields(nx, ny, seed, storage, vel=0.05):
    rng = np.random.default_rng(seed)
    f = {"p": workloads.gaussian2d(nx, ny, nx / 3, ny / 2, max(1.5, nx / 12)),
         "vx": vel * rng.normal(size=(ny, nx)),
         "vy": vel * rng.normal(size=(ny, nx))}
    return f


def gpu_acoustic(nx, ny, order, storage, comp, dt, rho, kappa, fields, nsteps,
                 energy_every=0, tile=0, scale_log2=0, dx=1.0):
    ntrace = (nsteps // energy_every + 2) if energy_every else 0
    pb = hw.Problem("acoustic2d", nx, ny, 1, order, storage, comp, dx, dt,
                    scale_log2, ntrace)
    plan = hw.Plan(pb)
    plan.set_tile(tile)
    plan.set_material([rho, kappa])
    plan.set_fields(fields)
    plan.advance(nsteps, energy_every)
    f, c = plan.get_fields(comps=True)
    e, steps = plan.energy_trace() if energy_every else (np.zeros(0), None)
    plan.close()
    return f, c, e


def oracle_acoustic(nx, ny, order, storage, comp, dt, rho, kappa, fields,
                    nsteps, energy_every=0, dx=1.0):
    fr = {k: oracle.round_to(v, storage) for k, v in fields.items()}
    return oracle.acoustic2d(nx, ny, order, dx, dt, rho, kappa, fr,
                             storage=storage,
                             stencil="f64" if storage == "f64" else "f32",
                             comp=comp, nsteps=nsteps,
                             energy_every=energy_every)


def smooth_medium3d(nx, ny, nz, seed):
    rng = np.random.default_rng(seed)
    rho = workloads.smooth_field3d(nx, ny, nz, rng, nmodes=6, kmax=2)
    lam = workloads.smooth_field3d(nx, ny, nz, rng, nmodes=6, kmax=2)
    mu = workloads.smooth_field3d(nx, ny, nz, rng, nmodes=6, kmax=2)
    # Courant number as the library measures it (faces, larger modulus)
    cp = float(np.sqrt((lam + 2 * mu).max() / rho.min()))
    return rho, lam, mu, cp


def elastic_fields(nx, ny, nz, seed, vel=0.05):
    rng = np.random.default_rng(seed)
    g = workloads.gaussian3d(nx, ny, nz, nx / 2, ny / 3, nz / 2, max(1.5, nx / 10))
    f = {k: vel * rng.normal(size=(nz, ny, nx)) for k in oracle.ELASTIC_FIELDS}
    for k in ("sxx", "syy", "szz"):
        f[k] = f[k] + g
    return f


def gpu_elastic(nx, ny, nz, storage, comp, dt, rho, lam, mu, fields, nsteps,
                energy_every=0, tile=0, dx=1.0):
    ntrace = (nsteps // energy_every + 2) if energy_every else 0
    pb = hw.Problem("elastic3d", nx, ny, nz, 2, storage, comp, dx, dt, 0, ntrace)
    plan = hw.Plan(pb)
    plan.set_tile(tile)
    plan.set_material([rho, lam, mu])
    plan.set_fields(fields)
    plan.advance(nsteps, energy_every)
    f, c = plan.get_fields(comps=True)
    e, _ = plan.energy_trace() if energy_every else (np.zeros(0), None)
    plan.close()
    return f, c, e


def oracle_elastic(nx, ny, nz, storage, comp, dt, rho, lam, mu, fields, nsteps,
                   energy_every=0, dx=1.0):
    fr = {k: oracle.round_to(v, storage) for k, v in fields.items()}
    return oracle.elastic3d(nx, ny, nz, dx, dt, rho, lam, mu, fr,
                            storage=storage,
                            stencil="f64" if storage == "f64" else "f32",
                            comp=comp, nsteps=nsteps, energy_every=energy_every)


def assert_bitexact(got, want, what=""):
    for k in want:
        if want[k] is None:
            continue
        g, w = np.asarray(got[k]), np.asarray(want[k])
        same = (g == w) | (np.isnan(g) & np.isnan(w))
        if not same.all():
            idx = np.argwhere(~same)[:5]
            raise AssertionError(
                f"{what} field {k}: {int((~same).sum())} of {same.size} differ; "
                f"first at {idx.tolist()}: gpu {g[tuple(idx[0])]!r} "
                f"oracle {w[tuple(idx[0])]!r}")
        # signed zeros must agree as well
        assert np.array_equal(np.signbit(g), np.signbit(w)), f"{what} {k} sign"


def rel_l2(a, b):
    num = sum(float(np.sum((a[k] - b[k]) ** 2)) for k in b)
    den = sum(float(np.sum(b[k] ** 2)) for k in b)
    return (num / den) ** 0.5


def rel_drift(e, e_ref):
    return float(np.max(np.abs(np.asarray(e) - np.asarray(e_ref))) / abs(e_ref[0]))
