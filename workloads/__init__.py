"""Seeded synthetic inputs for the wave-propagation workloads.

This module only draws inputs: initial fields, material models, batch and
request mixes.  It holds none of the numerical method's arithmetic and is the
one piece of code that both the oracle-side tests and the GPU-side callers
use.  Every generator takes an explicit seed; the same seed gives the same
arrays on every machine (numpy's PCG64 via default_rng).

Workloads (sizes are the ones the paper's experiments and the benchmark use;
the paper's own elastic medium is a dataset that is not available, so the
smooth random medium below stands in for it):

  small2d   2D acoustic, order 2, 128x128 periodic, rho = c = 1, dx = 1,
            CFL 0.5, Gaussian pressure pulse (sigma 8 cells) at the centre,
            zero velocity.
  layered2d 2D acoustic, order 4, 4096x4096 periodic, 4 horizontal layers
            (c ~ U[1.5, 4.5], rho ~ U[1.0, 2.5] per layer, 3 interface depths
            uniform in (0, ny)), CFL 0.4 on the largest layer speed, 4
            Gaussian pulses (sigma 8 cells) at uniform random positions.
  smooth3d  3D elastic, order 2, 512^3 periodic, rho, lambda, mu each a smooth
            periodic random field (16 Fourier modes, |k| <= 4) mapped to
            [1, 3], CFL 0.3 on the largest P-wave speed, explosive Gaussian
            (sigma 8 cells) on the three normal stresses.
  shots     64 independent layered 2D shots, sides U{256..2048}, step counts
            U{500..5000}.
  requests  Poisson stream of mixed 2D layered / 3D smooth requests.
  paper_elastic2d
            the elastic experiment of App. A: 2D, 600 x 600 cells of 1/125
            km, dt = 1e-4 s, 60000 steps, periodic in x, free surfaces at the
            top and bottom rows, at rest; a 5 Hz Ricker source on vy ten
            cells below the top surface at x = 200, a receiver at x = 400 at
            the same depth.  The paper's medium (a Marmousi2 subsection) is
            not available; a layered medium with undulating interfaces
            stands in for it, spanning the paper's stated extremes (minimum
            shear speed 1.0117 km/s, maximum compressional speed 4.6992
            km/s, density 2.0293 to 2.6230).
  paper2d   the acoustic experiment of Sec. 3: homogeneous rho = c = 1,
            600 x 600 cells of 1/125 m (ppw = 10; 1800 x 1800 of 1/375 m for
            ppw = 30), dt = 1e-4 s, 60000 steps, order 4, at rest; a point
            source on the pressure with a 5 Hz Ricker wavelet at one third
            of the domain in both directions, a receiver at two thirds.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 20231001


def seed_for(workload_id: int, instance: int = 0) -> int:
    return BASE_SEED + 1000 * workload_id + instance


# ------------------------------------------------------------ primitives --

def periodic_offsets(n: int, centre: float) -> np.ndarray:
    """Minimum-image offsets of grid indices 0..n-1 from `centre`."""
    d = np.arange(n, dtype=np.float64) - centre
    return d - n * np.round(d / n)


def gaussian2d(nx, ny, cx, cy, sigma, amplitude=1.0):
    dx = periodic_offsets(nx, cx)
    dy = periodic_offsets(ny, cy)
    r2 = dy[:, None] ** 2 + dx[None, :] ** 2
    return amplitude * np.exp(-r2 / (2.0 * sigma * sigma))


def gaussian3d(nx, ny, nz, cx, cy, cz, sigma, amplitude=1.0):
    """Periodic Gaussian, formed as the outer product of its 1D factors."""
    import torch
    g = [torch.from_numpy(amplitude ** (1.0 / 3.0) *
                          np.exp(-periodic_offsets(n, c) ** 2 / (2.0 * sigma * sigma)))
         for n, c in ((nz, cz), (ny, cy), (nx, cx))]
    out = g[0][:, None, None] * g[1][None, :, None]
    return (out * g[2][None, None, :]).numpy()


def layered_profile(ny, nlayers, rng, c_range=(1.5, 4.5), rho_range=(1.0, 2.5)):
    """Per-row (depth) wave speed and density of a layered medium."""
    depths = np.sort(rng.uniform(0.0, ny, size=nlayers - 1))
    c_layer = rng.uniform(*c_range, size=nlayers)
    rho_layer = rng.uniform(*rho_range, size=nlayers)
    rows = np.arange(ny, dtype=np.float64)
    layer = np.searchsorted(depths, rows, side="right")
    return c_layer[layer], rho_layer[layer], c_layer


def smooth_field3d(nx, ny, nz, rng, lo=1.0, hi=3.0, nmodes=16, kmax=4):
    """Smooth periodic random field: a sum of nmodes random Fourier modes with
    integer wave vectors |k| <= kmax, mapped affinely onto [lo, hi].

    Each mode a*cos(2 pi k.x + phase) is evaluated as
    a*(cos(A) cos(B) - sin(A) sin(B)) with A the x part and B the (y, z) part,
    accumulated in place in fp32 (torch's multi-threaded CPU kernels)."""
    import torch
    ks = []
    while len(ks) < nmodes:
        k = rng.integers(-kmax, kmax + 1, size=3)
        if 0 < np.dot(k, k) <= kmax * kmax:
            ks.append(k)
    x = np.arange(nx) / nx
    y = np.arange(ny) / ny
    z = np.arange(nz) / nz
    f = torch.zeros((nz, ny, nx), dtype=torch.float32)
    for k in ks:
        phase = rng.uniform(0, 2 * math.pi)
        a = rng.normal()
        A = 2 * math.pi * k[0] * x
        B = 2 * math.pi * (k[2] * z[:, None] + k[1] * y[None, :]) + phase
        ca = torch.from_numpy(np.cos(A).astype(np.float32))
        sa = torch.from_numpy(np.sin(A).astype(np.float32))
        cb = torch.from_numpy((a * np.cos(B)).astype(np.float32))[:, :, None]
        sb = torch.from_numpy((a * np.sin(B)).astype(np.float32))[:, :, None]
        f.addcmul_(cb, ca)
        f.addcmul_(sb, sa, value=-1.0)
    fmin, fmax = float(f.min()), float(f.max())
    if fmax == fmin:
        return np.full((nz, ny, nx), lo)
    f.sub_(fmin).mul_((hi - lo) / (fmax - fmin)).add_(lo)
    return f.numpy().astype(np.float64)


# ------------------------------------------------------------- workloads --

@dataclass
class Acoustic2D:
    nx: int
    ny: int
    order: int
    dx: float
    dt: float
    rho: np.ndarray          # [ny, nx] at p points
    kappa: np.ndarray        # [ny, nx] bulk modulus rho c^2 (= 1/beta)
    p0: np.ndarray           # [ny, nx] initial pressure
    vx0: np.ndarray | None = None
    vy0: np.ndarray | None = None
    nsteps: int = 0
    name: str = ""
    meta: dict = field(default_factory=dict)
    # point source on the pressure: (ix, iy, per-step samples), see paper2d
    source: tuple | None = None
    receivers: list | None = None      # [(ix, iy), ...]

    @property
    def cells(self) -> int:
        return self.nx * self.ny

    def fields(self):
        z = np.zeros((self.ny, self.nx))
        return {"vx": z if self.vx0 is None else self.vx0,
                "vy": z if self.vy0 is None else self.vy0, "p": self.p0}


@dataclass
class Elastic3D:
    nx: int
    ny: int
    nz: int
    dx: float
    dt: float
    rho: np.ndarray
    lam: np.ndarray
    mu: np.ndarray
    init: dict               # field name -> [nz, ny, nx] array (missing = 0)
    nsteps: int = 0
    name: str = ""
    meta: dict = field(default_factory=dict)
    order: int = 2

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    def fields(self):
        names = ("vx", "vy", "vz", "sxx", "syy", "szz", "sxy", "sxz", "syz")
        z = np.zeros((self.nz, self.ny, self.nx))
        return {k: self.init.get(k, z) for k in names}


@dataclass
class Elastic2D:
    """2D velocity-stress problem bounded in y by free surfaces (rows 0 and
    ny-1); arrays [ny, nx]."""
    nx: int
    ny: int
    dx: float
    dt: float
    rho: np.ndarray
    lam: np.ndarray
    mu: np.ndarray
    init: dict               # field name -> [ny, nx] array (missing = 0)
    nsteps: int = 0
    name: str = ""
    meta: dict = field(default_factory=dict)
    source: tuple | None = None        # (ix, iy, samples): vy at (ix, iy+1/2)
    receivers: list | None = None      # [(ix, iy), ...]
    order: int = 2

    @property
    def cells(self) -> int:
        return self.nx * self.ny

    def fields(self):
        z = np.zeros((self.ny, self.nx))
        return {k: self.init.get(k, z) for k in ("vx", "vy", "sxx", "syy", "sxy")}


# the extremes the paper states for its elastic medium (App. A), km/s and
# Gt/km^3
APP_A_CS_MIN = 1.0117
APP_A_CP_MAX = 4.6992
APP_A_RHO = (2.0293, 2.6230)


def layered_elastic2d(nx, ny, seed, nlayers=5, vpvs=1.85, swing=0.05):
    """rho, lambda, mu [ny, nx] of a layered medium whose interfaces
    undulate periodically in x: the normalised depth s = (j + d(i)) / (ny-1)
    (clipped to [0, 1]) with d a sum of two seeded periodic sines of
    amplitude swing*ny and swing*ny/2; the P speed grows with s, 70% as a
    gradient and 30% in nlayers equal steps, from APP_A_CS_MIN * vpvs to
    APP_A_CP_MAX; the S speed is the P speed / vpvs; the density follows the
    P speed linearly over APP_A_RHO.  Top and bottom rows reach the extremes
    wherever the interfaces rise above the top or sink below the bottom."""
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0.0, 2.0 * math.pi, size=2)
    x = 2.0 * math.pi * np.arange(nx) / nx
    d = swing * ny * (np.sin(x + ph[0]) + 0.5 * np.sin(3.0 * x + ph[1]))
    s = np.clip((np.arange(ny)[:, None] + d[None, :]) / (ny - 1), 0.0, 1.0)
    shape = 0.7 * s + 0.3 * np.minimum(np.floor(nlayers * s), nlayers - 1) / (nlayers - 1)
    cp_top = APP_A_CS_MIN * vpvs
    cp = cp_top + (APP_A_CP_MAX - cp_top) * shape
    cs = cp / vpvs
    rho = APP_A_RHO[0] + (APP_A_RHO[1] - APP_A_RHO[0]) * (cp - cp_top) / (APP_A_CP_MAX - cp_top)
    mu = rho * cs ** 2
    lam = rho * (cp ** 2 - 2.0 * cs ** 2)
    return rho, lam, mu


def paper_elastic2d(nsteps=60000, f0=5.0, delay=None, amplitude=1.0,
                    seed=None, n=600) -> Elastic2D:
    """The elastic setup of App. A on the medium of layered_elastic2d.

    n x n cells of dx = 1/125 km (ppw 10 at 12.5 Hz for the slowest shear
    wave), dt = 1e-4 s.  The vy update of step m is centred at t_m = m dt,
    so step m adds amplitude * dt / dx^2 * ricker(t_m - delay) (a point force
    per unit mass spread over one cell), delayed by 1.2 / f0 and cut after
    delay + 1.2 / f0.  Source on vy at (n/3, 10 + 1/2), receiver at cell
    (2n/3, 10): ten cells below the free surface at row 0."""
    dx = 1.0 / 125.0
    dt = 1e-4
    delay = 1.2 / f0 if delay is None else delay
    t = np.arange(nsteps) * dt - delay
    samples = amplitude * dt / (dx * dx) * ricker(t, f0)
    keep = int(np.ceil((delay + 1.2 / f0) / dt)) + 1
    samples = samples[:min(keep, nsteps)]
    rho, lam, mu = layered_elastic2d(n, n, seed_for(7) if seed is None else seed)
    return Elastic2D(n, n, dx, dt, rho, lam, mu, {}, nsteps=nsteps,
                     name=f"elastic2d-{n}x{n}-free-surface-ricker",
                     meta={"f0": f0, "delay": delay,
                           "cp_max": float(np.sqrt((lam + 2 * mu) / rho).max())},
                     source=(n // 3, 10, samples),
                     receivers=[(2 * n // 3, 10)])


def small2d(n=128, nsteps=1000, order=2, cfl=0.5, sigma=8.0) -> Acoustic2D:
    """Homogeneous rho = c = 1, dx = 1, centred Gaussian pressure pulse."""
    dt = cfl * 1.0 / 1.0
    ones = np.ones((n, n))
    return Acoustic2D(n, n, order, 1.0, dt, ones, ones.copy(),
                      gaussian2d(n, n, n // 2, n // 2, sigma), nsteps=nsteps,
                      name=f"acoustic2d-o{order}-{n}x{n}-homogeneous")


def ricker(t, f0):
    """Ricker wavelet of peak frequency f0 at times t (seconds, centred on
    the peak): (1 - 2a) exp(-a) with a = (pi f0 t)^2."""
    a = (math.pi * f0 * np.asarray(t, dtype=np.float64)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def paper2d(ppw=10, nsteps=60000, order=4, f0=5.0, delay=None,
            amplitude=1.0) -> Acoustic2D:
    """The acoustic setup of Sec. 3 (homogeneous, at rest, Ricker point
    source on the pressure, one receiver).

    The grid has 600 * ppw / 10 cells per side with dx = (1/125) * 10 / ppw
    (ppw points per wavelength of c = 1 at 12.5 Hz, 2.5 times the wavelet's
    peak frequency) and dt = 1e-4 s.  Per-step source samples: the scheme's
    right-hand sides already carry dt (the stencil weights are c_k dt/dx)
    and a point source spreads over one cell of area dx*dx, so step n adds
    amplitude * dt / dx^2 * ricker(t_{n+1/2} - delay) with t_{n+1/2} =
    (n + 1/2) dt, the time at which the pressure update is centred.  The
    wavelet is delayed by 1.2 / f0 so that it starts at rest (|r| < 2e-5 at
    t = 0)."""
    n = 600 * ppw // 10
    dx = (1.0 / 125.0) * 10.0 / ppw
    dt = 1e-4
    delay = 1.2 / f0 if delay is None else delay
    t = (np.arange(nsteps) + 0.5) * dt - delay
    samples = amplitude * dt / (dx * dx) * ricker(t, f0)
    # the wavelet is negligible after delay + 1.2/f0: keep only that part
    keep = int(np.ceil((delay + 1.2 / f0) / dt)) + 1
    samples = samples[:min(keep, nsteps)]
    ones = np.ones((n, n))
    return Acoustic2D(n, n, order, dx, dt, ones, ones.copy(), np.zeros((n, n)),
                      nsteps=nsteps, name=f"acoustic2d-o{order}-{n}x{n}-ricker-ppw{ppw}",
                      meta={"ppw": ppw, "f0": f0, "delay": delay},
                      source=(n // 3, n // 3, samples),
                      receivers=[(2 * n // 3, 2 * n // 3)])


def layered2d(nx=4096, ny=None, nsteps=10000, order=4, cfl=0.4, nlayers=4,
              npulses=4, sigma=8.0, seed=None) -> Acoustic2D:
    ny = nx if ny is None else ny
    rng = np.random.default_rng(seed_for(2) if seed is None else seed)
    c_row, rho_row, c_layer = layered_profile(ny, nlayers, rng)
    rho = np.repeat(rho_row[:, None], nx, axis=1)
    kappa = np.repeat((rho_row * c_row ** 2)[:, None], nx, axis=1)
    dx = 1.0
    dt = cfl * dx / float(c_layer.max())
    p0 = np.zeros((ny, nx))
    for _ in range(npulses):
        cx = rng.integers(0, nx)
        cy = rng.integers(0, ny)
        p0 += gaussian2d(nx, ny, cx, cy, sigma)
    return Acoustic2D(nx, ny, order, dx, dt, rho, kappa, p0, nsteps=nsteps,
                      name=f"acoustic2d-o{order}-{nx}x{ny}-layered",
                      meta={"c_max": float(c_layer.max())})


def smooth3d(n=512, nsteps=2000, cfl=0.3, sigma=8.0, seed=None,
             nx=None, ny=None, nz=None, nmodes=16) -> Elastic3D:
    nx = n if nx is None else nx
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    rng = np.random.default_rng(seed_for(3) if seed is None else seed)
    import torch
    rho = smooth_field3d(nx, ny, nz, rng, nmodes=nmodes)
    lam = smooth_field3d(nx, ny, nz, rng, nmodes=nmodes)
    mu = smooth_field3d(nx, ny, nz, rng, nmodes=nmodes)
    m = torch.from_numpy(mu).mul(2).add_(torch.from_numpy(lam))
    cp_max = float(m.div_(torch.from_numpy(rho)).max().sqrt())
    del m
    dx = 1.0
    dt = cfl * dx / cp_max
    g = gaussian3d(nx, ny, nz, nx // 2, ny // 2, nz // 2, sigma)
    init = {"sxx": g, "syy": g, "szz": g}       # read-only: shared
    return Elastic3D(nx, ny, nz, dx, dt, rho, lam, mu, init, nsteps=nsteps,
                     name=f"elastic3d-o2-{nx}x{ny}x{nz}-smooth",
                     meta={"cp_max": cp_max})


def shot_sizes(nshots=64, seed=None, side=(256, 2048), steps=(500, 5000)):
    """(nx, ny, nsteps) of each shot of the batched workload."""
    rng = np.random.default_rng(seed_for(4) if seed is None else seed)
    out = []
    for _ in range(nshots):
        nx = int(rng.integers(side[0], side[1] + 1))
        ny = int(rng.integers(side[0], side[1] + 1))
        ns = int(rng.integers(steps[0], steps[1] + 1))
        out.append((nx, ny, ns))
    return out


def shot(nx, ny, nsteps, index, order=4, cfl=0.4) -> Acoustic2D:
    """One shot of the batched workload: its own layered medium and pulse."""
    a = layered2d(nx, ny, nsteps=nsteps, order=order, cfl=cfl, npulses=1,
                  seed=seed_for(4, 1 + index))
    a.name = f"shot{index}-{nx}x{ny}"
    return a


@dataclass
class Request:
    arrival: float           # seconds after the stream starts
    kind: str                # 'acoustic2d' or 'elastic3d'
    size: int                # grid side
    nsteps: int
    precision: str           # 'f32' or 'f16+comp'
    index: int


def request_stream(nreq=500, rate=1.3, seed=None, frac2d=0.7,
                   side2d=(512, 4096), side3d=(128, 384),
                   steps=(1000, 10000)):
    """Poisson arrivals of mixed 2D/3D requests, precision 50/50."""
    rng = np.random.default_rng(seed_for(5) if seed is None else seed)
    t = 0.0
    out = []
    for i in range(nreq):
        t += rng.exponential(1.0 / rate)
        if rng.uniform() < frac2d:
            kind, size = "acoustic2d", int(rng.integers(side2d[0], side2d[1] + 1))
        else:
            kind, size = "elastic3d", int(rng.integers(side3d[0], side3d[1] + 1))
        ns = int(rng.integers(steps[0], steps[1] + 1))
        prec = "f32" if rng.uniform() < 0.5 else "f16+comp"
        out.append(Request(t, kind, size, ns, prec, i))
    return out


def request_problem(req: Request):
    """Concrete inputs of a request (own seed per request index)."""
    if req.kind == "acoustic2d":
        return layered2d(req.size, req.size, nsteps=req.nsteps, npulses=1,
                         seed=seed_for(5, 1 + req.index))
    # 3D requests draw 4 modes per medium field (the serving workload is about
    # sizes and arrival times; this keeps drawing the inputs cheap)
    return smooth3d(req.size, nsteps=req.nsteps, seed=seed_for(5, 1 + req.index),
                    nmodes=4)
