"""Closed-form discrete standing modes of the staggered leapfrog scheme.

TEST INFRASTRUCTURE ONLY (see the package docstring).

These are exact solutions of the *discrete* scheme of Sec. 3 (staggered grid,
staggered stencil, staggered leapfrog, periodic wrap) on a homogeneous medium,
so the FP64 oracle must reproduce them to roundoff after any number of steps.
They are derived here by substituting a separable trigonometric ansatz into
the update equations, independently of the oracle's code.

For the staggered first difference with weights w1, w2 (w_k = c_k dt/dx, as
fp32 values), applied to cos(k x) sampled half a cell either side of the
target point:
    w1 [f(x+h) - f(x-h)] + w2 [f(x+3h) - f(x-3h)],   h = dx/2
  = -2 sin(k x) [w1 sin(k h) + w2 sin(3 k h)] =: -sin(k x) * A(k)
and the same difference applied to sin(k x) gives +cos(k x) * A(k), with
A(k) = 2 [w1 sin(k dx/2) + w2 sin(3 k dx/2)]  (dt times the discrete
wavenumber).

Acoustic (Eq. 1, + signs): with p^n = cos(w n dt) cos(kx x_i) cos(ky y_j),
vx^{n+1/2} = -(Ax b / (2 s)) sin(w (n+1/2) dt) sin(kx x_{i+1/2}) cos(ky y_j)
(vy analogously), where s = sin(w dt / 2) and 4 s^2 = kappa b (Ax^2 + Ay^2).
"""
from __future__ import annotations

import math

import numpy as np

from . import round_to


def f32(x: float) -> float:
    return float(round_to(np.array([x]), "f32")[0])


def stencil_weights(order: int, dt: float, dx: float):
    r = dt / dx
    if order == 4:
        return f32((9.0 / 8.0) * r), f32((-1.0 / 24.0) * r)
    return f32(1.0 * r), 0.0


def amp(k: float, dx: float, w1: float, w2: float) -> float:
    """A(k) = 2 [w1 sin(k dx/2) + w2 sin(3 k dx/2)]."""
    return 2.0 * (w1 * math.sin(k * dx / 2) + w2 * math.sin(3 * k * dx / 2))


def acoustic_standing_mode(nx, ny, order, dx, dt, rho, kappa, mx, my, n):
    """State (vx^{n-1/2}, vy^{n-1/2}, p^n) of the standing mode with mx, my
    wavelengths across the periodic domain, homogeneous rho, kappa.

    Returns a dict of [ny, nx] arrays.  The material enters as the fp32
    values b = fp32(1/rho), kappa = fp32(kappa), as in the scheme."""
    w1, w2 = stencil_weights(order, dt, dx)
    b = f32(1.0 / rho)
    kap = f32(kappa)
    kx = 2 * math.pi * mx / (nx * dx)
    ky = 2 * math.pi * my / (ny * dx)
    ax = amp(kx, dx, w1, w2)
    ay = amp(ky, dx, w1, w2)
    s = 0.5 * math.sqrt(kap * b * (ax * ax + ay * ay))
    if not 0 < s < 1:
        raise ValueError("mode is not oscillatory at this time step")
    omega_dt = 2 * math.asin(s)
    x = np.arange(nx) * dx
    y = np.arange(ny) * dx
    xh = x + dx / 2
    yh = y + dx / 2
    t_half = (n - 0.5) * omega_dt   # v is stored at n - 1/2
    p = math.cos(n * omega_dt) * np.outer(np.cos(ky * y), np.cos(kx * x))
    vx = -(ax * b / (2 * s)) * math.sin(t_half) * np.outer(np.cos(ky * y),
                                                           np.sin(kx * xh))
    vy = -(ay * b / (2 * s)) * math.sin(t_half) * np.outer(np.sin(ky * yh),
                                                           np.cos(kx * x))
    return {"vx": vx, "vy": vy, "p": p}


def elastic_p_mode_x(nx, ny, nz, dx, dt, rho, lam, mu, m, n):
    """Compressional standing mode along x in a homogeneous elastic medium:
    sxx = cos(w n dt) cos(k x_i), syy = szz = lambda/(lambda+2mu) * sxx,
    vx at (i+1/2) follows the acoustic form with kappa -> lambda + 2 mu."""
    w = f32(1.0 * (dt / dx))
    b = f32(1.0 / rho)
    lam32, mu32 = f32(lam), f32(mu)
    l2m = lam32 + 2 * mu32
    k = 2 * math.pi * m / (nx * dx)
    a = amp(k, dx, w, 0.0)
    s = 0.5 * math.sqrt(l2m * b) * abs(a)
    omega_dt = 2 * math.asin(s)
    x = np.arange(nx) * dx
    shape = (nz, ny, nx)
    sxx = math.cos(n * omega_dt) * np.cos(k * x)
    vx = -(a * b / (2 * s)) * math.sin((n - 0.5) * omega_dt) * np.sin(k * (x + dx / 2))
    f = {key: np.zeros(shape) for key in
         ("vx", "vy", "vz", "sxx", "syy", "szz", "sxy", "sxz", "syz")}
    f["sxx"][...] = sxx
    f["syy"][...] = (lam32 / l2m) * sxx
    f["szz"][...] = (lam32 / l2m) * sxx
    f["vx"][...] = vx
    return f


def elastic_s_mode(nx, ny, nz, dx, dt, rho, lam, mu, m, n, axis_pair):
    """Shear standing mode in a homogeneous elastic medium.

    axis_pair = ('y', 'x'): particle velocity vy varying along x, with shear
    stress sxy (at x half points).  axis_pair = ('y', 'z'): vy varying along
    z with syz.  The velocity sits on integer points of the propagation axis
    and is updated first with the backward difference of the stress, the
    stress sits on half points and is updated with the forward difference:
        sigma^n_{i+1/2} = cos(w n dt) cos(k x_{i+1/2})
        v^{n+1/2}_i     = -(A b / (2 s)) sin(w (n+1/2) dt) sin(k x_i)
    with 4 s^2 = mu b A^2 (mu at the stress point is the mean of equal
    values, so it equals mu)."""
    w = f32(1.0 * (dt / dx))
    b = f32(1.0 / rho)
    mu32 = f32(mu)
    vel, prop = axis_pair
    nprop = {"x": nx, "y": ny, "z": nz}[prop]
    k = 2 * math.pi * m / (nprop * dx)
    a = amp(k, dx, w, 0.0)
    s = 0.5 * math.sqrt(mu32 * b) * abs(a)
    omega_dt = 2 * math.asin(s)
    c = np.arange(nprop) * dx
    sig = math.cos(n * omega_dt) * np.cos(k * (c + dx / 2))
    v = -(a * b / (2 * s)) * math.sin((n - 0.5) * omega_dt) * np.sin(k * c)
    shape = (nz, ny, nx)
    f = {key: np.zeros(shape) for key in
         ("vx", "vy", "vz", "sxx", "syy", "szz", "sxy", "sxz", "syz")}
    axis = {"x": 2, "y": 1, "z": 0}[prop]
    bshape = [1, 1, 1]
    bshape[axis] = nprop
    stress = {frozenset("xy"): "sxy", frozenset("xz"): "sxz",
              frozenset("yz"): "syz"}[frozenset(vel + prop)]
    f["v" + vel][...] = v.reshape(bshape)
    f[stress][...] = sig.reshape(bshape)
    return f


def elastic2d_surface_modes(nx, ny, dt, rho, lam, mu, m, n, kind):
    """Standing modes along y of the 2D elastic system of Eq. (A1) between
    the two free surfaces (rows 0 and L = ny-1), uniform in x, homogeneous
    medium, dx = 1, state (v^{n-1/2}, sigma^n).  k = m pi / L.

    kind 'p' (compressional, vy/syy/sxx):
        syy_j^n = A cos(w n dt) sin(k j)             (zero on both surfaces)
        vy_{j+1/2}^{n+1/2} = V sin(w (n+1/2) dt) cos(k (j+1/2))
        sxx_j^n = (lam / l2m) syy_j^n on interior rows, 0 on the surfaces
      with s = sin(w dt / 2) = w_ * sqrt(b l2m) sin(k/2)  (w_ = fp32 dt/dx),
      V = A b w_ sin(k/2) / s, and l2m = fp32(lam + 2 mu), b = fp32(1/rho).
    kind 's' (shear, vx/sxy):
        sxy_{j+1/2}^n = A cos(w n dt) sin(k (j+1/2))  (odd about each surface)
        vx_j^{n+1/2}  = V sin(w (n+1/2) dt) cos(k j)
      with s = w_ sqrt(b mu) sin(k/2), A = V s / (b w_ sin(k/2)).

    Both follow from substituting the ansatz into the update equations: the
    difference of sin(k j) across a half cell is 2 cos(k (j+1/2)) sin(k/2),
    the difference of cos across a half cell is -2 sin(.) sin(k/2), and
    the leapfrog difference of cos(w n dt) is -2 sin(w (n+1/2) dt) s.  For
    the shear mode the image rule of the surfaces (sxy half a cell outside
    equals minus sxy half a cell inside) holds for the ansatz because
    sin(k (L + 1/2)) = -sin(k (L - 1/2)) when k L is a multiple of pi.
    Returns a dict of the five fields, [ny, nx].
    """
    L = ny - 1
    k = m * math.pi / L
    w_ = f32(dt)                  # dx = 1
    b = f32(1.0 / rho)
    j = np.arange(ny, dtype=np.float64)[:, None] * np.ones((1, nx))
    z = np.zeros((ny, nx))
    out = {"vx": z.copy(), "vy": z.copy(), "sxx": z.copy(), "syy": z.copy(),
           "sxy": z.copy()}
    if kind == "p":
        l2m = f32(lam + 2.0 * mu)
        lm = f32(lam)
        s = w_ * math.sqrt(b * l2m) * math.sin(k / 2)
        om = 2.0 * math.asin(s)
        A = 1.0
        V = A * b * w_ * math.sin(k / 2) / s
        syy = A * math.cos(om * n) * np.sin(k * j)
        syy[0] = 0.0
        syy[-1] = 0.0
        # vy^{n+1/2} = V sin(w (n+1/2) dt) cos(k (j+1/2)); the state holds
        # the value half a step back
        vy = V * math.sin(om * (n - 0.5)) * np.cos(k * (j + 0.5))
        vy[-1] = 0.0
        sxx = (lm / l2m) * syy
        out.update(vy=vy, syy=syy, sxx=sxx)
    else:
        mq = f32(mu)
        s = w_ * math.sqrt(b * mq) * math.sin(k / 2)
        om = 2.0 * math.asin(s)
        V = 1.0
        A = V * s / (b * w_ * math.sin(k / 2))
        vx = V * math.sin(om * (n - 0.5)) * np.cos(k * j)
        sxy = A * math.cos(om * n) * np.sin(k * (j + 0.5))
        sxy[-1] = 0.0
        out.update(vx=vx, sxy=sxy)
    return out
