"""Dense operator matrices of the staggered scheme, built from coordinates.

TEST INFRASTRUCTURE ONLY (see the package docstring).

This is a second, deliberately different construction of the spatial
operators of Sec. 3 and App. A: every unknown is placed at its physical
position (in units of half a cell, so all coordinates are integers), and a
staggered derivative at a target point is assembled by looking up the source
unknowns that sit 1 and 3 half-cells away along the axis, by coordinate, with
periodic wrap.  No array-index arithmetic of the solvers is reused.  The
one-step update is then a sequence of dense matrix products in fp64.
Intended for tiny grids only.
"""
from __future__ import annotations

import numpy as np

from .closed_forms import f32, stencil_weights


class _Points:
    """Unknowns of one field: integer positions (in half cells) -> index."""

    def __init__(self, pos):
        self.pos = [tuple(p) for p in pos]
        self.index = {p: n for n, p in enumerate(self.pos)}

    def __len__(self):
        return len(self.pos)


def _derivative(target, source, axis, period, taps):
    """Matrix of sum_k c_k [f(x + o_k e) - f(x - o_k e)] from source points
    to target points; taps = [(offset_in_half_cells, coefficient), ...]."""
    m = np.zeros((len(target), len(source)))
    for t, pos in enumerate(target.pos):
        for off, c in taps:
            for sgn in (+1, -1):
                q = list(pos)
                q[axis] = (q[axis] + sgn * off) % period[axis]
                m[t, source.index[tuple(q)]] += sgn * c
    return m


def _average(target, cells, axes, period, values):
    """Mean of the cell-centred values at the 2**len(axes) cells lying half
    a cell away from each target point along each of the given axes."""
    out = np.zeros(len(target))
    for t, pos in enumerate(target.pos):
        acc = []
        for mask in range(1 << len(axes)):
            q = list(pos)
            for bit, ax in enumerate(axes):
                q[ax] = (q[ax] + (1 if mask >> bit & 1 else -1)) % period[ax]
            acc.append(values[cells.index[tuple(q)]])
        out[t] = sum(acc) / len(acc)
    return out


def acoustic2d_operators(nx, ny, order, dx, dt, rho, kappa):
    """Return (Gx, Gy, Dx, Dy, bx, by, kap, layout) for the 2D acoustic
    scheme.  Positions are (x, y) in half cells; p at even/even, vx at
    odd/even, vy at even/odd.  layout maps field name -> flat index order
    (row-major [ny][nx])."""
    period = (2 * nx, 2 * ny)
    grid = [(i, j) for j in range(ny) for i in range(nx)]
    P = _Points([(2 * i, 2 * j) for i, j in grid])
    VX = _Points([(2 * i + 1, 2 * j) for i, j in grid])
    VY = _Points([(2 * i, 2 * j + 1) for i, j in grid])
    w1, w2 = stencil_weights(order, dt, dx)
    taps = [(1, w1)] + ([(3, w2)] if order == 4 else [])
    Gx = _derivative(VX, P, 0, period, taps)
    Gy = _derivative(VY, P, 1, period, taps)
    Dx = _derivative(P, VX, 0, period, taps)
    Dy = _derivative(P, VY, 1, period, taps)
    rho = np.broadcast_to(np.asarray(rho, float), (ny, nx)).ravel()
    kappa = np.broadcast_to(np.asarray(kappa, float), (ny, nx)).ravel()
    b = np.array([f32(1.0 / r) for r in rho])
    kap = np.array([f32(k) for k in kappa])
    bx = _average(VX, P, [0], period, b)
    by = _average(VY, P, [1], period, b)
    return Gx, Gy, Dx, Dy, bx, by, kap


def acoustic2d_step(ops, vx, vy, p, source=None):
    """One fp64 leapfrog step with the dense operators (flattened fields).

    source: optional (flat index of a p point, value) -- a point source on
    the pressure equation (the s_p of Eq. 1), a unit vector at that point
    times the value, added to the divergence before the scaling by kappa."""
    Gx, Gy, Dx, Dy, bx, by, kap = ops
    vx = vx + bx * (Gx @ p)
    vy = vy + by * (Gy @ p)
    rhs = Dx @ vx + Dy @ vy
    if source is not None:
        e = np.zeros_like(rhs)
        e[source[0]] = 1.0
        rhs = rhs + source[1] * e
    p = p + kap * rhs
    return vx, vy, p


ELASTIC_POS = {   # offsets (x, y, z) in half cells relative to 2*(i, j, k)
    "vx": (1, 0, 0), "vy": (0, 1, 0), "vz": (0, 0, 1),
    "sxx": (0, 0, 0), "syy": (0, 0, 0), "szz": (0, 0, 0),
    "sxy": (1, 1, 0), "sxz": (1, 0, 1), "syz": (0, 1, 1),
}


def elastic3d_operators(nx, ny, nz, dx, dt, rho, lam, mu):
    period = (2 * nx, 2 * ny, 2 * nz)
    grid = [(i, j, k) for k in range(nz) for j in range(ny) for i in range(nx)]
    pts = {f: _Points([(2 * i + o[0], 2 * j + o[1], 2 * k + o[2])
                       for i, j, k in grid]) for f, o in ELASTIC_POS.items()}
    w = f32(1.0 * (dt / dx))
    taps = [(1, w)]

    def d(tf, sf, axis):
        return _derivative(pts[tf], pts[sf], axis, period, taps)

    shape = (nz, ny, nx)
    cells = pts["sxx"]
    b = np.array([f32(1.0 / r) for r in np.broadcast_to(rho, shape).ravel()])
    lm = np.array([f32(v) for v in np.broadcast_to(lam, shape).ravel()])
    m = np.array([f32(v) for v in np.broadcast_to(mu, shape).ravel()])
    ops = {
        "b": {f: _average(pts[f], cells, [a], period, b)
              for f, a in (("vx", 0), ("vy", 1), ("vz", 2))},
        "lam": lm, "mu": m,
        "mu_e": {f: _average(pts[f], cells, axes, period, m)
                 for f, axes in (("sxy", [0, 1]), ("sxz", [0, 2]),
                                 ("syz", [1, 2]))},
        # velocity rows: divergence of the stress tensor
        "vx": [d("vx", "sxx", 0), d("vx", "sxy", 1), d("vx", "sxz", 2)],
        "vy": [d("vy", "sxy", 0), d("vy", "syy", 1), d("vy", "syz", 2)],
        "vz": [d("vz", "sxz", 0), d("vz", "syz", 1), d("vz", "szz", 2)],
        # strain rates
        "exx": d("sxx", "vx", 0), "eyy": d("sxx", "vy", 1),
        "ezz": d("sxx", "vz", 2),
        "sxy": [d("sxy", "vy", 0), d("sxy", "vx", 1)],
        "sxz": [d("sxz", "vz", 0), d("sxz", "vx", 2)],
        "syz": [d("syz", "vz", 1), d("syz", "vy", 2)],
    }
    return ops


def elastic3d_step(ops, f):
    """One fp64 leapfrog step with dense operators; f maps field -> flat."""
    f = dict(f)
    src = {"vx": ("sxx", "sxy", "sxz"), "vy": ("sxy", "syy", "syz"),
           "vz": ("sxz", "syz", "szz")}
    for v in ("vx", "vy", "vz"):
        div = sum(M @ f[s] for M, s in zip(ops[v], src[v]))
        f[v] = f[v] + ops["b"][v] * div
    ex = ops["exx"] @ f["vx"]
    ey = ops["eyy"] @ f["vy"]
    ez = ops["ezz"] @ f["vz"]
    lam, mu = ops["lam"], ops["mu"]
    l2m = lam + 2 * mu
    f["sxx"] = f["sxx"] + l2m * ex + lam * (ey + ez)
    f["syy"] = f["syy"] + l2m * ey + lam * (ex + ez)
    f["szz"] = f["szz"] + l2m * ez + lam * (ex + ey)
    pairs = {"sxy": ("vy", "vx"), "sxz": ("vz", "vx"), "syz": ("vz", "vy")}
    for s, (a, c) in pairs.items():
        A, C = ops[s]
        f[s] = f[s] + ops["mu_e"][s] * (A @ f[a] + C @ f[c])
    return f
