"""Plain FP64 oracle of the source parameterisations of the paper's source
applications (TEST INFRASTRUCTURE ONLY: only the tests use this module).

* Earthquake location (Applications, "Earthquake Location and Source Time
  Function Retrieval"): f(x, t) = g(t) exp(-|x - x0|^2 / (2 sigma^2)) /
  (2 pi sigma^2), sampled at the grid nodes within `radius` cells of the node
  nearest to x0 (radius 3 at sigma = dx/2 drops terms below exp(-18)).  With
  a cell value of f times dx dz the footprint enters the discrete equation
  exactly as a point source r(t) does (value r(t), density r/(dx dz)).
* Rupture (Applications, "Earthquake Rupture Imaging"): point sources j with
  f_j(t) = A0_j exp(-(t - t0_j)^2 / (2 sigma_t^2)).

The gradients follow from dJ/dwav (the adjoint at each source cell, from
the oracle's or the library's adjoint sweep) by the chain rule.
"""
from __future__ import annotations

import numpy as np


def gaussian_footprint(x0, z0, sigma, dx, nx, nz, radius=3):
    """Cells (ix, iz) near (x0, z0) (metres, node (i, j) at (i dx, j dx))
    inside the grid, and their weights dx^2 exp(-r^2/(2 sigma^2))/(2 pi sigma^2)."""
    cx, cz = int(round(x0 / dx)), int(round(z0 / dx))
    cells, w = [], []
    for iz in range(cz - radius, cz + radius + 1):
        for ix in range(cx - radius, cx + radius + 1):
            if 0 <= ix < nx and 0 <= iz < nz:
                r2 = (ix * dx - x0) ** 2 + (iz * dx - z0) ** 2
                cells.append((ix, iz))
                w.append(dx * dx * np.exp(-r2 / (2 * sigma * sigma)) / (2 * np.pi * sigma * sigma))
    return np.array(cells, dtype=np.int32), np.array(w)


def gaussian_wavelets(g, w):
    """wav[j][k] = g(t_k) w_j."""
    return np.outer(np.asarray(w, dtype=np.float64), np.asarray(g, dtype=np.float64))


def gaussian_grad(gw, g, cells, x0, z0, sigma, dx):
    """(dJ/dg [nt], dJ/dx0, dJ/dz0) from dJ/dwav [nsrc][nt]."""
    gw = np.asarray(gw, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    xj, zj = cells[:, 0] * dx, cells[:, 1] * dx
    w = dx * dx * np.exp(-((xj - x0) ** 2 + (zj - z0) ** 2) / (2 * sigma ** 2)) / (2 * np.pi * sigma ** 2)
    dg = (gw * w[:, None]).sum(0)
    c = gw @ g                                   # sum_k dJ/dwav_jk g_k
    dx0 = float((c * w * (xj - x0) / sigma ** 2).sum())
    dz0 = float((c * w * (zj - z0) / sigma ** 2).sum())
    return dg, dx0, dz0


def rupture_wavelets(A0, t0, sigma_t, dt, nt):
    t = np.arange(nt) * dt
    A0, t0 = np.asarray(A0, dtype=np.float64), np.asarray(t0, dtype=np.float64)
    return A0[:, None] * np.exp(-(t[None, :] - t0[:, None]) ** 2 / (2 * sigma_t ** 2))


def rupture_grad(gw, A0, t0, sigma_t, dt):
    """(dJ/dA0 [np], dJ/dt0 [np]) from dJ/dwav [np][nt]."""
    gw = np.asarray(gw, dtype=np.float64)
    nt = gw.shape[1]
    t = np.arange(nt) * dt
    A0, t0 = np.asarray(A0, dtype=np.float64), np.asarray(t0, dtype=np.float64)
    e = np.exp(-(t[None, :] - t0[:, None]) ** 2 / (2 * sigma_t ** 2))
    return (gw * e).sum(1), (gw * A0[:, None] * e * (t[None, :] - t0[:, None]) / sigma_t ** 2).sum(1)


def plane_wave_wavelets(xs, theta_deg, c, f0, t0, dt, nt):
    """A row of source nodes at horizontal positions xs (metres) emitting a
    plane wave at angle theta from the vertical (the bottom-incident plane
    waves of the paper's layered-model inversion): node j fires the Ricker
    r(t - tau_j), tau_j = (x_j - x_ref) sin(theta) / c, with x_ref the first
    node to fire (all delays >= 0).  Positive theta: the front reaches small
    x first and travels towards +x."""
    xs = np.asarray(xs, dtype=np.float64)
    s = np.sin(np.radians(theta_deg))
    x_ref = xs.min() if s >= 0 else xs.max()
    tau = (xs - x_ref) * s / c
    t = np.arange(nt) * dt
    a = (np.pi * f0 * (t[None, :] - t0 - tau[:, None])) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)
