"""Source applications of the paper (Applications: earthquake location with
the source time function; rupture imaging) on the 2-D acoustic path, and
the bottom-incident plane waves of its layered-model inversion.

A shot may carry up to SG_MAX_SRC source nodes, each with its own wavelet;
adjoint_gradient then returns dJ/dwavelet per node.  The two
parameterisations map a few parameters to those wavelets and back:

* Gaussian footprint f(x, t) = g(t) exp(-|x - x0|^2/(2 sigma^2))/(2 pi
  sigma^2), sigma = dx/2, on the 7 x 7 nodes around the node nearest x0;
* rupture points with f_j(t) = A0_j exp(-(t - t0_j)^2/(2 sigma_t^2)).

Both the wavelets and the chain rules run in the library's kernels; this
module picks the footprint nodes (integer geometry) and marshals arguments.
"""
from __future__ import annotations

import numpy as np
import torch

from . import seisgrad as S


def footprint_nodes(x0, z0, dx, nx, nz, radius=3):
    """Nodes (ix, iz) within `radius` of the node nearest (x0, z0) [m], inside the grid."""
    cx, cz = int(round(x0 / dx)), int(round(z0 / dx))
    return np.array([(ix, iz) for iz in range(cz - radius, cz + radius + 1)
                     for ix in range(cx - radius, cx + radius + 1) if 0 <= ix < nx and 0 <= iz < nz],
                    dtype=np.int32)


class GaussianSource:
    """Wavelets of one shot's footprint nodes and the chain rule back to
    (g(t), x0, z0)."""

    def __init__(self, x0, z0, dx, nx, nz, sigma=None, radius=3):
        self.x0, self.z0, self.dx = float(x0), float(z0), float(dx)
        self.sigma = float(sigma if sigma is not None else dx / 2)
        self.nodes = footprint_nodes(x0, z0, dx, nx, nz, radius)
        self.cells = torch.tensor(self.nodes, device="cuda")

    def wavelets(self, g):
        wav = torch.empty((len(self.nodes), g.numel()), dtype=torch.float32, device=g.device)
        S._check(S.lib().source_gaussian(len(self.nodes), g.numel(), S._ptr(self.cells), self.x0, self.z0,
                                         self.sigma, self.dx, S._ptr(g), S._ptr(wav), S._stream()))
        return wav

    def grad(self, g, gw):
        """(dJ/dg [nt], dJ/dx0, dJ/dz0) from gw = dJ/dwav [nsrc][nt]."""
        dg = torch.empty_like(g)
        dxz = torch.empty(2, dtype=torch.float64, device=g.device)
        S._check(S.lib().source_gaussian_grad(len(self.nodes), g.numel(), S._ptr(self.cells), self.x0, self.z0,
                                              self.sigma, self.dx, S._ptr(g), S._ptr(gw.contiguous()), S._ptr(dg),
                                              S._ptr(dxz), S._stream()))
        d = dxz.cpu().numpy()
        return dg, float(d[0]), float(d[1])


def rupture_wavelets(A0, t0, sigma_t, dt, nt):
    wav = torch.empty((A0.numel(), nt), dtype=torch.float32, device=A0.device)
    S._check(S.lib().source_rupture(A0.numel(), nt, S._ptr(A0), S._ptr(t0), sigma_t, dt, S._ptr(wav), S._stream()))
    return wav


def plane_wave(ix, iz, theta_deg, c, f0, t0, dx, dt, nt):
    """Nodes and wavelets of one plane-wave shot: the row of nodes (ix[j], iz),
    ix consecutive, firing the Ricker wavelet with delays
    (x_j - x_ref) sin(theta)/c (library kernel source_plane_wave).
    Returns (nodes int32 [n][2], wavelets DEVICE FP32 [n][nt])."""
    ix = np.asarray(ix, dtype=np.int64)
    if ix.ndim != 1 or len(ix) < 1 or np.any(np.diff(ix) != 1):
        raise ValueError("plane-wave rows are consecutive nodes")
    nodes = np.stack([ix, np.full_like(ix, iz)], 1).astype(np.int32)
    wav = torch.empty((len(ix), nt), dtype=torch.float32, device="cuda")
    S._check(S.lib().source_plane_wave(len(ix), nt, float(ix[0] * dx), float(dx), float(theta_deg), float(c),
                                       float(f0), float(t0), float(dt), S._ptr(wav), S._stream()))
    return nodes, wav


def rupture_grad(A0, t0, sigma_t, dt, gw):
    dA = torch.empty(A0.numel(), dtype=torch.float64, device=A0.device)
    dt0 = torch.empty_like(dA)
    gw = gw.contiguous()
    S._check(S.lib().source_rupture_grad(A0.numel(), gw.shape[-1], S._ptr(A0), S._ptr(t0), sigma_t, dt, S._ptr(gw),
                                         S._ptr(dA), S._ptr(dt0), S._stream()))
    return dA, dt0


def locate(model_handle_factory, obs, x0, z0, g0, dx, nx, nz, rec, iters=60, lr_x=3.0, decay=0.97,
           fit_location=True, fit_stf=True, log=None):
    """Joint estimate of the location (x0, z0) and the source time function
    g(t) of one shot from its seismograms (the location test of the paper's
    source applications).  Per iteration: forward, misfit and adjoint give
    dJ/dg and dJ/d(x0, z0) through the footprint chain rule; g takes a
    steepest-descent step with the exact line search of the quadratic
    J(g + a p) (one more forward, FP64 inner products in the library); the
    two location coordinates take an Adam step, decaying geometrically by
    `decay` per iteration.  fit_location / fit_stf hold either part fixed.
    model_handle_factory() returns a seisgrad.Model of the velocity (reused).
    Returns (x0, z0, g, history)."""
    m = model_handle_factory()
    g = g0.clone().contiguous()
    mx = np.zeros(2)
    vx = np.zeros(2)
    b1, b2 = 0.9, 0.999
    xz = np.array([x0, z0], dtype=np.float64)
    hist = []
    for it in range(1, iters + 1):
        src = GaussianSource(xz[0], xz[1], dx, nx, nz)
        sh = S.Shots(src.nodes[None], rec, src.wavelets(g)[None].contiguous())
        pred = m.forward(sh, save_ckpt=True)
        J, resid = m.misfit(pred, obs)
        gw = torch.zeros_like(sh.wavelet)
        m.gradient(sh, resid, g_wavelet=gw)
        dg, dxx, dzz = src.grad(g, gw[0])
        hist.append((float(J.item()), float(xz[0]), float(xz[1])))
        if log:
            log(it, hist[-1])
        if fit_stf:
            p = (-dg).contiguous()
            fp = m.forward(S.Shots(src.nodes[None], rec, src.wavelets(p)[None].contiguous()), save_ckpt=False)
            num = S.dot_f64(resid.reshape(-1), fp.reshape(-1)).item()
            den = S.dot_f64(fp.reshape(-1), fp.reshape(-1)).item()
            if den > 0:
                g = (g + (-num / den) * p).contiguous()
        if fit_location:
            d = np.array([dxx, dzz])
            mx = b1 * mx + (1 - b1) * d
            vx = b2 * vx + (1 - b2) * d * d
            step = lr_x * decay ** (it - 1)
            xz -= step * (mx / (1 - b1 ** it)) / (np.sqrt(vx / (1 - b2 ** it)) + 1e-300)
            xz = np.clip(xz, [0.0, 0.0], [(nx - 1) * dx, (nz - 1) * dx])
    return float(xz[0]), float(xz[1]), g, hist
