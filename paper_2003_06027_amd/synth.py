"""Seeded synthetic inputs: velocity models, acquisition geometry, configs.

This module is the only code shared by the GPU path's tests and the CPU
oracle.  It generates inputs (models, source and receiver positions, wavelet
parameters) and contains none of the wave-propagation arithmetic: no
stencils, no time stepping, no adjoint, no wavelet evaluation.

Models are float64 numpy arrays, row-major [iz][ix] (2-D) or [iz][iy][ix]
(3-D), x fastest, z pointing down, 0-based indices.  Geometry arrays are
int32: sources [nshots][ndim] and receivers [nshots][nrec][ndim] with
coordinates ordered (ix, iz) in 2-D and (ix, iy, iz) in 3-D.

The paper's own FWI models (Marmousi; a layered crust with elliptical
anomalies) are not available here; the layered / anomaly / smooth-random
generators below stand in for them with comparable velocity ranges and
structure.
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy.ndimage import gaussian_filter


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    ndim: int
    nx: int
    nz: int
    ny: int = 1
    dx: float = 10.0
    dt: float = 1e-3
    nt: int = 500
    npml: int = 20
    f0: float = 10.0          # Ricker peak frequency (Hz)
    t0: float | None = None   # Ricker delay; None -> 1/f0
    nshots: int = 1
    physics: str = "acoustic"
    pml_R: float = 1e-3
    f0_pml: float = 10.0

    @property
    def ricker_t0(self) -> float:
        return 1.0 / self.f0 if self.t0 is None else self.t0

    @property
    def padded(self):
        p = 2 * self.npml
        if self.ndim == 2:
            return (self.nz + p, self.nx + p)
        return (self.nz + p, self.ny + p, self.nx + p)

    @property
    def padded_cells(self) -> int:
        return int(np.prod(self.padded))

    def replace(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)


# Workloads: 2-D acoustic layered (C1), 2-D acoustic dipping layers +
# anomalies with 64 shots (C2), 2-D elastic (C3), 3-D acoustic (C4).
C1 = Config("acoustic2d_101x101_nt500", 2, nx=101, nz=101, dx=10.0, dt=1e-3, nt=500,
            npml=20, f0=10.0, nshots=1)
C2 = Config("acoustic2d_1000x500_nt4000_64shots", 2, nx=1000, nz=500, dx=10.0, dt=0.8e-3,
            nt=4000, npml=32, f0=8.0, nshots=64)
C3 = Config("elastic2d_800x400_nt3000_16shots", 2, nx=800, nz=400, dx=5.0, dt=0.5e-3,
            nt=3000, npml=20, f0=10.0, nshots=16, physics="elastic", f0_pml=10.0)
C4 = Config("acoustic3d_400cube_nt2000", 3, nx=400, ny=400, nz=400, dx=10.0, dt=1e-3,
            nt=2000, npml=24, f0=8.0, nshots=1)
CONFIGS = {"c1": C1, "c2": C2, "c3": C3, "c4": C4}


# ------------------------------------------------------------------ models
def layered_c1(nx: int = 101, nz: int = 101) -> np.ndarray:
    """Three flat layers 1500 / 2200 / 3000 m/s split at thirds of the depth."""
    v = np.empty((nz, nx))
    z = np.arange(nz)
    v[z < 34] = 1500.0
    v[(z >= 34) & (z < 67)] = 2200.0
    v[z >= 67] = 3000.0
    return v


def smooth(v: np.ndarray, sigma: float = 10.0) -> np.ndarray:
    """Initial model of an inversion: Gaussian blur of the true model."""
    return gaussian_filter(v, sigma=sigma, mode="nearest")


def random_layered(seed: int, nx: int = 101, nz: int = 101) -> np.ndarray:
    """A 'C1-style' three-layer model with random interface depths and
    velocities (training / evaluation models of the learned preconditioner)."""
    rng = np.random.default_rng(seed)
    z1 = rng.uniform(20, 45)
    z2 = z1 + rng.uniform(20, 40)
    v1, v2, v3 = rng.uniform(1450, 1650), rng.uniform(1950, 2450), rng.uniform(2700, 3300)
    z = np.arange(nz)[:, None] * np.ones((1, nx))
    return np.where(z < z1, v1, np.where(z < z2, v2, v3)).astype(np.float64)


def dipping_layers_anomalies(seed: int = 2003, nx: int = 1000, nz: int = 500,
                             dx: float = 10.0) -> np.ndarray:
    """12 dipping interfaces plus 20 Gaussian anomalies, clipped to 1500-4500 m/s."""
    rng = np.random.default_rng(seed)
    x = np.arange(nx) * dx
    zc = np.arange(nz) * dx
    L = nx * dx
    H = nz * dx
    z0 = np.sort(rng.uniform(0.03 * H, 0.97 * H, size=12))
    theta = np.deg2rad(rng.uniform(-12.0, 12.0, size=12))
    base = 1500.0 + 3000.0 * (np.arange(13) / 12.0) ** 0.8 + rng.uniform(-150, 150, size=13)
    Z = zc[:, None] * np.ones((1, nx))
    layer = np.zeros((nz, nx), dtype=np.int64)
    for i in range(12):
        zi = z0[i] + (x - 0.5 * L) * np.tan(theta[i])
        layer += (Z > zi[None, :]).astype(np.int64)
    v = base[layer]
    X = np.ones((nz, 1)) * x[None, :]
    for _ in range(20):
        cx = rng.uniform(0, L)
        cz = rng.uniform(0.1 * H, H)
        sg = rng.uniform(40.0, 250.0)
        amp = rng.uniform(-400.0, 400.0)
        v = v + amp * np.exp(-((X - cx) ** 2 + (Z - cz) ** 2) / (2 * sg * sg))
    return np.clip(v, 1500.0, 4500.0)


def layered_ellipses(seed: int = 250, nx: int = 300, nz: int = 150, dx: float = 20.0, nlayers: int = 5,
                     nellipses: int = 4) -> np.ndarray:
    """A layered crust with embedded elliptical anomalies (stand-in for the
    paper's second FWI model, whose parameters are not given): flat layers
    with velocity increasing with depth (2500 -> 4500 m/s, random interface
    depths), plus ellipses of +-8..15 % velocity contrast with random centres,
    semi-axes and tilts, in the middle of the section."""
    rng = np.random.default_rng(seed)
    H, L = nz * dx, nx * dx
    zi = np.sort(rng.uniform(0.15 * H, 0.9 * H, size=nlayers - 1))
    vel = np.linspace(2500.0, 4500.0, nlayers) + rng.uniform(-100, 100, size=nlayers)
    X = np.ones((nz, 1)) * (np.arange(nx) * dx)[None, :]
    Z = (np.arange(nz) * dx)[:, None] * np.ones((1, nx))
    v = vel[np.searchsorted(zi, Z)]
    for _ in range(nellipses):
        cx, cz = rng.uniform(0.2 * L, 0.8 * L), rng.uniform(0.3 * H, 0.75 * H)
        a, b = rng.uniform(0.06 * L, 0.12 * L), rng.uniform(0.05 * H, 0.1 * H)
        th = rng.uniform(-0.5, 0.5)
        xr = (X - cx) * np.cos(th) + (Z - cz) * np.sin(th)
        zr = -(X - cx) * np.sin(th) + (Z - cz) * np.cos(th)
        inside = (xr / a) ** 2 + (zr / b) ** 2 <= 1.0
        v = np.where(inside, v * (1.0 + rng.choice([-1.0, 1.0]) * rng.uniform(0.08, 0.15)), v)
    return v


def smooth_random(seed: int, shape, sigma: float, vmin: float, vmax: float) -> np.ndarray:
    """Gaussian-filtered N(0,1) noise mapped affinely onto [vmin, vmax]."""
    rng = np.random.default_rng(seed)
    n = gaussian_filter(rng.standard_normal(shape), sigma=sigma, mode="wrap")
    n = (n - n.min()) / (n.max() - n.min())
    return vmin + (vmax - vmin) * n


def elastic_c3(seed: int = 6027, nx: int = 800, nz: int = 400):
    """vp from blurred noise in [1800, 4000]; vs = vp/1.73 with +-10 % noise;
    rho from Gardner's relation rho = 310 vp^0.25 (kg/m^3)."""
    vp = smooth_random(seed, (nz, nx), 15.0, 1800.0, 4000.0)
    rng = np.random.default_rng(seed + 1)
    vs = vp / 1.73 * (1.0 + rng.uniform(-0.1, 0.1, size=vp.shape))
    rho = 310.0 * vp ** 0.25
    return vp, vs, rho


def smooth_3d(seed: int = 4, n: int = 400) -> np.ndarray:
    return smooth_random(seed, (n, n, n), 12.0, 1500.0, 4000.0)


# ---------------------------------------------------------------- geometry
def surface_receivers_2d(nshots: int, nx: int, iz: int = 0, step: int = 1) -> np.ndarray:
    xs = np.arange(0, nx, step, dtype=np.int32)
    r = np.stack([xs, np.full_like(xs, iz)], axis=-1)
    return np.ascontiguousarray(np.broadcast_to(r, (nshots,) + r.shape)).astype(np.int32)


def c1_geometry():
    src = np.array([[50, 2]], dtype=np.int32)
    return src, surface_receivers_2d(1, 101)


def c2_geometry(nshots: int = 64, nx: int = 1000):
    ix = np.round((np.arange(nshots) + 0.5) * nx / nshots).astype(np.int32)
    src = np.stack([ix, np.full_like(ix, 2)], axis=-1).astype(np.int32)
    return src, surface_receivers_2d(nshots, nx)


def c3_geometry(seed: int = 6027, nx: int = 800):
    """Shots 0-7 explosive at depth 5, shots 8-15 double couples at depth 200;
    moment tensors (Mxx, Mzz, Mxz); 800 two-component surface receivers."""
    rng = np.random.default_rng(seed + 2)
    src = []
    mt = []
    for i in range(16):
        if i < 8:
            src.append((50 + 100 * i, 5))
            mt.append((1.0, 1.0, 0.0))
        else:
            th = rng.uniform(0.0, np.pi)
            src.append((50 + 100 * (i - 8), 200))
            mt.append((-np.sin(2 * th), np.sin(2 * th), np.cos(2 * th)))
    return (np.array(src, dtype=np.int32), np.array(mt, dtype=np.float64),
            surface_receivers_2d(16, nx))


def c4_geometry(n: int = 400):
    src = np.array([[n // 2, n // 2, 2]], dtype=np.int32)
    xs = np.arange(0, n, 2, dtype=np.int32)
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    rec = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size, dtype=np.int32)], axis=-1)
    return src, rec[None].astype(np.int32)


def random_field(seed: int, shape, scale: float = 1.0) -> np.ndarray:
    """Plain N(0, scale^2) values (dot tests, random seismogram adjoints)."""
    return scale * np.random.default_rng(seed).standard_normal(shape)
