"""Helpers of the GPU parity tests: run the HIP path through the C ABI and
the FP64 oracle on the same seeded inputs."""
import numpy as np
import torch

from oracle import pyoracle as O
from paper_2003_06027_amd import seisgrad as S
from paper_2003_06027_amd import synth


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_grid(cfg, pml_vmax, nt=None):
    return O.grid(ndim=2, nx=cfg.nx, nz=cfg.nz, npml=cfg.npml, nt=nt or cfg.nt, dx=cfg.dx,
                  dt=cfg.dt, pml_R=cfg.pml_R, pml_vmax=pml_vmax)


def gpu_desc(cfg, pml_vmax, nt=None, nmodels=1):
    return S.desc(ndim=2, nx=cfg.nx, nz=cfg.nz, npml=cfg.npml, nt=nt or cfg.nt, nmodels=nmodels,
                  dx=cfg.dx, dt=cfg.dt, pml_R=cfg.pml_R, pml_vmax=pml_vmax)


def gpu_wavelets(f0s, t0s, dt, nt):
    return torch.stack([S.ricker(f, t, dt, nt) for f, t in zip(f0s, t0s)])


def oracle_wavelets(f0s, t0s, dt, nt):
    return np.stack([O.ricker(f, t, dt, nt) for f, t in zip(f0s, t0s)])


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")
