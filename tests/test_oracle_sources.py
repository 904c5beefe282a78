"""Pins of the oracle's several-source-cells path and of the source
parameterisations: superposition (the forward map is linear in the
sources), a point source split into two coincident halves, the adjoint dot
identity of the wavelets -> seismograms map, and the chain rules for the
Gaussian earthquake location (g(t), x0, z0) and the rupture (A0, t0)
against central differences of the misfit."""
import numpy as np
import pytest

from oracle import pyoracle as O
from oracle import sources as SRC

NX, NZ, P, NT, DX, DT = 60, 50, 10, 260, 10.0, 1e-3


def _grid():
    return O.grid(ndim=2, nx=NX, nz=NZ, npml=P, nt=NT, dx=DX, dt=DT, pml_vmax=3000.0)


def _model():
    z = np.arange(NZ)[:, None] * np.ones((1, NX))
    return np.where(z < 25, 1800.0, 2500.0) + 10.0 * np.sin(np.arange(NX) / 7.0)[None, :]


def _rec():
    return np.array([[[ix, 0] for ix in range(0, NX, 3)]], dtype=np.int32)


def test_superposition_and_coincident_split():
    g, c, rec = _grid(), _model(), _rec()
    r = O.ricker(15.0, 1 / 15.0, DT, NT)
    a = O.ac2_forward(g, c, np.array([[20, 30]], np.int32), r[None], rec)
    b = O.ac2_forward(g, c, np.array([[41, 12]], np.int32), 0.5 * r[None], rec)
    ab = O.ac2_forward_ms(g, c, np.array([[[20, 30], [41, 12]]], np.int32), np.stack([r, 0.5 * r])[None], rec)
    assert np.abs(ab - (a + b)).max() <= 1e-13 * np.abs(a + b).max()
    half = O.ac2_forward_ms(g, c, np.array([[[20, 30], [20, 30]]], np.int32), np.stack([0.5 * r, 0.5 * r])[None], rec)
    assert np.abs(half - a).max() <= 1e-13 * np.abs(a).max()


def test_several_sources_adjoint_dot_identity():
    g, c, rec = _grid(), _model(), _rec()
    rng = np.random.default_rng(0)
    src = np.array([[[15, 20], [16, 20], [30, 35], [50, 5]]], np.int32)
    wav = rng.standard_normal((1, 4, NT))
    d = rng.standard_normal((1, NT, rec.shape[1]))
    seis = O.ac2_forward_ms(g, c, src, wav, rec)
    _, _, gw = O.ac2_gradient_ms(g, c, src, np.zeros_like(wav), rec, d)   # J = <seis, d> is linear
    lhs, rhs = float((seis * d).sum()), float((wav * gw).sum())
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def _J(c, src, wav, rec, obs):
    return 0.5 * float(((O.ac2_forward_ms(_grid(), c, src, wav, rec) - obs) ** 2).sum())


def test_gaussian_location_chain_rule_matches_central_differences():
    c, rec = _model(), _rec()
    sigma = DX / 2
    r = O.ricker(15.0, 1 / 15.0, DT, NT)
    cells_t, w_t = SRC.gaussian_footprint(302.0, 251.0, sigma, DX, NX, NZ)
    obs = O.ac2_forward_ms(_grid(), c, cells_t[None], SRC.gaussian_wavelets(r, w_t)[None], rec)
    x0, z0 = 296.7, 244.1                          # nearest node (30, 24) stays fixed under the steps below
    g = 0.9 * r
    cells, w = SRC.gaussian_footprint(x0, z0, sigma, DX, NX, NZ)
    wav = SRC.gaussian_wavelets(g, w)
    seis = O.ac2_forward_ms(_grid(), c, cells[None], wav[None], rec)
    _, _, gw = O.ac2_gradient_ms(_grid(), c, cells[None], wav[None], rec, seis - obs)
    dg, dx0, dz0 = SRC.gaussian_grad(gw[0], g, cells, x0, z0, sigma, DX)
    h = 0.05                                       # 4th-order central differences
    for name, grad, f in (("x0", dx0, lambda e: SRC.gaussian_footprint(x0 + e, z0, sigma, DX, NX, NZ)),
                          ("z0", dz0, lambda e: SRC.gaussian_footprint(x0, z0 + e, sigma, DX, NX, NZ))):
        J = lambda e: _J(c, f(e)[0][None], SRC.gaussian_wavelets(g, f(e)[1])[None], rec, obs)
        fd = (8 * (J(h) - J(-h)) - (J(2 * h) - J(-2 * h))) / (12 * h)
        assert abs(fd - grad) <= 1e-6 * abs(grad), (name, fd, grad)
    # the source time function: J is quadratic in g, so FD along a direction is exact up to rounding
    v = np.random.default_rng(1).standard_normal(NT)
    eps = 1e-3 * np.abs(g).max()
    Jp = _J(c, cells[None], SRC.gaussian_wavelets(g + eps * v, w)[None], rec, obs)
    Jm = _J(c, cells[None], SRC.gaussian_wavelets(g - eps * v, w)[None], rec, obs)
    assert abs((Jp - Jm) / (2 * eps) - dg @ v) <= 1e-8 * abs(dg @ v)


def test_rupture_chain_rule_matches_central_differences():
    c, rec = _model(), _rec()
    src = np.array([[[10 + 8 * j, 20] for j in range(4)]], np.int32)
    st = 0.01
    A_t, t_t = np.array([1.0, 0.8, 1.2, 0.6]), np.array([0.04, 0.06, 0.08, 0.10])
    obs = O.ac2_forward_ms(_grid(), c, src, SRC.rupture_wavelets(A_t, t_t, st, DT, NT)[None], rec)
    A0, t0 = np.full(4, 0.9), np.full(4, 0.07)
    wav = SRC.rupture_wavelets(A0, t0, st, DT, NT)
    seis = O.ac2_forward_ms(_grid(), c, src, wav[None], rec)
    _, _, gw = O.ac2_gradient_ms(_grid(), c, src, wav[None], rec, seis - obs)
    dA, dt0 = SRC.rupture_grad(gw[0], A0, t0, st, DT)
    for j in (0, 2):
        e = np.zeros(4)
        e[j] = 1.0
        hA, ht = 1e-4, 1e-6
        fdA = (_J(c, src, SRC.rupture_wavelets(A0 + hA * e, t0, st, DT, NT)[None], rec, obs)
               - _J(c, src, SRC.rupture_wavelets(A0 - hA * e, t0, st, DT, NT)[None], rec, obs)) / (2 * hA)
        fdt = (_J(c, src, SRC.rupture_wavelets(A0, t0 + ht * e, st, DT, NT)[None], rec, obs)
               - _J(c, src, SRC.rupture_wavelets(A0, t0 - ht * e, st, DT, NT)[None], rec, obs)) / (2 * ht)
        assert fdA == pytest.approx(dA[j], rel=1e-6)
        assert fdt == pytest.approx(dt0[j], rel=1e-5)
