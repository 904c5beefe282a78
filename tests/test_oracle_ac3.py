"""Pins of the FP64 oracle for the 3-D acoustic recursion and its adjoint:
the closed-form 3-D Green's function, discrete energy, dot-product
identities (with the edge/corner terms of the absorbing layer active), brute
force finite differences, reverse-mode AD in torch and checkpointing."""
import math

import numpy as np
import pytest
import torch

from paper_2003_06027_amd import synth
from test_oracle_ac2 import taylor_weights


def _greens(oracle, dt, n=61, f0=15.0, T=0.45, offs=(10, 15, 20)):
    c0, dx = 1500.0, 10.0
    nt = int(round(T / dt))
    g = oracle.grid(ndim=3, nx=n, ny=n, nz=n, npml=0, nt=nt, dx=dx, dt=dt, pml_vmax=c0)
    c = np.full((n, n, n), c0)
    wav = oracle.ricker(f0, 1.0 / f0, dt, nt)[None]
    m = n // 2
    src = np.array([[m, m, m]], dtype=np.int32)
    rec = np.array([[[m + k, m, m] for k in offs]], dtype=np.int32)
    s = oracle.ac3_forward(g, c, src, wav, rec)[0]
    t = (np.arange(nt) + 1) * dt
    errs = []
    for j, k in enumerate(offs):
        ref = oracle.greens3d_ricker(k * dx, c0, t, f0, 1.0 / f0)
        msk = t < (2 * (n - 1 - m) - k) * dx / c0
        errs.append(np.linalg.norm(s[msk, j] - ref[msk]) / np.linalg.norm(ref[msk]))
    return np.array(errs)


def test_forward_matches_3d_greens_function(oracle):
    """u = s(t - r/c) / (4 pi c^2 r) for a point source in 3-D."""
    e1 = _greens(oracle, 1e-3)
    e2 = _greens(oracle, 0.5e-3)
    assert np.all(e1 < 1.2e-2), e1
    assert np.all(e2 < 0.5 * e1), (e1, e2)


def _state(rng, shape, n=6, scale=1.0):
    return [scale * rng.standard_normal(shape) for _ in range(n)]


def _grid3(oracle, n=(9, 8, 7), P=6, nt=40, vmax=2500.0):
    nx, ny, nz = n
    return oracle.grid(ndim=3, nx=nx, ny=ny, nz=nz, npml=P, nt=nt, dx=10.0, dt=1e-3, pml_vmax=vmax)


def test_step_dot_product_identity_3d(oracle):
    g = _grid3(oracle)
    c = 1800.0 + 500.0 * synth.smooth_random(1, (g.nz, g.ny, g.nx), 1.5, 0.0, 1.0)
    cp, zx, zy, zz = oracle.ac3_pad(g, c)
    # edges and corners of the layer are present (products of two or three zetas)
    assert zx.max() > 0 and zy.max() > 0 and zz.max() > 0
    rng = np.random.default_rng(3)
    X = _state(rng, cp.shape)
    aY = _state(rng, cp.shape)
    Y, _ = oracle.ac3_step(g, cp, X)
    aX, _, _ = oracle.ac3_step_T(g, cp, X, aY)
    lhs = sum(np.vdot(a, b) for a, b in zip(Y, aY))
    rhs = sum(np.vdot(a, b) for a, b in zip(X, aX))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def _case3(oracle, nt=50):
    g = _grid3(oracle, nt=nt)
    c = 1800.0 + 500.0 * synth.smooth_random(2, (g.nz, g.ny, g.nx), 1.5, 0.0, 1.0)
    src = np.array([[4, 3, 1], [1, 6, 5]], dtype=np.int32)
    rec = np.array([[[x, y, 0] for x in range(0, 9, 2) for y in range(0, 8, 2)]] * 2, dtype=np.int32)
    wav = np.stack([oracle.ricker(40.0, 0.03, 1e-3, nt), oracle.ricker(35.0, 0.03, 1e-3, nt)])
    return g, c, src, wav, rec


def test_sweep_dot_product_identity_3d(oracle):
    g, c, src, wav, rec = _case3(oracle)
    rng = np.random.default_rng(4)
    s = rng.standard_normal(wav.shape)
    d = rng.standard_normal((2, g.nt, rec.shape[1]))
    Fs = oracle.ac3_forward(g, c, src, s, rec)
    _, _, FTd = oracle.ac3_gradient(g, c, src, s, rec, d, ckpt=7, want_wav=True)
    lhs, rhs = np.vdot(Fs, d), np.vdot(s, FTd)
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_gradient_fd_and_checkpointing_3d(oracle):
    g, c, src, wav, rec = _case3(oracle, nt=40)
    ct = c.copy()
    ct[2:5, 2:6, 3:7] += 120.0
    dobs = oracle.ac3_forward(g, ct, src, wav, rec)
    pred = oracle.ac3_forward(g, c, src, wav, rec)
    J, r = oracle.misfit(pred, dobs)
    grad, _ = oracle.ac3_gradient(g, c, src, wav, rec, r, ckpt=0)
    grad_k, _ = oracle.ac3_gradient(g, c, src, wav, rec, r, ckpt=6)
    assert np.array_equal(grad, grad_k)
    rng = np.random.default_rng(5)
    cells = [tuple(rng.integers(0, s) for s in c.shape) for _ in range(12)]
    cells += [(0, 0, 0), (g.nz - 1, g.ny - 1, g.nx - 1), (0, 3, g.nx - 1)]  # folded layer cells

    def Jat(cell, h):
        cc = c.copy()
        cc[cell] += h
        return oracle.misfit(oracle.ac3_forward(g, cc, src, wav, rec), dobs)[0]

    for cell in cells:
        h = 1e-4 * c[cell]
        fd = (8 * (Jat(cell, h) - Jat(cell, -h)) - (Jat(cell, 2 * h) - Jat(cell, -2 * h))) / (12 * h)
        assert fd == pytest.approx(grad[cell], rel=1e-6, abs=1e-9 * np.abs(grad).max()), cell


def _torch_forward3(c_pad, zx, zy, zz, dt, dx, nt, sidx, wav, ridx):
    """The same discrete 3-D recursion in torch FP64 ops (for reverse-mode AD)."""
    w2 = torch.tensor(taylor_weights(2, range(-4, 5)), dtype=torch.float64)
    w1 = torch.tensor(taylor_weights(1, range(-4, 5)), dtype=torch.float64)
    NZ, NY, NX = c_pad.shape
    zx = torch.tensor(zx)[None, None, :]
    zy = torch.tensor(zy)[None, :, None]
    zz = torch.tensor(zz)[:, None, None]
    zeta = [zx, zy, zz]

    def shift(a, axis, m):
        p = torch.nn.functional.pad(a, (4, 4, 4, 4, 4, 4))
        sl = [slice(4, 4 + NZ), slice(4, 4 + NY), slice(4, 4 + NX)]
        ax = {0: 2, 1: 1, 2: 0}[axis]
        n = (NX, NY, NZ)[axis]
        sl[ax] = slice(4 + m, 4 + m + n)
        return p[tuple(sl)]

    def lap(a):
        return sum(w2[m + 4] * (shift(a, 0, m) + shift(a, 1, m) + shift(a, 2, m)) for m in range(-4, 5)) / dx ** 2

    def d(a, axis):
        return sum(w1[m + 4] * shift(a, axis, m) for m in range(-4, 5)) / dx

    s1 = zx + zy + zz
    s2 = zx * zy + zy * zz + zz * zx
    s3 = zx * zy * zz
    alpha = 1.0 / (1.0 + 0.5 * s1 * dt)
    beta, gamma = 2.0 - dt * dt * s2, 1.0 - 0.5 * s1 * dt
    C = dt * dt * c_pad ** 2
    z = torch.zeros(NZ, NY, NX, dtype=torch.float64)
    u, um, psi = z.clone(), z.clone(), z.clone()
    ph = [z.clone(), z.clone(), z.clone()]
    out = []
    for k in range(nt):
        w = lap(u) + d(ph[0], 0) + d(ph[1], 1) + d(ph[2], 2)
        f = torch.zeros(NZ, NY, NX, dtype=torch.float64)
        f[sidx] = wav[k] / dx ** 3
        un = alpha * (beta * u - gamma * um - dt * dt * s3 * psi + C * w + dt * dt * f)
        psin = psi + dt * un
        new = []
        for j in range(3):
            oth = s1 - 2 * zeta[j]
            prod = zeta[(j + 1) % 3] * zeta[(j + 2) % 3]
            new.append(((1 - 0.5 * zeta[j] * dt) * ph[j] + dt * (oth * d(un, j) + prod * d(psin, j)))
                       / (1 + 0.5 * zeta[j] * dt))
        ph, um, u, psi = new, u, un, psin
        out.append(torch.stack([u[r] for r in ridx]))
    return torch.stack(out)


def test_adjoint_equals_reverse_mode_ad_3d(oracle):
    g, c, src, wav, rec = _case3(oracle, nt=25)
    P = g.npml
    cp, zx, zy, zz = oracle.ac3_pad(g, c)
    dobs = oracle.ac3_forward(g, c * 0.96, src[:1], wav[:1], rec[:1])
    cphys = torch.tensor(c, requires_grad=True)
    iz = np.clip(np.arange(cp.shape[0]) - P, 0, g.nz - 1)
    iy = np.clip(np.arange(cp.shape[1]) - P, 0, g.ny - 1)
    ix = np.clip(np.arange(cp.shape[2]) - P, 0, g.nx - 1)
    c_pad = cphys[iz][:, iy][:, :, ix]
    sidx = (int(src[0, 2]) + P, int(src[0, 1]) + P, int(src[0, 0]) + P)
    ridx = [(int(r[2]) + P, int(r[1]) + P, int(r[0]) + P) for r in rec[0]]
    dd = _torch_forward3(c_pad, zx, zy, zz, g.dt, g.dx, g.nt, sidx, torch.tensor(wav[0]), ridx)
    J = 0.5 * ((dd - torch.tensor(dobs[0])) ** 2).sum()
    J.backward()
    pred = oracle.ac3_forward(g, c, src[:1], wav[:1], rec[:1])
    Jo, r = oracle.misfit(pred, dobs)
    grad, _ = oracle.ac3_gradient(g, c, src[:1], wav[:1], rec[:1], r)
    assert float(J.detach()) == pytest.approx(Jo, rel=1e-12)
    ad = cphys.grad.numpy()
    assert np.linalg.norm(ad - grad) / np.linalg.norm(ad) < 1e-10


def test_energy_conservation_rigid_no_pml_3d(oracle):
    n, dx, dt = 16, 10.0, 1e-3
    g = oracle.grid(ndim=3, nx=n, ny=n, nz=n, npml=0, nt=1, dx=dx, dt=dt, pml_vmax=3000.0)
    c = 1500.0 + 1000.0 * synth.smooth_random(7, (n, n, n), 2.0, 0.0, 1.0)
    win = np.hanning(n)
    u0 = synth.smooth_random(8, (n, n, n), 1.5, -1.0, 1.0) * win[:, None, None] * win[None, :, None] * win[None, None, :]
    z = np.zeros_like(u0)
    X = [u0, u0 * 0.999, z, z, z, z]
    w = taylor_weights(2, range(-4, 5))

    def lapi(u):
        up = np.pad(u, 4)
        out = np.zeros_like(u)
        for m in range(-4, 5):
            out += w[m + 4] * (up[4 + m:4 + m + n, 4:4 + n, 4:4 + n] + up[4:4 + n, 4 + m:4 + m + n, 4:4 + n]
                               + up[4:4 + n, 4:4 + n, 4 + m:4 + m + n])
        return out / dx ** 2

    E = []
    for k in range(300):
        Y, _ = oracle.ac3_step(g, c, X)
        v = (Y[0] - X[0]) / dt
        E.append(0.5 * np.sum(v * v / c ** 2) + 0.5 * np.sum(Y[0] * -lapi(X[0])))
        X = Y
    E = np.array(E)
    assert np.max(np.abs(E - E[0])) / abs(E[0]) < 1e-11


def _homog3(oracle, n, P, src, rec, nt, f0, R=1e-3, c0=2000.0):
    g = oracle.grid(ndim=3, nx=n, ny=n, nz=n, npml=P, nt=nt, dx=10.0, dt=1e-3, pml_vmax=c0, pml_R=R)
    wav = oracle.ricker(f0, 1.0 / f0, 1e-3, nt)[None]
    return oracle.ac3_forward(g, np.full((n, n, n), c0), np.array([src], dtype=np.int32), wav,
                              np.array([rec], dtype=np.int32))[0]


def _layer_reflection(oracle, n, P, src, rec, f0, R=1e-3, pad=1):
    """Per-receiver rel-L2 of (run with the layer - run on a grid pad*n cells
    larger on every side without one), over the window before the larger
    grid's rigid walls can send anything back to a receiver."""
    off = pad * n
    nt = int((min(src) + off + min(min(r) for r in rec) + off) * 10.0 / 2000.0 / 1e-3)
    small = _homog3(oracle, n, P, src, rec, nt, f0, R)
    big = _homog3(oracle, (2 * pad + 1) * n, 0, [x + off for x in src], [[x + off for x in r] for r in rec], nt, f0, R)
    return np.linalg.norm(small - big, axis=0) / np.linalg.norm(big, axis=0)


def test_pml_absorbs_3d(oracle):
    """The 3-D layer with its edge (two damped axes) and corner (three) terms:
    a source 7 cells from a corner of the physical cube, receivers beside an
    edge, a face and the far corner; reflection against a 3x larger domain
    over the same window <= 1e-2 per receiver (measured 1.8e-3 to 6.8e-3)."""
    n = 24
    ratio = _layer_reflection(oracle, n, 10, [7, 7, 7],
                              [[2, 2, 2], [19, 2, 7], [7, n - 3, 2], [n - 3, n - 3, n - 3]], 15.0)
    assert np.all(ratio < 1e-2), ratio


def test_pml_corner_terms_3d(oracle):
    """A thick, strong layer (P = 20, R = 1e-6) and an 8 Hz wavelet starting 2
    cells from a corner, receivers in the corner and along its edges: the
    continuous layer is reflectionless, so what remains is discretisation
    error (measured 0.75e-3 to 2.9e-3).  The bar 4e-3 fails if the corner
    term s3*psi (8.3e-3) or the edge terms (prod zeta)*D psi (1.2e-2) are
    dropped or have their sign flipped (1.5e-2, 2.3e-2), or if the phi
    coefficient (sum of the other zetas - zeta_j) loses its -zeta_j (0.41):
    those mistakes make the corner and edge regions a non-matched layer."""
    ratio = _layer_reflection(oracle, 12, 20, [2, 2, 2], [[0, 0, 0], [2, 0, 0], [8, 8, 0]], 8.0, R=1e-6, pad=4)
    assert np.all(ratio < 4e-3), ratio


def test_pml_long_run_stable_3d(oracle):
    """Random state in every layer cell (faces, edges, corners), no source,
    3000 steps at 0.95 of the reference velocity: the field decays at every
    checkpoint and ends below 1e-3 of its start (measured 3.6e-5).  A flipped
    sign of s3*psi or of the edge terms grows without bound here."""
    n = 10
    g = oracle.grid(ndim=3, nx=n, ny=n, nz=n, npml=8, nt=1, dx=10.0, dt=1e-3, pml_vmax=4200.0)
    cp, zx, zy, zz = oracle.ac3_pad(g, np.full((n, n, n), 0.95 * 4200.0))
    rng = np.random.default_rng(2)
    mask = (zx[None, None, :] + zy[None, :, None] + zz[:, None, None]) > 0
    X = [rng.standard_normal(cp.shape) * mask for _ in range(2)] + [np.zeros(cp.shape)] * 4
    norms = [np.linalg.norm(X[0])]
    for k in range(1, 3001):
        X, _ = oracle.ac3_step(g, cp, X)
        if k % 250 == 0:
            norms.append(np.linalg.norm(X[0]))
    norms = np.array(norms)
    assert np.all(norms[1:] < norms[:-1]), norms
    assert norms[-1] < 1e-3 * norms[0], norms


def test_damping_profiles_3d_follow_definition(oracle):
    """zeta(d) = zeta_max (d/P)^2, zeta_max = 3 vmax ln(1/R) / (2 P dx), d the
    depth into the layer (1 on the first layer cell, P on the outermost), zero
    on the physical cells; each axis uses its own length."""
    g = oracle.grid(ndim=3, nx=9, ny=5, nz=7, npml=6, nt=1, dx=12.5, dt=1e-3, pml_vmax=3300.0, pml_R=1e-4)
    _, zx, zy, zz = oracle.ac3_pad(g, np.full((7, 5, 9), 2000.0))
    zmax = 3.0 * 3300.0 * np.log(1e4) / (2.0 * 6 * 12.5)
    for z, n in ((zx, 9), (zy, 5), (zz, 7)):
        i = np.arange(n + 12)
        depth = np.where(i < 6, 6 - i, np.where(i >= 6 + n, i - (5 + n), 0))
        assert np.allclose(z, zmax * (depth / 6.0) ** 2, rtol=1e-15, atol=0)
        assert z[6:6 + n].max() == 0.0 and z[0] == z[-1] == pytest.approx(zmax, rel=1e-15)
