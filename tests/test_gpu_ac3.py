"""GPU parity of the 3-D acoustic HIP path against the FP64 oracle, and GPU
self-consistency (dot-product identity, checkpointed == store-all bitwise).
Tolerances as in 2-D: seismograms rel-L2 <= 1e-4, gradients <= 1e-3."""
import numpy as np
import pytest
import torch

from gpu_common import O, S, synth, rel_l2, dev

pytestmark = pytest.mark.gpu

SEIS_TOL = 1e-4
GRAD_TOL = 1e-3


def _desc3(nx, ny, nz, P, nt, dt, dx=10.0, vmax=2800.0):
    return S.desc(ndim=3, nx=nx, ny=ny, nz=nz, npml=P, nt=nt, dx=dx, dt=dt, pml_vmax=vmax)


def _grid3(nx, ny, nz, P, nt, dt, dx=10.0, vmax=2800.0):
    return O.grid(ndim=3, nx=nx, ny=ny, nz=nz, npml=P, nt=nt, dx=dx, dt=dt, pml_vmax=vmax)


def _small_case():
    nx, ny, nz, P, nt, dt = 45, 37, 30, 12, 220, 1e-3     # padded 69 x 61 x 54: ragged tiles
    c = 1600.0 + 1200.0 * synth.smooth_random(21, (nz, ny, nx), 3.0, 0.0, 1.0)
    c0 = synth.smooth(c, 4.0)
    src = np.array([[22, 18, 2], [5, 30, 20]], dtype=np.int32)
    xs, ys = np.meshgrid(np.arange(0, nx, 3), np.arange(0, ny, 3), indexing="xy")
    r = np.stack([xs.ravel(), ys.ravel(), np.zeros(xs.size, dtype=int)], -1)
    rec = np.stack([r, r]).astype(np.int32)
    rec[1, :4] = rec[1, 4]                                  # duplicate receivers on one cell
    return (nx, ny, nz, P, nt, dt), c, c0, src, rec


def test_3d_forward_and_gradient_parity():
    (nx, ny, nz, P, nt, dt), c, c0, src, rec = _small_case()
    f0s, t0s = [20.0, 25.0], [0.05, 0.04]
    d = _desc3(nx, ny, nz, P, nt, dt)
    wav = torch.stack([S.ricker(f, t, dt, nt) for f, t in zip(f0s, t0s)])
    sh = S.Shots(src, rec, wav)
    mt = S.Model(d, dev(c), 2, rec.shape[1], 17)
    obs = mt.forward(sh, save_ckpt=False)
    m0 = S.Model(d, dev(c0), 2, rec.shape[1], 17)
    pred = m0.forward(sh)
    J, r = m0.misfit(pred, obs)
    g = m0.gradient(sh, r).cpu().numpy()[0]

    go = _grid3(nx, ny, nz, P, nt, dt)
    wo = np.stack([O.ricker(f, t, dt, nt) for f, t in zip(f0s, t0s)])
    oo = O.ac3_forward(go, c, src, wo, rec)
    op = O.ac3_forward(go, c0, src, wo, rec)
    Jo, ro = O.misfit(op, oo)
    og, _ = O.ac3_gradient(go, c0, src, wo, rec, ro, ckpt=15)
    ga = m0.gradient(sh, dev(ro[:, None])).cpu().numpy()[0]
    e1, e2 = rel_l2(obs.cpu().numpy()[:, 0], oo), rel_l2(pred.cpu().numpy()[:, 0], op)
    e3, e4 = rel_l2(g, og), rel_l2(ga, og)
    print(f"3-D seis {e1:.2e} {e2:.2e} grad {e3:.2e} (adjoint on the oracle residual {e4:.2e}) "
          f"J {J.item():.6e} vs {Jo:.6e}")
    assert e1 <= SEIS_TOL and e2 <= SEIS_TOL
    assert e3 <= GRAD_TOL and e4 <= GRAD_TOL


def test_3d_interior_tiles_two_chunks_parity():
    """A grid with xy tiles beyond the stencil reach of the layer (the tile
    passes' second launch, hx = hy = 0) and two z chunks (64 + 16 planes),
    sources and receivers inside those tiles on interior and slab planes."""
    nx, ny, nz, P, nt, dt = 100, 44, 60, 10, 150, 1e-3     # padded 120 x 64 x 80
    NX, NY = nx + 2 * P, ny + 2 * P
    interior = [(x0, y0) for x0 in range(0, NX, 32) for y0 in range(0, NY, 16)
                if x0 - 4 >= P and x0 + 36 <= P + nx and y0 - 4 >= P and y0 + 20 <= P + ny]
    assert len(interior) >= 4
    c = 1600.0 + 1200.0 * synth.smooth_random(22, (nz, ny, nx), 3.0, 0.0, 1.0)
    c0 = synth.smooth(c, 4.0)
    src = np.array([[50, 22, 2], [60, 20, 40]], dtype=np.int32)
    xs, ys = np.meshgrid(np.arange(0, nx, 4), np.arange(0, ny, 4), indexing="xy")
    surf = np.stack([xs.ravel(), ys.ravel(), np.zeros(xs.size, dtype=int)], -1)
    deep = np.stack([np.arange(30, 80, 2), np.full(25, 24), np.full(25, 30)], -1)
    r = np.concatenate([surf, deep])
    rec = np.stack([r, r]).astype(np.int32)
    d = _desc3(nx, ny, nz, P, nt, dt)
    wav = torch.stack([S.ricker(f, t, dt, nt) for f, t in ((20.0, 0.05), (25.0, 0.04))])
    sh = S.Shots(src, rec, wav)
    obs = S.Model(d, dev(c), 2, rec.shape[1], 14).forward(sh, save_ckpt=False)
    m0 = S.Model(d, dev(c0), 2, rec.shape[1], 14)
    pred = m0.forward(sh)
    J, r_ = m0.misfit(pred, obs)
    g = m0.gradient(sh, r_).cpu().numpy()[0]
    go = _grid3(nx, ny, nz, P, nt, dt)
    wo = np.stack([O.ricker(f, t, dt, nt) for f, t in ((20.0, 0.05), (25.0, 0.04))])
    oo = O.ac3_forward(go, c, src, wo, rec)
    op = O.ac3_forward(go, c0, src, wo, rec)
    _, ro = O.misfit(op, oo)
    og, _ = O.ac3_gradient(go, c0, src, wo, rec, ro, ckpt=14)
    e1, e2 = rel_l2(obs.cpu().numpy()[:, 0], oo), rel_l2(pred.cpu().numpy()[:, 0], op)
    e3 = rel_l2(g, og)
    print(f"3-D interior tiles ({len(interior)}), two chunks: seis {e1:.2e} {e2:.2e} grad {e3:.2e}")
    assert e1 <= SEIS_TOL and e2 <= SEIS_TOL
    assert e3 <= GRAD_TOL


def test_3d_no_layer_parity():
    """npml = 0: no layer passes and no tile within reach of a layer (one
    launch of the interior tile passes), rigid walls at the grid edge."""
    nx, ny, nz, nt, dt = 70, 40, 36, 150, 1e-3
    c = 1600.0 + 1000.0 * synth.smooth_random(23, (nz, ny, nx), 3.0, 0.0, 1.0)
    c0 = synth.smooth(c, 4.0)
    src = np.array([[3, 3, 2], [60, 30, 30]], dtype=np.int32)
    xs, ys = np.meshgrid(np.arange(0, nx, 3), np.arange(0, ny, 3), indexing="xy")
    r = np.stack([xs.ravel(), ys.ravel(), np.zeros(xs.size, dtype=int)], -1)
    rec = np.stack([r, r]).astype(np.int32)
    d = _desc3(nx, ny, nz, 0, nt, dt)
    wav = torch.stack([S.ricker(f, t, dt, nt) for f, t in ((20.0, 0.05), (25.0, 0.04))])
    sh = S.Shots(src, rec, wav)
    obs = S.Model(d, dev(c), 2, rec.shape[1], 12).forward(sh, save_ckpt=False)
    m0 = S.Model(d, dev(c0), 2, rec.shape[1], 12)
    pred = m0.forward(sh)
    J, r_ = m0.misfit(pred, obs)
    g = m0.gradient(sh, r_).cpu().numpy()[0]
    go = _grid3(nx, ny, nz, 0, nt, dt)
    wo = np.stack([O.ricker(f, t, dt, nt) for f, t in ((20.0, 0.05), (25.0, 0.04))])
    oo = O.ac3_forward(go, c, src, wo, rec)
    op = O.ac3_forward(go, c0, src, wo, rec)
    _, ro = O.misfit(op, oo)
    og, _ = O.ac3_gradient(go, c0, src, wo, rec, ro, ckpt=12)
    e1, e2 = rel_l2(obs.cpu().numpy()[:, 0], oo), rel_l2(pred.cpu().numpy()[:, 0], op)
    e3 = rel_l2(g, og)
    print(f"3-D no layer: seis {e1:.2e} {e2:.2e} grad {e3:.2e}")
    assert e1 <= SEIS_TOL and e2 <= SEIS_TOL
    assert e3 <= GRAD_TOL


def test_3d_checkpointed_equals_store_all_and_dot_identity():
    (nx, ny, nz, P, nt, dt), c, c0, src, rec = _small_case()
    nt = 120
    d = _desc3(nx, ny, nz, P, nt, dt)
    s = dev(synth.random_field(3, (2, nt)))
    sh = S.Shots(src, rec, s)
    outs = []
    for K in (nt, 11):
        m = S.Model(d, dev(c), 2, rec.shape[1], K)
        Fs = m.forward(sh)
        gw = torch.zeros((2, nt), dtype=torch.float32, device="cuda")
        g = m.gradient(sh, Fs, g_wavelet=gw)
        outs.append((Fs.clone(), gw.clone(), g.clone()))
        m.close()
    assert torch.equal(outs[0][0], outs[1][0])
    assert torch.equal(outs[0][1], outs[1][1])
    assert torch.equal(outs[0][2], outs[1][2])
    Fs, gw, _ = outs[0]
    lhs = S.dot_f64(Fs.reshape(-1), Fs.reshape(-1)).item()
    rhs = S.dot_f64(s.reshape(-1), gw.reshape(-1)).item()
    print(f"3-D dot test: {lhs:.12e} {rhs:.12e} rel {abs(lhs - rhs) / lhs:.2e}")
    assert abs(lhs - rhs) <= 1e-5 * lhs


def test_c4_full_grid_short_window_parity():
    """The full 400^3 + 24-cell layer launch configuration (448^3 padded,
    200 x 200 surface receivers, 8 Hz Ricker at (200, 200, 2)) over the first
    24 steps, against the oracle on the same grid; then a full-grid
    fwd+adjoint dot identity over 16 steps."""
    cfg = synth.C4
    n = cfg.nx
    c = synth.smooth_3d(4, n)
    src, rec = synth.c4_geometry(n)
    nt = 24
    d = _desc3(n, n, n, cfg.npml, nt, cfg.dt, cfg.dx, vmax=4000.0)
    wav = S.ricker(50.0, 0.02, cfg.dt, nt)[None]          # high-frequency pulse: signal within 24 steps
    sh = S.Shots(src, rec, wav)
    m = S.Model(d, dev(c), 1, rec.shape[1], 5)
    seis = m.forward(sh).cpu().numpy()[0, 0]
    go = _grid3(n, n, n, cfg.npml, nt, cfg.dt, cfg.dx, vmax=4000.0)
    ref = O.ac3_forward(go, c, src, O.ricker(50.0, 0.02, cfg.dt, nt)[None], rec)[0]
    e = rel_l2(seis, ref)
    print(f"C4 full grid, {nt} steps: seis rel-L2 {e:.2e}, max |ref| {np.abs(ref).max():.3e}")
    assert np.abs(ref).max() > 0 and e <= SEIS_TOL
    Fs = m.forward(sh)
    gw = torch.zeros((1, nt), dtype=torch.float32, device="cuda")
    g = m.gradient(sh, Fs, g_wavelet=gw)
    assert torch.isfinite(g).all()
    lhs = S.dot_f64(Fs.reshape(-1), Fs.reshape(-1)).item()
    rhs = S.dot_f64(wav.reshape(-1), gw.reshape(-1)).item()
    print(f"C4 dot test: rel {abs(lhs - rhs) / lhs:.2e}")
    assert abs(lhs - rhs) <= 1e-5 * lhs
