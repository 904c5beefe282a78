"""GPU parity of the divergence-form 2-D acoustic path (u_tt = div(c^2
grad u) + f, physics SG_ACOUSTIC_DIV, through the C ABI) against the FP64
oracle, and its self-consistency:

* point sources, two models batched, a grid of several tiles with ragged
  tails: seismograms rel-L2 <= 1e-4, gradient and dJ/dwavelet <= 1e-3;
* bottom-incident plane waves at -30, -10, 10, 30 degrees on a layered model
  with elliptical anomalies: the library's plane-wave wavelets against the
  oracle's (<= 1e-6), then seismograms and gradient as above; checkpoint
  interval, stored segments and repetition leave every output bitwise
  unchanged;
* without the layer, source-receiver reciprocity (FP32 rounding, <= 1e-5),
  and the sweep's dot identity <seis, d> = <wav, dJ/dwav> (<= 1e-5);
* a full 600 x 300 grid in a short window, on sampled traces and the whole
  gradient;
* the paper's layered-model inversion in small: L-BFGS from a smoothed model
  with the four plane waves lowers the misfit and the model error.
"""
import numpy as np
import pytest
import torch

from gpu_common import O, S, synth, rel_l2, dev
from oracle import sources as OSRC
from paper_2003_06027_amd import fwi
from paper_2003_06027_amd import sources as SRC

pytestmark = pytest.mark.gpu

SEIS_TOL, GRAD_TOL = 1e-4, 1e-3


def _desc(nx, nz, P, nt, dx, dt, nmodels=1, vmax=3000.0):
    return S.desc(ndim=2, physics=S.SG_ACOUSTIC_DIV, nx=nx, nz=nz, npml=P, nt=nt, nmodels=nmodels, dx=dx, dt=dt,
                  pml_R=1e-3, pml_vmax=vmax, f0_pml=10.0)


def _grid(nx, nz, P, nt, dx, dt, vmax=3000.0):
    return O.grid(ndim=2, nx=nx, nz=nz, npml=P, nt=nt, dx=dx, dt=dt, pml_R=1e-3, pml_vmax=vmax, f0_pml=10.0)


def _gpu_run(d, c, c_obs, sh, ckpt=0, store=0, want_gw=False):
    """forward on c_obs (data), then forward + misfit + adjoint on c."""
    ns, nrec = sh.nshots, sh.nrec
    mo = S.Model(d, dev(c_obs), ns, nrec, ckpt)
    obs = mo.forward(sh, save_ckpt=False).clone()
    m = S.Model(d, dev(c), ns, nrec, ckpt, store_segments=store)
    pred = m.forward(sh, save_ckpt=True)
    J, resid = m.misfit(pred, obs)
    gw = torch.zeros_like(sh.wavelet) if want_gw else None
    g = m.gradient(sh, resid, g_wavelet=gw)
    torch.cuda.synchronize()
    out = dict(obs=obs.cpu().numpy()[:, 0], pred=pred.cpu().numpy()[:, 0], J=float(J.item()), grad=g.cpu().numpy())
    if want_gw:
        out["gw"] = gw.cpu().numpy()
    mo.close()
    m.close()
    return out


def test_point_sources_two_models_parity():
    nx, nz, P, nt, dx, dt = 200, 120, 12, 500, 10.0, 1e-3
    B, spm = 2, 2
    c = np.stack([synth.smooth_random(11 + b, (nz, nx), 5.0, 1800.0, 2900.0) for b in range(B)])
    ct = c.copy()
    ct[:, 25:45, 40:160] *= 1.06      # residuals of 2-13 % of the data (FP32 differences stay accurate)
    src = np.array([[30, 4], [170, 6], [100, 2], [60, 90]], np.int32)
    rec = np.stack([np.array([[ix, 1] for ix in range(0, nx, 3)] + [[nx - 1, nz - 1]], np.int32)] * (B * spm))
    f0s, t0s = [15.0, 12.0, 18.0, 15.0], [0.07, 0.09, 0.06, 0.08]
    wav = torch.stack([S.ricker(f, t, dt, nt) for f, t in zip(f0s, t0s)])
    d = _desc(nx, nz, P, nt, dx, dt, nmodels=B)
    gpu = _gpu_run(d, c, ct, S.Shots(src, rec, wav), want_gw=True)
    g = _grid(nx, nz, P, nt, dx, dt)
    w = wav.cpu().numpy().astype(np.float64)
    for b in range(B):
        sl = slice(b * spm, (b + 1) * spm)
        obs = O.ad2_forward(g, ct[b], src[sl], w[sl], rec[sl])
        grad, pred, gw = O.ad2_gradient(g, c[b], src[sl], w[sl], rec[sl],
                                        O.ad2_forward(g, c[b], src[sl], w[sl], rec[sl]) - obs)
        es, eg = rel_l2(gpu["pred"][sl], pred), rel_l2(gpu["grad"][b], grad)
        ew = rel_l2(gpu["gw"][sl], gw[:, 0])
        print(f"model {b}: seis {es:.2e} grad {eg:.2e} dJ/dwav {ew:.2e}")
        assert rel_l2(gpu["obs"][sl], obs) <= SEIS_TOL and es <= SEIS_TOL
        assert eg <= GRAD_TOL and ew <= GRAD_TOL


def _plane_wave_case(nx, nz, dx, dt, nt, f0=6.0, t0=0.2, rec_z=0):
    c_true = synth.layered_ellipses(250, nx, nz, dx)
    c0 = synth.smooth(c_true, 6.0)
    cb = float(c_true[-1].mean())
    rows = [SRC.plane_wave(np.arange(nx), nz - 2, th, cb, f0, t0, dx, dt, nt) for th in (-30.0, -10.0, 10.0, 30.0)]
    src = np.stack([n for n, _ in rows])
    wav = torch.stack([w for _, w in rows]).contiguous()
    rec = np.stack([np.array([[ix, rec_z] for ix in range(0, nx, 2)], np.int32)] * 4)
    return c_true, c0, src, wav, rec, cb


def test_plane_waves_parity_and_bitwise_invariance():
    nx, nz, P, nt, dx, dt = 160, 80, 16, 900, 20.0, 2e-3
    c_true, c0, src, wav, rec, cb = _plane_wave_case(nx, nz, dx, dt, nt)
    ref = np.stack([OSRC.plane_wave_wavelets(np.arange(nx) * dx, th, cb, 6.0, 0.2, dt, nt)
                    for th in (-30.0, -10.0, 10.0, 30.0)])
    assert np.abs(wav.cpu().numpy() - ref).max() <= 1e-6
    d = _desc(nx, nz, P, nt, dx, dt, vmax=5000.0)
    sh = S.Shots(src, rec, wav)
    a = _gpu_run(d, c0, c_true, sh)
    b = _gpu_run(d, c0, c_true, sh, ckpt=7)
    c = _gpu_run(d, c0, c_true, sh, store=3)
    e = _gpu_run(d, c0, c_true, sh)
    for other in (b, c, e):
        for k in ("pred", "grad"):
            assert np.array_equal(a[k], other[k]), k
    g = _grid(nx, nz, P, nt, dx, dt, vmax=5000.0)
    w = wav.cpu().numpy().astype(np.float64)
    obs = O.ad2_forward(g, c_true, src, w, rec)
    pred = O.ad2_forward(g, c0, src, w, rec)
    grad, _, _ = O.ad2_gradient(g, c0, src, w, rec, pred - obs)
    es, eg = rel_l2(a["pred"], pred), rel_l2(a["grad"][0], grad)
    print(f"plane waves: seis {es:.2e} grad {eg:.2e}")
    assert rel_l2(a["obs"], obs) <= SEIS_TOL and es <= SEIS_TOL and eg <= GRAD_TOL


def test_reciprocity_and_dot_identity_without_layer():
    nx, nz, nt, dx, dt = 150, 90, 400, 10.0, 1e-3
    c = synth.smooth_random(21, (nz, nx), 4.0, 1800.0, 2800.0)
    d = _desc(nx, nz, 0, nt, dx, dt)
    r = S.ricker(15.0, 0.07, dt, nt)
    A, B = (17, 9), (121, 70)
    out = []
    for s_, r_ in ((A, B), (B, A)):
        m = S.Model(d, dev(c), 1, 1)
        out.append(m.forward(S.Shots(np.array([s_], np.int32), np.array([[r_]], np.int32), r[None].contiguous()),
                             save_ckpt=False).cpu().numpy().ravel())
        m.close()
    e = np.abs(out[0] - out[1]).max() / np.abs(out[0]).max()
    print(f"reciprocity: {e:.2e}")
    assert e <= 1e-5
    # dot identity of the whole sweep: J = <seis, d> is linear in the wavelets
    rng = np.random.default_rng(4)
    src = np.array([[[20, 10], [21, 10], [90, 60]]], np.int32)
    wav = dev(rng.standard_normal((1, 3, nt)))
    rec = np.array([[[ix, 2] for ix in range(0, nx, 5)]], np.int32)
    dd = dev(rng.standard_normal((1, 1, nt, rec.shape[1])))
    m = S.Model(d, dev(c), 1, rec.shape[1])
    sh = S.Shots(src, rec, wav)
    seis = m.forward(sh, save_ckpt=True)
    gw = torch.zeros_like(wav)
    m.gradient(sh, dd, g_wavelet=gw)
    lhs = S.dot_f64(seis.reshape(-1), dd.reshape(-1)).item()
    rhs = S.dot_f64(wav.reshape(-1), gw.reshape(-1)).item()
    print(f"dot identity: {lhs:.6e} vs {rhs:.6e}")
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)
    m.close()


def test_full_grid_short_window():
    """600 x 300 cells + 24-cell layer (a 12 x 6 km section at 20 m), 4 plane
    waves, 450 steps; receivers 1.2 km above the source row, so that the
    window holds the direct and scattered waves; whole seismograms and
    gradient."""
    nx, nz, P, nt, dx, dt = 600, 300, 24, 450, 20.0, 2e-3
    c_true, c0, src, wav, rec, cb = _plane_wave_case(nx, nz, dx, dt, nt, f0=8.0, t0=0.15, rec_z=nz - 62)
    d = _desc(nx, nz, P, nt, dx, dt, vmax=5000.0)
    gpu = _gpu_run(d, c0, c_true, S.Shots(src, rec, wav))
    g = _grid(nx, nz, P, nt, dx, dt, vmax=5000.0)
    w = wav.cpu().numpy().astype(np.float64)
    obs = O.ad2_forward(g, c_true, src, w, rec)
    pred = O.ad2_forward(g, c0, src, w, rec)
    grad, _, _ = O.ad2_gradient(g, c0, src, w, rec, pred - obs)
    es, eg = rel_l2(gpu["pred"], pred), rel_l2(gpu["grad"][0], grad)
    print(f"600x300: seis {es:.2e} grad {eg:.2e}")
    assert es <= SEIS_TOL and eg <= GRAD_TOL


def test_c2_configuration_sampled_shots():
    """The divergence form in the benchmark's launch configuration (1000 x 500
    + 32-cell CPML, all 64 point-source shots in one launch, checkpoints every
    64 steps) over a 250-step window: seismograms of two sampled shots, and
    the gradient driven by their residuals alone, against the oracle."""
    cfg = synth.C2
    nt = 250
    true = synth.dipping_layers_anomalies(2003, cfg.nx, cfg.nz, cfg.dx)
    c0 = synth.smooth(true, 10.0)
    src, rec = synth.c2_geometry(cfg.nshots, cfg.nx)
    vmax = 4500.0
    d = S.desc(ndim=2, physics=S.SG_ACOUSTIC_DIV, nx=cfg.nx, nz=cfg.nz, npml=cfg.npml, nt=nt, dx=cfg.dx,
               dt=cfg.dt, pml_R=cfg.pml_R, pml_vmax=vmax, f0_pml=cfg.f0)
    wav = S.ricker(cfg.f0, cfg.ricker_t0, cfg.dt, nt)[None].repeat(cfg.nshots, 1).contiguous()
    sh = S.Shots(src, rec, wav)
    m = S.Model(d, dev(c0), cfg.nshots, rec.shape[1], 64)
    seis = m.forward(sh)
    sel = [5, 40]
    g = O.grid(ndim=2, nx=cfg.nx, nz=cfg.nz, npml=cfg.npml, nt=nt, dx=cfg.dx, dt=cfg.dt, pml_R=cfg.pml_R,
               pml_vmax=vmax, f0_pml=cfg.f0)
    w = np.stack([O.ricker(cfg.f0, cfg.ricker_t0, cfg.dt, nt)] * len(sel))
    pred = O.ad2_forward(g, c0, src[sel], w, rec[sel])
    obs = O.ad2_forward(g, true, src[sel], w, rec[sel])
    dJ = torch.zeros_like(seis)
    dJ[sel, 0] = dev(pred - obs)
    gg = m.gradient(sh, dJ).cpu().numpy()[0]
    og, _, _ = O.ad2_gradient(g, c0, src[sel], w, rec[sel], pred - obs)
    es, eg = rel_l2(seis.cpu().numpy()[sel, 0], pred), rel_l2(gg, og)
    print(f"C2 divergence form, {nt} steps, shots {sel}: seis {es:.2e} grad {eg:.2e}")
    assert np.abs(pred).max() > 0 and np.abs(og).max() > 0
    assert es <= SEIS_TOL and eg <= GRAD_TOL
    m.close()


def test_layered_model_plane_wave_inversion():
    nx, nz, P, nt, dx, dt = 160, 80, 16, 900, 20.0, 2e-3
    c_true, c0, src, wav, rec, _ = _plane_wave_case(nx, nz, dx, dt, nt)
    d = _desc(nx, nz, P, nt, dx, dt, vmax=5000.0)
    sh = S.Shots(src, rec, wav)
    prop = fwi.Propagator(d, sh, store_segments=-1)
    obs = prop.forward(dev(c_true[None]), save_ckpt=False).clone()
    res = fwi.batched_lbfgs(prop, dev(c0[None]), obs, fwi.LBFGSConfig(iters=15, vmin=2000.0, vmax=5500.0))
    m = res.models.cpu().numpy()[0]
    J = np.asarray(res.J)[:, 0]
    e0, e1 = rel_l2(c0, c_true), rel_l2(m, c_true)
    # the update against the missing part of the model (cosine of the angle)
    du, dt_ = (m - c0).ravel(), (c_true - c0).ravel()
    cos = float(du @ dt_ / (np.linalg.norm(du) * np.linalg.norm(dt_)))
    print(f"J/J0 {J[-1] / J[0]:.3e}, model error {e0:.4f} -> {e1:.4f}, cos(update, true update) {cos:.3f}")
    assert np.all(np.diff(J) <= 0) and J[-1] <= 0.2 * J[0]
    assert e1 < e0 and cos > 0.1
