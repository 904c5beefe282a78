"""Parity over the workloads' full time length, in the launch configuration
the benchmark times, against stored oracle values (tests/golden/, written by
tests/golden/make_long_parity.py, which calls only the oracle and the seeded
input generators; the oracle takes 12-25 minutes per workload, too long to
run inside the test).

    c2: 1000 x 500 + 32-cell layer, 4000 steps: all 64 shots in one launch,
        two steps per launch on the blocked tiles, 64-step checkpoints, the
        last segments' snapshots kept; shots 0, 21, 42, 63 compared.
    c3: elastic 800 x 400 + 20-cell CPML, 3000 steps: all 16 shots in one
        launch (shot groups of 4), 55-step checkpoints; shot 0 (explosive)
        and shot 8 (double couple) compared, gradients in vp, vs, rho.
    c4: 3-D 128^3 + 24-cell layer, 2000 steps, 64 x 64 surface receivers,
        45-step checkpoints.

The gradient is driven by the residual of the compared shots only (zero for
the others, which then add nothing), so it equals the oracle's gradient for
those shots.  Compared: the predicted seismograms of a sample of receivers
at every time sample (rel-L2 <= 1e-4), each shot's whole-seismogram sum of
squares (rel <= 2e-4, twice the seismogram bar), the misfit J (relative
bound 2e-4 (|pred| + |obs|) / |pred - obs|, what a 1e-4 seismogram error
can move it), and the gradient (rel-L2 <= 1e-3: the whole array in 2-D;
every second cell and the whole array's norm and two inner products in
3-D)."""
import math
import os
import sys

import numpy as np
import pytest
import torch

from gpu_common import S, synth, rel_l2, dev

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_long_parity as G  # noqa: E402

SEIS_TOL, GRAD_TOL = 1e-4, 1e-3


def _golden(name):
    path = os.path.join(HERE, "golden", f"long_parity_{name}.npz")
    z = np.load(path)
    assert str(z["oracle_sha256"]) == G.oracle_sha256(), \
        f"{path} was written by other oracle sources; run tests/golden/make_long_parity.py {name}"
    return z


def _seis_checks(label, pred_all, obs_all, sel, z, rec_axis_sample):
    """pred_all, obs_all: FP32 device seismograms of every shot; sel: the
    compared shots."""
    p = pred_all[sel].double()
    o = obs_all[sel].double()
    samp = p.index_select(-1, torch.as_tensor(rec_axis_sample, device=p.device)).cpu().numpy()
    e_seis = rel_l2(samp, z["pred_sample"])
    n2p = (p ** 2).sum(dim=tuple(range(1, p.dim()))).cpu().numpy()
    n2o = (o ** 2).sum(dim=tuple(range(1, o.dim()))).cpu().numpy()
    e_np = np.max(np.abs(n2p / z["pred_norm2"] - 1.0))
    e_no = np.max(np.abs(n2o / z["obs_norm2"] - 1.0))
    J = 0.5 * float(((p - o) ** 2).sum())
    r = math.sqrt(2.0 * float(z["J"]))
    tol_J = 2e-4 * (math.sqrt(z["pred_norm2"].sum()) + math.sqrt(z["obs_norm2"].sum())) / r
    e_J = abs(J / float(z["J"]) - 1.0)
    print(f"{label}: sampled traces rel-L2 {e_seis:.2e}; sum of squares pred {e_np:.2e} obs {e_no:.2e}; "
          f"J {J:.6e} vs {float(z['J']):.6e} (rel {e_J:.2e}, bound {tol_J:.2e})")
    assert np.abs(z["pred_sample"]).max() > 0
    assert e_seis <= SEIS_TOL and e_np <= 2 * SEIS_TOL and e_no <= 2 * SEIS_TOL and e_J <= tol_J


def _residual_of(sel, pred, obs, m):
    J, r = m.misfit(pred, obs)
    mask = torch.zeros(pred.shape[0], dtype=torch.bool, device=pred.device)
    mask[sel] = True
    r[~mask] = 0.0
    return r


def test_c2_full_length_parity():
    z = _golden("c2")
    cfg = synth.C2
    true = synth.dipping_layers_anomalies(2003, cfg.nx, cfg.nz, cfg.dx)
    c0 = synth.smooth(true, 10.0)
    src, rec = synth.c2_geometry(cfg.nshots, cfg.nx)
    K = int(math.ceil(math.sqrt(cfg.nt)))
    d = S.desc(ndim=2, nx=cfg.nx, nz=cfg.nz, npml=cfg.npml, nt=cfg.nt, dx=cfg.dx, dt=cfg.dt, pml_R=cfg.pml_R,
               pml_vmax=4500.0, f0_pml=cfg.f0)
    wav = S.ricker(cfg.f0, cfg.ricker_t0, cfg.dt, cfg.nt)[None].repeat(cfg.nshots, 1).contiguous()
    sh = S.Shots(src, rec, wav)
    mo = S.Model(d, dev(true), cfg.nshots, rec.shape[1], K)
    obs = mo.forward(sh, save_ckpt=False)
    torch.cuda.synchronize()
    mo.close()
    del mo
    m = S.Model(d, dev(c0), cfg.nshots, rec.shape[1], K, store_segments=10)
    m.set_time_blocking(2)
    pred = m.forward(sh)
    sel = list(z["shots"])
    _seis_checks("C2 4000 steps", pred[:, 0], obs[:, 0], sel, z, z["rec_sample"])
    r = _residual_of(sel, pred, obs, m)
    g = m.gradient(sh, r).cpu().numpy()[0]
    e = rel_l2(g, z["grad"])
    print(f"C2 4000 steps: gradient rel-L2 {e:.2e}")
    assert e <= GRAD_TOL
    m.close()


def test_c3_full_length_parity():
    z = _golden("c3")
    cfg = synth.C3
    vp, vs, rho = synth.elastic_c3(6027, cfg.nx, cfg.nz)
    m0 = [synth.smooth(a, 10.0) for a in (vp, vs, rho)]
    src, mt, rec = synth.c3_geometry(6027, cfg.nx)
    K = int(math.ceil(math.sqrt(cfg.nt)))
    d = S.desc(ndim=2, physics=S.SG_ELASTIC, nx=cfg.nx, nz=cfg.nz, npml=cfg.npml, nt=cfg.nt, dx=cfg.dx,
               dt=cfg.dt, pml_R=cfg.pml_R, pml_vmax=4000.0, f0_pml=cfg.f0_pml)
    wav = S.ricker(cfg.f0, cfg.ricker_t0, cfg.dt, cfg.nt)[None].repeat(cfg.nshots, 1).contiguous()
    sh = S.Shots(src, rec, wav, mt=mt)
    mo = S.Model(d, dev(vp), cfg.nshots, rec.shape[1], K, vs=dev(vs), rho=dev(rho))
    obs = mo.forward(sh, save_ckpt=False)
    torch.cuda.synchronize()
    mo.close()
    m = S.Model(d, dev(m0[0]), cfg.nshots, rec.shape[1], K, vs=dev(m0[1]), rho=dev(m0[2]), store_segments=10)
    pred = m.forward(sh)
    sel = list(z["shots"])
    _seis_checks("C3 3000 steps", pred, obs, sel, z, z["rec_sample"])
    r = _residual_of(sel, pred, obs, m)
    gs = [t.cpu().numpy()[0] for t in m.gradient(sh, r)]
    es = [rel_l2(a, z[k]) for a, k in zip(gs, ("grad_vp", "grad_vs", "grad_rho"))]
    print(f"C3 3000 steps: gradient rel-L2 vp {es[0]:.2e} vs {es[1]:.2e} rho {es[2]:.2e}")
    assert max(es) <= GRAD_TOL
    m.close()


def test_c4_reduced_cube_full_length_parity():
    z = _golden("c4")
    cfg, true, c0, src, rec = G.c4_setup()
    K = int(math.ceil(math.sqrt(cfg.nt)))
    d = S.desc(ndim=3, nx=cfg.nx, ny=cfg.ny, nz=cfg.nz, npml=cfg.npml, nt=cfg.nt, dx=cfg.dx, dt=cfg.dt,
               pml_R=cfg.pml_R, pml_vmax=4000.0)
    wav = S.ricker(cfg.f0, cfg.ricker_t0, cfg.dt, cfg.nt)[None].contiguous()
    sh = S.Shots(src, rec, wav)
    mo = S.Model(d, dev(true), 1, rec.shape[1], K)
    obs = mo.forward(sh, save_ckpt=False)
    torch.cuda.synchronize()
    mo.close()
    m = S.Model(d, dev(c0), 1, rec.shape[1], K, store_segments=10)
    pred = m.forward(sh)
    _seis_checks("C4 128^3, 2000 steps", pred[:, 0], obs[:, 0], [0], z, z["rec_sample"])
    _, r = m.misfit(pred, obs)
    g = m.gradient(sh, r)[0].double()
    e_sub = rel_l2(g[::2, ::2, ::2].cpu().numpy(), z["grad_sub2"])
    e_norm = abs(float((g ** 2).sum()) / float(z["grad_norm2"]) - 1.0)
    probes = [float((g * torch.as_tensor(f, device=g.device)).sum()) for f in G.c4_probe_fields()]
    e_pr = [abs(a / b - 1.0) for a, b in zip(probes, z["grad_probes"])]
    print(f"C4 128^3, 2000 steps: gradient rel-L2 on every second cell {e_sub:.2e}; |g|^2 {e_norm:.2e}; "
          f"inner products {e_pr[0]:.2e} {e_pr[1]:.2e}")
    assert e_sub <= GRAD_TOL and e_norm <= 2 * GRAD_TOL and max(e_pr) <= GRAD_TOL
    m.close()
