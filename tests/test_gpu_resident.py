"""The CU-resident 2-D acoustic forward (one workgroup per shot holding the
whole field in LDS, a checkpoint segment per launch): seismograms and
gradients against the batched launches (same FP32 expressions per cell,
rel-L2 <= 1e-6) and against the FP64 oracle (seismograms 1e-4, gradients
1e-3), on a ragged grid with a layer, several models and shots, duplicate
receivers, an odd checkpoint interval, stored and recomputed segments; on a
grid without a layer; and the refusal of grids that do not fit."""
import numpy as np
import pytest
import torch

from gpu_common import O, S, synth, rel_l2, oracle_grid, gpu_desc, gpu_wavelets, oracle_wavelets, dev

pytestmark = pytest.mark.gpu

SEIS_TOL, GRAD_TOL, SAME_TOL = 1e-4, 1e-3, 1e-6


def _fwd_grad(d, c, sh, obs, ckpt, resident, tb=2, store=0):
    if store < 0:                                            # every segment's snapshots kept
        K = ckpt if ckpt > 0 else int(np.ceil(np.sqrt(d.nt)))
        store = -(-d.nt // K)
    m = S.Model(d, dev(c), sh.nshots, sh.nrec, ckpt, store_segments=store)
    m.set_time_blocking(tb)
    m.set_tuning(S.SG_TUNE_RESIDENT, int(resident))
    pred = m.forward(sh)
    J, r = m.misfit(pred, obs)
    g = m.gradient(sh, r)
    torch.cuda.synchronize()
    out = pred.cpu().numpy()[:, 0], g.cpu().numpy(), float(J.item())
    m.close()
    return out


def _case(cfg, ct, c0, src, rec, f0s, t0s, vmax, nmodels, ckpt):
    d = gpu_desc(cfg, vmax, nmodels=nmodels)
    wav = gpu_wavelets(f0s, t0s, cfg.dt, cfg.nt)
    sh = S.Shots(src, rec, wav)
    mo = S.Model(d, dev(ct), src.shape[0], rec.shape[1], ckpt)
    mo.set_tuning(S.SG_TUNE_RESIDENT, 1)
    obs_res = mo.forward(sh, save_ckpt=False).clone()
    mo.set_tuning(S.SG_TUNE_RESIDENT, 0)
    obs = mo.forward(sh, save_ckpt=False).clone()
    mo.close()
    e = rel_l2(obs_res.cpu().numpy(), obs.cpu().numpy())
    print(f"observed data, resident vs batched: rel-L2 {e:.2e} (bitwise: {torch.equal(obs_res, obs)})")
    assert e <= SAME_TOL
    runs = {}
    for label, res, tb, store in (("batched", False, 2, 0), ("batched 1 step", False, 1, 0),
                                  ("resident", True, 2, 0), ("resident, stored", True, 2, -1)):
        runs[label] = _fwd_grad(d, c0, sh, obs, ckpt, res, tb, store)
    p0, g0, J0 = runs["batched"]
    for label, (p, g, J) in runs.items():
        es, eg = rel_l2(p, p0), rel_l2(g, g0)
        print(f"{label}: vs batched seis {es:.2e} grad {eg:.2e} J {J:.8e} "
              f"(bitwise: {np.array_equal(p, p0)} {np.array_equal(g, g0)})")
        assert es <= SAME_TOL and eg <= SAME_TOL
    return d, obs.cpu().numpy()[:, 0], runs


def test_resident_ragged_multimodel_against_batched_and_oracle():
    cfg = synth.C1.replace(nx=150, nz=77, npml=10, nt=300, dt=1e-3)     # padded 170 x 97: ragged tiles
    rng = np.random.default_rng(31)
    cA = 1600.0 + 900.0 * synth.smooth_random(5, (cfg.nz, cfg.nx), 4.0, 0.0, 1.0)
    cB = cA[:, ::-1].copy()
    src = np.array([[5, 3], [140, 70], [75, 0], [0, 40]], dtype=np.int32)
    nr = 50
    rec = np.stack([np.stack([rng.integers(0, cfg.nx, nr), rng.integers(0, cfg.nz, nr)], -1)
                    for _ in range(4)]).astype(np.int32)
    rec[1, :3] = rec[1, 3]                                   # duplicate receivers on one cell
    f0s, t0s = [15.0, 12.0, 20.0, 18.0], [0.07, 0.08, 0.05, 0.06]
    vmax = 2600.0
    c0A, c0B = synth.smooth(cA, 3.0), synth.smooth(cB, 3.0)
    _, obs, runs = _case(cfg, np.stack([cA, cB]), np.stack([c0A, c0B]), src, rec, f0s, t0s, vmax, 2, 13)
    p, g, _ = runs["resident"]
    go = oracle_grid(cfg, vmax)
    wo = oracle_wavelets(f0s, t0s, cfg.dt, cfg.nt)
    for mi, (ci, c0i) in enumerate([(cA, c0A), (cB, c0B)]):
        sl = slice(2 * mi, 2 * mi + 2)
        oo = O.ac2_forward(go, ci, src[sl], wo[sl], rec[sl])
        op = O.ac2_forward(go, c0i, src[sl], wo[sl], rec[sl])
        _, ro = O.misfit(op, oo)
        og, _ = O.ac2_gradient(go, c0i, src[sl], wo[sl], rec[sl], ro, ckpt=0)
        e1, e2, e3 = rel_l2(obs[sl], oo), rel_l2(p[sl], op), rel_l2(g[mi], og)
        print(f"resident, model {mi} vs oracle: seis {e1:.2e} {e2:.2e} grad {e3:.2e}")
        assert e1 <= SEIS_TOL and e2 <= SEIS_TOL and e3 <= GRAD_TOL


def test_resident_c1_grid_and_no_layer():
    """The 141 x 141 padded grid of the 101 x 101 workload (one shot per
    model, 3 models), then a rigid box without a layer."""
    cfg = synth.C1.replace(nt=400)
    ct = np.stack([synth.random_layered(s) for s in range(3)])
    c0 = np.stack([synth.smooth(t, 10.0) for t in ct])
    src = np.array([[50, 2]] * 3, dtype=np.int32)
    rec = synth.surface_receivers_2d(3, cfg.nx)
    _case(cfg, ct, c0, src, rec, [cfg.f0] * 3, [cfg.ricker_t0] * 3, 3500.0, 3, 0)
    cfg0 = synth.C1.replace(nx=96, nz=130, npml=0, nt=250)
    c = 1500.0 + 1000.0 * synth.smooth_random(9, (cfg0.nz, cfg0.nx), 5.0, 0.0, 1.0)
    src0 = np.array([[48, 60], [10, 5]], dtype=np.int32)
    rec0 = np.stack([np.stack([np.arange(0, 96, 2), np.full(48, 3)], -1)] * 2).astype(np.int32)
    _case(cfg0, c, synth.smooth(c, 4.0), src0, rec0, [25.0, 20.0], [0.04, 0.05], 2500.0, 1, 16)


def test_resident_refuses_grids_that_do_not_fit():
    cfg = synth.C1.replace(nx=140, nz=140, npml=20, nt=10)               # 180 x 180 padded
    d = gpu_desc(cfg, 3000.0)
    m = S.Model(d, dev(np.full((140, 140), 2000.0)), 1, 1, 0)
    with pytest.raises(S.SeisError):
        m.set_tuning(S.SG_TUNE_RESIDENT, 1)
    m.close()
    d3 = S.desc(ndim=3, nx=8, ny=8, nz=8, npml=0, nt=4)
    m3 = S.Model(d3, dev(np.full((8, 8, 8), 2000.0)), 1, 1, 0)
    with pytest.raises(S.SeisError):
        m3.set_tuning(S.SG_TUNE_RESIDENT, 1)
    m3.close()
