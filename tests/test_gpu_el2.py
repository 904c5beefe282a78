"""GPU parity of the 2-D elastic HIP path (velocity-stress, staggered 4th
order, CPML) against the FP64 oracle: two-component seismograms (rel-L2 <=
1e-4) and gradients with respect to vp, vs and rho (rel-L2 <= 1e-3);
checkpointed == store-all bitwise; the dot-product identity with FP64
reductions."""
import numpy as np
import pytest
import torch

from gpu_common import O, S, synth, rel_l2, dev

pytestmark = pytest.mark.gpu

SEIS_TOL = 1e-4
GRAD_TOL = 1e-3


def _case(nx=150, nz=83, P=20, nt=700, dt=0.5e-3, dx=5.0):
    vp = 1800.0 + 2200.0 * synth.smooth_random(6027, (nz, nx), 8.0, 0.0, 1.0)
    rng = np.random.default_rng(6028)
    vs = vp / 1.73 * (1.0 + rng.uniform(-0.1, 0.1, size=vp.shape))
    rho = 310.0 * vp ** 0.25
    src = np.array([[40, 5], [110, 60], [75, 30]], dtype=np.int32)
    mt = np.array([[1.0, 1.0, 0.0], [-0.5, 0.5, 0.86], [0.3, -0.3, 0.95]])
    rec = np.stack([np.stack([np.arange(0, nx, 2), np.zeros(nx // 2 + nx % 2)], -1)] * 3).astype(np.int32)
    rec[2, :3] = rec[2, 3]                         # duplicate receivers on one cell
    cfg = dict(nx=nx, nz=nz, P=P, nt=nt, dt=dt, dx=dx)
    return cfg, vp, vs, rho, src, mt, rec


def _desc(c, vmax=4000.0, f0=15.0):
    return S.desc(ndim=2, physics=S.SG_ELASTIC, nx=c["nx"], nz=c["nz"], npml=c["P"], nt=c["nt"], dx=c["dx"],
                  dt=c["dt"], pml_vmax=vmax, f0_pml=f0)


def _grid(c, vmax=4000.0, f0=15.0):
    return O.grid(ndim=2, nx=c["nx"], nz=c["nz"], npml=c["P"], nt=c["nt"], dx=c["dx"], dt=c["dt"],
                  pml_vmax=vmax, f0_pml=f0)


def _model(d, vp, vs, rho, ns, nrec, ckpt=0):
    return S.Model(d, dev(vp), ns, nrec, ckpt, vs=dev(vs), rho=dev(rho))


def test_elastic_forward_and_gradient_parity():
    c, vp, vs, rho, src, mt, rec = _case()
    vp0, vs0, rho0 = (synth.smooth(a, 5.0) for a in (vp, vs, rho))
    d = _desc(c)
    f0s = [15.0, 12.0, 18.0]
    wav = torch.stack([S.ricker(f, 1.0 / f, c["dt"], c["nt"]) for f in f0s])
    sh = S.Shots(src, rec, wav, mt)
    mt_ = _model(d, vp, vs, rho, 3, rec.shape[1], 37)
    obs = mt_.forward(sh, save_ckpt=False)
    m0 = _model(d, vp0, vs0, rho0, 3, rec.shape[1], 37)
    pred = m0.forward(sh)
    J, r = m0.misfit(pred, obs)
    gv = [x.cpu().numpy()[0] for x in m0.gradient(sh, r)]
    go = _grid(c)
    wo = np.stack([O.ricker(f, 1.0 / f, c["dt"], c["nt"]) for f in f0s])
    oo = O.el2_forward(go, vp, vs, rho, src, mt, wo, rec)
    op = O.el2_forward(go, vp0, vs0, rho0, src, mt, wo, rec)
    Jo, ro = O.misfit(op, oo)
    og, _ = O.el2_gradient(go, vp0, vs0, rho0, src, mt, wo, rec, ro, ckpt=30)
    ga = [x.cpu().numpy()[0] for x in m0.gradient(sh, dev(ro))]
    e_obs, e_pred = rel_l2(obs.cpu().numpy(), oo), rel_l2(pred.cpu().numpy(), op)
    e_g = [rel_l2(a, b) for a, b in zip(gv, og)]
    e_a = [rel_l2(a, b) for a, b in zip(ga, og)]
    print(f"elastic seis {e_obs:.2e} {e_pred:.2e}; grad vp/vs/rho {e_g[0]:.2e} {e_g[1]:.2e} {e_g[2]:.2e}; "
          f"on the oracle residual {e_a[0]:.2e} {e_a[1]:.2e} {e_a[2]:.2e}; J {J.item():.6e} vs {Jo:.6e}")
    assert e_obs <= SEIS_TOL and e_pred <= SEIS_TOL
    assert max(e_a) <= GRAD_TOL
    assert max(e_g) <= GRAD_TOL


def test_elastic_gradient_shot_groups_parity():
    """The adjoint passes accumulate gradients over groups of the shots of a
    model (4 when the shots per model divide by 4, else 2, else 1): one model
    with 4 shots (groups of 4) and 2 models with 2 shots each (groups of 2),
    each on the oracle's residual, against the oracle's gradients."""
    c, vp, vs, rho, _, _, rec3 = _case(nx=100, nz=56, P=12, nt=380)
    src = np.array([[30, 5], [80, 40], [55, 25], [15, 45]], dtype=np.int32)
    mt = np.array([[1.0, 1.0, 0.0], [-0.5, 0.5, 0.86], [0.3, -0.3, 0.95], [0.7, 0.2, -0.4]])
    rec = np.stack([rec3[0]] * 4)
    f0s = [15.0, 12.0, 18.0, 14.0]
    wav = torch.stack([S.ricker(f, 1.0 / f, c["dt"], c["nt"]) for f in f0s])
    wo = np.stack([O.ricker(f, 1.0 / f, c["dt"], c["nt"]) for f in f0s])
    sh = S.Shots(src, rec, wav, mt)
    go = _grid(c)
    A = [vp, vs, rho]
    B = [a[::-1].copy() for a in A]
    A0 = [synth.smooth(a, 5.0) for a in A]
    B0 = [synth.smooth(a, 5.0) for a in B]
    for label, models, models0, spm in (("1 model x 4 shots", [A], [A0], 4),
                                        ("2 models x 2 shots", [A, B], [A0, B0], 2)):
        ro, og = [], []
        for mi, (t, t0) in enumerate(zip(models, models0)):
            sl = slice(mi * spm, (mi + 1) * spm)
            oo = O.el2_forward(go, *t, src[sl], mt[sl], wo[sl], rec[sl])
            op = O.el2_forward(go, *t0, src[sl], mt[sl], wo[sl], rec[sl])
            r = O.misfit(op, oo)[1]
            ro.append(r)
            og.append(O.el2_gradient(go, *t0, src[sl], mt[sl], wo[sl], rec[sl], r, ckpt=30)[0])
        d = S.desc(ndim=2, physics=S.SG_ELASTIC, nx=c["nx"], nz=c["nz"], npml=c["P"], nt=c["nt"], dx=c["dx"],
                   dt=c["dt"], pml_vmax=4000.0, f0_pml=15.0, nmodels=len(models))
        m0 = S.Model(d, dev(np.stack([t[0] for t in models0])), 4, rec.shape[1], 29,
                     vs=dev(np.stack([t[1] for t in models0])), rho=dev(np.stack([t[2] for t in models0])))
        m0.forward(sh)
        ga = [x.cpu().numpy() for x in m0.gradient(sh, dev(np.concatenate(ro)))]
        for mi in range(len(models)):
            e = [rel_l2(ga[q][mi], og[mi][q]) for q in range(3)]
            print(f"{label}, model {mi}: grad vp/vs/rho {e[0]:.2e} {e[1]:.2e} {e[2]:.2e}")
            assert max(e) <= GRAD_TOL


def test_elastic_no_layer_parity():
    """npml = 0: no CPML memories touched, rigid walls at the grid edge,
    sources next to two walls."""
    c, vp, vs, rho, src, mt, rec = _case(nx=120, nz=70, P=0, nt=400)
    src = np.array([[3, 2], [110, 60], [60, 35]], dtype=np.int32)
    vp0, vs0, rho0 = (synth.smooth(a, 5.0) for a in (vp, vs, rho))
    d = _desc(c)
    f0s = [15.0, 12.0, 18.0]
    wav = torch.stack([S.ricker(f, 1.0 / f, c["dt"], c["nt"]) for f in f0s])
    sh = S.Shots(src, rec, wav, mt)
    obs = _model(d, vp, vs, rho, 3, rec.shape[1], 21).forward(sh, save_ckpt=False)
    m0 = _model(d, vp0, vs0, rho0, 3, rec.shape[1], 21)
    pred = m0.forward(sh)
    J, r = m0.misfit(pred, obs)
    gv = [x.cpu().numpy()[0] for x in m0.gradient(sh, r)]
    go = _grid(c)
    wo = np.stack([O.ricker(f, 1.0 / f, c["dt"], c["nt"]) for f in f0s])
    oo = O.el2_forward(go, vp, vs, rho, src, mt, wo, rec)
    op = O.el2_forward(go, vp0, vs0, rho0, src, mt, wo, rec)
    _, ro = O.misfit(op, oo)
    og, _ = O.el2_gradient(go, vp0, vs0, rho0, src, mt, wo, rec, ro, ckpt=20)
    e_obs, e_pred = rel_l2(obs.cpu().numpy(), oo), rel_l2(pred.cpu().numpy(), op)
    e_g = [rel_l2(a, b) for a, b in zip(gv, og)]
    print(f"elastic no layer: seis {e_obs:.2e} {e_pred:.2e}; grad vp/vs/rho {e_g[0]:.2e} {e_g[1]:.2e} {e_g[2]:.2e}")
    assert e_obs <= SEIS_TOL and e_pred <= SEIS_TOL
    assert max(e_g) <= GRAD_TOL


def test_elastic_checkpointing_and_dot_identity():
    c, vp, vs, rho, src, mt, rec = _case(nt=300)
    d = _desc(c)
    s = dev(synth.random_field(9, (3, c["nt"])))
    sh = S.Shots(src, rec, s, mt)
    outs = []
    for K in (c["nt"], 13):
        m = _model(d, vp, vs, rho, 3, rec.shape[1], K)
        Fs = m.forward(sh)
        gw = torch.zeros((3, c["nt"]), dtype=torch.float32, device="cuda")
        g = m.gradient(sh, Fs, g_wavelet=gw)
        outs.append([Fs.clone(), gw.clone()] + [x.clone() for x in g])
        m.close()
    for a, b in zip(outs[0], outs[1]):
        assert torch.equal(a, b)
    Fs, gw = outs[0][0], outs[0][1]
    lhs = S.dot_f64(Fs.reshape(-1), Fs.reshape(-1)).item()
    rhs = S.dot_f64(s.reshape(-1), gw.reshape(-1)).item()
    print(f"elastic dot test: rel {abs(lhs - rhs) / lhs:.2e}")
    assert abs(lhs - rhs) <= 1e-5 * lhs


def test_c3_full_grid_short_window_parity():
    """The 800 x 400 (+20-cell CPML) launch configuration with all 16 shots
    (8 explosive, 8 double couples), 2-component receivers, over 150 steps."""
    cfg = synth.C3
    vp, vs, rho = synth.elastic_c3(6027, cfg.nx, cfg.nz)
    src, mt, rec = synth.c3_geometry(6027, cfg.nx)
    nt = 150
    c = dict(nx=cfg.nx, nz=cfg.nz, P=cfg.npml, nt=nt, dt=cfg.dt, dx=cfg.dx)
    d = _desc(c, f0=cfg.f0)
    wav = S.ricker(cfg.f0 * 4, 0.025, cfg.dt, nt)[None].repeat(16, 1).contiguous()
    sh = S.Shots(src, rec, wav, mt)
    m = _model(d, vp, vs, rho, 16, rec.shape[1], 12)
    seis = m.forward(sh).cpu().numpy()
    go = _grid(c, f0=cfg.f0)
    sel = [0, 9]                                   # one explosive, one double couple
    ref = O.el2_forward(go, vp, vs, rho, src[sel], mt[sel],
                        np.stack([O.ricker(cfg.f0 * 4, 0.025, cfg.dt, nt)] * 2), rec[sel])
    e = rel_l2(seis[sel], ref)
    print(f"C3 full grid, {nt} steps, shots {sel}: seis rel-L2 {e:.2e}")
    assert np.abs(ref).max() > 0 and e <= SEIS_TOL
