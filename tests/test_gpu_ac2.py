"""GPU parity of the 2-D acoustic HIP path (through the C ABI) against the
FP64 oracle, plus GPU self-consistency (dot-product identity with FP64
reductions, checkpointed == store-all bitwise, run-to-run determinism).

Tolerances: seismograms rel-L2 <= 1e-4, gradients rel-L2 <= 1e-3 over the
whole array; FP32 arithmetic in the kernels, FP64 in the oracle."""
import numpy as np
import pytest
import torch

from gpu_common import O, S, synth, rel_l2, oracle_grid, gpu_desc, gpu_wavelets, oracle_wavelets, dev

pytestmark = pytest.mark.gpu

SEIS_TOL = 1e-4
GRAD_TOL = 1e-3


def _run_case(cfg, c_true, c0, src, rec, f0s, t0s, pml_vmax, ckpt=0, nmodels=1, want_gw=False,
              ext_resid=None):
    """GPU: forward on c_true (observed), forward+misfit+adjoint on c0; with
    ext_resid also the adjoint driven by that (oracle) residual."""
    ns = src.shape[0]
    d = gpu_desc(cfg, pml_vmax, nmodels=nmodels)
    wav = gpu_wavelets(f0s, t0s, cfg.dt, cfg.nt)
    sh = S.Shots(src, rec, wav)
    mt = S.Model(d, dev(c_true), ns, rec.shape[1], ckpt)
    obs = mt.forward(sh, save_ckpt=False)
    m0 = S.Model(d, dev(c0), ns, rec.shape[1], ckpt)
    pred = m0.forward(sh, save_ckpt=True)
    J, resid = m0.misfit(pred, obs)
    gw = torch.zeros((ns, cfg.nt), dtype=torch.float32, device="cuda") if want_gw else None
    g = m0.gradient(sh, resid, g_wavelet=gw)
    torch.cuda.synchronize()
    out = dict(obs=obs.cpu().numpy()[:, 0], pred=pred.cpu().numpy()[:, 0], J=float(J.item()),
               grad=g.cpu().numpy(), wav=wav.cpu().numpy())
    if ext_resid is not None:
        out["grad_ext"] = m0.gradient(sh, dev(ext_resid[:, None])).cpu().numpy()
    if want_gw:
        out["gw"] = gw.cpu().numpy()
    mt.close()
    m0.close()
    return out


def _oracle_case(cfg, c_true, c0, src, rec, f0s, t0s, pml_vmax, ckpt=0):
    g = oracle_grid(cfg, pml_vmax)
    wav = oracle_wavelets(f0s, t0s, cfg.dt, cfg.nt)
    obs = O.ac2_forward(g, c_true, src, wav, rec)
    pred = O.ac2_forward(g, c0, src, wav, rec)
    J, r = O.misfit(pred, obs)
    grad, _ = O.ac2_gradient(g, c0, src, wav, rec, r, ckpt=ckpt)
    return dict(obs=obs, pred=pred, J=J, grad=grad, wav=wav, resid=r)


def test_ricker_matches_oracle():
    for f0, t0, dt, nt in [(10.0, 0.1, 1e-3, 500), (8.0, 0.125, 0.8e-3, 4000)]:
        a = S.ricker(f0, t0, dt, nt).cpu().numpy()
        b = O.ricker(f0, t0, dt, nt)
        assert np.max(np.abs(a - b)) <= 6e-8


def test_c1_forward_and_gradient_parity():
    """2-D acoustic 101x101, 3 layers, dt = 1 ms, 500 steps, 20-cell layer,
    10 Hz Ricker at (50, 2), 101 surface receivers; gradient of the L2
    misfit against the smoothed initial model."""
    cfg = synth.C1
    ct = synth.layered_c1()
    c0 = synth.smooth(ct, 10.0)
    src, rec = synth.c1_geometry()
    f0s, t0s = [cfg.f0], [cfg.ricker_t0]
    vmax = 3000.0
    ora = _oracle_case(cfg, ct, c0, src, rec, f0s, t0s, vmax)
    gpu = _run_case(cfg, ct, c0, src, rec, f0s, t0s, vmax, ext_resid=ora["resid"])
    e_obs, e_pred = rel_l2(gpu["obs"], ora["obs"]), rel_l2(gpu["pred"], ora["pred"])
    e_grad = rel_l2(gpu["grad"], ora["grad"])
    e_adj = rel_l2(gpu["grad_ext"], ora["grad"])
    print(f"C1 seis rel-L2 {e_obs:.2e} / {e_pred:.2e}  grad rel-L2 {e_grad:.2e} "
          f"(adjoint on the oracle residual {e_adj:.2e})  J {gpu['J']:.6e} vs {ora['J']:.6e}")
    assert e_obs <= SEIS_TOL and e_pred <= SEIS_TOL
    # the adjoint sweep alone, on the same residual
    assert e_adj <= GRAD_TOL
    # end to end: the FP32 residual carries the forward error amplified by
    # the cancellation pred - obs (the direct wave cancels)
    assert e_grad <= GRAD_TOL
    assert gpu["J"] == pytest.approx(ora["J"], rel=2e-3)


def test_ragged_multishot_multimodel_parity():
    """Grid not a multiple of the tile (ragged tiles in x and z), 4 shots over
    2 models batched in one launch, sources/receivers near and inside the
    layer's neighbourhood, odd checkpoint interval."""
    cfg = synth.C1.replace(nx=150, nz=77, npml=10, nt=300, dt=1e-3)
    rng = np.random.default_rng(12)
    cA = 1600.0 + 900.0 * synth.smooth_random(3, (cfg.nz, cfg.nx), 4.0, 0.0, 1.0)
    cB = cA[::-1].copy()
    src = np.array([[5, 3], [140, 70], [75, 0], [0, 40]], dtype=np.int32)
    nr = 60
    rec = np.stack([np.stack([rng.integers(0, cfg.nx, nr), rng.integers(0, cfg.nz, nr)], -1)
                    for _ in range(4)]).astype(np.int32)
    rec[0, :2] = rec[0, 2]                       # duplicate receivers on one cell
    f0s, t0s = [15.0, 12.0, 20.0, 18.0], [0.07, 0.08, 0.05, 0.06]
    vmax = 2600.0
    ct = np.stack([cA, cA, cB, cB])
    c0 = np.stack([synth.smooth(cA, 3.0)] * 2 + [synth.smooth(cB, 3.0)] * 2)
    d = gpu_desc(cfg, vmax, nmodels=2)
    wav = gpu_wavelets(f0s, t0s, cfg.dt, cfg.nt)
    sh = S.Shots(src, rec, wav)
    mt = S.Model(d, dev(np.stack([cA, cB])), 4, nr, 13)
    obs = mt.forward(sh, save_ckpt=False)
    m0 = S.Model(d, dev(np.stack([c0[0], c0[2]])), 4, nr, 13)
    pred = m0.forward(sh)
    J, r = m0.misfit(pred, obs)
    g = m0.gradient(sh, r).cpu().numpy()
    obs, pred = obs.cpu().numpy()[:, 0], pred.cpu().numpy()[:, 0]
    go = oracle_grid(cfg, vmax)
    wo = oracle_wavelets(f0s, t0s, cfg.dt, cfg.nt)
    for mi, (ci, c0i) in enumerate([(cA, c0[0]), (cB, c0[2])]):
        sl = slice(2 * mi, 2 * mi + 2)
        oo = O.ac2_forward(go, ci, src[sl], wo[sl], rec[sl])
        op = O.ac2_forward(go, c0i, src[sl], wo[sl], rec[sl])
        _, ro = O.misfit(op, oo)
        og, _ = O.ac2_gradient(go, c0i, src[sl], wo[sl], rec[sl], ro, ckpt=0)
        e1, e2, e3 = rel_l2(obs[sl], oo), rel_l2(pred[sl], op), rel_l2(g[mi], og)
        print(f"model {mi}: seis {e1:.2e} {e2:.2e} grad {e3:.2e}")
        assert e1 <= SEIS_TOL and e2 <= SEIS_TOL and e3 <= GRAD_TOL


def test_no_layer_rigid_box_parity():
    """npml = 0: no layer pass, rigid walls at the grid edge, the blocked
    tiles reaching to within 8 cells of the edge; reflections within the
    window (sources next to two walls)."""
    cfg = synth.C1.replace(nx=200, nz=120, npml=0, nt=300, dt=1e-3)
    c = 1700.0 + 800.0 * synth.smooth_random(5, (cfg.nz, cfg.nx), 4.0, 0.0, 1.0)
    c0 = synth.smooth(c, 3.0)
    src = np.array([[3, 2], [190, 110]], dtype=np.int32)
    xs = np.arange(0, cfg.nx, 3)
    rec = np.stack([np.stack([xs, np.zeros_like(xs)], -1), np.stack([xs, np.full_like(xs, 60)], -1)]).astype(np.int32)
    f0s, t0s = [15.0, 18.0], [0.07, 0.06]
    out = _run_case(cfg, c, c0, src, rec, f0s, t0s, 2500.0, ckpt=17)
    ref = _oracle_case(cfg, c, c0, src, rec, f0s, t0s, 2500.0)
    e1, e2, e3 = rel_l2(out["obs"], ref["obs"]), rel_l2(out["pred"], ref["pred"]), rel_l2(out["grad"][0], ref["grad"])
    print(f"no layer: seis {e1:.2e} {e2:.2e} grad {e3:.2e}")
    assert e1 <= SEIS_TOL and e2 <= SEIS_TOL and e3 <= GRAD_TOL


def test_degenerate_sizes():
    """One and two time steps; a 5 x 3 grid without a layer (one tile, most of
    it outside the grid); a shot without receivers (empty seismogram, J = 0,
    zero gradient)."""
    for nt in (1, 2):                                   # nt = 1: only the source term, zero gradient
        cfg = synth.C1.replace(nx=30, nz=20, npml=10, nt=nt, dt=1e-3)
        c = np.full((cfg.nz, cfg.nx), 2000.0)
        c[8:12, 8:14] = 2300.0
        src = np.array([[10, 9]], dtype=np.int32)
        rec = np.array([[[10, 9], [11, 9], [12, 10]]], dtype=np.int32)
        out = _run_case(cfg, c, synth.smooth(c, 2.0), src, rec, [15.0], [0.0], 2500.0)
        ref = _oracle_case(cfg, c, synth.smooth(c, 2.0), src, rec, [15.0], [0.0], 2500.0)
        assert rel_l2(out["obs"], ref["obs"]) <= SEIS_TOL and rel_l2(out["pred"], ref["pred"]) <= SEIS_TOL
        if nt == 1:
            assert np.all(ref["grad"] == 0.0) and np.all(out["grad"] == 0.0)
        else:
            assert np.abs(ref["grad"]).max() > 0 and rel_l2(out["grad"][0], ref["grad"]) <= GRAD_TOL
    cfg = synth.C1.replace(nx=5, nz=3, npml=0, nt=50, dt=1e-3)
    c = np.array([[2000.0, 2100, 2200, 2100, 2000]] * 3)
    src = np.array([[2, 1]], dtype=np.int32)
    rec = np.array([[[0, 0], [4, 2]]], dtype=np.int32)
    out = _run_case(cfg, c, np.full_like(c, 2100.0), src, rec, [15.0], [0.07], 2500.0)
    ref = _oracle_case(cfg, c, np.full_like(c, 2100.0), src, rec, [15.0], [0.07], 2500.0)
    e = (rel_l2(out["obs"], ref["obs"]), rel_l2(out["pred"], ref["pred"]), rel_l2(out["grad"][0], ref["grad"]))
    print(f"5 x 3 grid: seis {e[0]:.2e} {e[1]:.2e} grad {e[2]:.2e}")
    assert e[0] <= SEIS_TOL and e[1] <= SEIS_TOL and e[2] <= GRAD_TOL
    # no receivers
    cfg = synth.C1.replace(nx=40, nz=30, npml=10, nt=60, dt=1e-3)
    d = gpu_desc(cfg, 2500.0)
    sh = S.Shots(np.array([[20, 5]], dtype=np.int32), np.zeros((1, 0, 2), dtype=np.int32),
                 gpu_wavelets([15.0], [0.07], cfg.dt, cfg.nt))
    m = S.Model(d, dev(np.full((cfg.nz, cfg.nx), 2000.0)), 1, 0)
    seis = m.forward(sh)
    assert seis.shape == (1, 1, cfg.nt, 0)
    J, r = m.misfit(seis, seis)
    g = m.gradient(sh, r)
    torch.cuda.synchronize()
    assert J.item() == 0.0 and torch.count_nonzero(g).item() == 0
    m.close()


def test_c2_full_grid_short_window_parity():
    """The 1000 x 500 (+32-cell layer) launch configuration as timed: all 64
    shots in one launch, two steps per launch on the blocked tiles,
    checkpoints every 64 steps (here over a 250-step window).  Seismograms of
    two sampled shots against the oracle; the gradient driven by those two
    shots' residuals (zero residual for the others, which then add nothing)
    against the oracle's gradient for them."""
    cfg = synth.C2
    nt = 250
    true = synth.dipping_layers_anomalies(2003, cfg.nx, cfg.nz, cfg.dx)
    c0 = synth.smooth(true, 10.0)
    src, rec = synth.c2_geometry(cfg.nshots, cfg.nx)
    vmax = 4500.0
    d = S.desc(ndim=2, nx=cfg.nx, nz=cfg.nz, npml=cfg.npml, nt=nt, dx=cfg.dx, dt=cfg.dt,
               pml_R=cfg.pml_R, pml_vmax=vmax)
    wav = S.ricker(cfg.f0, cfg.ricker_t0, cfg.dt, nt)[None].repeat(cfg.nshots, 1).contiguous()
    sh = S.Shots(src, rec, wav)
    m = S.Model(d, dev(c0), cfg.nshots, rec.shape[1], 64)
    m.set_time_blocking(2)
    seis = m.forward(sh)
    sel = [5, 40]
    go = O.grid(ndim=2, nx=cfg.nx, nz=cfg.nz, npml=cfg.npml, nt=nt, dx=cfg.dx, dt=cfg.dt,
                pml_R=cfg.pml_R, pml_vmax=vmax)
    wo = np.stack([O.ricker(cfg.f0, cfg.ricker_t0, cfg.dt, nt)] * len(sel))
    op = O.ac2_forward(go, c0, src[sel], wo, rec[sel])
    oo = O.ac2_forward(go, true, src[sel], wo, rec[sel])
    _, ro = O.misfit(op, oo)
    dJ = torch.zeros_like(seis)
    dJ[sel, 0] = dev(ro)
    g = m.gradient(sh, dJ).cpu().numpy()[0]
    og, _ = O.ac2_gradient(go, c0, src[sel], wo, rec[sel], ro, ckpt=16)
    e1, e2 = rel_l2(seis.cpu().numpy()[sel, 0], op), rel_l2(g, og)
    print(f"C2 full grid, {nt} steps, shots {sel}: seis rel-L2 {e1:.2e}, grad rel-L2 {e2:.2e}")
    assert np.abs(op).max() > 0 and np.abs(og).max() > 0
    assert e1 <= SEIS_TOL and e2 <= GRAD_TOL
    m.close()


def test_checkpointed_equals_store_all_bitwise_and_deterministic():
    cfg = synth.C1.replace(nt=200)
    ct = synth.layered_c1()
    c0 = synth.smooth(ct, 10.0)
    src, rec = synth.c1_geometry()
    runs = [_run_case(cfg, ct, c0, src, rec, [10.0], [0.1], 3000.0, ckpt=k, want_gw=True)
            for k in (0, 200, 7, 0)]
    ref = runs[-1]
    for r in runs[:-1]:
        assert np.array_equal(r["grad"], ref["grad"])
        assert np.array_equal(r["gw"], ref["gw"])
        assert np.array_equal(r["pred"], ref["pred"])


def test_sweep_dot_product_identity_fp64():
    """<F s, d> = <s, F^T d> for the wavelet -> seismogram map with FP64
    reductions on the GPU (FP32 arithmetic in the sweeps)."""
    cfg = synth.C1.replace(nx=120, nz=90, npml=16, nt=400)
    c = 1700.0 + 800.0 * synth.smooth_random(5, (cfg.nz, cfg.nx), 5.0, 0.0, 1.0)
    src = np.array([[30, 4], [90, 60]], dtype=np.int32)
    rec = np.stack([synth.surface_receivers_2d(1, cfg.nx)[0]] * 2)
    d = gpu_desc(cfg, 2600.0)
    s = dev(synth.random_field(1, (2, cfg.nt)))
    dd = dev(synth.random_field(2, (2, 1, cfg.nt, cfg.nx)))
    sh = S.Shots(src, rec, s)
    m = S.Model(d, dev(c), 2, cfg.nx, 20)
    Fs = m.forward(sh)
    gw = torch.zeros((2, cfg.nt), dtype=torch.float32, device="cuda")
    m.gradient(sh, dd, g_wavelet=gw)
    lhs = S.dot_f64(Fs.reshape(-1), dd.reshape(-1)).item()
    rhs = S.dot_f64(s.reshape(-1), gw.reshape(-1)).item()
    nF = S.dot_f64(Fs.reshape(-1), Fs.reshape(-1)).item() ** 0.5
    nd = S.dot_f64(dd.reshape(-1), dd.reshape(-1)).item() ** 0.5
    # random-sign sums cancel: bound the defect by |F s| |d| (Cauchy-Schwarz)
    print(f"dot test (random d): {lhs:.12e} {rhs:.12e} defect/(|Fs||d|) {abs(lhs - rhs) / (nF * nd):.2e}")
    assert abs(lhs - rhs) <= 1e-5 * nF * nd
    # d = F s: <F s, F s> = <s, F^T F s>, no cancellation
    m.forward(sh)          # fresh checkpoints (same geometry)
    gw.zero_()
    m.gradient(sh, Fs, g_wavelet=gw)
    lhs2 = nF * nF
    rhs2 = S.dot_f64(s.reshape(-1), gw.reshape(-1)).item()
    print(f"dot test (d = F s): {lhs2:.12e} {rhs2:.12e} rel {abs(lhs2 - rhs2) / lhs2:.2e}")
    assert abs(lhs2 - rhs2) <= 1e-5 * lhs2


def test_misfit_fp64_matches_oracle():
    rng = np.random.default_rng(4)
    a = rng.standard_normal(3_000_001).astype(np.float32)
    b = rng.standard_normal(3_000_001).astype(np.float32)
    J, r = O.misfit(a.astype(np.float64), b.astype(np.float64))
    da, db = dev(a), dev(b)
    Jd = torch.empty(1, dtype=torch.float64, device="cuda")
    rd = torch.empty_like(da)
    assert S.lib().misfit(None, S._ptr(da), S._ptr(db), a.size, S._ptr(Jd), S._ptr(rd), S._stream()) == 0
    d = gpu_desc(synth.C1, 3000.0)
    m = S.Model(d, dev(synth.layered_c1()), 1, 101)
    J2, r2 = m.misfit(da, db)
    # the residual is rounded to FP32 before the FP64 accumulation
    assert Jd.item() == pytest.approx(J, rel=1e-8)
    assert J2.item() == pytest.approx(J, rel=1e-8)
    r32 = (a - b).astype(np.float64)
    assert Jd.item() == pytest.approx(0.5 * np.dot(r32, r32), rel=1e-12)
    assert np.array_equal(rd.cpu().numpy(), (a - b))
    assert np.array_equal(r2.cpu().numpy(), (a - b))


def test_error_paths_on_device():
    cfg = synth.C1
    d = gpu_desc(cfg, 3000.0)
    src, rec = synth.c1_geometry()
    wav = gpu_wavelets([10.0], [0.1], cfg.dt, cfg.nt)
    m = S.Model(d, dev(synth.layered_c1()), 1, 101)
    bad = src.copy()
    bad[0, 0] = cfg.nx
    with pytest.raises(S.SeisError) as e:
        m.forward(S.Shots(bad, rec, wav))
    assert e.value.code == S.SG_EINVAL
    # adjoint before a checkpointed forward of these shots
    m.forward(S.Shots(src, rec, wav), save_ckpt=False)
    with pytest.raises(S.SeisError) as e:
        m.gradient(S.Shots(src, rec, wav), torch.zeros((1, 1, cfg.nt, 101), device="cuda"))
    assert e.value.code == S.SG_ESTATE
    # unstable time step
    with pytest.raises(S.SeisError) as e:
        S.Model(gpu_desc(cfg.replace(dt=2e-3), 3000.0), dev(synth.layered_c1()), 1, 101)
    assert e.value.code == S.SG_EUNSTABLE


def test_discrete_energy_conserved_rigid_no_layer_fp32():
    """Rigid walls, no absorbing layer, the source switched off after 80
    steps: leapfrog conserves E^{n+1/2} = 1/2 sum (u^{n+1} - u^n)^2 / (dt^2 c^2)
    + 1/2 sum u^{n+1} (-L u^n) exactly (L the 8th-order Laplacian with zero
    values beyond the grid, a symmetric operator).  A receiver on every cell
    records the GPU's whole FP32 field at every step; the energy is summed in
    FP64 here.  Drift over 1400 steps <= 1e-5 of E."""
    n, dx, dt, nt, off = 64, 10.0, 1e-3, 1500, 80
    cfg = synth.C1.replace(nx=n, nz=n, npml=0, nt=nt, dx=dx, dt=dt)
    c = 1500.0 + 1500.0 * synth.smooth_random(31, (n, n), 4.0, 0.0, 1.0)
    rec = np.array([[[ix, iz] for iz in range(n) for ix in range(n)]], dtype=np.int32)
    wav = S.ricker(25.0, 0.04, dt, nt)
    wav[off:] = 0.0
    sh = S.Shots(np.array([[20, 29]], dtype=np.int32), rec, wav[None].contiguous())
    m = S.Model(gpu_desc(cfg, 3000.0), dev(c), 1, rec.shape[1])
    u = m.forward(sh, save_ckpt=False).cpu().numpy()[0, 0].reshape(nt, n, n).astype(np.float64)  # u^{k+1}
    m.close()
    a = [-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0]

    def lap(f):
        p = np.pad(f, 4)
        out = 2.0 * a[0] * f
        for k in range(1, 5):
            out += a[k] * (p[4 + k:4 + k + n, 4:4 + n] + p[4 - k:4 - k + n, 4:4 + n]
                           + p[4:4 + n, 4 + k:4 + k + n] + p[4:4 + n, 4 - k:4 - k + n])
        return out / dx ** 2

    E = np.array([0.5 * np.sum((u[j + 1] - u[j]) ** 2 / (dt * dt * c * c)) - 0.5 * np.sum(u[j + 1] * lap(u[j]))
                  for j in range(off, nt - 1)])
    drift = np.max(np.abs(E - E[0])) / E[0]
    print(f"energy drift over {nt - 1 - off} steps (FP32 fields, FP64 sums): {drift:.2e}")
    assert E[0] > 0 and drift <= 1e-5
