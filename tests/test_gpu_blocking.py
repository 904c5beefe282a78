"""Time blocking of the 2-D acoustic sweeps: two steps per launch on tiles
whose cells and 8-cell halo are physical and hold no receiver within 4 cells.

Every value is computed with the same operations as in the one-step
launches, so seismograms, gradients and wavelet gradients must be bitwise
equal with blocking on and off -- including segments of odd length, sources
inside blocked tiles and their halos, and receivers that exclude tiles.  The
blocked path is also compared with the FP64 oracle on a grid that has
blocked tiles (seismograms rel-L2 <= 1e-4, gradients <= 1e-3)."""
import numpy as np
import pytest
import torch

from gpu_common import O, S, synth, rel_l2, dev

pytestmark = pytest.mark.gpu

TX, TZ, HALO = 64, 32, 8


def blocked_tiles(nx, nz, P, rec):
    """Host mirror of the library's tile classification (for the test's own check)."""
    NX, NZ = nx + 2 * P, nz + 2 * P
    ntx, ntz = -(-NX // TX), -(-NZ // TZ)
    n = 0
    for tz in range(ntz):
        for tx in range(ntx):
            x0, z0 = tx * TX, tz * TZ
            inner = x0 - HALO >= P and x0 + TX + HALO <= P + nx and z0 - HALO >= P and z0 + TZ + HALO <= P + nz
            near_rec = any(x0 - 4 <= r[0] + P < x0 + TX + 4 and z0 - 4 <= r[1] + P < z0 + TZ + 4
                           for r in rec.reshape(-1, 2))
            n += inner and not near_rec
    return n


def _run(d, c_true, c0, src, rec, wav, ckpt, steps, pair=1):
    ns = src.shape[0]
    sh = S.Shots(src, rec, wav)
    mt = S.Model(d, dev(c_true), ns, rec.shape[1], ckpt)
    mt.set_time_blocking(steps)
    mt.set_tuning(S.SG_TUNE_PAIR, pair)
    obs = mt.forward(sh, save_ckpt=False)
    m = S.Model(d, dev(c0), ns, rec.shape[1], ckpt)
    m.set_time_blocking(steps)
    m.set_tuning(S.SG_TUNE_PAIR, pair)
    pred = m.forward(sh, save_ckpt=True)
    J, resid = m.misfit(pred, obs)
    gw = torch.zeros_like(wav)
    g = m.gradient(sh, resid, g_wavelet=gw)
    torch.cuda.synchronize()
    return obs.cpu(), pred.cpu(), J.item(), g.cpu(), gw.cpu()


@pytest.mark.parametrize("ckpt,nt", [(0, 250), (7, 251)])
def test_blocked_and_single_step_sweeps_are_bitwise_equal(ckpt, nt):
    nx, nz, P = 300, 180, 16
    ct = synth.smooth_random(5, (nz, nx), 8.0, 1600.0, 3200.0)
    c0 = synth.smooth(ct, 6.0)
    # shot 0 inside a blocked tile, shot 2 in the 4-cell halo of one
    src = np.array([[150, 90], [40, 5], [242, 100]], dtype=np.int32)
    rec = np.stack([synth.surface_receivers_2d(1, nx)[0]] * 3)
    rec[1, 7] = [200, 120]                                              # interior receivers exclude tiles
    rec[2, 3] = [90, 70]
    assert blocked_tiles(nx, nz, P, rec) >= 4
    d = S.desc(nx=nx, nz=nz, npml=P, nt=nt, dx=10.0, dt=1e-3, pml_vmax=3200.0)
    wav = torch.stack([S.ricker(f, 1.0 / f, 1e-3, nt) for f in (12.0, 10.0, 15.0)])
    a = _run(d, ct, c0, src, rec, wav, ckpt, 2)
    b = _run(d, ct, c0, src, rec, wav, ckpt, 1)
    for x, y, name in zip(a, b, ("obs", "pred", "J", "grad", "g_wavelet")):
        if isinstance(x, float):
            assert x == y, name
        else:
            assert torch.equal(x, y), name
    assert torch.count_nonzero(a[3]) > 0 and torch.count_nonzero(a[4][0]) > 0


@pytest.mark.parametrize("ckpt,nt", [(0, 250), (7, 251)])
def test_paired_launches_are_bitwise_equal(ckpt, nt):
    """With surface receivers only (no one-step tiles away from the layer),
    the near tiles' step and the blocked tiles' double step run as one grid
    by default; paired, apart and unblocked runs agree bit for bit."""
    nx, nz, P = 300, 180, 16
    ct = synth.smooth_random(5, (nz, nx), 8.0, 1600.0, 3200.0)
    c0 = synth.smooth(ct, 6.0)
    src = np.array([[150, 90], [40, 5], [242, 100]], dtype=np.int32)
    rec = np.stack([synth.surface_receivers_2d(1, nx)[0]] * 3)
    assert blocked_tiles(nx, nz, P, rec) >= 4
    d = S.desc(nx=nx, nz=nz, npml=P, nt=nt, dx=10.0, dt=1e-3, pml_vmax=3200.0)
    wav = torch.stack([S.ricker(f, 1.0 / f, 1e-3, nt) for f in (12.0, 10.0, 15.0)])
    a = _run(d, ct, c0, src, rec, wav, ckpt, 2, pair=1)
    b = _run(d, ct, c0, src, rec, wav, ckpt, 2, pair=0)
    c = _run(d, ct, c0, src, rec, wav, ckpt, 1)
    for x, y, z, name in zip(a, b, c, ("obs", "pred", "J", "grad", "g_wavelet")):
        if isinstance(x, float):
            assert x == y == z, name
        else:
            assert torch.equal(x, y) and torch.equal(x, z), name
    assert torch.count_nonzero(a[3]) > 0 and torch.count_nonzero(a[4][0]) > 0


def test_blocked_grid_matches_oracle():
    nx, nz, P, nt = 200, 120, 12, 400
    ct = synth.smooth_random(11, (nz, nx), 6.0, 1700.0, 3000.0)
    c0 = synth.smooth(ct, 8.0)
    src = np.array([[100, 60], [30, 3]], dtype=np.int32)
    rec = np.stack([synth.surface_receivers_2d(1, nx)[0]] * 2)
    assert blocked_tiles(nx, nz, P, rec) >= 4
    g = O.grid(ndim=2, nx=nx, nz=nz, npml=P, nt=nt, dx=10.0, dt=1e-3, pml_vmax=3000.0)
    d = S.desc(nx=nx, nz=nz, npml=P, nt=nt, dx=10.0, dt=1e-3, pml_vmax=3000.0)
    wav = torch.stack([S.ricker(12.0, 1.0 / 12.0, 1e-3, nt)] * 2)
    obs, pred, J, grad, _ = _run(d, ct, c0, src, rec, wav, 0, 2)
    wo = np.stack([O.ricker(12.0, 1.0 / 12.0, 1e-3, nt)] * 2)
    so = O.ac2_forward(g, c0, src, wo, rec)
    oo = O.ac2_forward(g, ct, src, wo, rec)
    es = rel_l2(pred.numpy()[:, 0], so)
    og, _ = O.ac2_gradient(g, c0, src, wo, rec, so - oo)
    eg = rel_l2(grad.numpy()[0], og)
    print(f"blocked grid: seismogram rel-L2 {es:.2e}, gradient rel-L2 {eg:.2e}")
    assert es <= 1e-4 and eg <= 1e-3
