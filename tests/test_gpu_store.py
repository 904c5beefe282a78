"""Workspace beyond the minimum holds the adjoint snapshots of the last
checkpoint segments: a checkpointed forward writes them and the adjoint
skips those segments' restore and recomputation.  The snapshots are the same
values either way, so seismograms and gradients must be bitwise equal with
0, some and all segments stored (2-D acoustic with time blocking, 3-D
acoustic, 2-D elastic)."""
import numpy as np
import pytest
import torch

from gpu_common import S, synth, dev

pytestmark = pytest.mark.gpu


def _grads(d, models, shots, nrec, ckpt, store):
    ns = shots.nshots
    kw = dict(vs=dev(models[1]), rho=dev(models[2])) if len(models) == 3 else {}
    mt = S.Model(d, dev(models[0] * 1.05), ns, nrec, ckpt, **kw)
    obs = mt.forward(shots, save_ckpt=False)
    m = S.Model(d, dev(models[0]), ns, nrec, ckpt, store_segments=store, **kw)
    pred = m.forward(shots, save_ckpt=True)
    _, resid = m.misfit(pred, obs)
    g = m.gradient(shots, resid)
    torch.cuda.synchronize()
    g = g if isinstance(g, tuple) else (g,)
    return [pred.cpu()] + [x.cpu() for x in g]


def _check(d, models, shots, nrec, ckpt, nseg):
    ref = _grads(d, models, shots, nrec, ckpt, 0)
    for store in (2, nseg):
        got = _grads(d, models, shots, nrec, ckpt, store)
        for a, b in zip(ref, got):
            assert torch.equal(a, b), store
    assert all(torch.count_nonzero(x) > 0 for x in ref[1:])


def test_stored_segments_2d_acoustic():
    nx, nz, P, nt, ckpt = 300, 180, 16, 250, 20
    c = synth.smooth_random(5, (nz, nx), 8.0, 1600.0, 3200.0)
    src = np.array([[150, 90], [40, 5]], dtype=np.int32)
    rec = np.stack([synth.surface_receivers_2d(1, nx)[0]] * 2)
    d = S.desc(nx=nx, nz=nz, npml=P, nt=nt, dx=10.0, dt=1e-3, pml_vmax=3400.0)
    wav = torch.stack([S.ricker(12.0, 1.0 / 12.0, 1e-3, nt)] * 2)
    _check(d, [c], S.Shots(src, rec, wav), nx, ckpt, -(-nt // ckpt))


def test_stored_segments_3d_acoustic():
    n, P, nt, ckpt = 40, 10, 120, 11
    c = synth.smooth_random(4, (n, n, n), 6.0, 1600.0, 2600.0)
    src = np.array([[20, 20, 5]], dtype=np.int32)
    rec = np.array([[[x, y, 0] for y in range(0, n, 4) for x in range(0, n, 4)]], dtype=np.int32)
    d = S.desc(ndim=3, nx=n, ny=n, nz=n, npml=P, nt=nt, dx=10.0, dt=1e-3, pml_vmax=2700.0)
    wav = S.ricker(15.0, 1.0 / 15.0, 1e-3, nt)[None].contiguous()
    _check(d, [c], S.Shots(src, rec, wav), rec.shape[1], ckpt, -(-nt // ckpt))


def test_stored_segments_2d_elastic():
    nx, nz, P, nt, ckpt = 90, 60, 16, 300, 17
    vp = 2000.0 + 1500.0 * synth.smooth_random(1, (nz, nx), 6.0, 0.0, 1.0)
    vs, rho = vp / 1.75, 310.0 * vp ** 0.25
    src = np.array([[45, 4]], dtype=np.int32)
    rec = np.stack([np.arange(nx), np.zeros(nx)], -1)[None].astype(np.int32)
    d = S.desc(ndim=2, physics=S.SG_ELASTIC, nx=nx, nz=nz, npml=P, nt=nt, dx=5.0, dt=0.5e-3,
               pml_vmax=3600.0, f0_pml=20.0)
    wav = S.ricker(20.0, 0.05, 0.5e-3, nt)[None].contiguous()
    _check(d, [vp, vs, rho], S.Shots(src, rec, wav, np.array([[1.0, 1.0, 0.0]])), nx, ckpt, -(-nt // ckpt))
