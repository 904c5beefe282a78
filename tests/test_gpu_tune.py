"""The sweep autotuner: its graph candidate (the library's segment graphs,
captured by the first checkpointed forward + misfit + adjoint and replayed
by the next) gives the eager results bit for bit on every step (with other
eager GPU work and synchronisations between steps), and the tuner caches its
choice per workload in JSON."""
import dataclasses
import json

import numpy as np
import pytest
import torch

from gpu_common import S, synth, dev
from paper_2003_06027_amd import tune

pytestmark = pytest.mark.gpu


def _problem(B=4, nt=300):
    cfg = synth.C1.replace(nt=nt)
    true = np.stack([synth.random_layered(s) for s in range(B)])
    init = np.stack([synth.smooth(t, 10.0) for t in true])
    d = S.desc(nx=cfg.nx, nz=cfg.nz, npml=cfg.npml, nt=nt, nmodels=B, dx=cfg.dx, dt=cfg.dt, pml_vmax=3500.0)
    wav = S.ricker(cfg.f0, cfg.ricker_t0, cfg.dt, nt)[None].repeat(B, 1).contiguous()
    sh = S.Shots(np.array([[50, 2]] * B, dtype=np.int32), synth.surface_receivers_2d(B, cfg.nx), wav)
    mt = S.Model(d, dev(true), B, cfg.nx)
    obs = mt.forward(sh, save_ckpt=False).clone()
    mt.close()
    return d, sh, dev(init), obs


def test_graph_replay_equals_eager_on_every_replay():
    d, sh, vp, obs = _problem()
    eager = tune.Runner(d, sh, vp, obs, tune.Strategy(2, False))
    g_ref = eager.step().clone()
    s_ref, J_ref = eager.seis.clone(), eager.J.clone()
    graph = tune.Runner(d, sh, vp, obs, tune.Strategy(2, True))
    for rep in range(3):
        graph.seis.zero_()
        if graph.out is not None:
            graph.out.zero_()
        torch.cuda.synchronize()
        g = graph.step()
        torch.cuda.synchronize()
        assert torch.equal(graph.seis, s_ref), rep
        assert torch.equal(g, g_ref), rep
        assert torch.equal(graph.J, J_ref), rep
        eager.step()                       # unrelated eager work between replays
        torch.cuda.synchronize()
    graph.close()
    eager.close()


def test_tuner_measures_once_then_reads_its_cache(tmp_path, monkeypatch):
    d, sh, vp, _ = _problem(B=2, nt=200)
    cache = str(tmp_path / "tune.json")
    best = tune.tune(d, sh, vp, cache=cache, log=print)
    table = json.load(open(cache))
    (entry,) = table.values()
    assert entry["strategy"] == dataclasses.asdict(best)
    assert len(entry["ms"]) == 4           # 1 or 2 steps per launch, eager or graph
    monkeypatch.setattr(tune, "measure", lambda *a, **k: (_ for _ in ()).throw(AssertionError("re-measured")))
    assert tune.tune(d, sh, vp, cache=cache) == best


def _run(m, sh, obs=None):
    seis = m.forward(sh)
    if obs is None:
        obs = (seis * 0.95).contiguous()
    _, r = m.misfit(seis, obs)
    g = m.gradient(sh, r)
    torch.cuda.synchronize()
    return seis.clone(), tuple(t.clone() for t in (g if isinstance(g, tuple) else (g,))), obs


def test_3d_chunk_settings_leave_results_bitwise_unchanged():
    """3-D z-chunk lengths of the forward and adjoint tile passes and of the
    layer work items (ragged last chunks, 64-plane adjoint chunks, 16-plane
    layer items) change the launch, not one value."""
    nx, ny, nz, P, nt = 45, 37, 70, 12, 60                  # padded 69 x 61 x 94: several chunks
    c = 1600.0 + 1200.0 * synth.smooth_random(21, (nz, ny, nx), 3.0, 0.0, 1.0)
    d = S.desc(ndim=3, nx=nx, ny=ny, nz=nz, npml=P, nt=nt, dx=10.0, dt=1e-3, pml_vmax=2800.0)
    src = np.array([[22, 18, 2], [5, 30, 60]], dtype=np.int32)
    xs, ys = np.meshgrid(np.arange(0, nx, 4), np.arange(0, ny, 4), indexing="xy")
    r = np.stack([xs.ravel(), ys.ravel(), np.zeros(xs.size, dtype=int)], -1)
    rec = np.stack([r, r]).astype(np.int32)
    wav = torch.stack([S.ricker(20.0, 0.05, 1e-3, nt), S.ricker(25.0, 0.04, 1e-3, nt)])
    sh = S.Shots(src, rec, wav)
    m = S.Model(d, dev(c), 2, rec.shape[1], 9)
    seis0, g0, obs = _run(m, sh)
    for fwd, adj, lay in ((16, 48, 64), (48, 32, 16), (64, 64, 32), (32, 64, 32)):
        m.set_tuning(S.SG_TUNE_CHUNK_FWD3, fwd)
        m.set_tuning(S.SG_TUNE_CHUNK_ADJ3, adj)
        m.set_tuning(S.SG_TUNE_CHUNK_LAYER3, lay)
        seis, g, _ = _run(m, sh, obs)
        assert torch.equal(seis, seis0), (fwd, adj, lay)
        assert torch.equal(g[0], g0[0]), (fwd, adj, lay)
    with pytest.raises(S.SeisError):
        m.set_tuning(S.SG_TUNE_CHUNK_FWD3, 20)             # not a multiple of 8
    with pytest.raises(S.SeisError):
        m.set_tuning(S.SG_TUNE_SHOT_GROUP, 2)              # an elastic setting on a 3-D model
    m.close()


def test_elastic_block_width_and_shot_groups():
    """Elastic cell blocks of 64 x 4 give the 32 x 8 results bit for bit; one
    shot per thread instead of groups of 4 changes only the gradient's
    summation order (rel-L2 within 1e-5 of each other)."""
    nx, nz, P, nt = 90, 57, 12, 300
    vp = 1800.0 + 2200.0 * synth.smooth_random(6027, (nz, nx), 8.0, 0.0, 1.0)
    vs = vp / 1.75
    rho = 310.0 * vp ** 0.25
    d = S.desc(ndim=2, physics=S.SG_ELASTIC, nx=nx, nz=nz, npml=P, nt=nt, dx=5.0, dt=0.5e-3, pml_vmax=4000.0,
               f0_pml=15.0)
    src = np.array([[20, 5], [45, 20], [70, 40], [30, 50]], dtype=np.int32)
    mt = np.array([[1.0, 1.0, 0.0], [-0.5, 0.5, 0.86], [0.3, -0.3, 0.95], [1.0, 0.2, 0.1]])
    rec = np.stack([np.stack([np.arange(0, nx, 3), np.zeros(nx // 3)], -1)] * 4).astype(np.int32)
    wav = S.ricker(20.0, 0.05, 0.5e-3, nt)[None].repeat(4, 1).contiguous()
    sh = S.Shots(src, rec, wav, mt=mt)
    m = S.Model(d, dev(vp), 4, rec.shape[1], 20, vs=dev(vs), rho=dev(rho))
    seis0, g0, obs = _run(m, sh)
    m.set_tuning(S.SG_TUNE_BLOCK_X, 64)
    seis, g, _ = _run(m, sh, obs)
    assert torch.equal(seis, seis0) and all(torch.equal(a, b) for a, b in zip(g, g0))
    m.set_tuning(S.SG_TUNE_SHOT_GROUP, 1)
    seis, g1, _ = _run(m, sh, obs)
    assert torch.equal(seis, seis0)
    errs = [float((a.double() - b.double()).norm() / b.double().norm()) for a, b in zip(g1, g0)]   # ~1e-25: FP64
    print("shot groups 1 vs 4: gradient rel-L2", errs)
    assert max(errs) <= 1e-5
    with pytest.raises(S.SeisError):
        m.set_tuning(S.SG_TUNE_SHOT_GROUP, 3)
    m.close()
