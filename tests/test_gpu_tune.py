"""The sweep autotuner: graph replay of a whole checkpointed forward + misfit
+ adjoint gives the eager results bit for bit on every replay (with other
eager GPU work and synchronisations between replays), and the tuner caches
its choice per workload in JSON."""
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
    assert entry["strategy"] == {"time_blocking": best.time_blocking, "graphs": best.graphs}
    assert len(entry["ms"]) == 4
    monkeypatch.setattr(tune, "measure", lambda *a, **k: (_ for _ in ()).throw(AssertionError("re-measured")))
    assert tune.tune(d, sh, vp, cache=cache) == best
