"""L-BFGS helpers on the GPU against the FP64 oracle (two-loop recursion
over each model's own ring of pairs, FP32 vectors with FP64 inner
products: rel-L2 <= 1e-5), and the batched L-BFGS inversion: the misfit
never increases and beats plain gradient descent at the same iteration
count on C1-style models."""
import numpy as np
import pytest
import torch

from gpu_common import S, synth, rel_l2, dev
from oracle import lbfgs as LB
from paper_2003_06027_amd import fwi

pytestmark = pytest.mark.gpu


def test_push_and_two_loop_match_oracle_per_model():
    rng = np.random.default_rng(3)
    B, n, mem = 3, 5000, 4
    counts = [0, 2, 4]                      # ragged histories, model 2 wraps around the ring
    S_ = torch.zeros((mem, B, n), device="cuda")
    Y_ = torch.zeros_like(S_)
    ysyy = torch.zeros((mem, B, 2), dtype=torch.float64, device="cuda")
    pairs = [[] for _ in range(B)]
    newest = [-1] * B
    for step in range(6):                   # push up to 6 pairs, keep the last `counts[b]`
        m_old = rng.standard_normal((B, n)).astype(np.float32)
        m_new = m_old + 0.1 * rng.standard_normal((B, n)).astype(np.float32)
        g_old = rng.standard_normal((B, n)).astype(np.float32)
        g_new = g_old + 2.0 * (m_new - m_old) + 0.01 * rng.standard_normal((B, n)).astype(np.float32)
        slot = np.array([(newest[b] + 1) % mem if step >= 6 - counts[b] else -1 for b in range(B)], np.int32)
        # device copies stay referenced until the launch has run (a dropped
        # temporary's block would be reused by the next allocation)
        args = [dev(slot, torch.int32), dev(m_new), dev(m_old), dev(g_new), dev(g_old)]
        S._check(S.lib().lbfgs_push(B, n, mem, *[S._ptr(t) for t in args], S._ptr(S_), S._ptr(Y_), S._ptr(ysyy),
                                    S._stream()))
        torch.cuda.synchronize()
        del args
        for b in range(B):
            if slot[b] >= 0:
                pairs[b].append((np.float32(m_new[b] - m_old[b]).astype(np.float64),
                                 np.float32(g_new[b] - g_old[b]).astype(np.float64)))
                newest[b] = slot[b]
    ys = ysyy.cpu().numpy()
    for b in range(B):
        for j, (s, y) in enumerate(pairs[b][::-1]):
            k = (newest[b] - j) % mem
            np.testing.assert_array_equal(S_[k, b].cpu().numpy(), s.astype(np.float32))
            assert ys[k, b, 0] == pytest.approx(float(y @ s), rel=1e-12)
    g = rng.standard_normal((B, n)).astype(np.float32)
    hist = dev(np.stack([counts, newest], 1).astype(np.int32), torch.int32)
    gd = dev(g)
    p = torch.empty((B, n), device="cuda")
    S._check(S.lib().lbfgs_direction(B, n, mem, S._ptr(hist), S._ptr(S_), S._ptr(Y_), S._ptr(ysyy),
                                     S._ptr(gd), S._ptr(p), S._stream()))
    for b in range(B):
        ref = LB.two_loop(g[b], [s for s, _ in pairs[b]], [y for _, y in pairs[b]])
        e = rel_l2(p[b].cpu().numpy(), ref)
        print(f"model {b} ({counts[b]} pairs): rel-L2 {e:.2e}")
        assert e <= 1e-5
    np.testing.assert_array_equal(p[0].cpu().numpy(), -g[0])


def test_batched_lbfgs_decreases_misfit_faster_than_gd():
    B = 3
    cfg = synth.C1.replace(nt=400)
    true = np.stack([synth.random_layered(200 + b) for b in range(B)])
    init = np.stack([synth.smooth(t, 10.0) for t in true])
    src = np.array([[50, 2]] * B, dtype=np.int32)
    rec = np.stack([synth.surface_receivers_2d(1, cfg.nx)[0]] * B)
    wav = S.ricker(cfg.f0, cfg.ricker_t0, cfg.dt, cfg.nt)[None].repeat(B, 1).contiguous()
    d = S.desc(nx=cfg.nx, nz=cfg.nz, npml=cfg.npml, nt=cfg.nt, nmodels=B, dx=cfg.dx, dt=cfg.dt, pml_vmax=3500.0)
    prop = fwi.Propagator(d, S.Shots(src, rec, wav), store_segments=-1)
    obs = prop.forward(dev(true), save_ckpt=False).clone()
    lb = fwi.batched_lbfgs(prop, dev(init), obs, fwi.LBFGSConfig(iters=10))
    gd = fwi.batched_gd(prop, dev(init), obs, fwi.GDConfig(iters=10))
    print("L-BFGS J/J0:", lb.J[-1] / lb.J[0], " GD J/J0:", gd.J[-1] / gd.J[0])
    assert np.all(np.diff(lb.J, axis=0) <= 0)
    assert np.median(lb.J[-1] / lb.J[0]) < np.median(gd.J[-1] / gd.J[0])
