"""Learned preconditioner for gradient-descent FWI: training-data generation,
training, and the time-to-misfit comparison with plain gradient descent.

* Models: three flat layers with random interface depths and velocities on
  the 101 x 101 grid of the single-shot acoustic configuration (10 Hz Ricker
  at (50, 2), 101 surface receivers, 20-cell absorbing layer, 500 steps of
  1 ms); the initial model is the sigma = 10 Gaussian blur of the true one.
  Training seeds 0..199, evaluation seeds 10000..10019.
* Data: the plain batched inversion of the training models (all in one
  launch), 50 iterations; each iteration i gives the pair
  (g_i / rms(g_i), (m_true - m_i) / rms(m_true - m_i)).
* Network and training: the 37,601-parameter CNN of
  :mod:`paper_2003_06027_amd.cnn`, Adam on the masked mean squared error,
  101 x 101 fields in the corners of 128 x 128 frames, four frames per
  256 x 256 patch.
* Use: safeguarded descent (the learned direction must satisfy <p, g> < 0
  and lower the misfit on its first trial, else the plain step is taken;
  after two consecutive rejections a model stops asking the network).
* Also timed: batched L-BFGS (the paper's optimizer family, two-loop
  direction in library kernels) from the same start, same iteration cap.
* Measure: a misfit target fixed in advance, tau = 0.9 (a 10 % reduction
  of J); the wall-clock seconds (device synchronised) until each model first
  reaches J / J0 <= tau, for plain and for preconditioned descent (and
  L-BFGS), same step rule, same GPU, 150-iteration caps.  A model that never
  reaches tau counts as infinitely slow, so a median is finite only when
  more than half of the models reach the target.  (The cap is set so that
  plain descent, which needs about 120 iterations for the median model,
  reaches it.)

Every forward, misfit, adjoint, network and optimizer step runs in the
library's HIP kernels; this module sequences calls and keeps scalar
bookkeeping on the host.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np
import torch

from . import cnn as N
from . import fwi
from . import seisgrad as S
from . import synth


@dataclasses.dataclass
class TTMConfig:
    train_seeds: tuple = tuple(range(200))
    eval_seeds: tuple = tuple(range(10000, 10020))
    train_iters: int = 50
    eval_iters: int = 150
    tau: float = 0.9          # misfit target J/J0, fixed before any run
    epochs: int = 20
    batch_patches: int = 8
    lr: float = 1e-3
    val_frac: float = 0.1
    max_rejects: int = 2
    seed: int = 0
    nt: int = 500


@dataclasses.dataclass
class Problem:
    prop: fwi.Propagator
    true: torch.Tensor
    init: torch.Tensor
    obs: torch.Tensor


def c1_problem(seeds, nt=500, graphs=True) -> Problem:
    """B random three-layer models, one shot each, batched in one launch; the
    propagator replays its checkpoint segments as HIP graphs unless graphs is
    False (these small grids are bound by the launches otherwise)."""
    cfg = synth.C1.replace(nt=nt)
    B = len(seeds)
    true = np.stack([synth.random_layered(s, cfg.nx, cfg.nz) for s in seeds])
    init = np.stack([synth.smooth(t, 10.0) for t in true])
    src = np.array([[50, 2]] * B, dtype=np.int32)
    rec = synth.surface_receivers_2d(B, cfg.nx)
    d = S.desc(nx=cfg.nx, nz=cfg.nz, npml=cfg.npml, nt=nt, nmodels=B, dx=cfg.dx, dt=cfg.dt,
               pml_R=cfg.pml_R, pml_vmax=3500.0)
    wav = S.ricker(cfg.f0, cfg.ricker_t0, cfg.dt, nt)[None].repeat(B, 1).contiguous()
    prop = fwi.Propagator(d, S.Shots(src, rec, wav), store_segments=-1, graphs=graphs)
    dev = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
    t_d, i_d = dev(true), dev(init)
    obs = prop.forward(t_d, save_ckpt=False, keep=True).clone()
    return Problem(prop, t_d, i_d, obs)


class Recorder:
    """Direction callback of the plain inversion that keeps (g, m) per iteration."""

    def __init__(self):
        self.g, self.m = [], []

    def __call__(self, g, m, it):
        self.g.append(g.clone())
        self.m.append(m.clone())
        return -g, torch.zeros(g.shape[0], dtype=torch.bool)


class LearnedDirection:
    """Safeguarded learned direction; a model stops asking the network after
    `max_rejects` consecutive rejections."""

    def __init__(self, pre: N.Preconditioner, max_rejects=2):
        self.pre, self.max_rejects = pre, max_rejects
        self.consec = None
        self.off = None

    def __call__(self, g, m, it):
        B = g.shape[0]
        if self.off is None:
            self.off = np.zeros(B, dtype=bool)
            self.consec = np.zeros(B, dtype=int)
        p = self.pre.direction(g)
        if self.off.any():
            idx = torch.as_tensor(np.nonzero(self.off)[0], device=g.device)
            p[idx] = -g[idx]
        return p, torch.as_tensor(~self.off)

    def report(self, it, rejected):
        self.consec = np.where(rejected, self.consec + 1, np.where(self.off, self.consec, 0))
        self.off |= self.consec >= self.max_rejects

    def state(self):
        """Switch-off bookkeeping, saved with the inversion state."""
        return {} if self.off is None else {"off": self.off.copy(), "consec": self.consec.copy()}

    def load_state(self, st):
        if st:
            self.off, self.consec = st["off"].astype(bool), st["consec"].astype(int)


def generate_pairs(prob: Problem, iters: int, frame=128, seed=0):
    """Run the plain inversion and pack its (g, m_true - m) pairs into
    patches in a seeded random slot order; returns (x, t, mask, seconds)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rec = Recorder()
    fwi.batched_gd(prob.prop, prob.init, prob.obs, fwi.GDConfig(iters=iters), direction=rec)
    G = torch.cat(rec.g)                                    # [iters * B, nz, nx], iteration-major
    M = torch.cat(rec.m)
    T = prob.true.repeat(len(rec.g), 1, 1).contiguous()
    order = torch.as_tensor(np.random.default_rng(seed).permutation(G.shape[0]).astype(np.int32), device="cuda")
    x, _, _ = N.pack(G, frame, order=order, with_mask=False)
    t, mask, _ = N.pack(T, frame, b=M, order=order)
    torch.cuda.synchronize()
    return x, t, mask, time.perf_counter() - t0


def evaluate_loss(pre: N.Preconditioner, x, t, mask):
    """Mean masked loss over patches (batches of the workspace size)."""
    tot, n = 0.0, 0
    for s in range(0, x.shape[0], pre.max_patches):
        e = min(s + pre.max_patches, x.shape[0])
        p = pre.forward(x[s:e])
        L, _ = N.loss(p, t[s:e], mask[s:e], pre.ws, want_grad=False)
        tot += L.item() * (e - s)
        n += e - s
    return tot / max(n, 1)


def train(pre: N.Preconditioner, x, t, mask, cfg: TTMConfig, log=None):
    """Adam over contiguous batches of patches, batch order reshuffled every
    epoch; the last val_frac of the patches is held out."""
    nval = max(1, int(round(cfg.val_frac * x.shape[0])))
    ntr = x.shape[0] - nval
    xv, tv, mv = x[ntr:], t[ntr:], mask[ntr:]
    hist = {"val0": evaluate_loss(pre, xv, tv, mv), "train": [], "val": []}
    rng = np.random.default_rng(cfg.seed + 1)
    starts = np.arange(0, ntr, cfg.batch_patches)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ep in range(cfg.epochs):
        acc = torch.zeros(1, dtype=torch.float64, device="cuda")
        for s in rng.permutation(starts):
            e = min(s + cfg.batch_patches, ntr)
            acc += pre.train_step(x[s:e], t[s:e], mask[s:e], cfg.lr)
        hist["train"].append(acc.item() / len(starts))
        hist["val"].append(evaluate_loss(pre, xv, tv, mv))
        if log:
            log(f"epoch {ep + 1}: train {hist['train'][-1]:.4f} val {hist['val'][-1]:.4f}")
    torch.cuda.synchronize()
    hist["seconds"] = time.perf_counter() - t0
    return hist


def time_to_target(res: fwi.GDResult, tau: float):
    """Per model: seconds and iterations until J/J0 <= tau first holds (inf if never)."""
    rel = res.J / res.J[0]
    secs, its = [], []
    for b in range(rel.shape[1]):
        hit = np.nonzero(rel[:, b] <= tau)[0]
        secs.append(res.times[hit[0]] if hit.size else np.inf)
        its.append(int(hit[0]) if hit.size else np.inf)
    return np.array(secs), np.array(its)


def run(cfg: TTMConfig = TTMConfig(), log=None) -> dict:
    """The whole experiment; returns the measured figures."""
    out = {}
    train_prob = c1_problem(cfg.train_seeds, cfg.nt)
    x, t, mask, t_data = generate_pairs(train_prob, cfg.train_iters, seed=cfg.seed)
    train_prob.prop.close()
    del train_prob
    if log:
        log(f"data: {x.shape[0]} patches from {len(cfg.train_seeds)} inversions x {cfg.train_iters} its "
            f"in {t_data:.1f} s")
    pre = N.Preconditioner(cfg.batch_patches, seed=cfg.seed)
    hist = train(pre, x, t, mask, cfg, log)
    del x, t, mask
    ev = c1_problem(cfg.eval_seeds, cfg.nt)
    gd = fwi.batched_gd(ev.prop, ev.init, ev.obs, fwi.GDConfig(iters=cfg.eval_iters))
    tau = cfg.tau
    ld = LearnedDirection(pre, cfg.max_rejects)
    pc = fwi.batched_gd(ev.prop, ev.init, ev.obs, fwi.GDConfig(iters=cfg.eval_iters), direction=ld)
    lb = fwi.batched_lbfgs(ev.prop, ev.init, ev.obs, fwi.LBFGSConfig(iters=cfg.eval_iters))
    s_gd, i_gd = time_to_target(gd, tau)
    s_pc, i_pc = time_to_target(pc, tau)
    s_lb, i_lb = time_to_target(lb, tau)
    offered = pc.guarded.sum()
    out.update({
        "tau": tau,
        "median_seconds_gd": float(np.median(s_gd)), "median_seconds_cnn": float(np.median(s_pc)),
        "median_iters_gd": float(np.median(i_gd)), "median_iters_cnn": float(np.median(i_pc)),
        "reached_gd": int(np.isfinite(s_gd).sum()), "reached_cnn": int(np.isfinite(s_pc).sum()),
        "models": len(cfg.eval_seeds),
        "seconds_per_iter_gd": float(gd.times[-1] / (len(gd.times) - 1)),
        "seconds_per_iter_cnn": float(pc.times[-1] / (len(pc.times) - 1)),
        "eval_iters": cfg.eval_iters,
        "final_rel_misfit_median_gd": float(np.median(gd.J[-1] / gd.J[0])),
        "final_rel_misfit_median_cnn": float(np.median(pc.J[-1] / pc.J[0])),
        "median_seconds_lbfgs": float(np.median(s_lb)), "median_iters_lbfgs": float(np.median(i_lb)),
        "reached_lbfgs": int(np.isfinite(s_lb).sum()),
        "final_rel_misfit_median_lbfgs": float(np.median(lb.J[-1] / lb.J[0])),
        "lbfgs_misfit_never_increases": bool(np.all(np.diff(lb.J, axis=0) <= 0)),
        "cnn_acceptance": float(1.0 - pc.rejected.sum() / offered) if offered else 0.0,
        "cnn_misfit_never_increases": bool(np.all(np.diff(pc.J, axis=0) <= 0)),
        "cnn_offered_steps": int(offered),
        "data_seconds": t_data, "train_seconds": hist["seconds"],
        "train_loss_first_last": [hist["train"][0], hist["train"][-1]],
        "val_loss_untrained_trained": [hist["val0"], hist["val"][-1]],
    })
    saved = out["median_seconds_gd"] - out["median_seconds_cnn"]
    cost = t_data + hist["seconds"]
    out["break_even_batches"] = float(cost / saved) if np.isfinite(saved) and saved > 0 else None
    ev.prop.close()
    return out
