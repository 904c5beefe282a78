"""Training-system forms around the plain method.

* :class:`Propagator` -- a reusable workspace plus model handle for one grid
  and acquisition: the velocity (and, elastic, vs and rho) can change between
  calls without reallocating.
* :class:`SeisForward` -- a ``torch.autograd.Function`` whose forward is the
  library's forward sweep (with wavefield checkpoints) and whose backward is
  the hand-written adjoint sweep: for any loss of the seismograms, autograd
  passes dL/dd and receives dL/dvp (elastic: dL/dvp, dL/dvs, dL/drho).  This
  is the paper's per-operator reverse rule (Method, the display after
  Eq. (5): dU_k/dU_{k-1} = A^T, dU_k/dtheta = dA/dtheta U_{k-1}) applied to
  the whole recursion at once.
* :func:`batched_gd` -- plain gradient descent FWI on B models batched in one
  launch (every model its own shots), with a normalised step and
  backtracking, the baseline the learned preconditioner is compared with.

All arithmetic of the forward, misfit and adjoint runs in the library's HIP
kernels; this module only sequences calls and does per-model scalar
bookkeeping.
"""
from __future__ import annotations

import dataclasses
import json
import os
import time

import numpy as np
import torch

from . import seisgrad as S


class Propagator:
    """Workspace + model for a fixed grid, shot batch and checkpoint interval."""

    def __init__(self, desc, shots: "S.Shots", ckpt_every: int = 0, device="cuda", store_segments: int = 0,
                 graphs: bool = False):
        """store_segments: checkpoint segments whose adjoint snapshots the
        checkpointed forward keeps in the workspace (-1: all of them), so the
        adjoint does not recompute them.  graphs: run every checkpoint
        segment as a replayed HIP graph (the library's segment graphs; the
        same results bit for bit, without the per-launch host cost).  The
        model is prepared once and its parameters replaced in place by later
        calls, so that the captured graphs stay valid while the forwards and
        misfits of the inversion loops write into the propagator's own
        seismogram and residual buffers (keep=True)."""
        self.d = desc
        self.graphs = graphs
        self._seis = {}            # save_ckpt -> the kept seismogram buffer
        self.resid = None          # the kept residual buffer
        self.shots = shots
        self.ckpt = ckpt_every
        self.elastic = desc.physics == S.SG_ELASTIC
        self.nbytes = S.workspace_bytes(desc, shots.nshots, shots.nrec, ckpt_every)
        if store_segments:
            K = ckpt_every if ckpt_every > 0 else int(np.ceil(np.sqrt(desc.nt)))
            nseg = -(-desc.nt // min(K, desc.nt))
            n = nseg if store_segments < 0 else min(store_segments, nseg)
            self.nbytes += n * S.snapshot_segment_bytes(desc, shots.nshots, ckpt_every)
        self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.model = None
        self.generation = 0

    def set_model(self, vp, vs=None, rho=None):
        """Prepare the model on the workspace (the first call), or give it
        new parameters (later calls: update_model keeps its lists, tables
        and graphs)."""
        vs = None if vs is None else vs.detach()
        rho = None if rho is None else rho.detach()
        if self.model is None:
            self.model = S.Model(self.d, vp.detach(), self.shots.nshots, self.shots.nrec, self.ckpt,
                                 vs=vs, rho=rho, ws=self.ws)
            if self.graphs:
                self.model.set_tuning(S.SG_TUNE_GRAPHS, 1)
        else:
            self.model.update(vp.detach(), vs, rho)
        self.generation += 1
        return self.model

    def forward(self, vp, vs=None, rho=None, save_ckpt=True, keep=False):
        """Seismograms of the shots for these parameters.  keep: into the
        propagator's buffer for this checkpoint mode, which the next kept
        forward of the same mode overwrites."""
        self.set_model(vp, vs, rho)
        seis = None
        if keep:
            seis = self._seis.get(bool(save_ckpt))
            if seis is None:
                shape = (self.shots.nshots, 2 if self.elastic else 1, self.d.nt, self.shots.nrec)
                seis = self._seis[bool(save_ckpt)] = torch.empty(shape, dtype=torch.float32, device=self.ws.device)
        return self.model.forward(self.shots, seis=seis, save_ckpt=save_ckpt)

    def close(self):
        if self.model is not None:
            self.model.close()
            self.model = None


class SeisForward(torch.autograd.Function):
    """seis = F(vp[, vs, rho]); backward = the library's adjoint sweep."""

    @staticmethod
    def forward(ctx, prop: Propagator, vp, vs=None, rho=None):
        seis = prop.forward(vp, vs, rho, save_ckpt=True)
        ctx.prop = prop
        ctx.generation = prop.generation
        ctx.elastic = prop.elastic
        return seis

    @staticmethod
    def backward(ctx, gseis):
        prop = ctx.prop
        if prop.generation != ctx.generation:
            raise RuntimeError("the propagator ran another forward before this backward; "
                               "its checkpoints belong to that call")
        g = prop.model.gradient(prop.shots, gseis.contiguous())
        if ctx.elastic:
            return (None,) + tuple(g)
        return None, g, None, None


def seis_forward(prop, vp, vs=None, rho=None):
    return SeisForward.apply(prop, vp, vs, rho)


# --------------------------------------------------------------- batched GD
@dataclasses.dataclass
class GDConfig:
    iters: int = 50
    alpha0: float = 50.0      # m/s, maximum model change of the first trial step
    shrink: float = 0.5       # backtracking factor
    max_backtracks: int = 4
    grow: float = 1.25        # step growth after a first-try success
    vmin: float = 1000.0
    vmax: float = 5000.0


@dataclasses.dataclass
class GDResult:
    models: torch.Tensor              # [B, nz, nx]
    J: np.ndarray                     # [iters + 1, B] misfit per iteration
    times: np.ndarray                 # [iters + 1] wall seconds since start (after device sync)
    accepted: np.ndarray              # [iters, B] step accepted
    guarded: np.ndarray = None        # [iters, B] a guarded (e.g. learned) direction was offered
    rejected: np.ndarray = None       # [iters, B] ... and replaced by the plain direction


def per_model_misfit(prop, pred, obs, nmodels, keep=False):
    """J_b = 1/2 sum over model b's samples (FP64 on the device), and the
    residual (FP32); keep: into the propagator's residual buffer, which the
    next kept misfit overwrites."""
    if keep:
        if prop.resid is None or prop.resid.shape != pred.shape:
            prop.resid = torch.empty_like(pred)
        resid = prop.resid
    else:
        resid = torch.empty_like(pred)
    J = torch.empty(nmodels, dtype=torch.float64, device=pred.device)
    per = pred.numel() // nmodels
    pv, ov, rv = pred.reshape(nmodels, per), obs.reshape(nmodels, per), resid.reshape(nmodels, per)
    for b in range(nmodels):
        S._check(S.lib().misfit(prop.model.handle, S._ptr(pv[b]), S._ptr(ov[b]), per, S._ptr(J[b:b + 1]),
                                S._ptr(rv[b]), S._stream()))
    return J, resid


def save_gd_state(path, it, m, alpha, Js, times, acc, offered, rej, direction=None):
    """The inversion state after iteration `it` (numpy arrays only, written
    atomically): models, step lengths, the misfit history and flags, and the
    direction object's state if it has one."""
    st = {"it": np.array(it), "models": m.detach().cpu().numpy(), "alpha": alpha.numpy(),
          "J": np.array(Js), "times": np.array(times), "accepted": np.array(acc),
          "guarded": np.array(offered), "rejected": np.array(rej)}
    if direction is not None and hasattr(direction, "state"):
        st.update({"dir_" + k: v for k, v in direction.state().items()})
    tmp = path + ".tmp.npz"
    np.savez(tmp, **st)
    os.replace(tmp, path)


def load_gd_state(path):
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def batched_gd(prop: Propagator, m0: torch.Tensor, obs: torch.Tensor, cfg: GDConfig = GDConfig(),
               direction=None, target=None, log=None, state_path=None, resume=False,
               jsonl=None) -> GDResult:
    """Gradient descent on B models at once.  Per iteration and model: fwd +
    misfit + adjoint gradient g_b; direction p_b = -g_b, or
    direction(g, models, it) if given (which returns p and a mask of models
    whose direction must pass the safeguard); normalised trial step
    m + alpha p / max|p| with backtracking until J decreases.  A safeguarded
    direction that is not a descent direction (<p, g> >= 0) or that fails to
    decrease J on its first trial is replaced by -g for that model and
    iteration; a direction object with a ``report(it, rejected)`` method is
    told which models that happened to.  Stops early when every model
    reaches J/J0 <= target.

    state_path: the state is saved there after every iteration; with
    resume=True and an existing file the run continues from it (the models
    are restored bit for bit, the misfit and residual recomputed from them,
    so the continued trajectory equals an uninterrupted one).  jsonl: one
    JSON line per iteration appended there (relative misfit, accepted and
    rejected steps, step lengths, seconds)."""
    B = prop.d.nmodels
    m = m0.clone().contiguous()
    alpha = torch.full((B,), cfg.alpha0, dtype=torch.float64)
    Js, times, acc, offered, rej = [], [], [], [], []
    start, t_prev = 0, 0.0
    if resume and state_path and os.path.exists(state_path):
        st = load_gd_state(state_path)
        m = torch.as_tensor(st["models"], device=m0.device).contiguous()
        alpha = torch.as_tensor(st["alpha"], dtype=torch.float64)
        Js = list(st["J"])
        times = list(st["times"])
        acc, offered, rej = list(st["accepted"]), list(st["guarded"]), list(st["rejected"])
        start, t_prev = int(st["it"]) + 1, float(st["times"][-1])
        if direction is not None and hasattr(direction, "load_state"):
            direction.load_state({k[4:]: v for k, v in st.items() if k.startswith("dir_")})
    torch.cuda.synchronize()
    t0 = time.perf_counter() - t_prev
    pred = prop.forward(m, save_ckpt=True, keep=True)
    J, r = per_model_misfit(prop, pred, obs, B, keep=True)
    if start == 0:
        Js.append(J.cpu().numpy().copy())
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    J0 = Js[0]
    for it in range(start, cfg.iters):
        g = prop.model.gradient(prop.shots, r)
        gflat = g.reshape(B, -1)
        p = -g
        guarded = torch.zeros(B, dtype=torch.bool)
        if direction is not None:
            p, guarded = direction(g, m, it)
            guarded = guarded.clone()
        offered.append(guarded.numpy().copy())
        pflat = p.reshape(B, -1)
        # a guarded direction must be a descent direction
        descent = (pflat.double() * gflat.double()).sum(1).cpu() < 0
        fallback = guarded & ~descent
        rejected = fallback.numpy().copy()
        guarded = guarded & descent
        if fallback.any():
            pflat[fallback.to(pflat.device)] = -gflat[fallback.to(pflat.device)]
        scale = pflat.abs().amax(1).clamp_min(1e-30)
        Jc = J.cpu().numpy()
        best = Jc.copy()
        done = np.zeros(B, dtype=bool)
        newm = m.clone()
        a = alpha.clone()
        first = np.ones(B, dtype=bool)
        for bt in range(cfg.max_backtracks + 1):
            trial = (m.reshape(B, -1) + (a.to(m.device, torch.float32) / scale)[:, None] * pflat).reshape(m.shape)
            trial = trial.clamp(cfg.vmin, cfg.vmax)
            tp = prop.forward(trial, save_ckpt=False, keep=True)
            Jt, _ = per_model_misfit(prop, tp, obs, B, keep=True)
            Jt = Jt.cpu().numpy()
            ok = (~done) & (Jt < Jc)
            if ok.any():
                idx = torch.as_tensor(np.nonzero(ok)[0], device=m.device)
                newm[idx] = trial[idx]
                best[ok] = Jt[ok]
            for b in np.nonzero(ok)[0]:
                alpha[b] = a[b] * (cfg.grow if first[b] else 1.0)
            done |= ok
            # guarded directions that fail their first trial fall back to -g,
            # which then gets a first trial of its own at the same step
            retry = np.zeros(B, dtype=bool)
            if bt == 0:
                retry = guarded.numpy() & ~ok
                if retry.any():
                    rejected |= retry
                    bi = torch.as_tensor(np.nonzero(retry)[0], device=m.device)
                    pflat[bi] = -gflat[bi]
                    scale[bi] = pflat[bi].abs().amax(1).clamp_min(1e-30)
                    guarded[torch.as_tensor(retry)] = False
            if done.all():
                break
            shrink = ~done & ~retry
            a[torch.as_tensor(shrink)] *= cfg.shrink
            first[shrink] = False
        for b in np.nonzero(~done)[0]:
            alpha[b] = a[b]
        acc.append(done.copy())
        rej.append(rejected)
        if direction is not None and hasattr(direction, "report"):
            direction.report(it, rejected)
        m = newm
        pred = prop.forward(m, save_ckpt=True, keep=True)
        J, r = per_model_misfit(prop, pred, obs, B, keep=True)
        Js.append(J.cpu().numpy().copy())
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        if log:
            log(it, Js[-1] / J0, done)
        if jsonl:
            with open(jsonl, "a") as f:
                f.write(json.dumps({"it": it, "seconds": times[-1], "J": Js[-1].tolist(),
                                    "J_rel": (Js[-1] / J0).tolist(), "accepted": done.tolist(),
                                    "rejected": rejected.tolist(), "alpha": alpha.tolist()}) + "\n")
        if state_path:
            save_gd_state(state_path, it, m, alpha, Js, times, acc, offered, rej, direction)
        if target is not None and np.all(Js[-1] / J0 <= target):
            break
    return GDResult(models=m, J=np.array(Js), times=np.array(times), accepted=np.array(acc),
                    guarded=np.array(offered), rejected=np.array(rej))


# --------------------------------------------------------------- batched L-BFGS
@dataclasses.dataclass
class LBFGSConfig:
    iters: int = 50
    mem: int = 8
    alpha0: float = 50.0      # m/s, maximum model change of the first steepest-descent step
    shrink: float = 0.5
    grow: float = 1.25        # steepest-descent step growth after a first-try success
    max_backtracks: int = 6
    vmin: float = 1000.0
    vmax: float = 5000.0


def batched_lbfgs(prop: Propagator, m0: torch.Tensor, obs: torch.Tensor, cfg: LBFGSConfig = LBFGSConfig(),
                  target=None, log=None) -> GDResult:
    """L-BFGS on B models at once, each with its own history (the paper's
    optimizer family; bounds by clipping).  Per iteration and model: the
    two-loop direction p = -H g (library kernel; -g with no history), the
    natural step m + p, halved until the misfit decreases.  Without history
    (the first step, and after a reset) the step is the normalised
    steepest-descent step alpha p / max|p| whose alpha persists across
    iterations as in plain descent (shrunk on failure, grown after a
    first-try success).  A model whose search fails, or whose direction is
    not a descent direction, drops its history.  Pairs (s, y) with y.s <= 0
    are not stored."""
    B = prop.d.nmodels
    dev = m0.device
    n = m0[0].numel()
    S_ = torch.zeros((cfg.mem, B, n), dtype=torch.float32, device=dev)
    Y_ = torch.zeros_like(S_)
    ysyy = torch.zeros((cfg.mem, B, 2), dtype=torch.float64, device=dev)
    count = np.zeros(B, dtype=np.int32)
    newest = np.full(B, -1, dtype=np.int32)
    alpha_sd = np.full(B, cfg.alpha0)
    m = m0.clone().contiguous()
    Js, times, acc = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred = prop.forward(m, save_ckpt=True, keep=True)
    J, r = per_model_misfit(prop, pred, obs, B, keep=True)
    J0 = J.cpu().numpy().copy()
    Js.append(J0.copy())
    torch.cuda.synchronize()
    times.append(time.perf_counter() - t0)
    g = prop.model.gradient(prop.shots, r).contiguous()
    p = torch.empty_like(g)
    lib = S.lib()
    for it in range(cfg.iters):
        hist = torch.as_tensor(np.stack([count, newest], 1).astype(np.int32), device=dev)
        S._check(lib.lbfgs_direction(B, n, cfg.mem, S._ptr(hist), S._ptr(S_), S._ptr(Y_), S._ptr(ysyy),
                                     S._ptr(g), S._ptr(p), S._stream()))
        pf, gf = p.reshape(B, -1), g.reshape(B, -1)
        descent = (pf.double() * gf.double()).sum(1).cpu().numpy() < 0
        for b in np.nonzero(~descent)[0]:
            pf[b] = -gf[b]
            count[b], newest[b] = 0, -1
        # natural step with history; without, the normalised steepest-descent
        # step whose length persists from iteration to iteration as in plain GD
        sd = count == 0
        scale = torch.where(torch.as_tensor(sd, device=dev), torch.as_tensor(alpha_sd, dtype=torch.float32, device=dev)
                            / pf.abs().amax(1).clamp_min(1e-30), torch.ones(B, device=dev))
        Jc = J.cpu().numpy()
        done = np.zeros(B, dtype=bool)
        newm = m.clone()
        a = torch.ones(B, device=dev)
        for bt in range(cfg.max_backtracks + 1):
            trial = (m.reshape(B, -1) + (a * scale)[:, None] * pf).reshape(m.shape).clamp(cfg.vmin, cfg.vmax)
            Jt, _ = per_model_misfit(prop, prop.forward(trial, save_ckpt=False, keep=True), obs, B, keep=True)
            Jt = Jt.cpu().numpy()
            ok = (~done) & (Jt < Jc)
            if ok.any():
                idx = torch.as_tensor(np.nonzero(ok)[0], device=dev)
                newm[idx] = trial[idx]
            done |= ok
            if done.all():
                break
            a[torch.as_tensor(~done, device=dev)] *= cfg.shrink
        ah = a.cpu().numpy().astype(np.float64)
        for b in np.nonzero(sd)[0]:
            if done[b]:
                alpha_sd[b] *= ah[b] * (cfg.grow if ah[b] == 1.0 else 1.0)
            else:
                alpha_sd[b] *= ah[b] * cfg.shrink
        for b in np.nonzero(~done)[0]:
            count[b], newest[b] = 0, -1          # failed search: restart from steepest descent
        acc.append(done.copy())
        m_old, g_old = m, g
        m = newm
        pred = prop.forward(m, save_ckpt=True, keep=True)
        J, r = per_model_misfit(prop, pred, obs, B, keep=True)
        g = prop.model.gradient(prop.shots, r).contiguous()
        # store (s, y) of the models that moved
        slot = np.where(done, (newest + 1) % cfg.mem, -1).astype(np.int32)
        slot_d = torch.as_tensor(slot, device=dev)
        S._check(lib.lbfgs_push(B, n, cfg.mem, S._ptr(slot_d), S._ptr(m), S._ptr(m_old), S._ptr(g), S._ptr(g_old),
                                S._ptr(S_), S._ptr(Y_), S._ptr(ysyy), S._stream()))
        ys = ysyy.cpu().numpy()
        for b in np.nonzero(done)[0]:
            if ys[slot[b], b, 0] > 0:
                newest[b] = slot[b]
                count[b] = min(count[b] + 1, cfg.mem)
            elif count[b] == cfg.mem:
                count[b] = cfg.mem - 1           # the rejected pair overwrote the oldest one
        Js.append(J.cpu().numpy().copy())
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        if log:
            log(it, Js[-1] / J0, done)
        if target is not None and np.all(Js[-1] / J0 <= target):
            break
    return GDResult(models=m, J=np.array(Js), times=np.array(times), accepted=np.array(acc))
