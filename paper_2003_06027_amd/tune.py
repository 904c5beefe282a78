"""Autotuner of the launch strategy for one workload (grid, shot batch,
physics), with a JSON cache.

Candidates (none changes what is computed; see set_tuning in the C ABI):
* 2-D acoustic: 1 or 2 steps per launch on the blocked tiles (results are
  bitwise identical, traffic and launch count differ), each eager or with
  the library's segment graphs (one HIP graph per checkpoint segment of the
  forward and of the adjoint sweep, captured once and replayed);
* 3-D acoustic: the z-chunk lengths of the forward tile passes (16-64
  planes), of the adjoint tile passes (32-64) and of the layer work items
  (16-64), searched one at a time from the defaults (each moves different
  kernels);
* 2-D elastic: shots of one model per thread (4, 2 or 1, those dividing the
  shots per model) and cell blocks of 32 x 8 or 64 x 4;
* every physics: eager launches or graph replay.

Each candidate is timed on a shortened run of the same grid and shots (a
few checkpoint segments; the cost per step does not depend on nt) and the
fastest is cached (graph replay only if it beats the best eager candidate
by more than 2%) under a key of the workload and the device, in
``$SEISGRAD_TUNE_CACHE`` or ``~/.cache/seisgrad/tune.json``.  Tuning runs
outside any timed region.
"""
from __future__ import annotations

import dataclasses
import hashlib
import json
import math
import os
import time

import torch

from . import seisgrad as S


GRAPH_MARGIN = 0.02


@dataclasses.dataclass(frozen=True)
class Strategy:
    time_blocking: int = 2     # 2-D acoustic
    graphs: bool = False
    chunk_fwd3: int = 32       # 3-D acoustic
    chunk_adj3: int = 64
    chunk_layer3: int = 32
    shot_group: int = 0        # elastic (0: the library's rule)
    block_x: int = 32

    def apply(self, m):
        """Set the strategy's launch settings on model m (those its physics has)."""
        d = m.d
        m.set_tuning(S.SG_TUNE_GRAPHS, int(self.graphs))
        if d.physics == S.SG_ACOUSTIC and d.ndim == 2:
            m.set_tuning(S.SG_TUNE_TIME_BLOCKING, self.time_blocking)
        elif d.physics == S.SG_ACOUSTIC and d.ndim == 3:
            m.set_tuning(S.SG_TUNE_CHUNK_FWD3, self.chunk_fwd3)
            m.set_tuning(S.SG_TUNE_CHUNK_ADJ3, self.chunk_adj3)
            m.set_tuning(S.SG_TUNE_CHUNK_LAYER3, self.chunk_layer3)
        elif d.physics == S.SG_ELASTIC:
            m.set_tuning(S.SG_TUNE_SHOT_GROUP, self.shot_group)
            m.set_tuning(S.SG_TUNE_BLOCK_X, self.block_x)

    def label(self):
        return ",".join(f"{k}={v}" for k, v in dataclasses.asdict(self).items()
                        if v != getattr(Strategy, k))  or "default"


def cache_path():
    return os.environ.get("SEISGRAD_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "seisgrad", "tune.json"))


def workload_key(d, nshots, nrec):
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    lib = S.LIB_PATH
    build = os.path.getmtime(lib) if os.path.exists(lib) else 0
    fields = (d.ndim, d.physics, d.nx, d.ny, d.nz, d.npml, d.nmodels, nshots, nrec, dev, build)
    return hashlib.sha1(repr(fields).encode()).hexdigest()[:16]


def candidates(d, nshots=1):
    """The first round of candidates; 3-D continues with coordinate search."""
    if d.ndim == 2 and d.physics == S.SG_ACOUSTIC:
        return [Strategy(time_blocking=tb, graphs=g) for tb in (2, 1) for g in (False, True)]
    if d.physics == S.SG_ELASTIC:
        spm = nshots // d.nmodels
        groups = [gs for gs in (4, 2, 1) if spm % gs == 0]
        return [Strategy(shot_group=gs, block_x=bx) for gs in groups for bx in (32, 64)] + [Strategy(graphs=True)]
    if d.ndim == 3:
        return [Strategy(chunk_fwd3=c) for c in (16, 32, 48, 64)]
    return [Strategy(), Strategy(graphs=True)]


# 3-D coordinate search after the forward chunk: the adjoint chunk, then the layer items
CHUNKS_ADJ3 = (32, 48, 64)
CHUNKS_LAYER3 = (16, 32, 64)


class Runner:
    """One checkpointed forward + misfit + adjoint of a shot batch with fixed
    buffers (so that the library's segment graphs, when the strategy has
    them, are captured by the first step and replayed by the next)."""

    def __init__(self, d, shots, vp, obs, strategy: Strategy, ckpt=0, vs=None, rho=None):
        self.shots = shots
        self.m = S.Model(d, vp, shots.nshots, shots.nrec, ckpt, vs=vs, rho=rho)
        strategy.apply(self.m)
        self.obs = obs
        self.seis = torch.empty_like(obs)
        self.resid = torch.empty_like(obs)
        self.out = None

    def _eager(self):
        self.m.forward(self.shots, seis=self.seis, save_ckpt=True)
        self.J, _ = self.m.misfit(self.seis, self.obs, resid=self.resid)
        if self.out is None:
            self.out = self.m.gradient(self.shots, self.resid)
        else:
            outs = self.out if isinstance(self.out, tuple) else (self.out,)
            g = self.m.gradient(self.shots, self.resid, g_vp=outs[0],
                                g_vs=outs[1] if len(outs) > 1 else None, g_rho=outs[2] if len(outs) > 2 else None)
            self.out = g
        return self.out

    def step(self):
        return self._eager()

    def close(self):
        self.m.close()


def measure(d, shots, vp, obs, strategy, reps=3, **kw):
    """Median seconds of one fwd + misfit + adjoint of the batch."""
    r = Runner(d, shots, vp, obs, strategy, **kw)
    r.step()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        r.step()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    r.close()
    ts.sort()
    return ts[len(ts) // 2]


def tune(d, shots, vp, vs=None, rho=None, ckpt=0, segments=4, cache=None, log=None, force=False):
    """Best Strategy for this workload (cached).  Times every candidate on a
    run of `segments` checkpoint segments of the same grid and shots."""
    cache = cache or cache_path()
    key = workload_key(d, shots.nshots, shots.nrec)
    table = {}
    if os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
    if key in table and not force:
        return Strategy(**table[key]["strategy"])
    K = ckpt if ckpt > 0 else int(math.ceil(math.sqrt(d.nt)))
    nt = min(d.nt, segments * K)
    dt = S.desc(ndim=d.ndim, physics=d.physics, nx=d.nx, ny=d.ny, nz=d.nz, npml=d.npml, nt=nt,
                nmodels=d.nmodels, dx=d.dx, dt=d.dt, pml_R=d.pml_R, pml_vmax=d.pml_vmax, f0_pml=d.f0_pml)
    wav = shots.wavelet[:, :nt].contiguous()
    sh = S.Shots(shots.src, shots.rec, wav, shots.mt)
    ref = S.Model(dt, vp, sh.nshots, sh.nrec, K, vs=vs, rho=rho)
    obs = (ref.forward(sh, save_ckpt=False) * 0.9).contiguous()   # any data of the right shape
    ref.close()
    times = {}

    def run(c):
        if c not in times:
            times[c] = measure(dt, sh, vp, obs, c, ckpt=K, vs=vs, rho=rho)
            if log:
                log(f"tune {key}: {c.label()} {times[c] * 1e3:.2f} ms for {nt} steps")
        return times[c]

    for c in candidates(d, shots.nshots):
        try:
            run(c)
        except S.SeisError as e:            # a setting this workload cannot take
            if log:
                log(f"tune {key}: {c.label()} skipped ({e})")
    if d.ndim == 3 and d.physics == S.SG_ACOUSTIC:
        best = min(times, key=times.get)
        for field, values in (("chunk_adj3", CHUNKS_ADJ3), ("chunk_layer3", CHUNKS_LAYER3)):
            for v in values:
                run(dataclasses.replace(best, **{field: v}))
            best = min(times, key=times.get)
        run(dataclasses.replace(best, graphs=True))
    # graph replay only where it beats the best eager candidate by more than 2%
    eager = min((c for c in times if not c.graphs), key=times.get)
    best = min(times, key=times.get)
    if best.graphs and times[best] > (1.0 - GRAPH_MARGIN) * times[eager]:
        best = eager
    table[key] = {"strategy": dataclasses.asdict(best), "nt_measured": nt,
                  "ms": {c.label(): round(t * 1e3, 3) for c, t in times.items()}}
    os.makedirs(os.path.dirname(cache), exist_ok=True)
    with open(cache + ".tmp", "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(cache + ".tmp", cache)
    return best
