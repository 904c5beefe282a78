"""Throughput benchmark of the fwd+adjoint hot path on one MI355X.

One step = one pass of the whole path over the batch: forward sweep of all
shots with wavefield checkpoints, FP64 misfit and residual, then the adjoint
sweep (checkpoint restore, segment recompute, adjoint steps) and the gradient
finalisation -- all in the library's HIP kernels, inputs resident in HBM.

Workload (default): 2-D acoustic, 8th-order Laplacian, 1000 x 500 cells
(dx = 10 m) + 32-cell absorbing layer, dt = 0.8 ms, 4000 steps, 64 shots of
an 8 Hz Ricker in one launch, 1000 receivers per shot, checkpoints every
ceil(sqrt(4000)) = 64 steps; velocity 1500-4500 m/s from 12 seeded dipping
layers + 20 Gaussian anomalies (a stand-in for the paper's Marmousi-class
FWI model), initial model its 10-cell Gaussian blur.

Second leg (the metric's "time-to-misfit w/ vs w/o CNN"): the learned
preconditioner experiment -- training data from 200 batched plain
inversions of random three-layer 101 x 101 models, CNN training with the
library's BF16 matrix-core kernels, then plain and preconditioned descent on
20 unseen models; reported under "time_to_misfit" (skip with --no-ttm).

Other workloads (--workload c3 | c4, --physics divergence) print their own
line with the same keys: the 2-D elastic (800 x 400, 16 shots) and 3-D
acoustic (400^3) sweeps, and the divergence-form acoustic kernels on the C2
workload.  The default run is the one above.

Prints ONE JSON line (rank 0, N = 1).
"""
import argparse
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gcell-updates/s fwd+adjoint (% HBM roofline); FWI time-to-misfit w/ vs w/o CNN"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bytes_per_cell_step(pml_fraction):
    """Algorithmic FP32 bytes per padded cell and step of each phase.
    forward: read u^k, u^{k-1}, chat, write u^{k+1} = 16 B; layer cells also
    read and write phi_x, phi_z (+16 B).  recompute: forward + the w~^k
    snapshot write (+4 B).  adjoint: read s^{k+2}, s^{k+3}, chat, w~^k,
    read+write the gradient, write s^{k+1} = 28 B; layer cells read and write
    b_x, b_z (+16 B)."""
    f = 16.0 + 16.0 * pml_fraction
    return {"forward": f, "recompute": f + 4.0, "adjoint": 28.0 + 16.0 * pml_fraction}


def bytes_per_cell_step_div(pml_fraction):
    """The same for the divergence form (staggered grid, CPML).  forward:
    read u^k, u^{k-1}, chat, write u^{k+1} = 16 B; layer cells read and write
    psi'x, psi'z, xi'x, xi'z (+32 B).  recompute: + the S'x, S'z snapshot
    writes (+8 B).  adjoint: read lambda^{k+1}, lambda^{k+2}, chat, S'x, S'z,
    read+write dJ/dchat, write lambda^k = 32 B; layer cells read and write
    Yx, Yz, Zx, Zz (+32 B)."""
    f = 16.0 + 32.0 * pml_fraction
    return {"forward": f, "recompute": f + 8.0, "adjoint": 32.0 + 32.0 * pml_fraction}


TRAFFIC_FILES = {   # workload -> committed counter summary, the kernel sources it was taken with
    "c2": ("ac2_c2_hbm_traffic.txt", ("ac2.hip", "sg_internal.h")),
    "div": ("ad2_c2_hbm_traffic.txt", ("ad2.hip", "ad2_internal.h", "sg_internal.h")),
    "c3": ("el2_c3_hbm_traffic.txt", ("el2.hip", "el2_internal.h", "sg_internal.h")),
    "c4": ("ac3_c4_hbm_traffic.txt", ("ac3.hip", "ac3_internal.h", "sg_internal.h")),
}


def measured_traffic(phase, workload="c2"):
    """HBM bytes per step of `phase` from the committed FETCH_SIZE/WRITE_SIZE
    summary (counters scaled by a plain copy of known size), or None when the
    kernels' source has changed since the counters were taken."""
    import hashlib
    name, files = TRAFFIC_FILES[workload]
    path = os.path.join(ROOT, "profiles", name)
    src = os.path.join(ROOT, "paper_2003_06027_amd", "csrc")
    try:
        text = open(path).read()
        h = hashlib.sha256()
        for f in files:
            h.update(open(os.path.join(src, f), "rb").read())
    except OSError:
        return None
    m = re.search(r"^kernel_source_sha256 (\w+)", text, re.M)
    if not m or m.group(1) != h.hexdigest():
        return None
    m = re.search(rf"^step_{phase} (\d+) bytes", text, re.M)
    return int(m.group(1)) if m else None


def el2_group(shots_per_model):
    """Shots of one model that the elastic passes take together (the
    library's rule): 4 when the model's shots divide by 4, else 2, else 1."""
    return 4 if shots_per_model % 4 == 0 else 2 if shots_per_model % 2 == 0 else 1


def bytes_per_cell_step_el2(pml_fraction, group=1):
    """2-D elastic, per shot and padded cell.  forward: read vx, vz, sxx, szz,
    sxz and write them = 40 B, plus the five model fields (lam, mu, muxz, bx,
    bz; 20 B) that a group of `group` shots reads once; layer cells read and
    write the eight CPML memory variables (+64 B).  recompute: + five
    snapshot fields (+20 B).  adjoint: read the five adjoint fields and the
    five snapshots, write five adjoint fields = 60 B, plus the model fields
    (20 B) and the five gradient accumulators read and written (40 B), once
    per group; +64 B on layer cells."""
    per_group = 20.0 / group
    return {"forward": 40.0 + per_group + 64.0 * pml_fraction,
            "recompute": 60.0 + per_group + 64.0 * pml_fraction,
            "adjoint": 60.0 + (20.0 + 40.0) / group + 64.0 * pml_fraction}


def bytes_per_cell_step_ac3(pml_fraction):
    """3-D acoustic: as the 2-D form, with phi_x, phi_y, phi_z and psi on
    layer cells (+32 B forward and adjoint)."""
    f = 16.0 + 32.0 * pml_fraction
    return {"forward": f, "recompute": f + 4.0, "adjoint": 28.0 + 32.0 * pml_fraction}


def copy_bandwidth(torch):
    """Best of five 1 GiB device-to-device copies (read + write bytes per
    second, GB/s), timed with HIP events on the current stream."""
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.ones_like(a)
    best = 0.0
    for _ in range(6):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        a.copy_(b)
        e1.record()
        torch.cuda.synchronize()
        best = max(best, 2.0 * a.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del a, b
    return best


def omp_threads(n):
    """Thread count of the oracle's OpenMP loops (the process's libgomp)."""
    import ctypes
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
    except OSError:
        pass


def host_cpu():
    """The host CPU as lscpu reports it, and the CPUs this process may use."""
    import subprocess
    info = {}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)",
                             "CPU max MHz"):
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    info["usable_cpus"] = len(os.sched_getaffinity(0))
    return info


def cpu_baseline_el2(cfg, m0, src, mt, rec, nshots, nt):
    from oracle import pyoracle as O
    g = O.grid(ndim=2, nx=cfg.nx, nz=cfg.nz, npml=cfg.npml, nt=nt, dx=cfg.dx, dt=cfg.dt,
               pml_R=cfg.pml_R, pml_vmax=4000.0, f0_pml=cfg.f0_pml)
    wav = np.stack([O.ricker(cfg.f0, cfg.ricker_t0, cfg.dt, nt)] * nshots)
    d = np.random.default_rng(0).standard_normal((nshots, 2, nt, rec.shape[1]))
    t0 = time.perf_counter()
    O.el2_gradient(g, m0[0], m0[1], m0[2], src[:nshots], mt[:nshots], wav, rec[:nshots], d,
                   ckpt=int(math.ceil(math.sqrt(nt))))
    t = time.perf_counter() - t0
    return 2.0 * cfg.padded_cells * nshots * nt / t / 1e9, t


def cpu_baseline_ac3(cfg, c0, src, rec, nt):
    from oracle import pyoracle as O
    g = O.grid(ndim=3, nx=cfg.nx, ny=cfg.ny, nz=cfg.nz, npml=cfg.npml, nt=nt, dx=cfg.dx, dt=cfg.dt,
               pml_R=cfg.pml_R, pml_vmax=4000.0)
    wav = O.ricker(cfg.f0, cfg.ricker_t0, cfg.dt, nt)[None]
    d = np.random.default_rng(0).standard_normal((1, nt, rec.shape[1]))
    t0 = time.perf_counter()
    O.ac3_gradient(g, c0, src, wav, rec, d, ckpt=int(math.ceil(math.sqrt(nt))))
    t = time.perf_counter() - t0
    return 2.0 * cfg.padded_cells * nt / t / 1e9, t


def cpu_baseline(cfg, c0, src, rec, nshots, nt, divergence=False):
    from oracle import pyoracle as O
    g = O.grid(ndim=2, nx=cfg.nx, nz=cfg.nz, npml=cfg.npml, nt=nt, dx=cfg.dx, dt=cfg.dt,
               pml_R=cfg.pml_R, pml_vmax=4500.0, f0_pml=cfg.f0)
    wav = np.stack([O.ricker(cfg.f0, cfg.ricker_t0, cfg.dt, nt)] * nshots)
    d = np.random.default_rng(0).standard_normal((nshots, nt, rec.shape[1]))
    t0 = time.perf_counter()
    grad = O.ad2_gradient if divergence else O.ac2_gradient
    grad(g, c0, src[:nshots], wav, rec[:nshots], d, ckpt=int(math.ceil(math.sqrt(nt))))
    t = time.perf_counter() - t0
    cells = cfg.padded_cells
    return 2.0 * cells * nshots * nt / t / 1e9, t


def measure(a, S, synth, torch):
    """Time K steps (fwd with checkpoints + misfit + adjoint) of workload
    a.workload; returns the JSON record and what the CPU baseline needs."""
    wl = a.workload
    cfg = {"c2": synth.C2, "c3": synth.C3, "c4": synth.C4}[wl]
    nt = a.nt or cfg.nt
    ckpt = int(math.ceil(math.sqrt(nt)))
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    div = a.physics == "divergence"
    if div and wl != "c2":
        log("--physics divergence applies to the c2 workload")
        sys.exit(2)
    if div or wl != "c2":
        a.no_ttm = True                    # the learned-preconditioner leg runs the headline form
    mt_ = None
    if wl == "c2":
        true_m = [synth.dipping_layers_anomalies(2003, cfg.nx, cfg.nz, cfg.dx)]
        src, rec = synth.c2_geometry(cfg.nshots, cfg.nx)
        vmax = 4500.0
        d = S.desc(ndim=2, physics=S.SG_ACOUSTIC_DIV if div else S.SG_ACOUSTIC, nx=cfg.nx, nz=cfg.nz,
                   npml=cfg.npml, nt=nt, dx=cfg.dx, dt=cfg.dt, pml_R=cfg.pml_R, pml_vmax=vmax, f0_pml=cfg.f0)
    elif wl == "c3":
        true_m = list(synth.elastic_c3(6027, cfg.nx, cfg.nz))
        src, mt_, rec = synth.c3_geometry(6027, cfg.nx)
        vmax = 4000.0
        d = S.desc(ndim=2, physics=S.SG_ELASTIC, nx=cfg.nx, nz=cfg.nz, npml=cfg.npml, nt=nt, dx=cfg.dx,
                   dt=cfg.dt, pml_R=cfg.pml_R, pml_vmax=vmax, f0_pml=cfg.f0_pml)
    else:
        true_m = [synth.smooth_3d(4, cfg.nx)]
        src, rec = synth.c4_geometry(cfg.nx)
        vmax = 4000.0
        d = S.desc(ndim=3, nx=cfg.nx, ny=cfg.ny, nz=cfg.nz, npml=cfg.npml, nt=nt, dx=cfg.dx, dt=cfg.dt,
                   pml_R=cfg.pml_R, pml_vmax=vmax)
    init_m = [synth.smooth(m, 10.0) for m in true_m]
    c0 = init_m[0]
    ns, nrec = src.shape[0], rec.shape[1]
    wav = S.ricker(cfg.f0, cfg.ricker_t0, cfg.dt, nt)
    wav = wav[None].repeat(ns, 1).contiguous()
    sh = S.Shots(src, rec, wav, mt=mt_)
    log(f"setup: {cfg.name} nt={nt} ckpt={ckpt} workspace={S.workspace_bytes(d, ns, nrec, ckpt) / 1e9:.1f} GB")

    def model(ms, **kw):
        extra = {} if len(ms) == 1 else {"vs": dev(ms[1]), "rho": dev(ms[2])}
        return S.Model(d, dev(ms[0]), ns, nrec, ckpt, **extra, **kw)

    mtrue = model(true_m)
    obs = mtrue.forward(sh, save_ckpt=False)
    torch.cuda.synchronize()
    mtrue.close()
    del mtrue
    # launch strategy from the autotuner (timed on a few checkpoint segments
    # of this grid and shot batch, cached, outside the timed region)
    from paper_2003_06027_amd import tune
    if a.time_blocking is not None:
        strategy = tune.Strategy(time_blocking=a.time_blocking)
    else:
        extra = {} if len(init_m) == 1 else {"vs": dev(init_m[1]), "rho": dev(init_m[2])}
        strategy = tune.tune(d, sh, dev(c0), ckpt=ckpt, log=log, segments=2 if wl == "c4" else 4, **extra)
        torch.cuda.empty_cache()
    # the timed run records per-phase HIP events, which need eager launches
    strategy = tune.dataclasses.replace(strategy, graphs=False)
    # workspace beyond the minimum keeps the adjoint snapshots of the last
    # checkpoint segments (their recomputation is skipped); leave a margin
    # for the seismogram and residual buffers
    nseg = -(-nt // ckpt)
    if a.store_segments is None:
        free = torch.cuda.mem_get_info()[0]
        spare = free - S.workspace_bytes(d, ns, nrec, ckpt) - 16 * (1 << 30)
        nstore = int(max(0, min(nseg, spare // S.snapshot_segment_bytes(d, ns, ckpt))))
    else:
        nstore = min(a.store_segments, nseg)
    m = model(init_m, store_segments=nstore)
    log(f"workspace {m.ws.numel() / 1e9:.1f} GB: {nstore} of {nseg} segments keep their snapshots")
    strategy.apply(m)
    seis = torch.empty_like(obs)
    resid = torch.empty_like(obs)
    J = torch.empty(1, dtype=torch.float64, device="cuda")
    gshape = (1, cfg.nz, cfg.nx) if cfg.ndim == 2 else (1, cfg.nz, cfg.ny, cfg.nx)
    g = torch.empty(gshape, dtype=torch.float32, device="cuda")
    gx = [torch.empty_like(g), torch.empty_like(g)] if wl == "c3" else [None, None]

    def step():
        m.forward(sh, seis=seis, save_ckpt=True)
        S._check(S.lib().misfit(m.handle, S._ptr(seis), S._ptr(obs), seis.numel(), S._ptr(J),
                                S._ptr(resid), S._stream()))
        m.gradient(sh, resid, g_vp=g, g_vs=gx[0], g_rho=gx[1])

    for i in range(a.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{a.warmup} done, J = {J.item():.6e}")
    m.set_profiling(True)
    m.phase_times()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        step()
        torch.cuda.synchronize()
        log(f"step {i + 1}/{a.steps} done at {time.perf_counter() - t0:.2f} s")
    t1 = time.perf_counter()
    phases = m.phase_times()
    m.set_profiling(False)
    if a.copy_probe:
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.ones_like(x)
        x.copy_(y)
        torch.cuda.synchronize()
        del x, y
    assert np.isfinite(J.item()) and np.isfinite(g.abs().max().item())
    copy_gbs = None if a.copy_probe else copy_bandwidth(torch)

    T = (t1 - t0) / a.steps
    cells = cfg.padded_cells
    updates = 2.0 * cells * ns * nt
    value = updates / T / 1e9
    pml_frac = 1.0 - cfg.nx * cfg.ny * cfg.nz / cells
    if wl == "c3":
        bpc = bytes_per_cell_step_el2(pml_frac, el2_group(ns // d.nmodels))
    else:
        bpc = (bytes_per_cell_step_div if div else bytes_per_cell_step_ac3 if wl == "c4"
               else bytes_per_cell_step)(pml_frac)
    ph = {}
    for name, (ms, steps) in phases.items():
        if steps == 0:
            continue
        per = ms / steps                      # ms per step of this phase
        gbs = cells * ns * bpc[name] / (per * 1e-3) / 1e9
        ph[name] = {"ms_per_step": round(per, 5), "gcell_per_s": round(cells * ns / (per * 1e-3) / 1e9, 2),
                    "alg_bytes_per_cell": round(bpc[name], 3), "gbs": round(gbs, 1),
                    "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
    dom = max(ph, key=lambda k: phases[k][0])
    traffic = measured_traffic(dom, "div" if div else wl)   # HBM bytes per step (all launches)
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gcell-updates/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(T * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (cfg.name if nt == cfg.nt else f"{cfg.name}_nt{nt}") + ("_divergence" if div else ""),
                   "grid_padded": list(cfg.padded),
                   "shots": ns, "nt": nt, "ckpt_every": ckpt, "stored_segments": nstore, "segments": nseg,
                   "launch_settings": strategy.label(),
                   "launch": "eager (per-phase HIP events need eager launches)",
                   "receivers": nrec,
                   "cell_updates_per_step": updates},
        "roofline": {"bound": "hbm",
                     "kernel": (f"ad2 {dom} step (one fused launch)" if div
                                else f"el2 {dom} step (velocity and stress passes)" if wl == "c3"
                                else f"ac3 {dom} step (layer and z-marching passes)" if wl == "c4"
                                else f"ac2 {dom} step (PML + interior launches)"),
                     "achieved": ph[dom]["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ph[dom]["frac_hbm"], "traffic": traffic,
                     "copy_gbs": None if copy_gbs is None else round(copy_gbs, 1),
                     "frac_of_copy": None if copy_gbs is None else round(ph[dom]["gbs"] / copy_gbs, 4)},
        "phases": ph,
    }
    ctx = dict(cfg=cfg, c0=c0, init_m=init_m, src=src, rec=rec, mt=mt_, ns=ns, div=div)
    m.close()
    return out, ctx


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nt", type=int, default=None, help="override time steps (profiling runs only)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-steps", type=int, default=400)
    ap.add_argument("--no-ttm", action="store_true", help="skip the learned-preconditioner time-to-misfit leg")
    ap.add_argument("--no-c4", action="store_true", help="skip the short 3-D record of the default run")
    ap.add_argument("--store-segments", type=int, default=None,
                    help="checkpoint segments whose adjoint snapshots the forward keeps "
                         "(default: as many as fit in free HBM)")
    ap.add_argument("--time-blocking", type=int, default=None, choices=(1, 2),
                    help="time steps per launch on the blocked tiles (results are identical); "
                         "default: the autotuner's choice")
    ap.add_argument("--workload", choices=("c2", "c3", "c4"), default="c2",
                    help="c2: 2-D acoustic 1000x500, 64 shots (default); c3: 2-D elastic 800x400, 16 shots; "
                         "c4: 3-D acoustic 400^3")
    ap.add_argument("--physics", choices=("constant-density", "divergence"), default="constant-density",
                    help="acoustic form: u_tt = c^2 lap(u) (the headline kernels) or u_tt = div(c^2 grad u) "
                         "(staggered grid, CPML; same grid, shots and steps)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the timed steps, run one plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU shot sharding "
              "is a design, not a build target.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2003_06027_amd import seisgrad as S
    from paper_2003_06027_amd import synth

    out, ctx = measure(args, S, synth, torch)
    if args.workload == "c2" and args.physics == "constant-density" and not args.no_c4:
        # a short 3-D record beside the headline: the full 400^3 grid, 200 of
        # its 2000 steps (15-step checkpoints, every segment recomputed, as
        # nearly all of them are at full length), one timed fwd+adjoint step
        # after one warm-up
        torch.cuda.empty_cache()
        sub = argparse.Namespace(**vars(args))
        sub.workload, sub.nt, sub.steps, sub.warmup = "c4", 200, 1, 1
        sub.store_segments, sub.time_blocking, sub.copy_probe, sub.no_ttm = 0, None, False, True
        c4, _ = measure(sub, S, synth, torch)
        out["c4"] = {k: c4[k] for k in ("value", "unit", "ms_per_step", "config", "roofline", "phases")}
        torch.cuda.empty_cache()
    cfg, c0, init_m, src, rec, mt_, ns, div = (ctx[k] for k in ("cfg", "c0", "init_m", "src", "rec", "mt", "ns",
                                                               "div"))
    wl = args.workload
    if not args.no_ttm:
        torch.cuda.empty_cache()
        from paper_2003_06027_amd import ttm
        log("time-to-misfit: data generation, CNN training and evaluation")
        r = ttm.run(ttm.TTMConfig(), log=log)

        def fin(v, nd=3):        # a median over models of which too few reach tau is infinite: null
            return round(float(v), nd) if v is not None and np.isfinite(v) else None
        out["time_to_misfit"] = {
            "metric": "seconds until J/J0 <= tau (median over 20 unseen 3-layer models batched in one launch; "
                      "null: fewer than half of the models reach tau within the iteration cap)",
            "tau": round(r["tau"], 4), "tau_rule": "fixed before the run", "iteration_cap": r["eval_iters"],
            "median_seconds_gd": fin(r["median_seconds_gd"]),
            "median_seconds_cnn": fin(r["median_seconds_cnn"]),
            "speedup": fin(r["median_seconds_gd"] / r["median_seconds_cnn"], 2),
            "median_iters_gd": fin(r["median_iters_gd"], 1), "median_iters_cnn": fin(r["median_iters_cnn"], 1),
            "reached_gd": r["reached_gd"], "reached_cnn": r["reached_cnn"], "models": r["models"],
            "final_rel_misfit_median_gd": round(r["final_rel_misfit_median_gd"], 4),
            "final_rel_misfit_median_cnn": round(r["final_rel_misfit_median_cnn"], 4),
            "median_seconds_lbfgs": fin(r["median_seconds_lbfgs"]),
            "median_iters_lbfgs": fin(r["median_iters_lbfgs"], 1), "reached_lbfgs": r["reached_lbfgs"],
            "final_rel_misfit_median_lbfgs": round(r["final_rel_misfit_median_lbfgs"], 4),
            "cnn_acceptance": round(r["cnn_acceptance"], 3),
            "data_seconds": round(r["data_seconds"], 2), "train_seconds": round(r["train_seconds"], 2),
            "break_even_batches": None if r["break_even_batches"] is None else round(r["break_even_batches"], 1),
            "val_loss_untrained_trained": [round(v, 4) for v in r["val_loss_untrained_trained"]],
        }
    if not args.no_cpu:
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        omp_threads(cores)

        def sample(nshots, nsteps):
            if wl == "c2":
                return cpu_baseline(cfg, c0, src, rec, nshots, nsteps, divergence=div)
            if wl == "c3":
                return cpu_baseline_el2(cfg, init_m, src, mt_, rec, nshots, nsteps)
            return cpu_baseline_ac3(cfg, c0, src, rec, nsteps)

        # all host threads (the oracle runs shots in parallel in 2-D acoustic,
        # rows / planes of every pass in the elastic and 3-D forms)
        ncpu, steps = {"c2": (max(1, min(cores, ns)), args.cpu_steps), "c3": (2, min(args.cpu_steps, 300)),
                       "c4": (1, 2)}[wl]
        log(f"cpu baseline: oracle, {ncpu} shot(s) x {steps} steps on {cores} threads")
        rate, t = sample(ncpu, steps)
        # one thread, a smaller sample of the same grid
        n1, s1 = {"c2": (1, max(1, steps // 2)), "c3": (1, max(1, steps // 10)), "c4": (1, 1)}[wl]
        omp_threads(1)
        log(f"cpu baseline: oracle, {n1} shot x {s1} steps on 1 thread")
        rate1, t1 = sample(n1, s1)
        omp_threads(cores)
        out["cpu_baseline"] = {"value": round(rate, 4), "unit": "Gcell-updates/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"{ncpu} shot(s) x {steps} steps of the same grid, FP64 "
                                         f"fwd+adjoint, {t:.1f} s",
                               "single_thread": {"value": round(rate1, 5),
                                                 "sample": f"{n1} shot x {s1} steps, {t1:.1f} s"},
                               "host": host_cpu()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
