"""Error paths of the C ABI that need a device: a non-finite misfit is
reported as SG_ENUMERIC at the next synchronising status query, and the host
arrays of a shot batch (src, rec, mt) are refused when they are device
pointers, before the host reads them and before any kernel runs."""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

from gpu_common import S, synth, dev, gpu_desc, gpu_wavelets

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_non_finite_misfit_is_reported_at_the_next_sync():
    cfg = synth.C1.replace(nt=120)
    src, rec = synth.c1_geometry()
    sh = S.Shots(src, rec, gpu_wavelets([10.0], [0.1], cfg.dt, cfg.nt))
    m = S.Model(gpu_desc(cfg, 3000.0), dev(synth.layered_c1()), 1, rec.shape[1])
    pred = m.forward(sh)
    obs = pred.clone()
    m.check_numeric()                          # a fresh model is clear
    J, _ = m.misfit(pred, obs)
    m.check_numeric()                          # finite: nothing to report
    assert J.item() == 0.0
    obs[0, 0, 37, 11] = float("nan")
    J, r = m.misfit(pred, obs)                 # enqueues; does not fail by itself
    with pytest.raises(S.SeisError) as e:
        m.check_numeric()
    assert e.value.code == S.SG_ENUMERIC
    assert not np.isfinite(J.item())
    m.check_numeric()                          # reading the flag cleared it
    obs[0, 0, 37, 11] = float("inf")
    m.misfit(pred, obs)
    m.misfit(pred, pred)                       # a later finite misfit does not hide the earlier one
    with pytest.raises(S.SeisError) as e:
        m.check_numeric()
    assert e.value.code == S.SG_ENUMERIC
    # the model keeps working: forward, misfit and adjoint after the report
    obs = m.forward(sh).clone()
    J, r = m.misfit(pred, obs)
    g = m.gradient(sh, r)
    m.check_numeric()
    torch.cuda.synchronize()
    assert torch.isfinite(g).all()
    m.close()


_CHILD = r"""
import sys, ctypes as C
import numpy as np, torch
sys.path.insert(0, {root!r})
from paper_2003_06027_amd import seisgrad as S
nx, nz, nt = 60, 40, 30
d = S.desc(ndim=2, physics=S.SG_ELASTIC, nx=nx, nz=nz, npml=10, nt=nt, dx=5.0, dt=0.5e-3,
           pml_vmax=3000.0, f0_pml=20.0)
vp = torch.full((nz, nx), 2500.0, device="cuda")
m = S.Model(d, vp, 1, 4, vs=vp / 1.8, rho=torch.full_like(vp, 2000.0))
src = np.array([[30, 5]], dtype=np.int32)
rec = np.array([[[10, 0], [20, 0], [30, 0], [40, 0]]], dtype=np.int32)
wav = S.ricker(20.0, 0.05, 0.5e-3, nt)[None].contiguous()
seis = torch.empty((1, 2, nt, 4), device="cuda")
mt_dev = torch.tensor([[1.0, 1.0, 0.0]], device="cuda")
src_dev = torch.as_tensor(src, device="cuda")
out = []
for name, sp, mp in (("mt", src.ctypes.data, mt_dev.data_ptr()), ("src", src_dev.data_ptr(), None)):
    mt_host = np.array([[1.0, 1.0, 0.0]], dtype=np.float32)
    st = S.SgShots(1, 4, sp, rec.ctypes.data, wav.data_ptr(), mp if mp else mt_host.ctypes.data, 1)
    rc = S.lib().forward_shots(m.handle, C.byref(st), S._ptr(seis), 1, S._stream())
    out.append((name, rc, S.lib().last_error().decode()))
# NULL moment tensors for elastic shots
st = S.SgShots(1, 4, src.ctypes.data, rec.ctypes.data, wav.data_ptr(), None, 1)
out.append(("mt NULL", S.lib().forward_shots(m.handle, C.byref(st), S._ptr(seis), 1, S._stream()),
            S.lib().last_error().decode()))
# the same model still runs a valid batch
sh = S.Shots(src, rec, wav, mt=np.array([[1.0, 1.0, 0.0]]))
m.forward(sh)
torch.cuda.synchronize()
for name, rc, msg in out:
    print(name + "|" + str(rc) + "|" + msg, flush=True)
print("DONE", flush=True)
"""


def test_device_pointers_for_host_arrays_are_refused():
    """The host reads src, rec and mt while it uploads the geometry.  A
    device address there used to be read on the host (a segmentation fault
    of the calling process); it is now refused with SG_EINVAL before any
    read or launch.  Run in a child process so that a regression fails this
    test instead of ending the test session."""
    p = subprocess.run([sys.executable, "-c", _CHILD.format(root=ROOT)], capture_output=True, text=True,
                       timeout=300)
    print(p.stdout[-2000:], p.stderr[-2000:])
    assert p.returncode == 0, p.returncode
    assert "DONE" in p.stdout.splitlines()
    got = {ln.split("|")[0]: ln.split("|") for ln in p.stdout.splitlines() if "|" in ln}
    for name in ("mt", "src", "mt NULL"):
        assert int(got[name][1]) == S.SG_EINVAL, got[name]
