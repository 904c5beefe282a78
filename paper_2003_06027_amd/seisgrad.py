"""Thin ctypes binding of libseisgrad (include/seisgrad.h).

Argument marshalling only: torch supplies device memory and the stream; every
step of the forward sweep, the misfit and the adjoint sweep runs in the HIP
kernels of the library.  There is no CPU fallback: loading fails loudly when
the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libseisgrad.so")

SG_OK, SG_EINVAL, SG_EUNSTABLE, SG_ENOMEM, SG_ESTATE, SG_EDEVICE, SG_EUNSUPPORTED, SG_ENUMERIC = \
    0, -1, -2, -3, -4, -5, -6, -7
SG_ACOUSTIC, SG_ELASTIC, SG_ACOUSTIC_DIV = 0, 1, 2
SG_TUNE_TIME_BLOCKING, SG_TUNE_CHUNK_FWD3, SG_TUNE_CHUNK_ADJ3, SG_TUNE_CHUNK_LAYER3, SG_TUNE_SHOT_GROUP, \
    SG_TUNE_BLOCK_X, SG_TUNE_GRAPHS, SG_TUNE_PAIR = 0, 1, 2, 3, 4, 5, 6, 7
_NAMES = {SG_EINVAL: "SG_EINVAL", SG_EUNSTABLE: "SG_EUNSTABLE", SG_ENOMEM: "SG_ENOMEM",
          SG_ESTATE: "SG_ESTATE", SG_EDEVICE: "SG_EDEVICE", SG_EUNSUPPORTED: "SG_EUNSUPPORTED",
          SG_ENUMERIC: "SG_ENUMERIC"}

EXPORTS = ("workspace_bytes", "init_model", "update_model", "forward_shots", "misfit", "adjoint_gradient",
           "free_model", "last_error", "ricker", "dot_f64", "set_profiling", "phase_times",
           "set_time_blocking", "set_tuning", "snapshot_segment_bytes", "numeric_status", "misfit_noalloc", "lbfgs_push", "lbfgs_direction",
           "source_gaussian", "source_gaussian_grad", "source_rupture", "source_rupture_grad",
           "source_plane_wave")


class SeisError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class SgDesc(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("physics", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("nz", C.c_int32), ("npml", C.c_int32), ("nt", C.c_int32), ("nmodels", C.c_int32),
                ("dx", C.c_double), ("dt", C.c_double), ("pml_R", C.c_double),
                ("pml_vmax", C.c_double), ("f0_pml", C.c_double)]


class SgShots(C.Structure):
    _fields_ = [("nshots", C.c_int32), ("nrec", C.c_int32), ("src", C.c_void_p),
                ("rec", C.c_void_p), ("wavelet", C.c_void_p), ("mt", C.c_void_p), ("nsrc", C.c_int32)]


_lib = None


def lib():
    """Open libseisgrad.so; raise if it is missing (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2003_06027_amd.build`")
        L = C.CDLL(LIB_PATH)
        L.workspace_bytes.restype = C.c_size_t
        L.workspace_bytes.argtypes = [C.POINTER(SgDesc), C.c_int32, C.c_int32, C.c_int32]
        L.snapshot_segment_bytes.restype = C.c_size_t
        L.snapshot_segment_bytes.argtypes = [C.POINTER(SgDesc), C.c_int32, C.c_int32]
        L.init_model.argtypes = [C.POINTER(SgDesc), C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                 C.c_int32, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                                 C.POINTER(C.c_void_p)]
        L.update_model.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.forward_shots.argtypes = [C.c_void_p, C.POINTER(SgShots), C.c_void_p, C.c_int32, C.c_void_p]
        L.misfit.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
        L.adjoint_gradient.argtypes = [C.c_void_p, C.POINTER(SgShots), C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p]
        L.free_model.argtypes = [C.c_void_p]
        L.last_error.restype = C.c_char_p
        L.ricker.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int32, C.c_void_p, C.c_void_p]
        L.dot_f64.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
        L.set_profiling.argtypes = [C.c_void_p, C.c_int32]
        L.set_time_blocking.argtypes = [C.c_void_p, C.c_int32]
        L.numeric_status.argtypes = [C.c_void_p, C.c_void_p]
        L.set_tuning.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]
        L.misfit_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
        v = C.c_void_p
        L.lbfgs_push.argtypes = [C.c_int32, C.c_int64, C.c_int32, v, v, v, v, v, v, v, v, v]
        L.lbfgs_direction.argtypes = [C.c_int32, C.c_int64, C.c_int32, v, v, v, v, v, v, v]
        i32, d = C.c_int32, C.c_double
        L.source_gaussian.argtypes = [i32, i32, v, d, d, d, d, v, v, v]
        L.source_gaussian_grad.argtypes = [i32, i32, v, d, d, d, d, v, v, v, v, v]
        L.source_rupture.argtypes = [i32, i32, v, v, d, d, v, v]
        L.source_rupture_grad.argtypes = [i32, i32, v, v, d, d, v, v, v, v]
        L.source_plane_wave.argtypes = [i32, i32, d, d, d, d, d, d, d, v, v]
        L.phase_times.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        _lib = L
    return _lib


def _check(rc):
    if rc != SG_OK:
        raise SeisError(rc, lib().last_error().decode())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return C.c_void_p(t.data_ptr())


def desc(ndim=2, physics=SG_ACOUSTIC, nx=1, ny=1, nz=1, npml=0, nt=1, nmodels=1, dx=10.0, dt=1e-3,
         pml_R=1e-3, pml_vmax=3000.0, f0_pml=10.0):
    return SgDesc(ndim, physics, nx, ny, nz, npml, nt, nmodels, dx, dt, pml_R, pml_vmax, f0_pml)


def workspace_bytes(d, max_shots, max_rec, ckpt_every=0):
    n = lib().workspace_bytes(C.byref(d), max_shots, max_rec, ckpt_every)
    if n == 0:
        raise SeisError(SG_EINVAL, lib().last_error().decode())
    return n


def snapshot_segment_bytes(d, max_shots, ckpt_every=0):
    """Workspace bytes per checkpoint segment whose adjoint snapshots the
    forward keeps (extra workspace beyond workspace_bytes)."""
    n = lib().snapshot_segment_bytes(C.byref(d), max_shots, ckpt_every)
    if n == 0:
        raise SeisError(SG_EINVAL, lib().last_error().decode())
    return n


def ricker(f0, t0, dt, nt, out=None, stream=None):
    out = out if out is not None else torch.empty(nt, dtype=torch.float32, device="cuda")
    _check(lib().ricker(f0, t0, dt, nt, _ptr(out), _stream(stream)))
    return out


def dot_f64(x, y, stream=None):
    out = torch.empty(1, dtype=torch.float64, device=x.device)
    _check(lib().dot_f64(_ptr(x), _ptr(y), x.numel(), _ptr(out), _stream(stream)))
    return out


class Shots:
    """Host geometry (int32), host moment tensors (elastic) and the device
    wavelet of one batch of shots."""

    def __init__(self, src, rec, wavelet, mt=None):
        """src [nshots][ndim] (one point source per shot) or [nshots][nsrc][ndim]
        (several source nodes, 2-D acoustic; wavelet then [nshots][nsrc][nt])."""
        self.src = np.ascontiguousarray(src, dtype=np.int32)
        self.rec = np.ascontiguousarray(rec, dtype=np.int32)
        assert self.src.ndim in (2, 3) and self.rec.ndim == 3 and self.rec.shape[0] == self.src.shape[0]
        self.nsrc = self.src.shape[1] if self.src.ndim == 3 else 1
        self.wavelet = wavelet.contiguous()
        self.mt = None if mt is None else np.ascontiguousarray(mt, dtype=np.float32)
        self.nshots, self.nrec = self.rec.shape[0], self.rec.shape[1]

    def struct(self):
        return SgShots(self.nshots, self.nrec, self.src.ctypes.data, self.rec.ctypes.data,
                       self.wavelet.data_ptr(), None if self.mt is None else self.mt.ctypes.data, self.nsrc)


class Model:
    """A model handle plus its workspace (a torch uint8 device tensor)."""

    def __init__(self, d, vp, max_shots, max_rec, ckpt_every=0, stream=None, vs=None, rho=None, ws=None,
                 store_segments=0):
        """ws: an existing workspace (uint8 device tensor) to reuse; all of it
        is handed to the library.  store_segments: when ws is None, allocate
        room for the adjoint snapshots of that many checkpoint segments, which
        a checkpointed forward then keeps (no recomputation of them)."""
        self.d = d
        self.max_shots, self.max_rec = max_shots, max_rec
        self.elastic = d.physics == SG_ELASTIC
        nbytes = workspace_bytes(d, max_shots, max_rec, ckpt_every)
        if ws is None and store_segments > 0:
            nbytes += store_segments * snapshot_segment_bytes(d, max_shots, ckpt_every)
        if ws is not None and ws.numel() < nbytes:
            raise SeisError(SG_ENOMEM, f"workspace of {ws.numel()} bytes, {nbytes} needed")
        self.ws = ws if ws is not None else torch.empty(nbytes, dtype=torch.uint8, device=vp.device)
        self.handle = C.c_void_p()
        self.vp = vp.contiguous()
        self.vs = None if vs is None else vs.contiguous()
        self.rho = None if rho is None else rho.contiguous()
        _check(lib().init_model(C.byref(d), _ptr(self.vp), _ptr(self.vs), _ptr(self.rho), max_shots, max_rec,
                                ckpt_every, _ptr(self.ws), self.ws.numel(), _stream(stream), C.byref(self.handle)))

    def update(self, vp, vs=None, rho=None, stream=None):
        """New parameters on the same grid, shots and workspace (the model's
        lists, tables and segment graphs are kept)."""
        vp = vp.contiguous()
        vs = None if vs is None else vs.contiguous()
        rho = None if rho is None else rho.contiguous()
        _check(lib().update_model(self.handle, _ptr(vp), _ptr(vs), _ptr(rho), _stream(stream)))
        self.vp, self.vs, self.rho = vp, vs, rho

    def forward(self, shots, seis=None, save_ckpt=True, stream=None):
        if seis is None:
            ncomp = 2 if self.elastic else 1
            seis = torch.empty((shots.nshots, ncomp, self.d.nt, shots.nrec), dtype=torch.float32,
                               device=self.ws.device)
        self._shots = shots.struct()
        _check(lib().forward_shots(self.handle, C.byref(self._shots), _ptr(seis), int(save_ckpt), _stream(stream)))
        return seis

    def misfit(self, pred, obs, resid=None, stream=None):
        J = torch.empty(1, dtype=torch.float64, device=pred.device)
        if resid is None:
            resid = torch.empty_like(pred)
        _check(lib().misfit(self.handle, _ptr(pred), _ptr(obs), pred.numel(), _ptr(J), _ptr(resid), _stream(stream)))
        return J, resid

    def gradient(self, shots, dJdd, g_vp=None, g_wavelet=None, stream=None, g_vs=None, g_rho=None):
        """dJ/dvp (acoustic) or (dJ/dvp, dJ/dvs, dJ/drho) (elastic)."""
        shape = (self.d.nmodels, self.d.nz, self.d.nx) if self.d.ndim == 2 else \
            (self.d.nmodels, self.d.nz, self.d.ny, self.d.nx)
        new = lambda: torch.empty(shape, dtype=torch.float32, device=dJdd.device)
        if g_vp is None:
            g_vp = new()
        if self.elastic:
            g_vs = new() if g_vs is None else g_vs
            g_rho = new() if g_rho is None else g_rho
        st = shots.struct()
        _check(lib().adjoint_gradient(self.handle, C.byref(st), _ptr(dJdd.contiguous()), _ptr(g_vp), _ptr(g_vs),
                                      _ptr(g_rho), _ptr(g_wavelet), _stream(stream)))
        return (g_vp, g_vs, g_rho) if self.elastic else g_vp

    def check_numeric(self, stream=None):
        """Wait for the stream; raise SeisError(SG_ENUMERIC) if a misfit on this
        model since the last check was not finite (the flag is then cleared)."""
        _check(lib().numeric_status(self.handle, _stream(stream)))

    def set_time_blocking(self, steps):
        """Steps per launch of the 2-D acoustic blocked tiles (1 or 2)."""
        _check(lib().set_time_blocking(self.handle, int(steps)))

    def set_tuning(self, key, value, stream=None):
        """A launch setting (SG_TUNE_*): 3-D chunk lengths, elastic shot group
        and cell block width, time blocking.  Results do not depend on it
        (the elastic shot group only fixes the gradient's summation order)."""
        _check(lib().set_tuning(self.handle, int(key), int(value), _stream(stream)))

    def set_profiling(self, on=True):
        _check(lib().set_profiling(self.handle, int(on)))

    def phase_times(self):
        """{phase: (milliseconds, steps)} for forward / recompute / adjoint."""
        ms = (C.c_double * 3)()
        st = (C.c_int64 * 3)()
        _check(lib().phase_times(self.handle, ms, st))
        return {name: (ms[i], st[i]) for i, name in enumerate(("forward", "recompute", "adjoint"))}

    def close(self):
        if self.handle:
            lib().free_model(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
