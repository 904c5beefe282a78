"""Thin ctypes binding of the preconditioner network (include/sg_cnn.h) and
the :class:`Preconditioner` that holds its parameters, Adam state and
workspace.

Argument marshalling only: the network's forward and backward, the loss,
Adam and the packing of gradient fields into patches all run in the
library's HIP kernels.  BF16 channels-last activations are passed as
torch.bfloat16 tensors of shape [n, h, w, 32].
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import seisgrad as S

NPARAMS = 37601
CHANNELS = 32
LAYERS = [(1, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 1)]   # (Cin, Cout)
EXPORTS = ("cnn_workspace_bytes", "cnn_forward", "cnn_backward", "cnn_loss", "cnn_adam", "cnn_pack",
           "cnn_unpack", "cnn_conv3x3", "cnn_conv3x3_wgrad")

_ready = False


def lib():
    global _ready
    L = S.lib()
    if not _ready:
        v, i32, i64, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_float
        L.cnn_workspace_bytes.restype = C.c_size_t
        L.cnn_workspace_bytes.argtypes = [i32, i32, i32]
        L.cnn_forward.argtypes = [v, v, i32, i32, i32, v, v, C.c_size_t, v]
        L.cnn_backward.argtypes = [v, v, v, i32, i32, i32, v, v, C.c_size_t, v]
        L.cnn_loss.argtypes = [v, v, v, i64, v, v, v, C.c_size_t, v]
        L.cnn_adam.argtypes = [v, v, v, v, i64, f32, f32, f32, f32, i32, v]
        L.cnn_pack.argtypes = [v, v, i32, v, i32, i32, i32, i32, i32, v, v, v, v]
        L.cnn_unpack.argtypes = [v, i32, i32, i32, i32, v, v]
        L.cnn_conv3x3.argtypes = [v, i32, i32, i32, v, v, v, v, i32, v, v, v]
        L.cnn_conv3x3_wgrad.argtypes = [v, v, i32, i32, i32, v, v, C.c_size_t, v]
        _ready = True
    return L


_ptr, _check, _stream = S._ptr, S._check, S._stream


def offsets():
    out, o = [], 0
    for cin, cout in LAYERS:
        out.append((o, o + 9 * cin * cout, cin, cout))
        o += 9 * cin * cout + cout
    return out


def workspace_bytes(n, h, w):
    nb = lib().cnn_workspace_bytes(n, h, w)
    if nb == 0:
        raise S.SeisError(S.SG_EINVAL, f"bad image extents {n}x{h}x{w}")
    return nb


def new_workspace(n, h, w, device="cuda"):
    return torch.empty(workspace_bytes(n, h, w), dtype=torch.uint8, device=device)


def forward(params, g, ws, stream=None):
    n, h, w = g.shape
    p = torch.empty_like(g)
    _check(lib().cnn_forward(_ptr(params), _ptr(g), n, h, w, _ptr(p), _ptr(ws), ws.numel(), _stream(stream)))
    return p


def backward(params, g, dp, ws, grad=None, stream=None):
    n, h, w = g.shape
    grad = grad if grad is not None else torch.empty(NPARAMS, dtype=torch.float32, device=g.device)
    _check(lib().cnn_backward(_ptr(params), _ptr(g), _ptr(dp), n, h, w, _ptr(grad), _ptr(ws), ws.numel(),
                              _stream(stream)))
    return grad


def loss(p, t, mask, ws, want_grad=True, stream=None):
    L = torch.empty(1, dtype=torch.float64, device=p.device)
    dp = torch.empty_like(p) if want_grad else None
    _check(lib().cnn_loss(_ptr(p), _ptr(t), _ptr(mask), p.numel(), _ptr(L), _ptr(dp), _ptr(ws), ws.numel(),
                          _stream(stream)))
    return L, dp


def adam(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().cnn_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), params.numel(), lr, beta1, beta2, eps,
                          step, _stream(stream)))


def pack(a, frame, b=None, order=None, normalise=True, stream=None, with_mask=True):
    """Fields [B, fh, fw] -> (patches, mask, inv_rms) per cnn_pack."""
    nf, fh, fw = a.shape if order is None else (order.numel(),) + tuple(a.shape[1:])
    npatch = (nf + 3) // 4
    patches = torch.empty(npatch, 2 * frame, 2 * frame, dtype=torch.float32, device=a.device)
    mask = torch.empty_like(patches) if with_mask else None
    inv = torch.empty(nf, dtype=torch.float64, device=a.device) if normalise else None
    _check(lib().cnn_pack(_ptr(a), _ptr(b), a.shape[0], _ptr(order), nf, fh, fw, frame, int(normalise), _ptr(inv),
                          _ptr(patches), _ptr(mask), _stream(stream)))
    return patches, mask, inv


def unpack(patches, nfields, fh, fw, frame, stream=None):
    out = torch.empty(nfields, fh, fw, dtype=torch.float32, device=patches.device)
    _check(lib().cnn_unpack(_ptr(patches), nfields, fh, fw, frame, _ptr(out), _stream(stream)))
    return out


def conv3x3(x, wgt, bias=None, res=None, gate=None, relu=False, want_fp32=False, stream=None):
    """One 32 -> 32 layer on BF16 [n, h, w, 32] tensors (weights [32, 3, 3, 32] BF16)."""
    n, h, w, c = x.shape
    assert c == CHANNELS and x.dtype == torch.bfloat16 and wgt.dtype == torch.bfloat16
    y = torch.empty_like(x)
    y32 = torch.empty(x.shape, dtype=torch.float32, device=x.device) if want_fp32 else None
    _check(lib().cnn_conv3x3(_ptr(x), n, h, w, _ptr(wgt), _ptr(bias), _ptr(res), _ptr(gate), int(relu),
                             _ptr(y), _ptr(y32), _stream(stream)))
    return (y, y32) if want_fp32 else y


def conv3x3_wgrad(dy, x, ws, stream=None):
    n, h, w, _ = x.shape
    dw = torch.empty(32 * 9 * 32 + 32, dtype=torch.float32, device=x.device)
    _check(lib().cnn_conv3x3_wgrad(_ptr(dy), _ptr(x), n, h, w, _ptr(dw), _ptr(ws), ws.numel(), _stream(stream)))
    return dw


def init_params(seed):
    """He-normal weights (std sqrt(2 / (9 Cin))), zero biases, and a zero last
    layer, so the untrained network returns the plain direction -g."""
    rng = np.random.default_rng(seed)
    p = np.zeros(NPARAMS, dtype=np.float32)
    for li, (wo, bo, cin, cout) in enumerate(offsets()):
        if li < 5:
            p[wo:bo] = rng.standard_normal(bo - wo) * np.sqrt(2.0 / (9 * cin))
    return p


class Preconditioner:
    """Parameters, Adam state and a workspace for batches of up to
    `max_patches` patches of size x size cells (frames of size / 2)."""

    def __init__(self, max_patches, size=256, seed=0, device="cuda", params=None):
        self.size, self.frame, self.max_patches = size, size // 2, max_patches
        p0 = init_params(seed) if params is None else np.asarray(params, dtype=np.float32)
        self.params = torch.tensor(p0, device=device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.step = 0
        self.ws = new_workspace(max_patches, size, size, device)

    def forward(self, x):
        assert x.shape[0] <= self.max_patches
        return forward(self.params, x, self.ws)

    def train_step(self, x, t, mask, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        """One Adam step on the masked MSE of p(x) against t; returns the loss (device FP64)."""
        p = self.forward(x)
        L, dp = loss(p, t, mask, self.ws)
        backward(self.params, x, dp, self.ws, grad=self.grad)
        self.step += 1
        adam(self.params, self.grad, self.m, self.v, self.step, lr, beta1, beta2, eps)
        return L

    def direction(self, g):
        """Search directions p [B, fh, fw] for gradient fields g [B, fh, fw]:
        each field divided by its RMS, framed, passed through the network."""
        B, fh, fw = g.shape
        out = torch.empty_like(g)
        for s in range(0, B, 4 * self.max_patches):
            gb = g[s:s + 4 * self.max_patches].contiguous()
            x, _, _ = pack(gb, self.frame, with_mask=False)
            out[s:s + gb.shape[0]] = unpack(self.forward(x), gb.shape[0], fh, fw, self.frame)
        return out


def _main():
    """Times training steps on seeded random patches (a profiling harness for
    the network kernels): python -m paper_2003_06027_amd.cnn --steps 50."""
    import argparse
    import json
    import time
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--size", type=int, default=256)
    a = ap.parse_args()
    rng = np.random.default_rng(0)
    shp = (a.batch, a.size, a.size)
    x = torch.tensor(rng.standard_normal(shp), dtype=torch.float32, device="cuda")
    t = torch.tensor(rng.standard_normal(shp), dtype=torch.float32, device="cuda")
    mask = torch.ones(shp, dtype=torch.float32, device="cuda")
    pre = Preconditioner(a.batch, a.size, seed=0)
    pre.params[N_LAST_W:] = torch.tensor(rng.standard_normal(NPARAMS - N_LAST_W) * 0.05, dtype=torch.float32,
                                         device="cuda")
    pre.train_step(x, t, mask, 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        pre.train_step(x, t, mask, 1e-4)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.steps
    flop = 3 * 2 * a.batch * a.size * a.size * sum(9 * ci * co for ci, co in LAYERS)
    print(json.dumps({"ms_per_train_step": round(dt * 1e3, 3), "patches": a.batch,
                      "tflops_fwd_bwd": round(flop / dt / 1e12, 2)}))


N_LAST_W = offsets()[5][0]

if __name__ == "__main__":
    _main()
