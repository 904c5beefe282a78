"""Plain FP64 CPU oracle of the learned gradient preconditioner
(TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU
baseline of the benchmark use this module; the product path never does).

The paper has no network.  Its Limitations section calls ill-conditioning
intrinsic to the inversion and notes that techniques which improve the
conditioning can be applied within the framework; this preconditioner is one
such technique, of the project's own design, written as plainly as possible
with torch FP64 CPU ops:

* six 3x3 convolutions with zero padding: c1 (1->32), c2..c5 (32->32) in two
  residual blocks, c6 (32->1);
      x1 = relu(c1(g)),  a2 = relu(c2(x1)),  x2 = relu(c3(a2) + x1),
      a4 = relu(c4(x2)), x3 = relu(c5(a4) + x2),  p = -g + c6(x3);
* flat parameter vector, layer by layer: weights [Cout][3][3][Cin], then the
  Cout biases; 37,601 numbers in all;
* masked mean-squared loss L = sum(mask (p - t)^2) / sum(mask);
* Adam (Kingma and Ba, Algorithm 1) with bias-corrected moments;
* the patch packing: each 2-D field (divided by its RMS) sits in the top-left
  corner of a zero frame x frame square; 2 x 2 frames form one patch.

``bf16=True`` mirrors where the accelerated path stores BF16: the weights of
c2..c5 and the stored activations x1, a2, x2, a4, x3 and back-propagated
pre-activation gradients are rounded to BF16 (round to nearest even), every
product and sum stays FP64.  The manual backward below is checked against
autograd and central differences in the CPU tests.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

C = 32
LAYERS = [(1, C), (C, C), (C, C), (C, C), (C, C), (C, 1)]     # (Cin, Cout)


def offsets():
    """[(w_off, b_off, cin, cout)] into the flat parameter vector."""
    out, o = [], 0
    for cin, cout in LAYERS:
        out.append((o, o + 9 * cin * cout, cin, cout))
        o += 9 * cin * cout + cout
    return out


NPARAMS = sum(9 * ci * co + co for ci, co in LAYERS)


def round_bf16(x):
    """Round to the nearest BF16 value (ties to even), returned in FP64.
    Values are first rounded to FP32, the precision the path holds them in."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _t(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64))


def unflatten(params, bf16=False):
    """Flat vector -> [(w [Cout][Cin][3][3] torch FP64, b [Cout])]."""
    params = np.asarray(params, dtype=np.float64)
    out = []
    for li, (wo, bo, cin, cout) in enumerate(offsets()):
        w = params[wo:bo].reshape(cout, 3, 3, cin)
        if bf16 and 1 <= li <= 4:
            w = round_bf16(w)
        out.append((_t(w).permute(0, 3, 1, 2).contiguous(), _t(params[bo:bo + cout])))
    return out


def flatten(layers):
    """Inverse of :func:`unflatten` (w in torch's [Cout][Cin][3][3])."""
    parts = []
    for w, b in layers:
        parts.append(np.asarray(w.detach().permute(0, 2, 3, 1).reshape(-1), dtype=np.float64))
        parts.append(np.asarray(b.detach().reshape(-1), dtype=np.float64))
    return np.concatenate(parts)


def conv3x3(x, w, b=None):
    """Cross-correlation with a 3x3 kernel and one cell of zero padding.
    x [N][Cin][H][W], w [Cout][Cin][3][3]."""
    return F.conv2d(x, w, b, padding=1)


def _store(x, bf16):
    return _t(round_bf16(x.numpy())) if bf16 else x


def forward(params, g, bf16=False):
    """p = -g + N(g) for g [N][H][W]; returns (p [N][H][W], activations)."""
    L = unflatten(params, bf16)
    x = _t(g)[:, None]
    relu = torch.relu
    x1 = _store(relu(conv3x3(x, *L[0])), bf16)
    a2 = _store(relu(conv3x3(x1, *L[1])), bf16)
    x2 = _store(relu(conv3x3(a2, *L[2]) + x1), bf16)
    a4 = _store(relu(conv3x3(x2, *L[3])), bf16)
    x3 = _store(relu(conv3x3(a4, *L[4]) + x2), bf16)
    p = -x[:, 0] + conv3x3(x3, *L[5])[:, 0]
    return p.numpy(), dict(x=x, x1=x1, a2=a2, x2=x2, a4=a4, x3=x3)


def conv3x3_input_grad(dy, w):
    """d/dx of sum(dy * conv3x3(x, w)): the transposed correlation."""
    return F.conv_transpose2d(dy, w, padding=1)


def conv3x3_weight_grad(dy, x):
    """d/dw[o][i][ky][kx] = sum_{n,y,x} dy[n][o][y][x] x[n][i][y+ky-1][x+kx-1]
    (zero outside), written out over the 9 taps."""
    N, Ci, H, W = x.shape
    xp = F.pad(x, (1, 1, 1, 1))
    dw = torch.zeros(dy.shape[1], Ci, 3, 3, dtype=torch.float64)
    for ky in range(3):
        for kx in range(3):
            sl = xp[:, :, ky:ky + H, kx:kx + W]
            dw[:, :, ky, kx] = torch.einsum("noyx,niyx->oi", dy, sl)
    return dw


def backward(params, acts, dp, bf16=False):
    """Gradient of sum(dp * p) with respect to the flat parameter vector,
    the chain rule taken layer by layer from c6 back to c1."""
    L = unflatten(params, bf16)
    dp = _t(dp)[:, None]
    st = lambda v: _store(v, bf16)
    grads = [None] * 6

    def wb(dz, xin):
        return conv3x3_weight_grad(dz, xin), dz.sum(dim=(0, 2, 3))

    grads[5] = wb(dp, acts["x3"])
    g5 = st(conv3x3_input_grad(dp, L[5][0]) * (acts["x3"] > 0))            # d pre-act of x3
    grads[4] = wb(g5, acts["a4"])
    g4 = st(conv3x3_input_grad(g5, L[4][0]) * (acts["a4"] > 0))
    grads[3] = wb(g4, acts["x2"])
    g3 = st((conv3x3_input_grad(g4, L[3][0]) + g5) * (acts["x2"] > 0))
    grads[2] = wb(g3, acts["a2"])
    g2 = st(conv3x3_input_grad(g3, L[2][0]) * (acts["a2"] > 0))
    grads[1] = wb(g2, acts["x1"])
    g1 = st((conv3x3_input_grad(g2, L[1][0]) + g3) * (acts["x1"] > 0))
    grads[0] = wb(g1, acts["x"])
    return flatten(grads)


def loss(p, t, mask):
    """(L, dL/dp) of the masked mean squared error."""
    p, t, mask = (np.asarray(a, dtype=np.float64) for a in (p, t, mask))
    n = mask.sum()
    r = (p - t) * mask
    return float((r * r).sum() / n), 2.0 * r / n


def adam(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (params, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v


def pack(fields, frame, minus=None, normalise=True, order=None):
    """Fields [B][fh][fw] (optionally fields - minus, optionally divided by
    the RMS of each field, optionally re-ordered: slot s takes field
    order[s]) -> patches [ceil(B/4)][2 frame][2 frame] and the 0/1 mask."""
    f = np.asarray(fields, dtype=np.float64)
    if minus is not None:
        f = f - np.asarray(minus, dtype=np.float64)
    if order is not None:
        f = f[np.asarray(order)]
    B, fh, fw = f.shape
    npatch = (B + 3) // 4
    out = np.zeros((npatch, 2 * frame, 2 * frame))
    mask = np.zeros_like(out)
    for b in range(B):
        v = f[b]
        if normalise:
            v = v / np.sqrt((v * v).mean())
        q, k = divmod(b, 4)
        y0, x0 = (k // 2) * frame, (k % 2) * frame
        out[q, y0:y0 + fh, x0:x0 + fw] = v
        mask[q, y0:y0 + fh, x0:x0 + fw] = 1.0
    return out, mask


def unpack(patches, nfields, fh, fw, frame):
    patches = np.asarray(patches, dtype=np.float64)
    out = np.zeros((nfields, fh, fw))
    for b in range(nfields):
        q, k = divmod(b, 4)
        y0, x0 = (k // 2) * frame, (k % 2) * frame
        out[b] = patches[q, y0:y0 + fh, x0:x0 + fw]
    return out
