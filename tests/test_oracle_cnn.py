"""Pins of the FP64 CNN oracle against things other than itself: brute-force
loops, torch autograd and BF16 conversion (library routines), central
differences, the adjoint identities of correlation, Adam's closed-form early
steps, and the invariants of the design (parameter count, zero-initialised
last layer = plain gradient direction, receptive radius 6)."""
import numpy as np
import pytest
import torch

from oracle import cnn as K


def _rand_params(seed, last_zero=False, scale=0.3):
    rng = np.random.default_rng(seed)
    p = np.zeros(K.NPARAMS)
    for li, (wo, bo, cin, cout) in enumerate(K.offsets()):
        p[wo:bo] = rng.standard_normal(bo - wo) * scale / np.sqrt(9 * cin)
        p[bo:bo + cout] = rng.standard_normal(cout) * 0.05
        if last_zero and li == 5:
            p[wo:bo + cout] = 0.0
    return p


def test_parameter_count_and_layout():
    assert K.NPARAMS == 37601
    offs = K.offsets()
    assert offs[0] == (0, 288, 1, 32)
    assert offs[1][0] == 320 and offs[5] == (37312, 37600, 32, 1)


def test_conv3x3_matches_brute_force_loop():
    rng = np.random.default_rng(1)
    N, Ci, Co, H, W = 2, 2, 3, 5, 4
    x = rng.standard_normal((N, Ci, H, W))
    w = rng.standard_normal((Co, Ci, 3, 3))
    b = rng.standard_normal(Co)
    ref = np.zeros((N, Co, H, W))
    for n in range(N):
        for o in range(Co):
            for y in range(H):
                for xx in range(W):
                    s = b[o]
                    for i in range(Ci):
                        for ky in range(3):
                            for kx in range(3):
                                yy, xs = y + ky - 1, xx + kx - 1
                                if 0 <= yy < H and 0 <= xs < W:
                                    s += w[o, i, ky, kx] * x[n, i, yy, xs]
                    ref[n, o, y, xx] = s
    got = K.conv3x3(torch.tensor(x), torch.tensor(w), torch.tensor(b)).numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13)


def test_correlation_adjoint_identities():
    rng = np.random.default_rng(2)
    x = torch.tensor(rng.standard_normal((2, 4, 7, 6)))
    w = torch.tensor(rng.standard_normal((5, 4, 3, 3)))
    y = torch.tensor(rng.standard_normal((2, 5, 7, 6)))
    lhs = float((K.conv3x3(x, w) * y).sum())
    assert abs(lhs - float((x * K.conv3x3_input_grad(y, w)).sum())) <= 1e-12 * abs(lhs)
    assert abs(lhs - float((w * K.conv3x3_weight_grad(y, x)).sum())) <= 1e-12 * abs(lhs)


def test_round_bf16_ties_and_library_conversion():
    vals = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 3.0e-39, 65504.0])
    exp = np.array([1.0, 1.0, 1 + 2.0 ** -6, -1.0], dtype=np.float64)
    np.testing.assert_array_equal(K.round_bf16(vals)[:4], exp)
    rng = np.random.default_rng(3)
    a = (rng.standard_normal(100000) * np.exp(rng.uniform(-20, 20, 100000))).astype(np.float32)
    ref = torch.tensor(a).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(K.round_bf16(a), ref)


def test_zero_last_layer_gives_plain_gradient_direction():
    rng = np.random.default_rng(4)
    g = rng.standard_normal((3, 12, 10))
    p, _ = K.forward(_rand_params(5, last_zero=True), g)
    np.testing.assert_array_equal(p, -g)


@pytest.mark.parametrize("bf16", [False, True])
def test_manual_backward_matches_autograd(bf16):
    rng = np.random.default_rng(6)
    params = _rand_params(7)
    g = rng.standard_normal((2, 9, 8))
    dp = rng.standard_normal((2, 9, 8))
    p, acts = K.forward(params, g)
    got = K.backward(params, acts, dp)
    # autograd of the same network written with torch.nn layers
    net = torch.nn.ModuleList([torch.nn.Conv2d(ci, co, 3, padding=1).double() for ci, co in K.LAYERS])
    with torch.no_grad():
        for layer, (w, b) in zip(net, K.unflatten(params)):
            layer.weight.copy_(w)
            layer.bias.copy_(b)
    x = torch.tensor(g)[:, None]
    r = torch.relu
    x1 = r(net[0](x))
    x2 = r(net[2](r(net[1](x1))) + x1)
    x3 = r(net[4](r(net[3](x2))) + x2)
    pt = -x[:, 0] + net[5](x3)[:, 0]
    np.testing.assert_allclose(pt.detach().numpy(), p, rtol=1e-12, atol=1e-12)
    (pt * torch.tensor(dp)).sum().backward()
    ref = K.flatten([(layer.weight.grad, layer.bias.grad) for layer in net])
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
    if bf16:
        # the BF16-storage mirror stays close to the exact gradient
        pb, ab = K.forward(params, g, bf16=True)
        gb = K.backward(params, ab, dp, bf16=True)
        assert np.linalg.norm(pb - p) <= 2e-2 * np.linalg.norm(p)
        assert np.linalg.norm(gb - ref) <= 5e-2 * np.linalg.norm(ref)


def test_backward_central_differences():
    rng = np.random.default_rng(8)
    params = _rand_params(9)
    g = rng.standard_normal((2, 6, 7))
    dp = rng.standard_normal((2, 6, 7))
    _, acts = K.forward(params, g)
    grad = K.backward(params, acts, dp)
    f = lambda q: float((K.forward(q, g)[0] * dp).sum())
    picks = []
    for wo, bo, cin, cout in K.offsets():
        picks += list(rng.integers(wo, bo, 3)) + [bo + int(rng.integers(0, cout))]
    h = 1e-6
    for i in picks:
        e = np.zeros_like(params)
        e[i] = h
        fd = (f(params + e) - f(params - e)) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(grad[i])), (i, fd, grad[i])


def test_receptive_radius_is_six():
    rng = np.random.default_rng(10)
    params = _rand_params(11)
    g = rng.standard_normal((1, 32, 32))
    p0, _ = K.forward(params, g)
    g2 = g.copy()
    g2[0, 16, 16] += 1.0
    p1, _ = K.forward(params, g2)
    d = np.abs(p1 - p0)[0]
    ys, xs = np.nonzero(d > 0)
    assert max(np.abs(ys - 16).max(), np.abs(xs - 16).max()) == 6


def test_loss_closed_form():
    p = np.array([[1.0, 2.0], [3.0, 4.0]])
    t = np.array([[0.0, 2.0], [1.0, 0.0]])
    m = np.array([[1.0, 1.0], [1.0, 0.0]])
    L, d = K.loss(p, t, m)
    assert L == pytest.approx((1 + 0 + 4) / 3)
    np.testing.assert_allclose(d, 2 * np.array([[1.0, 0.0], [2.0, 0.0]]) / 3)


def test_adam_early_steps_closed_form():
    rng = np.random.default_rng(12)
    p0 = rng.standard_normal(50)
    g = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    lr, eps = 1e-3, 1e-8
    p1, m, v = K.adam(p0, g, m, v, 1, lr, eps=eps)
    np.testing.assert_allclose(p1, p0 - lr * g / (np.abs(g) + eps), rtol=1e-14, atol=1e-15)
    # a constant gradient keeps the bias-corrected moments at g and g^2
    p2, m, v = K.adam(p1, g, m, v, 2, lr, eps=eps)
    np.testing.assert_allclose(p2, p1 - lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)


def test_pack_unpack_layout():
    rng = np.random.default_rng(13)
    f = rng.standard_normal((6, 5, 7)) * 3 + 1
    m = rng.standard_normal((6, 5, 7))
    order = rng.permutation(6)
    pk, mask = K.pack(f, 8, minus=m, order=order)
    assert pk.shape == (2, 16, 16) and mask.sum() == 6 * 35
    back = K.unpack(pk, 6, 5, 7, 8)
    for s in range(6):
        d = f[order[s]] - m[order[s]]
        np.testing.assert_allclose(back[s], d / np.sqrt((d * d).mean()), rtol=1e-14)
    # slot 5 lives in the second patch, top-right frame; everything outside frames is zero
    np.testing.assert_array_equal(pk[1, 0:5, 8:15], back[5])
    assert np.all(pk[mask == 0] == 0)
