"""Pins of the FP64 U-Net reference (oracle/unet.py) to plain loops, finite
differences and closed forms.  CPU only."""

import itertools

import numpy as np
import pytest
import torch

from oracle import unet


def _rng(s):
    return np.random.default_rng([s, 99])


def _loop_conv3(x, w, b):
    D, H, W, cin = x.shape
    cout = w.shape[0]
    out = np.zeros((D, H, W, cout))
    for z, y, xx in itertools.product(range(D), range(H), range(W)):
        for tap in range(27):
            dz, dy, dx = tap // 9 - 1, (tap // 3) % 3 - 1, tap % 3 - 1
            zz, yy, x2 = z + dz, y + dy, xx + dx
            if 0 <= zz < D and 0 <= yy < H and 0 <= x2 < W:
                out[z, y, xx] += w[:, :, tap] @ x[zz, yy, x2]
        out[z, y, xx] += b
    return out


def test_conv3_matches_loops():
    r = _rng(1)
    x = r.normal(size=(3, 4, 5, 2))
    w = r.normal(size=(3, 2, 27))
    b = r.normal(size=3)
    got = unet.conv3(torch.tensor(x), torch.tensor(w), torch.tensor(b)).numpy()
    np.testing.assert_allclose(got, _loop_conv3(x, w, b), rtol=1e-12, atol=1e-12)


def test_conv3_tap_order_single_tap():
    """A weight that is 1 only at tap (dz, dy, dx) = (+1, 0, -1) reads x[z+1, y, x-1]."""
    x = _rng(2).normal(size=(4, 4, 4, 1))
    w = np.zeros((1, 1, 27))
    w[0, 0, 2 * 9 + 1 * 3 + 0] = 1.0
    got = unet.conv3(torch.tensor(x), torch.tensor(w)).numpy()[..., 0]
    want = np.zeros((4, 4, 4))
    want[:3, :, 1:] = x[1:, :, :3, 0]
    np.testing.assert_array_equal(got, want)


def test_upconv2_matches_loops():
    r = _rng(3)
    x = r.normal(size=(2, 3, 2, 4))
    w = r.normal(size=(4, 3, 8))
    b = r.normal(size=3)
    got = unet.upconv2(torch.tensor(x), torch.tensor(w), torch.tensor(b)).numpy()
    want = np.zeros((4, 6, 4, 3)) + b
    for z, y, xx in itertools.product(range(2), range(3), range(2)):
        for a in range(8):
            az, ay, ax = a >> 2, (a >> 1) & 1, a & 1
            want[2 * z + az, 2 * y + ay, 2 * xx + ax] += x[z, y, xx] @ w[:, :, a]
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


def test_maxpool_forward_and_first_max_backward():
    r = _rng(4)
    x = np.round(r.normal(size=(4, 2, 4, 3)), 0)   # many ties
    d = r.normal(size=(2, 1, 2, 3))
    got = unet.maxpool2(torch.tensor(x)).numpy()
    gin = unet.maxpool2_backward(torch.tensor(x), torch.tensor(d)).numpy()
    want = np.zeros_like(got)
    wgin = np.zeros_like(x)
    for z, y, xx, c in itertools.product(range(2), range(1), range(2), range(3)):
        best, arg = -np.inf, None
        for a in range(8):   # ax fastest, then ay, az
            p = (2 * z + (a >> 2), 2 * y + ((a >> 1) & 1), 2 * xx + (a & 1))
            if x[p + (c,)] > best:
                best, arg = x[p + (c,)], p
        want[z, y, xx, c] = best
        wgin[arg + (c,)] += d[z, y, xx, c]
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(gin, wgin)


def test_bf16_rounding_ties_to_even():
    one = 1.0
    vals = np.array([one + 2.0 ** -8, one + 3 * 2.0 ** -8, one + 2.0 ** -9, -(one + 2.0 ** -7)])
    got = unet.bf16_round(vals).numpy()
    np.testing.assert_array_equal(got, [1.0, 1.0 + 2.0 ** -6, 1.0, -(1.0 + 2.0 ** -7)])


def test_zero_head_is_identity():
    p = unet.init_params(0)
    p["head.w"][:] = 0.0
    x = _rng(5).normal(size=(8, 8, 8))
    out = unet.forward(x, p).numpy()
    np.testing.assert_array_equal(out, x)


def test_gradients_match_central_differences():
    p = unet.init_params(6, head_std=0.5)
    for k in p:
        if k.endswith(".b"):
            p[k] = _rng(7).normal(0, 0.05, size=p[k].shape)
    r = _rng(8)
    x = r.uniform(0, 1, size=(8, 8, 4))
    t = x + 0.1 * r.normal(size=x.shape)
    loss, g = unet.loss_and_grads(x, t, p)
    assert np.isfinite(loss)
    probes = [("e1a.w", (3, 0, 13)), ("e1b.w", (5, 7, 0)), ("e2a.b", (4,)), ("bna.w", (10, 3, 26)),
              ("bnb.b", (33,)), ("up2.w", (12, 7, 5)), ("up2.b", (30,)), ("d2a.w", (2, 40, 4)),
              ("d2a.w", (2, 5, 4)), ("up1.w", (8, 3, 1)), ("d1a.w", (1, 20, 22)),
              ("d1b.w", (15, 15, 14)), ("head.w", (2,)), ("head.b", (0,))]
    h = 1e-6
    for name, idx in probes:
        pp, pm = {k: v.copy() for k, v in p.items()}, {k: v.copy() for k, v in p.items()}
        pp[name][idx] += h
        pm[name][idx] -= h
        fd = (float(unet.mse(unet.forward(x, pp), t)) - float(unet.mse(unet.forward(x, pm), t))) / (2 * h)
        an = g[name][idx]
        assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-3), (name, idx, fd, an)


def test_gradient_of_concatenation_order():
    """The first half of the decoder's input channels is the up-sampled path:
    with the weights on that half zeroed, nothing below level 1 receives a
    gradient, while the skip path still does."""
    p = unet.init_params(9, head_std=0.5)
    p["d1a.w"][:, :16, :] = 0.0
    x = _rng(10).uniform(size=(8, 8, 8))
    _, g = unet.loss_and_grads(x, x + 0.1, p)
    for name in ("e2a", "e2b", "bna", "bnb", "up2", "d2a", "d2b", "up1"):
        assert np.all(g[name + ".w"] == 0) and np.all(g[name + ".b"] == 0), name
    assert np.any(g["e1b.w"] != 0) and np.any(g["e1a.w"] != 0)


def test_adam_first_step_closed_form():
    r = _rng(11)
    p0, g = r.normal(size=50), r.normal(size=50)
    p1, m, v = unet.adam_step(p0, g, np.zeros(50), np.zeros(50), 1, lr=1e-3, eps=1e-8)
    np.testing.assert_allclose(p1, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_input_scale_is_a_change_of_units():
    """x + U(s x)/s equals (s x + U(s x)) / s: the scaled network is the
    unscaled one applied in units where the volume is s times larger."""
    p = unet.init_params(12, head_std=0.5)
    x = _rng(13).uniform(0, 0.01, size=(8, 8, 8))
    s = 256.0
    a = unet.forward(x, p, scale=s).numpy()
    b = unet.forward(s * x, p).numpy() / s
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-18)


def test_mask_confines_the_correction():
    p = unet.init_params(14, head_std=0.5)
    x = _rng(15).uniform(0, 1, size=(8, 8, 8))
    m = np.zeros((8, 8, 8))
    m[2:6, 2:6, 2:6] = 1.0
    full = unet.forward(x, p).numpy()
    got = unet.forward(x, p, mask=m).numpy()
    np.testing.assert_array_equal(got[m == 0], x[m == 0])
    np.testing.assert_allclose(got[m == 1], full[m == 1], rtol=1e-14, atol=1e-14)
