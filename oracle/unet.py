"""FP64 CPU reference of the learned correction network — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module; it shares nothing with the HIP library.

The paper proposes learned correction terms between physics-based operator
applications as the extension of its framework (Sec. 5) and specifies no
network.  The network used here (readings stated with the project's design):

* a 3-level 3D U-Net with 16 / 32 / 64 channels and one input channel: two
  3x3x3 convolutions (zero padding 1) with ReLU per level, 2x2x2 max pooling
  down, a 2x2x2 stride-2 transposed convolution up, skip concatenation
  [up-sampled, skip] along channels, a 1x1x1 head, and the residual output
  x + m U(s x) / s with a fixed input scale s (volumes stored per volume
  width are brought to O(1) values) and a per-voxel mask m confining the
  correction (the scanned field of view);
* one such network per unrolled stage: the pipeline applies a separate set
  of weights after each stage's physics iterations of Eq. (1) (this module
  evaluates one network; the stage loop is not part of the reference);
* MSE loss to the true volume, Adam.

Tensors are channels-last, [D][H][W][C], as torch float64 CPU tensors.
Weights use the layouts of the GPU library: 3x3x3 convolution [cout][cin][27]
with taps ordered (dz, dy, dx), dx fastest; transposed convolution
[cin][cout][8] with sub-positions (az, ay, ax), ax fastest.

Every convolution is a library call (torch conv3d / conv_transpose3d); the
module's tests pin them to plain loops and pin the network gradient to
central finite differences.
"""

from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

# (name, kind, cin, cout): the layers in forward order
LAYERS = (
    ("e1a", "conv", 1, 16),
    ("e1b", "conv", 16, 16),
    ("e2a", "conv", 16, 32),
    ("e2b", "conv", 32, 32),
    ("bna", "conv", 32, 64),
    ("bnb", "conv", 64, 64),
    ("up2", "up", 64, 32),
    ("d2a", "conv", 64, 32),
    ("d2b", "conv", 32, 32),
    ("up1", "up", 32, 16),
    ("d1a", "conv", 32, 16),
    ("d1b", "conv", 16, 16),
)


def weight_shape(kind, cin, cout):
    return (cout, cin, 27) if kind == "conv" else (cin, cout, 8)


def init_params(seed, head_std=1e-2):
    """He-normal weights, zero biases, a small random head (numpy float64)."""
    rng = np.random.default_rng([seed, 11])
    p = {}
    for name, kind, cin, cout in LAYERS:
        fan_in = cin * (27 if kind == "conv" else 1)
        p[name + ".w"] = rng.normal(0.0, np.sqrt(2.0 / fan_in), size=weight_shape(kind, cin, cout))
        p[name + ".b"] = np.zeros(cout)
    p["head.w"] = rng.normal(0.0, head_std, size=16)
    p["head.b"] = np.zeros(1)
    return p


def bf16_round(a):
    """Round float64 values to the nearest BF16 value (ties to even)."""
    t = torch.as_tensor(a, dtype=torch.float64)
    return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)


# ------------------------------------------------------------------ layers --
def _cf(x):
    """[D][H][W][C] -> [1][C][D][H][W]."""
    return x.permute(3, 0, 1, 2).unsqueeze(0)


def _cl(y):
    return y[0].permute(1, 2, 3, 0)


def conv3(x, w, b=None):
    """3x3x3 convolution, stride 1, zero padding 1 (cross-correlation)."""
    cout, cin, _ = w.shape
    return _cl(F.conv3d(_cf(x), w.reshape(cout, cin, 3, 3, 3), b, padding=1))


def upconv2(x, w, b=None):
    """2x2x2 stride-2 transposed convolution: out[2i + a] += x[i] w[a]."""
    cin, cout, _ = w.shape
    return _cl(F.conv_transpose3d(_cf(x), w.reshape(cin, cout, 2, 2, 2), b, stride=2))


def maxpool2(x):
    return _cl(F.max_pool3d(_cf(x), 2))


def maxpool2_backward(x, dout):
    """Gradient routed to the first maximum (ax fastest, then ay, az) of each
    2x2x2 window."""
    D, H, W, C = x.shape
    win = x.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).permute(0, 2, 4, 1, 3, 5, 6)
    win = win.reshape(D // 2, H // 2, W // 2, 8, C)
    arg = torch.argmax(win, dim=3, keepdim=True)   # first maximal index
    g = torch.zeros_like(win).scatter_(3, arg, dout.unsqueeze(3))
    g = g.reshape(D // 2, H // 2, W // 2, 2, 2, 2, C).permute(0, 3, 1, 4, 2, 5, 6)
    return g.reshape(D, H, W, C)


# ------------------------------------------------------------------- model --
def _t(p, requires_grad=False):
    return {k: torch.tensor(np.asarray(v), dtype=torch.float64, requires_grad=requires_grad)
            for k, v in p.items()}


def forward(x, params, round_activations=False, tensors=None, scale=1.0, mask=None):
    """U-Net correction of a volume: x + mask U(scale x) / scale.

    ``x`` is a [D][H][W] array; D, H, W divisible by 4.  With
    ``round_activations`` every stored activation is rounded to BF16, as a
    BF16-storage implementation keeps them (the arithmetic stays FP64).
    ``tensors`` optionally receives the intermediate activations by name.
    """
    P = params if isinstance(next(iter(params.values())), torch.Tensor) else _t(params)
    x = x if isinstance(x, torch.Tensor) else torch.as_tensor(np.asarray(x), dtype=torch.float64)
    r = bf16_round if round_activations else (lambda a: a)

    def cr(name, inp):
        return r(torch.relu(conv3(inp, P[name + ".w"], P[name + ".b"])))

    xin = r(scale * x.unsqueeze(-1))
    a1 = cr("e1a", xin)
    e1 = cr("e1b", a1)
    p1 = maxpool2(e1)
    a2 = cr("e2a", p1)
    e2 = cr("e2b", a2)
    p2 = maxpool2(e2)
    a3 = cr("bna", p2)
    b3 = cr("bnb", a3)
    u2 = r(upconv2(b3, P["up2.w"], P["up2.b"]))
    a4 = cr("d2a", torch.cat([u2, e2], dim=-1))
    d2 = cr("d2b", a4)
    u1 = r(upconv2(d2, P["up1.w"], P["up1.b"]))
    a5 = cr("d1a", torch.cat([u1, e1], dim=-1))
    d1 = cr("d1b", a5)
    corr = (P["head.b"][0] + d1 @ P["head.w"]) / scale
    if mask is not None:
        corr = corr * torch.as_tensor(np.asarray(mask), dtype=torch.float64)
    out = x + corr
    if tensors is not None:
        tensors.update(dict(xin=xin, a1=a1, e1=e1, p1=p1, a2=a2, e2=e2, p2=p2, a3=a3, b3=b3,
                            u2=u2, a4=a4, d2=d2, u1=u1, a5=a5, d1=d1))
    return out


def mse(a, t):
    a = a if isinstance(a, torch.Tensor) else torch.as_tensor(np.asarray(a), dtype=torch.float64)
    t = t if isinstance(t, torch.Tensor) else torch.as_tensor(np.asarray(t), dtype=torch.float64)
    return ((a - t) ** 2).mean()


def loss_and_grads(x, target, params, scale=1.0, mask=None):
    """MSE(x + mask U(scale x) / scale, target) and its gradient with respect
    to every parameter (reverse-mode differentiation of the FP64 forward)."""
    P = _t(params, requires_grad=True)
    loss = mse(forward(x, P, scale=scale, mask=mask), target)
    loss.backward()
    return loss.item(), {k: v.grad.numpy().copy() for k, v in P.items()}


def adam_step(param, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam update (numpy float64, returns new p, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return param - lr * mh / (np.sqrt(vh) + eps), m, v
