"""3D U-Net correction network on the libctrex learned-correction kernels.

The network (16 / 32 / 64 channels, three levels) corrects a volume between
unrolled SIRT iterations of Eq. (1), the learned correction term the paper
names as the extension of its operator framework (Sec. 5):

    level 1 (D x H x W):    conv 1->16, conv 16->16          -> e1 (skip)
    level 2 (D/2 ...):      pool, conv 16->32, conv 32->32   -> e2 (skip)
    level 3 (D/4 ...):      pool, conv 32->64, conv 64->64
    decoder level 2:        up 64->32, concat [up, e2], conv 64->32, conv 32->32
    decoder level 1:        up 32->16, concat [up, e1], conv 32->16, conv 16->16
    head:                   out = x + m (b + sum_c h_c d1_c) / s

with the network reading s x: the fixed input scale s brings volumes stored in
small physical units (attenuation per volume width) to the O(1) range the
biases work in, and the head maps the correction back.  The optional mask m
(per voxel) confines the correction, e.g. to the scanned field of view.

Every 3x3x3 convolution is followed by ReLU; the up-sampling is a 2x2x2
stride-2 transposed convolution.  Activations are BF16 channels-last in
device memory; the concatenations are written in place (the up-sampling and
the skip convolution write the two halves of one tensor).  Parameters, their
gradients and the Adam moments are FP32 in one flat device buffer.

This module only marshals arguments: every arithmetic step (convolutions,
their data and weight gradients, pooling, head, loss, Adam, weight packing)
runs in libctrex (include/ctrex_nn.h).
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check

# (name, kind, cin, cout) in forward order
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
_KIND = {name: (kind, cin, cout) for name, kind, cin, cout in LAYERS}
# resolution level of each layer's weight-gradient input (1 = full resolution;
# an up-sampling layer reads the coarser level below it)
_LEVEL = dict(e1a=1, e1b=1, e2a=2, e2b=2, bna=3, bnb=3, up2=3, d2a=2, d2b=2, up1=2, d1a=1, d1b=1)


def _wshape(kind, cin, cout):
    return (cout, cin, 27) if kind == "conv" else (cin, cout, 8)


def param_shapes():
    """Ordered {name: shape} of every parameter (master layouts)."""
    out = {}
    for name, kind, cin, cout in LAYERS:
        out[name + ".w"] = _wshape(kind, cin, cout)
        out[name + ".b"] = (cout,)
    out["head.w"] = (16,)
    out["head.b"] = (1,)
    return out


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


class UNet:
    """The correction network on one device.

    ``params``: optional {name: array} in the master layouts of
    ``param_shapes()`` (conv [cout][cin][27], up-sampling [cin][cout][8]);
    otherwise He-normal weights from ``seed`` with zero biases and a head of
    standard deviation ``head_std``.  ``scale``: the input scale s.
    """

    def __init__(self, device=None, params=None, seed=0, head_std=1e-2, scale=1.0):
        dev = torch.device(device if device is not None else "cuda")
        if dev.type != "cuda":
            raise ValueError("the network runs on a HIP device")
        self.device = torch.device("cuda", dev.index if dev.index is not None
                                   else torch.cuda.current_device())
        self._ctx = ctypes.c_void_p()
        L = _lib.lib()
        code = L.ctrex_create(ctypes.byref(self._ctx), self.device.index)
        if code != _lib.OK:
            raise _lib.CtrexError(code, "ctrex_create failed on %s" % self.device)
        shapes = param_shapes()
        self._offsets = {}
        n = 0
        for k, s in shapes.items():
            size = int(np.prod(s))
            # 16-byte aligned slices
            self._offsets[k] = (n, s)
            n += (size + 3) // 4 * 4
        self.n_params = n
        self.scale = float(scale)
        if not np.isfinite(self.scale) or self.scale <= 0:
            raise ValueError("scale must be a positive finite number")
        self.theta = torch.zeros(n, dtype=torch.float32, device=self.device)
        self.grad = torch.zeros_like(self.theta)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.step = 0
        if params is None:
            rng = np.random.default_rng([seed, 11])
            params = {}
            for name, kind, cin, cout in LAYERS:
                fan_in = cin * (27 if kind == "conv" else 1)
                params[name + ".w"] = rng.normal(0.0, np.sqrt(2.0 / fan_in),
                                                 size=_wshape(kind, cin, cout))
                params[name + ".b"] = np.zeros(cout)
            params["head.w"] = rng.normal(0.0, head_std, size=16)
            params["head.b"] = np.zeros(1)
        self.load_params(params)
        self._bufs = {}
        self._saved = None

    # ------------------------------------------------------------ lifecycle
    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            _lib.lib().ctrex_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()
        self._scr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _s(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _call(self, fn, *args):
        check(self._ctx, getattr(_lib.lib(), fn)(self._ctx, *args))

    # ----------------------------------------------------------- parameters
    def p(self, name, which=None):
        """View of parameter ``name`` in ``which`` (theta, grad, m or v)."""
        off, s = self._offsets[name]
        t = self.theta if which is None else which
        return t[off:off + int(np.prod(s))].view(*s)

    def load_params(self, params):
        for k, (off, s) in self._offsets.items():
            a = np.asarray(params[k], dtype=np.float32)
            if a.shape != tuple(s):
                raise ValueError("%s has shape %s, expected %s" % (k, a.shape, s))
            self.p(k).copy_(torch.from_numpy(np.ascontiguousarray(a)))
        self._pack()

    def params(self):
        """{name: float32 numpy array} of the current parameters."""
        return {k: self.p(k).detach().cpu().numpy().copy() for k in self._offsets}

    def grads(self):
        return {k: self.p(k, self.grad).detach().cpu().numpy().copy() for k in self._offsets}

    def state_dict(self):
        """Parameters, Adam moments and step (checkpoint)."""
        return dict(theta=self.theta.cpu().numpy().copy(), m=self.m.cpu().numpy().copy(),
                    v=self.v.cpu().numpy().copy(), step=self.step, scale=self.scale)

    def load_state_dict(self, st):
        for name in ("theta", "m", "v"):
            getattr(self, name).copy_(torch.from_numpy(np.asarray(st[name], dtype=np.float32)))
        self.step = int(st["step"])
        if "scale" in st:
            self.scale = float(st["scale"])
        self._pack()

    def _pack(self):
        """BF16 packings of every layer: forward and data-gradient layouts,
        rewritten in place after the first call (a captured forward graph
        reads them at fixed addresses)."""
        if not getattr(self, "_wt", None):
            self._wt, self._wd = {}, {}
        for name, kind, cin, cout in LAYERS:
            taps = 27 if kind == "conv" else 8
            wt, wd = self._wt.get(name), self._wd.get(name)
            if wt is None:
                wt = torch.empty(taps * cin * cout, dtype=torch.bfloat16, device=self.device)
                wd = torch.empty_like(wt)
            w = self.p(name + ".w")
            if kind == "conv":
                self._call("ctrex_nn_pack_conv3", _vp(w), cout, cin, _vp(wt), _vp(wd), self._s())
            else:
                self._call("ctrex_nn_pack_upconv2", _vp(w), cin, cout, _vp(wt), _vp(wd), self._s())
            self._wt[name], self._wd[name] = wt, wd

    # -------------------------------------------------------------- buffers
    def _buffers(self, shape, train):
        key = (shape, train)
        if key in self._bufs:
            return self._bufs[key]
        D, H, W = shape
        n1 = D * H * W
        n2, n3 = n1 // 8, n1 // 64

        def t(n, c):
            return torch.empty(n * c, dtype=torch.bfloat16, device=self.device)

        # the skip concatenations [u | e] are never stored: the decoder's first
        # convolution reads u and e, and its data gradient writes gu and ge
        b = dict(xb=t(n1, 1), a1=t(n1, 16), e1=t(n1, 16), u1=t(n1, 16), a5=t(n1, 16),
                 d1=t(n1, 16), p1=t(n2, 16), a2=t(n2, 32), e2=t(n2, 32), u2=t(n2, 32),
                 a4=t(n2, 32), d2=t(n2, 32), p2=t(n3, 32), a3=t(n3, 64), b3=t(n3, 64))
        if train:
            b.update(g1a=t(n1, 16), g1b=t(n1, 16), gu1=t(n1, 16), ge1=t(n1, 16),
                     g2a=t(n2, 32), g2b=t(n2, 32), gu2=t(n2, 32), ge2=t(n2, 32), gp1=t(n2, 16),
                     g3a=t(n3, 64), g3b=t(n3, 64), gp2=t(n3, 32),
                     dout=torch.empty(n1, dtype=torch.float32, device=self.device))
        # inference and training share nothing; keep the most recent of each
        self._bufs = {k: v for k, v in self._bufs.items() if k[1] != train}
        self._bufs[key] = b
        if train:
            self._attach_scratch((D, H, W))
        return b

    def _attach_scratch(self, shape):
        """Attach the device scratch the gradient and loss calls need at this
        volume shape (the maximum over the layers' needs)."""
        D, H, W = shape
        need = 0
        for name, kind, cin, cout in LAYERS:
            lv = _LEVEL[name]
            n = (D >> (lv - 1)) * (H >> (lv - 1)) * (W >> (lv - 1))
            sz = ctypes.c_size_t(0)
            check(self._ctx, _lib.lib().ctrex_nn_scratch_bytes(cin, cout, n, ctypes.byref(sz)))
            need = max(need, int(sz.value))
        self._grow_scratch(need)

    def _grow_scratch(self, need):
        """Attach at least ``need`` bytes of device scratch to the context."""
        if getattr(self, "_scr", None) is None or self._scr.numel() < need:
            check(self._ctx, _lib.lib().ctrex_set_scratch(self._ctx, None, 0))
            self._scr = None
            self._scr = torch.empty(need, dtype=torch.uint8, device=self.device)
            check(self._ctx, _lib.lib().ctrex_set_scratch(
                self._ctx, ctypes.c_void_p(self._scr.data_ptr()), need))

    @staticmethod
    def check_shape(shape):
        D, H, W = (int(s) for s in shape)
        if D % 4 or H % 4 or W % 4:
            raise ValueError("volume sides must be multiples of 4, got %s" % (shape,))
        if (D * H * W) % 4096:
            raise ValueError("D*H*W must be a multiple of 4096 (64 voxels at the coarsest level)")
        return D, H, W

    # -------------------------------------------------------------- forward
    def _conv(self, name, src, s_cs, s_off, dst, d_cs, d_off, dims, relu=True):
        kind, cin, cout = _KIND[name]
        D, H, W = dims
        self._call("ctrex_nn_conv3", _vp(src), s_cs, s_off, cin, _vp(self._wt[name]),
                   _vp(self.p(name + ".b")), _vp(dst), d_cs, d_off, cout, D, H, W,
                   _lib.NN_RELU if relu else 0, self._s())

    def _conv_cat(self, name, ua, ea, dst, dims):
        """Decoder convolution of the concatenation [ua | ea] (equal halves)."""
        kind, cin, cout = _KIND[name]
        D, H, W = dims
        h = cin // 2
        self._call("ctrex_nn_conv3_cat", _vp(ua), h, 0, h, _vp(ea), h, 0, h,
                   _vp(self._wt[name]), _vp(self.p(name + ".b")), _vp(dst), cout, 0, cout, None,
                   0, 0, 0, None, 0, 0, D, H, W, _lib.NN_RELU, self._s())

    def _up(self, name, src, dst, d_cs, d_off, dims):
        kind, cin, cout = _KIND[name]
        D, H, W = dims
        self._call("ctrex_nn_upconv2", _vp(src), cin, 0, cin, _vp(self._wt[name]),
                   _vp(self.p(name + ".b")), _vp(dst), d_cs, d_off, cout, D, H, W, 0, self._s())

    def _pool(self, src, cs, off, c, dst, dims):
        D, H, W = dims
        self._call("ctrex_nn_maxpool2", _vp(src), cs, off, c, _vp(dst), D, H, W, self._s())

    def forward(self, x, out=None, train=False, mask=None, keep_acts=False):
        """x + m U(s x) / s for a float32 volume ``x`` [D][H][W] on the device;
        ``mask``: optional float32 weights m of the same shape.  The last
        decoder activations are stored only with ``train`` or ``keep_acts``."""
        if x.dtype != torch.float32 or x.device != self.device or not x.is_contiguous():
            raise ValueError("x must be a contiguous float32 tensor on %s" % self.device)
        if mask is not None and (mask.dtype != torch.float32 or mask.shape != x.shape or
                                 mask.device != self.device or not mask.is_contiguous()):
            raise ValueError("mask must be a contiguous float32 tensor shaped like x")
        D, H, W = self.check_shape(x.shape)
        l1, l2, l3 = (D, H, W), (D // 2, H // 2, W // 2), (D // 4, H // 4, W // 4)
        b = self._buffers((D, H, W), train)
        n1 = D * H * W
        self._call("ctrex_nn_input", _vp(x), self.scale, _vp(b["xb"]), n1, self._s())
        self._conv("e1a", b["xb"], 1, 0, b["a1"], 16, 0, l1)
        self._conv("e1b", b["a1"], 16, 0, b["e1"], 16, 0, l1)
        self._pool(b["e1"], 16, 0, 16, b["p1"], l1)
        self._conv("e2a", b["p1"], 16, 0, b["a2"], 32, 0, l2)
        self._conv("e2b", b["a2"], 32, 0, b["e2"], 32, 0, l2)
        self._pool(b["e2"], 32, 0, 32, b["p2"], l2)
        self._conv("bna", b["p2"], 32, 0, b["a3"], 64, 0, l3)
        self._conv("bnb", b["a3"], 64, 0, b["b3"], 64, 0, l3)
        self._up("up2", b["b3"], b["u2"], 32, 0, l3)
        self._conv_cat("d2a", b["u2"], b["e2"], b["a4"], l2)
        self._conv("d2b", b["a4"], 32, 0, b["d2"], 32, 0, l2)
        self._up("up1", b["d2"], b["u1"], 16, 0, l2)
        self._conv_cat("d1a", b["u1"], b["e1"], b["a5"], l1)
        if out is None:
            out = torch.empty_like(x)
        # the last convolution with the head folded in; its activations are
        # stored only for the backward pass and activations()
        keep = train or keep_acts
        self._call("ctrex_nn_conv3_head", _vp(b["a5"]), 16, 0, _vp(self._wt["d1b"]),
                   _vp(self.p("d1b.b")), _vp(b["d1"]) if keep else None, 16, 0,
                   _vp(self.p("head.w")), _vp(self.p("head.b")), _vp(x), 1.0 / self.scale,
                   _vp(mask) if mask is not None else None, _vp(out), D, H, W, self._s())
        self._saved = (b, (l1, l2, l3), mask) if train else None
        return out

    def activations(self, x):
        """Run the forward pass and return the BF16 activations by name
        (channels-last [.., C] views), for inspection and tests."""
        self.forward(x, train=False, keep_acts=True)
        D, H, W = x.shape
        b = self._buffers((D, H, W), False)
        dims = {1: (D, H, W), 2: (D // 2, H // 2, W // 2), 3: (D // 4, H // 4, W // 4)}
        lay = dict(xb=(1, 1), a1=(1, 16), e1=(1, 16), u1=(1, 16), a5=(1, 16), d1=(1, 16),
                   p1=(2, 16), a2=(2, 32), e2=(2, 32), u2=(2, 32), a4=(2, 32), d2=(2, 32),
                   p2=(3, 32), a3=(3, 64), b3=(3, 64))
        return {k: b[k].view(*dims[lv], c) for k, (lv, c) in lay.items()}

    def capture_forward(self, x, out, mask=None):
        """The inference forward pass on ``x`` into ``out`` (and ``mask``), at
        their present addresses, captured once as a HIP graph: the returned
        object's ``replay()`` launches all of its kernels with one call on the
        current stream, without the host round trip per kernel.  Replays read
        the current parameters (biases in place, packed weights rewritten in
        place by every optimizer step) and the present contents of ``x`` and
        ``mask``; a change of the input scale needs a new capture."""
        self.forward(x, out=out, mask=mask)   # buffers and packings exist
        torch.cuda.synchronize(self.device)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.forward(x, out=out, mask=mask)
        return _ForwardGraph(self, g, (x, out, mask, self._buffers(tuple(x.shape), False),
                                       dict(self._wt)))

    # ------------------------------------------------------------- backward
    def _relu_bwd(self, y, g, cs, off, c, n):
        self._call("ctrex_nn_relu_backward", _vp(y), _vp(g), cs, off, c, n, self._s())

    def _wgrad(self, name, src, s_cs, s_off, dout, d_cs, d_off, dims):
        kind, cin, cout = _KIND[name]
        D, H, W = dims
        fn = "ctrex_nn_conv3_wgrad" if kind == "conv" else "ctrex_nn_upconv2_wgrad"
        self._call(fn, _vp(src), s_cs, s_off, cin, _vp(dout), d_cs, d_off, cout, D, H, W,
                   _vp(self.p(name + ".w", self.grad)), _vp(self.p(name + ".b", self.grad)),
                   self._s())

    def _wgrad_cat(self, name, ua, ea, dout, d_cs, dims):
        kind, cin, cout = _KIND[name]
        D, H, W = dims
        h = cin // 2
        self._call("ctrex_nn_conv3_wgrad_cat", _vp(ua), h, 0, h, _vp(ea), h, 0, h, _vp(dout),
                   d_cs, 0, cout, D, H, W, _vp(self.p(name + ".w", self.grad)),
                   _vp(self.p(name + ".b", self.grad)), self._s())

    def _dgrad_cat(self, name, dout, d_cs, gu, ge, dims):
        """Data gradient of a decoder convolution, split into the gradients of
        its two inputs (the up-sampled and the skip features)."""
        kind, cin, cout = _KIND[name]
        D, H, W = dims
        h = cin // 2
        self._call("ctrex_nn_conv3_cat", _vp(dout), d_cs, 0, cout, None, 0, 0, 0,
                   _vp(self._wd[name]), None, _vp(gu), h, 0, h, _vp(ge), h, 0, h, None, 0, 0, D, H,
                   W, 0, self._s())

    def _dgrad(self, name, dout, d_cs, d_off, dst, o_cs, o_off, dims, relu_of=None):
        """Data gradient of a convolution: the convolution with the mirrored,
        transposed packing (cin and cout swap roles).  ``relu_of``: the ReLU
        output (channels-last, cin channels) that the layer's input is; its
        derivative is applied in the same pass, giving the gradient at the
        producing layer's pre-activation."""
        kind, cin, cout = _KIND[name]
        D, H, W = dims
        if relu_of is None:
            self._call("ctrex_nn_conv3", _vp(dout), d_cs, d_off, cout, _vp(self._wd[name]), None,
                       _vp(dst), o_cs, o_off, cin, D, H, W, 0, self._s())
            return
        self._call("ctrex_nn_conv3_cat", _vp(dout), d_cs, d_off, cout, None, 0, 0, 0,
                   _vp(self._wd[name]), None, _vp(dst), o_cs, o_off, cin, None, 0, 0, 0,
                   _vp(relu_of), cin, 0, D, H, W, 0, self._s())

    def backward(self, dout):
        """Gradients of every parameter given d loss / d out (float32 [D][H][W]);
        needs the preceding ``forward(..., train=True)``.  Overwrites ``grad``."""
        if self._saved is None:
            raise RuntimeError("backward needs a forward pass with train=True")
        b, (l1, l2, l3), mask = self._saved
        n1 = l1[0] * l1[1] * l1[2]
        n2, n3 = n1 // 8, n1 // 64
        g = self.grad
        # head and decoder level 1
        # each ReLU's derivative is applied by the call producing its gradient
        self._call("ctrex_nn_head_relu_backward", _vp(b["d1"]), 16, _vp(self.p("head.w")),
                   1.0 / self.scale, _vp(mask) if mask is not None else None, _vp(dout),
                   _vp(b["g1a"]), _vp(self.p("head.w", g)), _vp(self.p("head.b", g)), n1,
                   self._s())
        self._wgrad("d1b", b["a5"], 16, 0, b["g1a"], 16, 0, l1)
        self._dgrad("d1b", b["g1a"], 16, 0, b["g1b"], 16, 0, l1, relu_of=b["a5"])
        self._wgrad_cat("d1a", b["u1"], b["e1"], b["g1b"], 16, l1)
        self._dgrad_cat("d1a", b["g1b"], 16, b["gu1"], b["ge1"], l1)
        # up-sampling 1 and decoder level 2
        self._wgrad("up1", b["d2"], 32, 0, b["gu1"], 16, 0, l2)
        self._call("ctrex_nn_upconv2_dgrad", _vp(b["gu1"]), 16, 0, 16, _vp(self._wd["up1"]),
                   _vp(b["g2a"]), 32, 0, 32, l2[0], l2[1], l2[2], 0, self._s())
        self._relu_bwd(b["d2"], b["g2a"], 32, 0, 32, n2)
        self._wgrad("d2b", b["a4"], 32, 0, b["g2a"], 32, 0, l2)
        self._dgrad("d2b", b["g2a"], 32, 0, b["g2b"], 32, 0, l2, relu_of=b["a4"])
        self._wgrad_cat("d2a", b["u2"], b["e2"], b["g2b"], 32, l2)
        self._dgrad_cat("d2a", b["g2b"], 32, b["gu2"], b["ge2"], l2)
        # up-sampling 2 and the bottom level
        self._wgrad("up2", b["b3"], 64, 0, b["gu2"], 32, 0, l3)
        self._call("ctrex_nn_upconv2_dgrad", _vp(b["gu2"]), 32, 0, 32, _vp(self._wd["up2"]),
                   _vp(b["g3a"]), 64, 0, 64, l3[0], l3[1], l3[2], 0, self._s())
        self._relu_bwd(b["b3"], b["g3a"], 64, 0, 64, n3)
        self._wgrad("bnb", b["a3"], 64, 0, b["g3a"], 64, 0, l3)
        self._dgrad("bnb", b["g3a"], 64, 0, b["g3b"], 64, 0, l3, relu_of=b["a3"])
        self._wgrad("bna", b["p2"], 32, 0, b["g3b"], 64, 0, l3)
        self._dgrad("bna", b["g3b"], 64, 0, b["gp2"], 32, 0, l3)
        # encoder level 2: pooled gradient joins the skip gradient in place
        self._call("ctrex_nn_maxpool2_relu_backward", _vp(b["e2"]), 32, 0, 32, _vp(b["gp2"]),
                   _vp(b["ge2"]), l2[0], l2[1], l2[2], self._s())
        self._wgrad("e2b", b["a2"], 32, 0, b["ge2"], 32, 0, l2)
        self._dgrad("e2b", b["ge2"], 32, 0, b["g2a"], 32, 0, l2, relu_of=b["a2"])
        self._wgrad("e2a", b["p1"], 16, 0, b["g2a"], 32, 0, l2)
        self._dgrad("e2a", b["g2a"], 32, 0, b["gp1"], 16, 0, l2)
        # encoder level 1
        self._call("ctrex_nn_maxpool2_relu_backward", _vp(b["e1"]), 16, 0, 16, _vp(b["gp1"]),
                   _vp(b["ge1"]), l1[0], l1[1], l1[2], self._s())
        self._wgrad("e1b", b["a1"], 16, 0, b["ge1"], 16, 0, l1)
        self._dgrad("e1b", b["ge1"], 16, 0, b["g1a"], 16, 0, l1, relu_of=b["a1"])
        self._wgrad("e1a", b["xb"], 1, 0, b["g1a"], 16, 0, l1)
        return self.grad

    # ------------------------------------------------------------- training
    def mse(self, a, t, grad=None, weight=1.0):
        """weight x mean squared error (FP64 sum), optionally its gradient into ``grad``."""
        loss = ctypes.c_double()
        sz = ctypes.c_size_t(0)
        check(self._ctx, _lib.lib().ctrex_nn_scratch_bytes(1, 16, 1, ctypes.byref(sz)))
        self._grow_scratch(int(sz.value))
        self._call("ctrex_nn_mse", _vp(a), _vp(t), a.numel(), float(weight), ctypes.byref(loss),
                   _vp(grad) if grad is not None else None, self._s())
        return loss.value

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        self._call("ctrex_nn_adam", _vp(self.theta), _vp(self.grad), _vp(self.m), _vp(self.v),
                   self.n_params, lr, beta1, beta2, eps, self.step, self._s())
        self._pack()

    def train_step(self, x, target, lr=1e-3, mask=None):
        """One Adam step on s^2 MSE(x + m U(s x) / s, target), the error in the
        network's own units; returns that loss before the step."""
        out = self.forward(x, train=True, mask=mask)
        b = self._saved[0]
        loss = self.mse(out, target, grad=b["dout"], weight=self.scale ** 2)
        self.backward(b["dout"].view_as(x))
        self.adam(lr)
        return loss


class _ForwardGraph:
    """A captured U-Net forward pass (see UNet.capture_forward); it keeps the
    tensors the graph reads and writes alive."""

    def __init__(self, net, graph, keep):
        self._net, self._graph, self._keep, self._scale = net, graph, keep, net.scale

    def replay(self):
        if self._net.scale != self._scale:
            raise RuntimeError("the input scale changed since the capture; capture again")
        self._graph.replay()
