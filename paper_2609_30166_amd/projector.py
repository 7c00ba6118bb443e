"""Python binding of the projector library: argument marshalling only.

Every computation runs in libctrex's HIP kernels; torch tensors supply device
memory and the current HIP stream.  Layouts: volumes [nz][ny][nx], sinograms
[n_views][n_v][n_u], view matrices [n_proj][n_sub][3][4] float64 (see
include/ctrex.h for the conventions).
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check

_DT = {torch.float32: _lib.F32, torch.bfloat16: _lib.BF16, torch.float16: _lib.F16}
_GATHER_FLAG = {torch.float32: 0, torch.bfloat16: _lib.BF16_GATHER,
                torch.float16: _lib.F16_GATHER}


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _views_arg(views):
    if views is None:
        return None, 0, None
    arr = np.ascontiguousarray(np.asarray(views, dtype=np.int32).ravel())
    return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(arr.size), arr


class Geometry:
    """A projector context: per-projection view matrices, detector and volume.

    ``P``: [n_proj][n_sub][3][4] (or [n_proj][3][4]) float64 view matrices;
    ``shape``: (nz, ny, nx); ``step``: ray-march step in voxels.
    ``U``/``tau``: optional displacement grid [gz][gy][gx][3] and time
    fractions [n_proj][n_sub] of the warp applied during ray traversal.
    """

    def __init__(self, P, n_u, n_v, shape, step=0.5, device=None, U=None, tau=None):
        P = np.ascontiguousarray(P, dtype=np.float64)
        if P.ndim == 3:
            P = P[:, None]
        if P.ndim != 4 or P.shape[2:] != (3, 4):
            raise ValueError("view matrices must be [n_proj][n_sub][3][4]")
        self.P = P
        self.n_proj, self.n_sub = P.shape[:2]
        self.n_u, self.n_v = int(n_u), int(n_v)
        self.shape = tuple(int(s) for s in shape)
        self.step = float(step)
        dev = torch.device(device if device is not None else "cuda")
        if dev.type != "cuda":
            raise ValueError("the projector runs on a HIP device")
        self.device = torch.device("cuda", dev.index if dev.index is not None
                                   else torch.cuda.current_device())
        self._ctx = ctypes.c_void_p()
        L = _lib.lib()
        code = L.ctrex_create(ctypes.byref(self._ctx), self.device.index)
        if code != _lib.OK:
            raise _lib.CtrexError(code, "ctrex_create failed on %s" % self.device)
        nz, ny, nx = self.shape
        check(self._ctx, L.ctrex_set_geometry(
            self._ctx, P.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), self.n_proj,
            self.n_sub, self.n_u, self.n_v, nx, ny, nz, self.step))
        self._U = None
        self._vw = None
        self._ws = {}
        self._scr = None
        if U is not None:
            self.set_motion(U, tau)

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

    # -------------------------------------------------------------- helpers
    def _check_tensor(self, t, shape, dtypes, name):
        if not isinstance(t, torch.Tensor):
            raise TypeError("%s must be a torch tensor" % name)
        if t.device != self.device:
            raise ValueError("%s is on %s, the projector on %s" % (name, t.device, self.device))
        if t.dtype not in dtypes:
            raise TypeError("%s has dtype %s (allowed: %s)" % (name, t.dtype, dtypes))
        if tuple(t.shape) != tuple(shape):
            raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)

    def _scratch(self, views=None):
        """Attach device scratch (a uint8 tensor this object owns) holding what
        the library's calls over ``views`` need; grown when a longer view list
        or a cylindrical domain needs more."""
        nv = 0 if views is None else self.n_views(views)
        n = ctypes.c_size_t(0)
        check(self._ctx, _lib.lib().ctrex_scratch_bytes(self._ctx, nv, ctypes.byref(n)))
        need = int(n.value)
        if self._scr is None or self._scr.numel() < need:
            check(self._ctx, _lib.lib().ctrex_set_scratch(self._ctx, None, 0))
            self._scr = None
            self._scr = torch.empty(need, dtype=torch.uint8, device=self.device)
            check(self._ctx, _lib.lib().ctrex_set_scratch(
                self._ctx, ctypes.c_void_p(self._scr.data_ptr()), need))

    def n_views(self, views):
        return self.n_proj if views is None else int(np.asarray(views).size)

    def sino_shape(self, views=None):
        return (self.n_views(views), self.n_v, self.n_u)

    # ------------------------------------------------------------- geometry
    def set_motion(self, U, tau):
        """Install (or with U=None remove) the displacement-field warp."""
        L = _lib.lib()
        if U is None:
            check(self._ctx, L.ctrex_set_motion(self._ctx, None, 0, 0, 0, None))
            self._U = None
            return
        U = torch.as_tensor(U, dtype=torch.float32, device=self.device).contiguous()
        if U.ndim != 4 or U.shape[3] != 3:
            raise ValueError("U must be [gz][gy][gx][3]")
        tau = np.ascontiguousarray(tau, dtype=np.float64).reshape(self.n_proj, self.n_sub)
        gz, gy, gx = U.shape[:3]
        check(self._ctx, L.ctrex_set_motion(self._ctx, ctypes.c_void_p(U.data_ptr()), gx, gy, gz,
                                            tau.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        self._U = U

    def set_voxel_weights(self, w):
        """Weighted backprojection (Sec. 3.2, 4.3.2): voxel weights w in [0, 1]
        scaling each voxel's correction in ``sirt``/``os_sirt``; None removes
        them.  The tensor is kept alive by this object while set."""
        L = _lib.lib()
        if w is None:
            check(self._ctx, L.ctrex_set_voxel_weights(self._ctx, None))
            self._vw = None
            return
        w = torch.as_tensor(w, dtype=torch.float32, device=self.device).contiguous()
        if tuple(w.shape) != self.shape:
            raise ValueError("weights must have the volume shape %s" % (self.shape,))
        check(self._ctx, L.ctrex_set_voxel_weights(self._ctx, ctypes.c_void_p(w.data_ptr())))
        self._vw = w

    # ------------------------------------------------------------ operators
    def forward(self, vol, views=None, out=None, out_dtype=torch.float32):
        """sino = A vol (Sec. 4.1 projection operator)."""
        self._check_tensor(vol, self.shape, _DT, "vol")
        shape = self.sino_shape(views)
        if out is None:
            out = torch.empty(shape, dtype=out_dtype, device=self.device)
        self._check_tensor(out, shape, _DT, "out")
        self._scratch(views)
        vp, nv, _keep = _views_arg(views)
        check(self._ctx, _lib.lib().ctrex_forward_project(
            self._ctx, ctypes.c_void_p(vol.data_ptr()), _DT[vol.dtype],
            ctypes.c_void_p(out.data_ptr()), _DT[out.dtype], vp, nv, _stream(self.device)))
        return out

    def back(self, sino, views=None, out=None, accumulate=False, scale=1.0):
        """vol (+)= scale A^T sino, the exact transpose of ``forward`` (the
        factor is applied inside the library's fixed-point sums)."""
        self._check_tensor(sino, self.sino_shape(views), _DT, "sino")
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
            accumulate = False
        self._check_tensor(out, self.shape, (torch.float32,), "out")
        self._scratch(views)
        vp, nv, _keep = _views_arg(views)
        if scale == 1.0:
            check(self._ctx, _lib.lib().ctrex_back_project(
                self._ctx, ctypes.c_void_p(sino.data_ptr()), _DT[sino.dtype],
                ctypes.c_void_p(out.data_ptr()), 1 if accumulate else 0, vp, nv,
                _stream(self.device)))
        else:
            check(self._ctx, _lib.lib().ctrex_back_project_scaled(
                self._ctx, ctypes.c_void_p(sino.data_ptr()), _DT[sino.dtype], float(scale),
                ctypes.c_void_p(out.data_ptr()), 1 if accumulate else 0, vp, nv,
                _stream(self.device)))
        return out

    def back_voxel(self, sino, views=None, out=None, accumulate=False):
        """vol (+)= B sino with the paper's voxel-driven backprojector (Sec. 4.1):
        voxel centres projected onto each image and sampled bilinearly; not the
        transpose of ``forward``.  No motion warp."""
        self._check_tensor(sino, self.sino_shape(views), _DT, "sino")
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
            accumulate = False
        self._check_tensor(out, self.shape, (torch.float32,), "out")
        vp, nv, _keep = _views_arg(views)
        check(self._ctx, _lib.lib().ctrex_back_project_voxel(
            self._ctx, ctypes.c_void_p(sino.data_ptr()), _DT[sino.dtype],
            ctypes.c_void_p(out.data_ptr()), 1 if accumulate else 0, vp, nv,
            _stream(self.device)))
        return out

    def workspace_bytes(self, views=None, gather_dtype=torch.float32):
        n = ctypes.c_size_t(0)
        nv = 0 if views is None else self.n_views(views)
        check(self._ctx, _lib.lib().ctrex_sirt_workspace_bytes(
            self._ctx, nv, _GATHER_FLAG[gather_dtype], ctypes.byref(n)))
        return int(n.value)

    def workspace(self, views=None, gather_dtype=torch.float32):
        """A caller-owned workspace buffer for ``sirt`` (uint8 tensor)."""
        return torch.empty(self.workspace_bytes(views, gather_dtype), dtype=torch.uint8,
                           device=self.device)

    def sirt(self, vol, sino, n_iter, alpha=1.0, nonneg=False, gather_dtype=torch.float32,
             views=None, workspace=None, norms=True, recompute_weights=False, voxel_bp=False):
        """Eq. (1): ``n_iter`` SIRT updates of ``vol`` (float32, in place).
        ``voxel_bp``: backproject with ``back_voxel``'s B (C = 1 / (B 1)).

        Returns the residual norms ||sino - A vol_k|| (numpy) when ``norms``,
        else None (and the call does not wait for the device).
        """
        self._check_tensor(vol, self.shape, (torch.float32,), "vol")
        self._check_tensor(sino, self.sino_shape(views), _DT, "sino")
        flags = _GATHER_FLAG[gather_dtype]
        if nonneg:
            flags |= _lib.NONNEG
        if recompute_weights:
            flags |= _lib.RECOMPUTE_WEIGHTS
        if voxel_bp:
            flags |= _lib.VOXEL_BP
        if workspace is None:
            # one workspace per view list, so ordered subsets keep their R and C
            key = (None if views is None else tuple(np.asarray(views).ravel().tolist()),
                   gather_dtype, bool(voxel_bp))
            workspace = self._ws.pop(key, None)
            if workspace is None:
                workspace = self.workspace(views, gather_dtype)
            self._ws[key] = workspace
            while len(self._ws) > 64:
                self._ws.pop(next(iter(self._ws)))
        self._scratch(views)
        vp, nv, _keep = _views_arg(views)
        out = np.zeros(max(int(n_iter), 0), dtype=np.float64) if norms else None
        check(self._ctx, _lib.lib().ctrex_sirt_iterate(
            self._ctx, ctypes.c_void_p(vol.data_ptr()), ctypes.c_void_p(sino.data_ptr()),
            _DT[sino.dtype], int(n_iter), float(alpha), flags, vp, nv,
            ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if norms else None,
            _stream(self.device)))
        return out

    def residual_norm(self, vol, sino, views=None):
        """||sino - A vol||_2 (FP64 sum, computed by the library; waits)."""
        self._check_tensor(vol, self.shape, _DT, "vol")
        self._check_tensor(sino, self.sino_shape(views), _DT, "sino")
        self._scratch(views)
        vp, nv, _keep = _views_arg(views)
        out = ctypes.c_double(0.0)
        check(self._ctx, _lib.lib().ctrex_residual_norm(
            self._ctx, ctypes.c_void_p(vol.data_ptr()), _DT[vol.dtype],
            ctypes.c_void_p(sino.data_ptr()), _DT[sino.dtype], vp, nv, ctypes.byref(out),
            _stream(self.device)))
        return out.value

    def data_residual(self, vol, b, views=None, scale=1.0, residual=True, sq_sum=True):
        """Data term of the loss (Eq. (1)'s residual): returns (r, s) with
        r = scale (A vol - b) in b's storage type (or None) and
        s = sum (A vol - b)^2 as a 0-d float64 device tensor (or None), both
        computed by the library's kernels, without a host wait."""
        self._check_tensor(vol, self.shape, _DT, "vol")
        self._check_tensor(b, self.sino_shape(views), _DT, "b")
        r = torch.empty_like(b) if residual else None
        s = torch.empty((), dtype=torch.float64, device=self.device) if sq_sum else None
        self._scratch(views)
        vp, nv, _keep = _views_arg(views)
        check(self._ctx, _lib.lib().ctrex_data_residual(
            self._ctx, ctypes.c_void_p(vol.data_ptr()), _DT[vol.dtype],
            ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(r.data_ptr()) if residual else None,
            _DT[b.dtype], float(scale), vp, nv,
            ctypes.c_void_p(s.data_ptr()) if sq_sum else None, _stream(self.device)))
        return r, s

    def os_sirt(self, vol, sino, subsets, n_epochs, alpha=1.0, nonneg=False,
                gather_dtype=torch.float32, norms=False, voxel_bp=False):
        """Ordered-subset SIRT (Sec. 2.3.2): each epoch applies Eq. (1) once per
        subset P_k of ``subsets`` (lists of projection indices), in order, with
        that subset's own R and C.  ``sino`` holds all projections
        [n_proj][n_v][n_u].  Returns, when ``norms``, the residual norm over
        each subset before its update, [n_epochs][n_subsets]."""
        subsets = [np.asarray(s, dtype=np.int32).ravel() for s in subsets]
        if not subsets or any(s.size == 0 for s in subsets):
            raise ValueError("subsets must be non-empty lists of projection indices")
        self._check_tensor(sino, self.sino_shape(), _DT, "sino")
        parts = getattr(self, "_os_parts", None)
        key = (sino.data_ptr(), tuple(tuple(s.tolist()) for s in subsets))
        if parts is None or parts[0] != key:
            idx = [torch.as_tensor(s, dtype=torch.long, device=self.device) for s in subsets]
            parts = (key, [sino.index_select(0, i).contiguous() for i in idx])
            self._os_parts = parts
        out = np.zeros((int(n_epochs), len(subsets))) if norms else None
        for e in range(int(n_epochs)):
            for k, (s, b) in enumerate(zip(subsets, parts[1])):
                r = self.sirt(vol, b, 1, alpha=alpha, nonneg=nonneg, gather_dtype=gather_dtype,
                              views=s, norms=norms, voxel_bp=voxel_bp)
                if norms:
                    out[e, k] = r[0]
        return out

    def sample_count(self, views=None):
        """Exact number of trilinear samples of one forward projection."""
        cnt = ctypes.c_int64(0)
        vp, nv, _keep = _views_arg(views)
        check(self._ctx, _lib.lib().ctrex_sample_count(self._ctx, vp, nv, ctypes.byref(cnt),
                                                       _stream(self.device)))
        return int(cnt.value)

    def profile(self, enable=True):
        """Start (or stop) recording kernel times inside ``sirt``."""
        check(self._ctx, _lib.lib().ctrex_profile_enable(self._ctx, 1 if enable else 0))

    def profile_read(self):
        """{phase: (total_ms, launches)} for 'forward', 'back', 'update' since the
        last read (waits for the device)."""
        ms = (ctypes.c_double * 3)()
        n = (ctypes.c_int64 * 3)()
        check(self._ctx, _lib.lib().ctrex_profile_read(self._ctx, ms, n))
        return {k: (ms[i], n[i]) for i, k in enumerate(("forward", "back", "update"))}

    def tv(self, x, eps=1e-5, weight=1.0, value=True, grad=False):
        """Total variation of a float32 volume: returns (TV(x) or None,
        weight * dTV/dx or None), both computed by the library's kernels."""
        if x.dtype != torch.float32 or not x.is_contiguous() or x.ndim != 3:
            raise ValueError("x must be a contiguous float32 [nz][ny][nx] tensor")
        if x.device != self.device:
            raise ValueError("x is on %s, the projector on %s" % (x.device, self.device))
        nz, ny, nx = x.shape
        g = torch.empty_like(x) if grad else None
        v = ctypes.c_double(0.0)
        check(self._ctx, _lib.lib().ctrex_tv(
            self._ctx, ctypes.c_void_p(x.data_ptr()), nx, ny, nz, float(eps), float(weight),
            ctypes.byref(v) if value else None, ctypes.c_void_p(g.data_ptr()) if grad else None,
            _stream(self.device)))
        return (v.value if value else None), g

    def convert(self, src, dtype):
        """Storage conversion (round to nearest even) through the library."""
        out = torch.empty(src.shape, dtype=dtype, device=self.device)
        check(self._ctx, _lib.lib().ctrex_convert(
            self._ctx, ctypes.c_void_p(src.data_ptr()), _DT[src.dtype],
            ctypes.c_void_p(out.data_ptr()), _DT[dtype], src.numel(), _stream(self.device)))
        return out


def ordered_subsets(n_proj, n_subsets, order="interleaved", seed=0):
    """Partition of the projections 0..n_proj-1 into ``n_subsets`` subsets
    (Sec. 2.3.2): "interleaved" (subset k = every n_subsets-th projection from
    k, so each subset spans the whole orbit), "bitreversal" (the interleaved
    subsets visited in bit-reversed index order, so consecutive subsets sit
    far apart on the orbit: the geometry-ordered schedule of ART/OS methods),
    "contiguous" (consecutive blocks), or "random" (a seeded permutation cut
    into blocks).  The list order is the visiting order."""
    n_proj, n_subsets = int(n_proj), int(n_subsets)
    if not 1 <= n_subsets <= n_proj:
        raise ValueError("need 1 <= n_subsets <= n_proj")
    if order in ("interleaved", "bitreversal"):
        subs = [list(range(k, n_proj, n_subsets)) for k in range(n_subsets)]
        if order == "bitreversal":
            bits = max(1, (n_subsets - 1).bit_length())
            rev = lambda k: int(format(k, "0%db" % bits)[::-1], 2)
            subs = [subs[k] for k in sorted(range(n_subsets), key=rev)]
        return subs
    if order == "contiguous":
        base = np.arange(n_proj)
    elif order == "random":
        base = np.random.default_rng([seed, 31]).permutation(n_proj)
    else:
        raise ValueError("order must be interleaved, bitreversal, contiguous or random")
    return [sorted(int(v) for v in part) for part in np.array_split(base, n_subsets)]


class ForwardProject(torch.autograd.Function):
    """y = A x with the exact-transpose backprojector as its backward."""

    @staticmethod
    def forward(ctx, vol, geom, views=None):
        ctx.geom = geom
        ctx.views = views
        return geom.forward(vol.contiguous(), views)

    @staticmethod
    def backward(ctx, grad_y):
        grad_x = None
        if ctx.needs_input_grad[0]:
            grad_x = ctx.geom.back(grad_y.contiguous().to(torch.float32), ctx.views)
        return grad_x, None, None


def project(vol, geom, views=None):
    """Differentiable forward projection (autograd tape through the HIP pair)."""
    return ForwardProject.apply(vol, geom, views)


class TotalVariation(torch.autograd.Function):
    """TV(x) (FP64 value) with the library's gradient kernel as backward."""

    @staticmethod
    def forward(ctx, vol, geom, eps=1e-5):
        v, _ = geom.tv(vol.contiguous(), eps)
        ctx.geom = geom
        ctx.eps = eps
        ctx.save_for_backward(vol)
        return torch.tensor(v, dtype=torch.float64, device=vol.device)

    @staticmethod
    def backward(ctx, grad_out):
        (vol,) = ctx.saved_tensors
        _, g = ctx.geom.tv(vol.contiguous(), ctx.eps, weight=1.0, value=False, grad=True)
        return g * grad_out.to(torch.float32), None, None


def total_variation(vol, geom, eps=1e-5):
    return TotalVariation.apply(vol, geom, eps)


class DataTerm(torch.autograd.Function):
    """||A x - b||^2 (Eq. (1)'s data term, summed in FP64) with the gradient
    2 A^T (A x - b): the forward projection with the residual epilogue, and
    the exact-transpose backprojector scaled by 2 in the backward.  ``b`` is
    data (no gradient)."""

    @staticmethod
    def forward(ctx, vol, b, geom, views=None):
        r, s = geom.data_residual(vol.contiguous(), b.contiguous(), views)
        ctx.geom = geom
        ctx.views = views
        ctx.save_for_backward(r)
        return s

    @staticmethod
    def backward(ctx, grad_out):
        grad_x = None
        if ctx.needs_input_grad[0]:
            (r,) = ctx.saved_tensors
            grad_x = ctx.geom.back(r, ctx.views, scale=2.0 * float(grad_out))
        return grad_x, None, None, None


def data_term(vol, b, geom, views=None):
    """Differentiable ||A x - b||^2 through the library's residual and
    backprojection kernels."""
    return DataTerm.apply(vol, b, geom, views)


def reconstruction_loss(vol, b, geom, lam=1e-3, eps=1e-5, views=None):
    """||A x - b||^2 + lam TV(x), differentiable through the HIP operators:
    the data term and its gradient from ``DataTerm``, TV and its gradient
    from the library's TV kernels."""
    return data_term(vol, b, geom, views) + lam * total_variation(vol, geom, eps)
