"""Python binding of the aligned cylindrical domain (include/ctrex.h,
``ctrex_set_cylinder`` and the ``*_cyl`` calls): argument marshalling only.

The volume is a polar grid [n_z][n_phi][n_r] about the z axis of a cylinder
frame (ring i at (i + 1/2) dr, angle 2 pi j / n_phi, slice (k - (n_z - 1)/2)
dz); ``pose`` = [R | t] (3x4) maps V-frame points of the view matrices to
that frame (identity when None).  ``forward`` is the ray-driven projector
clipped to the cylinder, ``back`` the voxel-driven backprojector over the
polar voxel centres, ``sirt`` Eq. (1) with them.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check
from .projector import _DT, Geometry, _stream, _views_arg


class CylinderGeometry:
    """Projector context on the aligned cylindrical domain (Sec. 3.5, 4.2.1, 4.3.1)."""

    def __init__(self, P, n_u, n_v, n_r, n_phi, n_z, dr=1.0, dz=1.0, step=0.5, pose=None,
                 device=None):
        # the view matrices and step live in a plain context; its box sides are not used
        self._g = Geometry(P, n_u, n_v, (2, 2, 2), step, device=device)
        self.P, self.n_proj, self.n_sub = self._g.P, self._g.n_proj, self._g.n_sub
        self.n_u, self.n_v, self.step, self.device = n_u, n_v, float(step), self._g.device
        self.n_r, self.n_phi, self.n_z = int(n_r), int(n_phi), int(n_z)
        self.dr, self.dz = float(dr), float(dz)
        self.shape = (self.n_z, self.n_phi, self.n_r)
        self.pose = None if pose is None else np.ascontiguousarray(pose, np.float64).reshape(3, 4)
        check(self._ctx, _lib.lib().ctrex_set_cylinder(
            self._ctx, self.n_r, self.n_phi, self.n_z, self.dr, self.dz,
            None if self.pose is None else self.pose.ctypes.data_as(
                ctypes.POINTER(ctypes.c_double))))
        self._ws = {}

    @property
    def _ctx(self):
        return self._g._ctx

    def close(self):
        self._g.close()

    def sino_shape(self, views=None):
        return self._g.sino_shape(views)

    def set_motion(self, U, tau):
        self._g.set_motion(U, tau)

    def forward(self, vol, views=None, out=None, out_dtype=torch.float32):
        """sino = A_cyl vol."""
        self._g._check_tensor(vol, self.shape, _DT, "vol")
        shape = self.sino_shape(views)
        if out is None:
            out = torch.empty(shape, dtype=out_dtype, device=self.device)
        self._g._check_tensor(out, shape, _DT, "out")
        self._g._scratch(views)
        vp, nv, _keep = _views_arg(views)
        check(self._ctx, _lib.lib().ctrex_forward_project_cyl(
            self._ctx, ctypes.c_void_p(vol.data_ptr()), _DT[vol.dtype],
            ctypes.c_void_p(out.data_ptr()), _DT[out.dtype], vp, nv, _stream(self.device)))
        return out

    def back(self, sino, views=None, out=None, accumulate=False):
        """vol (+)= B_cyl sino (voxel-driven, over the polar voxel centres)."""
        self._g._check_tensor(sino, self.sino_shape(views), _DT, "sino")
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
            accumulate = False
        self._g._check_tensor(out, self.shape, (torch.float32,), "out")
        vp, nv, _keep = _views_arg(views)
        check(self._ctx, _lib.lib().ctrex_back_project_cyl(
            self._ctx, ctypes.c_void_p(sino.data_ptr()), _DT[sino.dtype],
            ctypes.c_void_p(out.data_ptr()), 1 if accumulate else 0, vp, nv,
            _stream(self.device)))
        return out

    def sample_count(self, views=None):
        cnt = ctypes.c_int64(0)
        vp, nv, _keep = _views_arg(views)
        check(self._ctx, _lib.lib().ctrex_sample_count_cyl(self._ctx, vp, nv, ctypes.byref(cnt),
                                                           _stream(self.device)))
        return int(cnt.value)

    def workspace(self, views=None):
        n = ctypes.c_size_t(0)
        nv = 0 if views is None else int(np.asarray(views).size)
        check(self._ctx, _lib.lib().ctrex_sirt_workspace_bytes_cyl(self._ctx, nv,
                                                                   ctypes.byref(n)))
        return torch.empty(int(n.value), dtype=torch.uint8, device=self.device)

    def sirt(self, vol, sino, n_iter, alpha=1.0, nonneg=False, views=None, workspace=None,
             norms=True, recompute_weights=False):
        """Eq. (1) on the cylinder: vol <- vol + alpha C B R (sino - A vol), in place."""
        self._g._check_tensor(vol, self.shape, (torch.float32,), "vol")
        self._g._check_tensor(sino, self.sino_shape(views), _DT, "sino")
        flags = (_lib.NONNEG if nonneg else 0) | (_lib.RECOMPUTE_WEIGHTS if recompute_weights
                                                  else 0)
        if workspace is None:
            key = None if views is None else tuple(np.asarray(views).ravel().tolist())
            workspace = self._ws.get(key)
            if workspace is None:
                workspace = self._ws[key] = self.workspace(views)
        self._g._scratch(views)
        vp, nv, _keep = _views_arg(views)
        out = np.zeros(max(int(n_iter), 0), dtype=np.float64) if norms else None
        check(self._ctx, _lib.lib().ctrex_sirt_iterate_cyl(
            self._ctx, ctypes.c_void_p(vol.data_ptr()), ctypes.c_void_p(sino.data_ptr()),
            _DT[sino.dtype], int(n_iter), float(alpha), flags, vp, nv,
            ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if norms else None,
            _stream(self.device)))
        return out

    def profile(self, enable=True):
        self._g.profile(enable)

    def profile_read(self):
        return self._g.profile_read()
