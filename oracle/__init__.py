"""CPU FP64 oracle — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It is independent of the HIP library:
no shared kernels, headers, helpers or constants, and neither imports the
other.  The projector pair lives in plain C (``ctrex_oracle.c``, FP64); this
module adds the parts that are compositions of it:

* the SIRT iteration of Eq. (1): x_{k+1} = x_k + alpha C A^T R (b - A x_k), with
  R = 1 / (A 1) and C = 1 / (A^T 1) (zero where the sums are zero), x_0 = 0,
  and its ordered-subset form (Sec. 2.3.2), one update per subset of views;
* the total-variation term and its gradient, the least-squares loss, PSNR.

Functions take numpy arrays; geometry is a [n_proj][n_sub][3][4] float64 array
of view matrices (see ``synth.trajectories`` for the conventions).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ctrex_oracle.c")
_LIB = os.path.join(_HERE, "libctrex_oracle.so")
_lock = threading.Lock()
_lib = None

OK, EINVAL, ESINGULAR, ESOURCE_INSIDE = 0, -1, -3, -4


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__({EINVAL: "invalid argument", ESINGULAR: "singular view matrix",
                          ESOURCE_INSIDE: "source inside the volume hull"}.get(code, str(code)))
        self.code = code


def build(force=True):
    """Compile the C oracle (gcc, FP64, no fused multiply-add contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                           "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            lib = ctypes.CDLL(_LIB)
            dp = ctypes.POINTER(ctypes.c_double)
            ip = ctypes.POINTER(ctypes.c_int)
            i = ctypes.c_int
            lib.oracle_forward.argtypes = [dp, i, i, i, i, i, i, i, ctypes.c_double, dp, ip, i,
                                           dp, i, i, i, dp, dp, ctypes.POINTER(ctypes.c_int64)]
            lib.oracle_back.argtypes = [dp, i, i, i, i, i, i, i, ctypes.c_double, dp, ip, i,
                                        dp, i, i, i, dp, dp]
            lib.oracle_forward_indicator.argtypes = [dp, i, i, i, i, i, i, i, ctypes.c_double,
                                                     dp, dp, dp]
            lib.oracle_back_voxel.argtypes = [dp, i, i, i, i, i, i, i, dp, ip, i, dp]
            lib.oracle_back_voxel_points.argtypes = [dp, i, i, i, i, i, i, i, dp, ip, i, ip, i,
                                                     dp]
            d = ctypes.c_double
            lib.oracle_forward_cyl.argtypes = [dp, i, i, i, i, i, i, i, d, d, dp, d, dp, ip, i,
                                               dp, ctypes.POINTER(ctypes.c_int64)]
            lib.oracle_back_voxel_cyl.argtypes = [dp, i, i, i, i, i, i, i, d, d, dp, dp, ip, i,
                                                  dp]
            lib.oracle_num_threads.restype = i
            _lib = lib
    return _lib


def num_threads():
    return _load().oracle_num_threads()


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _views(views, n_proj):
    if views is None:
        return None, n_proj
    v = np.ascontiguousarray(views, dtype=np.int32)
    return v, len(v)


def _geom(P):
    P = _f64(P)
    if P.ndim == 3:
        P = P[:, None]
    return P, P.shape[0], P.shape[1]


def forward(P, shape, n_u, n_v, vol, step=0.5, views=None, U=None, tau=None, return_count=False):
    """y = A x, float64 [n_views][n_v][n_u] (Sec. 4.1 projection operator)."""
    P, n_proj, n_sub = _geom(P)
    nz, ny, nx = shape
    vol = _f64(vol).reshape(shape)
    v, nvw = _views(views, n_proj)
    U = _f64(U)
    tau = _f64(tau)
    g = U.shape[:3] if U is not None else (0, 0, 0)
    out = np.zeros((nvw, n_v, n_u))
    cnt = ctypes.c_int64(0)
    st = _load().oracle_forward(
        _dp(P), n_proj, n_sub, n_u, n_v, nx, ny, nz, float(step), _dp(vol),
        v.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if v is not None else None, nvw,
        _dp(U), g[2], g[1], g[0], _dp(tau), _dp(out), ctypes.byref(cnt))
    if st != OK:
        raise OracleError(st)
    return (out, cnt.value) if return_count else out


def back(P, shape, n_u, n_v, sino, step=0.5, views=None, U=None, tau=None):
    """x = A^T y, float64 [nz][ny][nx]: the exact transpose of ``forward``."""
    P, n_proj, n_sub = _geom(P)
    nz, ny, nx = shape
    v, nvw = _views(views, n_proj)
    sino = _f64(sino).reshape(nvw, n_v, n_u)
    U = _f64(U)
    tau = _f64(tau)
    g = U.shape[:3] if U is not None else (0, 0, 0)
    out = np.zeros(shape)
    st = _load().oracle_back(
        _dp(P), n_proj, n_sub, n_u, n_v, nx, ny, nz, float(step), _dp(sino),
        v.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if v is not None else None, nvw,
        _dp(U), g[2], g[1], g[0], _dp(tau), _dp(out))
    if st != OK:
        raise OracleError(st)
    return out


def back_voxel(P, shape, n_u, n_v, sino, views=None):
    """z = B y, float64 [nz][ny][nx]: the paper's voxel-driven backprojector
    (Sec. 4.1), each voxel centre projected onto every listed detector image
    and the image sampled bilinearly (zero outside), sub-views averaged."""
    P, n_proj, n_sub = _geom(P)
    nz, ny, nx = shape
    v, nvw = _views(views, n_proj)
    sino = _f64(sino).reshape(nvw, n_v, n_u)
    out = np.zeros(shape)
    st = _load().oracle_back_voxel(
        _dp(P), n_proj, n_sub, n_u, n_v, nx, ny, nz, _dp(sino),
        v.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if v is not None else None, nvw, _dp(out))
    if st != OK:
        raise OracleError(st)
    return out


def back_voxel_points(P, shape, n_u, n_v, sino, ijk, views=None):
    """``back_voxel`` at the voxels ``ijk`` ([n][3] (ix, iy, iz)) only."""
    P, n_proj, n_sub = _geom(P)
    nz, ny, nx = shape
    v, nvw = _views(views, n_proj)
    sino = _f64(sino).reshape(nvw, n_v, n_u)
    ijk = np.ascontiguousarray(np.asarray(ijk, dtype=np.int32).reshape(-1, 3))
    out = np.zeros(ijk.shape[0])
    st = _load().oracle_back_voxel_points(
        _dp(P), n_proj, n_sub, n_u, n_v, nx, ny, nz, _dp(sino),
        v.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if v is not None else None, nvw,
        ijk.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ijk.shape[0], _dp(out))
    if st != OK:
        raise OracleError(st)
    return out


def _pose(pose):
    if pose is None:
        return None
    pose = np.ascontiguousarray(pose, dtype=np.float64).reshape(3, 4)
    return pose


def forward_cyl(P, cyl, n_u, n_v, vol, step=0.5, views=None, pose=None, return_count=False):
    """y = A_cyl x, float64 [n_views][n_v][n_u]: the projector on the aligned
    cylindrical domain (Sec. 3.5, 4.2.1).  ``cyl`` = (n_r, n_phi, n_z, dr, dz);
    ``vol`` [n_z][n_phi][n_r]; ``pose`` an optional rigid 3x4 [R | t] taking V-frame
    points to the cylinder frame."""
    P, n_proj, n_sub = _geom(P)
    n_r, n_phi, n_z, dr, dz = cyl
    vol = _f64(vol).reshape(n_z, n_phi, n_r)
    v, nvw = _views(views, n_proj)
    out = np.zeros((nvw, n_v, n_u))
    cnt = ctypes.c_int64(0)
    pz = _pose(pose)
    st = _load().oracle_forward_cyl(
        _dp(P), n_proj, n_sub, n_u, n_v, int(n_r), int(n_phi), int(n_z), float(dr), float(dz),
        _dp(pz), float(step), _dp(vol),
        v.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if v is not None else None, nvw,
        _dp(out), ctypes.byref(cnt))
    if st != OK:
        raise OracleError(st)
    return (out, int(cnt.value)) if return_count else out


def back_voxel_cyl(P, cyl, n_u, n_v, sino, views=None, pose=None):
    """z = B_cyl y, float64 [n_z][n_phi][n_r]: the voxel-driven backprojector
    over the polar voxels (Sec. 4.3.1): each voxel centre, mapped back to the
    V frame, is projected and the image sampled bilinearly."""
    P, n_proj, n_sub = _geom(P)
    n_r, n_phi, n_z, dr, dz = cyl
    v, nvw = _views(views, n_proj)
    sino = _f64(sino).reshape(nvw, n_v, n_u)
    out = np.zeros((int(n_z), int(n_phi), int(n_r)))
    pz = _pose(pose)
    st = _load().oracle_back_voxel_cyl(
        _dp(P), n_proj, n_sub, n_u, n_v, int(n_r), int(n_phi), int(n_z), float(dr), float(dz),
        _dp(pz), _dp(sino),
        v.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if v is not None else None, nvw, _dp(out))
    if st != OK:
        raise OracleError(st)
    return out


def sirt_cyl(P, cyl, n_u, n_v, b, n_iter, alpha=1.0, step=0.5, views=None, pose=None, x0=None):
    """Eq. (1) on the cylindrical domain with the voxel-driven backprojector:
    x <- x + alpha C B R (b - A x), R = 1 / (A 1), C = 1 / (B 1)."""
    n_r, n_phi, n_z = int(cyl[0]), int(cyl[1]), int(cyl[2])
    shape = (n_z, n_phi, n_r)
    Rw = _safe_recip(forward_cyl(P, cyl, n_u, n_v, np.ones(shape), step, views, pose))
    Cw = _safe_recip(back_voxel_cyl(P, cyl, n_u, n_v, np.ones_like(Rw), views, pose))
    b = _f64(b).reshape(Rw.shape)
    x = np.zeros(shape) if x0 is None else _f64(x0).reshape(shape).copy()
    norms = []
    for _ in range(n_iter):
        res = b - forward_cyl(P, cyl, n_u, n_v, x, step, views, pose)
        norms.append(float(np.sqrt(np.sum(res * res))))
        x = x + alpha * Cw * back_voxel_cyl(P, cyl, n_u, n_v, Rw * res, views, pose)
    return x, norms


def forward_indicator(P, shape, n_u, n_v, Q, centre_idx, step=0.5):
    """The forward sampler applied to the indicator of one ellipsoid."""
    P, n_proj, n_sub = _geom(P)
    nz, ny, nx = shape
    out = np.zeros((n_proj, n_v, n_u))
    st = _load().oracle_forward_indicator(_dp(P), n_proj, n_sub, n_u, n_v, nx, ny, nz,
                                          float(step), _dp(_f64(Q)), _dp(_f64(centre_idx)),
                                          _dp(out))
    if st != OK:
        raise OracleError(st)
    return out


def _safe_recip(a):
    out = np.zeros_like(a)
    pos = a > 0
    out[pos] = 1.0 / a[pos]
    return out


def _bp(voxel, P, shape, n_u, n_v, y, step, views, U, tau):
    if voxel:
        if U is not None:
            raise ValueError("the voxel-driven backprojector has no motion warp")
        return back_voxel(P, shape, n_u, n_v, y, views)
    return back(P, shape, n_u, n_v, y, step, views, U, tau)


def sirt_weights(P, shape, n_u, n_v, step=0.5, views=None, U=None, tau=None, voxel_bp=False):
    """R = 1 / (A 1) in detector space and C = 1 / (B 1) in voxel space, B the
    backprojector (A^T, or the voxel-driven one)."""
    ones_v = np.ones(shape)
    Rw = _safe_recip(forward(P, shape, n_u, n_v, ones_v, step, views, U, tau))
    ones_s = np.ones_like(Rw)
    Cw = _safe_recip(_bp(voxel_bp, P, shape, n_u, n_v, ones_s, step, views, U, tau))
    return Rw, Cw


def sirt(P, shape, n_u, n_v, b, n_iter, alpha=1.0, step=0.5, views=None, U=None, tau=None,
         x0=None, nonneg=False, weights=None, voxel_weights=None, voxel_bp=False):
    """Eq. (1) with a single subset: returns (x_n, [||b - A x_k||_2 for k < n]).

    ``voxel_weights`` (weighted backprojection, Sec. 3.2): w_j in [0, 1]
    scaling the correction voxel j receives, x <- x + alpha C w A^T R (b - A x).
    ``voxel_bp``: the paper's voxel-driven backprojector B in place of A^T
    (and C = 1 / (B 1)).
    """
    Rw, Cw = weights if weights is not None else sirt_weights(P, shape, n_u, n_v, step, views,
                                                              U, tau, voxel_bp)
    b = _f64(b).reshape(Rw.shape)
    x = np.zeros(shape) if x0 is None else _f64(x0).reshape(shape).copy()
    norms = []
    for _ in range(n_iter):
        res = b - forward(P, shape, n_u, n_v, x, step, views, U, tau)
        norms.append(float(np.sqrt(np.sum(res * res))))
        corr = _bp(voxel_bp, P, shape, n_u, n_v, Rw * res, step, views, U, tau)
        if voxel_weights is not None:
            corr = _f64(voxel_weights).reshape(shape) * corr
        x = x + alpha * Cw * corr
        if nonneg:
            x = np.maximum(x, 0.0)
    return x, norms


def os_sirt(P, shape, n_u, n_v, b, subsets, n_epochs, alpha=1.0, step=0.5, U=None, tau=None,
            x0=None, nonneg=False):
    """Ordered subsets (Sec. 2.3.2): each epoch applies Eq. (1) once per subset
    P_k in order, with R_k = 1 / (A_k 1) and C_k = 1 / (A_k^T 1) of that
    subset.  ``b`` holds all projections; returns (x, [[||b_k - A_k x|| per
    subset] per epoch])."""
    b = _f64(b)
    x = np.zeros(shape) if x0 is None else _f64(x0).reshape(shape).copy()
    weights = [sirt_weights(P, shape, n_u, n_v, step, list(s), U, tau) for s in subsets]
    norms = []
    for _ in range(n_epochs):
        row = []
        for s, w in zip(subsets, weights):
            x, nk = sirt(P, shape, n_u, n_v, b[list(s)], 1, alpha, step, list(s), U, tau, x0=x,
                         nonneg=nonneg, weights=w)
            row.append(nk[0])
        norms.append(row)
    return x, norms


def _forward_diffs(x):
    dx = np.zeros_like(x)
    dy = np.zeros_like(x)
    dz = np.zeros_like(x)
    dx[:, :, :-1] = x[:, :, 1:] - x[:, :, :-1]
    dy[:, :-1, :] = x[:, 1:, :] - x[:, :-1, :]
    dz[:-1, :, :] = x[1:, :, :] - x[:-1, :, :]
    return dx, dy, dz


def tv(x, eps=1e-5):
    """Isotropic TV: sum_j sqrt(|grad+ x_j|^2 + eps^2), forward differences with a
    zero difference at the last index of each axis."""
    x = _f64(x)
    dx, dy, dz = _forward_diffs(x)
    return float(np.sum(np.sqrt(dx * dx + dy * dy + dz * dz + eps * eps)))


def tv_grad(x, eps=1e-5):
    """Gradient of ``tv`` with respect to every voxel."""
    x = _f64(x)
    dx, dy, dz = _forward_diffs(x)
    m = np.sqrt(dx * dx + dy * dy + dz * dz + eps * eps)
    g = -(dx + dy + dz) / m
    g[:, :, 1:] += (dx / m)[:, :, :-1]
    g[:, 1:, :] += (dy / m)[:, :-1, :]
    g[1:, :, :] += (dz / m)[:-1, :, :]
    return g


def psnr(x, x_true, mask=None):
    """10 log10(range^2 / MSE) with range = max - min of x_true, MSE in ``mask``."""
    x = _f64(x)
    t = _f64(x_true)
    rng = float(t.max() - t.min())
    d = (x - t) if mask is None else (x - t)[mask]
    mse = float(np.mean(d * d))
    return float("inf") if mse == 0 else 10.0 * np.log10(rng * rng / mse)
