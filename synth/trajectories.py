"""Trajectories expressed as per-projection 3x4 view matrices (Sec. 2.2).

Frame and pixel conventions used throughout the project:

* The volume frame V is in voxel units and centred on the volume: the centre of
  voxel (ix, iy, iz) sits at X = (ix - (nx-1)/2, iy - (ny-1)/2, iz - (nz-1)/2).
* A view matrix P (3x4, float64, row-major) maps homogeneous V coordinates to
  homogeneous detector coordinates, P @ (X, 1) ~ (u, v, 1), where (u, v) are in
  pixel-index units: pixel (iu, iv) has its centre at (u, v) = (iu, iv) and u
  runs fastest in memory.  P is only defined up to a non-zero scale.
* A trajectory is an array [n_proj][n_sub][3][4]: n_sub >= 1 sub-views per
  projection model the angular integration during one exposure (Sec. 3.4).

Everything here builds inputs; nothing evaluates rays.
"""

from __future__ import annotations

import math

import numpy as np


def view_matrix(src, det_centre, e_u, e_v, pitch_u, pitch_v, n_u, n_v):
    """3x4 matrix of a point source and a flat detector, all in the V frame.

    ``src`` is the source position, ``det_centre`` the position of the
    detector's geometric centre (the point between the middle pixels), and
    ``e_u``/``e_v`` orthonormal unit vectors along increasing u and v.  A point X
    projects to the intersection of the line src->X with the detector plane;
    the returned matrix expresses that central projection in pixel indices.
    """
    s = np.asarray(src, dtype=np.float64)
    c = np.asarray(det_centre, dtype=np.float64)
    eu = np.asarray(e_u, dtype=np.float64)
    ev = np.asarray(e_v, dtype=np.float64)
    nrm = np.cross(eu, ev)
    depth = float(np.dot(c - s, nrm))  # signed source-to-plane distance
    if abs(depth) < 1e-12:
        raise ValueError("source lies in the detector plane")
    cu = 0.5 * (n_u - 1)
    cv = 0.5 * (n_v - 1)
    # For a = X - src the plane is hit at src + a * depth / (a . n), i.e. at
    # detector offset (s - c) + a * depth / (a . n); u, v are its coordinates.
    row_u = (np.dot(s - c, eu) * nrm + depth * eu) / pitch_u + cu * nrm
    row_v = (np.dot(s - c, ev) * nrm + depth * ev) / pitch_v + cv * nrm
    row_w = nrm
    M = np.stack([row_u, row_v, row_w])
    P = np.empty((3, 4), dtype=np.float64)
    P[:, :3] = M
    P[:, 3] = -M @ s
    return P


def _circular_view(theta, sod, sdd, pitch, n_u, n_v, z=0.0, off_u=0.0, off_v=0.0):
    ct, st = math.cos(theta), math.sin(theta)
    radial = np.array([ct, st, 0.0])
    e_u = np.array([-st, ct, 0.0])
    e_v = np.array([0.0, 0.0, 1.0])
    src = sod * radial + np.array([0.0, 0.0, z])
    det = (sod - sdd) * radial + np.array([0.0, 0.0, z]) + off_u * e_u + off_v * e_v
    return view_matrix(src, det, e_u, e_v, pitch, pitch, n_u, n_v)


def _sub_angles(n_proj, n_sub, arc, theta0):
    """Sub-view angles at the midpoints of equal parts of each exposure window."""
    dth = arc / n_proj
    p = np.arange(n_proj)[:, None]
    s = np.arange(n_sub)[None, :]
    return theta0 + dth * (p + (s + 0.5) / n_sub - 0.5)


def circular_cone(n_proj, n_u, n_v, sod, sdd, pitch, n_sub=1, arc=2 * math.pi,
                  theta0=0.0, det_offset_u=0.0, det_offset_v=0.0):
    """Circular cone-beam scan about the V z axis, [n_proj][n_sub][3][4].

    ``det_offset_u`` shifts the detector sideways (an offset-detector scan);
    with n_sub > 1 the sub-views sample each projection's exposure window.
    """
    ang = _sub_angles(n_proj, n_sub, arc, theta0)
    out = np.empty((n_proj, n_sub, 3, 4))
    for p in range(n_proj):
        for s in range(n_sub):
            out[p, s] = _circular_view(ang[p, s], sod, sdd, pitch, n_u, n_v,
                                       off_u=det_offset_u, off_v=det_offset_v)
    return out


def helical_cone(n_proj, n_u, n_v, sod, sdd, pitch, pitch_per_rad, total_angle,
                 n_sub=1, theta0=0.0):
    """Helical scan (Sec. 2.2.2): rotation alpha about z plus a z shift p*alpha.

    The z shift is centred so that the middle of the scan is at z = 0.
    ``pitch_per_rad`` is the translation per radian of rotation.
    """
    ang = _sub_angles(n_proj, n_sub, total_angle, theta0)
    mid = theta0 + 0.5 * total_angle
    out = np.empty((n_proj, n_sub, 3, 4))
    for p in range(n_proj):
        for s in range(n_sub):
            a = ang[p, s]
            out[p, s] = _circular_view(a, sod, sdd, pitch, n_u, n_v,
                                       z=pitch_per_rad * (a - mid))
    return out


def medical_pitch_per_rad(pitch, n_v, det_pitch, sod, sdd):
    """Table feed per radian for a medical pitch (feed per turn / z coverage)."""
    h_iso = n_v * det_pitch * sod / sdd
    return pitch * h_iso / (2 * math.pi)


def _euler_xyz(rx, ry, rz):
    cx, sx = math.cos(rx), math.sin(rx)
    cy, sy = math.cos(ry), math.sin(ry)
    cz, sz = math.cos(rz), math.sin(rz)
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def rigid_jitter(P, sigma_t, sigma_rot_deg, rng):
    """Compose a seeded rigid perturbation of the volume pose into each projection.

    Per projection: translation ~ N(0, sigma_t^2) per axis and XYZ Euler angles
    ~ N(0, sigma_rot^2).  The pose T = [[R, t], [0, 1]] is held constant over the
    projection's sub-views: P' = P @ T (Sec. 2.2.3, rigid part of the pose).
    """
    P = np.array(P, dtype=np.float64, copy=True)
    n_proj = P.shape[0]
    sr = math.radians(sigma_rot_deg)
    for p in range(n_proj):
        t = rng.normal(0.0, sigma_t, size=3)
        ang = rng.normal(0.0, sr, size=3)
        T = np.eye(4)
        T[:3, :3] = _euler_xyz(*ang)
        T[:3, 3] = t
        for s in range(P.shape[1]):
            P[p, s] = P[p, s] @ T
    return P


def conveyor_belt(n_proj, n_u, n_v, sod, sdd, pitch, travel, rotation, n_sub=1):
    """Fixed source/detector; the object slides along x by ``travel`` voxels in
    total while turning by ``rotation`` radians about z (Sec. 2.2.2).

    In the V frame this is P_lab @ [[R_z(a), (x(t), 0, 0)], [0, 1]].
    """
    P0 = _circular_view(0.0, sod, sdd, pitch, n_u, n_v)
    out = np.empty((n_proj, n_sub, 3, 4))
    for p in range(n_proj):
        for s in range(n_sub):
            f = (p + (s + 0.5) / n_sub) / n_proj
            T = np.eye(4)
            T[:3, :3] = _euler_xyz(0.0, 0.0, rotation * f)
            T[0, 3] = travel * (f - 0.5)
            out[p, s] = P0 @ T
    return out


def exposure_time_fractions(n_proj, n_sub):
    """Normalised acquisition time in [0, 1] of each sub-view, linear in angle."""
    p = np.arange(n_proj)[:, None]
    s = np.arange(n_sub)[None, :]
    return ((p + (s + 0.5) / n_sub) / n_proj).astype(np.float64)


def smooth_displacement(g, max_disp, rng, n_modes=4):
    """Smooth seeded displacement grid U[g][g][g][3] (float32, voxel units).

    A sum of a few low-frequency cosine modes per component, rescaled so the
    largest displacement magnitude is exactly ``max_disp``.
    """
    ax = np.linspace(0.0, 1.0, g)
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
    U = np.zeros((g, g, g, 3))
    for comp in range(3):
        for _ in range(n_modes):
            k = rng.uniform(0.5, 2.0, size=3) * math.pi
            ph = rng.uniform(0, 2 * math.pi, size=3)
            a = rng.normal()
            U[..., comp] += a * (np.cos(k[0] * X + ph[0]) * np.cos(k[1] * Y + ph[1])
                                 * np.cos(k[2] * Z + ph[2]))
    mag = np.sqrt((U ** 2).sum(-1)).max()
    if mag > 0:
        U *= max_disp / mag
    return U.astype(np.float32)
