"""Seeded phantoms: random ellipsoids, a cylinder background and foams.

Coordinates are the centred voxel units of the V frame (voxel i of an axis of
length n has its centre at i - (n-1)/2).  Volumes are numpy arrays laid out
[nz][ny][nx] (x fastest).  Overlapping objects add their attenuation values,
so a line integral through a set of ellipsoids is the sum of mu times chord.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Ellipsoid:
    centre: np.ndarray   # (3,) V frame, order (x, y, z)
    axes: np.ndarray     # (3,) semi-axes, voxel units
    rot: np.ndarray      # (3,3) columns are the ellipsoid's axes in V
    mu: float

    def quadric(self):
        """Q with ||Q (X - centre)|| <= 1 exactly inside."""
        return np.diag(1.0 / self.axes) @ self.rot.T


def _random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def random_ellipsoids(n, shape, semi_range, mu_range, rng, fov_radius=None,
                      z_half=None):
    """``n`` ellipsoids whose bounding spheres lie inside the FOV cylinder.

    ``shape`` is (nz, ny, nx).  Semi-axes ~ U(semi_range), values ~ U(mu_range),
    orientation uniform on SO(3), centres uniform in the allowed region.
    """
    nz, ny, nx = shape
    if fov_radius is None:
        fov_radius = 0.5 * (min(nx, ny) - 1)
    if z_half is None:
        z_half = 0.5 * (nz - 1)
    out = []
    while len(out) < n:
        axes = rng.uniform(semi_range[0], semi_range[1], size=3)
        r = float(axes.max())
        rmax = fov_radius - r
        zmax = z_half - r
        if rmax <= 0 or zmax <= 0:
            # the largest draw does not fit: shrink it to the region
            axes = axes * min(fov_radius, z_half) / (r * 1.05)
            r = float(axes.max())
            rmax = fov_radius - r
            zmax = z_half - r
        rho = rmax * np.sqrt(rng.uniform())
        phi = rng.uniform(0, 2 * np.pi)
        cz = rng.uniform(-zmax, zmax)
        centre = np.array([rho * np.cos(phi), rho * np.sin(phi), cz])
        out.append(Ellipsoid(centre, axes, _random_rotation(rng),
                             float(rng.uniform(mu_range[0], mu_range[1]))))
    return out


def _centres(n):
    return np.arange(n, dtype=np.float64) - 0.5 * (n - 1)


def voxelise_ellipsoids(ells, shape, supersample=1, dtype=np.float64):
    """Point-sample (supersample=1) or box-average (k^3 sub-points) ellipsoids."""
    nz, ny, nx = shape
    vol = np.zeros(shape, dtype=np.float64)
    k = int(supersample)
    sub = (np.arange(k) + 0.5) / k - 0.5
    cx, cy, cz = _centres(nx), _centres(ny), _centres(nz)
    for e in ells:
        Q = e.quadric()
        r = float(e.axes.max()) + 1.0
        lo = np.floor(e.centre - r + 0.5 * (np.array([nx, ny, nz]) - 1)).astype(int)
        hi = np.ceil(e.centre + r + 0.5 * (np.array([nx, ny, nz]) - 1)).astype(int)
        lo = np.maximum(lo, 0)
        hi = np.minimum(hi, [nx - 1, ny - 1, nz - 1])
        if np.any(hi < lo):
            continue
        xs = cx[lo[0]:hi[0] + 1]
        ys = cy[lo[1]:hi[1] + 1]
        zs = cz[lo[2]:hi[2] + 1]
        acc = np.zeros((len(zs), len(ys), len(xs)))
        for dz in sub:
            for dy in sub:
                for dx in sub:
                    Z, Y, X = np.meshgrid(zs + dz, ys + dy, xs + dx, indexing="ij")
                    D = np.stack([X - e.centre[0], Y - e.centre[1], Z - e.centre[2]], -1)
                    q = D @ Q.T
                    acc += (np.einsum("...i,...i->...", q, q) <= 1.0)
        vol[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] += e.mu * acc / k ** 3
    return vol.astype(dtype)


def cylinder_background(shape, radius, height, mu, dtype=np.float64):
    """Uniform cylinder about the z axis, point-sampled at voxel centres."""
    nz, ny, nx = shape
    z = _centres(nz)
    y = _centres(ny)[:, None]
    x = _centres(nx)[None, :]
    disc = (x * x + y * y <= radius * radius)
    out = np.zeros(shape, dtype=dtype)
    out[np.abs(z) <= 0.5 * height] = mu * disc
    return out


def foam_phantom(shape, rng, radius_frac=0.4, mu=0.5, n_voids=(20, 200),
                 void_radius_frac=(0.01, 0.08), dtype=np.float64):
    """Cylinder (radius 0.4 N) minus random non-overlapping spherical voids."""
    nz, ny, nx = shape
    R, H, voids = foam_voids(shape, rng, radius_frac, n_voids, void_radius_frac)
    vol = cylinder_background(shape, R, H, mu)
    cz, cy, cx = _centres(nz), _centres(ny), _centres(nx)
    for c, r in voids:
        # clear the void inside its bounding box only
        lo = [max(int(np.floor(c[a] - r + 0.5 * (n - 1))), 0) for a, n in enumerate((nx, ny, nz))]
        hi = [min(int(np.ceil(c[a] + r + 0.5 * (n - 1))), n - 1) for a, n in enumerate((nx, ny, nz))]
        Z, Y, X = np.meshgrid(cz[lo[2]:hi[2] + 1], cy[lo[1]:hi[1] + 1], cx[lo[0]:hi[0] + 1],
                              indexing="ij")
        d2 = (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2
        sub = vol[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1]
        sub[d2 <= r * r] = 0.0
    return vol.astype(dtype)


def fov_mask(shape, radius):
    """Boolean cylinder mask about the z axis (used for PSNR)."""
    nz, ny, nx = shape
    y = _centres(ny)[:, None]
    x = _centres(nx)[None, :]
    return np.broadcast_to((x * x + y * y) <= radius * radius, shape)


# ------------------------------------------------------------- torch variants --
# The same point-sampled definitions evaluated with torch on any device, so
# large training sets can be synthesised where the volumes are used.  Object
# parameters still come from the numpy generators above.

def _torch_centres(n, device):
    import torch
    return torch.arange(n, dtype=torch.float64, device=device) - 0.5 * (n - 1)


def voxelise_ellipsoids_torch(ells, shape, device, dtype=None):
    """Point-sampled ellipsoids (``voxelise_ellipsoids`` with supersample=1)."""
    import torch
    nz, ny, nx = shape
    vol = torch.zeros(shape, dtype=torch.float64, device=device)
    cx, cy, cz = (_torch_centres(n, device) for n in (nx, ny, nz))
    for e in ells:
        Q = torch.as_tensor(e.quadric(), dtype=torch.float64, device=device)
        r = float(e.axes.max()) + 1.0
        lo = np.floor(e.centre - r + 0.5 * (np.array([nx, ny, nz]) - 1)).astype(int)
        hi = np.ceil(e.centre + r + 0.5 * (np.array([nx, ny, nz]) - 1)).astype(int)
        lo = np.maximum(lo, 0)
        hi = np.minimum(hi, [nx - 1, ny - 1, nz - 1])
        if np.any(hi < lo):
            continue
        xs = cx[lo[0]:hi[0] + 1] - float(e.centre[0])
        ys = cy[lo[1]:hi[1] + 1] - float(e.centre[1])
        zs = cz[lo[2]:hi[2] + 1] - float(e.centre[2])
        Z, Y, X = torch.meshgrid(zs, ys, xs, indexing="ij")
        D = torch.stack([X, Y, Z], -1)
        q = D @ Q.T
        inside = (q * q).sum(-1) <= 1.0
        vol[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] += e.mu * inside.to(torch.float64)
    return vol if dtype is None else vol.to(dtype)


def foam_voids(shape, rng, radius_frac=0.4, n_voids=(20, 200), void_radius_frac=(0.01, 0.08)):
    """The cylinder radius, height and void list of ``foam_phantom`` (same draws)."""
    nz, ny, nx = shape
    N = min(nx, ny)
    R = radius_frac * N
    H = 0.9 * nz
    k = int(rng.integers(n_voids[0], n_voids[1] + 1))
    voids = []
    tries = 0
    while len(voids) < k and tries < 20000:
        tries += 1
        r = rng.uniform(void_radius_frac[0], void_radius_frac[1]) * N
        rho = (R - r) * np.sqrt(rng.uniform())
        phi = rng.uniform(0, 2 * np.pi)
        z = rng.uniform(-(0.5 * H - r), 0.5 * H - r)
        c = np.array([rho * np.cos(phi), rho * np.sin(phi), z])
        if all(np.linalg.norm(c - c2) > r + r2 for c2, r2 in voids):
            voids.append((c, r))
    return R, H, voids


def foam_phantom_torch(shape, rng, device, mu=0.5, dtype=None, **kw):
    """``foam_phantom`` evaluated with torch (identical draws from ``rng``)."""
    import torch
    nz, ny, nx = shape
    R, H, voids = foam_voids(shape, rng, **kw)
    cz, cy, cx = (_torch_centres(n, device) for n in (nz, ny, nx))
    disc = (cx[None, :] ** 2 + cy[:, None] ** 2) <= R * R
    vol = torch.zeros(shape, dtype=torch.float64, device=device)
    vol[torch.abs(cz) <= 0.5 * H] = mu * disc.to(torch.float64)
    for c, r in voids:
        lo = [max(int(np.floor(c[a] - r + 0.5 * (n - 1))), 0) for a, n in enumerate((nx, ny, nz))]
        hi = [min(int(np.ceil(c[a] + r + 0.5 * (n - 1))), n - 1) for a, n in enumerate((nx, ny, nz))]
        Z, Y, X = torch.meshgrid(cz[lo[2]:hi[2] + 1], cy[lo[1]:hi[1] + 1], cx[lo[0]:hi[0] + 1],
                                 indexing="ij")
        d2 = (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2
        sub = vol[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1]
        sub[d2 <= r * r] = 0.0
    return vol if dtype is None else vol.to(dtype)


def vial_polar(n_r, n_phi, n_z, dr, dz, rng, dtype=np.float32):
    """A vial-like object on the polar grid [n_z][n_phi][n_r] of the aligned
    cylindrical domain (ring i at (i + 1/2) dr, angle 2 pi j / n_phi, slice
    (k - (n_z - 1)/2) dz): a glass wall (mu 1.0) at 80-90 % of the radius, a
    fill (mu 0.3) below 75 % of the height with concentric layers of +-0.05
    and seeded spherical voids, empty above."""
    r = (np.arange(n_r) + 0.5) * dr
    z = (np.arange(n_z) - 0.5 * (n_z - 1)) * dz
    R, H = n_r * dr, 0.5 * (n_z - 1) * dz
    wall = ((r >= 0.8 * R) & (r <= 0.9 * R)).astype(np.float64)
    fill = (r < 0.8 * R) * (0.3 + 0.05 * np.sign(np.sin(r / (0.04 * R))))
    vol = np.empty((n_z, n_phi, n_r), dtype=dtype)
    below = z < 0.5 * H
    prof = wall[None, :] + fill[None, :] * below[:, None]          # [n_z][n_r]
    vol[:] = prof[:, None, :]
    # voids: balls in the fill, carved on the polar grid
    phi = 2 * np.pi * np.arange(n_phi) / n_phi
    for _ in range(int(rng.integers(8, 16))):
        cr, cphi = rng.uniform(0.1, 0.6) * R, rng.uniform(0, 2 * np.pi)
        cz, rad = rng.uniform(-H, 0.4 * H), rng.uniform(0.03, 0.08) * R
        ks = np.nonzero(np.abs(z - cz) <= rad)[0]
        for k in ks:
            d2 = (r[None, :] * np.cos(phi)[:, None] - cr * np.cos(cphi)) ** 2 + \
                 (r[None, :] * np.sin(phi)[:, None] - cr * np.sin(cphi)) ** 2 + (z[k] - cz) ** 2
            vol[k][d2 <= rad * rad] = 0.0
    return vol
