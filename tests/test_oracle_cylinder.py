"""Pins of the oracle's aligned cylindrical domain (Sec. 3.5; projector and
backprojector geometry-level modifications, Sec. 4.2.1 / 4.3.1): ray-cylinder
chords in closed form, exact line integrals of volumes linear in z, the
radial and angular index maps against the Cartesian coordinates they
encode, the rigid pose as a change of view matrices, and the voxel-driven
backprojector over polar voxel centres.  CPU only."""

import math

import numpy as np
import pytest

import oracle
import synth


def rigid(rx, ry, rz, t):
    """3x4 [R | t] with R = Rz Ry Rx."""
    cx, sx, cy, sy, cz, sz = (math.cos(rx), math.sin(rx), math.cos(ry), math.sin(ry),
                              math.cos(rz), math.sin(rz))
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    return np.hstack([Rz @ Ry @ Rx, np.asarray(t, float).reshape(3, 1)])


def rays(P, n_u, n_v):
    """Source and unit directions (V frame) of every pixel ray, with numpy."""
    M, p4 = P[:, :3], P[:, 3]
    S = -np.linalg.solve(M, p4)
    uu, vv = np.meshgrid(np.arange(n_u, dtype=float), np.arange(n_v, dtype=float))
    pix = np.stack([uu, vv, np.ones_like(uu)], -1)
    d = np.linalg.solve(M, pix.reshape(-1, 3).T).T.reshape(n_v, n_u, 3)
    return S, d / np.linalg.norm(d, axis=-1, keepdims=True)


def chords(S, d, cyl, pose):
    """[t0, t1] of each ray inside the hull r <= (n_r - 1/2) dr, |z| <= (n_z - 1) dz / 2
    of the cylinder frame (empty where t1 <= t0)."""
    n_r, n_phi, n_z, dr, dz = cyl
    R, t = (np.eye(3), np.zeros(3)) if pose is None else (pose[:, :3], pose[:, 3])
    Sc, dc = R @ S + t, d @ R.T
    Rh, Hz = (n_r - 0.5) * dr, 0.5 * (n_z - 1) * dz
    a = dc[..., 0] ** 2 + dc[..., 1] ** 2
    b = Sc[0] * dc[..., 0] + Sc[1] * dc[..., 1]
    c = Sc[0] ** 2 + Sc[1] ** 2 - Rh ** 2
    disc = b * b - a * c
    sq = np.sqrt(np.maximum(disc, 0))
    # numerically stable roots of a t^2 + 2 b t + c
    q = -(b + np.copysign(sq, b))
    r1, r2 = q / a, c / q
    lo, hi = np.minimum(r1, r2), np.maximum(r1, r2)
    z1, z2 = (-Hz - Sc[2]) / dc[..., 2], (Hz - Sc[2]) / dc[..., 2]
    lo = np.maximum(lo, np.minimum(z1, z2))
    hi = np.minimum(hi, np.maximum(z1, z2))
    hit = (disc >= 0) & (hi > lo)
    return np.where(hit, lo, 0.0), np.where(hit, hi, 0.0), Sc, dc


CYL = (6, 32, 8, 1.5, 1.25)
POSES = [None, rigid(0.15, -0.1, 0.4, [1.5, -0.75, 0.5])]


def scan(n_views=8, n_u=40, n_v=22):
    return synth.circular_cone(n_views, n_u, n_v, 60.0, 120.0, 1.0), n_u, n_v


@pytest.mark.parametrize("pose", POSES, ids=["aligned", "posed"])
def test_ones_volume_gives_the_hull_chord(pose):
    P, n_u, n_v = scan()
    n_r, n_phi, n_z = CYL[:3]
    y, cnt = oracle.forward_cyl(P, CYL, n_u, n_v, np.ones((n_z, n_phi, n_r)), 0.5, pose=pose,
                                return_count=True)
    want, n_want = np.zeros_like(y), 0
    for p in range(P.shape[0]):
        S, d = rays(P[p, 0], n_u, n_v)
        t0, t1, _, _ = chords(S, d, CYL, pose)
        L = t1 - t0
        want[p] = L
        n_want += int(np.sum(np.ceil(L[L > 0] / 0.5)))
    assert np.count_nonzero(want == 0) > 0 and np.count_nonzero(want) > 0   # misses and hits
    # exact up to the conditioning of near-tangent chords (naive vs stable roots)
    np.testing.assert_allclose(y, want, rtol=1e-9, atol=1e-9)
    assert cnt == n_want


@pytest.mark.parametrize("pose", POSES, ids=["aligned", "posed"])
def test_volume_linear_in_z_is_integrated_exactly(pose):
    """f = 0.3 + 0.2 z_k: trilinear sampling reproduces it and the midpoint
    rule integrates it exactly, so A f = L (0.3 + 0.2 z at the chord's middle)."""
    P, n_u, n_v = scan()
    n_r, n_phi, n_z, dr, dz = CYL
    zk = (np.arange(n_z) - 0.5 * (n_z - 1)) * dz
    vol = np.broadcast_to((0.3 + 0.2 * zk)[:, None, None], (n_z, n_phi, n_r))
    y = oracle.forward_cyl(P, CYL, n_u, n_v, vol, 0.5, pose=pose)
    for p in range(P.shape[0]):
        S, d = rays(P[p, 0], n_u, n_v)
        t0, t1, Sc, dc = chords(S, d, CYL, pose)
        zmid = Sc[2] + 0.5 * (t0 + t1) * dc[..., 2]
        np.testing.assert_allclose(y[p], (t1 - t0) * (0.3 + 0.2 * zmid), rtol=1e-11,
                                   atol=1e-11)


def _quadrature(P, n_u, n_v, cyl, pose, f, n=4000):
    """Line integrals of f(xc, yc, zc) over each chord by a fine midpoint rule."""
    out = np.zeros((P.shape[0], n_v, n_u))
    for p in range(P.shape[0]):
        S, d = rays(P[p, 0], n_u, n_v)
        t0, t1, Sc, dc = chords(S, d, cyl, pose)
        s = (np.arange(n) + 0.5) / n
        tt = t0[..., None] + (t1 - t0)[..., None] * s
        X = Sc[:, None, None, None] + dc.transpose(2, 0, 1)[..., None] * tt[None]
        out[p] = (t1 - t0) * f(X[0], X[1], X[2]).mean(-1)
    return out


def test_radial_index_map():
    """f = r_i = (i + 1/2) dr on every ring: the sampled value is max(r, dr/2)
    (linear between rings, the innermost ring's value inside the core)."""
    P, n_u, n_v = scan(4, 24, 18)
    cyl = (12, 64, 10, 1.0, 1.0)
    n_r, n_phi, n_z, dr, dz = cyl
    ri = (np.arange(n_r) + 0.5) * dr
    vol = np.broadcast_to(ri[None, None, :], (n_z, n_phi, n_r))
    y = oracle.forward_cyl(P, cyl, n_u, n_v, vol, 0.02)
    want = _quadrature(P, n_u, n_v, cyl, None,
                       lambda x, yy, z: np.maximum(np.hypot(x, yy), 0.5 * dr))
    np.testing.assert_allclose(y, want, rtol=2e-4, atol=2e-4)


@pytest.mark.parametrize("pose", POSES, ids=["aligned", "posed"])
def test_angular_index_map_and_storage_order(pose):
    """f = r_i cos(phi_j) and r_i sin(phi_j) encode the cylinder-frame x and y;
    with 256 angles their interpolation errs by under r (2 pi / 256)^2 / 8, so
    the integrals match those of xc and yc to 1e-3 relative (a swapped angle,
    a sign or a transposed layout is off by O(1))."""
    P, n_u, n_v = scan(4, 24, 18)
    cyl = (12, 256, 10, 1.0, 1.0)
    n_r, n_phi, n_z, dr, dz = cyl
    ri = (np.arange(n_r) + 0.5) * dr
    phj = 2 * np.pi * np.arange(n_phi) / n_phi
    for trig, comp in ((np.cos, 0), (np.sin, 1)):
        vol = np.broadcast_to((trig(phj)[:, None] * ri[None, :])[None], (n_z, n_phi, n_r))
        y = oracle.forward_cyl(P, cyl, n_u, n_v, vol, 0.5, pose=pose)
        for p in range(P.shape[0]):
            S, d = rays(P[p, 0], n_u, n_v)
            t0, t1, Sc, dc = chords(S, d, cyl, pose)
            mid = Sc[comp] + 0.5 * (t0 + t1) * dc[..., comp]
            want = (t1 - t0) * mid
            # inside the core (r < dr/2) the map holds ring 0's values: allow that
            scale = np.abs(want).max()
            assert np.max(np.abs(y[p] - want)) <= 1e-3 * scale + 0.02 * (t1 - t0).max()
            # and most rays away from the axis agree much more closely
            assert np.median(np.abs(y[p] - want)) <= 2e-3 * scale


def test_pose_is_a_change_of_view_matrices():
    """A rigid pose T (V frame -> cylinder frame) equals projecting with the
    matrices P T^-1 and no pose, for both operators."""
    P, n_u, n_v = scan(6, 20, 16)
    T = rigid(0.2, 0.1, -0.7, [2.0, 1.0, -1.5])
    T4 = np.vstack([T, [0, 0, 0, 1]])
    P2 = P @ np.linalg.inv(T4)
    rng = np.random.default_rng(5)
    vol = rng.uniform(0, 1, (CYL[2], CYL[1], CYL[0]))
    a = oracle.forward_cyl(P, CYL, n_u, n_v, vol, 0.5, pose=T)
    b = oracle.forward_cyl(P2, CYL, n_u, n_v, vol, 0.5)
    np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-9)
    img = rng.uniform(-1, 1, (6, n_v, n_u))
    np.testing.assert_allclose(oracle.back_voxel_cyl(P, CYL, n_u, n_v, img, pose=T),
                               oracle.back_voxel_cyl(P2, CYL, n_u, n_v, img), rtol=1e-10,
                               atol=1e-10)


@pytest.mark.parametrize("pose", POSES, ids=["aligned", "posed"])
def test_voxel_backprojector_samples_affine_images_at_polar_centres(pose):
    P = synth.circular_cone(5, 64, 60, 60.0, 120.0, 1.0, n_sub=2)
    n_u, n_v = 64, 60
    n_r, n_phi, n_z, dr, dz = CYL
    rng = np.random.default_rng(8)
    coef = rng.normal(size=(5, 3))
    uu, vv = np.meshgrid(np.arange(n_u), np.arange(n_v))
    img = np.stack([a * uu + b * vv + c for a, b, c in coef])
    got = oracle.back_voxel_cyl(P, CYL, n_u, n_v, img, pose=pose)
    ri = (np.arange(n_r) + 0.5) * dr
    phj = 2 * np.pi * np.arange(n_phi) / n_phi
    zk = (np.arange(n_z) - 0.5 * (n_z - 1)) * dz
    Z, PH, RR = np.meshgrid(zk, phj, ri, indexing="ij")
    Xc = np.stack([RR * np.cos(PH), RR * np.sin(PH), Z], -1)
    R, t = (np.eye(3), np.zeros(3)) if pose is None else (pose[:, :3], pose[:, 3])
    X = (Xc - t) @ R
    H = np.concatenate([X, np.ones(X.shape[:-1] + (1,))], -1)
    want = np.zeros(got.shape)
    for p in range(5):
        for s in range(2):
            q = H @ P[p, s].T
            u, v = q[..., 0] / q[..., 2], q[..., 1] / q[..., 2]
            assert u.min() > 1 and u.max() < n_u - 2 and v.min() > 1 and v.max() < n_v - 2
            want += (coef[p, 0] * u + coef[p, 1] * v + coef[p, 2]) / 2
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-11)


def test_sirt_cyl_is_the_matrix_iteration():
    P, n_u, n_v = scan(6, 10, 8)
    cyl = (3, 8, 3, 2.0, 2.0)
    pose = rigid(0.1, 0.0, 0.3, [0.5, 0.0, 0.0])
    shape = (3, 8, 3)
    nvox = int(np.prod(shape))
    A = np.zeros((6 * n_v * n_u, nvox))
    for j in range(nvox):
        e = np.zeros(nvox)
        e[j] = 1.0
        A[:, j] = oracle.forward_cyl(P, cyl, n_u, n_v, e.reshape(shape), 0.5, pose=pose).ravel()
    B = np.zeros((nvox, A.shape[0]))
    for i in range(A.shape[0]):
        e = np.zeros(A.shape[0])
        e[i] = 1.0
        B[:, i] = oracle.back_voxel_cyl(P, cyl, n_u, n_v, e.reshape(6, n_v, n_u),
                                        pose=pose).ravel()
    b = np.random.default_rng(2).uniform(0, 3, A.shape[0])
    R = np.where(A.sum(1) > 0, 1 / np.maximum(A.sum(1), 1e-300), 0)
    C = np.where(B.sum(1) > 0, 1 / np.maximum(B.sum(1), 1e-300), 0)
    x = np.zeros(nvox)
    for _ in range(3):
        x = x + 0.9 * C * (B @ (R * (b - A @ x)))
    got, _ = oracle.sirt_cyl(P, cyl, n_u, n_v, b, 3, alpha=0.9, pose=pose)
    np.testing.assert_allclose(got.ravel(), x, rtol=1e-10, atol=1e-12)


def test_source_inside_the_cylinder_is_rejected():
    P, n_u, n_v = scan(2, 8, 8)
    with pytest.raises(oracle.OracleError):
        oracle.forward_cyl(P, (50, 16, 8, 1.5, 1.0), n_u, n_v, np.zeros((8, 16, 50)))
