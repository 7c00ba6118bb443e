"""Pins of the oracle's voxel-driven backprojector (the paper's Sec. 4.1
backprojection operator: voxel centre projected onto each detector image,
image sampled bilinearly).  CPU only."""

import numpy as np

import oracle
import synth


def _project(P, shape):
    """(u, v) of every voxel centre under each 3x4 matrix, written out with
    numpy (independent of the oracle's loops)."""
    nz, ny, nx = shape
    Z, Y, X = np.meshgrid(np.arange(nz) - 0.5 * (nz - 1), np.arange(ny) - 0.5 * (ny - 1),
                          np.arange(nx) - 0.5 * (nx - 1), indexing="ij")
    H = np.stack([X, Y, Z, np.ones_like(X)], -1)
    q = H @ P.T
    return q[..., 0] / q[..., 2], q[..., 1] / q[..., 2]


def test_linear_images_are_sampled_exactly():
    """Bilinear sampling reproduces an affine image exactly, so B r equals the
    sum over views of a_p u + b_p v + c_p at the projected voxel centres."""
    shape = (5, 6, 7)
    n_u = n_v = 64
    P = synth.circular_cone(9, n_u, n_v, 40.0, 80.0, 1.0, n_sub=2)
    rng = np.random.default_rng(3)
    coef = rng.normal(size=(9, 3))
    uu, vv = np.meshgrid(np.arange(n_u), np.arange(n_v))
    img = np.stack([a * uu + b * vv + c for a, b, c in coef])
    got = oracle.back_voxel(P, shape, n_u, n_v, img)
    want = np.zeros(shape)
    for p in range(9):
        for s in range(2):
            u, v = _project(P[p, s], shape)
            assert u.min() > 1 and u.max() < n_u - 2 and v.min() > 1 and v.max() < n_v - 2
            want += (coef[p, 0] * u + coef[p, 1] * v + coef[p, 2]) / 2
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-11)


def test_affine_view_hand_values_with_zero_outside():
    """One affine view with u = x + 0.25, v = y - 0.5 (index coordinates) on a
    3 x 2 detector: hand-computed bilinear values, zero beyond the border."""
    shape = (1, 3, 4)                    # x in {-1.5, ..., 1.5}, y in {-1, 0, 1}
    P = np.array([[[1.0, 0, 0, 1.5 + 0.25], [0, 1.0, 0, 1.0 - 0.5], [0, 0, 0, 1.0]]])
    img = np.array([[[1.0, 2.0, 4.0], [8.0, 16.0, 32.0]]])   # [v][u], 2 rows x 3 cols
    got = oracle.back_voxel(P, shape, 3, 2, img)[0]
    want = np.zeros((3, 4))
    for iy in range(3):
        for ix in range(4):
            u, v = ix + 0.25, iy - 0.5
            acc = 0.0
            for du in (0, 1):
                for dv in (0, 1):
                    iu, iv = int(np.floor(u)) + du, int(np.floor(v)) + dv
                    if 0 <= iu < 3 and 0 <= iv < 2:
                        wu = (u - np.floor(u)) if du else 1 - (u - np.floor(u))
                        wv = (v - np.floor(v)) if dv else 1 - (v - np.floor(v))
                        acc += wu * wv * img[0, iv, iu]
            want[iy, ix] = acc
    # spot values: voxel (0, 0) at (0.25, -0.5) sees half of row 0 at u = 0.25
    assert abs(want[0, 0] - 0.5 * (0.75 * 1 + 0.25 * 2)) < 1e-15
    # u = 2.25 keeps one column (weight 0.75), v = -0.5 / 1.5 one row (0.5)
    assert want[0, 2] == 0.5 * 0.75 * 4 and want[2, 2] == 0.5 * 0.75 * 32
    assert want[0, 3] == 0.0             # u = 3.25: both columns off the detector
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)


def test_ones_count_the_views_that_see_a_voxel():
    shape = (4, 4, 4)
    n_u = n_v = 48
    P = synth.circular_cone(12, n_u, n_v, 30.0, 60.0, 1.0, n_sub=1)
    got = oracle.back_voxel(P, shape, n_u, n_v, np.ones((12, n_v, n_u)))
    np.testing.assert_allclose(got, 12.0, rtol=0, atol=1e-12)
    sub = oracle.back_voxel(P, shape, n_u, n_v, np.ones((3, n_v, n_u)), views=[0, 5, 9])
    np.testing.assert_allclose(sub, 3.0, rtol=0, atol=1e-12)


def test_sirt_with_voxel_backprojector_is_the_matrix_iteration():
    """x <- x + a C B R (b - A x) with C = 1 / (B 1), B and A as explicit
    matrices built column by column from the oracle's operators."""
    shape = (3, 4, 4)
    n_u = n_v = 6
    P = synth.circular_cone(10, n_u, n_v, 20.0, 40.0, 1.2, n_sub=1)
    nvox = int(np.prod(shape))
    A = np.zeros((10 * n_u * n_v, nvox))
    for j in range(nvox):
        e = np.zeros(nvox)
        e[j] = 1.0
        A[:, j] = oracle.forward(P, shape, n_u, n_v, e.reshape(shape)).ravel()
    B = np.zeros((nvox, 10 * n_u * n_v))
    for i in range(B.shape[1]):
        e = np.zeros(B.shape[1])
        e[i] = 1.0
        B[:, i] = oracle.back_voxel(P, shape, n_u, n_v, e.reshape(10, n_v, n_u)).ravel()
    rng = np.random.default_rng(4)
    b = rng.uniform(0, 2, A.shape[0])
    R = np.where(A.sum(1) > 0, 1 / np.maximum(A.sum(1), 1e-300), 0)
    C = np.where(B.sum(1) > 0, 1 / np.maximum(B.sum(1), 1e-300), 0)
    x = np.zeros(nvox)
    for _ in range(3):
        x = x + 0.7 * C * (B @ (R * (b - A @ x)))
    got, _ = oracle.sirt(P, shape, n_u, n_v, b, 3, alpha=0.7, voxel_bp=True)
    np.testing.assert_allclose(got.ravel(), x, rtol=1e-10, atol=1e-12)


def test_points_variant_agrees_with_the_volume():
    shape = (6, 5, 7)
    n_u, n_v = 20, 18
    P = synth.circular_cone(8, n_u, n_v, 25.0, 50.0, 1.0, n_sub=2)
    rng = np.random.default_rng(11)
    img = rng.uniform(-1, 1, (5, n_v, n_u))
    views = [7, 0, 3, 3, 5]
    vol = oracle.back_voxel(P, shape, n_u, n_v, img, views=views)
    ijk = np.stack([rng.integers(0, n, 40) for n in (7, 5, 6)], 1)
    pts = oracle.back_voxel_points(P, shape, n_u, n_v, img, ijk, views=views)
    np.testing.assert_array_equal(pts, vol[ijk[:, 2], ijk[:, 1], ijk[:, 0]])
