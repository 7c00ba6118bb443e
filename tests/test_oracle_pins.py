"""Pins of the CPU oracle's projector pair against closed forms and invariants.

Each test fixes a property that a plausible slip in the oracle (a transposed
axis, a wrong sign or offset in the sample positions, a dropped weight, a
transpose that is not one) would break.  Geometry: Sec. 2.2; projection
operator: Sec. 4.1; warp: Sec. 3.1 / 4.2.1; sub-views: Sec. 3.4 / 4.2.2.
"""

import json
import math
import os

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

import oracle
import synth
from ray_reference import box_chord, ellipsoid_chord, source_and_dir

SHAPE = (10, 14, 18)          # (nz, ny, nx): unequal axes catch axis mix-ups
N_U, N_V = 12, 9


def _trajectories():
    rng = np.random.default_rng(11)
    circ = synth.circular_cone(7, N_U, N_V, 40.0, 80.0, 2.0, arc=2.0)
    hel = synth.helical_cone(5, N_U, N_V, 40.0, 80.0, 2.0, pitch_per_rad=2.0,
                             total_angle=5.0, n_sub=1)
    hel = synth.rigid_jitter(hel, 0.5, 2.0, rng)
    off = synth.circular_cone(5, N_U, N_V, 45.0, 70.0, 1.7, det_offset_u=4.0,
                              det_offset_v=-2.0)
    belt = synth.conveyor_belt(5, N_U, N_V, 40.0, 80.0, 2.0, travel=6.0, rotation=1.0)
    return {"circular": circ, "helical_jitter": hel, "offset": off, "conveyor": belt}


@pytest.mark.parametrize("name", ["circular", "helical_jitter", "offset", "conveyor"])
def test_ones_projection_is_hull_chord(name):
    """A 1 equals the chord of the voxel-centre hull, from face intersections."""
    P = _trajectories()[name]
    y = oracle.forward(P, SHAPE, N_U, N_V, np.ones(SHAPE))
    hits = 0
    for p in range(P.shape[0]):
        for iv in range(N_V):
            for iu in range(N_U):
                S, d = source_and_dir(P[p, 0], iu, iv, SHAPE)
                ch = box_chord(S, d, SHAPE)
                want = 0.0 if ch is None else ch[1] - ch[0]
                hits += want > 0
                assert y[p, iv, iu] == pytest.approx(want, rel=1e-12, abs=1e-12)
    assert hits > 0.3 * y.size


def test_linear_volume_is_integrated_exactly():
    """Midpoint rule + trilinear reproduce the integral of a linear field:
    A x = L (a . c_mid + b) with c_mid the chord midpoint."""
    P = _trajectories()["helical_jitter"]
    nz, ny, nx = SHAPE
    a = np.array([0.3, -0.7, 1.1])
    b0 = 2.5
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    vol = a[0] * X + a[1] * Y + a[2] * Z + b0
    y = oracle.forward(P, SHAPE, N_U, N_V, vol)
    for p in range(P.shape[0]):
        for iv in range(N_V):
            for iu in range(N_U):
                S, d = source_and_dir(P[p, 0], iu, iv, SHAPE)
                ch = box_chord(S, d, SHAPE)
                if ch is None:
                    assert y[p, iv, iu] == 0.0
                    continue
                L = ch[1] - ch[0]
                mid = S + 0.5 * (ch[0] + ch[1]) * d
                assert y[p, iv, iu] == pytest.approx(L * (a @ mid + b0), rel=1e-10, abs=1e-9)


def test_indicator_quadrature_bound():
    """Sampling the indicator of an ellipsoid errs from its exact chord by at
    most one adjusted step h <= step per ray (midpoint rule at two edges)."""
    shape = (40, 44, 48)
    P = synth.circular_cone(9, 40, 36, 150.0, 300.0, 1.5, arc=3.0)
    rng = np.random.default_rng(5)
    e = synth.random_ellipsoids(1, shape, (5.0, 14.0), (1.0, 1.0), rng, fov_radius=18.0)[0]
    off = 0.5 * (np.array([48, 44, 40]) - 1)
    Q = e.quadric()
    y = oracle.forward_indicator(P, shape, 40, 36, Q, e.centre + off, step=0.5)
    errs = []
    for p in range(P.shape[0]):
        for iv in range(36):
            for iu in range(40):
                S, d = source_and_dir(P[p, 0], iu, iv, shape)
                want = ellipsoid_chord(S, d, Q, e.centre + off)
                err = abs(y[p, iv, iu] - want)
                assert err <= 0.5 + 1e-9
                if want > 0:
                    errs.append(err)
    errs = np.array(errs)
    assert len(errs) > 200
    # the two edge errors are independent and uniform in [0, h/2]: mean ~ h/4
    assert 0.05 < errs.mean() < 0.2


def test_trilinear_samples_match_library_interpolator():
    """Each ray value equals sum_i h * RGI(c_i) with scipy's trilinear
    RegularGridInterpolator, samples at the midpoints of n = ceil(L/step)
    equal parts of the chord."""
    rng = np.random.default_rng(3)
    P = _trajectories()["offset"]
    vol = rng.uniform(0, 1, SHAPE)
    nz, ny, nx = SHAPE
    interp = RegularGridInterpolator((np.arange(nz), np.arange(ny), np.arange(nx)), vol,
                                     method="linear")
    y = oracle.forward(P, SHAPE, N_U, N_V, vol, step=0.37)
    checked = 0
    for p in range(P.shape[0]):
        for iv in range(0, N_V, 2):
            for iu in range(0, N_U, 3):
                S, d = source_and_dir(P[p, 0], iu, iv, SHAPE)
                ch = box_chord(S, d, SHAPE)
                if ch is None:
                    continue
                L = ch[1] - ch[0]
                n = math.ceil(L / 0.37)
                h = L / n
                t = ch[0] + (np.arange(n) + 0.5) * h
                c = S[None, :] + t[:, None] * d[None, :]
                c = np.clip(c, 0, np.array([nx, ny, nz]) - 1)
                want = h * interp(c[:, ::-1]).sum()
                assert y[p, iv, iu] == pytest.approx(want, rel=1e-11)
                checked += 1
    assert checked > 30


def _voxelised_error(N):
    """rel-L2 of A(voxelised ellipsoids) against sum_e mu_e chord_e."""
    shape = (N, N, N)
    sod = 3.125 * N
    nd = N
    P = synth.circular_cone(8, nd, nd, sod, 2 * sod, 1.5, arc=math.pi)
    rng = np.random.default_rng(21)
    ells = synth.random_ellipsoids(4, (64, 64, 64), (6.0, 14.0), (0.2, 1.0), rng,
                                   fov_radius=20.0)
    s = N / 64.0
    scaled = [synth.Ellipsoid(e.centre * s, e.axes * s, e.rot, e.mu) for e in ells]
    vol = synth.voxelise_ellipsoids(scaled, shape, supersample=3)
    y = oracle.forward(P, shape, nd, nd, vol)
    off = 0.5 * (N - 1)
    exact = np.zeros_like(y)
    for p in range(P.shape[0]):
        for iv in range(nd):
            for iu in range(nd):
                S, d = source_and_dir(P[p, 0], iu, iv, shape)
                exact[p, iv, iu] = sum(e.mu * ellipsoid_chord(S, d, e.quadric(), e.centre + off)
                                       for e in scaled)
    return np.linalg.norm(y - exact) / np.linalg.norm(exact)


def test_voxelised_phantom_converges_first_order():
    e32, e64, e128 = (_voxelised_error(n) for n in (32, 64, 128))
    assert e32 > e64 > e128
    assert e32 / e64 > 1.5 and e64 / e128 > 1.5
    assert e128 < 0.02


def _dot_test(P, shape, n_u, n_v, U=None, tau=None, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=shape)
    y = rng.normal(size=(P.shape[0], n_v, n_u))
    Ax = oracle.forward(P, shape, n_u, n_v, x, U=U, tau=tau)
    ATy = oracle.back(P, shape, n_u, n_v, y, U=U, tau=tau)
    lhs = float(np.sum(Ax * y))
    rhs = float(np.sum(x * ATy))
    return lhs, rhs


@pytest.mark.parametrize("case", ["plain", "subviews", "warp"])
def test_adjoint_dot_product(case):
    """<A x, y> = <x, A^T y> for random x, y."""
    rng = np.random.default_rng(4)
    U = tau = None
    if case == "plain":
        P = _trajectories()["circular"]
    else:
        P = synth.helical_cone(6, N_U, N_V, 40.0, 80.0, 2.0, 2.0, 5.0, n_sub=4)
        P = synth.rigid_jitter(P, 0.5, 2.0, rng)
        if case == "warp":
            U = synth.smooth_displacement(5, 2.0, rng)
            tau = synth.exposure_time_fractions(6, 4)
    lhs, rhs = _dot_test(P, SHAPE, N_U, N_V, U, tau)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_explicit_matrix_transpose():
    """Build A column by column on a tiny case; A^T y must equal A_mat^T y."""
    shape = (5, 6, 7)
    n_u, n_v = 6, 5
    rng = np.random.default_rng(8)
    P = synth.helical_cone(4, n_u, n_v, 25.0, 50.0, 2.0, 1.0, 3.0, n_sub=2)
    U = synth.smooth_displacement(3, 1.0, rng)
    tau = synth.exposure_time_fractions(4, 2)
    nvox = int(np.prod(shape))
    A = np.zeros((4 * n_v * n_u, nvox))
    for j in range(nvox):
        e = np.zeros(nvox)
        e[j] = 1.0
        A[:, j] = oracle.forward(P, shape, n_u, n_v, e.reshape(shape), U=U, tau=tau).ravel()
    assert np.count_nonzero(A) > 0.05 * A.size
    for k in range(3):
        y = rng.normal(size=(4, n_v, n_u))
        got = oracle.back(P, shape, n_u, n_v, y, U=U, tau=tau).ravel()
        np.testing.assert_allclose(got, A.T @ y.ravel(), rtol=1e-12, atol=1e-12)
    # unit rows
    for i in rng.choice(A.shape[0], 8, replace=False):
        e = np.zeros(A.shape[0])
        e[i] = 1.0
        got = oracle.back(P, shape, n_u, n_v, e.reshape(4, n_v, n_u), U=U, tau=tau).ravel()
        np.testing.assert_allclose(got, A[i], rtol=1e-13, atol=1e-14)


def test_identical_subviews_equal_plain():
    P1 = _trajectories()["circular"]
    P4 = np.repeat(P1, 4, axis=1)
    vol = np.random.default_rng(1).uniform(size=SHAPE)
    np.testing.assert_allclose(oracle.forward(P4, SHAPE, N_U, N_V, vol),
                               oracle.forward(P1, SHAPE, N_U, N_V, vol), rtol=1e-13)


def test_subviews_are_the_mean_of_plain_projections():
    P = synth.circular_cone(5, N_U, N_V, 40.0, 80.0, 2.0, n_sub=3)
    vol = np.random.default_rng(2).uniform(size=SHAPE)
    got = oracle.forward(P, SHAPE, N_U, N_V, vol)
    want = np.mean([oracle.forward(P[:, s], SHAPE, N_U, N_V, vol) for s in range(3)], axis=0)
    np.testing.assert_allclose(got, want, rtol=1e-13)
    sino = np.random.default_rng(3).normal(size=got.shape)
    gotb = oracle.back(P, SHAPE, N_U, N_V, sino)
    wantb = np.mean([oracle.back(P[:, s], SHAPE, N_U, N_V, sino) for s in range(3)], axis=0)
    np.testing.assert_allclose(gotb, wantb, rtol=1e-12, atol=1e-13)


def test_zero_displacement_is_plain():
    P = _trajectories()["helical_jitter"]
    vol = np.random.default_rng(2).uniform(size=SHAPE)
    U = np.zeros((4, 4, 4, 3))
    tau = np.full((P.shape[0], 1), 0.7)
    np.testing.assert_array_equal(oracle.forward(P, SHAPE, N_U, N_V, vol, U=U, tau=tau),
                                  oracle.forward(P, SHAPE, N_U, N_V, vol))


def test_linear_displacement_field_is_exact():
    """With U(c) = B (c - m) sampled at the grid nodes k (n-1)/(g-1) (m the
    volume centre), trilinear interpolation reproduces it, so the warped
    samples are c + tau B (c - m).  B contracts the hull into itself, so for a
    linear volume every ray equals L (a . c'_mid + b0) with
    c'_mid = mid + tau B (mid - m): this pins the node placement, the pull-back
    direction and the time scale tau."""
    nz, ny, nx = SHAPE
    g = (4, 5, 6)   # (gz, gy, gx)
    m = 0.5 * (np.array([nx, ny, nz]) - 1.0)
    B = np.array([[-0.06, 0.01, 0.015], [0.01, -0.06, 0.02], [-0.015, 0.01, -0.06]])
    U = np.zeros(g + (3,))
    for kz in range(g[0]):
        for ky in range(g[1]):
            for kx in range(g[2]):
                node = np.array([kx * (nx - 1) / (g[2] - 1), ky * (ny - 1) / (g[1] - 1),
                                 kz * (nz - 1) / (g[0] - 1)])
                U[kz, ky, kx] = B @ (node - m)
    P = _trajectories()["circular"]
    tau = np.linspace(0.2, 0.9, P.shape[0])[:, None]
    a = np.array([0.4, 0.9, -0.6])
    b0 = 3.0
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    vol = a[0] * X + a[1] * Y + a[2] * Z + b0
    y = oracle.forward(P, SHAPE, N_U, N_V, vol, U=U, tau=tau)
    plain = oracle.forward(P, SHAPE, N_U, N_V, vol)
    checked = 0
    for p in range(P.shape[0]):
        for iv in range(N_V):
            for iu in range(N_U):
                S, d = source_and_dir(P[p, 0], iu, iv, SHAPE)
                ch = box_chord(S, d, SHAPE)
                if ch is None:
                    continue
                L = ch[1] - ch[0]
                mid = S + 0.5 * (ch[0] + ch[1]) * d
                wmid = mid + tau[p, 0] * B @ (mid - m)
                assert y[p, iv, iu] == pytest.approx(L * (a @ wmid + b0), rel=1e-10)
                checked += 1
    assert checked > 100
    assert np.max(np.abs(y - plain)) > 0.1   # the warp really moved the samples


def test_projection_is_scale_and_sign_invariant():
    P = _trajectories()["conveyor"]
    vol = np.random.default_rng(9).uniform(size=SHAPE)
    np.testing.assert_allclose(oracle.forward(-2.5 * P, SHAPE, N_U, N_V, vol),
                               oracle.forward(P, SHAPE, N_U, N_V, vol), rtol=1e-12, atol=1e-13)


def test_view_subset_selects_rows():
    P = _trajectories()["circular"]
    vol = np.random.default_rng(10).uniform(size=SHAPE)
    full = oracle.forward(P, SHAPE, N_U, N_V, vol)
    sub = oracle.forward(P, SHAPE, N_U, N_V, vol, views=[5, 1, 1])
    np.testing.assert_array_equal(sub, full[[5, 1, 1]])


def test_invalid_geometry_is_rejected():
    P = _trajectories()["circular"].copy()
    bad = P.copy()
    bad[0, 0, :, :3] = 0.0
    with pytest.raises(oracle.OracleError) as e:
        oracle.forward(bad, SHAPE, N_U, N_V, np.ones(SHAPE))
    assert e.value.code == oracle.ESINGULAR
    inside = synth.view_matrix([0.5, 0.0, 0.0], [-30.0, 0, 0], [0, 1, 0], [0, 0, 1],
                               1.0, 1.0, N_U, N_V)
    with pytest.raises(oracle.OracleError) as e:
        oracle.forward(inside[None, None], SHAPE, N_U, N_V, np.ones(SHAPE))
    assert e.value.code == oracle.ESOURCE_INSIDE


def test_hand_worked_examples():
    """Hand-derived single-ray values (tests/golden/hand_cases.json)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "hand_cases.json")
    with open(path) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        shape = tuple(c["shape"])
        P = synth.view_matrix(c["src"], c["det"], c["e_u"], c["e_v"], 1.0, 1.0, 1, 1)
        vol = np.array(c["vol"], dtype=float).reshape(shape)
        y = oracle.forward(P[None, None], shape, 1, 1, vol, step=c["step"])
        assert y[0, 0, 0] == pytest.approx(c["expected"], rel=1e-13), c["name"]
