"""Pins of the oracle's SIRT iteration (Eq. 1) and helper terms on tiny problems.

The projector is turned into an explicit matrix column by column, so the
iteration can be checked against linear algebra that does not run it: the
closed-form power series, the spectral bound of the normalised operator, the
monotone weighted residual, and convergence to the exact solution.
"""

import numpy as np
import pytest

import oracle
import synth

SHAPE = (3, 4, 4)
N_U = N_V = 6


def _problem(n_proj=12):
    P = synth.circular_cone(n_proj, N_U, N_V, 20.0, 40.0, 1.2, n_sub=1)
    nvox = int(np.prod(SHAPE))
    A = np.zeros((n_proj * N_V * N_U, nvox))
    for j in range(nvox):
        e = np.zeros(nvox)
        e[j] = 1.0
        A[:, j] = oracle.forward(P, SHAPE, N_U, N_V, e.reshape(SHAPE)).ravel()
    return P, A


def _recip(v):
    out = np.zeros_like(v)
    out[v > 0] = 1.0 / v[v > 0]
    return out


def test_weights_are_inverse_row_and_column_sums():
    P, A = _problem()
    Rw, Cw = oracle.sirt_weights(P, SHAPE, N_U, N_V)
    np.testing.assert_allclose(Rw.ravel(), _recip(A.sum(1)), rtol=1e-12)
    np.testing.assert_allclose(Cw.ravel(), _recip(A.sum(0)), rtol=1e-12)


@pytest.mark.parametrize("alpha", [1.0, 1.7])
def test_iterates_equal_power_series(alpha):
    """x_k = sum_{j<k} (I - a C A^T R A)^j a C A^T R b for x_0 = 0."""
    P, A = _problem()
    rng = np.random.default_rng(1)
    b = rng.uniform(0, 3, A.shape[0])
    R = np.diag(_recip(A.sum(1)))
    C = np.diag(_recip(A.sum(0)))
    T = np.eye(A.shape[1]) - alpha * C @ A.T @ R @ A
    g = alpha * C @ A.T @ R @ b
    xk = np.zeros(A.shape[1])
    term = g.copy()
    for k in range(1, 6):
        xk = xk + term
        term = T @ term
    x5, norms = oracle.sirt(P, SHAPE, N_U, N_V, b, 5, alpha=alpha)
    np.testing.assert_allclose(x5.ravel(), xk, rtol=1e-10, atol=1e-12)
    # the reported norms are ||b - A x_k|| for k = 0..4
    x = np.zeros(A.shape[1])
    want = []
    for k in range(5):
        want.append(np.linalg.norm(b - A @ x))
        x = x + g + (T - np.eye(A.shape[1])) @ x
    np.testing.assert_allclose(norms, want, rtol=1e-10)


def test_normalised_operator_norm_at_most_one():
    """||R^1/2 A C^1/2||_2 <= 1 for row/column-sum normalisations."""
    _, A = _problem()
    r = np.sqrt(_recip(A.sum(1)))
    c = np.sqrt(_recip(A.sum(0)))
    s = np.linalg.norm(r[:, None] * A * c[None, :], 2)
    assert s <= 1.0 + 1e-12
    assert s > 0.99   # attained by the positive Perron vector


@pytest.mark.parametrize("alpha", [0.5, 1.0, 1.9])
def test_weighted_residual_is_non_increasing(alpha):
    P, A = _problem()
    rng = np.random.default_rng(2)
    b = A @ rng.uniform(0, 1, A.shape[1]) + 0.05 * rng.normal(size=A.shape[0])
    Rw, Cw = oracle.sirt_weights(P, SHAPE, N_U, N_V)
    x = np.zeros(SHAPE)
    prev = np.inf
    for _ in range(15):
        res = b.reshape(Rw.shape) - oracle.forward(P, SHAPE, N_U, N_V, x)
        wr = float(np.sum(Rw * res * res))
        assert wr <= prev * (1 + 1e-12)
        prev = wr
        x, _ = oracle.sirt(P, SHAPE, N_U, N_V, b, 1, alpha=alpha, x0=x, weights=(Rw, Cw))


def test_converges_to_exact_solution_of_consistent_system():
    """Full column rank and b = A x_true: in w = C^-1/2 (x - x_true) one step is
    the symmetric map I - a H, H = C^1/2 A^T R A C^1/2 with spectrum in (0, 1],
    so ||x_k - x_true||_{C^-1} <= rho^k ||x_0 - x_true||_{C^-1} with
    rho = max |1 - a lambda|; the bound is checked every 25 iterations."""
    P, A = _problem(n_proj=16)
    assert np.linalg.matrix_rank(A) == A.shape[1]
    rng = np.random.default_rng(3)
    x_true = rng.uniform(0, 1, A.shape[1])
    b = A @ x_true
    alpha = 1.9
    r = _recip(A.sum(1))
    c = _recip(A.sum(0))
    H = np.sqrt(c)[:, None] * (A.T @ (r[:, None] * A)) * np.sqrt(c)[None, :]
    lam = np.linalg.eigvalsh(H)
    assert lam.min() > 0 and lam.max() <= 1 + 1e-12
    rho = max(abs(1 - alpha * lam.min()), abs(1 - alpha * lam.max()))
    Rw, Cw = oracle.sirt_weights(P, SHAPE, N_U, N_V)
    cinv = _recip(Cw.ravel())
    x = np.zeros(SHAPE)
    e0 = float(np.sqrt(np.sum(cinv * x_true * x_true)))
    for j in range(1, 21):
        x, _ = oracle.sirt(P, SHAPE, N_U, N_V, b, 25, alpha=alpha, x0=x, weights=(Rw, Cw))
        e = x.ravel() - x_true
        ek = float(np.sqrt(np.sum(cinv * e * e)))
        assert ek <= rho ** (25 * j) * e0 * (1 + 1e-9) + 1e-12
    assert ek < 0.05 * e0


def test_nonneg_clamps_iterates():
    P, A = _problem()
    b = -np.ones(A.shape[0])
    x, _ = oracle.sirt(P, SHAPE, N_U, N_V, b, 3, nonneg=True)
    assert x.min() == 0.0


def test_tv_closed_form_ramp():
    nz, ny, nx = 4, 5, 6
    a, eps = 0.3, 1e-5
    x = np.broadcast_to(a * np.arange(nx), (nz, ny, nx)).copy()
    want = (nx - 1) * ny * nz * np.sqrt(a * a + eps * eps) + ny * nz * eps
    assert oracle.tv(x, eps) == pytest.approx(want, rel=1e-13)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_tv_closed_form_ramp_each_axis(axis):
    """A ramp along one axis (z, y or x): every voxel before the last index of
    that axis has |grad+ x| = a, the last layer only eps.  A difference taken
    along the wrong axis, or one axis' difference counted twice, fails."""
    shape = (4, 5, 6)
    a, eps = 0.7, 1e-5
    idx = np.indices(shape)[axis].astype(np.float64)
    x = a * idx
    n_axis = shape[axis]
    layer = int(np.prod(shape)) // n_axis
    want = (n_axis - 1) * layer * np.sqrt(a * a + eps * eps) + layer * eps
    assert oracle.tv(x, eps) == pytest.approx(want, rel=1e-13)


def test_tv_brute_force_loops():
    """TV written as an explicit triple loop over voxels with each forward
    difference taken by index arithmetic, on a random 4x5x6 volume."""
    rng = np.random.default_rng(21)
    nz, ny, nx = 4, 5, 6
    x = rng.normal(size=(nz, ny, nx))
    eps = 1e-3
    total = 0.0
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                gx = x[k, j, i + 1] - x[k, j, i] if i + 1 < nx else 0.0
                gy = x[k, j + 1, i] - x[k, j, i] if j + 1 < ny else 0.0
                gz = x[k + 1, j, i] - x[k, j, i] if k + 1 < nz else 0.0
                total += (gx * gx + gy * gy + gz * gz + eps * eps) ** 0.5
    assert oracle.tv(x, eps) == pytest.approx(total, rel=1e-13)


def test_tv_gradient_matches_central_differences():
    rng = np.random.default_rng(4)
    x = rng.normal(size=(5, 6, 7))
    eps = 1e-2
    g = oracle.tv_grad(x, eps)
    h = 1e-6
    for idx in [(0, 0, 0), (4, 5, 6), (2, 3, 1), (1, 0, 6), (3, 5, 0)]:
        xp = x.copy()
        xm = x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (oracle.tv(xp, eps) - oracle.tv(xm, eps)) / (2 * h)
        assert g[idx] == pytest.approx(fd, rel=1e-6, abs=1e-8)


def test_psnr_closed_form():
    t = np.zeros((2, 3, 4))
    t[0, 0, 0] = 2.0
    x = t + 0.1
    assert oracle.psnr(x, t) == pytest.approx(10 * np.log10(4.0 / 0.01), rel=1e-12)


def test_poisson_log_transform_is_unbiased_at_high_dose():
    rng = np.random.default_rng(5)
    y = np.full(200000, 1.3)
    b = synth.poisson_log_transform(y, 1e6, rng)
    assert abs(b.mean() - 1.3) < 2e-4
    # standard deviation of -ln(counts / I0) ~ 1 / sqrt(I0 exp(-y))
    assert b.std() == pytest.approx(1 / np.sqrt(1e6 * np.exp(-1.3)), rel=0.02)


def _rows(views, n_proj):
    """Row indices of the explicit matrix belonging to the listed projections."""
    per = N_V * N_U
    return np.concatenate([np.arange(v * per, (v + 1) * per) for v in views])


def test_os_sirt_equals_block_matrix_iteration():
    """Each subset update is x <- x + a C_k A_k^T R_k (b_k - A_k x) with the
    subset's own row/column-sum weights, written with the explicit matrix."""
    P, A = _problem()
    rng = np.random.default_rng(7)
    b = rng.uniform(0, 3, A.shape[0])
    subsets = [[0, 4, 8], [1, 5, 9], [2, 6, 10], [3, 7, 11]]
    x, norms = oracle.os_sirt(P, SHAPE, N_U, N_V, b.reshape(12, N_V, N_U), subsets, 2,
                              alpha=0.9)
    xr = np.zeros(A.shape[1])
    want = []
    for _ in range(2):
        row = []
        for s in subsets:
            rows = _rows(s, 12)
            Ak, bk = A[rows], b[rows]
            Rk, Ck = _recip(Ak.sum(1)), _recip(Ak.sum(0))
            r = bk - Ak @ xr
            row.append(np.linalg.norm(r))
            xr = xr + 0.9 * Ck * (Ak.T @ (Rk * r))
        want.append(row)
    np.testing.assert_allclose(x.ravel(), xr, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(norms, want, rtol=1e-10)


def test_os_sirt_with_one_subset_is_sirt():
    P, A = _problem()
    b = np.random.default_rng(8).uniform(0, 3, (12, N_V, N_U))
    x1, n1 = oracle.os_sirt(P, SHAPE, N_U, N_V, b, [list(range(12))], 3)
    x2, n2 = oracle.sirt(P, SHAPE, N_U, N_V, b, 3)
    # equal up to the summation order of the oracle's threaded backprojection
    np.testing.assert_allclose(x1, x2, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(np.ravel(n1), n2, rtol=1e-12)


def test_os_sirt_converges_faster_per_data_pass_on_consistent_data():
    """On consistent data one ordered-subset epoch (as many projections as one
    SIRT iteration) lowers the error more than one SIRT iteration."""
    P, A = _problem()
    xt = np.random.default_rng(9).uniform(0, 1, A.shape[1])
    b = (A @ xt).reshape(12, N_V, N_U)
    subsets = [[k, k + 4, k + 8] for k in range(4)]
    xo, _ = oracle.os_sirt(P, SHAPE, N_U, N_V, b, subsets, 3)
    xs, _ = oracle.sirt(P, SHAPE, N_U, N_V, b, 3)
    assert np.linalg.norm(xo.ravel() - xt) < np.linalg.norm(xs.ravel() - xt)


def test_ordered_subsets_partition_the_projections():
    from paper_2609_30166_amd.projector import ordered_subsets
    for order in ("interleaved", "bitreversal", "contiguous", "random"):
        for n, k in ((720, 10), (13, 4), (5, 5), (7, 1)):
            s = ordered_subsets(n, k, order)
            assert len(s) == k
            flat = sorted(v for part in s for v in part)
            assert flat == list(range(n)), (order, n, k)
    assert ordered_subsets(8, 4)[1] == [1, 5]
    assert ordered_subsets(8, 4, "contiguous")[1] == [2, 3]
    # bit-reversed visiting order of the interleaved subsets: 0, 4, 2, 6, 1, 5, 3, 7
    br = ordered_subsets(16, 8, "bitreversal")
    assert [part[0] for part in br] == [0, 4, 2, 6, 1, 5, 3, 7]
    assert [part[0] for part in ordered_subsets(30, 6, "bitreversal")] == [0, 4, 2, 1, 5, 3]
    with pytest.raises(ValueError):
        ordered_subsets(4, 5)


def test_weighted_backprojection_equals_diagonal_weight_iteration():
    """Weighted backprojection (Sec. 3.2): x <- x + a C W A^T R (b - A x) with a
    diagonal W; weight 0 keeps the reference value, weight 1 everywhere is SIRT."""
    P, A = _problem()
    rng = np.random.default_rng(10)
    b = rng.uniform(0, 3, A.shape[0])
    x0 = rng.uniform(0, 1, A.shape[1])
    w = rng.uniform(0, 1, A.shape[1])
    w[:8] = 0.0
    x, _ = oracle.sirt(P, SHAPE, N_U, N_V, b, 3, alpha=0.8, x0=x0.reshape(SHAPE),
                       voxel_weights=w.reshape(SHAPE))
    R, C = _recip(A.sum(1)), _recip(A.sum(0))
    xr = x0.copy()
    for _ in range(3):
        xr = xr + 0.8 * C * w * (A.T @ (R * (b - A @ xr)))
    np.testing.assert_allclose(x.ravel(), xr, rtol=1e-10, atol=1e-12)
    np.testing.assert_array_equal(x.ravel()[:8], x0[:8])
    x1, _ = oracle.sirt(P, SHAPE, N_U, N_V, b, 2, voxel_weights=np.ones(SHAPE))
    x2, _ = oracle.sirt(P, SHAPE, N_U, N_V, b, 2)
    np.testing.assert_allclose(x1, x2, rtol=1e-12, atol=1e-15)
