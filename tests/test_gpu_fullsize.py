"""HIP path vs the oracle at the configurations' full sizes (needs an MI355X).

The oracle cannot redo whole 512^3 x 720 projections in a test, so these
compare sampled projections of runs made in the benchmark's launch
configuration, view subsets, and properties that hold at any size.
"""

import numpy as np
import pytest

import oracle
from synth.configs import make_config, make_phantom
from synth.noise import poisson_log_transform

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL = 1e-5


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda", 0)


@pytest.fixture(scope="module")
def full(dev):
    from paper_2609_30166_amd import Geometry

    cfg = make_config("full")
    x, _ = make_phantom(cfg, seed=0)
    g = Geometry(cfg.P, cfg.n_u, cfg.n_v, cfg.shape, cfg.step, device=dev)
    return cfg, x, g


# Projections 0 and 357 put the source near +x / -x (rays mainly along x: the
# y-fastest gather copy), 180 and 540 near +y / -y (rays mainly along y: the
# x-fastest copy), 90 and 270 on the diagonals (the copy chosen per detector
# tile from its central ray, so both are used within one projection).
FULL_VIEWS = [0, 90, 180, 270, 357, 540]


@pytest.fixture(scope="module")
def full_forward_ref(full):
    cfg, x, g = full
    return oracle.forward(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, x.astype(np.float64), cfg.step,
                          views=FULL_VIEWS)


def test_full_forward_sampled_projections(full, full_forward_ref, dev):
    """All 720 projections in one launch (the benchmark's configuration);
    six projections covering both gather copies against the oracle, each on
    its own and together."""
    cfg, x, g = full
    xt = torch.from_numpy(x).to(dev)
    y = g.forward(xt)
    got = y[FULL_VIEWS].cpu().numpy()
    for k, v in enumerate(FULL_VIEWS):
        assert rel_l2(got[k], full_forward_ref[k]) <= TOL, v
    assert rel_l2(got, full_forward_ref) <= TOL


def test_full_forward_16bit_storage(full, full_forward_ref, dev):
    """BF16 and FP16 volumes at 512^3 through the 16-bit corner-packed
    copies (x- and y-fastest): against the oracle on the same rounded volume
    at 1e-5 with an FP32 sinogram, and against FP64 of the unrounded volume
    within the storage rounding with a 16-bit sinogram."""
    cfg, x, g = full
    xt = torch.from_numpy(x).to(dev)
    for dt, bound in ((torch.bfloat16, 8e-3), (torch.float16, 2e-3)):
        x16 = xt.to(dt)
        y32 = g.forward(x16, views=FULL_VIEWS, out_dtype=torch.float32).cpu().numpy()
        xr = x16.float().cpu().numpy().astype(np.float64)
        ref = oracle.forward(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, xr, cfg.step, views=FULL_VIEWS)
        for k, v in enumerate(FULL_VIEWS):
            assert rel_l2(y32[k], ref[k]) <= TOL, (dt, v)
        y16 = g.forward(x16, views=FULL_VIEWS, out_dtype=dt)
        assert rel_l2(y16.float().cpu().numpy(), full_forward_ref) <= bound, dt


def test_full_back_view_subset(full, dev):
    cfg, x, g = full
    views = [5, 400]
    rng = np.random.default_rng(11)
    s = rng.normal(0.0, 1.0, (2, cfg.n_v, cfg.n_u)).astype(np.float32)
    z = g.back(torch.from_numpy(s).to(dev), views=views).cpu().numpy()
    z_ref = oracle.back(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, s.astype(np.float64), cfg.step,
                        views=views)
    assert rel_l2(z, z_ref) <= TOL


def test_full_voxel_back_sampled_voxels(full, dev):
    """The voxel-driven backprojector over all 720 projections in one launch
    (as in the benchmark's SIRT run), 320 sampled voxels (random, the volume
    corners and centre) against the oracle's per-voxel sums."""
    cfg, x, g = full
    rng = np.random.default_rng(12)
    s = rng.standard_normal((cfg.n_proj, cfg.n_v, cfg.n_u), dtype=np.float32)
    z = g.back_voxel(torch.from_numpy(s).to(dev)).cpu().numpy()
    nz, ny, nx = cfg.shape
    ijk = [rng.integers(0, n, 311) for n in (nx, ny, nz)]
    ijk = np.stack(ijk, 1).tolist()
    ijk += [[i, j, k] for i in (0, nx - 1) for j in (0, ny - 1) for k in (0, nz - 1)]
    ijk.append([nx // 2, ny // 2, nz // 2])
    ijk = np.asarray(ijk)
    ref = oracle.back_voxel_points(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, s, ijk)
    got = z[ijk[:, 2], ijk[:, 1], ijk[:, 0]]
    assert rel_l2(got, ref) <= TOL
    # every sampled voxel to the FP32 accumulation bound of 720 terms
    scale = np.sqrt(cfg.n_proj) * 4.0
    assert np.max(np.abs(got - ref)) <= 1e-5 * scale


def test_full_adjoint_all_projections(full, dev):
    """<A x, y> = <x, A^T y> over all 720 projections at 512^3."""
    cfg, x, g = full
    gen = torch.Generator(device=dev).manual_seed(3)
    xr = torch.randn(cfg.shape, device=dev, generator=gen)
    yr = torch.randn(g.sino_shape(), device=dev, generator=gen)
    Ax = g.forward(xr).double()
    lhs = float((Ax * yr.double()).sum())
    rhs = float((xr.double() * g.back(yr).double()).sum())
    assert abs(lhs - rhs) <= 1e-6 * float(Ax.norm() * yr.double().norm())


def test_full_sirt_residual_decreases(full, dev):
    """Three SIRT iterations at full size: the R-weighted residual of Eq. (1)
    never grows (alpha = 1), and the plain residual falls."""
    cfg, x, g = full
    b = g.forward(torch.from_numpy(x).to(dev))
    v = torch.zeros(cfg.shape, device=dev)
    norms = g.sirt(v, b, 3)
    assert norms[1] < norms[0] and norms[2] < norms[1]


def test_full_sirt_iteration_view_subset(full, dev):
    """One SIRT iteration with a 2-projection subset P_k (R and C from that
    subset) against the oracle."""
    cfg, x, g = full
    views = [90, 450]
    b = oracle.forward(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, x.astype(np.float64), cfg.step,
                       views=views)
    v = torch.zeros(cfg.shape, device=dev)
    norms = g.sirt(v, torch.from_numpy(b.astype(np.float32)).to(dev), 1, views=views)
    v_ref, n_ref = oracle.sirt(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, b, 1, step=cfg.step,
                               views=views)
    assert rel_l2(v.cpu().numpy(), v_ref) <= TOL
    np.testing.assert_allclose(norms, n_ref, rtol=TOL)


def test_helical_warp_subviews_subset(dev):
    """Helical scan with jitter, 4 angular sub-views and the 32^3 warp at the
    real 256^3 x 512x256 size, on a subset of 3 of the 1200 projections."""
    from paper_2609_30166_amd import Geometry

    cfg = make_config("helical")
    x, _ = make_phantom(cfg, seed=0)
    g = Geometry(cfg.P, cfg.n_u, cfg.n_v, cfg.shape, cfg.step, device=dev, U=cfg.U,
                 tau=cfg.tau)
    views = [0, 600, 1199]
    y = g.forward(torch.from_numpy(x).to(dev), views=views).cpu().numpy()
    y_ref, cnt = oracle.forward(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, x.astype(np.float64),
                                cfg.step, views=views, U=cfg.U, tau=cfg.tau, return_count=True)
    assert rel_l2(y, y_ref) <= TOL
    assert g.sample_count(views) == cnt
    rng = np.random.default_rng(12)
    s = rng.normal(size=y_ref.shape).astype(np.float32)
    z = g.back(torch.from_numpy(s).to(dev), views=views).cpu().numpy()
    z_ref = oracle.back(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, s.astype(np.float64), cfg.step,
                        views=views, U=cfg.U, tau=cfg.tau)
    assert rel_l2(z, z_ref) <= TOL


@pytest.fixture(scope="module")
def diff(dev):
    from paper_2609_30166_amd import Geometry

    cfg = make_config("diff")
    x_true, _ = make_phantom(cfg, seed=0)
    g = Geometry(cfg.P, cfg.n_u, cfg.n_v, cfg.shape, cfg.step, device=dev)
    y = g.forward(torch.from_numpy(x_true).to(dev)).cpu().numpy()
    b = poisson_log_transform(y, cfg.extra["I0"], np.random.default_rng([0, 4, 1]))
    x0 = 0.8 * x_true + 0.05 * x_true.max() * np.random.default_rng(5).random(cfg.shape)
    return cfg, g, x0.astype(np.float32), b.astype(np.float32)


def test_tv_matches_oracle(diff, dev):
    cfg, g, x0, b = diff
    xs = x0[:40, 50:83, 60:87].copy()
    val, grad = g.tv(torch.from_numpy(xs).to(dev), eps=1e-5, weight=1.0, grad=True)
    assert val == pytest.approx(oracle.tv(xs.astype(np.float64), 1e-5), rel=1e-6)
    assert rel_l2(grad.cpu().numpy(), oracle.tv_grad(xs.astype(np.float64), 1e-5)) <= TOL


def test_diff_gradient_matches_oracle_on_subset(diff, dev):
    """Autograd gradient of ||A x - b||^2 + 1e-3 TV(x) (36-projection subset)
    against the oracle's 2 A^T (A x - b) + 1e-3 grad TV."""
    from paper_2609_30166_amd import reconstruction_loss

    cfg, g, x0, b = diff
    views = list(range(0, 360, 10))
    xt = torch.from_numpy(x0).to(dev).requires_grad_(True)
    bt = torch.from_numpy(b[views]).to(dev)
    loss = reconstruction_loss(xt, bt, g, lam=1e-3, eps=1e-5, views=views)
    loss.backward()
    xd = x0.astype(np.float64)
    res = oracle.forward(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, xd, cfg.step, views=views) - \
        b[views].astype(np.float64)
    want = 2 * oracle.back(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, res, cfg.step, views=views) + \
        1e-3 * oracle.tv_grad(xd, 1e-5)
    # the residual is about 0.2 A x (x0 = 0.8 x_true + noise), so the FP32
    # projection's error against FP64 (~1e-7 relative) grows about 5-fold in
    # it: within 1e-5
    assert rel_l2(xt.grad.cpu().numpy(), want) <= TOL
    assert float(loss) == pytest.approx(float(np.sum(res * res)) + 1e-3 * oracle.tv(xd, 1e-5),
                                        rel=1e-5)


def test_diff_gradient_central_differences(diff, dev):
    """All 360 projections: autograd gradient against central differences of
    the loss on 64 seeded voxels inside the field of view."""
    from paper_2609_30166_amd import reconstruction_loss

    cfg, g, x0, b = diff
    bt = torch.from_numpy(b).to(dev)
    xt = torch.from_numpy(x0).to(dev).requires_grad_(True)
    reconstruction_loss(xt, bt, g, lam=1e-3).backward()
    grad = xt.grad.cpu().numpy()
    rng = np.random.default_rng(6)
    N = cfg.shape[0]
    picks = []
    while len(picks) < 64:
        i, j, k = rng.integers(N // 4, 3 * N // 4, size=3)
        picks.append((int(i), int(j), int(k)))
    h = 3e-4
    with torch.no_grad():
        base = torch.from_numpy(x0).to(dev)
        for idx in picks:
            xp = base.clone()
            xm = base.clone()
            xp[idx] += h
            xm[idx] -= h
            step = float(xp[idx]) - float(xm[idx])
            fd = (float(reconstruction_loss(xp, bt, g, lam=1e-3)) -
                  float(reconstruction_loss(xm, bt, g, lam=1e-3))) / step
            assert grad[idx] == pytest.approx(fd, rel=1e-3, abs=1e-3 * np.abs(grad).max())


def test_full_cylinder_sampled_views(dev):
    """The aligned cylindrical domain at the benchmark's size: a 256 x 1608 x 512
    polar grid under the 720 x 768^2 scan, all projections in one launch,
    views 0 and 357 against the oracle; the voxel-driven backprojector of two
    views over all 210.8e6 polar voxels against the oracle."""
    from paper_2609_30166_amd import CylinderGeometry
    from synth.phantoms import vial_polar

    cfg = make_config("full")
    cyl = (256, 1608, 512, 1.0, 1.0)
    g = CylinderGeometry(cfg.P, cfg.n_u, cfg.n_v, *cyl, step=cfg.step, device=dev)
    x = vial_polar(256, 1608, 512, 1.0, 1.0, np.random.default_rng(17))
    y = g.forward(torch.from_numpy(x).to(dev))
    views = [0, 357]
    y_ref = oracle.forward_cyl(cfg.P, cyl, cfg.n_u, cfg.n_v, x, cfg.step, views=views)
    assert rel_l2(y[views].cpu().numpy(), y_ref) <= TOL
    del y
    rng = np.random.default_rng(13)
    s = rng.standard_normal((2, cfg.n_v, cfg.n_u), dtype=np.float32)
    z = g.back(torch.from_numpy(s).to(dev), views=[5, 400]).cpu().numpy()
    z_ref = oracle.back_voxel_cyl(cfg.P, cyl, cfg.n_u, cfg.n_v, s, views=[5, 400])
    assert rel_l2(z, z_ref) <= TOL
    g.close()
