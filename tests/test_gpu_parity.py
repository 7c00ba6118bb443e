"""HIP path vs the CPU FP64 oracle through the C ABI (needs an MI355X).

Bar: FP32 results within relative L2 1e-5 of the FP64 oracle on the same
seeded inputs; integer results (sample counts) exact; error statuses exact.
"""

import ctypes

import numpy as np
import pytest

import oracle
import synth
from synth.configs import make_config, make_phantom

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
def tiny(dev):
    from paper_2609_30166_amd import Geometry

    cfg = make_config("tiny")
    x, _ = make_phantom(cfg, seed=0)
    g = Geometry(cfg.P, cfg.n_u, cfg.n_v, cfg.shape, cfg.step, device=dev)
    y_ref, n_ref = oracle.forward(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, x.astype(np.float64),
                                  cfg.step, return_count=True)
    return cfg, x, g, y_ref, n_ref


def test_forward_tiny_matches_oracle(tiny, dev):
    cfg, x, g, y_ref, _ = tiny
    y = g.forward(torch.from_numpy(x).to(dev)).cpu().numpy()
    assert rel_l2(y, y_ref) <= TOL


def test_sample_count_is_exact(tiny):
    cfg, x, g, _, n_ref = tiny
    assert g.sample_count() == n_ref
    assert g.sample_count(views=[3, 7]) == oracle.forward(
        cfg.P, cfg.shape, cfg.n_u, cfg.n_v, np.zeros(cfg.shape), cfg.step, views=[3, 7],
        return_count=True)[1]


def test_back_tiny_matches_oracle(tiny, dev):
    cfg, x, g, y_ref, _ = tiny
    rng = np.random.default_rng(1)
    s = (y_ref + rng.normal(0, 0.5, y_ref.shape)).astype(np.float32)
    z = g.back(torch.from_numpy(s).to(dev)).cpu().numpy()
    z_ref = oracle.back(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, s.astype(np.float64), cfg.step)
    assert rel_l2(z, z_ref) <= TOL


def test_back_accumulates(tiny, dev):
    cfg, x, g, y_ref, _ = tiny
    s = torch.from_numpy(y_ref.astype(np.float32)).to(dev)
    z1 = g.back(s)
    z2 = torch.ones_like(z1)
    g.back(s, out=z2, accumulate=True)
    np.testing.assert_allclose(z2.cpu().numpy(), z1.cpu().numpy() + 1.0, rtol=TOL, atol=1e-5)


def test_sirt_five_iterations_match_oracle(tiny, dev):
    cfg, x, g, y_ref, _ = tiny
    b = y_ref.astype(np.float32)
    v = torch.zeros(cfg.shape, dtype=torch.float32, device=dev)
    norms = g.sirt(v, torch.from_numpy(b).to(dev), 5)
    v_ref, n_ref = oracle.sirt(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, b.astype(np.float64), 5,
                               step=cfg.step)
    assert rel_l2(v.cpu().numpy(), v_ref) <= TOL
    np.testing.assert_allclose(norms, n_ref, rtol=TOL)
    # a second call continues from the iterate, reusing the cached weights
    norms2 = g.sirt(v, torch.from_numpy(b).to(dev), 2)
    v_ref2, n_ref2 = oracle.sirt(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, b.astype(np.float64), 2,
                                 step=cfg.step, x0=v_ref)
    assert rel_l2(v.cpu().numpy(), v_ref2) <= TOL
    np.testing.assert_allclose(norms2, n_ref2, rtol=TOL)


def test_adjoint_dot_product_on_gpu(tiny, dev):
    cfg, x, g, _, _ = tiny
    rng = np.random.default_rng(2)
    xr = torch.from_numpy(rng.normal(size=cfg.shape).astype(np.float32)).to(dev)
    yr = torch.from_numpy(rng.normal(size=(cfg.n_proj, cfg.n_v, cfg.n_u)).astype(np.float32)).to(dev)
    Ax = g.forward(xr).double()
    lhs = float((Ax * yr.double()).sum())
    rhs = float((xr.double() * g.back(yr).double()).sum())
    # random signs cancel in the sums, so normalise by ||A x|| ||y|| (Cauchy-Schwarz)
    scale = float(Ax.norm() * yr.double().norm())
    assert abs(lhs - rhs) <= 1e-6 * scale


@pytest.mark.parametrize("n_u,n_v,shape", [(37, 23, (21, 26, 30)), (16, 16, (2, 2, 2)),
                                           (1, 1, (9, 9, 9)), (70, 9, (40, 12, 17))])
def test_ragged_tiles_and_odd_volumes(dev, n_u, n_v, shape):
    from paper_2609_30166_amd import Geometry

    P = synth.circular_cone(7, n_u, n_v, 60.0, 110.0, 0.9, arc=4.0, det_offset_u=1.3)
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, shape).astype(np.float32)
    g = Geometry(P, n_u, n_v, shape, 0.5, device=dev)
    y = g.forward(torch.from_numpy(x).to(dev)).cpu().numpy()
    y_ref = oracle.forward(P, shape, n_u, n_v, x.astype(np.float64))
    assert rel_l2(y, y_ref) <= TOL
    s = rng.normal(size=y_ref.shape).astype(np.float32)
    z = g.back(torch.from_numpy(s).to(dev)).cpu().numpy()
    z_ref = oracle.back(P, shape, n_u, n_v, s.astype(np.float64))
    assert rel_l2(z, z_ref) <= TOL


def test_tube_gather_is_bitwise_the_direct_gather(tiny, dev, monkeypatch):
    """The LDS-staged tube gather (CTREX_FP_GATHER=lds, read when the context
    is created) walks the same samples with the same arithmetic as the direct
    gather: bitwise equal forward projections, plain and in the SIRT modes,
    and the oracle's at 1e-5; also on a ragged volume and detector."""
    from paper_2609_30166_amd import Geometry

    cfg, x, g, y_ref, _ = tiny
    xt = torch.from_numpy(x).to(dev)
    monkeypatch.setenv("CTREX_FP_GATHER", "lds")
    gt = Geometry(cfg.P, cfg.n_u, cfg.n_v, cfg.shape, cfg.step, device=dev)
    monkeypatch.delenv("CTREX_FP_GATHER")
    y1 = g.forward(xt)
    y2 = gt.forward(xt)
    assert torch.equal(y1, y2)
    assert rel_l2(y2.cpu().numpy(), y_ref) <= TOL
    b = torch.from_numpy(y_ref.astype(np.float32)).to(dev) * 1.01
    v1 = torch.zeros_like(xt)
    v2 = torch.zeros_like(xt)
    n1 = g.sirt(v1, b, 2)
    n2 = gt.sirt(v2, b, 2)
    assert torch.equal(v1, v2)
    np.testing.assert_array_equal(np.asarray(n1), np.asarray(n2))
    shape = (21, 26, 30)
    P = synth.circular_cone(7, 37, 23, 60.0, 110.0, 0.9, arc=4.0, det_offset_u=1.3)
    xr = np.random.default_rng(3).uniform(0, 1, shape).astype(np.float32)
    monkeypatch.setenv("CTREX_FP_GATHER", "lds")
    gr = Geometry(P, 37, 23, shape, 0.5, device=dev)
    monkeypatch.delenv("CTREX_FP_GATHER")
    yr = gr.forward(torch.from_numpy(xr).to(dev)).cpu().numpy()
    assert rel_l2(yr, oracle.forward(P, shape, 37, 23, xr.astype(np.float64))) <= TOL


def test_interior_bricks_match_oracle(dev):
    """A volume large enough that some 32 x 16 x 16 backprojection bricks
    touch no face (x0 >= 1 and x0 + e <= n - 2 on every axis): these walk
    their samples without the corner clamps, and their lanes hand rays over
    to each other as in any brick.  Against the oracle at 1e-5."""
    from paper_2609_30166_amd import Geometry

    shape = (100, 52, 52)
    P = synth.circular_cone(12, 64, 48, 180.0, 360.0, 1.6, arc=3.0, det_offset_u=0.7)
    rng = np.random.default_rng(5)
    g = Geometry(P, 64, 48, shape, 0.5, device=dev)
    s = rng.normal(size=(12, 48, 64)).astype(np.float32)
    z = g.back(torch.from_numpy(s).to(dev)).cpu().numpy()
    z_ref = oracle.back(P, shape, 64, 48, s.astype(np.float64))
    assert rel_l2(z, z_ref) <= TOL
    # the interior voxels alone (bricks 1-2 on each axis), so that an error
    # there cannot hide in the norm of the whole volume
    sl = (slice(33, 95), slice(17, 47), slice(17, 47))
    assert rel_l2(z[sl], z_ref[sl]) <= TOL


def test_view_subsets_with_repeats_and_empty(tiny, dev):
    cfg, x, g, y_ref, _ = tiny
    views = [59, 0, 17, 17, 30]
    xt = torch.from_numpy(x).to(dev)
    y = g.forward(xt, views=views).cpu().numpy()
    assert rel_l2(y, y_ref[views]) <= TOL
    empty = g.forward(xt, views=[])
    assert empty.shape == (0, cfg.n_v, cfg.n_u)
    z = g.back(torch.zeros((0, cfg.n_v, cfg.n_u), device=dev), views=[])
    assert float(z.abs().max()) == 0.0
    s = y_ref[views].astype(np.float32)
    zb = g.back(torch.from_numpy(s).to(dev), views=views).cpu().numpy()
    z_ref = oracle.back(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, s.astype(np.float64), views=views)
    assert rel_l2(zb, z_ref) <= TOL


def _helical_small(warp):
    shape = (24, 28, 32)
    n_u, n_v = 48, 20
    rng = np.random.default_rng(4)
    P = synth.helical_cone(10, n_u, n_v, 90.0, 180.0, 1.5, 3.0, 6.0, n_sub=4)
    P = synth.rigid_jitter(P, 0.5, 0.2, rng)
    U = tau = None
    if warp:
        U = synth.smooth_displacement(6, 2.5, rng)
        tau = synth.exposure_time_fractions(10, 4)
    return shape, n_u, n_v, P, U, tau


@pytest.mark.parametrize("warp", [False, True])
def test_subviews_and_warp_match_oracle(dev, warp):
    from paper_2609_30166_amd import Geometry

    shape, n_u, n_v, P, U, tau = _helical_small(warp)
    rng = np.random.default_rng(5)
    ells = synth.random_ellipsoids(5, shape, (3.0, 8.0), (0.1, 1.0), rng, fov_radius=10.0)
    x = synth.voxelise_ellipsoids(ells, shape).astype(np.float32)
    g = Geometry(P, n_u, n_v, shape, 0.5, device=dev, U=U, tau=tau)
    y = g.forward(torch.from_numpy(x).to(dev)).cpu().numpy()
    y_ref, cnt = oracle.forward(P, shape, n_u, n_v, x.astype(np.float64), U=U, tau=tau,
                                return_count=True)
    assert rel_l2(y, y_ref) <= TOL
    assert g.sample_count() == cnt
    s = (y_ref + rng.normal(0, 0.2, y_ref.shape)).astype(np.float32)
    z = g.back(torch.from_numpy(s).to(dev)).cpu().numpy()
    z_ref = oracle.back(P, shape, n_u, n_v, s.astype(np.float64), U=U, tau=tau)
    assert rel_l2(z, z_ref) <= TOL
    v = torch.zeros(shape, dtype=torch.float32, device=dev)
    norms = g.sirt(v, torch.from_numpy(y_ref.astype(np.float32)).to(dev), 3)
    v_ref, n_ref = oracle.sirt(P, shape, n_u, n_v, y_ref, 3, U=U, tau=tau)
    assert rel_l2(v.cpu().numpy(), v_ref) <= TOL
    np.testing.assert_allclose(norms, n_ref, rtol=TOL)
    if warp:
        g.set_motion(None, None)
        y0 = g.forward(torch.from_numpy(x).to(dev)).cpu().numpy()
        assert rel_l2(y0, oracle.forward(P, shape, n_u, n_v, x.astype(np.float64))) <= TOL


@pytest.mark.parametrize("dtype,bound", [("bfloat16", 8e-3), ("float16", 1e-3)])
def test_16bit_storage_error_against_fp64(tiny, dev, dtype, bound):
    """Storage precision extension: 16-bit volume and sinogram, FP32 arithmetic.
    The error against FP64 is dominated by the output rounding (2^-9 for BF16,
    2^-12 for FP16 relative, per value)."""
    cfg, x, g, y_ref, _ = tiny
    dt = getattr(torch, dtype)
    x16 = torch.from_numpy(x).to(dev).to(dt)
    y16 = g.forward(x16, out_dtype=dt).float().cpu().numpy()
    err = rel_l2(y16, y_ref)
    assert err <= bound
    # the 16-bit gather itself (FP32 output) equals FP64 projection of the rounded volume
    y32 = g.forward(x16).cpu().numpy()
    xr = x16.float().cpu().numpy().astype(np.float64)
    assert rel_l2(y32, oracle.forward(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, xr, cfg.step)) <= TOL
    # SIRT with the 16-bit shadow converges like FP32 within the storage error
    b = torch.from_numpy(y_ref.astype(np.float32)).to(dev).to(dt)
    v = torch.zeros(cfg.shape, dtype=torch.float32, device=dev)
    n16 = g.sirt(v, b, 5, gather_dtype=dt)
    v_ref, n_ref = oracle.sirt(cfg.P, cfg.shape, cfg.n_u, cfg.n_v,
                               b.float().cpu().numpy().astype(np.float64), 5, step=cfg.step)
    assert rel_l2(v.cpu().numpy(), v_ref) <= 4 * bound
    assert n16[-1] < n16[0]


def test_conversion_rounds_to_nearest_even(tiny, dev):
    cfg, x, g, _, _ = tiny
    vals = torch.tensor([1.0, 1.00390625, 1.01171875, -3.3, 65504.0, 1e-8, 0.0],
                        dtype=torch.float32, device=dev)
    for dt in (torch.bfloat16, torch.float16):
        got = g.convert(vals, dt)
        assert torch.equal(got.cpu(), vals.cpu().to(dt))


def test_autograd_gradient_is_exact_transpose(tiny, dev):
    """Autograd through the projector (backward = the exact-transpose
    backprojector) against the oracle's 2 A^T (A x - b).  The residual is
    0.2 A x here, so the FP32 projection's relative error (~1e-7 against
    FP64) grows 5.5-fold in it: well inside 1e-5."""
    from paper_2609_30166_amd import project

    cfg, x, g, y_ref, _ = tiny
    b = torch.from_numpy((y_ref * 0.9).astype(np.float32)).to(dev)
    xt = torch.from_numpy(x * 1.1).to(dev).requires_grad_(True)
    loss = ((project(xt, g) - b) ** 2).sum()
    loss.backward()
    res = oracle.forward(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, x.astype(np.float64) * 1.1) - \
        (y_ref * 0.9).astype(np.float32).astype(np.float64)
    want = 2 * oracle.back(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, res)
    assert rel_l2(xt.grad.cpu().numpy(), want) <= TOL


def test_data_term_and_gradient_from_library(tiny, dev):
    """``data_term`` (the library's residual epilogue and scaled
    backprojector): value sum (A x - b)^2 and gradient 2 A^T (A x - b)
    against the oracle, on all projections and on a subset with repeats."""
    from paper_2609_30166_amd import data_term

    cfg, x, g, y_ref, _ = tiny
    b32 = (y_ref * 0.9).astype(np.float32)
    for views in (None, [3, 17, 17, 41, 59]):
        bsel = b32 if views is None else b32[views]
        xt = torch.from_numpy(x * 1.1).to(dev).requires_grad_(True)
        loss = data_term(xt, torch.from_numpy(bsel).to(dev), g, views)
        assert loss.dtype == torch.float64 and loss.device == xt.device
        loss.backward()
        res = oracle.forward(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, x.astype(np.float64) * 1.1,
                             views=views) - bsel.astype(np.float64)
        want = 2 * oracle.back(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, res, views=views)
        assert rel_l2(xt.grad.cpu().numpy(), want) <= TOL, views
        assert float(loss) == pytest.approx(float(np.sum(res * res)), rel=TOL), views


def test_data_residual_scaled_and_backprojection_scaled(tiny, dev):
    """r = scale (A x - b) from the correction epilogue; the scaled
    backprojector: bitwise twice the plain one for scale 2 (the fixed-point
    scale absorbs the power of two), and within rounding for 0.37; an empty
    view list zeroes the sum."""
    cfg, x, g, y_ref, _ = tiny
    xt = torch.from_numpy(x).to(dev)
    bt = torch.from_numpy((y_ref * 0.8).astype(np.float32)).to(dev)
    r, s = g.data_residual(xt, bt, scale=-3.0)
    want = -3.0 * (oracle.forward(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, x.astype(np.float64)) -
                   bt.cpu().numpy().astype(np.float64))
    assert rel_l2(r.cpu().numpy(), want) <= TOL
    assert float(s) == pytest.approx(float(np.sum((want / 3.0) ** 2)), rel=TOL)
    r_only, none = g.data_residual(xt, bt, scale=1.0, sq_sum=False)
    assert none is None
    s_only = g.data_residual(xt, bt, residual=False)[1]
    assert float(s_only) == pytest.approx(float(s), rel=1e-12)
    rng = np.random.default_rng(9)
    y = torch.from_numpy(rng.normal(size=g.sino_shape()).astype(np.float32)).to(dev)
    z1 = g.back(y)
    assert torch.equal(g.back(y, scale=2.0), 2.0 * z1)
    z37 = g.back(y, scale=0.37).cpu().numpy()
    assert rel_l2(z37, 0.37 * z1.cpu().numpy().astype(np.float64)) <= 1e-6
    e = torch.full((1, cfg.n_v, cfg.n_u), 5.0, device=dev)[:0]
    _, s0 = g.data_residual(xt, e.reshape(0, cfg.n_v, cfg.n_u), views=[])
    assert float(s0) == 0.0


def test_calls_need_attached_scratch(tiny, dev):
    """Without caller scratch the projector calls fail before launching
    (CTREX_EWORKSPACE, message with the size); with ctrex_scratch_bytes'
    size attached they run."""
    from paper_2609_30166_amd._lib import lib

    cfg, x, g, _, _ = tiny
    L = lib()
    ctx = ctypes.c_void_p()
    assert L.ctrex_create(ctypes.byref(ctx), 0) == 0
    P = np.ascontiguousarray(cfg.P, np.float64)
    nz, ny, nx = cfg.shape
    assert L.ctrex_set_geometry(ctx, P.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                cfg.n_proj, 1, cfg.n_u, cfg.n_v, nx, ny, nz, cfg.step) == 0
    xt = torch.from_numpy(x).to(dev)
    y = torch.full((cfg.n_proj, cfg.n_v, cfg.n_u), -1.0, device=dev)
    args = (ctypes.c_void_p(xt.data_ptr()), 0, ctypes.c_void_p(y.data_ptr()), 0, None, 0, None)
    assert L.ctrex_forward_project(ctx, *args) == -6
    assert b"scratch" in L.ctrex_last_error(ctx)
    torch.cuda.synchronize()
    assert float(y.min()) == -1.0 and float(y.max()) == -1.0   # nothing launched
    n = ctypes.c_size_t()
    assert L.ctrex_scratch_bytes(ctx, 0, ctypes.byref(n)) == 0
    assert n.value >= 36 * x.size
    small = torch.empty(n.value // 2, dtype=torch.uint8, device=dev)
    assert L.ctrex_set_scratch(ctx, ctypes.c_void_p(small.data_ptr()), small.numel()) == 0
    assert L.ctrex_forward_project(ctx, *args) == -6
    scr = torch.empty(n.value, dtype=torch.uint8, device=dev)
    assert L.ctrex_set_scratch(ctx, ctypes.c_void_p(scr.data_ptr()), scr.numel()) == 0
    assert L.ctrex_forward_project(ctx, *args) == 0
    torch.cuda.synchronize()
    assert rel_l2(y.cpu().numpy(), g.forward(xt).cpu().numpy()) == 0.0
    assert L.ctrex_set_scratch(ctx, None, 5) == -1
    # a pointer off the 256-byte alignment is refused (its 16-byte partial
    # sums would be misaligned)
    assert L.ctrex_set_scratch(ctx, ctypes.c_void_p(scr.data_ptr() + 8), scr.numel() - 8) == -1
    assert L.ctrex_set_scratch(ctx, None, 0) == 0
    L.ctrex_destroy(ctx)


def test_error_statuses(dev):
    from paper_2609_30166_amd import Geometry, CtrexError
    from paper_2609_30166_amd._lib import lib

    shape = (8, 8, 8)
    P = synth.circular_cone(4, 8, 8, 30.0, 60.0, 1.0)
    bad = P.copy()
    bad[2, 0, :, :3] = 0
    with pytest.raises(CtrexError) as e:
        Geometry(bad, 8, 8, shape, device=dev)
    assert e.value.code == -3
    inside = synth.view_matrix([0.5, 0, 0], [-30, 0, 0], [0, 1, 0], [0, 0, 1], 1, 1, 8, 8)
    with pytest.raises(CtrexError) as e:
        Geometry(inside[None, None], 8, 8, shape, device=dev)
    assert e.value.code == -4
    with pytest.raises(CtrexError) as e:
        Geometry(P, 8, 8, (1, 8, 8), device=dev)
    assert e.value.code == -2
    g = Geometry(P, 8, 8, shape, device=dev)
    x = torch.zeros(shape, device=dev)
    with pytest.raises(CtrexError) as e:
        g.forward(x, views=[0, 4])
    assert e.value.code == -2
    ws = torch.empty(16, dtype=torch.uint8, device=dev)
    with pytest.raises(CtrexError) as e:
        g.sirt(x, torch.zeros(g.sino_shape(), device=dev), 1, workspace=ws)
    assert e.value.code == -6
    # a context without geometry
    L = lib()
    ctx = ctypes.c_void_p()
    assert L.ctrex_create(ctypes.byref(ctx), 0) == 0
    cnt = ctypes.c_int64()
    assert L.ctrex_sample_count(ctx, None, 0, ctypes.byref(cnt), None) == -7
    assert b"geometry" in L.ctrex_last_error(ctx)
    L.ctrex_destroy(ctx)
    # non-finite residuals are reported
    b = torch.full(g.sino_shape(), float("nan"), device=dev)
    with pytest.raises(CtrexError) as e:
        g.sirt(x, b, 1)
    assert e.value.code == -8


def test_backprojection_is_bitwise_reproducible(tiny, dev):
    """The brick accumulators sum fixed-point integers, so the order of the
    atomics cannot change the result (one projection chunk per brick)."""
    from paper_2609_30166_amd import Geometry

    shape = (48, 40, 64)
    P = synth.circular_cone(24, 48, 40, 150.0, 300.0, 1.5)
    g = Geometry(P, 48, 40, shape, 0.5, device=dev)
    rng = np.random.default_rng(7)
    s = torch.from_numpy(rng.normal(size=(24, 40, 48)).astype(np.float32)).to(dev)
    z1 = g.back(s)
    z2 = g.back(s)
    assert torch.equal(z1, z2)
    z_ref = oracle.back(P, shape, 48, 40, s.cpu().numpy().astype(np.float64))
    assert rel_l2(z1.cpu().numpy(), z_ref) <= TOL


def test_backprojection_propagates_nan(tiny, dev):
    cfg, x, g, y_ref, _ = tiny
    s = torch.from_numpy(y_ref.astype(np.float32)).to(dev)
    s[3, 10, 10] = float("nan")
    z = g.back(s)
    assert torch.isnan(z).any()


def test_residual_norm_matches_oracle(tiny, dev):
    """||b - A x|| from the library equals the oracle's (FP64 sum of FP32
    residuals versus FP64 throughout: relative 1e-5), on all views, a subset
    and bf16 storage of the sinogram."""
    cfg, x, g, y_ref, _ = tiny
    rng = np.random.default_rng(5)
    b = (y_ref + rng.normal(0, 0.3, y_ref.shape)).astype(np.float32)
    want = float(np.linalg.norm(b.astype(np.float64) - y_ref))
    got = g.residual_norm(torch.from_numpy(x).to(dev), torch.from_numpy(b).to(dev))
    assert abs(got - want) <= TOL * want
    views = [2, 9, 31]
    bs = np.ascontiguousarray(b[views])
    got_s = g.residual_norm(torch.from_numpy(x).to(dev), torch.from_numpy(bs).to(dev), views=views)
    want_s = float(np.linalg.norm(bs.astype(np.float64) - y_ref[views]))
    assert abs(got_s - want_s) <= TOL * want_s
    bb = torch.from_numpy(b).to(dev).bfloat16()
    want_b = float(np.linalg.norm(bb.double().cpu().numpy() - y_ref))
    got_b = g.residual_norm(torch.from_numpy(x).to(dev), bb)
    assert abs(got_b - want_b) <= TOL * want_b
    # the residual of the exact projection is zero up to FP32 rounding
    y = g.forward(torch.from_numpy(x).to(dev))
    assert g.residual_norm(torch.from_numpy(x).to(dev), y) <= 1e-6 * np.linalg.norm(y_ref)
    empty = torch.zeros((0, cfg.n_v, cfg.n_u), dtype=torch.float32, device=dev)
    assert g.residual_norm(torch.from_numpy(x).to(dev), empty, views=[]) == 0.0


def test_os_sirt_matches_oracle(tiny, dev):
    """Ordered subsets (4 interleaved subsets, 2 epochs = 8 updates) against
    the oracle; subset weights are cached per workspace and stay valid while
    the subsets cycle."""
    from paper_2609_30166_amd import ordered_subsets
    cfg, x, g, y_ref, _ = tiny
    subsets = ordered_subsets(cfg.n_proj, 4)
    b = torch.from_numpy(y_ref.astype(np.float32)).to(dev)
    vol = torch.zeros(cfg.shape, dtype=torch.float32, device=dev)
    norms = g.os_sirt(vol, b, subsets, 2, norms=True)
    x_ref, n_ref = oracle.os_sirt(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, y_ref, subsets, 2,
                                  step=cfg.step)
    assert rel_l2(vol.cpu().numpy(), x_ref) <= TOL
    np.testing.assert_allclose(norms, n_ref, rtol=TOL)
    # one subset holding every projection is plain SIRT, bit for bit
    v1 = torch.zeros_like(vol)
    g.os_sirt(v1, b, [list(range(cfg.n_proj))], 2)
    v2 = torch.zeros_like(vol)
    g.sirt(v2, b, 2, views=list(range(cfg.n_proj)), norms=False)
    assert torch.equal(v1, v2)


def test_weighted_backprojection_matches_oracle(tiny, dev):
    """Voxel weights in [0, 1] (zero in a slab) from a reference volume: 3
    weighted SIRT updates against the oracle; zero-weight voxels keep their
    reference values bit for bit."""
    cfg, x, g, y_ref, _ = tiny
    rng = np.random.default_rng(11)
    w = rng.uniform(0, 1, cfg.shape).astype(np.float32)
    w[:, :, :10] = 0.0
    ref = (0.7 * x).astype(np.float32)
    b = torch.from_numpy(y_ref.astype(np.float32)).to(dev)
    vol = torch.from_numpy(ref.copy()).to(dev)
    g.set_voxel_weights(torch.from_numpy(w).to(dev))
    try:
        g.sirt(vol, b, 3, norms=False, recompute_weights=True)
    finally:
        g.set_voxel_weights(None)
    want, _ = oracle.sirt(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, y_ref, 3, step=cfg.step,
                          x0=ref.astype(np.float64), voxel_weights=w.astype(np.float64))
    got = vol.cpu().numpy()
    assert rel_l2(got, want) <= TOL
    np.testing.assert_array_equal(got[:, :, :10], ref[:, :, :10])
    # without weights the same call is plain SIRT again
    v2 = torch.from_numpy(ref.copy()).to(dev)
    g.sirt(v2, b, 1, norms=False)
    want2, _ = oracle.sirt(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, y_ref, 1, step=cfg.step,
                           x0=ref.astype(np.float64))
    assert rel_l2(v2.cpu().numpy(), want2) <= TOL


def test_one_voxel_edge_bricks(dev):
    """Volume sides 32 + 1, 15 + 1 and 16 + 1 voxels: the backprojector's last
    brick along every axis is one voxel thick, so its halo cells in x and y
    and its clamped planes in z are all exercised.  Forward, back and two
    SIRT iterations (which also build the weight sums) against the oracle."""
    from paper_2609_30166_amd import Geometry

    shape, n_u, n_v = (17, 16, 33), 80, 40
    P = synth.circular_cone(9, n_u, n_v, 60.0, 110.0, 0.9, arc=5.0, det_offset_u=0.7)
    rng = np.random.default_rng(11)
    x = rng.uniform(0, 1, shape).astype(np.float32)
    g = Geometry(P, n_u, n_v, shape, 0.5, device=dev)
    y = g.forward(torch.from_numpy(x).to(dev)).cpu().numpy()
    y_ref = oracle.forward(P, shape, n_u, n_v, x.astype(np.float64))
    assert rel_l2(y, y_ref) <= TOL
    s = rng.normal(size=y_ref.shape).astype(np.float32)
    z = g.back(torch.from_numpy(s).to(dev)).cpu().numpy()
    z_ref = oracle.back(P, shape, n_u, n_v, s.astype(np.float64))
    # the one-voxel slabs receive rays
    assert np.abs(z_ref[16]).sum() > 0 and np.abs(z_ref[:, 15]).sum() > 0
    assert np.abs(z_ref[:, :, 32]).sum() > 0
    assert rel_l2(z, z_ref) <= TOL
    for sl in (np.s_[16], np.s_[:, 15], np.s_[:, :, 32]):
        assert rel_l2(z[sl], z_ref[sl]) <= TOL
    b = y_ref.astype(np.float32)
    v = torch.zeros(shape, dtype=torch.float32, device=dev)
    norms = g.sirt(v, torch.from_numpy(b).to(dev), 2)
    v_ref, n_ref = oracle.sirt(P, shape, n_u, n_v, b.astype(np.float64), 2)
    assert rel_l2(v.cpu().numpy(), v_ref) <= TOL
    np.testing.assert_allclose(norms, n_ref, rtol=TOL)


@pytest.mark.parametrize("dtype", ["bfloat16", "float16"])
def test_16bit_gather_sirt_first_iteration_exact(tiny, dev, dtype):
    """SIRT with a 16-bit gather, started from a volume that 16 bits hold
    exactly: the first iteration's rays see no rounding, so its increment and
    residual norm equal the FP64 oracle's (FP32 data, FP32 update)."""
    cfg, x, g, y_ref, _ = tiny
    dt = getattr(torch, dtype)
    x0 = torch.from_numpy(0.5 * x).to(dev).to(dt).float()
    b = y_ref.astype(np.float32)
    v = x0.clone()
    norms = g.sirt(v, torch.from_numpy(b).to(dev), 1, gather_dtype=dt)
    x0d = x0.cpu().numpy().astype(np.float64)
    v_ref, n_ref = oracle.sirt(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, b.astype(np.float64), 1,
                               step=cfg.step, x0=x0d)
    assert rel_l2(v.cpu().numpy() - x0d, v_ref - x0d) <= TOL
    np.testing.assert_allclose(norms, n_ref, rtol=TOL)


@pytest.mark.parametrize("dtype", ["bfloat16", "float16"])
def test_residual_norm_of_a_16bit_volume(tiny, dev, dtype):
    """||b - A x|| with the volume stored in 16 bits: the rays gather the
    16-bit values exactly, so the norm equals the oracle's for the rounded
    volume (relative 1e-5)."""
    cfg, x, g, y_ref, _ = tiny
    dt = getattr(torch, dtype)
    x16 = torch.from_numpy(x).to(dev).to(dt)
    xr = x16.float().cpu().numpy().astype(np.float64)
    y_r = oracle.forward(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, xr, cfg.step)
    b = (y_ref + np.random.default_rng(8).normal(0, 0.3, y_ref.shape)).astype(np.float32)
    want = float(np.linalg.norm(b.astype(np.float64) - y_r))
    got = g.residual_norm(x16, torch.from_numpy(b).to(dev))
    assert abs(got - want) <= TOL * want
