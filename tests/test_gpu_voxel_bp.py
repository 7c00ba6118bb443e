"""The voxel-driven backprojector (the paper's Sec. 4.1 form) on the GPU
against the FP64 oracle, through the C ABI: plain and tilted orbits (the
column fast path and the per-voxel path), sub-views, view lists with
repeats, 16-bit images, ragged tiles, SIRT with it, edge cases."""

import math

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
    y_ref = oracle.forward(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, x.astype(np.float64), cfg.step)
    return cfg, x, g, y_ref


def tilted(P, angle):
    """The orbit seen by an object turned by `angle` about x: P [R 0; 0 1]
    (the depth row then has a z coefficient, so each voxel is projected on
    its own)."""
    c, s = math.cos(angle), math.sin(angle)
    T = np.eye(4)
    T[1:3, 1:3] = [[c, -s], [s, c]]
    return P @ T


def test_voxel_back_tiny_matches_oracle(tiny, dev):
    cfg, x, g, y_ref = tiny
    rng = np.random.default_rng(21)
    s = (y_ref + rng.normal(0, 0.5, y_ref.shape)).astype(np.float32)
    z = g.back_voxel(torch.from_numpy(s).to(dev)).cpu().numpy()
    z_ref = oracle.back_voxel(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, s.astype(np.float64))
    assert rel_l2(z, z_ref) <= TOL
    # one thread sums each voxel in a fixed order: bitwise reproducible
    z2 = g.back_voxel(torch.from_numpy(s).to(dev)).cpu().numpy()
    assert np.array_equal(z, z2)


@pytest.mark.parametrize("angle", [0.0, 0.3])
@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16, torch.float16])
def test_voxel_back_ragged_subviews_truncated(dev, angle, dtype):
    """Volume sides off the 16 x 16 x 8 tiles, two sub-views, a truncated
    detector (borders exercised), repeats in the view list; 16-bit images are
    compared with the oracle on the same rounded values."""
    from paper_2609_30166_amd import Geometry

    shape, n_u, n_v = (21, 37, 45), 48, 40
    P = tilted(synth.circular_cone(24, n_u, n_v, 80.0, 160.0, 1.2, n_sub=2), angle)
    g = Geometry(P, n_u, n_v, shape, 0.5, device=dev)
    views = [5, 0, 23, 5, 11]
    rng = np.random.default_rng(22)
    s = torch.from_numpy(rng.uniform(-1, 1, (5, n_v, n_u)).astype(np.float32)).to(dtype)
    z = g.back_voxel(s.to(dev), views=views).cpu().numpy()
    z_ref = oracle.back_voxel(P, shape, n_u, n_v, s.float().numpy().astype(np.float64),
                              views=views)
    assert np.count_nonzero(z_ref == 0) > 0      # some voxels are seen by no listed view
    assert rel_l2(z, z_ref) <= TOL
    # accumulate onto a non-zero volume
    out = torch.full(shape, 2.0, device=dev)
    g.back_voxel(s.to(dev), views=views, out=out, accumulate=True)
    assert rel_l2(out.cpu().numpy(), z_ref + 2.0) <= TOL


def test_voxel_sirt_matches_oracle(tiny, dev):
    """Eq. (1) with B in place of A^T and C = 1 / (B 1), three iterations,
    then two more from the iterate with the cached weights."""
    cfg, x, g, y_ref = tiny
    b = y_ref.astype(np.float32)
    bt = torch.from_numpy(b).to(dev)
    v = torch.zeros(cfg.shape, dtype=torch.float32, device=dev)
    norms = g.sirt(v, bt, 3, voxel_bp=True)
    v_ref, n_ref = oracle.sirt(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, b.astype(np.float64), 3,
                               step=cfg.step, voxel_bp=True)
    assert rel_l2(v.cpu().numpy(), v_ref) <= TOL
    np.testing.assert_allclose(norms, n_ref, rtol=TOL)
    norms2 = g.sirt(v, bt, 2, voxel_bp=True)
    v_ref2, n_ref2 = oracle.sirt(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, b.astype(np.float64), 2,
                                 step=cfg.step, voxel_bp=True, x0=v_ref)
    assert rel_l2(v.cpu().numpy(), v_ref2) <= TOL
    np.testing.assert_allclose(norms2, n_ref2, rtol=TOL)
    # the exact-transpose SIRT on the same view list keeps its own weights
    w = torch.zeros_like(v)
    g.sirt(w, bt, 1)
    w_ref, _ = oracle.sirt(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, b.astype(np.float64), 1,
                           step=cfg.step)
    assert rel_l2(w.cpu().numpy(), w_ref) <= TOL


def test_voxel_sirt_on_a_tilted_subset_with_subviews(dev):
    from paper_2609_30166_amd import Geometry

    shape, n_u, n_v = (19, 24, 26), 40, 36
    P = tilted(synth.circular_cone(16, n_u, n_v, 60.0, 120.0, 1.0, n_sub=3), 0.25)
    g = Geometry(P, n_u, n_v, shape, 0.5, device=dev)
    views = [1, 4, 9, 12, 15]
    x, _ = make_phantom(make_config("tiny"), seed=5)
    x = np.ascontiguousarray(x[22:41, 20:44, 19:45])
    b = oracle.forward(P, shape, n_u, n_v, x.astype(np.float64), 0.5, views=views)
    v = torch.zeros(shape, dtype=torch.float32, device=dev)
    norms = g.sirt(v, torch.from_numpy(b.astype(np.float32)).to(dev), 2, alpha=0.8,
                   views=views, voxel_bp=True)
    v_ref, n_ref = oracle.sirt(P, shape, n_u, n_v, b.astype(np.float32).astype(np.float64), 2,
                               alpha=0.8, step=0.5, views=views, voxel_bp=True)
    assert rel_l2(v.cpu().numpy(), v_ref) <= TOL
    np.testing.assert_allclose(norms, n_ref, rtol=TOL)


def test_voxel_back_edge_cases(dev):
    from paper_2609_30166_amd import Geometry, CtrexError

    shape = (8, 8, 8)
    P = synth.circular_cone(4, 8, 8, 30.0, 60.0, 1.0)
    g = Geometry(P, 8, 8, shape, device=dev)
    # empty list: overwrite -> zeros, accumulate -> unchanged
    out = torch.full(shape, 3.0, device=dev)
    g.back_voxel(torch.empty((0, 8, 8), device=dev), views=[], out=out)
    assert torch.count_nonzero(out) == 0
    out.fill_(3.0)
    g.back_voxel(torch.empty((0, 8, 8), device=dev), views=[], out=out, accumulate=True)
    assert torch.all(out == 3.0)
    # an all-ones image gives the weight sums B 1 (< views where the border cuts)
    ones = g.back_voxel(torch.ones(g.sino_shape(), device=dev)).cpu().numpy()
    ref = oracle.back_voxel(P, shape, 8, 8, np.ones((4, 8, 8)))
    assert rel_l2(ones, ref) <= TOL
    # a motion field is not supported by this backprojector
    g.set_motion(np.zeros((2, 2, 2, 3), np.float32), np.ones(4))
    with pytest.raises(CtrexError) as e:
        g.back_voxel(torch.ones(g.sino_shape(), device=dev))
    assert e.value.code == -7
    with pytest.raises(CtrexError) as e:
        g.sirt(torch.zeros(shape, device=dev), torch.ones(g.sino_shape(), device=dev), 1,
               voxel_bp=True)
    assert e.value.code == -7
    g.set_motion(None, None)
    # a detector one pixel high cannot be sampled bilinearly
    P1 = synth.circular_cone(4, 8, 1, 30.0, 60.0, 1.0)
    g1 = Geometry(P1, 8, 1, shape, device=dev)
    with pytest.raises(CtrexError) as e:
        g1.back_voxel(torch.ones(g1.sino_shape(), device=dev))
    assert e.value.code == -2
