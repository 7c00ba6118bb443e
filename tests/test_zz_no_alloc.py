"""The allocation-free backprojector (ctrex_back_project_noalloc) against
ctrex_back_project, through the C ABI (needs an MI355X).

The variant keeps its scratch (view list, max |r| cell, per-chunk partial
volumes) in the library's fixed per-device array and runs the direct form of
the brick backprojector (each brick writes its own voxels); the regular entry
point runs the owner form (bricks add into a 64-bit integer volume).  Both
are the same operator summed in fixed point at different scales, so they
agree to about 1e-9 relative; the test holds them to 1e-6 (inside the 1e-5
parity bar) on consecutive calls of different sizes, the array keeping the
previous call's contents in between, and checks each call's reproducibility
bit for bit.
"""

import ctypes

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda", 0)


def _noalloc(g, sino, views=None, out=None, accumulate=False):
    from paper_2609_30166_amd._lib import check, lib

    if out is None:
        out = torch.empty(g.shape, dtype=torch.float32, device=g.device)
    arr = None if views is None else np.ascontiguousarray(views, dtype=np.int32)
    vp = None if arr is None else arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    nv = 0 if arr is None else int(arr.size)
    check(g._ctx, lib().ctrex_back_project_noalloc(
        g._ctx, ctypes.c_void_p(sino.data_ptr()), 0, ctypes.c_void_p(out.data_ptr()),
        1 if accumulate else 0, vp, nv,
        ctypes.c_void_p(torch.cuda.current_stream(g.device).cuda_stream)))
    return out


def _case(dev, shape, n_proj, n_u, n_v, sod, seed):
    from paper_2609_30166_amd import Geometry

    P = synth.circular_cone(n_proj, n_u, n_v, sod, 2 * sod, 1.5)
    g = Geometry(P, n_u, n_v, shape, 0.5, device=dev)
    rng = np.random.default_rng(seed)
    s = torch.from_numpy(rng.normal(size=(n_proj, n_v, n_u)).astype(np.float32)).to(dev)
    return P, g, s


def test_noalloc_matches_back_project_on_consecutive_calls(dev):
    # 1: 64^3 under 60 views (15 projection chunks, each with a partial volume
    #    in the array)
    P, g, s = _case(dev, (64, 64, 64), 60, 64, 64, 200.0, 1)
    z_ref = g.back(s)
    z = _noalloc(g, s)
    torch.cuda.synchronize()
    assert rel_l2(z.cpu().numpy(), z_ref.cpu().numpy()) <= 1e-6
    z_or = oracle.back(P, g.shape, 64, 64, s.cpu().numpy().astype(np.float64))
    assert rel_l2(z.cpu().numpy(), z_or) <= 1e-5
    # 2: a smaller input right after it (ragged 17 x 16 x 33 volume, a view
    #    list with repeats, accumulate into a non-zero volume)
    P2, g2, s2 = _case(dev, (17, 16, 33), 7, 40, 27, 80.0, 2)
    views = [6, 0, 3, 3]
    sv = s2[views].contiguous()
    base = torch.ones(g2.shape, dtype=torch.float32, device=dev)
    z2_ref = g2.back(sv, views=views, out=base.clone(), accumulate=True)
    z2 = _noalloc(g2, sv, views=views, out=base.clone(), accumulate=True)
    torch.cuda.synchronize()
    assert rel_l2(z2.cpu().numpy() - 1.0, z2_ref.cpu().numpy() - 1.0) <= 1e-6
    z2_or = 1.0 + oracle.back(P2, g2.shape, 40, 27, sv.cpu().numpy().astype(np.float64),
                              views=views)
    assert rel_l2(z2.cpu().numpy(), z2_or) <= 1e-5
    # 3: a volume whose partial volumes do not fit the array: fewer chunks,
    #    the same operator up to the rounding of the fixed-point scale
    P3, g3, s3 = _case(dev, (160, 160, 160), 24, 128, 128, 500.0, 3)
    z3_ref = g3.back(s3)
    z3 = _noalloc(g3, s3)
    torch.cuda.synchronize()
    assert rel_l2(z3.cpu().numpy(), z3_ref.cpu().numpy()) <= 1e-6
    # the first case again: the array's leftover contents do not matter
    assert torch.equal(_noalloc(g, s), z)


def test_noalloc_rejects_oversized_view_list(dev):
    from paper_2609_30166_amd._lib import lib

    P, g, s = _case(dev, (16, 16, 16), 4, 16, 16, 60.0, 4)
    views = np.zeros(262145, dtype=np.int32)
    out = torch.full(g.shape, 3.0, device=dev)
    L = lib()
    code = L.ctrex_back_project_noalloc(
        g._ctx, ctypes.c_void_p(s.data_ptr()), 0, ctypes.c_void_p(out.data_ptr()), 0,
        views.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(views.size), None)
    assert code == -2
    assert b"exceeds" in L.ctrex_last_error(g._ctx)
    torch.cuda.synchronize()
    assert bool((out == 3.0).all())
