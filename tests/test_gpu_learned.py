"""The learned-correction pipeline on the GPU: the residual acceptance rule
and its plain-SIRT fallback, training checkpoint/resume, and what the trained
network gains over SIRT without it."""

import os

import numpy as np
import pytest
import torch

from synth.configs import make_config, make_phantom

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2609_30166_amd", "weights", "unet_learned_256.npz")


@pytest.fixture(scope="module")
def tiny():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2609_30166_amd import Geometry

    cfg = make_config("tiny")
    x, _ = make_phantom(cfg, seed=3)
    dev = torch.device("cuda", 0)
    g = Geometry(cfg.P, cfg.n_u, cfg.n_v, cfg.shape, cfg.step, device=dev)
    xt = torch.from_numpy(x).to(dev)
    b = g.forward(xt)
    return cfg, g, xt, b


def _net(head_std, seed=0, scale=1.0):
    from paper_2609_30166_amd.unet import UNet
    return UNet("cuda:0", seed=seed, head_std=head_std, scale=scale)


def test_broken_network_falls_back_to_plain_sirt(tiny):
    """A network with an absurd head makes the data residual worse, so the
    first correction is rejected and the result is plain SIRT, bit for bit."""
    from paper_2609_30166_amd.learned import LearnedSirt
    cfg, g, xt, b = tiny
    net = _net(head_std=50.0)
    x, stages = LearnedSirt(g, net, n_stages=4)(b)
    assert not stages[0]["corrected"] and stages[0]["fallback"]
    assert stages[0]["rho_corrected"] > stages[0]["rho_sirt"]
    assert all(s["fallback"] and not s["corrected"] for s in stages[1:])
    ref = torch.zeros_like(x)
    g.sirt(ref, b, 4, norms=False)
    assert torch.equal(x, ref)


def test_identity_network_is_kept_and_changes_nothing(tiny):
    """With a zero head x + U(x) = x: the residual does not grow, every
    correction is kept, and the result is plain SIRT."""
    from paper_2609_30166_amd.learned import LearnedSirt
    cfg, g, xt, b = tiny
    net = _net(head_std=0.0)
    x, stages = LearnedSirt(g, net, n_stages=3)(b)
    assert all(s["corrected"] for s in stages)
    assert all(s["rho_corrected"] == s["rho_sirt"] for s in stages)
    ref = torch.zeros_like(x)
    g.sirt(ref, b, 3, norms=False)
    assert torch.equal(x, ref)


def test_ordered_subset_stages_with_identity_network_are_os_sirt(tiny):
    """With ordered-subset physics steps (Sec. 2.3.2) and a zero head, the
    pipeline is exactly OS-SIRT: one epoch per stage over the same subsets."""
    from paper_2609_30166_amd import ordered_subsets
    from paper_2609_30166_amd.learned import LearnedSirt
    cfg, g, xt, b = tiny
    net = _net(head_std=0.0)
    x, stages = LearnedSirt(g, net, n_stages=3, subsets=4)(b)
    assert all(s["corrected"] for s in stages)
    ref = torch.zeros_like(x)
    g.os_sirt(ref, b, ordered_subsets(cfg.n_proj, 4), 3)
    assert torch.equal(x, ref)


def test_rejection_happens_at_the_stage_that_hurts(tiny):
    """Stage-by-stage check of the rule against residual norms recomputed
    independently by the library."""
    from paper_2609_30166_amd.learned import LearnedSirt
    cfg, g, xt, b = tiny
    net = _net(head_std=0.5, seed=4)
    x, stages = LearnedSirt(g, net, n_stages=4)(b)
    for s in stages:
        if "rho_sirt" in s:
            assert s["corrected"] == (s["rho_corrected"] <= s["rho_sirt"])
    assert abs(g.residual_norm(x, b) - np.linalg.norm(
        (b - g.forward(x)).double().cpu().numpy())) <= 1e-5 * g.residual_norm(x, b)


def test_training_checkpoint_resume_is_bitwise(tiny):
    """Two Adam steps equal one step, a save/load of parameters and moments,
    and a second step: the kernels are deterministic."""
    from paper_2609_30166_amd.unet import UNet
    cfg, g, xt, b = tiny
    x = torch.zeros_like(xt)
    g.sirt(x, b, 1, norms=False)
    a = _net(head_std=0.05, seed=7, scale=4.0)
    a.train_step(x, xt)
    a.train_step(x, xt)
    c = _net(head_std=0.05, seed=7, scale=4.0)
    c.train_step(x, xt)
    st = c.state_dict()
    d = UNet("cuda:0", params=c.params(), scale=st["scale"])
    d.load_state_dict(st)
    d.train_step(x, xt)
    assert torch.equal(a.theta, d.theta)
    assert torch.equal(a.m, d.m) and torch.equal(a.v, d.v)


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="trained weights not present")
def test_trained_network_gains_over_plain_sirt():
    """On a held-out phantom of the learned-correction configuration (256^3,
    180 x 384^2, Poisson I0 = 1e4), the staged pipeline beats its own physics
    steps without corrections (the same SIRT iterations or OS-SIRT epochs) in
    PSNR and keeps its corrections."""
    from paper_2609_30166_amd import learned
    from paper_2609_30166_amd.train_unet import load
    from synth import configs

    import json

    cfg, geom = learned.learned_geometry(device="cuda:0")
    nets = load(WEIGHTS, "cuda:0")
    meta = json.loads(str(np.load(WEIGHTS, allow_pickle=False)["meta"]))
    per = int(meta["iters_per_stage"])
    seed = list(configs.TEST_SEEDS)[2]   # an ellipsoid phantom
    stages = int(meta["stages"])
    res = learned.compare(geom, nets, cfg, [seed], sirt_iters=stages * per, n_stages=stages,
                          iters_per_stage=per, fov=bool(meta.get("fov_mask", False)),
                          subsets=int(meta.get("subsets", 0)) or None)
    r = res["rows"][0]
    assert r["accepted"] >= 1
    assert r["psnr_learned"] >= r["psnr_sirt_same_budget"] + 1.0, r
