"""The torch input synthesisers reproduce the numpy definitions (CPU)."""

import numpy as np
import torch

from synth import configs, noise, phantoms


def test_ellipsoids_torch_matches_numpy():
    rng = np.random.default_rng([3, 1])
    shape = (40, 48, 56)
    ells = phantoms.random_ellipsoids(6, shape, (3.0, 12.0), (0.1, 1.0), rng)
    a = phantoms.voxelise_ellipsoids(ells, shape)
    b = phantoms.voxelise_ellipsoids_torch(ells, shape, "cpu").numpy()
    # identical up to voxel centres lying on a surface to rounding precision
    assert np.mean(a != b) < 1e-4
    np.testing.assert_allclose(a.sum(), b.sum(), rtol=1e-3)


def test_foam_torch_matches_numpy():
    shape = (32, 40, 40)
    a = phantoms.foam_phantom(shape, np.random.default_rng([5, 2]))
    b = phantoms.foam_phantom_torch(shape, np.random.default_rng([5, 2]), "cpu").numpy()
    assert np.mean(a != b) < 1e-4
    assert a.max() == 0.5 and (a == 0).mean() > 0.3


def test_learned_phantoms_alternate_kinds_and_units():
    cfg = configs.make_config("learned", n_proj=4)
    cfg.shape = (32, 32, 32)
    cfg.extra = dict(cfg.extra, semi=(2.0, 10.0))
    ell = configs.make_learned_phantom(cfg, 0, "cpu").numpy()
    foam = configs.make_learned_phantom(cfg, 1, "cpu").numpy()
    assert foam.max() == 0.5 / 32
    assert 0 < ell.max() <= cfg.extra["n_ellipsoids"] * 1.0 / 32   # additive overlaps
    assert set(configs.TRAIN_SEEDS).isdisjoint(configs.TEST_SEEDS)
    assert len(configs.TRAIN_SEEDS) == 512 and len(configs.TEST_SEEDS) == 32


def test_poisson_torch_statistics():
    g = torch.Generator().manual_seed(0)
    y = torch.full((200000,), 1.0)
    b = noise.poisson_log_transform_torch(y, 1e4, g)
    # E[-ln(N / I0)] ~ y for large counts; variance ~ 1 / (I0 e^-y)
    assert abs(float(b.mean()) - 1.0) < 2e-3
    assert abs(float(b.var()) - np.exp(1.0) / 1e4) < 0.05 * np.exp(1.0) / 1e4
    z = noise.poisson_log_transform_torch(torch.full((1000,), 30.0), 1e4, g)
    assert torch.all(z == float(np.log(1e4)))   # zero counts clamp to 1
