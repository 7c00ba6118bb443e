"""Measurement noise for the transmission model (input synthesis only)."""

from __future__ import annotations

import numpy as np


def poisson_log_transform(y, I0, rng):
    """Noisy line integrals from clean ones: counts ~ Poisson(I0 exp(-y)),
    clamped to >= 1 so the log stays finite, then b = -ln(counts / I0).

    ``y`` is a numpy array of clean line integrals; returns float64.
    """
    lam = I0 * np.exp(-np.asarray(y, dtype=np.float64))
    counts = np.maximum(rng.poisson(lam), 1)
    return -np.log(counts / I0)


def poisson_log_transform_torch(y, I0, generator):
    """``poisson_log_transform`` with torch on the tensor's device: counts ~
    Poisson(I0 exp(-y)) drawn from ``generator``, clamped to >= 1,
    b = -ln(counts / I0); returns float32."""
    import torch
    lam = I0 * torch.exp(-y.to(torch.float64))
    counts = torch.clamp(torch.poisson(lam, generator=generator), min=1.0)
    return (-torch.log(counts / I0)).to(torch.float32)
