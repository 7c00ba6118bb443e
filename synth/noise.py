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
