"""Independent ray geometry used by the pins (not the oracle's code path).

The oracle clips rays with the slab method; these helpers compute the same
chords by intersecting the ray with each face of the box, and chords through
ellipsoids from the quadric's quadratic equation.  Source and direction come
from numpy.linalg on the 3x4 matrix.
"""

from __future__ import annotations

import numpy as np


def source_and_dir(P, u, v, shape):
    """Source (index coordinates) and unit direction of the pixel ray (u, v)."""
    nz, ny, nx = shape
    off = 0.5 * (np.array([nx, ny, nz]) - 1)
    M = P[:, :3]
    S = -np.linalg.solve(M, P[:, 3]) + off
    d = np.linalg.solve(M, np.array([u, v, 1.0]))
    return S, d / np.linalg.norm(d)


def box_chord(S, d, shape, tol=1e-9):
    """Entry/exit parameters of S + t d through [0, n-1]^3 via face hits."""
    nz, ny, nx = shape
    hi = np.array([nx, ny, nz], dtype=float) - 1
    ts = []
    for a in range(3):
        if d[a] == 0:
            continue
        for face in (0.0, hi[a]):
            t = (face - S[a]) / d[a]
            q = S + t * d
            ok = all(-tol <= q[b] <= hi[b] + tol for b in range(3) if b != a)
            if ok:
                ts.append(t)
    if len(ts) < 2:
        return None
    t0, t1 = min(ts), max(ts)
    if t1 - t0 <= tol:
        return None
    return t0, t1


def ellipsoid_chord(S, d, Q, centre):
    """Length of S + t d inside ||Q (c - centre)|| <= 1 (0 if it misses)."""
    qd = Q @ d
    qs = Q @ (S - centre)
    a = qd @ qd
    b = 2 * qd @ qs
    c = qs @ qs - 1.0
    disc = b * b - 4 * a * c
    if disc <= 0:
        return 0.0
    r = np.sqrt(disc)
    return (r / a) * np.linalg.norm(d)
