"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package builds inputs only: view matrices for a trajectory, voxelised
phantoms, displacement grids and measurement noise.  It holds none of the
projector's arithmetic (no ray clipping, sampling or interpolation), so the
CPU oracle and the HIP path can both consume it without sharing any of the
method's code.
"""

from .trajectories import (  # noqa: F401
    view_matrix,
    circular_cone,
    helical_cone,
    rigid_jitter,
    conveyor_belt,
    exposure_time_fractions,
    smooth_displacement,
)
from .phantoms import (  # noqa: F401
    Ellipsoid,
    random_ellipsoids,
    voxelise_ellipsoids,
    cylinder_background,
    foam_phantom,
    fov_mask,
)
from .noise import poisson_log_transform  # noqa: F401
from .configs import CONFIGS, make_config  # noqa: F401
