"""MI355X-native ray-driven projector pair and SIRT loop (CTrex hot path).

Public Python API (argument marshalling over the C ABI in include/ctrex.h):

* ``Geometry`` — projector context over per-projection 3x4 view matrices;
  ``forward`` (A), ``back`` (A^T), ``sirt`` (Eq. 1), ``sample_count``.
* ``project`` — differentiable forward projection (autograd).
* ``total_variation``, ``reconstruction_loss`` — ||Ax - b||^2 + lambda TV(x).
"""

from .projector import (  # noqa: F401
    Geometry, ForwardProject, project, TotalVariation, total_variation, reconstruction_loss,
)
from ._lib import CtrexError, library_path  # noqa: F401

__all__ = ["Geometry", "ForwardProject", "project", "TotalVariation", "total_variation",
           "reconstruction_loss", "CtrexError", "library_path"]
