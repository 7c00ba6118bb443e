"""MI355X-native ray-driven projector pair and SIRT loop (CTrex hot path).

Public Python API (argument marshalling over the C ABI in include/ctrex.h):

* ``Geometry`` — projector context over per-projection 3x4 view matrices;
  ``forward`` (A), ``back`` (A^T), ``sirt`` (Eq. 1), ``os_sirt`` (ordered
  subsets, Sec. 2.3.2), ``residual_norm``, ``sample_count``.
* ``ordered_subsets`` — interleaved / contiguous / random projection subsets.
* ``CylinderGeometry`` — the aligned cylindrical domain (polar grid, rigid
  pose; Sec. 3.5, 4.2.1, 4.3.1): ``forward``, voxel-driven ``back``, ``sirt``.
* ``project`` — differentiable forward projection (autograd).
* ``data_term`` — differentiable ||Ax - b||^2 (library residual epilogue and
  scaled backprojection); ``total_variation``, ``reconstruction_loss`` —
  ||Ax - b||^2 + lambda TV(x).
* ``unet.UNet``, ``learned.LearnedSirt`` — the learned correction between
  unrolled SIRT iterations (Sec. 5 extension; include/ctrex_nn.h).
"""

from .projector import (  # noqa: F401
    Geometry, ForwardProject, project, DataTerm, data_term, TotalVariation, total_variation,
    reconstruction_loss, ordered_subsets,
)
from .cylinder import CylinderGeometry  # noqa: F401
from ._lib import CtrexError, library_path  # noqa: F401

__all__ = ["Geometry", "ForwardProject", "project", "DataTerm", "data_term", "TotalVariation",
           "total_variation",
           "reconstruction_loss", "ordered_subsets", "CylinderGeometry", "CtrexError",
           "library_path"]
