"""dfr: per-pixel astronomical image reprojection on AMD Instinct MI355X.

The method of "dfreproject: A Python package for astronomical reprojection"
(target WCS -> sky -> source WCS, TAN + SIP, nearest / bilinear / bicubic
interpolation, footprint normalisation) as hand-written HIP kernels for
gfx950 behind the C ABI of ``include/dfr.h``; this package is the thin Python
binding (``_lib``: the C entry points by name; ``api``: torch helpers).
"""
from . import _lib
from ._lib import DfrError
from .api import (Plan, ReprojectFn, Wcs, as_wcs, autotune, calculate_reprojection, cell_model,
                  batch_boxes, coadd_batch, release, reproject_batch_cropped,
                  reproject, reproject_backward, reproject_batch, reproject_differentiable,
                  sq_residual, wcs_from_header, wcs_params, wcs_with_params)

__all__ = ["DfrError", "Plan", "ReprojectFn", "Wcs", "as_wcs", "autotune", "calculate_reprojection",
           "batch_boxes", "cell_model", "coadd_batch", "reproject_batch_cropped",
           "release", "reproject", "reproject_backward", "reproject_batch",
           "reproject_differentiable", "sq_residual", "wcs_from_header", "wcs_params",
           "wcs_with_params"]
