"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This package only *creates* inputs: star-field images, TAN/SIP world
coordinate headers and the fitted inverse SIP coefficients that a real FITS
header would carry.  It holds none of the reprojection arithmetic (no
celestial transform, no interpolation), so the oracle and the HIP path can
both consume its outputs without sharing any of the method's code.
"""
from .wcsparams import WcsParams
from .starfield import star_field
from .sipfit import draw_sip, fit_inverse_sip
from . import configs

__all__ = ["WcsParams", "star_field", "draw_sip", "fit_inverse_sip", "configs"]
