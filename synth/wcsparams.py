"""Plain container for the WCS keywords the method reads (paper section 3.1
and the definitions list of section 3.2): CRPIX, CRVAL, the CD matrix and
the four SIP polynomials A, B, AP, BP (Shupe et al. 2005).

No arithmetic of the method lives here; only construction helpers.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
import math
from typing import Optional

import numpy as np


def _coeffs(c) -> Optional[np.ndarray]:
    if c is None:
        return None
    c = np.array(c, dtype=np.float64)
    if c.ndim != 2 or c.shape[0] != c.shape[1]:
        raise ValueError("SIP coefficients must be a square (order+1, order+1) array")
    return c


@dataclass
class WcsParams:
    """FITS TAN (+SIP) world coordinate system.

    crpix : FITS 1-based reference pixel (CRPIX1, CRPIX2); x is the column
            (NAXIS1, contiguous in memory), y the row.
    crval : (RA, Dec) of the reference point in degrees.
    cd    : 2x2 CD matrix in degrees per pixel, [[CD1_1, CD1_2], [CD2_1, CD2_2]].
    a, b  : forward SIP polynomials, arrays [p, q] = coefficient of u**p v**q.
    ap, bp: inverse SIP polynomials, same layout.
    An absent polynomial is ``None`` (order 0).
    """

    crpix: tuple
    crval: tuple
    cd: np.ndarray
    a: Optional[np.ndarray] = None
    b: Optional[np.ndarray] = None
    ap: Optional[np.ndarray] = None
    bp: Optional[np.ndarray] = None

    def __post_init__(self):
        self.crpix = (float(self.crpix[0]), float(self.crpix[1]))
        self.crval = (float(self.crval[0]), float(self.crval[1]))
        self.cd = np.array(self.cd, dtype=np.float64).reshape(2, 2)
        self.a = _coeffs(self.a)
        self.b = _coeffs(self.b)
        self.ap = _coeffs(self.ap)
        self.bp = _coeffs(self.bp)

    @staticmethod
    def order_of(c: Optional[np.ndarray]) -> int:
        return 0 if c is None else c.shape[0] - 1

    @property
    def a_order(self) -> int:
        return self.order_of(self.a)

    @property
    def b_order(self) -> int:
        return self.order_of(self.b)

    @property
    def ap_order(self) -> int:
        return self.order_of(self.ap)

    @property
    def bp_order(self) -> int:
        return self.order_of(self.bp)

    def copy(self, **changes) -> "WcsParams":
        base = replace(self)
        base.cd = self.cd.copy()
        for name in ("a", "b", "ap", "bp"):
            v = getattr(self, name)
            setattr(base, name, None if v is None else v.copy())
        for k, v in changes.items():
            setattr(base, k, v)
        base.__post_init__()
        return base

    @staticmethod
    def tan(crval, scale_arcsec: float, rot_deg: float, shape_hw, crpix_offset=(0.0, 0.0),
            a=None, b=None, ap=None, bp=None) -> "WcsParams":
        """TAN header with the reference pixel at the image centre (plus an
        offset), east to the left: CD = s * [[-cos r, sin r], [sin r, cos r]]."""
        h, w = shape_hw
        s = scale_arcsec / 3600.0
        r = math.radians(rot_deg)
        cd = s * np.array([[-math.cos(r), math.sin(r)], [math.sin(r), math.cos(r)]])
        crpix = ((w + 1) / 2.0 + crpix_offset[0], (h + 1) / 2.0 + crpix_offset[1])
        return WcsParams(crpix=crpix, crval=crval, cd=cd, a=a, b=b, ap=ap, bp=bp)
