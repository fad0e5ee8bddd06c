"""The five seeded workloads (and small variants of them for parity tests).

Each builder returns a :class:`Case`.  Sizes follow the paper's benchmark
range (256x256 to 4000x6000 pixels, section 4.2); a shape is written (rows,
cols) = (H, W) and "6000x4000" means W=6000, H=4000.  All randomness comes
from ``numpy.random.default_rng(seed)``.

  plain   (seed 1): 256x256 N(100,5) sky + 50 stars, TAN at (150, +2) deg,
                    2.85"/px; target CRPIX + (3.7, -2.2) px, rotated 0.5 deg.
  sip3    (seed 2): 6000x4000 N(300,10) sky + 2000 stars, 2.85"/px, forward
                    SIP order 3 and fitted inverse order 4; target 6000x4000
                    TAN, CRVAL moved 40 px along the source +x axis (RA
                    decreases, east-left), rotated 0.3 deg, no SIP.
  batch   (seed 3): 64 frames with sides U{2048..6000}, CRVAL dither
                    U(+-0.1 deg) on the sky, rotation U(+-2 deg), scale
                    U(2.5, 3.2)"/px, SIP order U{2,3,4} with inverse order+1,
                    83.3 stars per Mpix; target 8192x8192 TAN at (150, +2),
                    2.85"/px.
  grad    (seed 4): 2048x2048 N(100,5) + 350 stars, SIP order 3 with inverse
                    order 3 (10+10 coefficients), target 2048x2048 TAN with
                    CRPIX + (3.7, -2.2), rotated 0.5 deg; the perturbed WCS moves
                    CRVAL by U(+-1"), CRPIX by U(+-0.5 px), CD by (1+U(+-1e-4)).
  pole    (seed 5): target 8192x8192 TAN at (150, +89.5), 0.2"/px; source
                    8192x8192 at (152.0, +89.48), rotated 45 deg, CRPIX +
                    (3.7, -2.2), SIP order 4 with inverse order 4.
  demo            : 50x50 frames, 0.5 px CRPIX offset and 0.005 deg CRVAL
                    offset (the paper's demo set-up, section 4.1).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math
from typing import List, Optional

import numpy as np

from .wcsparams import WcsParams
from .starfield import star_field
from .sipfit import draw_sip, fit_inverse_sip

NEAREST, BILINEAR, BICUBIC = 0, 1, 2
STAR_DENSITY_PER_MPIX = 2000.0 / 24.0  # the 6000x4000 frame's density, 83.3 per Mpix


@dataclass
class Case:
    name: str
    src: object                      # float32 [H, W] array, or a list of them (batch)
    src_wcs: object                  # WcsParams, or a list of them (batch)
    tgt_wcs: WcsParams
    out_shape: tuple                 # (H_out, W_out)
    interp: int
    extra: dict = field(default_factory=dict)


def _scaled(n: int, scale: float) -> int:
    return max(1, int(round(n * scale)))


def plain(seed: int = 1, size: int = 256, interp: int = BILINEAR) -> Case:
    rng = np.random.default_rng(seed)
    h = w = size
    n_stars = max(1, int(round(50 * size * size / 65536)))
    src = star_field(h, w, 100.0, 5.0, n_stars, seed, rng=rng)
    sw = WcsParams.tan((150.0, 2.0), 2.85, 0.0, (h, w))
    tw = WcsParams.tan((150.0, 2.0), 2.85, 0.5, (h, w), crpix_offset=(3.7, -2.2))
    return Case("plain", src, sw, tw, (h, w), interp)


def sip3(seed: int = 2, scale: float = 1.0, interp: int = BILINEAR,
         sip_order: int = 3, inv_order: int = 4) -> Case:
    """The 6000x4000 SIP frame; ``scale`` < 1 gives a smaller frame with the
    same star density and the same edge displacement per SIP order."""
    rng = np.random.default_rng(seed)
    w = _scaled(6000, scale)
    h = _scaled(4000, scale)
    n_stars = _scaled(2000, scale * scale)
    src = star_field(h, w, 300.0, 10.0, n_stars, seed, rng=rng)
    half = 0.5 * max(h, w)
    a, b = draw_sip(sip_order, half, rng)
    sw = WcsParams.tan((150.0, 2.0), 2.85, 0.0, (h, w), a=a, b=b)
    ap, bp, resid = fit_inverse_sip(a, b, inv_order, sw.crpix, (h, w))
    sw = sw.copy(ap=ap, bp=bp)
    s_deg = 2.85 / 3600.0
    ra_t = 150.0 - 40.0 * s_deg / math.cos(math.radians(2.0))
    tw = WcsParams.tan((ra_t, 2.0), 2.85, 0.3, (h, w))
    return Case("sip3", src, sw, tw, (h, w), interp, extra={"inverse_fit_resid_px": resid})


def sweep(shape_hw, sip: bool = True, seed: int = 8, interp: int = BILINEAR) -> Case:
    """One point of the size sweep: an (h, w) frame with the 6000x4000 frame's
    recipe (star density, sky, 2.85"/px at (150, +2)); with ``sip`` a SIP
    order-3 distortion scaled to the frame and its fitted order-4 inverse.
    The target is the same size, its CRVAL 40 px along +x and rotated 0.3 deg."""
    rng = np.random.default_rng(seed)
    h, w = shape_hw
    n_stars = max(1, int(round(STAR_DENSITY_PER_MPIX * h * w / 1e6)))
    src = star_field(h, w, 300.0, 10.0, n_stars, seed, rng=rng)
    sw = WcsParams.tan((150.0, 2.0), 2.85, 0.0, (h, w))
    if sip:
        a, b = draw_sip(3, 0.5 * max(h, w), rng)
        ap, bp, _ = fit_inverse_sip(a, b, 4, sw.crpix, (h, w))
        sw = sw.copy(a=a, b=b, ap=ap, bp=bp)
    s_deg = 2.85 / 3600.0
    ra_t = 150.0 - 40.0 * s_deg / math.cos(math.radians(2.0))
    tw = WcsParams.tan((ra_t, 2.0), 2.85, 0.3, (h, w))
    return Case("sweep", src, sw, tw, (h, w), interp)


def batch(seed: int = 3, n_frames: int = 64, target_side: int = 8192,
          side_range=(2048, 6000), interp: int = BILINEAR, images: bool = True) -> Case:
    """64 uneven sub-exposures onto one target.  Frame parameters come from
    ``default_rng(seed)``; frame k's pixels from ``default_rng(seed*1000+k)``.
    ``images=False`` returns the frame shapes only (src entries are shapes)."""
    rng = np.random.default_rng(seed)
    tw = WcsParams.tan((150.0, 2.0), 2.85, 0.0, (target_side, target_side))
    srcs, wcss, orders = [], [], []
    for k in range(n_frames):
        w = int(rng.integers(side_range[0], side_range[1] + 1))
        h = int(rng.integers(side_range[0], side_range[1] + 1))
        dra = rng.uniform(-0.1, 0.1)
        ddec = rng.uniform(-0.1, 0.1)
        rot = rng.uniform(-2.0, 2.0)
        sc = rng.uniform(2.5, 3.2)
        order = int(rng.integers(2, 5))
        dec = 2.0 + ddec
        ra = 150.0 + dra / math.cos(math.radians(dec))
        half = 0.5 * max(h, w)
        a, b = draw_sip(order, half, rng)
        sw = WcsParams.tan((ra, dec), sc, rot, (h, w), a=a, b=b)
        ap, bp, _ = fit_inverse_sip(a, b, order + 1, sw.crpix, (h, w))
        wcss.append(sw.copy(ap=ap, bp=bp))
        orders.append(order)
        if images:
            n_stars = int(round(STAR_DENSITY_PER_MPIX * h * w / 1e6))
            srcs.append(star_field(h, w, 300.0, 10.0, n_stars, seed * 1000 + k))
        else:
            srcs.append((h, w))
    return Case("batch", srcs, wcss, tw, (target_side, target_side), interp,
                extra={"sip_orders": orders})


def grad(seed: int = 4, size: int = 2048, interp: int = BICUBIC) -> Case:
    rng = np.random.default_rng(seed)
    h = w = size
    n_stars = max(1, int(round(350 * size * size / 2048.0 ** 2)))
    src = star_field(h, w, 100.0, 5.0, n_stars, seed, rng=rng)
    half = 0.5 * size
    a, b = draw_sip(3, half, rng)
    sw = WcsParams.tan((150.0, 2.0), 2.85, 0.0, (h, w), a=a, b=b)
    ap, bp, _ = fit_inverse_sip(a, b, 3, sw.crpix, (h, w))
    sw = sw.copy(ap=ap, bp=bp)
    tw = WcsParams.tan((150.0, 2.0), 2.85, 0.5, (h, w), crpix_offset=(3.7, -2.2))
    dec = sw.crval[1]
    d_ra = rng.uniform(-1.0, 1.0) / 3600.0 / math.cos(math.radians(dec))
    d_dec = rng.uniform(-1.0, 1.0) / 3600.0
    d_crpix = rng.uniform(-0.5, 0.5, 2)
    cd_fac = 1.0 + rng.uniform(-1e-4, 1e-4, (2, 2))
    pert = sw.copy(crval=(sw.crval[0] + d_ra, sw.crval[1] + d_dec),
                   crpix=(sw.crpix[0] + d_crpix[0], sw.crpix[1] + d_crpix[1]),
                   cd=sw.cd * cd_fac)
    return Case("grad", src, pert, tw, (h, w), interp, extra={"src_wcs_true": sw})


def pole(seed: int = 5, size: int = 8192, interp: int = BILINEAR) -> Case:
    """Dec +89.5 target; ``size`` < 8192 shrinks both frames with the pixel
    scale fixed (the SIP scale follows the frame)."""
    rng = np.random.default_rng(seed)
    h = w = size
    n_stars = int(round(STAR_DENSITY_PER_MPIX * h * w / 1e6))
    src = star_field(h, w, 300.0, 10.0, n_stars, seed, rng=rng)
    half = 0.5 * size
    a, b = draw_sip(4, half, rng)
    sw = WcsParams.tan((152.0, 89.48), 0.2, 45.0, (h, w), crpix_offset=(3.7, -2.2), a=a, b=b)
    ap, bp, resid = fit_inverse_sip(a, b, 4, sw.crpix, (h, w))
    sw = sw.copy(ap=ap, bp=bp)
    tw = WcsParams.tan((150.0, 89.5), 0.2, 0.0, (h, w))
    return Case("pole", src, sw, tw, (h, w), interp, extra={"inverse_fit_resid_px": resid})


def strong_sip(seed: int = 11, size: int = 256, order: int = 7, sigma: float = 1e-5,
               interp: int = BILINEAR) -> Case:
    """A stress map for the local cubic models: an inverse SIP made of the
    terms of one high order only, sigma * N(0, 1) px at the frame edge per
    term.  Its local quartic terms grow as the cube of the distance from
    CRPIX, so with the default sigma cells near the centre admit a cubic
    model within 1e-6 px and cells towards the edges do not."""
    rng = np.random.default_rng(seed)
    S = 0.5 * size
    ap = np.zeros((order + 1, order + 1))
    bp = np.zeros((order + 1, order + 1))
    for p in range(order + 1):
        q = order - p
        ap[p, q] = rng.normal(0.0, sigma) * S / S ** order
        bp[p, q] = rng.normal(0.0, sigma) * S / S ** order
    src = star_field(size, size, 100.0, 5.0, max(1, size * size // 1300), seed, rng=rng)
    sw = WcsParams.tan((150.0, 2.0), 2.85, 0.0, (size, size), ap=ap, bp=bp)
    tw = WcsParams.tan((150.0, 2.0), 2.85, 0.5, (size, size), crpix_offset=(3.7, -2.2))
    return Case("strong_sip", src, sw, tw, (size, size), interp)


def demo(seed: int = 6, interp: int = BILINEAR) -> Case:
    rng = np.random.default_rng(seed)
    src = star_field(50, 50, 100.0, 5.0, 3, seed, rng=rng)
    sw = WcsParams.tan((150.0, 2.0), 2.85, 0.0, (50, 50))
    tw = WcsParams.tan((150.005, 2.005), 2.85, 0.0, (50, 50), crpix_offset=(0.5, 0.5))
    return Case("demo", src, sw, tw, (50, 50), interp)
