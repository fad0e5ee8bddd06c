"""Seeded synthetic star fields standing in for the paper's Dragonfly frames
(sizes 256x256 to 4000x6000, section 4.2); the paper's own FITS files are not
available, so these images replace them.

Recipe (all draws from ``numpy.random.default_rng(seed)``, PCG64):
  1. sky    = mu + sigma * standard_normal((h, w), float32)
  2. star x ~ U(0, w-1), star y ~ U(0, h-1), amplitude = 10**U(2, 5)
  3. each star adds amp * exp(-r^2 / (2 * 1.5^2)) to the pixel centres within
     9 px of it (stamp computed in float64, added in float32).
"""
from __future__ import annotations

import numpy as np

STAR_SIGMA_PX = 1.5
STAR_RADIUS_PX = 9


def star_field(h: int, w: int, sky_mu: float, sky_sigma: float, n_stars: int,
               seed: int, rng: np.random.Generator | None = None) -> np.ndarray:
    """Return a C-contiguous float32 [h, w] star field."""
    if rng is None:
        rng = np.random.default_rng(seed)
    img = rng.standard_normal((h, w), dtype=np.float32)
    img *= np.float32(sky_sigma)
    img += np.float32(sky_mu)
    if n_stars <= 0 or h == 0 or w == 0:
        return img
    xs = rng.uniform(0.0, w - 1, n_stars)
    ys = rng.uniform(0.0, h - 1, n_stars)
    amps = 10.0 ** rng.uniform(2.0, 5.0, n_stars)
    r = STAR_RADIUS_PX
    inv2s2 = 1.0 / (2.0 * STAR_SIGMA_PX * STAR_SIGMA_PX)
    for x, y, a in zip(xs, ys, amps):
        x0 = max(int(np.ceil(x - r)), 0)
        x1 = min(int(np.floor(x + r)), w - 1)
        y0 = max(int(np.ceil(y - r)), 0)
        y1 = min(int(np.floor(y + r)), h - 1)
        gx = np.arange(x0, x1 + 1, dtype=np.float64) - x
        gy = np.arange(y0, y1 + 1, dtype=np.float64) - y
        d2 = gy[:, None] ** 2 + gx[None, :] ** 2
        stamp = np.where(d2 <= r * r, a * np.exp(-d2 * inv2s2), 0.0)
        img[y0:y1 + 1, x0:x1 + 1] += stamp.astype(np.float32)
    return img
