"""Synthetic SIP distortion headers.

``draw_sip`` draws a forward A/B pair; ``fit_inverse_sip`` produces the
inverse AP/BP that a real header would carry, by linear least squares on a
grid (the usual way SIP inverses are produced; Shupe et al. 2005).  Both only
make header *values*; evaluation uses numpy's polynomial library.

Recipe: order-n terms (2 <= n <= N) ~ N(0, (1e-6 * S**(2-n))**2) with S half
the larger image side, so every order moves the frame edge by ~1e-6*S**2 px.
The inverse is fitted for 0 <= p+q <= order on a 161 x 121 grid spanning the
frame plus a 20 px margin, with design columns scaled by S**(p+q).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import polynomial as P


def draw_sip(order: int, half_side: float, rng: np.random.Generator):
    """Return forward SIP arrays (A, B), each (order+1, order+1)."""
    a = np.zeros((order + 1, order + 1))
    b = np.zeros((order + 1, order + 1))
    for n in range(2, order + 1):
        sd = 1e-6 * half_side ** (2 - n)
        for p in range(n + 1):
            q = n - p
            a[p, q] = rng.normal(0.0, sd)
            b[p, q] = rng.normal(0.0, sd)
    return a, b


def fit_inverse_sip(a: np.ndarray, b: np.ndarray, inv_order: int, crpix, shape_hw,
                    margin: float = 20.0, grid=(161, 121)):
    """Least-squares inverse SIP (AP, BP) of order ``inv_order`` for a frame of
    ``shape_hw`` with 1-based reference pixel ``crpix``.

    Returns (AP, BP, max_residual_px): max_residual_px is how far the fitted
    inverse misses the exact inverse at the grid nodes (a property of the
    data, reported, never a tolerance)."""
    h, w = shape_hw
    s = 0.5 * max(h, w)
    x = np.linspace(-margin, w - 1 + margin, grid[0])
    y = np.linspace(-margin, h - 1 + margin, grid[1])
    xx, yy = np.meshgrid(x, y)
    u = (xx - (crpix[0] - 1.0)).ravel()
    v = (yy - (crpix[1] - 1.0)).ravel()
    uu = u + P.polyval2d(u, v, a)
    vv = v + P.polyval2d(u, v, b)
    n = inv_order
    full = P.polyvander2d(uu / s, vv / s, [n, n])
    keep = [i * (n + 1) + j for i in range(n + 1) for j in range(n + 1) if i + j <= n]
    design = full[:, keep]
    cu, *_ = np.linalg.lstsq(design, u - uu, rcond=None)
    cv, *_ = np.linalg.lstsq(design, v - vv, rcond=None)
    ap = np.zeros((n + 1, n + 1))
    bp = np.zeros((n + 1, n + 1))
    k = 0
    for i in range(n + 1):
        for j in range(n + 1):
            if i + j <= n:
                ap[i, j] = cu[k] / s ** (i + j)
                bp[i, j] = cv[k] / s ** (i + j)
                k += 1
    res_u = design @ cu - (u - uu)
    res_v = design @ cv - (v - vv)
    resid = float(np.max(np.hypot(res_u, res_v)))
    return ap, bp, resid
