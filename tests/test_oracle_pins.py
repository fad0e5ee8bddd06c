"""Pins of the FP64 oracle against what the definitions fix (CPU only).

The paper prints no numeric example (its figures are not available), so the
oracle is tied to closed forms, an independent formulation of the same
geometry, exact special cases and brute force:

  * CRPIX maps to CRVAL (section 3.2.1 with u = v = 0);
  * an independent tangent-plane (vector) formulation of the gnomonic
    projection, in 40-digit arithmetic, for both stages of section 3.2;
  * closed forms on the central meridian and at the celestial pole;
  * pixel -> sky -> pixel round trips with an exact (Newton) SIP inverse;
  * SIP single-term closed forms and library polynomial evaluation;
  * identity, integer-shift and 90-degree-rotation reprojections;
  * interpolation: affine / quadratic reproduction, brute force on 8x8,
    nearest = closest pixel, footprint closed forms;
  * gradients: adjoint identity and central finite differences.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from numpy.polynomial import polynomial as P

from synth import WcsParams, configs, draw_sip, fit_inverse_sip

mp.mp.dps = 40

# ---------------------------------------------------------------- helpers --


def geometries():
    """The WCS of every workload (and the pole at exactly +90 deg)."""
    c1 = configs.plain()
    c2 = configs.sip3(scale=0.1)
    c4 = configs.grad(size=256)
    c5 = configs.pole(size=512)
    polar = WcsParams.tan((33.0, 90.0), 1.0, 17.0, (300, 300))
    south = WcsParams.tan((310.0, -45.0), 4.0, -30.0, (400, 500), crpix_offset=(10.3, -7.1))
    return {
        "plain_src": c1.src_wcs, "plain_tgt": c1.tgt_wcs,
        "sip3_src": c2.src_wcs, "sip3_tgt": c2.tgt_wcs,
        "grad_src": c4.src_wcs, "pole_src": c5.src_wcs, "pole_tgt": c5.tgt_wcs,
        "polar": polar, "south": south,
    }


def frame_points(w, n, rng, span=None):
    """n random pixel coordinates over a frame around CRPIX."""
    span = span or 2.0 * max(w.crpix)
    cx, cy = w.crpix[0] - 1, w.crpix[1] - 1
    x = cx + rng.uniform(-span / 2, span / 2, n)
    y = cy + rng.uniform(-span / 2, span / 2, n)
    return np.stack([x, y], axis=1)


def unit(ra_deg, dec_deg):
    ra = np.radians(ra_deg)
    de = np.radians(dec_deg)
    return np.stack([np.cos(de) * np.cos(ra), np.cos(de) * np.sin(ra), np.sin(de)], axis=-1)


def separation_rad(radec1, radec2):
    a = unit(radec1[:, 0], radec1[:, 1])
    b = unit(radec2[:, 0], radec2[:, 1])
    return np.arctan2(np.linalg.norm(np.cross(a, b), axis=-1), np.sum(a * b, axis=-1))


def pixel_scale_rad(w):
    return math.radians(math.sqrt(abs(np.linalg.det(w.cd))))


def sip(c, u, v):
    return 0.0 if c is None else float(P.polyval2d(u, v, c))


def tangent_basis(w):
    a0 = mp.radians(w.crval[0])
    d0 = mp.radians(w.crval[1])
    c0 = [mp.cos(d0) * mp.cos(a0), mp.cos(d0) * mp.sin(a0), mp.sin(d0)]
    e = [-mp.sin(a0), mp.cos(a0), mp.mpf(0)]
    n = [-mp.sin(d0) * mp.cos(a0), -mp.sin(d0) * mp.sin(a0), mp.cos(d0)]
    return c0, e, n


def vec_pix2world(w, x, y):
    """Gnomonic deprojection as a point on the tangent plane: the direction is
    c0 + xi*east + eta*north (standard coordinates in radians)."""
    u = x - (w.crpix[0] - 1.0)
    v = y - (w.crpix[1] - 1.0)
    u, v = u + sip(w.a, u, v), v + sip(w.b, u, v)
    cd = [[mp.mpf(float(w.cd[i, j])) for j in range(2)] for i in range(2)]
    xi = mp.radians(cd[0][0] * u + cd[0][1] * v)
    eta = mp.radians(cd[1][0] * u + cd[1][1] * v)
    c0, e, n = tangent_basis(w)
    d = [c0[k] + xi * e[k] + eta * n[k] for k in range(3)]
    nd = mp.sqrt(sum(t * t for t in d))
    d = [t / nd for t in d]
    ra = mp.degrees(mp.atan2(d[1], d[0])) % 360
    dec = mp.degrees(mp.asin(d[2]))
    return float(ra), float(dec)


def vec_world2pix(w, ra, dec):
    """Inverse of vec_pix2world through AP/BP: xi = d.east / d.c0, eta likewise."""
    ra, dec = mp.radians(ra), mp.radians(dec)
    d = [mp.cos(dec) * mp.cos(ra), mp.cos(dec) * mp.sin(ra), mp.sin(dec)]
    c0, e, n = tangent_basis(w)
    dc = sum(d[k] * c0[k] for k in range(3))
    if dc <= 0:
        return None
    xi = mp.degrees(sum(d[k] * e[k] for k in range(3)) / dc)
    eta = mp.degrees(sum(d[k] * n[k] for k in range(3)) / dc)
    M = mp.matrix([[float(w.cd[0, 0]), float(w.cd[0, 1])], [float(w.cd[1, 0]), float(w.cd[1, 1])]])
    uv = mp.lu_solve(M, mp.matrix([xi, eta]))
    u, v = float(uv[0]), float(uv[1])
    u, v = u + sip(w.ap, u, v), v + sip(w.bp, u, v)
    return u + (w.crpix[0] - 1.0), v + (w.crpix[1] - 1.0)


# ------------------------------------------------------- coordinate pins --


@pytest.mark.parametrize("name", list(geometries().keys()))
def test_crpix_maps_to_crval(orc, name):
    w = geometries()[name]
    got = orc.pix2world(w, [[w.crpix[0] - 1.0, w.crpix[1] - 1.0]])
    sep = separation_rad(got, np.array([w.crval]))
    assert sep[0] <= 1e-12


@pytest.mark.parametrize("name", list(geometries().keys()))
def test_pix2world_matches_tangent_plane_vectors(orc, name):
    w = geometries()[name]
    rng = np.random.default_rng(11)
    xy = frame_points(w, 150, rng)
    got = orc.pix2world(w, xy)
    ref = np.array([vec_pix2world(w, x, y) for x, y in xy])
    err_px = separation_rad(got, ref) / pixel_scale_rad(w)
    assert err_px.max() <= 1e-9, err_px.max()


@pytest.mark.parametrize("name", list(geometries().keys()))
def test_world2pix_matches_tangent_plane_vectors(orc, name):
    w = geometries()[name]
    rng = np.random.default_rng(12)
    xy = frame_points(w, 150, rng)
    radec = np.array([vec_pix2world(w.copy(a=None, b=None), x, y) for x, y in xy])
    got, valid = orc.world2pix(w, radec)
    assert valid.all()
    ref = np.array([vec_world2pix(w, r, d) for r, d in radec])
    err = np.hypot(*(got - ref).T)
    assert err.max() <= 1e-9, err.max()


def test_central_meridian_closed_form(orc):
    """x' = 0: ra = ra0 and dec = dec0 + atan(y' in radians)."""
    for dec0 in (2.0, -45.0, 60.0):
        w = WcsParams(crpix=(1.0, 1.0), crval=(150.0, dec0), cd=[[-1e-3, 0.0], [0.0, 1e-3]])
        y = np.linspace(-3000, 3000, 41)
        got = orc.pix2world(w, np.stack([np.zeros_like(y), y], 1))
        assert np.all(np.abs(got[:, 0] - 150.0) <= 1e-12)
        ref = dec0 + np.degrees(np.arctan(np.radians(1e-3 * y)))
        assert np.abs(got[:, 1] - ref).max() <= 1e-11


def test_pole_closed_form(orc):
    """dec0 = +90: dec = atan2(r0, r) and ra = ra0 + atan2(x', -y')."""
    w = WcsParams(crpix=(1.0, 1.0), crval=(40.0, 90.0), cd=[[-2e-3, 5e-4], [7e-4, 1.5e-3]])
    rng = np.random.default_rng(3)
    xy = rng.uniform(-800, 800, (200, 2))
    got = orc.pix2world(w, xy)
    xp = w.cd[0, 0] * xy[:, 0] + w.cd[0, 1] * xy[:, 1]
    yp = w.cd[1, 0] * xy[:, 0] + w.cd[1, 1] * xy[:, 1]
    r = np.hypot(xp, yp)
    dec = np.degrees(np.arctan2(180.0 / np.pi, r))
    ra = (40.0 + np.degrees(np.arctan2(xp, -yp))) % 360.0
    sep = separation_rad(got, np.stack([ra, dec], 1))
    assert sep.max() <= 1e-13


def test_equator_ra_shift_closed_form(orc):
    """Along the equator row, a target at ra_t maps into a source tangent at
    ra_s with x'_s = r0 * tan(ra - ra_s)."""
    s = 1e-3
    tw = WcsParams(crpix=(1.0, 1.0), crval=(10.0, 0.0), cd=[[-s, 0.0], [0.0, s]])
    sw = WcsParams(crpix=(1.0, 1.0), crval=(10.7, 0.0), cd=[[-s, 0.0], [0.0, s]])
    x = np.linspace(-2000, 2000, 51)
    radec = orc.pix2world(tw, np.stack([x, np.zeros_like(x)], 1))
    xs, valid = orc.world2pix(sw, radec)
    ra = 10.0 + np.degrees(np.arctan(np.radians(-s * x)))
    xp = np.degrees(np.tan(np.radians(ra - 10.7)))
    assert valid.all()
    assert np.abs(xs[:, 0] - (-xp / s)).max() <= 1e-9
    assert np.abs(xs[:, 1]).max() <= 1e-9


@pytest.mark.parametrize("name", list(geometries().keys()))
def test_round_trip_exact_inverse(orc, name):
    """pixel -> sky -> pixel closes to < 1e-9 px (SIP inverted exactly)."""
    w = geometries()[name]
    rng = np.random.default_rng(5)
    xy = frame_points(w, 20000, rng)
    radec = orc.pix2world(w, xy)
    back, valid = orc.world2pix(w, radec, exact=True)
    assert valid.all()
    err = np.hypot(*(back - xy).T)
    assert err.max() < 1e-9, err.max()


def test_round_trip_tan_only(orc):
    w = configs.pole(size=512).tgt_wcs
    xy = frame_points(w, 20000, np.random.default_rng(6), span=8192)
    back, valid = orc.world2pix(w, orc.pix2world(w, xy))
    assert valid.all() and np.hypot(*(back - xy).T).max() < 1e-9


def test_fitted_inverse_close_to_exact(orc):
    """AP/BP is a fit: its miss against the exact inverse stays near the fit
    residual the generator reports (a property of the data)."""
    c = configs.sip3(scale=0.25)
    w = c.src_wcs
    xy = frame_points(w, 5000, np.random.default_rng(7), span=max(c.src.shape))
    radec = orc.pix2world(w, xy)
    a, _ = orc.world2pix(w, radec)
    b, _ = orc.world2pix(w, radec, exact=True)
    assert np.hypot(*(a - b).T).max() < 10 * c.extra["inverse_fit_resid_px"] + 1e-6


def test_sip_single_term_closed_form(orc):
    """Only A_20 = c: the pixel is seen by the TAN part at u + c u^2."""
    c = 3e-5
    base = WcsParams.tan((150.0, 2.0), 2.85, 0.3, (400, 400))
    a = np.zeros((3, 3))
    a[2, 0] = c
    ws = base.copy(a=a, b=np.zeros((3, 3)))
    rng = np.random.default_rng(8)
    xy = frame_points(base, 200, rng)
    u = xy[:, 0] - (base.crpix[0] - 1)
    got = orc.pix2world(ws, xy)
    ref = orc.pix2world(base, np.stack([xy[:, 0] + c * u * u, xy[:, 1]], 1))
    assert separation_rad(got, ref).max() <= 1e-14
    # inverse: only BP_11 = k adds k*u*v to y after the TAN inverse
    k = -2e-5
    bp = np.zeros((3, 3))
    bp[1, 1] = k
    wi = base.copy(ap=np.zeros((3, 3)), bp=bp)
    radec = orc.pix2world(base, xy)
    p1, _ = orc.world2pix(wi, radec)
    p0, _ = orc.world2pix(base, radec)
    uu = p0[:, 0] - (base.crpix[0] - 1)
    vv = p0[:, 1] - (base.crpix[1] - 1)
    assert np.abs(p1[:, 0] - p0[:, 0]).max() == 0.0
    assert np.abs(p1[:, 1] - (p0[:, 1] + k * uu * vv)).max() <= 1e-10


def test_sip_eval_matches_library_polynomial(orc):
    rng = np.random.default_rng(9)
    for order in (2, 3, 4, 5, 9):
        c = rng.normal(0, 1, (order + 1, order + 1))
        for p in range(order + 1):
            for q in range(order + 1):
                if p + q > order:
                    c[p, q] = 0.0
        for _ in range(20):
            u, v = rng.uniform(-3, 3, 2)
            ref = P.polyval2d(np.longdouble(u), np.longdouble(v), c.astype(np.longdouble))
            got = orc.sip_eval(c, u, v)
            scale = P.polyval2d(abs(u), abs(v), np.abs(c))
            assert abs(got - float(ref)) <= 1e-14 * max(scale, 1.0)


# -------------------------------------------------- whole-image special cases --


@pytest.mark.parametrize("interp", [0, 1, 2])
def test_identity_wcs_returns_image(orc, interp):
    c = configs.plain(size=96)
    out, fp, pos = orc.reproject(c.src, c.src_wcs, c.src_wcs, c.src.shape, interp, want_pos=True)
    src = c.src.astype(np.float64)
    y, x = np.mgrid[0:96, 0:96]
    assert np.hypot(pos[..., 0] - x, pos[..., 1] - y).max() <= 1e-10
    if interp == 0:
        assert np.array_equal(out, src) and np.all(fp == 1.0)
    else:
        # positions are integers to ~1e-11 px: the value moves by at most that
        # times the steepest neighbour difference
        grad = max(np.abs(np.diff(src, axis=0)).max(), np.abs(np.diff(src, axis=1)).max())
        assert np.abs(out - src).max() <= 1e-10 * 4 * grad
        # at the frame edge a position 1e-11 px outside loses that much footprint
        assert np.abs(fp - 1.0).max() <= 1e-10
        inner = (slice(2, -2), slice(2, -2))
        assert np.abs(fp[inner] - 1.0).max() <= 1e-12


@pytest.mark.parametrize("interp", [0, 1])
def test_integer_crpix_shift_is_array_shift(orc, interp):
    c = configs.plain(size=80)
    d1, d2 = 7, -4
    tw = c.src_wcs.copy(crpix=(c.src_wcs.crpix[0] + d1, c.src_wcs.crpix[1] + d2))
    out, fp = orc.reproject(c.src, c.src_wcs, tw, (70, 90), interp)
    exp = np.zeros((70, 90))
    efp = np.zeros((70, 90))
    h, w = c.src.shape
    for y in range(70):
        for x in range(90):
            ys, xs = y - d2, x - d1
            if 0 <= ys < h and 0 <= xs < w:
                exp[y, x] = c.src[ys, xs]
                efp[y, x] = 1.0
    if interp == 0:
        assert np.array_equal(out, exp) and np.array_equal(fp, efp)
    else:
        inner = efp == 1.0
        grad = np.abs(np.diff(c.src.astype(np.float64), axis=1)).max()
        assert np.abs(out - exp)[inner].max() <= 4e-10 * grad
        assert np.abs(fp - efp)[inner].max() <= 1e-10


def test_rotation_by_90_degrees(orc):
    """Same tangent point, target CD = source CD * Rot(90): nearest output is
    the source read at (col, row) = (c + (y - c) * -1 ... ) exactly."""
    n = 65
    rng = np.random.default_rng(4)
    src = rng.normal(0, 1, (n, n)).astype(np.float32)
    sw = WcsParams.tan((150.0, 2.0), 2.85, 0.0, (n, n))
    rot = np.array([[0.0, -1.0], [1.0, 0.0]])
    tw = sw.copy(cd=sw.cd @ rot)
    out, fp = orc.reproject(src, sw, tw, (n, n), 0)
    c = (n - 1) // 2
    y, x = np.mgrid[0:n, 0:n]
    xs = c - (y - c)  # (u_s, v_s) = Rot (u, v) = (-v, u)
    ys = c + (x - c)
    assert np.array_equal(out, src[ys, xs].astype(np.float64)) and np.all(fp == 1.0)


def test_behind_tangent_plane_is_uncovered(orc):
    """A source whose tangent point is > 90 deg away covers nothing."""
    c = configs.plain(size=32)
    sw = c.src_wcs.copy(crval=(330.0, -2.0))
    out, fp = orc.reproject(c.src, sw, c.tgt_wcs, (32, 32), 1)
    assert np.all(out == 0.0) and np.all(fp == 0.0)
    out, fp = orc.reproject(c.src, sw, c.tgt_wcs, (32, 32), 1, nan_outside=True)
    assert np.all(np.isnan(out))


# ------------------------------------------------------- interpolation pins --


def _interp_points(orc, src, pts, interp, a=-0.5):
    S = np.empty(len(pts))
    F = np.empty(len(pts))
    out, fp, _ = orc.interp_at(src, pts, interp, a)
    return out, fp


def test_bilinear_reproduces_affine(orc):
    y, x = np.mgrid[0:24, 0:32]
    src = (3.0 + 0.5 * x - 0.25 * y).astype(np.float32)
    rng = np.random.default_rng(1)
    pts = rng.uniform([0, 0], [31, 23], (500, 2))
    out, fp = _interp_points(orc, src, pts, 1)
    assert np.abs(out - (3.0 + 0.5 * pts[:, 0] - 0.25 * pts[:, 1])).max() <= 1e-12
    assert np.abs(fp - 1.0).max() <= 1e-14


def test_bicubic_reproduces_quadratic_and_constants(orc):
    y, x = np.mgrid[0:24, 0:32]
    q = lambda X, Y: 1.0 + 0.25 * X - 0.5 * Y + 0.125 * X * X - 0.0625 * X * Y + 0.03125 * Y * Y
    src = q(x, y).astype(np.float32)
    assert np.array_equal(src.astype(np.float64), q(x, y))
    rng = np.random.default_rng(2)
    pts = rng.uniform([1, 1], [29, 21], (500, 2))
    out, fp = _interp_points(orc, src, pts, 2, -0.5)
    assert np.abs(out - q(pts[:, 0], pts[:, 1])).max() <= 1e-10
    const = np.full((24, 32), 7.0, np.float32)
    for a in (-0.5, -0.75):
        out, fp = _interp_points(orc, const, pts, 2, a)
        assert np.abs(out - 7.0).max() <= 1e-12 and np.abs(fp - 1.0).max() <= 1e-13
    # a = -0.75 does not reproduce linear fields (the reason a = -0.5 is the default)
    lin = (0.5 * x).astype(np.float32)
    out, _ = _interp_points(orc, lin, pts, 2, -0.75)
    assert np.abs(out - 0.5 * pts[:, 0]).max() > 1e-3


def _kernel(s, interp, a):
    s = np.abs(s)
    if interp == 1:
        return np.clip(1.0 - s, 0.0, None)
    return np.where(s <= 1, (a + 2) * s ** 3 - (a + 3) * s ** 2 + 1,
                    np.where(s < 2, a * s ** 3 - 5 * a * s ** 2 + 8 * a * s - 4 * a, 0.0))


@pytest.mark.parametrize("interp", [1, 2])
def test_brute_force_8x8(orc, interp):
    """Sum over every source pixel of K(x-k) K(y-l) src[l, k] equals the
    windowed gather, for positions inside, across and beyond the edges."""
    rng = np.random.default_rng(3)
    src = rng.normal(10, 3, (8, 8)).astype(np.float32)
    pts = rng.uniform(-3.5, 10.5, (400, 2))
    k = np.arange(8)
    S = np.array([np.sum(_kernel(px - k, interp, -0.5)[None, :] * _kernel(py - k, interp, -0.5)[:, None]
                         * src.astype(np.float64)) for px, py in pts])
    F = np.array([np.sum(_kernel(px - k, interp, -0.5)[None, :] * _kernel(py - k, interp, -0.5)[:, None])
                  for px, py in pts])
    out, fp, _ = orc.interp_at(src, pts, interp)
    cov = F > 0
    assert np.array_equal(fp > 0, cov)
    assert np.abs(fp[cov] - F[cov]).max() <= 1e-13
    assert np.abs(out[cov] - S[cov] / F[cov]).max() <= 1e-10 * np.abs(S[cov] / F[cov]).max()
    assert np.all(out[~cov] == 0.0)


@pytest.mark.parametrize("interp", [1, 2])
def test_condition_scale_brute_force_and_closed_form(orc, interp):
    """The scale the value tolerance is measured against, sum |w v| / F:
    brute force over every source pixel on an 8x8 source of both signs, and
    for a constant source c the closed forms c (bilinear, weights >= 0) and
    c (1 + t(1-t)) (1 + s(1-s)) (interior bicubic with a = -0.5, whose outer
    weights a t (1-t)^2 and a t^2 (1-t) are <= 0)."""
    rng = np.random.default_rng(13)
    src = rng.normal(0, 3, (8, 8)).astype(np.float32)
    pts = rng.uniform(-2.5, 9.5, (400, 2))
    k = np.arange(8)
    A = np.array([np.sum(np.abs(_kernel(px - k, interp, -0.5)[None, :] *
                                _kernel(py - k, interp, -0.5)[:, None] * src.astype(np.float64)))
                  for px, py in pts])
    _, fp, cond = orc.interp_at(src, pts, interp)
    cov = fp > 0
    assert cov.sum() > 200 and (~cov).sum() > 10
    assert np.abs(cond[cov] - A[cov] / fp[cov]).max() <= 1e-12 * np.abs(A[cov] / fp[cov]).max()
    assert np.all(cond[~cov] == 0.0)
    const = np.full((16, 16), 2.5, np.float32)
    inner = rng.uniform(2.0, 13.0, (300, 2))
    _, _, cc = orc.interp_at(const, inner, interp)
    if interp == 1:
        assert np.abs(cc - 2.5).max() <= 1e-14
    else:
        t = inner - np.floor(inner)
        ref = 2.5 * (1 + t[:, 0] * (1 - t[:, 0])) * (1 + t[:, 1] * (1 - t[:, 1]))
        assert np.abs(cc - ref).max() <= 1e-13


def test_nearest_is_closest_pixel_ties_to_even(orc):
    rng = np.random.default_rng(4)
    src = rng.permutation(64).astype(np.float32).reshape(8, 8)
    pts = rng.uniform(-0.49, 7.49, (300, 2))
    pts = np.concatenate([pts, [[2.5, 3.0], [3.5, 3.0], [1.0, 4.5], [0.5, 0.5]]])
    out, fp, _ = orc.interp_at(src, pts, 0)
    for (px, py), o in zip(pts, out):
        d = np.abs(np.arange(8) - px)
        cand = np.flatnonzero(d == d.min())
        ix = cand[0] if len(cand) == 1 else cand[cand % 2 == 0][0]
        d = np.abs(np.arange(8) - py)
        cand = np.flatnonzero(d == d.min())
        iy = cand[0] if len(cand) == 1 else cand[cand % 2 == 0][0]
        assert o == src[iy, ix]
    assert np.all(fp == 1.0)


def test_footprint_closed_forms(orc):
    src = np.ones((16, 16), np.float32)
    pts = np.array([[-0.5, 8.0], [-1.0, 8.0], [15.5, 8.0], [8.0, -0.5], [8.3, 8.7]])
    _, fb, _ = orc.interp_at(src, pts, 1)
    assert np.allclose(fb, [0.5, 0.0, 0.5, 0.5, 1.0], atol=1e-15)
    _, fc, _ = orc.interp_at(src, pts, 2, -0.5)
    assert np.allclose(fc, [0.5, 0.0, 0.5, 0.5, 1.0], atol=1e-15)


# ---------------------------------------------------------------- gradient --


def _small_grad_case(interp=2):
    c = configs.grad(size=48, interp=interp)
    return c, c.extra["src_wcs_true"]


def test_adjoint_identity_source_gradient(orc):
    """<A s, g> = <s, A^T g>: A is linear in the source for a fixed WCS."""
    c, _ = _small_grad_case()
    rng = np.random.default_rng(5)
    g = rng.normal(0, 1, c.out_shape)
    out, _ = orc.reproject(c.src, c.src_wcs, c.tgt_wcs, c.out_shape, c.interp)
    gs, _ = orc.grad(c.src, c.src_wcs, c.tgt_wcs, c.out_shape, c.interp, g)
    lhs = np.sum(out * g)
    rhs = np.sum(c.src.astype(np.float64) * gs)
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(out * g))


def _loss(orc, c, wcs, ref, mask):
    out, _ = orc.reproject(c.src, wcs, c.tgt_wcs, c.out_shape, c.interp, threads=1)
    return np.sum(mask * (out - ref) ** 2)


def _param_views(wcs):
    """(getter, setter) per parameter in the oracle's gradient order."""
    n_ap = (wcs.ap_order + 1) ** 2
    items = []
    items += [("crval", 0), ("crval", 1), ("crpix", 0), ("crpix", 1)]
    items += [("cd", k) for k in range(4)]
    items += [("ap", k) for k in range(n_ap)]
    items += [("bp", k) for k in range((wcs.bp_order + 1) ** 2)]
    return items


def _perturbed(wcs, name, k, h):
    """WCS with parameter (name, k) moved by h; also returns the step that
    was actually taken after rounding (CRVAL ~150 deg quantises a 1e-9 deg
    step by ~1e-5 relative)."""
    if name in ("crval", "crpix"):
        v = list(getattr(wcs, name))
        old = v[k]
        v[k] = old + h
        return wcs.copy(**{name: tuple(v)}), v[k] - old
    arr = getattr(wcs, name).copy()
    old = arr.flat[k]
    arr.flat[k] = old + h
    return wcs.copy(**{name: arr}), arr.flat[k] - old


def _check_fd(orc, c, ref, mask, only=None):
    """Analytic FP64 gradient of L = sum mask (out - ref)^2 at c.src_wcs
    against central differences with steps of 1e-6 px of induced
    displacement, for every parameter (or those named in ``only``).
    Returns the number of parameters checked."""
    out, _ = orc.reproject(c.src, c.src_wcs, c.tgt_wcs, c.out_shape, c.interp)
    g = 2.0 * mask * (out - ref)
    _, gp = orc.grad(c.src, c.src_wcs, c.tgt_wcs, c.out_shape, c.interp, g, want_src=False)
    wcs = c.src_wcs
    s = 0.5 * max(c.src.shape)
    scale_deg = math.sqrt(abs(np.linalg.det(wcs.cd)))
    o = wcs.ap_order
    checked = 0
    for i, (name, k) in enumerate(_param_views(wcs)):
        if only is not None and name not in only:
            continue
        if name == "crval":
            h = 1e-6 * scale_deg
        elif name == "crpix":
            h = 1e-6
        elif name == "cd":
            h = 1e-6 * scale_deg / s
        else:
            p, q = divmod(k, o + 1)
            if p + q > o:
                assert gp[i] == 0.0
                continue
            h = 1e-6 / s ** (p + q)
        wp, hp = _perturbed(wcs, name, k, h)
        wm, hm = _perturbed(wcs, name, k, -h)
        fd = (_loss(orc, c, wp, ref, mask) - _loss(orc, c, wm, ref, mask)) / (hp - hm)
        # Central differences over a 1e-6 px step carry the oracle's position
        # rounding divided by the step.  Through the explicit RA of section
        # 3.2 (RA ~150 deg, ulp 2.8e-14 deg ~ 2e-11 px at 2.85"/px) that is
        # ~2e-5 relative for CRVAL; every other parameter moves the position
        # after the sky stage, where the rounding is ~1e-12 px.
        rel = 2e-5 if name == "crval" else 5e-6
        assert abs(gp[i] - fd) <= rel * abs(fd), (name, k, gp[i], fd)
        checked += 1
    return checked


@pytest.mark.parametrize("interp", [1, 2])
def test_parameter_gradient_vs_central_differences(orc, interp):
    """Analytic FP64 gradient vs central differences with steps of 1e-6 px
    of induced displacement; interior mask so no tap crosses the edge."""
    c, true_w = _small_grad_case(interp)
    ref, _ = orc.reproject(c.src, true_w, c.tgt_wcs, c.out_shape, c.interp)
    pos = orc.reproject(c.src, true_w, c.tgt_wcs, c.out_shape, c.interp, want_pos=True)[2]
    h_, w_ = c.src.shape
    mask = ((pos[..., 0] >= 3) & (pos[..., 0] <= w_ - 4) & (pos[..., 1] >= 3) & (pos[..., 1] <= h_ - 4))
    mask = mask.astype(np.float64)
    _check_fd(orc, c, ref, mask)


@pytest.mark.parametrize("interp", [1, 2])
def test_parameter_gradient_edge_band_vs_central_differences(orc, interp):
    """Analytic gradient vs central differences on the pixels whose taps
    straddle the source edge (footprint strictly between 0 and 1 and not
    near 0): there out = S/F moves with F, so d out / d position carries
    the term -out dF/dposition / F of the footprint normalisation (section
    3.1), which the interior check never sees."""
    c, true_w = _small_grad_case(interp)
    ref, fp_true = orc.reproject(c.src, true_w, c.tgt_wcs, c.out_shape, c.interp)
    mask = ((fp_true > 0.05) & (np.abs(fp_true - 1.0) > 1e-6)).astype(np.float64)
    assert mask.sum() >= 40, mask.sum()
    o = c.src_wcs.ap_order
    assert _check_fd(orc, c, ref, mask) >= 8 + 2 * (o + 1) * (o + 2) // 2


def _wide_field_case():
    """A 64 x 64 frame of 150"/px (2.7 deg across) at Dec +55, rotated 25
    deg, with SIP order 2 and its fitted inverse of order 3; the target is
    offset by a few pixels and rotated 24.5 deg.  Across such a field the
    spherical terms of the sky stages are ~1e-3 of the linear ones, far above
    the finite-difference resolution (on the 2.85"/px frames they are ~1e-6)."""
    rng = np.random.default_rng(31)
    h = w = 64
    from synth.starfield import star_field
    src = star_field(h, w, 100.0, 5.0, 12, 31, rng=rng)
    a, b = draw_sip(2, 32.0, rng)
    true_w = WcsParams.tan((200.0, 55.0), 150.0, 25.0, (h, w), a=a, b=b)
    ap, bp, _ = fit_inverse_sip(a, b, 3, true_w.crpix, (h, w))
    true_w = true_w.copy(ap=ap, bp=bp)
    tw = WcsParams.tan((200.02, 55.01), 150.0, 24.5, (h, w), crpix_offset=(-2.1, 1.3))
    s_deg = 150.0 / 3600.0
    pert = true_w.copy(crval=(true_w.crval[0] + 0.3 * s_deg / math.cos(math.radians(55.0)),
                              true_w.crval[1] - 0.2 * s_deg),
                       crpix=(true_w.crpix[0] + 0.2, true_w.crpix[1] - 0.1),
                       cd=true_w.cd * (1.0 + np.array([[1e-4, -2e-4], [1.5e-4, -1e-4]])))
    return configs.Case("wide", src, pert, tw, (h, w), 1), true_w


def test_sky_gradient_wide_field_vs_central_differences(orc):
    """CRVAL, CRPIX and CD gradients on a wide field, where the derivatives
    of the spherical rotation (section 3.2) weigh in."""
    c, true_w = _wide_field_case()
    ref, _, pos = orc.reproject(c.src, true_w, c.tgt_wcs, c.out_shape, 1, want_pos=True)
    h, w = c.src.shape
    mask = ((pos[..., 0] >= 1) & (pos[..., 0] <= w - 2) & (pos[..., 1] >= 1) &
            (pos[..., 1] <= h - 2)).astype(np.float64)
    assert _check_fd(orc, c, ref, mask, only=("crval", "crpix", "cd")) == 8


def test_gradient_abs_scales_bound_the_sums(orc):
    """The magnitude sums the oracle reports beside its gradient bound the
    gradient entry by entry, equal it for a gradient of one sign per term
    (CRPIX with g > 0 on a ramp whose slope is positive everywhere), and
    scale linearly with g."""
    c, _ = _small_grad_case(2)
    rng = np.random.default_rng(11)
    g = rng.normal(0, 1, c.out_shape)
    gs, gp, gsa, ga = orc.grad(c.src, c.src_wcs, c.tgt_wcs, c.out_shape, 2, g, want_abs=True)
    assert np.all(ga >= np.abs(gp) * (1 - 1e-12)) and np.all(gsa >= np.abs(gs) * (1 - 1e-12))
    gs2, gp2, gsa2, ga2 = orc.grad(c.src, c.src_wcs, c.tgt_wcs, c.out_shape, 2, -3.0 * g,
                                   want_abs=True)
    assert np.allclose(ga2, 3.0 * ga, rtol=1e-13) and np.allclose(gsa2, 3.0 * gsa, rtol=1e-13)
    # ramp source increasing in x: d out / d x > 0 on the interior, so with
    # g = 1 on interior pixels every CRPIX1 term is positive
    h, w = c.src.shape
    ramp = np.tile(np.arange(w, dtype=np.float32) * 2.0 + 5.0, (h, 1))
    pos = orc.reproject(ramp, c.src_wcs, c.tgt_wcs, c.out_shape, 1, want_pos=True)[2]
    inner = ((pos[..., 0] >= 3) & (pos[..., 0] <= w - 4) & (pos[..., 1] >= 3) &
             (pos[..., 1] <= h - 4)).astype(np.float64)
    _, gp3, _, ga3 = orc.grad(ramp, c.src_wcs, c.tgt_wcs, c.out_shape, 1, inner, want_src=False,
                              want_abs=True)
    assert gp3[2] > 0 and abs(ga3[2] - gp3[2]) <= 1e-12 * ga3[2]
    assert abs(gp3[2] - 2.0 * inner.sum()) <= 1e-9 * gp3[2]


# ----------------------------------------------------------------- coadd --
# The stack is defined from the per-frame result (out_i, F_i); these pins tie
# the oracle's sums to closed forms where the footprints are known exactly.


def _half_pixel_pair():
    """Target = frame B's grid; frame A has the same WCS with CRPIX1 + 0.5,
    so A's column of target column x is x + 0.5 and A (30 columns wide)
    covers x <= 28 fully, x = 29 with footprint 1/2 (bilinear) and nothing
    beyond."""
    wb = WcsParams.tan((150.0, 2.0), 2.85, 0.0, (40, 60))
    wa = wb.copy(crpix=(wb.crpix[0] + 0.5, wb.crpix[1]))
    return wa, wb


def test_coadd_half_pixel_edge_closed_form(orc):
    wa, wb = _half_pixel_pair()
    ca, cb = 3.0, 11.0
    sa = np.full((40, 30), ca, np.float32)
    sb = np.full((40, 60), cb, np.float32)
    img, swf, sf = orc.coadd([sa, sb], [wa, wb], wb, (40, 60), "bilinear")
    assert np.allclose(sf[:, :29], 2.0, atol=1e-8) and np.allclose(img[:, :29], (ca + cb) / 2, atol=1e-8)
    assert np.allclose(sf[:, 29], 1.5, atol=1e-8)
    assert np.allclose(img[:, 29], (0.5 * ca + cb) / 1.5, atol=1e-8)
    assert np.allclose(swf[:, 29], 0.5 * ca + cb, atol=1e-7)
    assert np.allclose(sf[:, 30:], 1.0, atol=1e-8) and np.allclose(img[:, 30:], cb, atol=1e-8)


@pytest.mark.parametrize("interp", ["nearest", "bilinear", "bicubic"])
def test_coadd_of_constant_frames_is_constant(orc, interp):
    """Footprint normalisation reproduces a constant frame wherever it
    covers, so a stack of frames of one constant is that constant wherever
    any frame covers, whatever the frames' geometry."""
    tw = WcsParams.tan((150.0, 2.0), 2.85, 0.0, (90, 100))
    rng = np.random.default_rng(5)
    srcs, wcss = [], []
    for k in range(4):
        h, w = int(rng.integers(20, 70)), int(rng.integers(20, 70))
        wcss.append(WcsParams.tan((150.0 + rng.uniform(-0.01, 0.01), 2.0 + rng.uniform(-0.01, 0.01)),
                                  rng.uniform(2.0, 3.5), rng.uniform(-30, 30), (h, w)))
        srcs.append(np.full((h, w), 7.25, np.float32))
    img, swf, sf = orc.coadd(srcs, wcss, tw, (90, 100), interp)
    cov = sf > 0
    assert cov.sum() > 2000 and (~cov).sum() > 100
    assert np.allclose(img[cov], 7.25, rtol=1e-12, atol=0)
    assert np.all(img[~cov] == 0) and np.all(swf[~cov] == 0)


def test_coadd_of_copies_and_invariances(orc):
    c = configs.plain()
    out, fp = orc.reproject(c.src, c.src_wcs, c.tgt_wcs, c.out_shape, "bicubic")
    img, swf, sf = orc.coadd([c.src] * 3, [c.src_wcs] * 3, c.tgt_wcs, c.out_shape, "bicubic")
    cov = fp > 0
    assert np.array_equal(sf > 0, cov)
    assert np.allclose(sf[cov], 3 * fp[cov], rtol=1e-14)
    assert np.allclose(img[cov], out[cov], rtol=1e-12, atol=1e-9)
    # frame order and a common scale of the sources
    w2 = c.src_wcs.copy(crval=(c.src_wcs.crval[0] + 2e-4, c.src_wcs.crval[1] - 1e-4))
    s2 = (c.src * 0.5 + 3.0).astype(np.float32)
    a = orc.coadd([c.src, s2], [c.src_wcs, w2], c.tgt_wcs, c.out_shape, "bilinear")
    b = orc.coadd([s2, c.src], [w2, c.src_wcs], c.tgt_wcs, c.out_shape, "bilinear")
    assert np.allclose(a[0], b[0], rtol=1e-13, atol=1e-10)
    k = orc.coadd([c.src * np.float32(4), s2 * np.float32(4)], [c.src_wcs, w2], c.tgt_wcs,
                  c.out_shape, "bilinear")
    assert np.allclose(k[0], 4 * a[0], rtol=1e-12, atol=1e-9)
    assert np.array_equal(k[2], a[2])


def test_coadd_rows_and_empty_stack(orc):
    c = configs.plain()
    rows = np.array([0, 17, 200, 255], dtype=np.int64)
    full = orc.coadd([c.src], [c.src_wcs], c.tgt_wcs, c.out_shape, "bilinear")
    part = orc.coadd([c.src], [c.src_wcs], c.tgt_wcs, c.out_shape, "bilinear", rows=rows)
    for f, p in zip(full, part):
        assert np.array_equal(f[rows], p)
    img, swf, sf = orc.coadd([], [], c.tgt_wcs, (5, 7), nan_outside=True)
    assert np.all(np.isnan(img)) and not swf.any() and not sf.any()
