"""The per-cell position models of the default FP32 path, checked on the CPU
against the FP64 oracle (which the pins tie to the WCS definitions).

For a cell of 32x32 output pixels the library returns the FP32 coefficients
of the cubic its kernels evaluate and a bound it claims on the distance
between that cubic and the exact position map over the whole cell.  Every
pixel of the cell is mapped by the oracle (target pixel -> sky -> source
pixel, section 3.2) and the model, evaluated exactly in FP64, must lie within
the claimed bound.  Maps built to defeat the model (coarse pixels far from
the source tangent point, strong high-order SIP) must come back uncertified
and must still honour their (larger) bound, which is where a wrong remainder
term would show.
"""
import math

import numpy as np
import pytest

from synth import WcsParams, configs
from synth.sipfit import draw_sip

CELL = 32
HALF = 15.5
POWERS = [(0, 0), (0, 1), (0, 2), (0, 3), (1, 0), (1, 1), (1, 2), (2, 0), (2, 1), (3, 0)]


@pytest.fixture(scope="module")
def dfr():
    import paper_2505_03932_amd as d
    return d


def cell_positions(orc, src_wcs, tgt_wcs, cx, cy):
    """Oracle source positions of the cell's pixels: ([32, 32, 2], valid)."""
    ys, xs = np.mgrid[0:CELL, 0:CELL]
    xy = np.stack([xs.ravel() + cx * CELL, ys.ravel() + cy * CELL], axis=1).astype(np.float64)
    pos, valid = orc.world2pix(src_wcs, orc.pix2world(tgt_wcs, xy))
    return pos.reshape(CELL, CELL, 2), valid.reshape(CELL, CELL)


def model_positions(m):
    ys, xs = np.mgrid[0:CELL, 0:CELL]
    a = xs.astype(np.float64) - HALF
    b = ys.astype(np.float64) - HALF
    out = np.zeros((CELL, CELL, 2))
    for k, (i, j) in enumerate(POWERS):
        t = a ** i * b ** j
        out[..., 0] += m["coef_x"][k] * t
        out[..., 1] += m["coef_y"][k] * t
    out[..., 0] += m["base"][0]
    out[..., 1] += m["base"][1]
    return out


def check_cell(dfr, orc, src_wcs, tgt_wcs, cx, cy):
    m = dfr.cell_model(src_wcs, tgt_wcs, cx, cy)
    if m["bound"] >= 1e29:
        assert not m["certified"]
        return m, None
    pos, valid = cell_positions(orc, src_wcs, tgt_wcs, cx, cy)
    assert valid.all()
    err = np.abs(model_positions(m) - pos).max()
    # the oracle's trigonometric chain and the composed map agree to ~1e-10 px
    assert err <= m["bound"] + 1e-8, (cx, cy, err, m["bound"])
    # the bound = truncation (<= 1e-6 when certified) + FP32 coefficient rounding
    a = np.array([HALF ** (i + j) for i, j in POWERS])
    rnd = 2.0 ** -24 * (np.abs(m["coef_x"]) * a).sum() + 2.0 ** -24 * (np.abs(m["coef_y"]) * a).sum()
    if m["certified"]:
        assert m["bound"] <= 1e-6 + rnd * (1 + 1e-6) + 1e-9
    else:
        assert m["bound"] > 1e-6
    return m, err


def sample_cells(out_shape, n, seed):
    h, w = out_shape
    ncx, ncy = (w + CELL - 1) // CELL, (h + CELL - 1) // CELL
    rng = np.random.default_rng(seed)
    cells = {(0, 0), (ncx - 1, 0), (0, ncy - 1), (ncx - 1, ncy - 1), (ncx // 2, ncy // 2)}
    while len(cells) < n:
        cells.add((int(rng.integers(ncx)), int(rng.integers(ncy))))
    return sorted(cells)


@pytest.mark.parametrize("name", ["plain", "sip3", "grad", "pole"])
def test_models_certified_and_within_bound(dfr, orc, name):
    c = {"plain": lambda: configs.plain(),
         "sip3": lambda: configs.sip3(),
         "grad": lambda: configs.grad(size=2048),
         "pole": lambda: configs.pole(size=2048)}[name]()
    worst = 0.0
    for cx, cy in sample_cells(c.out_shape, 12, 7):
        m, err = check_cell(dfr, orc, c.src_wcs, c.tgt_wcs, cx, cy)
        assert m["certified"], (name, cx, cy, m["bound"])
        worst = max(worst, m["bound"])
    print(name, "largest certified bound", worst)


def test_batch_frames_certified(dfr, orc):
    c = configs.batch(images=False)
    for k in (0, 17, 41, 63):
        for cx, cy in sample_cells(c.out_shape, 6, k):
            m, _ = check_cell(dfr, orc, c.src_wcs[k], c.tgt_wcs, cx, cy)
            assert m["certified"]


def test_target_sip_has_no_model(dfr):
    c = configs.plain()
    a, b = draw_sip(2, 128.0, np.random.default_rng(1))
    m = dfr.cell_model(c.src_wcs, c.tgt_wcs.copy(a=a, b=b), 3, 4)
    assert not m["certified"] and m["bound"] >= 1e29


def test_coarse_far_field_is_uncertified_but_bounded(dfr, orc):
    """10 arcmin pixels 25 deg from the source tangent point: the projective
    terms of a cell are too large for a cubic, and the bound says so."""
    tw = WcsParams.tan((150.0, 2.0), 600.0, 10.0, (256, 256))
    sw = WcsParams.tan((151.0, 27.0), 600.0, -5.0, (256, 256))
    seen = 0
    for cx, cy in [(0, 0), (7, 7), (3, 5)]:
        m, err = check_cell(dfr, orc, sw, tw, cx, cy)
        if err is not None:
            assert not m["certified"] and m["bound"] > 1e-6
            seen += 1
    assert seen >= 2


@pytest.mark.parametrize("sigma", [1e-5, 1e-3, 0.1])
def test_high_order_sip_bounded_and_mixed(dfr, orc, sigma):
    """Inverse SIP of order 7 only: its local quartic terms grow with the cube
    of the distance from CRPIX.  Weak (1e-5): cells near the centre certify
    and the outer ones do not; stronger: none certify.  Every model stays
    within its bound, which here is 1e-7 .. 1 px, so a wrong remainder term
    shows."""
    c = configs.strong_sip(sigma=sigma)
    states = []
    for cx, cy in [(0, 0), (7, 0), (0, 7), (7, 7), (3, 3), (4, 4), (3, 4), (1, 5)]:
        m, err = check_cell(dfr, orc, c.src_wcs, c.tgt_wcs, cx, cy)
        assert err is not None
        states.append(m["certified"])
    if sigma == 1e-5:
        assert states.count(False) >= 4 and states.count(True) >= 3, states
    else:
        assert not any(states)


def test_argument_errors(dfr):
    from paper_2505_03932_amd import _lib
    c = configs.plain()
    from paper_2505_03932_amd.api import CWcs
    s = _lib.dfr_cell_model(CWcs(c.src_wcs).s, CWcs(c.tgt_wcs).s, -1, 0)[0]
    assert s == 7  # DFR_E_ARG
    bad = c.src_wcs.copy(cd=np.zeros((2, 2)))
    s = _lib.dfr_cell_model(CWcs(bad).s, CWcs(c.tgt_wcs).s, 0, 0)[0]
    assert s == 3  # DFR_E_WCS
