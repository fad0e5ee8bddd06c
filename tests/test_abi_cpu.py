"""C-ABI checks that need no GPU: the library loads and exports every entry
point the header declares, host helpers, and every argument error is
reported by its documented status before any device work is enqueued."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from synth import WcsParams, configs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2505_03932_amd import _lib
    return _lib


def declared_functions():
    text = open(os.path.join(ROOT, "include", "dfr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dfr_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L.lib, n), n
    assert set(names) == set(L.EXPORTED)
    assert L.dfr_abi_version() == 3


def test_struct_sizes_match_header(L):
    # dfr_wcs: 8 doubles + 4 int32 + 4 pointers; dfr_options: 40 bytes on LP64
    assert C.sizeof(L.dfr_wcs) == 8 * 8 + 4 * 4 + 4 * 8
    assert C.sizeof(L.dfr_options) == 40
    o = L.dfr_options()
    L.dfr_options_init(o)
    assert o.size == 40 and o.precision == 0 and o.cubic_a == -0.5 and o.tile == 0
    assert o.deterministic == 0 and o.reserved_ == 0


def test_tiles_and_helpers(L):
    assert L.dfr_tile_count() == 12
    shapes = [L.dfr_tile_shape(t) for t in range(1, 13)]
    assert all(s == 0 and w * h in (1024, 2048, 4096) for s, w, h in shapes)
    assert L.dfr_tile_shape(0)[0] == 7 and L.dfr_tile_shape(13)[0] == 7
    assert L.dfr_cd_from_pc_cdelt([0.5, 0.2, -0.1, 0.9], [-2e-4, 3e-4]) == pytest.approx(
        [-1e-4, -4e-5, -3e-5, 2.7e-4])
    assert "WCS" in L.dfr_strerror(3)


def _wcs(L, w):
    from paper_2505_03932_amd.api import CWcs
    return CWcs(w)


def _call(L, src_wcs, tgt_wcs, src_h=8, src_w=8, pitch=8, out_h=4, out_w=4, interp=1,
          out=1, src=1, opt=None):
    return L.dfr_reproject(src, src_h, src_w, pitch, src_wcs.s, tgt_wcs.s, out_h, out_w, interp,
                           out, None, opt, None)


def test_argument_errors(L):
    c = configs.plain(size=16)
    S, T = _wcs(L, c.src_wcs), _wcs(L, c.tgt_wcs)
    # empty output: nothing to do, no device needed
    assert _call(L, S, T, out_h=0) == 0
    assert _call(L, S, T, out_h=-1) == 2
    assert _call(L, S, T, pitch=7) == 2
    assert _call(L, S, T, src=None) == 1
    assert _call(L, S, T, out=None) == 1
    assert _call(L, S, T, interp=3) == 4
    assert L.lib.dfr_reproject(1, 8, 8, 8, None, T.s, 4, 4, 1, 1, None, None, None) == 1
    o = L.dfr_options()
    L.dfr_options_init(o)
    o.size = 8
    assert _call(L, S, T, opt=o) == 7
    L.dfr_options_init(o)
    o.precision = 9
    assert _call(L, S, T, opt=o) == 4
    L.dfr_options_init(o)
    o.tile = 13
    assert _call(L, S, T, opt=o) == 7
    L.dfr_options_init(o)
    o.cubic_a = float("nan")
    assert _call(L, S, T, opt=o) == 7
    L.dfr_options_init(o)
    o.reserved_ = 1
    assert _call(L, S, T, opt=o) == 7


def test_noalloc_limit_and_errors(L):
    """The allocation-free call refuses an output whose model table exceeds
    its fixed scratch (DFR_E_LIMIT) before any device work, and reports the
    other argument errors as dfr_reproject does."""
    c = configs.plain(size=16)
    S, T = _wcs(L, c.src_wcs), _wcs(L, c.tgt_wcs)

    def call(out_h, out_w, opt=None, **kw):
        a = dict(src=1, src_h=8, src_w=8, pitch=8, out=1, interp=1)
        a.update(kw)
        return L.dfr_reproject_noalloc(a["src"], a["src_h"], a["src_w"], a["pitch"], S.s, T.s,
                                       out_h, out_w, a["interp"], a["out"], None, opt, None)

    cells = L.DFR_NOALLOC_SCRATCH_BYTES // 112
    assert cells == 74898
    assert call(9000, 9000) == L.DFR_E_LIMIT  # 282 x 282 cells
    assert call(32, 32 * (cells + 1)) == L.DFR_E_LIMIT
    assert "limit" in L.dfr_strerror(L.DFR_E_LIMIT)
    assert call(0, 9000) == 0
    assert call(4, 4, pitch=7) == 2
    assert call(4, 4, src=None) == 1
    assert call(4, 4, out=None) == 1
    assert call(4, 4, interp=3) == 4
    o = L.dfr_options()
    L.dfr_options_init(o)
    o.size = 8
    assert call(4, 4, opt=o) == 7


@pytest.mark.parametrize("change,code", [
    (dict(crval=(150.0, 90.5)), 3),
    (dict(crval=(float("nan"), 2.0)), 3),
    (dict(crpix=(float("inf"), 1.0)), 3),
    (dict(cd=[[1e-3, 2e-3], [0.5e-3, 1e-3]]), 3),  # singular
])
def test_wcs_errors(L, change, code):
    c = configs.plain(size=16)
    bad = c.src_wcs.copy(**change)
    T = _wcs(L, c.tgt_wcs)
    assert _call(L, _wcs(L, bad), T) == code
    assert _call(L, T, _wcs(L, bad)) == code
    assert L.dfr_check_wcs(_wcs(L, bad).s, True) == code


def test_sip_errors(L):
    c = configs.sip3(scale=0.02)
    T = _wcs(L, c.tgt_wcs)
    w = c.src_wcs
    ap = w.ap.copy()
    ap[4, 4] = 1e-9  # p + q > order
    assert _call(L, _wcs(L, w.copy(ap=ap)), T) == 3
    big = np.zeros((11, 11))
    assert _call(L, _wcs(L, w.copy(ap=big)), T) == 3  # order 10 > DFR_MAX_SIP_ORDER
    nan = w.ap.copy()
    nan[1, 1] = float("nan")
    assert _call(L, _wcs(L, w.copy(ap=nan)), T) == 3
    # a source with forward SIP but no inverse is not supported
    assert _call(L, _wcs(L, w.copy(ap=None, bp=None)), T) == 4
    # ... but a target with forward SIP only is fine (validated as target)
    assert L.dfr_check_wcs(_wcs(L, w.copy(ap=None, bp=None)).s, False) == 0
    s = _wcs(L, w)
    s.s.ap = None  # order > 0 with a NULL coefficient pointer
    assert _call(L, s, T) == 1


def test_batch_backward_loss_errors(L):
    c = configs.plain(size=16)
    S, T = _wcs(L, c.src_wcs), _wcs(L, c.tgt_wcs)
    frames = (L.dfr_frame * 1)()
    frames[0].src = 1
    frames[0].h = 8
    frames[0].w = 8
    frames[0].pitch = 4
    frames[0].wcs = S.s
    outs = (C.c_void_p * 1)(1)
    assert L.dfr_reproject_batch(-1, frames, T.s, 4, 4, 1, outs, None, None, None) == 7
    assert L.dfr_reproject_batch(1, frames, T.s, 4, 4, 1, outs, None, None, None) == 2  # pitch
    frames[0].pitch = 8
    assert L.dfr_reproject_batch(1, frames, T.s, 4, 4, 5, outs, None, None, None) == 4
    assert L.dfr_reproject_batch(0, None, T.s, 4, 4, 1, None, None, None, None) == 0
    o = L.dfr_options()
    L.dfr_options_init(o)
    o.precision = 1
    assert L.dfr_reproject_batch(1, frames, T.s, 4, 4, 1, outs, None, o, None) == 4
    # coadd: the same frame checks, both sums required, FP32 only
    frames[0].pitch = 4
    assert L.dfr_coadd_batch(1, frames, T.s, 4, 4, 1, 1, 1, None, 0, None, None) == 2
    frames[0].pitch = 8
    assert L.dfr_coadd_batch(-1, frames, T.s, 4, 4, 1, 1, 1, None, 0, None, None) == 7
    assert L.dfr_coadd_batch(1, None, T.s, 4, 4, 1, 1, 1, None, 0, None, None) == 1
    assert L.dfr_coadd_batch(1, frames, T.s, 4, 4, 3, 1, 1, None, 0, None, None) == 4
    assert L.dfr_coadd_batch(1, frames, T.s, 4, 4, 1, None, 1, None, 0, None, None) == 1
    assert L.dfr_coadd_batch(1, frames, T.s, 4, 4, 1, 1, None, 1, 0, None, None) == 1
    assert L.dfr_coadd_batch(1, frames, T.s, 4, 4, 1, 1, 1, None, 0, o, None) == 4
    assert L.dfr_coadd_batch(1, frames, T.s, -4, 4, 1, 1, 1, None, 0, None, None) == 2
    assert L.dfr_coadd_batch(1, frames, T.s, 0, 4, 1, None, None, None, 0, None, None) == 0
    # cropped batch and boxes: the same frame checks, boxes inside the output
    bx = (C.c_int32 * 4)(0, 0, 2, 2)
    assert L.dfr_batch_boxes(1, frames, T.s, 4, 4, 1, None, None, None) == 1
    assert L.dfr_batch_boxes(-1, frames, T.s, 4, 4, 1, None, None, bx) == 7
    assert L.dfr_reproject_batch_cropped(1, frames, T.s, 4, 4, 1, None, outs, None, None, None) == 1
    assert L.dfr_reproject_batch_cropped(1, frames, T.s, 4, 4, 1, bx, None, None, None, None) == 1
    bad = (C.c_int32 * 4)(3, 0, 2, 2)  # x0 + w > out_w
    assert L.dfr_reproject_batch_cropped(1, frames, T.s, 4, 4, 1, bad, outs, None, None, None) == 2
    neg = (C.c_int32 * 4)(0, -1, 2, 2)
    assert L.dfr_reproject_batch_cropped(1, frames, T.s, 4, 4, 1, neg, outs, None, None, None) == 2
    nul = (C.c_void_p * 1)(None)
    assert L.dfr_reproject_batch_cropped(1, frames, T.s, 4, 4, 1, bx, nul, None, None, None) == 1
    assert L.dfr_reproject_batch_cropped(1, frames, T.s, 4, 4, 1, bx, outs, None, o, None) == 4
    # plans: argument errors before any device work
    raw = L.lib
    assert raw.dfr_plan_create(8, 8, C.byref(S.s), C.byref(T.s), 4, 4, 1, None, None, None) == 1
    h = C.c_void_p()
    assert raw.dfr_plan_create(8, 8, None, C.byref(T.s), 4, 4, 1, None, None, C.byref(h)) == 1
    assert raw.dfr_plan_create(-8, 8, C.byref(S.s), C.byref(T.s), 4, 4, 1, None, None,
                               C.byref(h)) == 2
    assert raw.dfr_plan_create(8, 8, C.byref(S.s), C.byref(T.s), 4, 4, 3, None, None,
                               C.byref(h)) == 4
    assert raw.dfr_plan_create(8, 8, C.byref(S.s), C.byref(T.s), 4, 4, 1, C.byref(o), None,
                               C.byref(h)) == 4  # FP64 form: no plan
    assert h.value is None
    assert raw.dfr_plan_execute(None, 1, 8, 1, None, None) == 1
    assert raw.dfr_plan_destroy(None) == 0
    # backward: FP32 only, inverse SIP order <= 5, gradient input required
    assert L.dfr_reproject_backward(1, 8, 8, 8, S.s, T.s, 4, 4, 1, None, None, None, None,
                                    None) == 1
    assert L.dfr_reproject_backward(1, 8, 8, 8, S.s, T.s, 4, 4, 1, 1, None, None, o, None) == 4
    hi = c.src_wcs.copy(ap=np.zeros((7, 7)), bp=np.zeros((7, 7)))
    assert L.dfr_reproject_backward(1, 8, 8, 8, _wcs(L, hi).s, T.s, 4, 4, 1, 1, None, None, None,
                                    None) == 4
    assert L.dfr_sq_residual(1, 1, None, -1, 1, None, None) == 2
    assert L.dfr_sq_residual(None, 1, None, 4, 1, None, None) == 1
    assert L.dfr_sq_residual(1, 1, None, 4, None, None, None) == 1
    n = L.dfr_wcs_grad_size(_wcs(L, configs.grad(size=32).src_wcs).s)
    assert n == 8 + 16 + 16


def test_header_front_end(L):
    """FITS-style header -> WCS, CD from PC x CDELT (section 3.1)."""
    from paper_2505_03932_amd.api import wcs_from_header
    h = {"CRPIX1": 10.5, "CRPIX2": 20.0, "CRVAL1": 150.0, "CRVAL2": 2.0, "CDELT1": -2e-4,
         "CDELT2": 2e-4, "PC1_1": 0.9, "PC1_2": 0.1, "PC2_1": -0.1, "PC2_2": 0.9,
         "A_ORDER": 2, "A_2_0": 1e-6, "B_ORDER": 2, "B_0_2": -2e-6,
         "AP_ORDER": 2, "AP_2_0": -1e-6, "BP_ORDER": 2, "BP_0_2": 2e-6}
    w = wcs_from_header(h)
    assert w.cd == pytest.approx(np.array([[-1.8e-4, -2e-5], [-2e-5, 1.8e-4]]))
    assert w.a[2, 0] == 1e-6 and w.b[0, 2] == -2e-6 and w.ap.shape == (3, 3)
    assert L.dfr_check_wcs(_wcs(L, w).s, True) == 0


@pytest.mark.parametrize("keys,ok", [
    ({"CTYPE1": "RA---TAN", "CTYPE2": "DEC--TAN"}, True),
    ({"CTYPE1": "RA---TAN-SIP", "CTYPE2": "DEC--TAN-SIP", "CUNIT1": "deg", "CUNIT2": "deg"}, True),
    ({"CTYPE1": "GLON-TAN", "CTYPE2": "GLAT-TAN"}, True),
    ({"CTYPE1": "RA---SIN", "CTYPE2": "DEC--SIN"}, False),    # another projection
    ({"CTYPE1": "RA---TAN", "CTYPE2": "DEC--ZEA"}, False),
    ({"CTYPE1": "DEC--TAN", "CTYPE2": "RA---TAN"}, False),    # swapped axes
    ({"CTYPE1": "GLON-TAN", "CTYPE2": "DEC--TAN"}, False),    # mismatched pair
    ({"CTYPE1": "RA---TAN"}, False),                          # one axis only
    ({"CUNIT1": "rad"}, False),
    ({"LONPOLE": 180.0, "LATPOLE": 5.0}, True),
    ({"LONPOLE": 0.0}, False),
])
def test_header_axes(keys, ok):
    """The header front end accepts only the gnomonic projection with a
    celestial longitude/latitude pair in degrees (section 3.2)."""
    from paper_2505_03932_amd.api import wcs_from_header
    h = {"CRPIX1": 1.0, "CRPIX2": 1.0, "CRVAL1": 10.0, "CRVAL2": 5.0, "CD1_1": -1e-4,
         "CD2_2": 1e-4, **keys}
    if ok:
        assert wcs_from_header(h).cd[0, 0] == -1e-4
    else:
        with pytest.raises(ValueError):
            wcs_from_header(h)


def test_missing_library_fails_loudly(tmp_path):
    """Without libdfr.so the package refuses to import: no fallback path."""
    import shutil
    import subprocess
    import sys
    import paper_2505_03932_amd as pkg
    src = os.path.dirname(pkg.__file__)
    dst = tmp_path / "paper_2505_03932_amd"
    shutil.copytree(src, dst, ignore=shutil.ignore_patterns("*.so", "__pycache__", "csrc"))
    r = subprocess.run([sys.executable, "-c", "import paper_2505_03932_amd"], cwd=tmp_path,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "libdfr.so is missing" in r.stderr and "no fallback" in r.stderr
