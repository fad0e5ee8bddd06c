"""ctypes wrapper of the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU
baseline of the benchmark may import this package; the product path may not.
It shares no code with the HIP implementation: its only input contract is the
plain :class:`synth.WcsParams` container.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

NEAREST, BILINEAR, BICUBIC = 0, 1, 2
INTERP = {"nearest": 0, "nearest-neighbor": 0, "bilinear": 1, "bicubic": 2}


class OrcWcs(C.Structure):
    _fields_ = [("crpix", C.c_double * 2), ("crval", C.c_double * 2), ("cd", C.c_double * 4),
                ("a_order", C.c_int32), ("b_order", C.c_int32), ("ap_order", C.c_int32),
                ("bp_order", C.c_int32), ("a", C.c_void_p), ("b", C.c_void_p),
                ("ap", C.c_void_p), ("bp", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = _configure(C.CDLL(LIB_PATH))
    return _lib


class use_library:
    """Context manager: route this module's calls to another build of
    oracle.c (the mutation tests plant mistakes in a copy of the source)."""

    def __init__(self, path):
        self.L = _configure(C.CDLL(path))

    def __enter__(self):
        global _lib
        lib()
        self.saved = _lib
        _lib = self.L
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _configure(L):
    dp = C.POINTER(C.c_double)
    L.orc_pix2world.argtypes = [C.POINTER(OrcWcs), C.c_double, C.c_double, dp, dp]
    L.orc_world2pix.argtypes = [C.POINTER(OrcWcs), C.c_double, C.c_double, dp, dp]
    L.orc_world2pix.restype = C.c_int
    L.orc_world2pix_exact.argtypes = [C.POINTER(OrcWcs), C.c_double, C.c_double, dp, dp]
    L.orc_world2pix_exact.restype = C.c_int
    L.orc_pix2world_n.argtypes = [C.POINTER(OrcWcs), C.c_void_p, C.c_int64, C.c_void_p]
    L.orc_world2pix_n.argtypes = [C.POINTER(OrcWcs), C.c_void_p, C.c_int64, C.c_void_p,
                                  C.c_void_p, C.c_int]
    L.orc_reproject_rows.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_int64,
                                     C.POINTER(OrcWcs), C.POINTER(OrcWcs), C.c_int64,
                                     C.c_void_p, C.c_int64, C.c_int, C.c_double, C.c_int,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
    L.orc_interp_at.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_void_p,
                                C.c_int64, C.c_int, C.c_double, C.c_void_p, C.c_void_p,
                                C.c_void_p]
    L.orc_interp.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_double,
                             C.c_double, C.c_int, C.c_double, dp, dp, dp]
    L.orc_n_params.argtypes = [C.POINTER(OrcWcs)]
    L.orc_n_params.restype = C.c_int64
    L.orc_grad.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.POINTER(OrcWcs),
                           C.POINTER(OrcWcs), C.c_int64, C.c_int64, C.c_int, C.c_double,
                           C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_sip_eval.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double]
    L.orc_sip_eval.restype = C.c_double
    L.orc_online_cores.restype = C.c_int
    return L


class _W:
    """Keeps the ctypes struct and the coefficient buffers it points to alive."""

    def __init__(self, w):
        self.keep = []
        s = OrcWcs()
        s.crpix[:] = list(w.crpix)
        s.crval[:] = list(w.crval)
        s.cd[:] = list(np.asarray(w.cd, dtype=np.float64).ravel())
        for name in ("a", "b", "ap", "bp"):
            c = getattr(w, name)
            if c is None:
                setattr(s, name + "_order", 0)
                setattr(s, name, None)
            else:
                c = np.ascontiguousarray(c, dtype=np.float64)
                self.keep.append(c)
                setattr(s, name + "_order", c.shape[0] - 1)
                setattr(s, name, c.ctypes.data)
        self.s = s

    @property
    def ref(self):
        return C.byref(self.s)


def _interp_id(interp):
    return INTERP[interp] if isinstance(interp, str) else int(interp)


def pix2world(w, xy):
    """xy: [n, 2] pixel coordinates -> [n, 2] (ra, dec) degrees."""
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    out = np.empty_like(xy)
    W = _W(w)
    lib().orc_pix2world_n(W.ref, xy.ctypes.data, xy.shape[0], out.ctypes.data)
    return out


def world2pix(w, radec, exact=False):
    """[n, 2] (ra, dec) -> ([n, 2] pixel, [n] valid).  exact=True inverts A/B by
    Newton iteration instead of using AP/BP."""
    radec = np.ascontiguousarray(radec, dtype=np.float64).reshape(-1, 2)
    out = np.empty_like(radec)
    valid = np.empty(radec.shape[0], dtype=np.int32)
    W = _W(w)
    lib().orc_world2pix_n(W.ref, radec.ctypes.data, radec.shape[0], out.ctypes.data,
                          valid.ctypes.data, 1 if exact else 0)
    return out, valid.astype(bool)


def sip_eval(c, u, v):
    c = np.ascontiguousarray(c, dtype=np.float64)
    return lib().orc_sip_eval(c.ctypes.data, c.shape[0] - 1, float(u), float(v))


def reproject(src, src_wcs, tgt_wcs, out_shape=None, interp="bilinear", cubic_a=-0.5,
              rows=None, threads=0, nan_outside=False, want_pos=False):
    """FP64 reprojection of the target rows ``rows`` (default: all).

    Returns (out, fp[, pos]) as float64 arrays of shape [len(rows), W_out]
    (pos: [len(rows), W_out, 2])."""
    src = np.ascontiguousarray(src, dtype=np.float32)
    h, w = src.shape
    if out_shape is None:
        out_shape = (h, w)
    oh, ow = out_shape
    rows = np.arange(oh, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    n = rows.shape[0]
    out = np.empty((n, ow), dtype=np.float64)
    fp = np.empty((n, ow), dtype=np.float64)
    pos = np.empty((n, ow, 2), dtype=np.float64) if want_pos else None
    S, T = _W(src_wcs), _W(tgt_wcs)
    lib().orc_reproject_rows(src.ctypes.data, h, w, w, S.ref, T.ref, ow, rows.ctypes.data, n,
                             _interp_id(interp), float(cubic_a), 1 if nan_outside else 0,
                             out.ctypes.data, fp.ctypes.data,
                             pos.ctypes.data if pos is not None else None, int(threads))
    return (out, fp, pos) if want_pos else (out, fp)


def coadd(srcs, src_wcss, tgt_wcs, out_shape, interp="bilinear", cubic_a=-0.5, rows=None,
          threads=0, nan_outside=False):
    """Footprint-weighted stack of frames on the target rows ``rows``.

    The stacking use of reprojection (section 1) written out from the
    per-frame result of section 3.1: with out_i, F_i the reprojection of
    frame i, sum_wf = sum of out_i * F_i and sum_f = sum of F_i over the
    frames with F_i > 0 (an uncovered pixel has F_i = 0 and contributes
    nothing), and coadd = sum_wf / sum_f where sum_f > 0, else 0 (NaN with
    nan_outside).  Returns (coadd, sum_wf, sum_f), float64 [len(rows), W]."""
    oh, ow = out_shape
    n = oh if rows is None else len(rows)
    sum_wf = np.zeros((n, ow))
    sum_f = np.zeros((n, ow))
    for src, w in zip(srcs, src_wcss):
        if src.size == 0:
            continue
        out, fp = reproject(src, w, tgt_wcs, out_shape, interp, cubic_a, rows=rows,
                            threads=threads)
        cov = fp > 0
        sum_wf[cov] += out[cov] * fp[cov]
        sum_f[cov] += fp[cov]
    img = np.full((n, ow), np.nan if nan_outside else 0.0)
    cov = sum_f > 0
    img[cov] = sum_wf[cov] / sum_f[cov]
    return img, sum_wf, sum_f


def interp_at(src, pos, interp="bilinear", cubic_a=-0.5):
    """Interpolate ``src`` at source positions pos [n, 2].

    Returns (out, fp, cond) with cond = sum|w*src| / F (the scale against
    which a relative error of the normalised value is measured)."""
    src = np.ascontiguousarray(src, dtype=np.float32)
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 2)
    n = pos.shape[0]
    out = np.empty(n)
    fp = np.empty(n)
    cond = np.empty(n)
    h, w = src.shape
    lib().orc_interp_at(src.ctypes.data, h, w, w, pos.ctypes.data, n, _interp_id(interp),
                        float(cubic_a), out.ctypes.data, fp.ctypes.data, cond.ctypes.data)
    return out, fp, cond


def n_params(src_wcs) -> int:
    return int(lib().orc_n_params(_W(src_wcs).ref))


def grad(src, src_wcs, tgt_wcs, out_shape, interp, grad_out, cubic_a=-0.5, want_src=True,
         want_abs=False):
    """Gradient of a loss with dL/dout = grad_out [H_out, W_out].

    Returns (grad_src [H, W] float64 or None, grad_params [n_params]) with the
    parameter order crval(2), crpix(2), cd(4), ap[(o+1)^2], bp[(o+1)^2]; with
    want_abs also (grad_src_abs or None, grad_params_abs): every entry's sum
    of the magnitudes of its per-pixel (and per-tap) terms."""
    src = np.ascontiguousarray(src, dtype=np.float32)
    g = np.ascontiguousarray(grad_out, dtype=np.float64)
    h, w = src.shape
    oh, ow = out_shape
    assert g.shape == (oh, ow)
    S, T = _W(src_wcs), _W(tgt_wcs)
    gp = np.zeros(lib().orc_n_params(S.ref))
    gs = np.zeros((h, w)) if want_src else None
    ga = np.zeros_like(gp) if want_abs else None
    gsa = np.zeros((h, w)) if (want_abs and want_src) else None
    ptr = lambda a: a.ctypes.data if a is not None else None
    lib().orc_grad(src.ctypes.data, h, w, w, S.ref, T.ref, oh, ow, _interp_id(interp),
                   float(cubic_a), g.ctypes.data, ptr(gs), gp.ctypes.data, ptr(gsa), ptr(ga))
    if want_abs:
        return gs, gp, gsa, ga
    return gs, gp


def online_cores() -> int:
    return int(lib().orc_online_cores())
