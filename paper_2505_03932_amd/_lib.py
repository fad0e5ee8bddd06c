"""ctypes binding of libdfr.so: the C-ABI entry points under their C names,
with the structs of ``include/dfr.h`` mirrored.  Pure argument marshalling:
every step of the computation runs in the library's HIP kernels.

Importing this module loads the library and raises if it is missing: there
is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdfr.so")

DFR_MAX_SIP_ORDER = 9
DFR_NEAREST, DFR_BILINEAR, DFR_BICUBIC = 0, 1, 2
DFR_PREC_F32, DFR_PREC_F64, DFR_PREC_TRIG_F64, DFR_PREC_F32_ANCHOR = 0, 1, 2, 3
DFR_OK = 0
STATUS_NAMES = {0: "DFR_OK", 1: "DFR_E_NULL", 2: "DFR_E_SHAPE", 3: "DFR_E_WCS",
                4: "DFR_E_UNSUPPORTED", 5: "DFR_E_DEVICE", 6: "DFR_E_NOMEM", 7: "DFR_E_ARG",
                8: "DFR_E_LIMIT"}
DFR_E_LIMIT = 8
DFR_NOALLOC_SCRATCH_BYTES = 8 << 20

EXPORTED = [
    "dfr_options_init", "dfr_reproject", "dfr_reproject_noalloc", "dfr_plan_create", "dfr_plan_execute",
    "dfr_plan_destroy", "dfr_reproject_batch", "dfr_batch_boxes", "dfr_reproject_batch_cropped",
    "dfr_coadd_batch",
    "dfr_wcs_grad_size",
    "dfr_reproject_backward", "dfr_sq_residual", "dfr_autotune", "dfr_autotune_batch",
    "dfr_tile_count", "dfr_tile_shape", "dfr_cd_from_pc_cdelt", "dfr_check_wcs",
    "dfr_cell_model", "dfr_release", "dfr_strerror", "dfr_abi_version",
]


class dfr_wcs(C.Structure):
    _fields_ = [("crpix", C.c_double * 2), ("crval", C.c_double * 2), ("cd", C.c_double * 4),
                ("a_order", C.c_int32), ("b_order", C.c_int32), ("ap_order", C.c_int32),
                ("bp_order", C.c_int32), ("a", C.c_void_p), ("b", C.c_void_p),
                ("ap", C.c_void_p), ("bp", C.c_void_p)]


class dfr_options(C.Structure):
    _fields_ = [("size", C.c_uint32), ("precision", C.c_int32), ("cubic_a", C.c_double),
                ("nan_outside", C.c_int32), ("tile", C.c_int32),
                ("debug_positions", C.c_void_p), ("deterministic", C.c_int32),
                ("reserved_", C.c_int32)]


class dfr_frame(C.Structure):
    _fields_ = [("src", C.c_void_p), ("h", C.c_int32), ("w", C.c_int32), ("pitch", C.c_int64),
                ("wcs", dfr_wcs)]


class DfrError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)} ({dfr_strerror(status)})")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2505_03932_amd.build` "
            "(hipcc, gfx950).  There is no fallback implementation.")
    # libdfr needs libamdhip64.so.7, and torch ships its own copy under the
    # same soname: whichever is loaded first serves both.  Loading torch
    # first makes the library run on torch's HIP runtime, so torch's streams
    # and device pointers are valid in it (the other order leaves torch and
    # libdfr on different runtime instances).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, st = C.c_void_p, C.c_int32, C.c_int64, C.c_int
    W = C.POINTER(dfr_wcs)
    O = C.POINTER(dfr_options)
    L.dfr_options_init.argtypes = [O]
    L.dfr_options_init.restype = None
    L.dfr_reproject.argtypes = [vp, i32, i32, i64, W, W, i32, i32, st, vp, vp, O, vp]
    L.dfr_reproject.restype = st
    L.dfr_reproject_noalloc.argtypes = [vp, i32, i32, i64, W, W, i32, i32, st, vp, vp, O, vp]
    L.dfr_reproject_noalloc.restype = st
    L.dfr_plan_create.argtypes = [i32, i32, W, W, i32, i32, st, O, vp, C.POINTER(vp)]
    L.dfr_plan_create.restype = st
    L.dfr_plan_execute.argtypes = [vp, vp, i64, vp, vp, vp]
    L.dfr_plan_execute.restype = st
    L.dfr_plan_destroy.argtypes = [vp]
    L.dfr_plan_destroy.restype = st
    L.dfr_reproject_batch.argtypes = [i32, C.POINTER(dfr_frame), W, i32, i32, st, vp, vp, O, vp]
    L.dfr_reproject_batch.restype = st
    L.dfr_batch_boxes.argtypes = [i32, C.POINTER(dfr_frame), W, i32, i32, st, O, vp, vp]
    L.dfr_batch_boxes.restype = st
    L.dfr_reproject_batch_cropped.argtypes = [i32, C.POINTER(dfr_frame), W, i32, i32, st, vp, vp,
                                              vp, O, vp]
    L.dfr_reproject_batch_cropped.restype = st
    L.dfr_coadd_batch.argtypes = [i32, C.POINTER(dfr_frame), W, i32, i32, st, vp, vp, vp, i32,
                                  O, vp]
    L.dfr_coadd_batch.restype = st
    L.dfr_wcs_grad_size.argtypes = [W]
    L.dfr_wcs_grad_size.restype = i64
    L.dfr_reproject_backward.argtypes = [vp, i32, i32, i64, W, W, i32, i32, st, vp, vp, vp, O, vp]
    L.dfr_reproject_backward.restype = st
    L.dfr_sq_residual.argtypes = [vp, vp, vp, i64, vp, vp, vp]
    L.dfr_sq_residual.restype = st
    L.dfr_autotune.argtypes = [vp, i32, i32, i64, W, W, i32, i32, st, vp, vp, O, vp,
                               C.POINTER(i32)]
    L.dfr_autotune.restype = st
    L.dfr_autotune_batch.argtypes = [i32, C.POINTER(dfr_frame), W, i32, i32, st, vp, vp, O, vp,
                                     C.POINTER(i32)]
    L.dfr_autotune_batch.restype = st
    L.dfr_tile_count.argtypes = []
    L.dfr_tile_count.restype = i32
    L.dfr_tile_shape.argtypes = [i32, C.POINTER(i32), C.POINTER(i32)]
    L.dfr_tile_shape.restype = st
    L.dfr_cd_from_pc_cdelt.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.POINTER(C.c_double)]
    L.dfr_cd_from_pc_cdelt.restype = None
    L.dfr_check_wcs.argtypes = [W, i32]
    L.dfr_check_wcs.restype = st
    D = C.POINTER(C.c_double)
    L.dfr_cell_model.argtypes = [W, W, i32, i32, D, D, C.POINTER(i32), D, C.POINTER(i32), D]
    L.dfr_cell_model.restype = st
    L.dfr_release.argtypes = []
    L.dfr_release.restype = st
    L.dfr_strerror.argtypes = [st]
    L.dfr_strerror.restype = C.c_char_p
    L.dfr_abi_version.argtypes = []
    L.dfr_abi_version.restype = i32
    return L


lib = _load()


# ------------------------------------------------ the C entry points, 1:1 --

def dfr_options_init(opt: dfr_options) -> None:
    lib.dfr_options_init(C.byref(opt))


def dfr_reproject(src, src_h, src_w, src_pitch, src_wcs, tgt_wcs, out_h, out_w, interp, out,
                  footprint, opt, stream) -> int:
    return lib.dfr_reproject(src, src_h, src_w, src_pitch, C.byref(src_wcs), C.byref(tgt_wcs),
                             out_h, out_w, interp, out, footprint,
                             C.byref(opt) if opt is not None else None, stream)


def dfr_reproject_noalloc(src, src_h, src_w, src_pitch, src_wcs, tgt_wcs, out_h, out_w, interp,
                          out, footprint, opt, stream) -> int:
    return lib.dfr_reproject_noalloc(src, src_h, src_w, src_pitch, C.byref(src_wcs),
                                     C.byref(tgt_wcs), out_h, out_w, interp, out, footprint,
                                     C.byref(opt) if opt is not None else None, stream)


def dfr_reproject_batch(n, frames, tgt_wcs, out_h, out_w, interp, outs, footprints, opt,
                        stream) -> int:
    return lib.dfr_reproject_batch(n, frames, C.byref(tgt_wcs), out_h, out_w, interp, outs,
                                   footprints, C.byref(opt) if opt is not None else None, stream)


def dfr_plan_create(src_h, src_w, src_wcs, tgt_wcs, out_h, out_w, interp, opt, stream):
    """Returns (status, plan handle or None)."""
    h = C.c_void_p()
    s = lib.dfr_plan_create(src_h, src_w, C.byref(src_wcs), C.byref(tgt_wcs), out_h, out_w, interp,
                            C.byref(opt) if opt is not None else None, stream, C.byref(h))
    return s, h.value


def dfr_plan_execute(plan, src, src_pitch, out, footprint, stream) -> int:
    return lib.dfr_plan_execute(plan, src, src_pitch, out, footprint, stream)


def dfr_plan_destroy(plan) -> int:
    return lib.dfr_plan_destroy(plan)


def dfr_batch_boxes(n, frames, tgt_wcs, out_h, out_w, interp, opt, stream, boxes) -> int:
    return lib.dfr_batch_boxes(n, frames, C.byref(tgt_wcs), out_h, out_w, interp,
                               C.byref(opt) if opt is not None else None, stream, boxes)


def dfr_reproject_batch_cropped(n, frames, tgt_wcs, out_h, out_w, interp, boxes, outs, footprints,
                                opt, stream) -> int:
    return lib.dfr_reproject_batch_cropped(n, frames, C.byref(tgt_wcs), out_h, out_w, interp,
                                           boxes, outs, footprints,
                                           C.byref(opt) if opt is not None else None, stream)


def dfr_coadd_batch(n, frames, tgt_wcs, out_h, out_w, interp, sum_wf, sum_f, coadd, accumulate,
                    opt, stream) -> int:
    return lib.dfr_coadd_batch(n, frames, C.byref(tgt_wcs), out_h, out_w, interp, sum_wf, sum_f,
                               coadd, accumulate, C.byref(opt) if opt is not None else None,
                               stream)


def dfr_wcs_grad_size(src_wcs) -> int:
    return int(lib.dfr_wcs_grad_size(C.byref(src_wcs)))


def dfr_reproject_backward(src, src_h, src_w, src_pitch, src_wcs, tgt_wcs, out_h, out_w, interp,
                           grad_out, grad_src, grad_wcs, opt, stream) -> int:
    return lib.dfr_reproject_backward(src, src_h, src_w, src_pitch, C.byref(src_wcs),
                                      C.byref(tgt_wcs), out_h, out_w, interp, grad_out, grad_src,
                                      grad_wcs, C.byref(opt) if opt is not None else None, stream)


def dfr_sq_residual(out, ref, mask, n, loss, grad_out, stream) -> int:
    return lib.dfr_sq_residual(out, ref, mask, n, loss, grad_out, stream)


def dfr_autotune(src, src_h, src_w, src_pitch, src_wcs, tgt_wcs, out_h, out_w, interp, out,
                 footprint, opt, stream):
    t = C.c_int32(0)
    s = lib.dfr_autotune(src, src_h, src_w, src_pitch, C.byref(src_wcs), C.byref(tgt_wcs), out_h,
                         out_w, interp, out, footprint, C.byref(opt) if opt is not None else None,
                         stream, C.byref(t))
    return s, t.value


def dfr_autotune_batch(n, frames, tgt_wcs, out_h, out_w, interp, outs, footprints, opt, stream):
    t = C.c_int32(0)
    s = lib.dfr_autotune_batch(n, frames, C.byref(tgt_wcs), out_h, out_w, interp, outs,
                               footprints, C.byref(opt) if opt is not None else None, stream,
                               C.byref(t))
    return s, t.value


def dfr_tile_count() -> int:
    return int(lib.dfr_tile_count())


def dfr_tile_shape(tile: int):
    w, h = C.c_int32(0), C.c_int32(0)
    s = lib.dfr_tile_shape(tile, C.byref(w), C.byref(h))
    return s, w.value, h.value


def dfr_cd_from_pc_cdelt(pc, cdelt):
    p = (C.c_double * 4)(*[float(v) for v in pc])
    d = (C.c_double * 2)(*[float(v) for v in cdelt])
    out = (C.c_double * 4)()
    lib.dfr_cd_from_pc_cdelt(p, d, out)
    return list(out)


def dfr_check_wcs(wcs, as_source: bool) -> int:
    return lib.dfr_check_wcs(C.byref(wcs), 1 if as_source else 0)


def dfr_cell_model(src_wcs, tgt_wcs, cx: int, cy: int):
    """Returns (status, coef_x[10], coef_y[10], (base_x, base_y), bound, certified, tie)."""
    cxs, cys = (C.c_double * 10)(), (C.c_double * 10)()
    base = (C.c_int32 * 2)()
    bound, cert, tie = C.c_double(0.0), C.c_int32(0), C.c_double(0.0)
    s = lib.dfr_cell_model(C.byref(src_wcs), C.byref(tgt_wcs), cx, cy, cxs, cys, base,
                           C.byref(bound), C.byref(cert), C.byref(tie))
    return s, list(cxs), list(cys), (base[0], base[1]), bound.value, cert.value, tie.value


def dfr_release() -> int:
    return lib.dfr_release()


def dfr_strerror(status: int) -> str:
    r = lib.dfr_strerror(status)
    return r.decode() if r else "?"


def dfr_abi_version() -> int:
    return int(lib.dfr_abi_version())
