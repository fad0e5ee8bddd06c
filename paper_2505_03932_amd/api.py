"""Torch-facing API over the C ABI (argument marshalling only).

PyTorch provides device memory and streams; every step of the reprojection
runs in libdfr's HIP kernels.

  reproject(src, src_wcs, tgt_wcs, shape_out, order)       single image
  Plan(src_shape, src_wcs, tgt_wcs, shape_out).execute(src) one geometry, many images
  calculate_reprojection(source_hdus, target_wcs, ...)     the paper's call
  reproject_batch(srcs, src_wcss, tgt_wcs, shape_out)      many frames
  reproject_batch_cropped(srcs, src_wcss, tgt_wcs, shape)  per-frame windows (batch_boxes)
  coadd_batch(srcs, src_wcss, tgt_wcs, shape_out)          footprint-weighted stack
  ReprojectFn / reproject_differentiable(...)              autograd
  sq_residual(out, ref, mask)                              alignment loss

A WCS is any object with ``crpix``, ``crval``, ``cd`` (2x2) and optional SIP
arrays ``a``, ``b``, ``ap``, ``bp`` ((order+1, order+1), [p, q] = coefficient
of u**p v**q), or a FITS-style header mapping (see :func:`wcs_from_header`).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import DfrError

ORDERS = {"nearest": 0, "nearest-neighbor": 0, "nearest_neighbor": 0, "bilinear": 1,
          "bicubic": 2, 0: 0, 1: 1, 2: 2}
PRECISIONS = {"f32": 0, "fp32": 0, "f64": 1, "fp64": 1, "trig": 2, "trig_f64": 2,
              "f32_anchor": 3, 0: 0, 1: 1, 2: 2, 3: 3}


@dataclass
class Wcs:
    """TAN (+SIP) world coordinate system (FITS conventions, degrees)."""

    crpix: tuple
    crval: tuple
    cd: np.ndarray
    a: Optional[np.ndarray] = None
    b: Optional[np.ndarray] = None
    ap: Optional[np.ndarray] = None
    bp: Optional[np.ndarray] = None


def _sip_from_header(h, name):
    order = int(h.get(f"{name}_ORDER", 0))
    if order <= 0:
        return None
    c = np.zeros((order + 1, order + 1))
    for p in range(order + 1):
        for q in range(order + 1 - p):
            c[p, q] = float(h.get(f"{name}_{p}_{q}", 0.0))
    return c


_LON_LAT = {"RA": "DEC", "GLON": "GLAT", "ELON": "ELAT", "SLON": "SLAT", "HLON": "HLAT"}


def _check_axes(h):
    """The transform is the gnomonic (TAN) one of section 3.2 with axis 1
    the longitude, in degrees.  A header that names another projection,
    swapped or non-celestial axes, another LONPOLE or other units is refused
    rather than reprojected as if it were TAN; a header without CTYPEs is
    taken as TAN."""
    c1, c2 = h.get("CTYPE1"), h.get("CTYPE2")
    if c1 is not None or c2 is not None:
        if c1 is None or c2 is None:
            raise ValueError("CTYPE1 and CTYPE2 must both be given or both be absent")
        c1, c2 = str(c1).strip().upper(), str(c2).strip().upper()
        t1, p1 = c1[:4].rstrip("-"), c1[4:]
        t2, p2 = c2[:4].rstrip("-"), c2[4:]
        for c, p in ((c1, p1), (c2, p2)):
            if p not in ("-TAN", "-TAN-SIP"):
                raise ValueError(f"CTYPE {c!r}: only the gnomonic projection (TAN, TAN-SIP) "
                                 "is supported")
        lat = _LON_LAT.get(t1)
        if lat is None and len(t1) == 4 and t1.endswith("LN"):
            lat = t1[:2] + "LT"
        if lat is None or t2 != lat:
            raise ValueError(f"CTYPE1/CTYPE2 {c1!r}/{c2!r}: axis 1 must be a celestial "
                             "longitude and axis 2 its latitude")
    lp = h.get("LONPOLE")
    if lp is not None and float(lp) != 180.0:
        raise ValueError(f"LONPOLE = {lp!r}: the transform places the celestial pole at "
                         "native longitude 180 deg")
    for k in ("CUNIT1", "CUNIT2"):
        u = h.get(k)
        if u is not None and str(u).strip().lower() not in ("deg", ""):
            raise ValueError(f"{k} = {u!r}: world coordinates must be in degrees")


def wcs_from_header(h) -> Wcs:
    """WCS from a FITS-style header mapping (CRPIXi, CRVALi, CDi_j or
    PCi_j x CDELTi (paper section 3.1), A/B/AP/BP_ORDER and A_p_q ...)."""
    _check_axes(h)
    crpix = (float(h["CRPIX1"]), float(h["CRPIX2"]))
    crval = (float(h["CRVAL1"]), float(h["CRVAL2"]))
    if "CD1_1" in h:
        cd = [float(h.get(k, 0.0)) for k in ("CD1_1", "CD1_2", "CD2_1", "CD2_2")]
    else:
        pc = [float(h.get(k, 1.0 if k in ("PC1_1", "PC2_2") else 0.0))
              for k in ("PC1_1", "PC1_2", "PC2_1", "PC2_2")]
        cdelt = [float(h.get("CDELT1", 1.0)), float(h.get("CDELT2", 1.0))]
        cd = _lib.dfr_cd_from_pc_cdelt(pc, cdelt)
    return Wcs(crpix, crval, np.array(cd).reshape(2, 2), _sip_from_header(h, "A"),
               _sip_from_header(h, "B"), _sip_from_header(h, "AP"), _sip_from_header(h, "BP"))


def as_wcs(w):
    if isinstance(w, dict) or (hasattr(w, "keys") and "CRPIX1" in w):
        return wcs_from_header(w)
    return w


class CWcs:
    """A dfr_wcs struct with the coefficient buffers it points to."""

    def __init__(self, w):
        w = as_wcs(w)
        self.keep = []
        s = _lib.dfr_wcs()
        s.crpix[:] = [float(v) for v in w.crpix]
        s.crval[:] = [float(v) for v in w.crval]
        s.cd[:] = [float(v) for v in np.asarray(w.cd, dtype=np.float64).ravel()]
        for name in ("a", "b", "ap", "bp"):
            c = getattr(w, name, None)
            if c is None:
                setattr(s, name + "_order", 0)
                setattr(s, name, None)
            else:
                c = np.ascontiguousarray(c, dtype=np.float64)
                self.keep.append(c)
                setattr(s, name + "_order", c.shape[0] - 1)
                setattr(s, name, c.ctypes.data)
        self.s = s


def _opts(precision="f32", cubic_a=-0.5, nan_outside=False, tile=0, debug=None,
          deterministic=False):
    o = _lib.dfr_options()
    _lib.dfr_options_init(o)
    o.precision = PRECISIONS[precision]
    o.cubic_a = float(cubic_a)
    o.nan_outside = 1 if nan_outside else 0
    o.tile = int(tile)
    o.debug_positions = debug
    o.deterministic = 1 if deterministic else 0
    return o


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def _check(status: int, where: str):
    if status != _lib.DFR_OK:
        raise DfrError(status, where)


def _src_tensor(src) -> torch.Tensor:
    if not isinstance(src, torch.Tensor):
        src = torch.as_tensor(np.ascontiguousarray(src, dtype=np.float32))
    if not src.is_cuda:
        src = src.cuda()
    if src.dtype != torch.float32:
        src = src.float()
    if src.dim() != 2:
        raise ValueError("source image must be 2-D [rows, cols]")
    if src.stride(1) != 1:
        src = src.contiguous()
    return src


def reproject(src, src_wcs, tgt_wcs, shape_out=None, order="bilinear", *, footprint=True,
              out=None, fp=None, precision="f32", cubic_a=-0.5, nan_outside=False, tile=0,
              debug_positions=False):
    """Reproject one image.  Returns (out, footprint) float32 tensors on the
    source's device (footprint None if footprint=False); with
    debug_positions=True also the float64 [H, W, 2] source positions."""
    src = _src_tensor(src)
    if shape_out is None:
        shape_out = tuple(src.shape)
    oh, ow = int(shape_out[0]), int(shape_out[1])
    dev = src.device
    if out is None:
        out = torch.empty((oh, ow), dtype=torch.float32, device=dev)
    if footprint and fp is None:
        fp = torch.empty((oh, ow), dtype=torch.float32, device=dev)
    pos = torch.empty((oh, ow, 2), dtype=torch.float64, device=dev) if debug_positions else None
    sw, tw = CWcs(src_wcs), CWcs(tgt_wcs)
    o = _opts(precision, cubic_a, nan_outside, tile, _ptr(pos))
    s = _lib.dfr_reproject(src.data_ptr(), src.shape[0], src.shape[1], src.stride(0), sw.s, tw.s,
                           oh, ow, ORDERS[order], _ptr(out), _ptr(fp if footprint else None), o,
                           _stream(dev))
    _check(s, "dfr_reproject")
    if debug_positions:
        return out, (fp if footprint else None), pos
    return out, (fp if footprint else None)


class Plan:
    """A reprojection geometry prepared once (``dfr_plan_create``) and run on
    many images of its source shape (``dfr_plan_execute``): results equal
    :func:`reproject` with the same arguments bit for bit; the per-cell
    models are not recomputed per image."""

    def __init__(self, src_shape, src_wcs, tgt_wcs, shape_out=None, order="bilinear", *,
                 precision="f32", cubic_a=-0.5, nan_outside=False, tile=0, device=None):
        self.src_shape = (int(src_shape[0]), int(src_shape[1]))
        shape_out = self.src_shape if shape_out is None else shape_out
        self.shape_out = (int(shape_out[0]), int(shape_out[1]))
        dev = torch.device(device if device is not None else "cuda")
        self.device = dev if dev.index is not None else torch.device("cuda", torch.cuda.current_device())
        self._handle = None
        sw, tw = CWcs(src_wcs), CWcs(tgt_wcs)
        with torch.cuda.device(self.device):
            s, h = _lib.dfr_plan_create(self.src_shape[0], self.src_shape[1], sw.s, tw.s,
                                        self.shape_out[0], self.shape_out[1], ORDERS[order],
                                        _opts(precision, cubic_a, nan_outside, tile),
                                        _stream(self.device))
        _check(s, "dfr_plan_create")
        self._handle = h

    def execute(self, src, out=None, fp=None, footprint=True):
        """Returns (out, footprint or None) for ``src`` (the plan's shape)."""
        if self._handle is None:
            raise ValueError("plan is closed")
        src = _src_tensor(src)
        if tuple(src.shape) != self.src_shape:
            raise ValueError(f"source shape {tuple(src.shape)} is not the plan's {self.src_shape}")
        oh, ow = self.shape_out
        if out is None:
            out = torch.empty((oh, ow), dtype=torch.float32, device=src.device)
        if footprint and fp is None:
            fp = torch.empty((oh, ow), dtype=torch.float32, device=src.device)
        with torch.cuda.device(src.device):
            s = _lib.dfr_plan_execute(self._handle, src.data_ptr(), src.stride(0), _ptr(out),
                                      _ptr(fp if footprint else None), _stream(src.device))
        _check(s, "dfr_plan_execute")
        return out, (fp if footprint else None)

    def close(self):
        if self._handle is not None:
            torch.cuda.synchronize(self.device)
            h, self._handle = self._handle, None
            _check(_lib.dfr_plan_destroy(h), "dfr_plan_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def calculate_reprojection(source_hdus, target_wcs, shape_out=None, order="bilinear", *,
                           return_footprint=False, device=None):
    """The paper's single call (section 2): ``source_hdus`` is a (data, wcs)
    pair (or an object with .data and .header); ``target_wcs`` a WCS or a
    header mapping; ``shape_out`` defaults to the source shape."""
    if hasattr(source_hdus, "data") and hasattr(source_hdus, "header"):
        data, wcs = source_hdus.data, source_hdus.header
    else:
        data, wcs = source_hdus
    src = torch.as_tensor(np.ascontiguousarray(data, dtype=np.float32)) \
        if not isinstance(data, torch.Tensor) else data
    src = src.to(device or ("cuda" if not src.is_cuda else src.device))
    out, fp = reproject(src, wcs, target_wcs, shape_out, order)
    return (out, fp) if return_footprint else out


def _frames(srcs, wcss):
    frames = (_lib.dfr_frame * len(srcs))()
    keep = []
    for i, (s, w) in enumerate(zip(srcs, wcss)):
        cw = CWcs(w)
        keep.append(cw)
        frames[i].src = s.data_ptr()
        frames[i].h = s.shape[0]
        frames[i].w = s.shape[1]
        frames[i].pitch = s.stride(0)
        frames[i].wcs = cw.s
    return frames, keep


def reproject_batch(srcs: Sequence[torch.Tensor], src_wcss, tgt_wcs, shape_out, order="bilinear",
                    *, outs=None, fps=None, footprint=True, cubic_a=-0.5, nan_outside=False,
                    tile=0, autotune=False):
    """Reproject many frames onto one target grid in one persistent launch.
    Returns (outs, fps): lists of [H, W] float32 tensors."""
    srcs = [_src_tensor(s) for s in srcs]
    oh, ow = int(shape_out[0]), int(shape_out[1])
    dev = srcs[0].device
    if outs is None:
        outs = [torch.empty((oh, ow), dtype=torch.float32, device=dev) for _ in srcs]
    if footprint and fps is None:
        fps = [torch.empty((oh, ow), dtype=torch.float32, device=dev) for _ in srcs]
    frames, keep = _frames(srcs, src_wcss)
    n = len(srcs)
    out_ptrs = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
    fp_ptrs = (C.c_void_p * n)(*[f.data_ptr() for f in fps]) if footprint else None
    tw = CWcs(tgt_wcs)
    o = _opts("f32", cubic_a, nan_outside, tile)
    if autotune:
        s, t = _lib.dfr_autotune_batch(n, frames, tw.s, oh, ow, ORDERS[order], out_ptrs, fp_ptrs,
                                       o, _stream(dev))
        _check(s, "dfr_autotune_batch")
    s = _lib.dfr_reproject_batch(n, frames, tw.s, oh, ow, ORDERS[order], out_ptrs, fp_ptrs, o,
                                 _stream(dev))
    _check(s, "dfr_reproject_batch")
    return outs, (fps if footprint else None)


def batch_boxes(srcs: Sequence[torch.Tensor], src_wcss, tgt_wcs, shape_out, order="bilinear", *,
                cubic_a=-0.5):
    """[n, 4] int array of (x0, y0, w, h): the window of the target grid each
    frame can cover (outside it a frame's batch output is uncovered)."""
    srcs = [_src_tensor(s) for s in srcs]
    n = len(srcs)
    boxes = np.zeros((n, 4), dtype=np.int32)
    if n == 0:
        return boxes
    frames, keep = _frames(srcs, src_wcss)
    tw = CWcs(tgt_wcs)
    s = _lib.dfr_batch_boxes(n, frames, tw.s, int(shape_out[0]), int(shape_out[1]), ORDERS[order],
                             _opts("f32", cubic_a), _stream(srcs[0].device),
                             boxes.ctypes.data_as(C.c_void_p))
    _check(s, "dfr_batch_boxes")
    return boxes


def reproject_batch_cropped(srcs: Sequence[torch.Tensor], src_wcss, tgt_wcs, shape_out,
                            order="bilinear", *, boxes=None, footprint=True, cubic_a=-0.5,
                            nan_outside=False, tile=0):
    """The batch with one window per frame (default: :func:`batch_boxes`).
    Returns (outs, fps, boxes): frame i's [h, w] crops of target pixels
    x0 .. x0+w-1, y0 .. y0+h-1, and the [n, 4] boxes used."""
    srcs = [_src_tensor(s) for s in srcs]
    oh, ow = int(shape_out[0]), int(shape_out[1])
    if boxes is None:
        boxes = batch_boxes(srcs, src_wcss, tgt_wcs, shape_out, order, cubic_a=cubic_a)
    boxes = np.ascontiguousarray(boxes, dtype=np.int32).reshape(len(srcs), 4)
    dev = srcs[0].device if srcs else torch.device("cuda")
    outs = [torch.empty((int(b[3]), int(b[2])), dtype=torch.float32, device=dev) for b in boxes]
    fps = [torch.empty((int(b[3]), int(b[2])), dtype=torch.float32, device=dev)
           for b in boxes] if footprint else None
    n = len(srcs)
    if n == 0:
        return outs, fps, boxes
    frames, keep = _frames(srcs, src_wcss)
    out_ptrs = (C.c_void_p * n)(*[o.data_ptr() if o.numel() else None for o in outs])
    fp_ptrs = (C.c_void_p * n)(*[f.data_ptr() if f.numel() else None for f in fps]) \
        if footprint else None
    tw = CWcs(tgt_wcs)
    s = _lib.dfr_reproject_batch_cropped(n, frames, tw.s, oh, ow, ORDERS[order],
                                         boxes.ctypes.data_as(C.c_void_p), out_ptrs, fp_ptrs,
                                         _opts("f32", cubic_a, nan_outside, tile), _stream(dev))
    _check(s, "dfr_reproject_batch_cropped")
    return outs, fps, boxes


def coadd_batch(srcs: Sequence[torch.Tensor], src_wcss, tgt_wcs, shape_out, order="bilinear",
                *, sum_wf=None, sum_f=None, coadd=True, accumulate=False, cubic_a=-0.5,
                nan_outside=False, tile=0):
    """Stack many frames onto one target grid, each weighted by its footprint.

    Returns (coadd, sum_wf, sum_f): [H, W] float32 tensors with
    sum_wf = sum of out_i * F_i and sum_f = sum of F_i over the frames, and
    coadd = sum_wf / sum_f where sum_f > 0 (None when ``coadd`` is False).
    With ``accumulate`` the given ``sum_wf`` / ``sum_f`` are added to."""
    srcs = [_src_tensor(s) for s in srcs]
    oh, ow = int(shape_out[0]), int(shape_out[1])
    if accumulate and (sum_wf is None or sum_f is None):
        raise ValueError("accumulate needs sum_wf and sum_f")
    dev = srcs[0].device if srcs else (sum_wf.device if sum_wf is not None else torch.device("cuda"))
    if sum_wf is None:
        sum_wf = torch.empty((oh, ow), dtype=torch.float32, device=dev)
    if sum_f is None:
        sum_f = torch.empty((oh, ow), dtype=torch.float32, device=dev)
    for t in (sum_wf, sum_f):
        if t.dtype != torch.float32 or t.shape != (oh, ow) or not t.is_contiguous() or not t.is_cuda:
            raise ValueError("sum_wf and sum_f must be contiguous float32 [H, W] device tensors")
    img = torch.empty((oh, ow), dtype=torch.float32, device=dev) if coadd else None
    frames, keep = _frames(srcs, src_wcss) if srcs else (None, [])
    tw = CWcs(tgt_wcs)
    o = _opts("f32", cubic_a, nan_outside, tile)
    s = _lib.dfr_coadd_batch(len(srcs), frames, tw.s, oh, ow, ORDERS[order], sum_wf.data_ptr(),
                             sum_f.data_ptr(), img.data_ptr() if img is not None else None,
                             1 if accumulate else 0, o, _stream(dev))
    _check(s, "dfr_coadd_batch")
    return img, sum_wf, sum_f


def autotune(src, src_wcs, tgt_wcs, shape_out, order="bilinear", cubic_a=-0.5) -> int:
    """Time every tile shape for this reprojection and cache the fastest."""
    src = _src_tensor(src)
    oh, ow = int(shape_out[0]), int(shape_out[1])
    out = torch.empty((oh, ow), dtype=torch.float32, device=src.device)
    fp = torch.empty_like(out)
    sw, tw = CWcs(src_wcs), CWcs(tgt_wcs)
    s, t = _lib.dfr_autotune(src.data_ptr(), src.shape[0], src.shape[1], src.stride(0), sw.s, tw.s,
                             oh, ow, ORDERS[order], out.data_ptr(), fp.data_ptr(),
                             _opts("f32", cubic_a), _stream(src.device))
    _check(s, "dfr_autotune")
    return t


# ------------------------------------------------------------ gradients --

def wcs_params(w) -> np.ndarray:
    """Source-WCS parameter vector in the gradient order of the C ABI:
    CRVAL(2), CRPIX(2), CD(4), AP[(o+1)^2], BP[(o+1)^2]."""
    w = as_wcs(w)
    parts = [np.asarray(w.crval, float), np.asarray(w.crpix, float),
             np.asarray(w.cd, float).ravel()]
    for c in (w.ap, w.bp):
        if c is not None:
            parts.append(np.asarray(c, float).ravel())
    return np.concatenate(parts)


def wcs_with_params(template, theta) -> Wcs:
    """The template WCS with the parameters of :func:`wcs_params` replaced."""
    t = np.asarray(theta, dtype=np.float64)
    w = as_wcs(template)
    ap = bp = None
    k = 8
    if w.ap is not None:
        n = w.ap.shape[0]
        ap = t[k:k + n * n].reshape(n, n)
        k += n * n
    if w.bp is not None:
        n = w.bp.shape[0]
        bp = t[k:k + n * n].reshape(n, n)
        k += n * n
    return Wcs((t[2], t[3]), (t[0], t[1]), t[4:8].reshape(2, 2), w.a, w.b, ap, bp)


def reproject_backward(src, src_wcs, tgt_wcs, shape_out, order, grad_out, *, want_src=True,
                       want_wcs=True, cubic_a=-0.5, tile=0, deterministic=False):
    """(grad_src float32 [H, W] or None, grad_wcs float64 [n] or None).
    deterministic=True: grad_src bitwise reproducible across runs and tile
    shapes (exact integer sums of contributions on a fixed grid)."""
    src = _src_tensor(src)
    oh, ow = int(shape_out[0]), int(shape_out[1])
    sw, tw = CWcs(src_wcs), CWcs(tgt_wcs)
    gs = torch.empty(src.shape, dtype=torch.float32, device=src.device) if want_src else None
    gw = torch.empty(_lib.dfr_wcs_grad_size(sw.s), dtype=torch.float64,
                     device=src.device) if want_wcs else None
    g = grad_out.contiguous().float()
    s = _lib.dfr_reproject_backward(src.data_ptr(), src.shape[0], src.shape[1], src.stride(0),
                                    sw.s, tw.s, oh, ow, ORDERS[order], g.data_ptr(), _ptr(gs),
                                    _ptr(gw), _opts("f32", cubic_a, tile=tile,
                                                    deterministic=deterministic),
                                    _stream(src.device))
    _check(s, "dfr_reproject_backward")
    return gs, gw


class ReprojectFn(torch.autograd.Function):
    """out = reproject(src, WCS(theta)); differentiable in src and theta
    (theta as in :func:`wcs_params`, float64)."""

    @staticmethod
    def forward(ctx, src, theta, template, tgt_wcs, shape_out, order, cubic_a):
        w = wcs_with_params(template, theta.detach().cpu().numpy())
        out, _ = reproject(src, w, tgt_wcs, shape_out, order, footprint=False, cubic_a=cubic_a)
        ctx.save_for_backward(src)
        ctx.cfg = (w, tgt_wcs, shape_out, order, cubic_a, theta.device)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        (src,) = ctx.saved_tensors
        w, tgt, shape_out, order, a, tdev = ctx.cfg
        gs, gw = reproject_backward(src, w, tgt, shape_out, order, grad_out,
                                    want_src=ctx.needs_input_grad[0],
                                    want_wcs=ctx.needs_input_grad[1], cubic_a=a)
        return gs, (gw.to(tdev) if gw is not None else None), None, None, None, None, None


def reproject_differentiable(src, theta, template, tgt_wcs, shape_out, order="bicubic",
                             cubic_a=-0.5):
    return ReprojectFn.apply(src, theta, template, tgt_wcs, shape_out, order, cubic_a)


def sq_residual(out, ref, mask=None, want_grad=True):
    """(loss [1] float64 tensor, grad_out or None) with
    loss = sum mask*(out-ref)^2 and grad_out = 2*mask*(out-ref)."""
    out = out.contiguous()
    ref = ref.contiguous()
    n = out.numel()
    loss = torch.empty(1, dtype=torch.float64, device=out.device)
    g = torch.empty_like(out) if want_grad else None
    m = mask.contiguous().float() if mask is not None else None
    s = _lib.dfr_sq_residual(out.data_ptr(), ref.data_ptr(), _ptr(m), n, loss.data_ptr(),
                             _ptr(g), _stream(out.device))
    _check(s, "dfr_sq_residual")
    return loss, g


def cell_model(src_wcs, tgt_wcs, cx: int, cy: int) -> dict:
    """The local position model of output cell (cx, cy) the default FP32 path
    evaluates (host only): FP32 coefficients, integer base, certified bound,
    and the distance from a rounding tie within which nearest decides in FP64."""
    s, mx, my, base, bound, cert, tie = _lib.dfr_cell_model(CWcs(src_wcs).s, CWcs(tgt_wcs).s,
                                                           int(cx), int(cy))
    _check(s, "dfr_cell_model")
    return {"coef_x": np.array(mx), "coef_y": np.array(my), "base": base, "bound": bound,
            "certified": bool(cert), "tie": tie}


def release():
    _check(_lib.dfr_release(), "dfr_release")
