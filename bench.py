#!/usr/bin/env python3
"""Benchmark of the reprojection hot path on one MI355X.

Headline: output Mpix/s of the bilinear forward reprojection of the
6000x4000 frame with SIP A/B order 3 and fitted inverse AP/BP order 4
(target 6000x4000 TAN, 40 px offset, rotated 0.3 deg), output and footprint
float32, inputs resident in HBM.  One step = one full forward pass over the
frame through the C ABI: host set-up, the per-cell position-model prepass and
the tile kernel (two launches on the caller's stream).

Four buffer sets (source, output, footprint) are rotated, so the sources
alone (4 x 96 MB) exceed the 256 MB last-level cache and every step reads its
source from HBM.

Beside it: the roofline of the dominant kernel, the tile kernel
(algorithmic bytes per launch over its average duration, HIP events on its
stream around launches of that kernel alone through a plan that holds the
frame's cell models, against 8 TB/s), the same for the whole step, a
measured device-copy bandwidth, the HBM traffic the committed rocprofv3 PMC
summary measured, the other forms of the path (nearest and bicubic, the
FP64 and trigonometric forms, forward+backward on the 2048^2 alignment case,
the 64-frame batch and its coadd, the +89.5 deg precision case), a short run
of the paper's size sweep, and the oracle leg: the FP64 CPU oracle timed on
this host (all the cores the process may use, and one thread) and the
position error of every form against it, in pixels.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-extras]
                    [--extras forms,grad,pole,batch,sweep] [--no-cpu-baseline]
                    [--calibrate-copy] [--sweep]

--sweep prints, instead, one JSON line with the size sweep of the paper's
scaling benchmark: 256^2 .. 4000x6000 x {nearest, bilinear, bicubic} x
{with, without SIP}, with the given steps per point (the default line holds
the same sweep at 5 timed steps per point).

--calibrate-copy adds, after the timed steps, three plain device copies of a
512,000,000-byte buffer, each from a source pushed out of the caches by a
512 MB fill just before it: the PMC runs read FETCH_SIZE and WRITE_SIZE of
that known-size copy to scale the counters.
"""
from __future__ import annotations

import argparse
import ctypes as C
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2505_03932_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp", ".cpp")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def stored_profile(name: str, tag: str):
    """A record of a committed rocprofv3 summary (`<!--tag {json}-->`), if it
    was taken on the current kernel sources."""
    p = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(p):
        return None
    with open(p) as f:
        for line in f:
            if line.startswith(f"<!--{tag} "):
                d = json.loads(line[len(f"<!--{tag} "):].rsplit("-->", 1)[0])
                if d.get("kernel_source_hash") == kernel_source_hash():
                    return d
    return None


class Frame:
    """Device buffers and prebuilt C structs for repeated launches."""

    def __init__(self, dfr, src_np, sw, tw, shape, interp, n_sets=4, precision="f32", fp=True):
        import torch
        from paper_2505_03932_amd import api
        self.api = api
        self.lib = api._lib
        self.shape = shape
        self.interp = api.ORDERS[interp]
        self.sets = []
        for _ in range(n_sets):
            s = torch.from_numpy(src_np).cuda()
            o = torch.empty(shape, dtype=torch.float32, device="cuda")
            f = torch.empty(shape, dtype=torch.float32, device="cuda") if fp else None
            self.sets.append((s, o, f))
        self.sw = api.CWcs(sw)
        self.tw = api.CWcs(tw)
        self.opt = api._opts(precision)
        self.stream = torch.cuda.current_stream().cuda_stream
        self.k = 0

    def step(self):
        s, o, f = self.sets[self.k % len(self.sets)]
        self.k += 1
        st = self.lib.dfr_reproject(s.data_ptr(), s.shape[0], s.shape[1], s.stride(0), self.sw.s,
                                    self.tw.s, self.shape[0], self.shape[1], self.interp,
                                    o.data_ptr(), f.data_ptr() if f is not None else None,
                                    self.opt, self.stream)
        if st != 0:
            raise RuntimeError(f"dfr_reproject failed: {st}")


def time_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def time_tile_kernel(dfr, frame, case, steps, warmup):
    """Average duration of the tile kernel alone over `steps` launches: a
    plan holds the frame's cell models, each dfr_plan_execute is one launch
    (raw C calls with prebuilt arguments, alternating the frame's buffer
    sets like the step)."""
    from paper_2505_03932_amd import api
    plan = api.Plan(case.src.shape, case.src_wcs, case.tgt_wcs, case.out_shape, "bilinear")
    lib, stream, k = api._lib, frame.stream, [0]

    def launch():
        s, o, f = frame.sets[k[0] % len(frame.sets)]
        k[0] += 1
        st = lib.dfr_plan_execute(plan._handle, s.data_ptr(), s.stride(0), o.data_ptr(),
                                  f.data_ptr(), stream)
        if st != 0:
            raise RuntimeError(f"dfr_plan_execute failed: {st}")

    ms, _ = time_steps(launch, steps, warmup)
    plan.close()
    return ms


def touched_source_pixels(dfr, src_t, sw, tw, shape, interp):
    """Distinct source pixels the interpolation reads: the support of the
    adjoint applied to an all-ones output gradient."""
    import torch
    g = torch.ones(shape, dtype=torch.float32, device="cuda")
    gs, _ = dfr.reproject_backward(src_t, sw, tw, shape, interp, g, want_wcs=False)
    torch.cuda.synchronize()
    return int(torch.count_nonzero(gs).item())


def cpu_threads():
    """Threads the oracle may use here: the CPUs this process may run on,
    capped by OMP_NUM_THREADS where the host sets it (a host shared between
    GPUs gives each GPU's jobs a share of its cores)."""
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count() or 1
    cap = os.environ.get("OMP_NUM_THREADS", "")
    n = aff
    if cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n), aff, cap or None


def cpu_baseline(case, interp):
    """The FP64 oracle on this host: whole passes over the headline frame on
    every core the process may use until about 12 s of CPU work (wall time
    x threads) are done (at most 8 passes), then one thread on every 4th row
    of the frame."""
    import oracle
    threads, aff, cap = cpu_threads()
    oh, ow = case.out_shape
    rows8 = np.arange(8, dtype=np.int64)
    oracle.reproject(case.src, case.src_wcs, case.tgt_wcs, case.out_shape, interp, rows=rows8,
                     threads=threads)
    passes = 0
    t0 = time.perf_counter()
    while True:
        oracle.reproject(case.src, case.src_wcs, case.tgt_wcs, case.out_shape, interp,
                         threads=threads)
        passes += 1
        dt = time.perf_counter() - t0
        if dt * threads >= 12.0 or passes >= 8:
            break
    npx = passes * oh * ow
    rows = np.arange(0, oh, 4, dtype=np.int64)
    t1 = time.perf_counter()
    oracle.reproject(case.src, case.src_wcs, case.tgt_wcs, case.out_shape, interp, rows=rows,
                     threads=1)
    dt1 = time.perf_counter() - t1
    npx1 = len(rows) * ow
    return {"value": round(npx / dt / 1e6, 3), "unit": "Mpix/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{passes} whole passes over the 6000x4000 SIP frame ({npx} px, {interp}), "
                      f"FP64, {dt:.1f} s wall on {threads} threads",
            "host_cpus": os.cpu_count(), "affinity_cpus": aff, "omp_num_threads": cap,
            "one_thread": {"value": round(npx1 / dt1 / 1e6, 3), "unit": "Mpix/s", "cores": 1,
                           "sample": f"every 4th row of the same frame ({npx1} px), "
                                     f"{dt1:.1f} s wall"}}


def _pos_err(dfr, src_t, src_np, sw, tw, shape, interp, rows, precision="f32"):
    """Max and RMS distance (px) between the source positions a GPU run
    interpolated at (its debug output) and the oracle's FP64 positions, on
    the target rows `rows`."""
    import torch
    import oracle
    _, _, pos = dfr.reproject(src_t, sw, tw, shape, interp, precision=precision,
                              debug_positions=True)
    gp = pos[torch.from_numpy(rows).to(pos.device)].cpu().numpy()
    del pos
    _, _, op = oracle.reproject(src_np, sw, tw, shape, interp, rows=rows, want_pos=True)
    ok = np.isfinite(gp[..., 0]) & np.isfinite(op[..., 0])
    d = np.hypot(*(gp[ok] - op[ok]).T) if ok.any() else np.zeros(1)
    return {"max": float(d.max()), "rms": float(np.sqrt(np.mean(d * d))),
            "px_compared": int(ok.sum())}


def _rows(h, n):
    return np.unique(np.linspace(0, h - 1, n).round().astype(np.int64))


def position_errors(dfr, case, forms):
    """Position error against the oracle for the headline and every form in
    `forms` (sampled rows of each workload)."""
    import torch
    from synth import configs
    out = {}
    src = torch.from_numpy(case.src).cuda()
    rows = _rows(case.out_shape[0], 16)
    args = (src, case.src, case.src_wcs, case.tgt_wcs, case.out_shape)
    out["sip3_bilinear"] = _pos_err(dfr, *args, "bilinear", rows)
    for key, interp, prec in (("sip3_nearest", "nearest", "f32"),
                              ("sip3_bicubic", "bicubic", "f32"),
                              ("sip3_bilinear_f32_anchor", "bilinear", "f32_anchor"),
                              ("sip3_bilinear_f64", "bilinear", "f64"),
                              ("sip3_bilinear_trig", "bilinear", "trig")):
        if key in forms:
            out[key] = _pos_err(dfr, *args, interp, rows, prec)
    del src
    if "grad2048_bicubic_fwd" in forms:
        c = configs.grad()
        s = torch.from_numpy(c.src).cuda()
        e = _pos_err(dfr, s, c.src, c.src_wcs, c.tgt_wcs, c.out_shape, "bicubic",
                     _rows(c.out_shape[0], 16))
        out["grad2048_bicubic_fwd"] = e
        out["grad2048_bicubic_fwd_bwd"] = e
        out["grad2048_bicubic_fwd_bwd_deterministic"] = e
    if "pole8192_bilinear_f32" in forms:
        c = configs.pole()
        s = torch.from_numpy(c.src).cuda()
        for prec in ("f32", "f64"):
            out[f"pole8192_bilinear_{prec}"] = _pos_err(dfr, s, c.src, c.src_wcs, c.tgt_wcs,
                                                        c.out_shape, "bilinear",
                                                        _rows(c.out_shape[0], 8), prec)
        del s
    if "batch64_8192_bilinear" in forms:
        c = configs.batch()
        worst = None
        for i in (0, 21, 42, 63):
            s = torch.from_numpy(c.src[i]).cuda()
            e = _pos_err(dfr, s, c.src[i], c.src_wcs[i], c.tgt_wcs, c.out_shape, "bilinear",
                         _rows(c.out_shape[0], 8))
            if worst is None or e["max"] > worst["max"]:
                worst = dict(e, frame=i)
        for key in ("batch64_8192_bilinear", "batch64_8192_bilinear_cropped",
                    "coadd64_8192_bilinear"):
            out[key] = dict(worst, note="frames 0, 21, 42, 63; the largest")
    torch.cuda.empty_cache()
    return out


def copy_bandwidth():
    """A plain device-to-device copy of 1 GiB (torch copy_), best of 5, as
    read + write bytes per second: what a streaming kernel reaches here."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = 1e30
    for _ in range(5):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    torch.cuda.empty_cache()
    return {"copy_gbs": round(2 * 4 * n / best / 1e6, 1), "copy_bytes": 2 * 4 * n,
            "copy_how": "torch copy_ of a 1 GiB float32 buffer on the device, best of 5"}


# ------------------------------------------------------------------ extras --

def extra_forms(dfr, case, steps):
    """Nearest/bicubic and the FP64 forms on the same frame."""
    res = {}
    npx = case.out_shape[0] * case.out_shape[1]
    for interp in ("nearest", "bicubic"):
        fr = Frame(dfr, case.src, case.src_wcs, case.tgt_wcs, case.out_shape, interp)
        ms, _ = time_steps(fr.step, steps, 2)
        res[f"sip3_{interp}"] = {"mpix_s": round(npx / ms / 1e3, 1), "ms": round(ms, 4)}
        del fr
    fr = Frame(dfr, case.src, case.src_wcs, case.tgt_wcs, case.out_shape, "bilinear",
               precision="f32_anchor")
    ms, _ = time_steps(fr.step, steps, 2)
    res["sip3_bilinear_f32_anchor"] = {"mpix_s": round(npx / ms / 1e3, 1), "ms": round(ms, 4)}
    del fr
    for prec in ("f64", "trig"):
        fr = Frame(dfr, case.src, case.src_wcs, case.tgt_wcs, case.out_shape, "bilinear",
                   precision=prec, n_sets=1)
        ms, _ = time_steps(fr.step, max(2, steps // 4), 1)
        res[f"sip3_bilinear_{prec}"] = {"mpix_s": round(npx / ms / 1e3, 1), "ms": round(ms, 4)}
        del fr
    return res


def extra_grad(dfr, steps):
    """Forward + loss + backward on the 2048^2 bicubic alignment case."""
    import torch
    from synth import configs
    c = configs.grad()
    src = torch.from_numpy(c.src).cuda()
    true_w = c.extra["src_wcs_true"]
    ref, _ = dfr.reproject(src, true_w, c.tgt_wcs, c.out_shape, "bicubic")
    n = c.out_shape[0] * c.out_shape[1]

    def fwd():
        out, _ = dfr.reproject(src, c.src_wcs, c.tgt_wcs, c.out_shape, "bicubic", footprint=False)
        return out

    def step():
        out = fwd()
        loss, g = dfr.sq_residual(out, ref)
        dfr.reproject_backward(src, c.src_wcs, c.tgt_wcs, c.out_shape, "bicubic", g)

    def step_det():
        out = fwd()
        loss, g = dfr.sq_residual(out, ref)
        dfr.reproject_backward(src, c.src_wcs, c.tgt_wcs, c.out_shape, "bicubic", g,
                               deterministic=True)

    ms_f, _ = time_steps(fwd, steps, 2)
    ms_fb, _ = time_steps(step, steps, 2)
    ms_fbd, _ = time_steps(step_det, steps, 2)
    return {"grad2048_bicubic_fwd": {"mpix_s": round(n / ms_f / 1e3, 1), "ms": round(ms_f, 4)},
            "grad2048_bicubic_fwd_bwd": {"mpix_s": round(n / ms_fb / 1e3, 1),
                                         "ms": round(ms_fb, 4)},
            "grad2048_bicubic_fwd_bwd_deterministic": {"mpix_s": round(n / ms_fbd / 1e3, 1),
                                                       "ms": round(ms_fbd, 4)}}


def extra_batch(dfr, steps):
    """64 uneven frames onto one 8192^2 grid in one graph-replayed launch, the
    same frames into per-frame windows (the boxes each frame can cover), and
    coadded (footprint-weighted sums, no per-frame output)."""
    import torch
    from synth import configs
    t0 = time.perf_counter()
    c = configs.batch()
    log(f"batch inputs generated in {time.perf_counter() - t0:.1f} s")
    srcs = [torch.from_numpy(s).cuda() for s in c.src]
    oh, ow = c.out_shape
    outs = [torch.empty((oh, ow), dtype=torch.float32, device="cuda") for _ in srcs]
    fps = [torch.empty((oh, ow), dtype=torch.float32, device="cuda") for _ in srcs]
    tile = dfr.api.reproject_batch(srcs, c.src_wcs, c.tgt_wcs, c.out_shape, "bilinear",
                                   outs=outs, fps=fps, autotune=True)
    ms, _ = time_steps(lambda: dfr.reproject_batch(srcs, c.src_wcs, c.tgt_wcs, c.out_shape,
                                                   "bilinear", outs=outs, fps=fps),
                       max(2, steps // 4), 1)
    npx = len(srcs) * oh * ow
    src_bytes = sum(s.numel() * 4 for s in srcs)
    byts = npx * 8 + src_bytes
    res = {"batch64_8192_bilinear": {"mpix_s": round(npx / ms / 1e3, 1), "ms": round(ms, 3),
                                     "gbs_alg": round(byts / ms / 1e6, 1),
                                     "hbm_frac": round(byts / ms / 1e6 / HBM_PEAK_GBS, 4)}}
    del outs, fps
    torch.cuda.empty_cache()
    # the same stack into per-frame windows (the boxes each frame can cover)
    from paper_2505_03932_amd import api
    import ctypes as C
    boxes = dfr.batch_boxes(srcs, c.src_wcs, c.tgt_wcs, c.out_shape, "bilinear")
    couts = [torch.empty((int(b[3]), int(b[2])), dtype=torch.float32, device="cuda") for b in boxes]
    cfps = [torch.empty_like(t) for t in couts]
    n = len(srcs)
    frames, keep = api._frames(srcs, c.src_wcs)
    tw, opts = api.CWcs(c.tgt_wcs), api._opts("f32")
    optrs = (C.c_void_p * n)(*[t.data_ptr() for t in couts])
    fptrs = (C.c_void_p * n)(*[t.data_ptr() for t in cfps])
    bptr = boxes.ctypes.data_as(C.c_void_p)
    stream = torch.cuda.current_stream().cuda_stream

    def cropped():
        st = api._lib.dfr_reproject_batch_cropped(n, frames, tw.s, oh, ow, 1, bptr, optrs, fptrs,
                                                  opts, stream)
        if st != 0:
            raise RuntimeError(f"dfr_reproject_batch_cropped failed: {st}")

    ms_x, _ = time_steps(cropped, max(2, steps // 2), 1)
    crop_px = int(sum(int(b[2]) * int(b[3]) for b in boxes))
    byts_x = 8 * crop_px + src_bytes
    res["batch64_8192_bilinear_cropped"] = {
        "ms": round(ms_x, 3), "window_px": crop_px, "window_mpix_s": round(crop_px / ms_x / 1e3, 1),
        "dense_equiv_mpix_s": round(npx / ms_x / 1e3, 1), "gbs_alg": round(byts_x / ms_x / 1e6, 1),
        "hbm_frac": round(byts_x / ms_x / 1e6 / HBM_PEAK_GBS, 4)}
    del couts, cfps
    torch.cuda.empty_cache()
    # the same stack coadded: sources read once, three target images written
    swf = torch.empty((oh, ow), dtype=torch.float32, device="cuda")
    sf = torch.empty_like(swf)
    ms_c, _ = time_steps(lambda: dfr.coadd_batch(srcs, c.src_wcs, c.tgt_wcs, c.out_shape,
                                                 "bilinear", sum_wf=swf, sum_f=sf),
                         max(2, steps // 2), 1)
    byts_c = src_bytes + 3 * oh * ow * 4
    res["coadd64_8192_bilinear"] = {"mpix_s": round(npx / ms_c / 1e3, 1), "ms": round(ms_c, 3),
                                    "gbs_alg": round(byts_c / ms_c / 1e6, 1),
                                    "hbm_frac": round(byts_c / ms_c / 1e6 / HBM_PEAK_GBS, 4)}
    del swf, sf, srcs
    torch.cuda.empty_cache()
    return res


def extra_pole(dfr, steps):
    """+89.5 deg, 0.2"/px, 8192^2, rotated 45 deg, SIP 4: FP32 vs FP64 path."""
    import torch
    from synth import configs
    c = configs.pole()
    src = torch.from_numpy(c.src).cuda()
    npx = c.out_shape[0] * c.out_shape[1]
    res = {}
    pos = {}
    for prec in ("f32", "f64"):
        _, _, p = dfr.reproject(src, c.src_wcs, c.tgt_wcs, c.out_shape, "bilinear",
                                precision=prec, debug_positions=True)
        pos[prec] = p
        fr = Frame(dfr, c.src, c.src_wcs, c.tgt_wcs, c.out_shape, "bilinear", precision=prec,
                   n_sets=1)
        ms, _ = time_steps(fr.step, max(2, steps // 4), 1)
        res[f"pole8192_bilinear_{prec}"] = {"mpix_s": round(npx / ms / 1e3, 1), "ms": round(ms, 3)}
        del fr
    ok = torch.isfinite(pos["f32"][..., 0]) & torch.isfinite(pos["f64"][..., 0])
    d = torch.linalg.norm(pos["f32"][ok] - pos["f64"][ok], dim=-1)
    res["pole8192_fp32_vs_fp64_pos_err_px"] = {"max": float(d.max()), "rms": float(
        torch.sqrt(torch.mean(d * d)))}
    del pos, src
    torch.cuda.empty_cache()
    return res


SWEEP_SIZES = [(256, 256), (512, 512), (1024, 1024), (2048, 2048), (4000, 6000)]


def sweep(dfr, steps, warmup):
    """The paper's scaling benchmark (section 4): image sizes 256^2 to
    4000x6000, each interpolation, with and without SIP; per point the whole
    forward step (cell models + tiles) on device-resident buffers."""
    import torch
    from synth import configs
    rows = []
    for shape in SWEEP_SIZES:
        for sip in (False, True):
            c = configs.sweep(shape, sip=sip)
            for interp in ("nearest", "bilinear", "bicubic"):
                fr = Frame(dfr, c.src, c.src_wcs, c.tgt_wcs, c.out_shape, interp)
                ms, _ = time_steps(fr.step, steps, warmup)
                npx = shape[0] * shape[1]
                rows.append({"h": shape[0], "w": shape[1], "sip": sip, "interp": interp,
                             "us": round(ms * 1e3, 2), "mpix_s": round(npx / ms / 1e3, 1),
                             "hbm_frac_12Bpx": round(12 * npx / ms / 1e6 / HBM_PEAK_GBS, 4)})
                log(json.dumps(rows[-1]))
                del fr
            torch.cuda.empty_cache()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--extras", default="forms,grad,pole,batch,sweep",
                    help="comma-separated extras to run: forms, grad, pole, batch, sweep")
    ap.add_argument("--sweep", action="store_true",
                    help="print the size x interpolation x SIP sweep instead of the headline")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build runs the reprojection on a single MI355X "
              "(no multi-GPU path); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2505_03932_amd as dfr
    from synth import configs

    if args.sweep:
        rows = sweep(dfr, args.steps, args.warmup)
        print(json.dumps({"metric": "output Mpix/s per size, interpolation and SIP",
                          "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps,
                          "warmup": args.warmup, "dtype": "f32", "data": "synthetic",
                          "config": {"workload": "size sweep 256^2 .. 4000x6000"},
                          "sweep": rows}), flush=True)
        return

    t0 = time.perf_counter()
    case = configs.sip3(interp=1)
    log(f"sip3 inputs generated in {time.perf_counter() - t0:.1f} s")
    oh, ow = case.out_shape
    npx = oh * ow
    frame = Frame(dfr, case.src, case.src_wcs, case.tgt_wcs, case.out_shape, "bilinear")
    ms, wall = time_steps(frame.step, args.steps, args.warmup)
    value = npx / ms / 1e3  # Mpix/s
    src_t = frame.sets[0][0]
    touched = touched_source_pixels(dfr, src_t, case.src_wcs, case.tgt_wcs, case.out_shape,
                                    "bilinear")
    alg_bytes = 8 * npx + 4 * touched
    # the dominant kernel alone: the same frame through a plan (models made
    # once), so each timed launch is exactly one reproject_tiles
    kms = time_tile_kernel(dfr, frame, case, args.steps, args.warmup)
    achieved = alg_bytes / kms / 1e6  # GB/s
    step_gbs = alg_bytes / ms / 1e6
    traffic = stored_profile("reproject_sip3_bilinear_pmc.md", "traffic")
    split = stored_profile("reproject_sip3_bilinear_kernel_trace.md", "split")
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": (traffic or {}).get("bytes_per_launch"),
            "alg_bytes_per_launch": alg_bytes, "kernel": "reproject_tiles",
            "kernel_ms": round(kms, 5),
            "timing": "HIP events on the launch stream around the timed launches of the tile "
                      "kernel alone (dfr_plan_execute)",
            "step_ms": round(ms, 5), "step_gbs": round(step_gbs, 1),
            "step_frac": round(step_gbs / HBM_PEAK_GBS, 4),
            "step_launches": "cell_models_kernel + reproject_tiles",
            "touched_src_px": touched}
    if split:
        # the same launches (the plan executes) in the committed kernel trace
        # of this measurement, and every launch of the tile kernel there
        roof["trace_tiles_us"] = split["tiles_us"]
        roof["trace_tiles_all_launches_us"] = split.get("tiles_all_us")
        roof["trace_models_us"] = split["models_us"]
        roof["frac_from_trace"] = round(alg_bytes / (split["tiles_us"] * 1e3) / HBM_PEAK_GBS, 4)
    roof["buffer_sets"] = len(frame.sets)
    del frame
    torch.cuda.empty_cache()
    roof.update(copy_bandwidth())
    if args.calibrate_copy:
        n = 128_000_000  # 512,000,000 bytes, twice the last-level cache
        a = torch.full((n,), 1.0, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        evict = torch.empty_like(a)
        for _ in range(3):
            evict.fill_(2.0)
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b, evict
        torch.cuda.empty_cache()

    forms = {}
    sweep_rows = None
    if not args.no_extras:
        chosen = set(args.extras.split(","))
        extras = {"forms": lambda: extra_forms(dfr, case, args.steps),
                  "grad": lambda: extra_grad(dfr, args.steps),
                  "pole": lambda: extra_pole(dfr, args.steps),
                  "batch": lambda: extra_batch(dfr, args.steps)}
        for fn in [f for k, f in extras.items() if k in chosen]:
            try:
                forms.update(fn())
            except Exception as e:  # an extra must not hide the headline
                forms.setdefault("errors", []).append(repr(e))
            log("extras so far:", json.dumps(forms))
        if "sweep" in chosen:
            try:
                sweep_rows = sweep(dfr, 5, 2)
            except Exception as e:
                forms.setdefault("errors", []).append(repr(e))
    cpu = None
    pos_err = None
    if not args.no_cpu_baseline:
        # the oracle leg: its timing on this host, and the position error of
        # every result against it
        cpu = cpu_baseline(case, "bilinear")
        try:
            errs = position_errors(dfr, case, forms)
            pos_err = errs.pop("sip3_bilinear")
            for k, e in errs.items():
                if k in forms:
                    forms[k]["pos_err_px"] = e
        except Exception as e:
            forms.setdefault("errors", []).append(repr(e))

    line = {
        "metric": "output Mpix/s (bilinear/bicubic, SIP-3) + % HBM roofline; fwd+bwd Mpix/s",
        "value": round(value, 1), "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded star field, SIP order 3 + fitted inverse order 4)",
        "config": {"workload": "6000x4000 SIP-3 frame -> 6000x4000 TAN target, bilinear, "
                               "out+footprint f32", "out_px": npx},
        "roofline": roof, "cpu_baseline": cpu, "pos_err_px": pos_err, "forms": forms,
    }
    if sweep_rows is not None:
        line["sweep"] = {"steps": 5, "warmup": 2, "note": "whole forward step per point",
                         "rows": sweep_rows}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
