#!/usr/bin/env python3
"""Benchmark of the reprojection hot path on one MI355X.

Headline: output Mpix/s of the bilinear forward reprojection of the
6000x4000 frame with SIP A/B order 3 and fitted inverse AP/BP order 4
(target 6000x4000 TAN, 40 px offset, rotated 0.3 deg), output and footprint
float32, inputs resident in HBM.  One step = one full forward pass over the
frame through the C ABI: host set-up, the per-cell position-model prepass and
the tile kernel (two launches on the caller's stream).

Beside it: the roofline of the dominant kernel, the tile kernel
(algorithmic bytes per launch over its average duration, HIP events on its
stream around launches of that kernel alone through a plan that holds the
frame's cell models, against 8 TB/s), the same for the whole step, the HBM
traffic the committed rocprofv3 PMC summary measured, the FP64 CPU oracle
timed on this host, and the other forms of the path (nearest and bicubic,
the FP64 and trigonometric forms, forward+backward on the 2048^2 alignment
case, the 64-frame batch and its coadd, the +89.5 deg precision case).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-extras]
                    [--extras forms,grad,pole,batch] [--no-cpu-baseline]
                    [--calibrate-copy] [--sweep]

--sweep prints, instead, one JSON line with the size sweep of the paper's
scaling benchmark: 256^2 .. 4000x6000 x {nearest, bilinear, bicubic} x
{with, without SIP}.

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

    def __init__(self, dfr, src_np, sw, tw, shape, interp, n_sets=2, precision="f32", fp=True):
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


def cpu_baseline(case, interp):
    """The FP64 oracle on this host's cores (at most 16 threads): whole
    passes over the headline frame until about 12 s of CPU work (wall time
    x threads) are done, at most 8 passes."""
    import oracle
    threads = max(1, min(os.cpu_count() or 1, 16))
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
    npx = passes * case.out_shape[0] * case.out_shape[1]
    return {"value": round(npx / dt / 1e6, 3), "unit": "Mpix/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{passes} whole passes over the 6000x4000 SIP frame ({npx} px, {interp}), "
                      f"FP64, {dt:.1f} s wall on {threads} threads"}


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

    ms_f, _ = time_steps(fwd, steps, 2)
    ms_fb, _ = time_steps(step, steps, 2)
    return {"grad2048_bicubic_fwd": {"mpix_s": round(n / ms_f / 1e3, 1), "ms": round(ms_f, 4)},
            "grad2048_bicubic_fwd_bwd": {"mpix_s": round(n / ms_fb / 1e3, 1),
                                         "ms": round(ms_fb, 4)}}


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
    ap.add_argument("--extras", default="forms,grad,pole,batch",
                    help="comma-separated extras to run: forms, grad, pole, batch")
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
        # the tile kernel alone, from the committed kernel trace of this command
        roof["trace_tiles_us"] = split["tiles_us"]
        roof["trace_models_us"] = split["models_us"]
        roof["tiles_frac_from_trace"] = round(alg_bytes / (split["tiles_us"] * 1e3) / HBM_PEAK_GBS, 4)
    del frame
    torch.cuda.empty_cache()
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
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(case, "bilinear")

    line = {
        "metric": "output Mpix/s (bilinear/bicubic, SIP-3) + % HBM roofline; fwd+bwd Mpix/s",
        "value": round(value, 1), "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded star field, SIP order 3 + fitted inverse order 4)",
        "config": {"workload": "6000x4000 SIP-3 frame -> 6000x4000 TAN target, bilinear, "
                               "out+footprint f32", "out_px": npx},
        "roofline": roof, "cpu_baseline": cpu, "forms": forms,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
