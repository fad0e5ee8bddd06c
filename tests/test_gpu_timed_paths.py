"""Parity of the launch configurations the benchmark times, against the FP64
oracle (section 3.1: positions by the two stages of section 3.2, then
interpolation and footprint normalisation).

The timed calls run without debug positions, which is what enables the
all-model position branch, the unchecked interior gather and the skip of
tiles that cannot reach the source.  Each case here runs that configuration,
checks that a debug run (which reports the positions but takes the general
branches) gives the same bits over the whole output, and compares the timed
output with the oracle on sampled rows at the debug run's positions.
Also: the FP64 forms at full size, the 64-frame stack at full size, the
cropped batch windows and the header front end against the oracle.
"""
import numpy as np
import pytest
import torch

from synth import configs
from tests.parity import compare

pytestmark = pytest.mark.gpu

INTERPS = {0: "nearest", 1: "bilinear", 2: "bicubic"}


@pytest.fixture(scope="module")
def dfr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_03932_amd as d
    return d


def _rows(h, n, seed):
    rng = np.random.default_rng(seed)
    r = np.unique(np.concatenate([[0, 1, h // 2, h - 2, h - 1], rng.integers(0, h, n)]))
    return r.astype(np.int64)


def _timed_and_debug(dfr, c, interp, rows, **kw):
    """The timed call, the debug call, their bitwise equality; the timed
    output on `rows` with the debug positions."""
    src = torch.from_numpy(c.src).cuda()
    out, fp = dfr.reproject(src, c.src_wcs, c.tgt_wcs, c.out_shape, INTERPS[interp], **kw)
    dout, dfp, pos = dfr.reproject(src, c.src_wcs, c.tgt_wcs, c.out_shape, INTERPS[interp],
                                   debug_positions=True, **kw)
    torch.cuda.synchronize()
    assert torch.equal(torch.nan_to_num(out, nan=-3.0), torch.nan_to_num(dout, nan=-3.0))
    assert torch.equal(fp, dfp)
    r = torch.from_numpy(rows).cuda()
    return out[r].cpu().numpy(), fp[r].cpu().numpy(), pos[r].cpu().numpy()


@pytest.mark.parametrize("interp", [0, 1, 2])
def test_sip3_full_size_timed_configuration(dfr, orc, interp):
    """The 6000x4000 SIP-3 frame exactly as the benchmark runs it."""
    c = configs.sip3(interp=interp)
    rows = _rows(4000, 24, 17)
    print(f"timed sip3 interp={interp} rows={len(rows)}", flush=True)
    go, gf, gp = _timed_and_debug(dfr, c, interp, rows)
    oo, of, op = orc.reproject(c.src, c.src_wcs, c.tgt_wcs, c.out_shape, interp, rows=rows,
                               want_pos=True)
    rep = compare(orc, c.src, go, gf, gp, oo, of, op, interp)
    print(rep, flush=True)
    if interp == 0:
        assert rep["ties"] == 0


@pytest.mark.parametrize("interp", [0, 1])
def test_pole_full_size_timed_configuration(dfr, orc, interp):
    c = configs.pole(interp=interp)
    rows = _rows(8192, 12, 18)
    print(f"timed pole interp={interp} rows={len(rows)}", flush=True)
    go, gf, gp = _timed_and_debug(dfr, c, interp, rows)
    oo, of, op = orc.reproject(c.src, c.src_wcs, c.tgt_wcs, c.out_shape, interp, rows=rows,
                               want_pos=True)
    rep = compare(orc, c.src, go, gf, gp, oo, of, op, interp)
    print(rep, flush=True)


def test_anchor_chain_full_size_timed_configuration(dfr, orc):
    """The anchored FP32 chain (Horner per pixel), as the benchmark times it."""
    c = configs.sip3()
    rows = _rows(4000, 12, 19)
    go, gf, gp = _timed_and_debug(dfr, c, 1, rows, precision="f32_anchor")
    oo, of, op = orc.reproject(c.src, c.src_wcs, c.tgt_wcs, c.out_shape, 1, rows=rows,
                               want_pos=True)
    print(compare(orc, c.src, go, gf, gp, oo, of, op, 1), flush=True)


@pytest.mark.parametrize("precision", ["f64", "trig"])
def test_fp64_forms_full_size_pole(dfr, orc, precision):
    """Both FP64 forms on the 8192^2 frame at Dec +89.5: positions within
    1e-9 px of the oracle (different routes, both FP64)."""
    c = configs.pole()
    rows = _rows(8192, 10, 20)
    print(f"fp64 form {precision} at 8192^2 rows={len(rows)}", flush=True)
    go, gf, gp = _timed_and_debug(dfr, c, 1, rows, precision=precision)
    oo, of, op = orc.reproject(c.src, c.src_wcs, c.tgt_wcs, c.out_shape, 1, rows=rows,
                               want_pos=True)
    rep = compare(orc, c.src, go, gf, gp, oo, of, op, 1)
    print(rep, flush=True)
    assert rep["pos_max"] <= 1e-9


def _frame_positions(dfr, src, w, tw, shape, rows):
    _, _, pos = dfr.reproject(src, w, tw, shape, "bilinear", debug_positions=True)
    r = torch.from_numpy(rows).cuda()
    p = pos[r].cpu().numpy()
    del pos
    return p


def test_batch64_full_size(dfr, orc):
    """The 64-frame stack onto 8192^2 in the benchmark's launch: every 97th
    row of every frame, and every row of the cover box of 4 frames, against
    the oracle (positions from single-image debug runs, which the batch
    equals bit for bit)."""
    c = configs.batch()
    shape = c.out_shape
    srcs = [torch.from_numpy(s).cuda() for s in c.src]
    outs, fps = dfr.reproject_batch(srcs, c.src_wcs, c.tgt_wcs, shape, "bilinear")
    torch.cuda.synchronize()
    rows = np.arange(0, shape[0], 97, dtype=np.int64)
    r = torch.from_numpy(rows).cuda()
    for i in range(len(srcs)):
        pos = _frame_positions(dfr, srcs[i], c.src_wcs[i], c.tgt_wcs, shape, rows)
        oo, of, op = orc.reproject(c.src[i], c.src_wcs[i], c.tgt_wcs, shape, 1, rows=rows,
                                   want_pos=True)
        rep = compare(orc, c.src[i], outs[i][r].cpu().numpy(), fps[i][r].cpu().numpy(), pos,
                      oo, of, op, 1)
        if i % 8 == 0:
            print(f"batch64 frame {i}: {rep}", flush=True)
    boxes = dfr.batch_boxes(srcs, c.src_wcs, c.tgt_wcs, shape, "bilinear")
    for i in (0, 21, 42, 63):
        x0, y0, w, h = (int(v) for v in boxes[i])
        outside = torch.ones(shape, dtype=torch.bool, device="cuda")
        outside[y0:y0 + h, x0:x0 + w] = False
        assert not torch.any(fps[i][outside] != 0)
        print(f"batch64 frame {i}: all {h} rows of its box", flush=True)
        for y in range(y0, y0 + h, 1024):
            rows_i = np.arange(y, min(y + 1024, y0 + h), dtype=np.int64)
            ri = torch.from_numpy(rows_i).cuda()
            pos = _frame_positions(dfr, srcs[i], c.src_wcs[i], c.tgt_wcs, shape, rows_i)
            oo, of, op = orc.reproject(c.src[i], c.src_wcs[i], c.tgt_wcs, shape, 1, rows=rows_i,
                                       want_pos=True)
            compare(orc, c.src[i], outs[i][ri].cpu().numpy(), fps[i][ri].cpu().numpy(), pos, oo,
                    of, op, 1)
    del outs, fps
    torch.cuda.empty_cache()


@pytest.mark.parametrize("interp", [0, 1, 2])
def test_cropped_windows_vs_oracle(dfr, orc, interp):
    """Per-frame windows of the batch against the oracle on the target
    pixels each window holds."""
    c = configs.batch(n_frames=7, target_side=700, side_range=(120, 520))
    shape = (700, 640)
    srcs = [torch.from_numpy(s).cuda() for s in c.src]
    co, cf, boxes = dfr.reproject_batch_cropped(srcs, c.src_wcs, c.tgt_wcs, shape,
                                                INTERPS[interp])
    torch.cuda.synchronize()
    for i, (x0, y0, w, h) in enumerate(boxes):
        if w * h == 0:
            continue
        rows = np.arange(y0, y0 + h, dtype=np.int64)
        _, _, pos = dfr.reproject(srcs[i], c.src_wcs[i], c.tgt_wcs, shape, INTERPS[interp],
                                  debug_positions=True)
        pos = pos.cpu().numpy()[y0:y0 + h, x0:x0 + w]
        oo, of, op = orc.reproject(c.src[i], c.src_wcs[i], c.tgt_wcs, shape, interp, rows=rows,
                                   want_pos=True)
        rep = compare(orc, c.src[i], co[i].cpu().numpy(), cf[i].cpu().numpy(), pos,
                      oo[:, x0:x0 + w], of[:, x0:x0 + w], op[:, x0:x0 + w], interp)
        print(f"crop interp={interp} frame {i} box {(x0, y0, w, h)}: {rep}", flush=True)


def _header(w, pc_form):
    """FITS-style header mapping of a WCS; pc_form writes PCi_j x CDELTi."""
    h = {"CRPIX1": w.crpix[0], "CRPIX2": w.crpix[1], "CRVAL1": w.crval[0], "CRVAL2": w.crval[1],
         "CTYPE1": "RA---TAN-SIP", "CTYPE2": "DEC--TAN-SIP", "CUNIT1": "deg", "CUNIT2": "deg"}
    if pc_form:
        s = np.sqrt(abs(np.linalg.det(w.cd)))
        h.update({"CDELT1": -s, "CDELT2": s, "PC1_1": w.cd[0, 0] / -s, "PC1_2": w.cd[0, 1] / -s,
                  "PC2_1": w.cd[1, 0] / s, "PC2_2": w.cd[1, 1] / s})
    else:
        h.update({"CD1_1": w.cd[0, 0], "CD1_2": w.cd[0, 1], "CD2_1": w.cd[1, 0],
                  "CD2_2": w.cd[1, 1]})
    for name in ("A", "B", "AP", "BP"):
        cf = getattr(w, name.lower())
        if cf is None:
            continue
        h[f"{name}_ORDER"] = cf.shape[0] - 1
        for p in range(cf.shape[0]):
            for q in range(cf.shape[1]):
                if cf[p, q] != 0.0:
                    h[f"{name}_{p}_{q}"] = float(cf[p, q])
    return h


@pytest.mark.parametrize("pc_form", [False, True])
@pytest.mark.parametrize("interp", [0, 1, 2])
def test_front_end_vs_oracle(dfr, orc, interp, pc_form):
    """The paper's call with header mappings (CD, or PC x CDELT) against the
    oracle run on the WCS the headers were written from."""
    c = configs.sip3(scale=0.07, interp=interp)
    sh, th = _header(c.src_wcs, pc_form), _header(c.tgt_wcs, pc_form)
    out, fp = dfr.calculate_reprojection((c.src, sh), th, c.out_shape, INTERPS[interp],
                                         return_footprint=True)
    _, _, pos = dfr.reproject(torch.from_numpy(c.src).cuda(), c.src_wcs, c.tgt_wcs, c.out_shape,
                              INTERPS[interp], debug_positions=True)
    torch.cuda.synchronize()
    oo, of, op = orc.reproject(c.src, c.src_wcs, c.tgt_wcs, c.out_shape, interp, want_pos=True)
    rep = compare(orc, c.src, out.cpu().numpy(), fp.cpu().numpy(), pos.cpu().numpy(), oo, of, op,
                  interp)
    print(f"front end interp={interp} pc={pc_form}: {rep}", flush=True)
