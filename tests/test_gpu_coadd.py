"""Coadd (footprint-weighted stack) of many frames onto one target grid.

  * one frame: the sums are the single-image out * F and F, bit for bit;
  * many frames: the sums equal those of the per-frame batch outputs, summed
    in frame order, to FP32 accumulation rounding;
  * deterministic: every tile shape, and a stack split over calls with
    accumulate, give bit-identical sums;
  * parity with the FP64 oracle's stack on sampled rows (smooth frames, so
    the tolerance is set by the position error, not by image gradients);
  * empty stack, empty and out-of-reach frames, nan_outside.
"""
import numpy as np
import pytest
import torch

from synth import configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dfr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_03932_amd as d
    return d


SHAPE = (700, 640)


@pytest.fixture(scope="module")
def small_batch():
    # uneven frames with inverse SIP orders 3..5, partly off a 700x640 grid
    return configs.batch(n_frames=7, target_side=700, side_range=(120, 520))


def smooth(h, w, k):
    """A smooth frame: value gradients below 0.3 per pixel."""
    y, x = np.mgrid[0:h, 0:w].astype(np.float64)
    return (100.0 + 10.0 * k + 5.0 * np.sin(x / 37.0 + k) * np.cos(y / 23.0 - k)
            + 0.01 * x).astype(np.float32)


@pytest.mark.parametrize("interp", ["nearest", "bilinear", "bicubic"])
def test_single_frame_equals_reproject(dfr, small_batch, interp):
    c = small_batch
    src = torch.from_numpy(c.src[2]).cuda()
    out, fp = dfr.reproject(src, c.src_wcs[2], c.tgt_wcs, SHAPE, interp)
    img, swf, sf = dfr.coadd_batch([src], [c.src_wcs[2]], c.tgt_wcs, SHAPE, interp)
    cov = fp > 0
    print(f"coadd single interp={interp} covered={int(cov.sum())}", flush=True)
    assert torch.equal(sf, torch.where(cov, fp, torch.zeros_like(fp)))
    assert torch.equal(swf, torch.where(cov, out * fp, torch.zeros_like(fp)))
    ratio = torch.where(cov, swf / torch.where(cov, sf, torch.ones_like(sf)), torch.zeros_like(sf))
    assert torch.equal(img, ratio)


@pytest.mark.parametrize("interp", ["bilinear", "bicubic"])
def test_sums_equal_batch_outputs(dfr, small_batch, interp):
    c = small_batch
    srcs = [torch.from_numpy(s).cuda() for s in c.src]
    outs, fps = dfr.reproject_batch(srcs, c.src_wcs, c.tgt_wcs, SHAPE, interp)
    img, swf, sf = dfr.coadd_batch(srcs, c.src_wcs, c.tgt_wcs, SHAPE, interp)
    ref_wf = np.zeros(SHAPE)
    ref_f = np.zeros(SHAPE)
    mag = np.zeros(SHAPE)
    for o, f in zip(outs, fps):
        o = o.cpu().numpy().astype(np.float64)
        f = f.cpu().numpy().astype(np.float64)
        cov = f > 0
        ref_wf[cov] += o[cov] * f[cov]
        ref_f[cov] += f[cov]
        mag[cov] += np.abs(o[cov] * f[cov])
    n = len(srcs)
    swf = swf.cpu().numpy()
    sf = sf.cpu().numpy()
    # FP32 accumulation: one rounding per frame of at most half an ulp of the
    # running sum, plus the rounding of each product
    assert np.all(np.abs(swf - ref_wf) <= n * 2.0 ** -23 * mag + 1e-30)
    assert np.all(np.abs(sf - ref_f) <= n * 2.0 ** -23 * ref_f + 1e-30)
    cov = ref_f > 0
    assert cov.sum() > 0.3 * cov.size and (~cov).sum() > 0
    img = img.cpu().numpy()
    assert np.all(img[~cov] == 0)
    rel = np.abs(img[cov] - ref_wf[cov] / ref_f[cov]) / np.maximum(np.abs(ref_wf[cov] / ref_f[cov]), 1.0)
    print(f"coadd vs batch interp={interp} max rel {rel.max():.2e}", flush=True)
    assert rel.max() < 4 * n * 2.0 ** -23


def test_tiles_and_accumulate_bit_identical(dfr, small_batch):
    c = small_batch
    srcs = [torch.from_numpy(s).cuda() for s in c.src]
    ref = dfr.coadd_batch(srcs, c.src_wcs, c.tgt_wcs, SHAPE, "bilinear")
    for tile in (1, 2, 4, 5, 7, 10, 12):
        r = dfr.coadd_batch(srcs, c.src_wcs, c.tgt_wcs, SHAPE, "bilinear", tile=tile)
        for a, b in zip(ref, r):
            assert torch.equal(a, b), tile
    # the stack split over three calls, the sums carried with accumulate
    _, swf, sf = dfr.coadd_batch(srcs[:2], c.src_wcs[:2], c.tgt_wcs, SHAPE, "bilinear",
                                 coadd=False)
    dfr.coadd_batch(srcs[2:5], c.src_wcs[2:5], c.tgt_wcs, SHAPE, "bilinear", sum_wf=swf,
                    sum_f=sf, accumulate=True, coadd=False)
    img, swf, sf = dfr.coadd_batch(srcs[5:], c.src_wcs[5:], c.tgt_wcs, SHAPE, "bilinear",
                                   sum_wf=swf, sum_f=sf, accumulate=True)
    assert torch.equal(swf, ref[1]) and torch.equal(sf, ref[2]) and torch.equal(img, ref[0])
    # repeated calls give the same bits
    again = dfr.coadd_batch(srcs, c.src_wcs, c.tgt_wcs, SHAPE, "bilinear")
    assert all(torch.equal(a, b) for a, b in zip(ref, again))


@pytest.mark.parametrize("interp", ["bilinear", "bicubic"])
def test_parity_against_oracle(dfr, orc, small_batch, interp):
    c = small_batch
    imgs = [smooth(s.shape[0], s.shape[1], k) for k, s in enumerate(c.src)]
    srcs = [torch.from_numpy(s).cuda() for s in imgs]
    img, swf, sf = dfr.coadd_batch(srcs, c.src_wcs, c.tgt_wcs, SHAPE, interp)
    rows = np.arange(1, SHAPE[0], 29, dtype=np.int64)
    oimg, owf, of = orc.coadd(imgs, c.src_wcs, c.tgt_wcs, SHAPE, interp, rows=rows)
    img = img.cpu().numpy()[rows].astype(np.float64)
    swf = swf.cpu().numpy()[rows].astype(np.float64)
    sf = sf.cpu().numpy()[rows].astype(np.float64)
    n = len(imgs)
    # positions agree to ~2e-5 px, footprints move at most 1.5 per px (bicubic
    # edge), values at most 0.3 per px: per frame |dF| <= 5e-5, |d(out F)| <=
    # 5e-5 * 170 + FP32 rounding
    dF = np.abs(sf - of)
    dWF = np.abs(swf - owf)
    print(f"coadd vs oracle interp={interp} max |dF| {dF.max():.2e} max |d(wf)| {dWF.max():.2e}",
          flush=True)
    assert dF.max() <= n * 5e-5
    assert np.all(dWF <= n * (5e-5 * 170.0) + 1e-6 * np.abs(owf))
    # where every frame is fully in or out (sum F integral) the ratio is set
    # by value and rounding errors only; elsewhere a footprint error dF_i
    # moves weight between frames whose values differ by at most 70
    whole = (of >= 1) & (np.abs(of - np.round(of)) < 1e-9)
    part = (of > 0.05) & ~whole
    assert whole.sum() > 0.3 * whole.size and part.sum() > 0
    rel = np.abs(img[whole] - oimg[whole]) / np.abs(oimg[whole])
    d = np.abs(img[part] - oimg[part])
    tol = n * 5e-5 * 70.0 / of[part] + 1e-5 * np.abs(oimg[part])
    print(f"coadd vs oracle interp={interp} max rel (whole) {rel.max():.2e} "
          f"max |d| / tol (partial) {(d / tol).max():.2e}", flush=True)
    assert rel.max() < 1e-5
    assert np.all(d <= tol)
    # where the oracle covers nothing, at most a sliver of footprint appears
    assert np.all(sf[of == 0] <= n * 5e-5)


def test_empty_stack_empty_and_outside_frames(dfr, small_batch):
    c = small_batch
    shape = (300, 260)
    empty = torch.zeros((0, 0), dtype=torch.float32, device="cuda")
    far = c.src_wcs[1].copy(crval=(330.0, -2.0))
    s0 = torch.from_numpy(c.src[0]).cuda()
    img, swf, sf = dfr.coadd_batch([s0, empty, torch.from_numpy(c.src[1]).cuda()],
                                   [c.src_wcs[0], c.src_wcs[2], far], c.tgt_wcs, shape, "bicubic")
    r = dfr.coadd_batch([s0], [c.src_wcs[0]], c.tgt_wcs, shape, "bicubic")
    assert torch.equal(img, r[0]) and torch.equal(swf, r[1]) and torch.equal(sf, r[2])
    # nothing covers: NaN with nan_outside
    img, swf, sf = dfr.coadd_batch([empty], [c.src_wcs[0]], c.tgt_wcs, shape, "bilinear",
                                   nan_outside=True)
    assert torch.all(torch.isnan(img)) and not swf.any() and not sf.any()
    # an empty stack zeroes the sums, or keeps them with accumulate
    w = torch.full(shape, 6.0, device="cuda")
    f = torch.full(shape, 2.0, device="cuda")
    img, _, _ = dfr.coadd_batch([], [], c.tgt_wcs, shape, "bilinear", sum_wf=w, sum_f=f,
                                accumulate=True)
    assert torch.all(img == 3.0) and torch.all(w == 6.0) and torch.all(f == 2.0)
    img, _, _ = dfr.coadd_batch([], [], c.tgt_wcs, shape, "bilinear", sum_wf=w, sum_f=f)
    assert not img.any() and not w.any() and not f.any()
