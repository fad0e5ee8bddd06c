"""Plans: one geometry prepared once (FP64 set-up and per-cell models), many
images executed with only the per-pixel kernel.  Every execute must equal
dfr_reproject with the same geometry and options bit for bit."""
import numpy as np
import pytest
import torch

from synth import configs
from synth.sipfit import draw_sip

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dfr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_03932_amd as d
    return d


def _same(a, b):
    return torch.equal(torch.nan_to_num(a, nan=-7.0), torch.nan_to_num(b, nan=-7.0))


@pytest.mark.parametrize("interp", ["nearest", "bilinear", "bicubic"])
def test_plan_equals_reproject(dfr, interp):
    c = configs.sip3(scale=0.1)
    rng = np.random.default_rng(3)
    print(f"plan sip3 x0.1 interp={interp} shape={c.src.shape}", flush=True)
    with dfr.Plan(c.src.shape, c.src_wcs, c.tgt_wcs, c.out_shape, interp) as plan:
        for k in range(3):
            img = c.src if k == 0 else (c.src * rng.uniform(0.5, 2.0) + k).astype(np.float32)
            src = torch.from_numpy(img).cuda()
            o1, f1 = plan.execute(src)
            o2, f2 = dfr.reproject(src, c.src_wcs, c.tgt_wcs, c.out_shape, interp)
            assert torch.equal(o1, o2) and torch.equal(f1, f2), k


@pytest.mark.parametrize("shape", [(301, 207), (17, 3)])
def test_plan_ragged_and_options(dfr, shape):
    c = configs.plain()
    src = torch.from_numpy(c.src).cuda()
    for kw in ({"nan_outside": True}, {"tile": 3}, {"precision": "f32_anchor"},
               {"cubic_a": -0.75}):
        interp = "bicubic" if "cubic_a" in kw else "bilinear"
        with dfr.Plan(c.src.shape, c.src_wcs, c.tgt_wcs, shape, interp, **kw) as plan:
            o1, f1 = plan.execute(src)
            o3, _ = plan.execute(src, footprint=False)
        o2, f2 = dfr.reproject(src, c.src_wcs, c.tgt_wcs, shape, interp, **kw)
        assert _same(o1, o2) and _same(f1, f2) and _same(o3, o2), kw


def test_plan_target_sip_and_pitch(dfr):
    """A target with SIP has no model table (anchored chain); a source with
    a row pitch wider than its width."""
    c = configs.plain()
    a, b = draw_sip(2, 128.0, np.random.default_rng(1))
    tw = c.tgt_wcs.copy(a=a, b=b)
    big = torch.zeros((256, 300), dtype=torch.float32, device="cuda")
    big[:, :256] = torch.from_numpy(c.src).cuda()
    view = big[:, :256]
    with dfr.Plan((256, 256), c.src_wcs, tw, (256, 256), "bicubic") as plan:
        o1, f1 = plan.execute(view)
    o2, f2 = dfr.reproject(view, c.src_wcs, tw, (256, 256), "bicubic")
    assert torch.equal(o1, o2) and torch.equal(f1, f2)


def test_plan_errors(dfr):
    c = configs.plain()
    plan = dfr.Plan(c.src.shape, c.src_wcs, c.tgt_wcs, (64, 64))
    with pytest.raises(ValueError):
        plan.execute(torch.zeros((10, 10), device="cuda"))
    plan.close()
    with pytest.raises(ValueError):
        plan.execute(torch.from_numpy(c.src).cuda())
    with pytest.raises(dfr.DfrError):
        dfr.Plan(c.src.shape, c.src_wcs, c.tgt_wcs, (64, 64), precision="f64")


def _header(w):
    """FITS-style header mapping of a WCS (CD form, SIP terms by keyword)."""
    h = {"CRPIX1": w.crpix[0], "CRPIX2": w.crpix[1], "CRVAL1": w.crval[0], "CRVAL2": w.crval[1],
         "CD1_1": w.cd[0, 0], "CD1_2": w.cd[0, 1], "CD2_1": w.cd[1, 0], "CD2_2": w.cd[1, 1],
         "CTYPE1": "RA---TAN-SIP", "CTYPE2": "DEC--TAN-SIP", "CUNIT1": "deg", "CUNIT2": "deg"}
    for name in ("A", "B", "AP", "BP"):
        c = getattr(w, name.lower())
        if c is None:
            continue
        h[f"{name}_ORDER"] = c.shape[0] - 1
        for p in range(c.shape[0]):
            for q in range(c.shape[1]):
                if c[p, q] != 0.0:
                    h[f"{name}_{p}_{q}"] = float(c[p, q])
    return h


def test_calculate_reprojection_front_end(dfr):
    """The paper's call: (data, header) source, header target, shape_out
    defaulting to the source shape; equals reproject with the same WCS."""
    c = configs.sip3(scale=0.05)
    src = torch.from_numpy(c.src).cuda()
    sh, th = _header(c.src_wcs), _header(c.tgt_wcs)
    out, fp = dfr.calculate_reprojection((c.src, sh), th, c.out_shape, "bicubic",
                                         return_footprint=True)
    o2, f2 = dfr.reproject(src, c.src_wcs, c.tgt_wcs, c.out_shape, "bicubic")
    assert torch.equal(out, o2) and torch.equal(f2, fp)
    only = dfr.calculate_reprojection((c.src, sh), th, order="nearest-neighbor")
    o3, _ = dfr.reproject(src, c.src_wcs, c.tgt_wcs, c.src.shape, "nearest")
    assert only.shape == c.src.shape and torch.equal(only, o3)
