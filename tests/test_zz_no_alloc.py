"""The allocation-free entry point (dfr_reproject_noalloc, through the C
ABI) against dfr_reproject: bit-identical outputs and footprints on two
calls in a row, the second with a smaller input, for every interpolation
and the FP32 forms; outputs beyond its fixed scratch are refused."""
import numpy as np
import pytest
import torch

from synth import configs

pytestmark = pytest.mark.gpu

INTERPS = {0: "nearest", 1: "bilinear", 2: "bicubic"}


@pytest.fixture(scope="module")
def dfr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_03932_amd as d
    return d


def _noalloc(dfr, src, sw, tw, shape, interp, precision="f32"):
    from paper_2505_03932_amd import _lib
    from paper_2505_03932_amd.api import CWcs, _opts
    oh, ow = shape
    out = torch.full((oh, ow), -7.0, dtype=torch.float32, device="cuda")
    fp = torch.full((oh, ow), -7.0, dtype=torch.float32, device="cuda")
    S, T = CWcs(sw), CWcs(tw)
    s = _lib.dfr_reproject_noalloc(src.data_ptr(), src.shape[0], src.shape[1], src.stride(0),
                                   S.s, T.s, oh, ow, interp, out.data_ptr(), fp.data_ptr(),
                                   _opts(precision), torch.cuda.current_stream().cuda_stream)
    assert s == 0, _lib.dfr_strerror(s)
    return out, fp


@pytest.mark.parametrize("precision", ["f32", "f32_anchor"])
@pytest.mark.parametrize("interp", [0, 1, 2])
def test_noalloc_equals_reproject_twice(dfr, interp, precision):
    big = configs.sip3(scale=0.25, interp=interp)    # 1500 x 1000
    small = configs.sip3(scale=0.06, interp=interp)  # 360 x 240
    results = []
    for c in (big, small):
        print(f"noalloc interp={interp} precision={precision} out={c.out_shape}", flush=True)
        src = torch.from_numpy(c.src).cuda()
        out, fp = _noalloc(dfr, src, c.src_wcs, c.tgt_wcs, c.out_shape, interp, precision)
        ref_out, ref_fp = dfr.reproject(src, c.src_wcs, c.tgt_wcs, c.out_shape, INTERPS[interp],
                                        precision=precision)
        torch.cuda.synchronize()
        assert torch.equal(out, ref_out) and torch.equal(fp, ref_fp)
        assert fp.max().item() > 0.5  # the frame is covered
        results.append(out)
    assert results[1].shape[0] < results[0].shape[0]


def test_noalloc_largest_grid_and_limit(dfr):
    """The largest table that fits (close to 8 MiB) and one cell more."""
    from paper_2505_03932_amd import _lib
    from paper_2505_03932_amd.api import CWcs, _opts
    c = configs.plain(size=256)
    src = torch.from_numpy(c.src).cuda()
    cells = _lib.DFR_NOALLOC_SCRATCH_BYTES // 112
    shape = (273 * 32, 274 * 32)  # 74,802 cells, 96 short of the limit
    assert 273 * 274 <= cells < 274 * 274
    print(f"noalloc full table out={shape}", flush=True)
    out, fp = _noalloc(dfr, src, c.src_wcs, c.tgt_wcs, shape, 1)
    ref_out, ref_fp = dfr.reproject(src, c.src_wcs, c.tgt_wcs, shape, "bilinear")
    torch.cuda.synchronize()
    assert torch.equal(out, ref_out) and torch.equal(fp, ref_fp)
    S, T = CWcs(c.src_wcs), CWcs(c.tgt_wcs)
    o = torch.zeros(1, device="cuda")
    s = _lib.dfr_reproject_noalloc(src.data_ptr(), 256, 256, 256, S.s, T.s, 274 * 32, 274 * 32,
                                   1, o.data_ptr(), None, _opts("f32"),
                                   torch.cuda.current_stream().cuda_stream)
    assert s == _lib.DFR_E_LIMIT
    # the FP64 form uses no scratch: no limit (a small grid here)
    out, fp = _noalloc(dfr, src, c.src_wcs, c.tgt_wcs, (64, 80), 1, precision="f64")
    ref_out, ref_fp = dfr.reproject(src, c.src_wcs, c.tgt_wcs, (64, 80), "bilinear",
                                    precision="f64")
    torch.cuda.synchronize()
    assert torch.equal(out, ref_out) and torch.equal(fp, ref_fp)
