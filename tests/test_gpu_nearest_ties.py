"""Nearest-neighbour rounding decisions next to ties (section 3.3: the value
of the closest source pixel; ties to even), against the FP64 oracle.

Source and target share CRVAL and CD and have no SIP, so the map is a pure
translation by the CRPIX difference; a difference of half a pixel plus a
small delta puts every output pixel's source position delta away from a
rounding tie on each axis.  The FP32 positions cannot tell such pixels
apart, so every pixel takes the kernels' FP64 decision (from the cell's
model where its certified bound allows, else from the full FP64 chain),
and the result must equal the oracle's bit for bit on every pixel.
"""
import numpy as np
import pytest
import torch

from synth import WcsParams
from synth.starfield import star_field
from tests.parity import compare

pytestmark = pytest.mark.gpu

SRC_SHAPE = (256, 256)
OUT_SHAPE = (300, 260)
# (delta_x, delta_y): 3e-6 and 7e-7 px lie beyond the cell models' bound
# for this map, 1e-8 and 2e-8 px within it (those pixels take the chain)
DELTAS = [(3e-6, -7e-7), (1e-8, 2e-6), (-2e-8, -1e-8)]


@pytest.fixture(scope="module")
def dfr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_03932_amd as d
    return d


def _case(delta, seed):
    h, w = SRC_SHAPE
    src = star_field(h, w, 100.0, 5.0, 40, seed, rng=np.random.default_rng(seed))
    sw = WcsParams.tan((150.0, 2.0), 2.85, 0.0, SRC_SHAPE)
    # x_src = x_out + crpix_src - crpix_out: fractional part 0.5 + delta
    tw = WcsParams.tan((150.0, 2.0), 2.85, 0.0, OUT_SHAPE,
                       crpix_offset=(0.5 - delta[0], 0.5 - delta[1]))
    return src, sw, tw


@pytest.mark.parametrize("delta", DELTAS)
def test_near_tie_translation_single(dfr, orc, delta):
    src, sw, tw = _case(delta, 31)
    print(f"near-tie translation delta={delta}", flush=True)
    s = torch.from_numpy(src).cuda()
    out, fp = dfr.reproject(s, sw, tw, OUT_SHAPE, "nearest")
    dout, dfp, pos = dfr.reproject(s, sw, tw, OUT_SHAPE, "nearest", debug_positions=True)
    torch.cuda.synchronize()
    assert torch.equal(out, dout) and torch.equal(fp, dfp)
    oo, of, op = orc.reproject(src, sw, tw, OUT_SHAPE, 0, want_pos=True)
    # every oracle position is delta from a tie on both axes
    fr = np.abs(op - np.floor(op) - 0.5)
    ok = np.isfinite(op[..., 0])
    assert np.all(np.abs(fr[ok] - np.abs(np.array(delta))) < 1e-10)
    rep = compare(orc, src, out.cpu().numpy(), fp.cpu().numpy(), pos.cpu().numpy(), oo, of, op, 0)
    print(rep, flush=True)
    assert rep["ties"] == 0
    assert (fp.cpu().numpy() > 0).sum() > 0.5 * src.size


def test_near_tie_translation_batch(dfr, orc):
    """The persistent batch kernel takes the same decisions, frame by frame."""
    cases = [_case(d, 40 + i) for i, d in enumerate(DELTAS)]
    srcs = [torch.from_numpy(c[0]).cuda() for c in cases]
    outs, fps = dfr.reproject_batch(srcs, [c[1] for c in cases], cases[0][2], OUT_SHAPE, "nearest")
    torch.cuda.synchronize()
    for i, (src, sw, _) in enumerate(cases):
        # every frame is reprojected onto the first frame's target grid
        tw = cases[0][2]
        oo, of, op = orc.reproject(src, sw, tw, OUT_SHAPE, 0, want_pos=True)
        _, _, pos = dfr.reproject(srcs[i], sw, tw, OUT_SHAPE, "nearest", debug_positions=True)
        rep = compare(orc, src, outs[i].cpu().numpy(), fps[i].cpu().numpy(), pos.cpu().numpy(),
                      oo, of, op, 0)
        print(f"batch frame {i}: {rep}", flush=True)
        assert rep["ties"] == 0
