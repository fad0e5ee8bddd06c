"""Batch into per-frame windows: the boxes dfr_batch_boxes reports are
rigorous (every pixel of the full batch outside a frame's box is
uncovered), and the cropped outputs equal the same pixels of the full batch
bit for bit, for the reported boxes and for arbitrary, unaligned, empty and
partly unreachable ones."""
import numpy as np
import pytest
import torch

from synth import configs

pytestmark = pytest.mark.gpu

SHAPE = (700, 640)


@pytest.fixture(scope="module")
def dfr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_03932_amd as d
    return d


@pytest.fixture(scope="module")
def small_batch():
    return configs.batch(n_frames=7, target_side=700, side_range=(120, 520))


@pytest.mark.parametrize("interp", ["nearest", "bilinear", "bicubic"])
def test_boxes_rigorous_and_crops_identical(dfr, small_batch, interp):
    c = small_batch
    srcs = [torch.from_numpy(s).cuda() for s in c.src]
    outs, fps = dfr.reproject_batch(srcs, c.src_wcs, c.tgt_wcs, SHAPE, interp)
    boxes = dfr.batch_boxes(srcs, c.src_wcs, c.tgt_wcs, SHAPE, interp)
    print(f"cropped interp={interp} boxes={boxes.tolist()}", flush=True)
    for i, (x0, y0, w, h) in enumerate(boxes):
        assert 0 <= x0 and 0 <= y0 and x0 + w <= SHAPE[1] and y0 + h <= SHAPE[0]
        mask = torch.ones(SHAPE, dtype=torch.bool, device="cuda")
        mask[y0:y0 + h, x0:x0 + w] = False
        assert not torch.any(fps[i][mask] != 0), i  # nothing covered outside the box
    co, cf, cb = dfr.reproject_batch_cropped(srcs, c.src_wcs, c.tgt_wcs, SHAPE, interp)
    assert np.array_equal(cb, boxes)
    for i, (x0, y0, w, h) in enumerate(boxes):
        assert co[i].shape == (h, w)
        assert torch.equal(co[i], outs[i][y0:y0 + h, x0:x0 + w]), i
        assert torch.equal(cf[i], fps[i][y0:y0 + h, x0:x0 + w]), i
    # the stack's frames cover a fraction of the grid each
    assert sum(int(w) * int(h) for _, _, w, h in boxes) < len(srcs) * SHAPE[0] * SHAPE[1]


def test_arbitrary_boxes(dfr, small_batch):
    """Unaligned, empty, whole-grid and unreachable windows, tile shapes,
    NaN outside: always the same pixels as the full batch."""
    c = small_batch
    srcs = [torch.from_numpy(s).cuda() for s in c.src]
    boxes = np.array([[3, 5, 101, 77], [0, 0, 0, 0], [0, 0, 640, 700], [637, 698, 3, 2],
                      [17, 333, 1, 300], [200, 0, 55, 1], [0, 650, 640, 50]], dtype=np.int32)
    for tile, nan in ((0, False), (7, True), (3, False)):
        outs, fps = dfr.reproject_batch(srcs, c.src_wcs, c.tgt_wcs, SHAPE, "bilinear", tile=tile,
                                        nan_outside=nan)
        co, cf, _ = dfr.reproject_batch_cropped(srcs, c.src_wcs, c.tgt_wcs, SHAPE, "bilinear",
                                                boxes=boxes, tile=tile, nan_outside=nan)
        for i, (x0, y0, w, h) in enumerate(boxes):
            a, b = co[i], outs[i][y0:y0 + h, x0:x0 + w]
            assert torch.equal(torch.nan_to_num(a, nan=-5.0), torch.nan_to_num(b, nan=-5.0)), (tile, i)
            assert torch.equal(cf[i], fps[i][y0:y0 + h, x0:x0 + w]), (tile, i)


def test_unreachable_frame_box_is_empty(dfr, small_batch):
    c = small_batch
    far = c.src_wcs[1].copy(crval=(330.0, -2.0))
    empty = torch.zeros((0, 0), dtype=torch.float32, device="cuda")
    srcs = [torch.from_numpy(c.src[0]).cuda(), torch.from_numpy(c.src[1]).cuda(), empty]
    boxes = dfr.batch_boxes(srcs, [c.src_wcs[0], far, c.src_wcs[2]], c.tgt_wcs, SHAPE)
    assert boxes[0, 2] * boxes[0, 3] > 0
    assert boxes[1].tolist() == [0, 0, 0, 0] and boxes[2].tolist() == [0, 0, 0, 0]
    co, cf, _ = dfr.reproject_batch_cropped(srcs, [c.src_wcs[0], far, c.src_wcs[2]], c.tgt_wcs,
                                            SHAPE, boxes=boxes)
    assert co[1].numel() == 0 and co[2].numel() == 0


def test_target_sip_whole_grid_boxes(dfr, small_batch):
    """A target with SIP has no model table: every box is the whole grid,
    and crops still equal the full batch's pixels."""
    from synth.sipfit import draw_sip
    c = small_batch
    a, b = draw_sip(2, 350.0, np.random.default_rng(4))
    tw = c.tgt_wcs.copy(a=a, b=b)
    srcs = [torch.from_numpy(s).cuda() for s in c.src[:3]]
    boxes = dfr.batch_boxes(srcs, c.src_wcs[:3], tw, SHAPE)
    assert all(bx.tolist() == [0, 0, SHAPE[1], SHAPE[0]] for bx in boxes)
    sub = np.array([[40, 60, 300, 200], [0, 0, 64, 64], [600, 690, 40, 10]], dtype=np.int32)
    outs, fps = dfr.reproject_batch(srcs, c.src_wcs[:3], tw, SHAPE, "bicubic")
    co, cf, _ = dfr.reproject_batch_cropped(srcs, c.src_wcs[:3], tw, SHAPE, "bicubic", boxes=sub)
    for i, (x0, y0, w, h) in enumerate(sub):
        assert torch.equal(co[i], outs[i][y0:y0 + h, x0:x0 + w]), i
        assert torch.equal(cf[i], fps[i][y0:y0 + h, x0:x0 + w]), i
