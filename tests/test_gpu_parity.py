"""GPU forward parity: the HIP path (through the C ABI) against the FP64 oracle.

Sizes span many tiles with ragged tails; full-size workloads are checked on
sampled rows the oracle computes one by one.
"""
import numpy as np
import pytest
import torch

from synth import WcsParams, configs, draw_sip, fit_inverse_sip
from tests.parity import compare

pytestmark = pytest.mark.gpu

INTERPS = {0: "nearest", 1: "bilinear", 2: "bicubic"}


@pytest.fixture(scope="module")
def dfr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_03932_amd as d
    return d


def run_gpu(dfr, src, sw, tw, shape, interp, **kw):
    out, fp, pos = dfr.reproject(torch.from_numpy(src).cuda(), sw, tw, shape, INTERPS[interp],
                                 debug_positions=True, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy(), fp.cpu().numpy(), pos.cpu().numpy()


def check_case(dfr, orc, src, sw, tw, shape, interp, rows=None, **kw):
    print(f"case shape={shape} interp={interp} src={src.shape} rows={'all' if rows is None else len(rows)}",
          flush=True)
    go, gf, gp = run_gpu(dfr, src, sw, tw, shape, interp, **kw)
    if rows is not None:
        go, gf, gp = go[rows], gf[rows], gp[rows]
    oo, of, op = orc.reproject(src, sw, tw, shape, interp, rows=rows, want_pos=True,
                               cubic_a=kw.get("cubic_a", -0.5))
    rep = compare(orc, src, go, gf, gp, oo, of, op, interp, kw.get("cubic_a", -0.5))
    print(rep, flush=True)
    return rep, (go, gf, gp)


def test_plain_bilinear(dfr, orc):
    c = configs.plain()
    check_case(dfr, orc, c.src, c.src_wcs, c.tgt_wcs, c.out_shape, c.interp)


@pytest.mark.parametrize("interp", [0, 1, 2])
def test_sip3_reduced(dfr, orc, interp):
    c = configs.sip3(scale=0.1, interp=interp)
    check_case(dfr, orc, c.src, c.src_wcs, c.tgt_wcs, c.out_shape, interp)


@pytest.mark.parametrize("interp", [1, 2])
def test_bicubic_a(dfr, orc, interp):
    c = configs.plain(size=200, interp=interp)
    check_case(dfr, orc, c.src, c.src_wcs, c.tgt_wcs, c.out_shape, interp, cubic_a=-0.75)


@pytest.mark.parametrize("interp", [0, 1, 2])
def test_target_side_sip(dfr, orc, interp):
    """SIP A/B on the target (no workload has it): a distorted target grid."""
    rng = np.random.default_rng(21)
    c = configs.plain(size=300)
    a, b = draw_sip(3, 150.0, rng)
    tw = c.tgt_wcs.copy(a=a * 50, b=b * 50)
    check_case(dfr, orc, c.src, c.src_wcs, tw, (290, 310), interp)


def test_demo_analogue(dfr, orc):
    c = configs.demo()
    check_case(dfr, orc, c.src, c.src_wcs, c.tgt_wcs, c.out_shape, c.interp)


@pytest.mark.parametrize("interp", [0, 1, 2])
def test_pole_reduced(dfr, orc, interp):
    c = configs.pole(size=640, interp=interp)
    check_case(dfr, orc, c.src, c.src_wcs, c.tgt_wcs, c.out_shape, interp)


@pytest.mark.parametrize("shape", [(301, 207), (1, 1), (17, 3), (5, 1023)])
def test_ragged_outputs(dfr, orc, shape):
    c = configs.sip3(scale=0.05)
    check_case(dfr, orc, c.src, c.src_wcs, c.tgt_wcs, shape, 1)


def test_ragged_source_pitch(dfr, orc):
    """A source that is a column slice of a wider buffer (row pitch > width)."""
    c = configs.plain(size=128)
    wide = np.zeros((128, 160), np.float32)
    wide[:, :128] = c.src
    t = torch.from_numpy(wide).cuda()[:, :128]
    assert t.stride(0) == 160
    out, fp, pos = dfr.reproject(t, c.src_wcs, c.tgt_wcs, (128, 128), "bicubic",
                                 debug_positions=True)
    oo, of, op = orc.reproject(c.src, c.src_wcs, c.tgt_wcs, (128, 128), 2, want_pos=True)
    compare(orc, c.src, out.cpu().numpy(), fp.cpu().numpy(), pos.cpu().numpy(), oo, of, op, 2)


def test_empty_and_uncovered(dfr, orc):
    c = configs.plain(size=64)
    src = torch.from_numpy(c.src).cuda()
    out, fp = dfr.reproject(src, c.src_wcs, c.tgt_wcs, (0, 10))
    assert out.shape == (0, 10)
    empty = torch.zeros((0, 0), dtype=torch.float32, device="cuda")
    out, fp = dfr.reproject(empty, c.src_wcs, c.tgt_wcs, (40, 44))
    assert torch.all(out == 0) and torch.all(fp == 0)
    far = c.src_wcs.copy(crval=(330.0, -2.0))  # tangent point > 90 deg away
    out, fp = dfr.reproject(src, far, c.tgt_wcs, (64, 64), nan_outside=True)
    assert torch.all(torch.isnan(out)) and torch.all(fp == 0)
    shifted = c.src_wcs.copy(crpix=(c.src_wcs.crpix[0] + 5000.0, c.src_wcs.crpix[1]))
    out, fp = dfr.reproject(src, shifted, c.tgt_wcs, (64, 64))
    assert torch.all(out == 0) and torch.all(fp == 0)


def test_package_imported_before_torch():
    """The library must run on torch's HIP runtime whatever the import order
    (libdfr and torch both need libamdhip64.so.7)."""
    import subprocess
    import sys
    code = ("import paper_2505_03932_amd as d\n"
            "import torch\n"
            "from synth import configs\n"
            "c = configs.plain(size=96)\n"
            "out, fp = d.reproject(torch.from_numpy(c.src).cuda(), c.src_wcs, c.tgt_wcs, c.out_shape)\n"
            "torch.cuda.synchronize()\n"
            "print('ok', float(fp.sum()))\n")
    root = __file__.rsplit("/tests/", 1)[0]
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                       timeout=180)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stderr[-2000:]


def test_identity_nearest_bit_exact(dfr):
    c = configs.plain(size=130)
    out, fp = dfr.reproject(torch.from_numpy(c.src).cuda(), c.src_wcs, c.src_wcs, c.src.shape,
                            "nearest")
    assert torch.equal(out.cpu(), torch.from_numpy(c.src)) and torch.all(fp == 1)


def test_tile_shapes_bit_identical(dfr):
    """The fixed anchor grid makes results independent of the tile shape."""
    c = configs.sip3(scale=0.08)
    src = torch.from_numpy(c.src).cuda()
    for interp in ("nearest", "bilinear", "bicubic"):
        ref = None
        for t in range(1, 13):
            out, fp = dfr.reproject(src, c.src_wcs, c.tgt_wcs, (333, 470), interp, tile=t)
            if ref is None:
                ref = (out.clone(), fp.clone())
            else:
                assert torch.equal(out, ref[0]) and torch.equal(fp, ref[1]), (interp, t)


@pytest.mark.parametrize("interp", [0, 1, 2])
def test_anchor_chain_form(dfr, orc, interp):
    """The FP32 chain evaluated per pixel from FP64 anchors (no cell models)."""
    c = configs.sip3(scale=0.1, interp=interp)
    check_case(dfr, orc, c.src, c.src_wcs, c.tgt_wcs, c.out_shape, interp, precision="f32_anchor")


def test_models_and_anchor_chain_agree(dfr):
    """Positions of the two FP32 forms differ by their FP32 rounding only."""
    c = configs.sip3(scale=0.15)
    src = torch.from_numpy(c.src).cuda()
    _, _, pm = dfr.reproject(src, c.src_wcs, c.tgt_wcs, c.out_shape, "bilinear",
                             debug_positions=True)
    _, _, pa = dfr.reproject(src, c.src_wcs, c.tgt_wcs, c.out_shape, "bilinear",
                             debug_positions=True, precision="f32_anchor")
    d = (pm - pa).abs()
    ok = torch.isfinite(d)
    assert ok.float().mean() > 0.95
    assert d[ok].max().item() < 2e-5


@pytest.mark.parametrize("interp", [0, 1, 2])
def test_mixed_model_and_anchor_cells(dfr, orc, interp):
    """A map whose central cells have certified models and whose outer cells
    do not: tiles mix both kinds of cell."""
    c = configs.strong_sip(interp=interp)
    check_case(dfr, orc, c.src, c.src_wcs, c.tgt_wcs, c.out_shape, interp)
    src = torch.from_numpy(c.src).cuda()
    ref = None
    for t in range(1, 13):
        out, fp = dfr.reproject(src, c.src_wcs, c.tgt_wcs, c.out_shape, INTERPS[interp], tile=t)
        if ref is None:
            ref = (out.clone(), fp.clone())
        else:
            assert torch.equal(out, ref[0]) and torch.equal(fp, ref[1]), t


@pytest.mark.parametrize("precision", ["f64", "trig"])
@pytest.mark.parametrize("interp", [0, 1, 2])
def test_fp64_forms(dfr, orc, precision, interp):
    """Both FP64 paths: positions within 1e-9 px of the oracle (different
    arithmetic routes, both FP64)."""
    c = configs.pole(size=384, interp=interp)
    rep, _ = check_case(dfr, orc, c.src, c.src_wcs, c.tgt_wcs, c.out_shape, interp,
                        precision=precision)
    assert rep["pos_max"] <= 1e-9


def _rows(h, n, seed):
    rng = np.random.default_rng(seed)
    r = np.unique(np.concatenate([[0, 1, h // 2, h - 2, h - 1], rng.integers(0, h, n)]))
    return r.astype(np.int64)


@pytest.mark.parametrize("interp", [0, 1, 2])
def test_sip3_full_size_sampled_rows(dfr, orc, interp):
    """The 6000x4000 SIP frame at full size, in the launch configuration the
    benchmark times, checked on sampled rows."""
    c = configs.sip3(interp=interp)
    check_case(dfr, orc, c.src, c.src_wcs, c.tgt_wcs, c.out_shape, interp, rows=_rows(4000, 20, 7))


def test_pole_full_size_sampled_rows(dfr, orc):
    c = configs.pole()
    rep, _ = check_case(dfr, orc, c.src, c.src_wcs, c.tgt_wcs, c.out_shape, 1,
                        rows=_rows(8192, 12, 8))
    print("pole FP32 position error max/rms px:", rep["pos_max"], rep["pos_rms"])
