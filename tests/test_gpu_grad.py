"""Backward pass on the GPU: source-image adjoint and WCS-parameter gradient
against the FP64 oracle gradient (which the CPU tests pin to central finite
differences), the adjoint identity, the loss kernel and autograd."""
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


def grad_case(size):
    c = configs.grad(size=size)
    return c, c.extra["src_wcs_true"]


def interior_mask(orc, c, true_w):
    _, _, pos = orc.reproject(c.src, true_w, c.tgt_wcs, c.out_shape, 2, want_pos=True)
    h, w = c.src.shape
    return ((pos[..., 0] >= 3) & (pos[..., 0] <= w - 4) & (pos[..., 1] >= 3) &
            (pos[..., 1] <= h - 4))


# Per-entry tolerance of the WCS gradient, relative to the entry's own sum of
# term magnitudes sum_p |g_p * d out_p / d theta_i| (the oracle computes it
# beside the gradient).  Each per-pixel term is formed in FP32 (a few ulp,
# ~6e-7 of its magnitude) at a position within ~2e-6 px of the oracle's (an
# interpolant-derivative change of ~1e-6 relative for the star profiles), and
# the terms of a work-group are summed in FP32 over <= 2048 terms by a
# binary tree (<= 11 roundings, ~7e-7 of the magnitudes) before the FP64
# sums: together ~2e-6 of sum|terms| at worst, gated with a 5x margin.
WCS_TOL_ABS = 1e-5


def _compare_wcs_grad(gw, ref, ref_abs, tol=WCS_TOL_ABS, rel_tol=None):
    """Every entry: |gpu - oracle| <= tol * sum|terms|; entries that do not
    exist (p + q > order) must be exactly 0.  With rel_tol also
    |gpu - oracle| <= rel_tol * |oracle| per entry.  Returns the worst ratios."""
    gw = np.asarray(gw, np.float64)
    live = ref_abs > 0
    assert np.all(gw[~live] == 0.0), gw[~live]
    err = np.abs(gw - ref)
    r_abs = err[live] / ref_abs[live]
    r_rel = err[live] / np.abs(ref[live])
    print(f"wcs grad: max err/sum|terms| {r_abs.max():.3e}, max err/|ref| {r_rel.max():.3e}",
          flush=True)
    assert r_abs.max() <= tol, (np.argmax(r_abs), r_abs.max(), gw[live], ref[live])
    if rel_tol is not None:
        assert r_rel.max() <= rel_tol, (np.argmax(r_rel), r_rel.max(), gw[live], ref[live])
    return r_abs.max(), r_rel.max()


# Source adjoint: each source pixel sums <= 16 taps per output pixel (a few
# output pixels per source pixel at these scales) of g * w / F; with positions
# within ~2e-6 px of the oracle's a weight moves by <= max|W'| * 2e-6 ~ 4e-6,
# so a source entry moves by <= ~6.4e-5 * max|g|.
SRC_TOL = 1e-4


@pytest.mark.parametrize("interp", [1, 2])
def test_gradients_vs_oracle(dfr, orc, interp):
    """Unmasked g: pixels whose taps leave the source (0 < F < 1, the
    footprint-normalisation terms of the gradient) and uncovered pixels
    are included."""
    c, true_w = grad_case(160)
    print(f"grad interp={interp} size=160", flush=True)
    src = torch.from_numpy(c.src).cuda()
    rng = np.random.default_rng(3)
    g = rng.normal(0, 1, c.out_shape).astype(np.float32)
    _, of = orc.reproject(c.src, c.src_wcs, c.tgt_wcs, c.out_shape, interp)
    assert ((of > 1e-3) & (of < 1 - 1e-3)).sum() > 100  # the edge band is exercised
    gs, gw = dfr.reproject_backward(src, c.src_wcs, c.tgt_wcs, c.out_shape, INTERPS[interp],
                                    torch.from_numpy(g).cuda())
    torch.cuda.synchronize()
    ogs, ogw, _, oga = orc.grad(c.src, c.src_wcs, c.tgt_wcs, c.out_shape, interp,
                                g.astype(np.float64), want_abs=True)
    gs = gs.cpu().numpy().astype(np.float64)
    assert np.abs(gs - ogs).max() <= SRC_TOL * np.abs(g).max()
    _compare_wcs_grad(gw.cpu().numpy(), ogw, oga)


@pytest.mark.parametrize("interp", [1, 2])
def test_gradients_edge_band_only(dfr, orc, interp):
    """g nonzero only where the footprint is strictly between 0 and 1: the
    gradient there is carried by the derivative of the normalisation
    (out = S / F), so a mistake in those terms cannot hide behind the
    interior's."""
    c, _ = grad_case(192)
    src = torch.from_numpy(c.src).cuda()
    _, of = orc.reproject(c.src, c.src_wcs, c.tgt_wcs, c.out_shape, interp)
    band = (of > 1e-3) & (of < 1 - 1e-3)
    g = (np.random.default_rng(11).normal(0, 1, c.out_shape) * band).astype(np.float32)
    print(f"edge band interp={interp} pixels={int(band.sum())}", flush=True)
    gs, gw = dfr.reproject_backward(src, c.src_wcs, c.tgt_wcs, c.out_shape, INTERPS[interp],
                                    torch.from_numpy(g).cuda())
    torch.cuda.synchronize()
    ogs, ogw, _, oga = orc.grad(c.src, c.src_wcs, c.tgt_wcs, c.out_shape, interp,
                                g.astype(np.float64), want_abs=True)
    assert np.abs(gs.cpu().numpy() - ogs).max() <= SRC_TOL * np.abs(g).max()
    _compare_wcs_grad(gw.cpu().numpy(), ogw, oga)


def test_adjoint_identity_on_gpu(dfr):
    c, _ = grad_case(200)
    src = torch.from_numpy(c.src).cuda()
    g = torch.randn(c.out_shape, device="cuda", generator=torch.Generator("cuda").manual_seed(1))
    out, _ = dfr.reproject(src, c.src_wcs, c.tgt_wcs, c.out_shape, "bicubic")
    gs, _ = dfr.reproject_backward(src, c.src_wcs, c.tgt_wcs, c.out_shape, "bicubic", g,
                                   want_wcs=False)
    lhs = torch.sum(out.double() * g.double())
    rhs = torch.sum(src.double() * gs.double())
    scale = torch.sum(torch.abs(out.double() * g.double()))
    assert abs((lhs - rhs).item()) <= 1e-5 * scale.item()


def test_nearest_backward(dfr, orc):
    c, _ = grad_case(96)
    src = torch.from_numpy(c.src).cuda()
    g = np.random.default_rng(5).normal(0, 1, c.out_shape).astype(np.float32)
    gs, gw = dfr.reproject_backward(src, c.src_wcs, c.tgt_wcs, c.out_shape, "nearest",
                                    torch.from_numpy(g).cuda())
    ogs, ogw = orc.grad(c.src, c.src_wcs, c.tgt_wcs, c.out_shape, 0, g.astype(np.float64))
    assert np.abs(gs.cpu().numpy() - ogs).max() <= 1e-5 * np.abs(g).max()
    assert np.all(gw.cpu().numpy()[[0, 1, 4, 5, 6, 7]] == 0.0)


def test_full_size_alignment_gradient(dfr, orc):
    """The 2048^2 bicubic alignment case: loss against the reference
    reprojection under the true WCS, gradient at the perturbed WCS."""
    c, true_w = grad_case(2048)
    src = torch.from_numpy(c.src).cuda()
    mask = torch.from_numpy(interior_mask(orc, c, true_w).astype(np.float32)).cuda()
    ref, _ = dfr.reproject(src, true_w, c.tgt_wcs, c.out_shape, "bicubic")
    out, _ = dfr.reproject(src, c.src_wcs, c.tgt_wcs, c.out_shape, "bicubic")
    loss, g = dfr.sq_residual(out, ref, mask)
    gs, gw = dfr.reproject_backward(src, c.src_wcs, c.tgt_wcs, c.out_shape, "bicubic", g)
    torch.cuda.synchronize()
    gn = g.cpu().numpy().astype(np.float64)
    ogs, ogw, _, oga = orc.grad(c.src, c.src_wcs, c.tgt_wcs, c.out_shape, 2, gn, want_abs=True)
    print("loss", loss.item(), "grad_wcs", gw.cpu().numpy()[:8], "oracle", ogw[:8], flush=True)
    # every entry, CRVAL through the cubic AP/BP terms, within 1e-4 of itself
    _compare_wcs_grad(gw.cpu().numpy(), ogw, oga, rel_tol=1e-4)
    assert np.abs(gs.cpu().numpy() - ogs).max() <= SRC_TOL * np.abs(gn).max()


def test_full_size_gradient_unmasked(dfr, orc):
    """The 2048^2 bicubic case with g over the whole output (edges and
    uncovered pixels included), per entry against the oracle."""
    c, _ = grad_case(2048)
    src = torch.from_numpy(c.src).cuda()
    g = np.random.default_rng(12).normal(0, 1, c.out_shape).astype(np.float32)
    print("grad 2048 unmasked", flush=True)
    gs, gw = dfr.reproject_backward(src, c.src_wcs, c.tgt_wcs, c.out_shape, "bicubic",
                                    torch.from_numpy(g).cuda())
    torch.cuda.synchronize()
    ogs, ogw, _, oga = orc.grad(c.src, c.src_wcs, c.tgt_wcs, c.out_shape, 2,
                                g.astype(np.float64), want_abs=True)
    _compare_wcs_grad(gw.cpu().numpy(), ogw, oga)
    assert np.abs(gs.cpu().numpy() - ogs).max() <= SRC_TOL * np.abs(g).max()


def test_sq_residual_kernel(dfr):
    gen = torch.Generator("cuda").manual_seed(2)
    a = torch.randn(1000, 777, device="cuda", generator=gen)
    b = torch.randn(1000, 777, device="cuda", generator=gen)
    m = (torch.rand(1000, 777, device="cuda", generator=gen) > 0.3).float()
    loss, g = dfr.sq_residual(a, b, m)
    r = (a - b).double()
    ref = torch.sum(m.double() * r * r)
    assert abs(loss.item() - ref.item()) <= 1e-12 * abs(ref.item())
    assert torch.equal(g, 2.0 * m * (a - b))
    loss2, _ = dfr.sq_residual(a, b)
    assert abs(loss2.item() - torch.sum(r * r).item()) <= 1e-12 * torch.sum(r * r).item()


def test_autograd_function(dfr):
    c, true_w = grad_case(128)
    src = torch.from_numpy(c.src).cuda().requires_grad_(True)
    theta = torch.tensor(dfr.wcs_params(c.src_wcs), dtype=torch.float64,
                         requires_grad=True)
    ref, _ = dfr.reproject(src.detach(), true_w, c.tgt_wcs, c.out_shape, "bicubic")
    out = dfr.reproject_differentiable(src, theta, c.src_wcs, c.tgt_wcs, c.out_shape, "bicubic")
    loss = torch.sum((out - ref) ** 2)
    loss.backward()
    g = 2.0 * (out.detach() - ref)
    gs, gw = dfr.reproject_backward(src.detach(), c.src_wcs, c.tgt_wcs, c.out_shape, "bicubic", g)
    assert torch.allclose(src.grad, gs, rtol=0, atol=1e-5 * gs.abs().max().item())
    assert torch.allclose(theta.grad, gw.cpu(), rtol=1e-6, atol=0)


def test_gradient_descent_reduces_misalignment(dfr):
    """WCS alignment by gradient descent on image residuals: normalised
    gradient steps on CRPIX with backtracking recover a 0.5 px offset."""
    c, true_w = grad_case(256)
    src = torch.from_numpy(c.src).cuda()
    ref, _ = dfr.reproject(src, true_w, c.tgt_wcs, c.out_shape, "bicubic")

    def loss_and_grad(w):
        out, _ = dfr.reproject(src, w, c.tgt_wcs, c.out_shape, "bicubic")
        loss, g = dfr.sq_residual(out, ref)
        _, gw = dfr.reproject_backward(src, w, c.tgt_wcs, c.out_shape, "bicubic", g,
                                       want_src=False)
        return loss.item(), gw.cpu().numpy()[2:4]

    w = true_w.copy(crpix=(true_w.crpix[0] + 0.4, true_w.crpix[1] - 0.3))
    err0 = np.hypot(w.crpix[0] - true_w.crpix[0], w.crpix[1] - true_w.crpix[1])
    lr = 0.25
    cur, g = loss_and_grad(w)
    for _ in range(40):
        step = lr * g / (np.linalg.norm(g) + 1e-300)
        trial = w.copy(crpix=(w.crpix[0] - step[0], w.crpix[1] - step[1]))
        l_new, g_new = loss_and_grad(trial)
        if l_new < cur:
            w, cur, g = trial, l_new, g_new
        else:
            lr *= 0.5
    err1 = np.hypot(w.crpix[0] - true_w.crpix[0], w.crpix[1] - true_w.crpix[1])
    print("CRPIX error", err0, "->", err1, flush=True)
    assert err1 < 0.05 * err0


@pytest.mark.parametrize("interp", [1, 2])
def test_deterministic_source_gradient(dfr, orc, interp):
    """grad_src has the same bits on repeated runs and for every tile shape
    (exact integer sums), with or without the deterministic request, and
    matches the oracle to the source-adjoint tolerance."""
    c, _ = grad_case(300)
    src = torch.from_numpy(c.src).cuda()
    g = np.random.default_rng(21).normal(0, 1, c.out_shape).astype(np.float32)
    gt = torch.from_numpy(g).cuda()
    ref = None
    for tile in (0, 1, 2, 4, 5, 7, 8, 10, 11):
        for _ in range(2):
            gs, _ = dfr.reproject_backward(src, c.src_wcs, c.tgt_wcs, c.out_shape, INTERPS[interp],
                                           gt, want_wcs=False, tile=tile, deterministic=True)
            torch.cuda.synchronize()
            if ref is None:
                ref = gs.clone()
            else:
                assert torch.equal(gs, ref), tile
    ogs, _ = orc.grad(c.src, c.src_wcs, c.tgt_wcs, c.out_shape, interp, g.astype(np.float64),
                      want_src=True)
    d = np.abs(ref.cpu().numpy().astype(np.float64) - ogs).max()
    print(f"deterministic grad_src interp={interp}: max |gpu - oracle| / max|g| = "
          f"{d / np.abs(g).max():.3e}", flush=True)
    assert d <= SRC_TOL * np.abs(g).max()
    # the default request gives the same bits (the adjoint is always exact)
    gs0, _ = dfr.reproject_backward(src, c.src_wcs, c.tgt_wcs, c.out_shape, INTERPS[interp], gt,
                                    want_wcs=False)
    assert torch.equal(gs0, ref)


def test_deterministic_full_size_alignment(dfr, orc):
    """The 2048^2 bicubic alignment gradient in the deterministic mode: two
    runs give the same bits (source and WCS gradients) and both match the
    oracle."""
    c, true_w = grad_case(2048)
    src = torch.from_numpy(c.src).cuda()
    mask = torch.from_numpy(interior_mask(orc, c, true_w).astype(np.float32)).cuda()
    ref, _ = dfr.reproject(src, true_w, c.tgt_wcs, c.out_shape, "bicubic")
    out, _ = dfr.reproject(src, c.src_wcs, c.tgt_wcs, c.out_shape, "bicubic")
    _, g = dfr.sq_residual(out, ref, mask)
    a = dfr.reproject_backward(src, c.src_wcs, c.tgt_wcs, c.out_shape, "bicubic", g,
                               deterministic=True)
    b = dfr.reproject_backward(src, c.src_wcs, c.tgt_wcs, c.out_shape, "bicubic", g,
                               deterministic=True)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    gn = g.cpu().numpy().astype(np.float64)
    ogs, ogw, _, oga = orc.grad(c.src, c.src_wcs, c.tgt_wcs, c.out_shape, 2, gn, want_abs=True)
    _compare_wcs_grad(a[1].cpu().numpy(), ogw, oga, rel_tol=1e-4)
    assert np.abs(a[0].cpu().numpy() - ogs).max() <= SRC_TOL * np.abs(gn).max()


def test_backward_streams_and_gradient_scales(dfr):
    """Backward calls on two streams in turn, with gradients of very
    different magnitudes in turn (so max|g|, kept per stream in two
    alternating control words, changes from call to call), give the bits a
    call on the default stream gives for the same gradient."""
    c, _ = grad_case(300)
    src = torch.from_numpy(c.src).cuda()
    rng = np.random.default_rng(22)
    grads = [torch.from_numpy((rng.normal(0, 1, c.out_shape) * sc).astype(np.float32)).cuda()
             for sc in (1.0, 1e-6, 3e4)]
    want = []
    for g in grads:
        gs, gw = dfr.reproject_backward(src, c.src_wcs, c.tgt_wcs, c.out_shape, "bicubic", g)
        torch.cuda.synchronize()
        want.append((gs.clone(), gw.clone()))
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for rep in range(3):
        for k, g in enumerate(grads):
            st = streams[(rep + k) % 2]
            st.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(st):
                gs, gw = dfr.reproject_backward(src, c.src_wcs, c.tgt_wcs, c.out_shape, "bicubic",
                                                g)
            st.synchronize()
            assert torch.equal(gs, want[k][0]), (rep, k)
            assert torch.equal(gw, want[k][1]), (rep, k)
    # an argument error leaves the next call's result unchanged
    with pytest.raises(Exception):
        dfr.reproject_backward(src, c.src_wcs, c.tgt_wcs, (-1, 5), "bicubic", grads[0])
    gs, gw = dfr.reproject_backward(src, c.src_wcs, c.tgt_wcs, c.out_shape, "bicubic", grads[2])
    torch.cuda.synchronize()
    assert torch.equal(gs, want[2][0]) and torch.equal(gw, want[2][1])
