"""Comparison helpers for the GPU-vs-oracle parity tests.

Criteria (FP32 path against the FP64 oracle):
  position   |pos_gpu - pos_oracle| <= 1e-3 px (both from the same target
             pixel; the GPU reports the exact position it interpolated at);
  value      |out_gpu - O(pos_gpu)| <= 1e-5 * max(|O|, C, 1), where O is the
             oracle's FP64 interpolation at the GPU's own position and
             C = sum|w v| / F the magnitude of the terms being combined (the
             scale a relative FP32 error of a weighted sum refers to);
  footprint  |F_gpu - F_oracle(pos_gpu)| <= 1e-6 (FP32 sums of <= 4 weights per axis
             and their product: a few ulp of 1; measured <= 3.5e-7);
  coverage   covered on one side and not the other only where the oracle's
             footprint at the GPU position is below 1e-6 (a decision of F > 0
             within rounding of zero);
  nearest    bit-exact values and footprint, except pixels whose oracle
             position lies within 1e-9 px of a rounding tie (counted).
"""
from __future__ import annotations

import numpy as np

POS_TOL = 1e-3
REL_TOL = 1e-5
FP_TOL = 1e-6
F_EDGE = 1e-6


def compare(orc, src, gpu_out, gpu_fp, gpu_pos, ora_out, ora_fp, ora_pos, interp, cubic_a=-0.5,
            pos_tol=POS_TOL):
    """Check one set of rows; returns a dict of measured errors."""
    gpu_out = np.asarray(gpu_out, np.float64)
    gpu_fp = np.asarray(gpu_fp, np.float64)
    gv = np.isfinite(gpu_pos[..., 0])
    ov = np.isfinite(ora_pos[..., 0])
    rep = {}
    both = gv & ov
    # validity may only differ where the position is far outside the source
    h, w = src.shape
    far = lambda p: (np.abs(p[..., 0]) > 4 * max(h, w)) | (np.abs(p[..., 1]) > 4 * max(h, w))
    mism = gv != ov
    assert np.all(~mism | far(np.where(np.isfinite(ora_pos), ora_pos, 1e30))), "validity differs"
    d = np.hypot(*(gpu_pos[both] - ora_pos[both]).T) if both.any() else np.zeros(1)
    rep["pos_max"] = float(d.max()) if d.size else 0.0
    rep["pos_rms"] = float(np.sqrt(np.mean(d ** 2))) if d.size else 0.0
    assert rep["pos_max"] <= pos_tol, f"position error {rep['pos_max']:.3e} px"
    flat_pos = gpu_pos.reshape(-1, 2)
    sel = np.flatnonzero(gv.ravel())
    O = np.zeros(gpu_out.size)
    F = np.zeros(gpu_out.size)
    cond = np.zeros(gpu_out.size)
    if sel.size:
        o, f, c = orc.interp_at(src, flat_pos[sel], interp, cubic_a)
        O[sel], F[sel], cond[sel] = o, f, c
    go = gpu_out.ravel()
    gf = gpu_fp.ravel()
    if interp == 0:
        # ties: oracle position within 1e-9 of a half-integer on either axis
        op = ora_pos.reshape(-1, 2)
        with np.errstate(invalid="ignore"):
            fr = np.abs(np.abs(op - np.floor(op)) - 0.5)
        tie = np.any(fr < 1e-9, axis=1) & np.isfinite(op[:, 0])
        rep["ties"] = int(tie.sum())
        ok = ~tie
        assert np.array_equal(gf[ok], ora_fp.ravel()[ok]), "nearest footprint differs"
        assert np.array_equal(go[ok], ora_out.ravel()[ok]), "nearest value differs"
        return rep
    cov_g = gf > 0
    cov_o = F > 0
    edge = np.abs(F) < F_EDGE
    assert np.all((cov_g == cov_o) | edge), "coverage differs away from F ~ 0"
    m = cov_g & cov_o & ~edge
    scale = np.maximum(np.maximum(np.abs(O[m]), cond[m]), 1.0)
    rel = np.abs(go[m] - O[m]) / scale
    rep["val_rel_max"] = float(rel.max()) if rel.size else 0.0
    assert rep["val_rel_max"] <= REL_TOL, f"value error {rep['val_rel_max']:.3e}"
    fe = np.abs(gf[m] - F[m])
    rep["fp_max"] = float(fe.max()) if fe.size else 0.0
    assert rep["fp_max"] <= FP_TOL, f"footprint error {rep['fp_max']:.3e}"
    # uncovered pixels are exactly zero
    unc = ~cov_g
    assert np.all(go[unc] == 0.0) and np.all(gf[unc] == 0.0)
    # end-to-end against the oracle's own output (reported, not gated)
    oo = ora_out.ravel()
    ofp = ora_fp.ravel()
    mm = m & (ofp > F_EDGE)
    if mm.any():
        rep["e2e_max_abs"] = float(np.max(np.abs(go[mm] - oo[mm])))
    return rep
