"""The pins are strong enough to catch plausible mistakes in the oracle.

Each case plants one mistake (a flipped sign, a dropped term, a transposed
operand, a swapped weight, a sequential instead of simultaneous update) in a
copy of ``oracle/oracle.c``, builds it with gcc into a temporary library,
routes the oracle wrapper to it and runs the pin battery of
``test_oracle_pins.py``: at least one pin must fail for every mutant.  All of
this runs on the CPU; the real oracle is untouched.
"""
import os
import shutil
import tempfile

import pytest

import oracle
from oracle import build as obuild

import tests.test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "sip_sign": ("  u += du;\n  v += dv;\n  /* CD matrix", "  u -= du;\n  v -= dv;\n  /* CD matrix"),
    "crpix_shift": ("double u = x - (w->crpix[0] - 1.0);", "double u = x - w->crpix[0];"),
    "cd_transposed": ("double up = w->cd[0] * u + w->cd[1] * v;",
                      "double up = w->cd[0] * u + w->cd[2] * v;"),
    "phi_sign": ("double phi = atan2(-up, vp);", "double phi = atan2(up, vp);"),
    "rotation_term": ("double Y = st * cos(d0) - ct * sin(d0) * cp;",
                      "double Y = st * cos(d0) + ct * sin(d0) * cp;"),
    "inverse_cd": ("*u = (w->cd[3] * up - w->cd[1] * vp) / det;",
                   "*u = (w->cd[3] * up - w->cd[2] * vp) / det;"),
    "inverse_sequential_sip": (
        "  double du = orc_sip_eval(w->ap, w->ap_order, u, v);\n"
        "  double dv = orc_sip_eval(w->bp, w->bp_order, u, v);\n  u += du;\n  v += dv;",
        "  double du = orc_sip_eval(w->ap, w->ap_order, u, v);\n  u += du;\n"
        "  double dv = orc_sip_eval(w->bp, w->bp_order, u, v);\n  v += dv;"),
    "dropped_sip_term": ("for (int q = 0; q + p <= order; ++q) s +=",
                         "for (int q = 0; q + p < order; ++q) s +="),
    "bilinear_weights": ("    wt[0] = 1.0 - t;\n    dwt[0] = -1.0;", "    wt[0] = t;\n    dwt[0] = -1.0;"),
    "keys_kernel": ("return (a + 2.0) * s * s * s - (a + 3.0) * s * s + 1.0;",
                    "return (a + 2.0) * s * s * s - (a + 2.0) * s * s + 1.0;"),
    "bicubic_tap_offset": ("double d = x - (double)(i0 - 1 + k);", "double d = x - (double)(i0 + k);"),
    "no_normalisation": ("if (J->out) J->out[o] = cov ? S / F", "if (J->out) J->out[o] = cov ? S"),
    "nearest_rounding": ("idx[0] = (int64_t)rint(x);", "idx[0] = (int64_t)floor(x + 0.5);"),
    "edge_taps_counted": ("if (ix[i] < 0 || ix[i] >= w) continue;\n        double val",
                          "if (ix[i] < -1 || ix[i] > w) continue;\n        double val"),
    "behind_plane_valid": ("if (!(Z > 0.0)) return 0;             /* behind the tangent plane */",
                           ""),
    "grad_crpix_axis": ("gp[2] += gx;", "gp[2] += gy;"),
    "grad_cd_sign": ("double du = -cinv_col[k][0] * uv[l];", "double du = cinv_col[k][0] * uv[l];"),
    "grad_scatter_weight": ("if (grad_src) grad_src[iy[j] * w + ix[i]] += g * wx[i] * wy[j] / F;",
                            "if (grad_src) grad_src[iy[j] * w + ix[i]] += g * wx[i] * wy[j];"),
    # the footprint-normalisation terms of d out / d position (edge pixels)
    "grad_footprint_sign": ("double ox = (Sx - o * Fx) / F,", "double ox = (Sx + o * Fx) / F,"),
    "grad_footprint_dropped_y": (", oy = (Sy - o * Fy) / F;", ", oy = Sy / F;"),
    "grad_ap_monomial": ("gp[8 + p * (sw->ap_order + 1) + q] += gx * ipow(u, p) * ipow(v, q);",
                         "gp[8 + p * (sw->ap_order + 1) + q] += gx * ipow(u, q) * ipow(v, p);"),
    "grad_bp_axis": ("gp[8 + na + p * (sw->bp_order + 1) + q] += gy * ipow(u, p) * ipow(v, q);",
                     "gp[8 + na + p * (sw->bp_order + 1) + q] += gx * ipow(u, p) * ipow(v, q);"),
    "grad_crval_dz": ("dZ[1] = Y * D2R;", "dZ[1] = -Y * D2R;"),
    "condition_scale_signed": ("as += fabs(ww * val);", "as += ww * val;"),
    "grad_inverse_sip_jacobian": ("double gu = gx * (1.0 + apu) + gy * bpu; /* dL/du */",
                                  "double gu = gx * (1.0 + apu) + gy * apv; /* dL/du */"),
}


def _battery():
    """Run every pin with the currently routed oracle; return failures."""
    failed = []
    g = pins.geometries()
    checks = []
    for name in g:
        checks += [("crpix", lambda n=name: pins.test_crpix_maps_to_crval(oracle, n)),
                   ("p2w_vec", lambda n=name: pins.test_pix2world_matches_tangent_plane_vectors(oracle, n)),
                   ("w2p_vec", lambda n=name: pins.test_world2pix_matches_tangent_plane_vectors(oracle, n)),
                   ("roundtrip", lambda n=name: pins.test_round_trip_exact_inverse(oracle, n))]
    checks += [
        ("meridian", lambda: pins.test_central_meridian_closed_form(oracle)),
        ("pole", lambda: pins.test_pole_closed_form(oracle)),
        ("equator", lambda: pins.test_equator_ra_shift_closed_form(oracle)),
        ("sip_single", lambda: pins.test_sip_single_term_closed_form(oracle)),
        ("sip_eval", lambda: pins.test_sip_eval_matches_library_polynomial(oracle)),
        ("fit", lambda: pins.test_fitted_inverse_close_to_exact(oracle)),
        ("behind", lambda: pins.test_behind_tangent_plane_is_uncovered(oracle)),
        ("rot90", lambda: pins.test_rotation_by_90_degrees(oracle)),
        ("affine", lambda: pins.test_bilinear_reproduces_affine(oracle)),
        ("quadratic", lambda: pins.test_bicubic_reproduces_quadratic_and_constants(oracle)),
        ("nearest", lambda: pins.test_nearest_is_closest_pixel_ties_to_even(oracle)),
        ("footprint", lambda: pins.test_footprint_closed_forms(oracle)),
        ("adjoint", lambda: pins.test_adjoint_identity_source_gradient(oracle)),
        ("fd2", lambda: pins.test_parameter_gradient_vs_central_differences(oracle, 2)),
        ("fd_edge1", lambda: pins.test_parameter_gradient_edge_band_vs_central_differences(oracle, 1)),
        ("fd_edge2", lambda: pins.test_parameter_gradient_edge_band_vs_central_differences(oracle, 2)),
        ("grad_abs", lambda: pins.test_gradient_abs_scales_bound_the_sums(oracle)),
        ("fd_wide", lambda: pins.test_sky_gradient_wide_field_vs_central_differences(oracle)),
    ]
    for interp in (0, 1, 2):
        checks.append(("identity", lambda i=interp: pins.test_identity_wcs_returns_image(oracle, i)))
    for interp in (1, 2):
        checks.append(("brute8", lambda i=interp: pins.test_brute_force_8x8(oracle, i)))
        checks.append(("cond", lambda i=interp:
                       pins.test_condition_scale_brute_force_and_closed_form(oracle, i)))
    for interp in (0, 1):
        checks.append(("shift", lambda i=interp: pins.test_integer_crpix_shift_is_array_shift(oracle, i)))
    for tag, fn in checks:
        try:
            fn()
        except AssertionError:
            failed.append(tag)
        except Exception as e:  # a crash in a mutant counts as caught too
            failed.append(f"{tag}:{type(e).__name__}")
    return failed


@pytest.fixture(scope="module")
def workdir():
    d = tempfile.mkdtemp(prefix="orc_mut_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


def test_unmutated_source_passes_battery(workdir):
    out = obuild.compile_library(SRC, os.path.join(workdir, "lib_orig.so"))
    with oracle.use_library(out):
        assert _battery() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(workdir, name):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site for {name} not unique"
    src = os.path.join(workdir, f"{name}.c")
    with open(src, "w") as f:
        f.write(text.replace(old, new))
    shutil.copy(os.path.join(os.path.dirname(SRC), "oracle.h"), workdir)
    out = obuild.compile_library(src, os.path.join(workdir, f"lib_{name}.so"))
    with oracle.use_library(out):
        failed = _battery()
    assert failed, f"no pin caught the planted mistake {name}"
