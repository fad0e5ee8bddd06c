// Host-side FP64 set-up: validation of the C-ABI arguments and the
// composition of everything the kernels consume.
#pragma once

#include "common.hpp"
#include "launch.hpp"

namespace dfr {

dfr_status check_wcs(const dfr_wcs *w, bool as_source);

// Fill `P` for one source frame onto the target grid.  Requires validated
// WCS.  Composes H = A_s^-1 R A_t (FP64), packs the SIP coefficients and
// their FP32 scaled copies.
void build_plan(const float *src, int32_t src_h, int32_t src_w, int64_t pitch,
                const dfr_wcs &sw, const dfr_wcs &tw, int32_t out_h, int32_t out_w, float *out,
                float *fp, FramePlan &P);

void build_trig_plan(const dfr_wcs &sw, const dfr_wcs &tw, TrigPlan &T);

// Floats of LDS a tile of shape `s` needs for its source box, estimated from
// the Jacobian of the map sampled over the output frame (never below the
// exact need of an affine map; the kernel falls back to global gathers for
// a tile whose exact box is larger).
int estimate_lds_floats(const FramePlan &P, int32_t out_h, int32_t out_w, const TileShape &s,
                        int interp);

// Largest |d source / d target| over the output frame (for tile choice).
double max_magnification(const FramePlan &P, int32_t out_h, int32_t out_w);

// d H / d theta for theta = source (CRVAL1, CRVAL2, CD1_1, CD1_2, CD2_1,
// CD2_2) in degrees: jac[9 * 6], column-major by parameter.
void h_jacobian(const dfr_wcs &sw, const dfr_wcs &tw, double jac[54]);

}  // namespace dfr
