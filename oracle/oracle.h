/*
 * Plain FP64 CPU oracle for per-pixel astronomical reprojection.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call this
 * library: only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code with the HIP implementation.
 *
 * It follows the paper's method step by step (section 3.1 overview,
 * section 3.2.1 "to celestial coordinates", section 3.2.2 "to source
 * coordinates"), then interpolates with zero padding and normalises by the
 * footprint (section 3.1, final paragraph).  Every value is FP64.
 *
 * Conventions: x = 0-based column, y = 0-based row, integer coordinates are
 * pixel centres; CRPIX is FITS 1-based (hence the "- 1" shift of section
 * 3.2); CRVAL and CD are in degrees.  SIP arrays are (order+1)^2 doubles,
 * element [p*(order+1)+q] = coefficient of u^p v^q.
 */
#ifndef DFR_ORACLE_H
#define DFR_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_wcs {
  double crpix[2];
  double crval[2];
  double cd[4];          /* CD1_1, CD1_2, CD2_1, CD2_2 */
  int32_t a_order, b_order, ap_order, bp_order;
  const double *a, *b, *ap, *bp;
} orc_wcs;

enum { ORC_NEAREST = 0, ORC_BILINEAR = 1, ORC_BICUBIC = 2 };

/* Section 3.2.1: pixel (x, y) of `w` -> (ra, dec) in degrees, ra in [0, 360). */
void orc_pix2world(const orc_wcs *w, double x, double y, double *ra, double *dec);

/* Section 3.2.2: (ra, dec) -> pixel of `w` through the inverse SIP AP/BP.
 * Returns 0 when the direction is on or behind the tangent plane (invalid). */
int orc_world2pix(const orc_wcs *w, double ra, double dec, double *x, double *y);

/* As orc_world2pix, but inverts the forward SIP A/B by Newton iteration
 * instead of using AP/BP (exact inverse; used for round-trip checks). */
int orc_world2pix_exact(const orc_wcs *w, double ra, double dec, double *x, double *y);

/* Target pixel -> source pixel position (both stages of section 3.2). */
int orc_position(const orc_wcs *src, const orc_wcs *tgt, double x, double y,
                 double *xs, double *ys);

/* Interpolation at one source position with zero padding (section 3.1 step 3
 * and footprint paragraph).  Returns S = sum of in-bounds w*src, F = sum of
 * in-bounds w; `absS` (nullable) = sum of |w*src| over in-bounds taps. */
void orc_interp(const float *src, int64_t h, int64_t w, int64_t pitch, double xs, double ys,
                int interp, double cubic_a, double *S, double *F, double *absS);

/* Full reprojection of the target rows listed in `rows` (n_rows of them) into
 * out/fp/pos ([n_rows][out_w], pos [n_rows][out_w][2]; each nullable).
 * out = S/F and fp = F where F > 0; else out = 0 (NaN when nan_outside) and
 * fp = 0.  pos receives the source position (NaN for invalid pixels).
 * Rows are split over `threads` POSIX threads (<= 0: all online cores). */
void orc_reproject_rows(const float *src, int64_t h, int64_t w, int64_t pitch,
                        const orc_wcs *src_wcs, const orc_wcs *tgt_wcs,
                        int64_t out_w, const int64_t *rows, int64_t n_rows,
                        int interp, double cubic_a, int nan_outside,
                        double *out, double *fp, double *pos, int threads);

/* Interpolation at n given source positions (pos [n][2]); writes the
 * normalised value, footprint and the condition scale sum|w*src|/|F|. */
void orc_interp_at(const float *src, int64_t h, int64_t w, int64_t pitch,
                   const double *pos, int64_t n, int interp, double cubic_a,
                   double *out, double *fp, double *cond);

/* Number of WCS parameters orc_grad reports for a source WCS:
 * crval(2), crpix(2), cd(4), ap[(ap_order+1)^2], bp[(bp_order+1)^2]. */
int64_t orc_n_params(const orc_wcs *src_wcs);

/* Gradient of a scalar loss L given g = dL/dout [out_h][out_w]:
 *   grad_src[k] = sum_p g_p * w_{k,p} / F_p                 ([h][w], nullable)
 *   grad_params = dL/d(source WCS parameters) in the order of orc_n_params
 *                 (degrees for CRVAL and CD; entries of AP/BP with
 *                 p+q > order are 0).                         (nullable)
 *   grad_src_abs, grad_params_abs: the same sums with every term replaced
 *                 by its magnitude (nullable).
 * Pixels with F <= 0 or an invalid position contribute nothing. */
void orc_grad(const float *src, int64_t h, int64_t w, int64_t pitch,
              const orc_wcs *src_wcs, const orc_wcs *tgt_wcs,
              int64_t out_h, int64_t out_w, int interp, double cubic_a,
              const double *grad_out, double *grad_src, double *grad_params,
              double *grad_src_abs, double *grad_params_abs);

/* Array forms of the two stages (xy, radec: [n][2]; valid may be NULL). */
void orc_pix2world_n(const orc_wcs *w, const double *xy, int64_t n, double *radec);
void orc_world2pix_n(const orc_wcs *w, const double *radec, int64_t n, double *xy, int32_t *valid,
                     int exact);

/* SIP polynomial sum_{p+q<=order} c[p][q] u^p v^q (plain power sums). */
double orc_sip_eval(const double *c, int order, double u, double v);

int orc_online_cores(void);

#ifdef __cplusplus
}
#endif
#endif
