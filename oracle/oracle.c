/*
 * Plain FP64 CPU oracle for per-pixel astronomical reprojection.
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product path.  Shares no
 * code with the HIP implementation.
 *
 * Written from the paper's section 3 (method overview, the two coordinate
 * stages of section 3.2 and the footprint normalisation), the SIP convention
 * of Shupe et al. (2005) and the TAN projection of Calabretta & Greisen
 * (2002).  Readings where the paper is silent or garbled:
 *   - the garbled two-argument arctangent is atan2(numerator, denominator);
 *   - the arcsine of section 3.2 is evaluated as atan2(z, hypot(x, y)) of the
 *     same unit vector (same function, numerically stable near the tangent
 *     point); the arcsine of the inverse stage likewise;
 *   - SIP corrections are added (the SIP convention the paper says it
 *     follows) and both coordinates use the pre-update (u, v);
 *   - a direction on or behind the source tangent plane (sin theta <= 0) has
 *     no source position and is uncovered;
 *   - taps outside the source contribute nothing to the value or the
 *     footprint (zero padding); output = value / footprint where the
 *     footprint is > 0, otherwise 0 and footprint 0;
 *   - nearest = round half to even; bicubic = Keys cubic convolution with
 *     parameter a (default -0.5).
 */
#define _GNU_SOURCE
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

static const double R0 = 180.0 / M_PI; /* r_0 of section 3.2.1 */
static const double D2R = M_PI / 180.0;

/* ------------------------------------------------------------------ SIP -- */

static double ipow(double x, int n) {
  double r = 1.0;
  for (int i = 0; i < n; ++i) r *= x;
  return r;
}

/* f(u, v) = sum_{p+q<=order} c[p][q] u^p v^q  (SIP convention) */
double orc_sip_eval(const double *c, int order, double u, double v) {
  if (!c || order <= 0) return 0.0;
  double s = 0.0;
  for (int p = 0; p <= order; ++p)
    for (int q = 0; q + p <= order; ++q) s += c[p * (order + 1) + q] * ipow(u, p) * ipow(v, q);
  return s;
}

/* partial derivatives of the same polynomial */
static void sip_partials(const double *c, int order, double u, double v, double *fu, double *fv) {
  double su = 0.0, sv = 0.0;
  if (c && order > 0) {
    for (int p = 0; p <= order; ++p)
      for (int q = 0; q + p <= order; ++q) {
        double k = c[p * (order + 1) + q];
        if (p > 0) su += k * p * ipow(u, p - 1) * ipow(v, q);
        if (q > 0) sv += k * q * ipow(u, p) * ipow(v, q - 1);
      }
  }
  *fu = su;
  *fv = sv;
}

/* -------------------------------------------- section 3.2.1: to the sky -- */

void orc_pix2world(const orc_wcs *w, double x, double y, double *ra, double *dec) {
  /* shift (0-based pixels) */
  double u = x - (w->crpix[0] - 1.0);
  double v = y - (w->crpix[1] - 1.0);
  /* SIP distortion A/B, both evaluated at the undistorted (u, v) */
  double du = orc_sip_eval(w->a, w->a_order, u, v);
  double dv = orc_sip_eval(w->b, w->b_order, u, v);
  u += du;
  v += dv;
  /* CD matrix: intermediate coordinates in degrees */
  double up = w->cd[0] * u + w->cd[1] * v;
  double vp = w->cd[2] * u + w->cd[3] * v;
  /* gnomonic deprojection to native spherical (phi, theta) */
  double r = hypot(up, vp);
  double phi = atan2(-up, vp);
  double theta = atan2(R0, r);
  /* spherical rotation to (ra, dec) about the reference point */
  double d0 = w->crval[1] * D2R;
  double st = sin(theta), ct = cos(theta), sp = sin(phi), cp = cos(phi);
  double Z = st * sin(d0) + ct * cos(d0) * cp;
  double X = -ct * sp;
  double Y = st * cos(d0) - ct * sin(d0) * cp;
  double de = atan2(Z, hypot(X, Y)); /* = asin(Z) for the unit vector (X, Y, Z) */
  double a = w->crval[0] + atan2(X, Y) / D2R;
  a = fmod(a, 360.0);
  if (a < 0) a += 360.0;
  *ra = a;
  *dec = de / D2R;
}

/* ------------------------------------ section 3.2.2: to source coords -- */

/* native (phi, theta) -> projection plane (u', v') -> CD^-1 -> (u, v) */
static int sky_to_intermediate(const orc_wcs *w, double ra, double dec, double *u, double *v) {
  double d0 = w->crval[1] * D2R;
  double dra = (ra - w->crval[0]) * D2R;
  double de = dec * D2R;
  double X = -cos(de) * sin(dra);
  double Y = sin(de) * cos(d0) - cos(de) * sin(d0) * cos(dra);
  double Z = sin(de) * sin(d0) + cos(de) * cos(d0) * cos(dra);
  double phi = atan2(X, Y);
  double theta = atan2(Z, hypot(X, Y)); /* = asin(Z) */
  if (!(Z > 0.0)) return 0;             /* behind the tangent plane */
  double r = R0 * cos(theta) / sin(theta);
  double up = -r * sin(phi);
  double vp = r * cos(phi);
  double det = w->cd[0] * w->cd[3] - w->cd[1] * w->cd[2];
  *u = (w->cd[3] * up - w->cd[1] * vp) / det;
  *v = (-w->cd[2] * up + w->cd[0] * vp) / det;
  return 1;
}

int orc_world2pix(const orc_wcs *w, double ra, double dec, double *x, double *y) {
  double u, v;
  if (!sky_to_intermediate(w, ra, dec, &u, &v)) {
    *x = NAN;
    *y = NAN;
    return 0;
  }
  /* inverse SIP AP/BP, both evaluated at the same (u, v) */
  double du = orc_sip_eval(w->ap, w->ap_order, u, v);
  double dv = orc_sip_eval(w->bp, w->bp_order, u, v);
  u += du;
  v += dv;
  /* shift back */
  *x = u + (w->crpix[0] - 1.0);
  *y = v + (w->crpix[1] - 1.0);
  return 1;
}

int orc_world2pix_exact(const orc_wcs *w, double ra, double dec, double *x, double *y) {
  double U, V;
  if (!sky_to_intermediate(w, ra, dec, &U, &V)) {
    *x = NAN;
    *y = NAN;
    return 0;
  }
  /* solve u + A(u,v) = U, v + B(u,v) = V by Newton's method */
  double u = U, v = V;
  for (int it = 0; it < 60; ++it) {
    double fu = u + orc_sip_eval(w->a, w->a_order, u, v) - U;
    double fv = v + orc_sip_eval(w->b, w->b_order, u, v) - V;
    double au, av, bu, bv;
    sip_partials(w->a, w->a_order, u, v, &au, &av);
    sip_partials(w->b, w->b_order, u, v, &bu, &bv);
    double j00 = 1.0 + au, j01 = av, j10 = bu, j11 = 1.0 + bv;
    double det = j00 * j11 - j01 * j10;
    double su = (j11 * fu - j01 * fv) / det;
    double sv = (-j10 * fu + j00 * fv) / det;
    u -= su;
    v -= sv;
    if (fabs(su) + fabs(sv) < 1e-15 * (1.0 + fabs(u) + fabs(v))) break;
  }
  *x = u + (w->crpix[0] - 1.0);
  *y = v + (w->crpix[1] - 1.0);
  return 1;
}

void orc_pix2world_n(const orc_wcs *w, const double *xy, int64_t n, double *radec) {
  for (int64_t k = 0; k < n; ++k) orc_pix2world(w, xy[2 * k], xy[2 * k + 1], &radec[2 * k], &radec[2 * k + 1]);
}

void orc_world2pix_n(const orc_wcs *w, const double *radec, int64_t n, double *xy, int32_t *valid,
                     int exact) {
  for (int64_t k = 0; k < n; ++k) {
    int ok = exact ? orc_world2pix_exact(w, radec[2 * k], radec[2 * k + 1], &xy[2 * k], &xy[2 * k + 1])
                   : orc_world2pix(w, radec[2 * k], radec[2 * k + 1], &xy[2 * k], &xy[2 * k + 1]);
    if (valid) valid[k] = ok;
  }
}

int orc_position(const orc_wcs *src, const orc_wcs *tgt, double x, double y, double *xs,
                 double *ys) {
  double ra, dec;
  orc_pix2world(tgt, x, y, &ra, &dec);
  return orc_world2pix(src, ra, dec, xs, ys);
}

/* ------------------------------------------------------- interpolation -- */

/* Keys (1981) cubic convolution kernel with parameter a */
static double keys(double s, double a) {
  s = fabs(s);
  if (s <= 1.0) return (a + 2.0) * s * s * s - (a + 3.0) * s * s + 1.0;
  if (s < 2.0) return a * s * s * s - 5.0 * a * s * s + 8.0 * a * s - 4.0 * a;
  return 0.0;
}

/* d/ds of keys(s) for s >= 0 */
static double keys_d(double s, double a) {
  double sg = s < 0 ? -1.0 : 1.0;
  s = fabs(s);
  if (s <= 1.0) return sg * (3.0 * (a + 2.0) * s * s - 2.0 * (a + 3.0) * s);
  if (s < 2.0) return sg * (3.0 * a * s * s - 10.0 * a * s + 8.0 * a);
  return 0.0;
}

/* 1-D taps: index, weight and d(weight)/d(position) */
static int taps1d(double x, int interp, double a, int64_t *idx, double *wt, double *dwt) {
  if (interp == ORC_NEAREST) {
    idx[0] = (int64_t)rint(x); /* half to even in the default rounding mode */
    wt[0] = 1.0;
    dwt[0] = 0.0;
    return 1;
  }
  double f = floor(x);
  double t = x - f;
  int64_t i0 = (int64_t)f;
  if (interp == ORC_BILINEAR) {
    idx[0] = i0;
    wt[0] = 1.0 - t;
    dwt[0] = -1.0;
    idx[1] = i0 + 1;
    wt[1] = t;
    dwt[1] = 1.0;
    return 2;
  }
  /* bicubic: distances from the position to taps i0-1 .. i0+2 */
  for (int k = 0; k < 4; ++k) {
    double d = x - (double)(i0 - 1 + k); /* 1+t, t, t-1, t-2 */
    idx[k] = i0 - 1 + k;
    wt[k] = keys(d, a);
    dwt[k] = keys_d(d, a);
  }
  return 4;
}

/* generic interpolation with derivatives (any pointer may be NULL) */
static void interp_full(const float *src, int64_t h, int64_t w, int64_t pitch, double xs, double ys,
                        int interp, double a, double *S, double *F, double *absS, double *Sx,
                        double *Sy, double *Fx, double *Fy) {
  double s = 0, f = 0, as = 0, sx = 0, sy = 0, fx = 0, fy = 0;
  if (isfinite(xs) && isfinite(ys) && fabs(xs) < 4e15 && fabs(ys) < 4e15) {
    int64_t ix[4], iy[4];
    double wx[4], wy[4], dx[4], dy[4];
    int nx = taps1d(xs, interp, a, ix, wx, dx);
    int ny = taps1d(ys, interp, a, iy, wy, dy);
    for (int j = 0; j < ny; ++j) {
      if (iy[j] < 0 || iy[j] >= h) continue;
      for (int i = 0; i < nx; ++i) {
        if (ix[i] < 0 || ix[i] >= w) continue;
        double val = (double)src[iy[j] * pitch + ix[i]];
        double ww = wx[i] * wy[j];
        s += ww * val;
        f += ww;
        as += fabs(ww * val);
        sx += dx[i] * wy[j] * val;
        sy += wx[i] * dy[j] * val;
        fx += dx[i] * wy[j];
        fy += wx[i] * dy[j];
      }
    }
  }
  if (S) *S = s;
  if (F) *F = f;
  if (absS) *absS = as;
  if (Sx) *Sx = sx;
  if (Sy) *Sy = sy;
  if (Fx) *Fx = fx;
  if (Fy) *Fy = fy;
}

void orc_interp(const float *src, int64_t h, int64_t w, int64_t pitch, double xs, double ys,
                int interp, double cubic_a, double *S, double *F, double *absS) {
  interp_full(src, h, w, pitch, xs, ys, interp, cubic_a, S, F, absS, NULL, NULL, NULL, NULL);
}

void orc_interp_at(const float *src, int64_t h, int64_t w, int64_t pitch, const double *pos,
                   int64_t n, int interp, double cubic_a, double *out, double *fp, double *cond) {
  for (int64_t k = 0; k < n; ++k) {
    double S, F, aS;
    interp_full(src, h, w, pitch, pos[2 * k], pos[2 * k + 1], interp, cubic_a, &S, &F, &aS, NULL,
                NULL, NULL, NULL);
    int cov = F > 0.0;
    if (out) out[k] = cov ? S / F : 0.0;
    if (fp) fp[k] = cov ? F : 0.0;
    if (cond) cond[k] = cov ? aS / F : 0.0;
  }
}

/* ------------------------------------------------------- reprojection -- */

typedef struct {
  const float *src;
  int64_t h, w, pitch;
  const orc_wcs *sw, *tw;
  int64_t out_w;
  const int64_t *rows;
  int64_t n_rows;
  int interp;
  double a;
  int nan_outside;
  double *out, *fp, *pos;
  int tid, nthreads;
} job_t;

static void reproject_one_row(const job_t *J, int64_t r) {
  int64_t y = J->rows[r];
  for (int64_t x = 0; x < J->out_w; ++x) {
    double xs = NAN, ys = NAN, S = 0.0, F = 0.0;
    int ok = orc_position(J->sw, J->tw, (double)x, (double)y, &xs, &ys);
    if (ok && J->h > 0 && J->w > 0)
      interp_full(J->src, J->h, J->w, J->pitch, xs, ys, J->interp, J->a, &S, &F, NULL, NULL, NULL,
                  NULL, NULL);
    int cov = ok && F > 0.0;
    int64_t o = r * J->out_w + x;
    if (J->out) J->out[o] = cov ? S / F : (J->nan_outside ? NAN : 0.0);
    if (J->fp) J->fp[o] = cov ? F : 0.0;
    if (J->pos) {
      J->pos[2 * o] = ok ? xs : NAN;
      J->pos[2 * o + 1] = ok ? ys : NAN;
    }
  }
}

static void *reproject_worker(void *arg) {
  const job_t *J = (const job_t *)arg;
  for (int64_t r = J->tid; r < J->n_rows; r += J->nthreads) reproject_one_row(J, r);
  return NULL;
}

int orc_online_cores(void) {
  long n = sysconf(_SC_NPROCESSORS_ONLN);
  return n > 0 ? (int)n : 1;
}

void orc_reproject_rows(const float *src, int64_t h, int64_t w, int64_t pitch,
                        const orc_wcs *src_wcs, const orc_wcs *tgt_wcs, int64_t out_w,
                        const int64_t *rows, int64_t n_rows, int interp, double cubic_a,
                        int nan_outside, double *out, double *fp, double *pos, int threads) {
  if (threads <= 0) threads = orc_online_cores();
  if (threads > n_rows) threads = n_rows > 0 ? (int)n_rows : 1;
  job_t *jobs = (job_t *)calloc((size_t)threads, sizeof(job_t));
  pthread_t *th = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
  for (int t = 0; t < threads; ++t) {
    job_t J = {src, h, w, pitch, src_wcs, tgt_wcs, out_w, rows, n_rows, interp, cubic_a,
               nan_outside, out, fp, pos, t, threads};
    jobs[t] = J;
  }
  if (threads == 1) {
    reproject_worker(&jobs[0]);
  } else {
    for (int t = 0; t < threads; ++t) pthread_create(&th[t], NULL, reproject_worker, &jobs[t]);
    for (int t = 0; t < threads; ++t) pthread_join(th[t], NULL);
  }
  free(th);
  free(jobs);
}

/* ----------------------------------------------------------- gradient -- */

int64_t orc_n_params(const orc_wcs *sw) {
  int64_t na = sw->ap_order > 0 ? (int64_t)(sw->ap_order + 1) * (sw->ap_order + 1) : 0;
  int64_t nb = sw->bp_order > 0 ? (int64_t)(sw->bp_order + 1) * (sw->bp_order + 1) : 0;
  return 8 + na + nb;
}

/* Each gradient entry is a sum of one term per output pixel (and, for the
 * source, per tap); the *_abs outputs, when non-null, receive the sums of
 * the terms' magnitudes: the scale against which the rounding of such a sum
 * is measured. */
void orc_grad(const float *src, int64_t h, int64_t w, int64_t pitch, const orc_wcs *sw,
              const orc_wcs *tw, int64_t out_h, int64_t out_w, int interp, double a,
              const double *grad_out, double *grad_src, double *grad_params,
              double *grad_src_abs, double *grad_params_abs) {
  int64_t np = orc_n_params(sw);
  int na = sw->ap_order > 0 ? (sw->ap_order + 1) * (sw->ap_order + 1) : 0;
  if (grad_src)
    for (int64_t k = 0; k < h * w; ++k) grad_src[k] = 0.0;
  if (grad_src_abs)
    for (int64_t k = 0; k < h * w; ++k) grad_src_abs[k] = 0.0;
  double *gp = (double *)calloc((size_t)np, sizeof(double));
  double *ga = (double *)calloc((size_t)np, sizeof(double));
  double det = sw->cd[0] * sw->cd[3] - sw->cd[1] * sw->cd[2];
  /* CD^-1 */
  double ci00 = sw->cd[3] / det, ci01 = -sw->cd[1] / det;
  double ci10 = -sw->cd[2] / det, ci11 = sw->cd[0] / det;
  double d0 = sw->crval[1] * D2R;
  for (int64_t y = 0; y < out_h; ++y) {
    for (int64_t x = 0; x < out_w; ++x) {
      double g = grad_out[y * out_w + x];
      if (g == 0.0) continue;
      double ra, dec;
      orc_pix2world(tw, (double)x, (double)y, &ra, &dec);
      double dra = (ra - sw->crval[0]) * D2R, de = dec * D2R;
      double X = -cos(de) * sin(dra);
      double Y = sin(de) * cos(d0) - cos(de) * sin(d0) * cos(dra);
      double Z = sin(de) * sin(d0) + cos(de) * cos(d0) * cos(dra);
      if (!(Z > 0.0)) continue;
      double u, v, xs, ys;
      sky_to_intermediate(sw, ra, dec, &u, &v);
      orc_world2pix(sw, ra, dec, &xs, &ys);
      double S, F, Sx, Sy, Fx, Fy;
      interp_full(src, h, w, pitch, xs, ys, interp, a, &S, &F, NULL, &Sx, &Sy, &Fx, &Fy);
      if (!(F > 0.0)) continue;
      double o = S / F;
      /* d out / d (xs, ys) */
      double ox = (Sx - o * Fx) / F, oy = (Sy - o * Fy) / F;
      double gx = g * ox, gy = g * oy; /* dL/dxs, dL/dys */
      /* d pos / d (u, v) through the inverse SIP */
      double apu, apv, bpu, bpv;
      sip_partials(sw->ap, sw->ap_order, u, v, &apu, &apv);
      sip_partials(sw->bp, sw->bp_order, u, v, &bpu, &bpv);
      double gu = gx * (1.0 + apu) + gy * bpu; /* dL/du */
      double gv = gx * apv + gy * (1.0 + bpv); /* dL/dv */
      /* projection plane (x', y') = R0 * (-X/Z, Y/Z); derivatives wrt CRVAL */
      double dX[2], dY[2], dZ[2];
      dX[0] = cos(de) * cos(dra) * D2R;
      dY[0] = -cos(de) * sin(d0) * sin(dra) * D2R;
      dZ[0] = cos(de) * cos(d0) * sin(dra) * D2R;
      dX[1] = 0.0;
      dY[1] = -Z * D2R;
      dZ[1] = Y * D2R;
      for (int k = 0; k < 2; ++k) {
        double dxp = -R0 * (dX[k] * Z - X * dZ[k]) / (Z * Z);
        double dyp = R0 * (dY[k] * Z - Y * dZ[k]) / (Z * Z);
        double du = ci00 * dxp + ci01 * dyp;
        double dv = ci10 * dxp + ci11 * dyp;
        gp[k] += gu * du + gv * dv;
        ga[k] += fabs(gu * du + gv * dv);
      }
      /* CRPIX */
      gp[2] += gx;
      gp[3] += gy;
      ga[2] += fabs(gx);
      ga[3] += fabs(gy);
      /* CD_kl: d(u,v) = -CD^-1 E_kl (u,v) */
      double uv[2] = {u, v};
      double cinv_col[2][2] = {{ci00, ci10}, {ci01, ci11}}; /* column k of CD^-1 */
      for (int k = 0; k < 2; ++k)
        for (int l = 0; l < 2; ++l) {
          double du = -cinv_col[k][0] * uv[l];
          double dv = -cinv_col[k][1] * uv[l];
          gp[4 + 2 * k + l] += gu * du + gv * dv;
          ga[4 + 2 * k + l] += fabs(gu * du + gv * dv);
        }
      /* AP, BP coefficients */
      for (int p = 0; p <= sw->ap_order && sw->ap_order > 0; ++p)
        for (int q = 0; q + p <= sw->ap_order; ++q)
        {
          gp[8 + p * (sw->ap_order + 1) + q] += gx * ipow(u, p) * ipow(v, q);
          ga[8 + p * (sw->ap_order + 1) + q] += fabs(gx * ipow(u, p) * ipow(v, q));
        }
      for (int p = 0; p <= sw->bp_order && sw->bp_order > 0; ++p)
        for (int q = 0; q + p <= sw->bp_order; ++q)
        {
          gp[8 + na + p * (sw->bp_order + 1) + q] += gy * ipow(u, p) * ipow(v, q);
          ga[8 + na + p * (sw->bp_order + 1) + q] += fabs(gy * ipow(u, p) * ipow(v, q));
        }
      /* source image: scatter of the interpolation weights */
      if (grad_src || grad_src_abs) {
        int64_t ix[4], iy[4];
        double wx[4], wy[4], dxw[4], dyw[4];
        int nx = taps1d(xs, interp, a, ix, wx, dxw);
        int ny = taps1d(ys, interp, a, iy, wy, dyw);
        for (int j = 0; j < ny; ++j) {
          if (iy[j] < 0 || iy[j] >= h) continue;
          for (int i = 0; i < nx; ++i) {
            if (ix[i] < 0 || ix[i] >= w) continue;
            if (grad_src) grad_src[iy[j] * w + ix[i]] += g * wx[i] * wy[j] / F;
            if (grad_src_abs) grad_src_abs[iy[j] * w + ix[i]] += fabs(g * wx[i] * wy[j] / F);
          }
        }
      }
    }
  }
  if (grad_params) memcpy(grad_params, gp, (size_t)np * sizeof(double));
  if (grad_params_abs) memcpy(grad_params_abs, ga, (size_t)np * sizeof(double));
  free(gp);
  free(ga);
}
