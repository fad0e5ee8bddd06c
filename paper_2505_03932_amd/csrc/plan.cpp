// Host FP64 set-up (validation, composition of the projective map, SIP
// packing, LDS sizing, parameter Jacobian of the map).
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace dfr {

namespace {

const double kD2R = M_PI / 180.0;
const double kR2D = 180.0 / M_PI;

bool finite_all(const double *v, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

dfr_status check_poly(int order, const double *c) {
  if (order < 0 || order > DFR_MAX_SIP_ORDER) return DFR_E_WCS;
  if (order == 0) return DFR_OK;
  if (!c) return DFR_E_NULL;
  for (int p = 0; p <= order; ++p)
    for (int q = 0; q <= order; ++q) {
      double v = c[p * (order + 1) + q];
      if (!std::isfinite(v)) return DFR_E_WCS;
      if (p + q > order && v != 0.0) return DFR_E_WCS;
    }
  return DFR_OK;
}

// Tangent frame of a reference point: columns east, north, centre (unit
// vectors in equatorial Cartesian coordinates); row-major M[r * 3 + c].
void tangent_frame(double ra_deg, double dec_deg, double M[9]) {
  double a = ra_deg * kD2R, d = dec_deg * kD2R;
  double sa = std::sin(a), ca = std::cos(a), sd = std::sin(d), cd = std::cos(d);
  double e[3] = {-sa, ca, 0.0};
  double n[3] = {-sd * ca, -sd * sa, cd};
  double c[3] = {cd * ca, cd * sa, sd};
  for (int r = 0; r < 3; ++r) {
    M[r * 3 + 0] = e[r];
    M[r * 3 + 1] = n[r];
    M[r * 3 + 2] = c[r];
  }
}

void matmul3(const double A[9], const double B[9], double C[9]) {
  double T[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += A[i * 3 + k] * B[k * 3 + j];
      T[i * 3 + j] = s;
    }
  std::memcpy(C, T, sizeof(T));
}

// R = Ms^T Mt
void rotation(const double Ms[9], const double Mt[9], double R[9]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int r = 0; r < 3; ++r) s += Ms[r * 3 + i] * Mt[r * 3 + j];
      R[i * 3 + j] = s;
    }
}

void cd_inverse(const double cd[4], double ci[4]) {
  double det = cd[0] * cd[3] - cd[1] * cd[2];
  ci[0] = cd[3] / det;
  ci[1] = -cd[1] / det;
  ci[2] = -cd[2] / det;
  ci[3] = cd[0] / det;
}

// A_t: SIP-corrected target offset -> standard coordinates (radians), w = 1
void a_target(const double cd[4], double A[9]) {
  double v[9] = {cd[0] * kD2R, cd[1] * kD2R, 0.0, cd[2] * kD2R, cd[3] * kD2R, 0.0, 0.0, 0.0, 1.0};
  std::memcpy(A, v, sizeof(v));
}

// A_s^-1: standard coordinates (radians, projective) -> source offset
void a_source_inv(const double cd[4], double A[9]) {
  double ci[4];
  cd_inverse(cd, ci);
  double v[9] = {ci[0] * kR2D, ci[1] * kR2D, 0.0, ci[2] * kR2D, ci[3] * kR2D, 0.0, 0.0, 0.0, 1.0};
  std::memcpy(A, v, sizeof(v));
}

void pack(const double *c, int order, double *out) {
  for (int i = 0; i < kMaxCoef; ++i) out[i] = 0.0;
  if (!c || order <= 0) return;
  for (int p = 0; p <= order; ++p)
    for (int q = 0; p + q <= order; ++q) out[tri9(p, q)] = c[p * (order + 1) + q];
}

void scale_pack(const double *in, double S, float *out) {
  for (int p = 0; p <= kMaxOrder; ++p)
    for (int q = 0; p + q <= kMaxOrder; ++q)
      out[tri9(p, q)] = (float)(in[tri9(p, q)] * std::pow(S, p + q));
}

}  // namespace

dfr_status check_wcs(const dfr_wcs *w, bool as_source) {
  if (!w) return DFR_E_NULL;
  if (!finite_all(w->crpix, 2) || !finite_all(w->crval, 2) || !finite_all(w->cd, 4))
    return DFR_E_WCS;
  if (std::fabs(w->crval[1]) > 90.0) return DFR_E_WCS;
  double det = w->cd[0] * w->cd[3] - w->cd[1] * w->cd[2];
  if (!(det != 0.0) || !std::isfinite(det)) return DFR_E_WCS;
  dfr_status s;
  if ((s = check_poly(w->a_order, w->a)) != DFR_OK) return s;
  if ((s = check_poly(w->b_order, w->b)) != DFR_OK) return s;
  if ((s = check_poly(w->ap_order, w->ap)) != DFR_OK) return s;
  if ((s = check_poly(w->bp_order, w->bp)) != DFR_OK) return s;
  if (as_source && (w->a_order > 0 || w->b_order > 0) && w->ap_order == 0 && w->bp_order == 0)
    return DFR_E_UNSUPPORTED;
  return DFR_OK;
}

void build_plan(const float *src, int32_t src_h, int32_t src_w, int64_t pitch,
                const dfr_wcs &sw, const dfr_wcs &tw, int32_t out_h, int32_t out_w, float *out,
                float *fp, FramePlan &P) {
  std::memset(&P, 0, sizeof(P));
  P.crop[2] = out_w;
  P.crop[3] = out_h;
  double Ms[9], Mt[9], R[9], At[9], Asi[9], T[9];
  tangent_frame(sw.crval[0], sw.crval[1], Ms);
  tangent_frame(tw.crval[0], tw.crval[1], Mt);
  rotation(Ms, Mt, R);
  a_target(tw.cd, At);
  a_source_inv(sw.cd, Asi);
  matmul3(R, At, T);
  matmul3(Asi, T, P.H);
  P.tcr[0] = tw.crpix[0] - 1.0;
  P.tcr[1] = tw.crpix[1] - 1.0;
  P.scr[0] = sw.crpix[0] - 1.0;
  P.scr[1] = sw.crpix[1] - 1.0;
  double St = std::max(1.0, 0.5 * std::max(out_h, out_w));
  double Ss = std::max(1.0, 0.5 * std::max(src_h, src_w));
  P.t_inv_scale = 1.0 / St;
  P.s_inv_scale = 1.0 / Ss;
  P.s_scale = Ss;
  P.src = src;
  P.pitch = pitch;
  P.src_h = src_h;
  P.src_w = src_w;
  P.out = out;
  P.fp = fp;
  P.t_order = std::max(tw.a_order, tw.b_order);
  P.s_order = std::max(sw.ap_order, sw.bp_order);
  pack(tw.a, tw.a_order, P.tA);
  pack(tw.b, tw.b_order, P.tB);
  pack(sw.ap, sw.ap_order, P.sA);
  pack(sw.bp, sw.bp_order, P.sB);
  scale_pack(P.tA, St, P.ftA);
  scale_pack(P.tB, St, P.ftB);
  scale_pack(P.sA, Ss, P.fsA);
  scale_pack(P.sB, Ss, P.fsB);
  // The projective denominator over a cell is 1 + e with |e| <= (|H20| +
  // |H21|) * 31 / w.  w is linear in the target offset, so its minimum over
  // the output frame (grown by a margin for target SIP) is at a corner.  When
  // |e| < 1e-3 everywhere, 1/(1+e) is evaluated as 1 - e + e^2 (relative
  // error below 1e-9) instead of a reciprocal instruction.
  {
    double mg = 64.0 + 0.1 * std::max(out_h, out_w);
    double wmin = 1e300;
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        double u = (cx ? out_w - 1 + mg : -mg) - P.tcr[0];
        double v = (cy ? out_h - 1 + mg : -mg) - P.tcr[1];
        wmin = std::min(wmin, P.H[6] * u + P.H[7] * v + P.H[8]);
      }
    double kap = wmin > 0.0 ? 1.2 * (std::fabs(P.H[6]) + std::fabs(P.H[7])) * (kCell - 1) / wmin
                            : 1e300;
    P.series = kap < 1e-3 ? 1 : 0;
  }
}

void build_trig_plan(const dfr_wcs &sw, const dfr_wcs &tw, TrigPlan &T) {
  for (int i = 0; i < 4; ++i) T.tcd[i] = tw.cd[i];
  cd_inverse(sw.cd, T.scdi);
  T.tcrval[0] = tw.crval[0] * kD2R;
  T.tcrval[1] = tw.crval[1] * kD2R;
  T.scrval[0] = sw.crval[0] * kD2R;
  T.scrval[1] = sw.crval[1] * kD2R;
}

namespace {

// Jacobian d(source position)/d(target pixel) at (x, y) by FP64 differences.
bool jacobian_at(const FramePlan &P, double x, double y, double J[4]) {
  const double h = 4.0;
  double x0, y0, x1, y1, x2, y2;
  if (!position_f64(P, x, y, x0, y0) || !position_f64(P, x + h, y, x1, y1) ||
      !position_f64(P, x, y + h, x2, y2))
    return false;
  J[0] = (x1 - x0) / h;
  J[1] = (x2 - x0) / h;
  J[2] = (y1 - y0) / h;
  J[3] = (y2 - y0) / h;
  return std::isfinite(J[0] + J[1] + J[2] + J[3]);
}

}  // namespace

int estimate_lds_floats(const FramePlan &P, int32_t out_h, int32_t out_w, const TileShape &s,
                        int interp) {
  const int support = interp == DFR_NEAREST ? 1 : (interp == DFR_BILINEAR ? 2 : 4);
  double best = 0.0;
  bool any = false;
  for (int iy = 0; iy < 5; ++iy)
    for (int ix = 0; ix < 5; ++ix) {
      double x = (out_w - 1) * ix / 4.0, y = (out_h - 1) * iy / 4.0;
      double J[4];
      if (!jacobian_at(P, x, y, J)) continue;
      any = true;
      // the kernel's box: extreme tap origins grown by the support and 2 px,
      // rows padded by up to 3 floats (LDS bank spread)
      double bw = std::fabs(J[0]) * (s.width - 1) + std::fabs(J[1]) * (s.height - 1) + support + 9.0;
      double bh = std::fabs(J[2]) * (s.width - 1) + std::fabs(J[3]) * (s.height - 1) + support + 6.0;
      best = std::max(best, bw * bh);
    }
  if (!any) best = 2.0 * s.width * s.height;
  double f = std::ceil(best * 1.1 + 64.0);
  return (int)std::min(f, 1.0e9);
}

double max_magnification(const FramePlan &P, int32_t out_h, int32_t out_w) {
  double m = 0.0;
  for (int iy = 0; iy < 3; ++iy)
    for (int ix = 0; ix < 3; ++ix) {
      double J[4];
      if (!jacobian_at(P, (out_w - 1) * ix / 2.0, (out_h - 1) * iy / 2.0, J)) continue;
      m = std::max(m, std::max(std::fabs(J[0]) + std::fabs(J[1]), std::fabs(J[2]) + std::fabs(J[3])));
    }
  return m;
}

void h_jacobian(const dfr_wcs &sw, const dfr_wcs &tw, double jac[54]) {
  double Ms[9], Mt[9], At[9], Asi[9], R[9];
  tangent_frame(sw.crval[0], sw.crval[1], Ms);
  tangent_frame(tw.crval[0], tw.crval[1], Mt);
  a_target(tw.cd, At);
  a_source_inv(sw.cd, Asi);
  rotation(Ms, Mt, R);
  double RAt[9];
  matmul3(R, At, RAt);
  double a = sw.crval[0] * kD2R, d = sw.crval[1] * kD2R;
  double sa = std::sin(a), ca = std::cos(a), sd = std::sin(d), cd = std::cos(d);
  // derivatives of the source tangent frame (columns east, north, centre)
  double dMa[9] = {-ca, sd * sa, -cd * sa,   //
                   -sa, -sd * ca, cd * ca,   //
                   0.0, 0.0, 0.0};
  double dMd[9] = {0.0, -cd * ca, -sd * ca,  //
                   0.0, -cd * sa, -sd * sa,  //
                   0.0, -sd, cd};
  double dR[9], T[9], out[9];
  // CRVAL1, CRVAL2 (per degree)
  const double *dM[2] = {dMa, dMd};
  for (int k = 0; k < 2; ++k) {
    rotation(dM[k], Mt, dR);
    matmul3(dR, At, T);
    matmul3(Asi, T, out);
    for (int i = 0; i < 9; ++i) jac[k * 9 + i] = out[i] * kD2R;
  }
  // CD_kl: d(CD^-1) = -CD^-1 E_kl CD^-1 in the upper-left block of A_s^-1
  double ci[4];
  cd_inverse(sw.cd, ci);
  for (int kl = 0; kl < 4; ++kl) {
    int k = kl / 2, l = kl % 2;
    double dA[9] = {0};
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) dA[i * 3 + j] = -ci[i * 2 + k] * ci[l * 2 + j] * kR2D;
    matmul3(dA, RAt, out);
    for (int i = 0; i < 9; ++i) jac[(2 + kl) * 9 + i] = out[i];
  }
}

}  // namespace dfr
