// Shared device-side definitions of the reprojection kernels (gfx950).
//
// Geometry (paper section 3.2).  Stage one takes a target pixel to the sky
// (shift, SIP A/B, CD, gnomonic deprojection, rotation to RA/Dec); stage two
// takes the sky to the source plane (rotation, gnomonic projection, CD^-1,
// SIP AP/BP, shift).  With tangent-plane standard coordinates, the rotation
// between the two tangent frames and both gnomonic steps compose exactly
// into one projective map of the SIP-corrected target offset (u, v):
//     (p, q, w) = H (u, v, 1),   (U, V) = (p / w, q / w),   valid iff w > 0,
// H = A_s^-1 R A_t, A = [[CD * pi/180, 0], [0, 1]], R = M_s^T M_t, and
// M = [east | north | centre] the tangent frame of each reference point.
// H is composed on the host in FP64.
//
// Precision split.  Per 32x32 cell of output pixels (a fixed grid, so tile
// shape and batching never change results) one lane evaluates the map in
// FP64 at the cell's anchor pixel and reduces it to small FP32 coefficients:
// every pixel of the cell then evaluates only offsets from the anchor in
// FP32, whose rounding is ~1e-7 of a few tens of pixels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dfr.h"

namespace dfr {

constexpr int kMaxOrder = DFR_MAX_SIP_ORDER;
constexpr int kMaxCoef = (kMaxOrder + 1) * (kMaxOrder + 2) / 2;  // 55
constexpr int kCellLog2 = 5;
constexpr int kCell = 1 << kCellLog2;  // anchor grid pitch in output pixels (both axes)
constexpr int kThreads = 256;   // work-group size of every tile kernel
constexpr int kRun = 4;         // consecutive output pixels per thread and row
constexpr int kMaxAnchors = 16; // anchors a tile covers at most

// Packed index of the SIP coefficient of u^p v^q (p + q <= kMaxOrder).
__host__ __device__ constexpr int tri9(int p, int q) {
  return p * (kMaxOrder + 1) - p * (p - 1) / 2 + q;
}

// Packed index of (p, q) among the (n+1)(n+2)/2 terms of an order-n polynomial.
__host__ __device__ constexpr int tri_n(int n, int p, int q) {
  return p * (n + 1) - p * (p - 1) / 2 + q;
}

struct CellModel;

// Everything a kernel needs about one source frame and the target grid.
// Built on the host in FP64 (plan.cpp); passed by value (single image) or
// through a device table (batch).
struct FramePlan {
  double H[9];              // source-from-target projective map, row-major
  double tcr[2];            // target CRPIX - 1
  double scr[2];            // source CRPIX - 1
  double t_inv_scale;       // 1 / S_t: target SIP arguments are (u, v) / S_t
  double s_inv_scale;       // 1 / S_s: source SIP arguments are (U, V) / S_s
  double s_scale;           // S_s
  const float *src;         // device source image
  int64_t pitch;            // source row pitch in elements
  int32_t src_h, src_w;
  float *out;               // device [out_h][out_w]
  float *fp;                // device [out_h][out_w] or null
  int32_t t_order;          // target A/B order (0 = none)
  int32_t s_order;          // source AP/BP order (0 = none)
  int32_t series;           // 1: |k.d| < 1e-3 over the frame, 1/(1+e) = 1 - e + e^2
  int32_t pad_;
  const CellModel *models;  // device table of per-cell position models, or null
  int32_t *reach;           // batch: the frame's reach box of cells (see kReachBig), or null
  int32_t crop[4];          // x0, y0, w, h of the frame's output window (full grid unless cropped)
  int32_t item0;            // cropped batch: first work item of the frame
  int32_t tile0[2];         // cropped batch: first tile column and row of the window
  int32_t ntx;              // cropped batch: tile columns of the window
  double tA[kMaxCoef], tB[kMaxCoef];   // FP64 coefficients, packed by tri9
  double sA[kMaxCoef], sB[kMaxCoef];
  float ftA[kMaxCoef], ftB[kMaxCoef];  // FP32, scaled: c * S^(p+q)
  float fsA[kMaxCoef], fsB[kMaxCoef];
};

// Launch-wide settings shared by every tile.
struct TileGeom {
  int32_t out_h, out_w;
  int32_t tiles_x, n_tiles;   // tiles per row of the output, tiles per frame
  int32_t txt_log2;           // threads per tile row = 1 << txt_log2 (each kRun px)
  int32_t lds_cap;            // floats of dynamic LDS for the staged source tile
  float cubic_a;
  int32_t nan_outside;
  int32_t allow_skip;         // skip provably uncovered tiles (off with debug output)
  double *debug;              // [out_h][out_w][2] source positions, or null
};

// Outputs of the coadd kernel: device [out_h][out_w] float32 each, not
// overlapping; coadd nullable.
struct CoaddOut {
  float *sum_wf;       // sum over frames of out * F
  float *sum_f;        // sum over frames of F
  float *coadd;        // sum_wf / sum_f where sum_f > 0
  int32_t accumulate;  // add to the sums already there instead of starting at 0
};

// Per-cell quantities from the FP64 anchor evaluation (kept in LDS).
struct alignas(16) Anchor {
  float g1, g2, f1, f2, k1, k2;  // dU = (g.d)/(1 + k.d), dV = (f.d)/(1 + k.d)
  float u0s, v0s;                // (U0, V0) / S_s
  float c0x, c0y;                // X0 - bx, Y0 - by in [0, 1)
  float tus, tvs;                // target anchor offset / S_t
  float ta0, tb0;                // FP32 target SIP at the anchor (for differencing)
  float sgn;                     // sign of w at the anchor
  float inv_w0;                  // 1 / w0 (gradient of H needs 1/w)
  float tu0, tv0;                // SIP-corrected target offset of the anchor (u, v)
  int32_t bx, by;                // integer parts of the anchor source position
  int32_t touch;                 // 0 when no pixel of the cell can reach the source
  int32_t ok;                    // every pixel of the cell has a valid, finite position
  float jx[2], jy[2];            // d(source position)/d(target pixel) at the anchor
  float sx0, sy0;                // source position at the anchor minus (bx, by)
  float ex, ey;                  // bound on |position - linear model| over the cell
};

// ------------------------------------------------------ SIP polynomials --

// Horner evaluation of sum_{p+q<=N} c[p][q] x^p y^q, compile-time order.
template <int N>
__device__ __forceinline__ float sip_f32(const float *__restrict__ c, float x, float y) {
  if constexpr (N <= 0) {
    return 0.0f;
  } else {
    float f = 0.0f;
#pragma unroll
    for (int p = N; p >= 0; --p) {
      float in = c[tri9(p, N - p)];
#pragma unroll
      for (int q = N - p - 1; q >= 0; --q) in = fmaf(in, y, c[tri9(p, q)]);
      f = (p == N) ? in : fmaf(f, x, in);
    }
    return f;
  }
}

// Same with a run-time order n <= kMaxOrder.  Fully unrolled over the
// maximum order with uniform guards, so the coefficient array is never
// indexed dynamically (a dynamically indexed kernel-argument array can make
// the compiler copy the whole plan to private memory).  The coefficients
// past order n are zero, so fma(0, y, c) = c keeps this bit-identical to a
// loop over the first n orders.
__device__ __forceinline__ float sip_f32_rt(const float *__restrict__ c, int n, float x, float y) {
  if (n <= 0) return 0.0f;
  float f = 0.0f;
#pragma unroll
  for (int p = kMaxOrder; p >= 0; --p) {
    if (p > n) continue;
    float in = 0.0f;
#pragma unroll
    for (int q = kMaxOrder - p; q >= 0; --q)
      if (p + q <= n) in = fmaf(in, y, c[tri9(p, q)]);
    f = fmaf(f, x, in);
  }
  return f;
}

// Value and partial derivatives (compile-time order), for the backward pass.
template <int N>
__device__ __forceinline__ void sip_f32_grad(const float *__restrict__ c, float x, float y,
                                             float &f, float &fx, float &fy) {
  f = 0.0f;
  fx = 0.0f;
  fy = 0.0f;
  if constexpr (N > 0) {
#pragma unroll
    for (int p = N; p >= 0; --p) {
      float in = c[tri9(p, N - p)];
      float din = 0.0f;
#pragma unroll
      for (int q = N - p - 1; q >= 0; --q) {
        din = fmaf(din, y, in);
        in = fmaf(in, y, c[tri9(p, q)]);
      }
      if (p == N) {
        f = in;
        fy = din;
      } else {
        fx = fmaf(fx, x, f);
        f = fmaf(f, x, in);
        fy = fmaf(fy, x, din);
      }
    }
  }
}

// Value and partial derivatives with a run-time order (unrolled as above).
__device__ __forceinline__ void sip_f32_grad_rt(const float *__restrict__ c, int n, float x,
                                                float y, float &f, float &fx, float &fy) {
  f = 0.0f;
  fx = 0.0f;
  fy = 0.0f;
  if (n <= 0) return;
#pragma unroll
  for (int p = kMaxOrder; p >= 0; --p) {
    if (p > n) continue;
    float in = 0.0f, din = 0.0f;
#pragma unroll
    for (int q = kMaxOrder - p; q >= 0; --q) {
      if (p + q > n) continue;
      din = fmaf(din, y, in);
      in = fmaf(in, y, c[tri9(p, q)]);
    }
    fx = fmaf(fx, x, f);
    f = fmaf(f, x, in);
    fy = fmaf(fy, x, din);
  }
}

// FP64, run-time order, unrolled (device).
__device__ __forceinline__ double sip_f64_dev(const double *__restrict__ c, int n, double x,
                                              double y) {
  if (n <= 0) return 0.0;
  double f = 0.0;
#pragma unroll
  for (int p = kMaxOrder; p >= 0; --p) {
    if (p > n) continue;
    double in = 0.0;
#pragma unroll
    for (int q = kMaxOrder - p; q >= 0; --q)
      if (p + q <= n) in = fma(in, y, c[tri9(p, q)]);
    f = fma(f, x, in);
  }
  return f;
}

// Host: loops (used by the FP64 set-up on the host).
__host__ __device__ __forceinline__ double sip_f64(const double *__restrict__ c, int n, double x, double y) {
  if (n <= 0) return 0.0;
  double f = 0.0;
  for (int p = n; p >= 0; --p) {
    double in = c[tri9(p, n - p)];
    for (int q = n - p - 1; q >= 0; --q) in = __builtin_fma(in, y, c[tri9(p, q)]);
    f = (p == n) ? in : __builtin_fma(f, x, in);
  }
  return f;
}

// FP64 Horner with a compile-time order (N < 0: run-time order n).
template <int N>
__device__ __forceinline__ double sip_f64_ct(const double *__restrict__ c, int n, double x,
                                             double y) {
  if constexpr (N < 0) {
    return sip_f64_dev(c, n, x, y);
  } else if constexpr (N == 0) {
    return 0.0;
  } else {
    double f = 0.0;
#pragma unroll
    for (int p = N; p >= 0; --p) {
      double in = c[tri9(p, N - p)];
#pragma unroll
      for (int q = N - p - 1; q >= 0; --q) in = fma(in, y, c[tri9(p, q)]);
      f = (p == N) ? in : fma(f, x, in);
    }
    return f;
  }
}

// ----------------------------------------------------------- positions --

// Source position of target pixel (x, y) entirely in FP64 (no anchor).
__host__ __device__ __forceinline__ bool position_f64(const FramePlan &P, double x, double y, double &xs,
                                             double &ys) {
  double u = x - P.tcr[0], v = y - P.tcr[1];
  if (P.t_order > 0) {
    double du = sip_f64(P.tA, P.t_order, u, v);
    double dv = sip_f64(P.tB, P.t_order, u, v);
    u += du;
    v += dv;
  }
  double p = __builtin_fma(P.H[0], u, __builtin_fma(P.H[1], v, P.H[2]));
  double q = __builtin_fma(P.H[3], u, __builtin_fma(P.H[4], v, P.H[5]));
  double w = __builtin_fma(P.H[6], u, __builtin_fma(P.H[7], v, P.H[8]));
  if (!(w > 0.0)) return false;
  double iw = 1.0 / w;
  double U = p * iw, V = q * iw;
  if (P.s_order > 0) {
    double dU = sip_f64(P.sA, P.s_order, U, V);
    double dV = sip_f64(P.sB, P.s_order, U, V);
    U += dU;
    V += dV;
  }
  xs = U + P.scr[0];
  ys = V + P.scr[1];
  return __builtin_isfinite(xs) && __builtin_isfinite(ys);
}

// position_f64 with the source SIP order known at compile time (when SORD
// >= 0; the padded coefficients make it equal to the run-time version);
// the target SIP is compiled in only when TSIP.
template <int SORD, bool TSIP>
__device__ __forceinline__ bool position_f64_ct(const FramePlan &P, double x, double y,
                                                double &xs, double &ys) {
  double u = x - P.tcr[0], v = y - P.tcr[1];
  if (TSIP && P.t_order > 0) {
    double du = sip_f64_dev(P.tA, P.t_order, u, v);
    double dv = sip_f64_dev(P.tB, P.t_order, u, v);
    u += du;
    v += dv;
  }
  double p = fma(P.H[0], u, fma(P.H[1], v, P.H[2]));
  double q = fma(P.H[3], u, fma(P.H[4], v, P.H[5]));
  double w = fma(P.H[6], u, fma(P.H[7], v, P.H[8]));
  if (!(w > 0.0)) return false;
  double iw = 1.0 / w;
  double U = p * iw, V = q * iw;
  double dU = sip_f64_ct<SORD>(P.sA, P.s_order, U, V);
  double dV = sip_f64_ct<SORD>(P.sB, P.s_order, U, V);
  xs = U + dU + P.scr[0];
  ys = V + dV + P.scr[1];
  return isfinite(xs) && isfinite(ys);
}

// Reach box of a frame in cell units, encoded so that all zeros means
// "empty": {max(kReachBig - cx), max(cx + 1), max(kReachBig - cy), max(cy + 1)}
// over the cells that may reach the source.
constexpr int32_t kReachBig = 1 << 24;

constexpr double kFar = 268435456.0;  // 2^28: anchors beyond this are out of any image

// Sum over the terms of order >= 2 of |c| (p+q)(p+q-1) R^(p+q-2): bounds
// every second partial derivative of the polynomial on [-R, R]^2.
template <int SORD>
__device__ __forceinline__ float sip_hess_bound(const float *__restrict__ c, int n, float R) {
  constexpr int N = SORD >= 0 ? SORD : kMaxOrder;
  float b = 0.0f;
#pragma unroll
  for (int p = 0; p <= N; ++p)
#pragma unroll
    for (int q = 0; p + q <= N; ++q) {
      const int m = p + q;
      if (m < 2 || (SORD < 0 && m > n)) continue;
      float rp = 1.0f;
#pragma unroll
      for (int i = 0; i < m - 2; ++i) rp *= R;
      b = fmaf(fabsf(c[tri9(p, q)]) * (float)(m * (m - 1)), rp, b);
    }
  return b;
}

// FP64 evaluation at the anchor pixel (xa, ya) of a cell.  `support` is how
// far interpolation taps reach beyond the position (0, 1 or 2 px).  SORD is
// the source SIP order when known at compile time (< 0: read at run time);
// TSIP compiles in the target SIP (kernels without it require t_order 0).
template <int SORD, bool TSIP>
__device__ __forceinline__ void compute_anchor(const FramePlan &P, int xa, int ya, int support,
                                               Anchor &A) {
  double u = (double)xa - P.tcr[0], v = (double)ya - P.tcr[1];
  A.tus = 0.0f;
  A.tvs = 0.0f;
  A.ta0 = 0.0f;
  A.tb0 = 0.0f;
  if (TSIP && P.t_order > 0) {
    A.tus = (float)(u * P.t_inv_scale);
    A.tvs = (float)(v * P.t_inv_scale);
    A.ta0 = sip_f32_rt(P.ftA, P.t_order, A.tus, A.tvs);
    A.tb0 = sip_f32_rt(P.ftB, P.t_order, A.tus, A.tvs);
    double du = sip_f64_dev(P.tA, P.t_order, u, v);
    double dv = sip_f64_dev(P.tB, P.t_order, u, v);
    u += du;
    v += dv;
  }
  A.tu0 = (float)u;
  A.tv0 = (float)v;
  const double *H = P.H;
  double p = fma(H[0], u, fma(H[1], v, H[2]));
  double q = fma(H[3], u, fma(H[4], v, H[5]));
  double w = fma(H[6], u, fma(H[7], v, H[8]));
  double iw = 1.0 / w;
  double U0 = p * iw, V0 = q * iw;
  A.g1 = (float)((H[0] - U0 * H[6]) * iw);
  A.g2 = (float)((H[1] - U0 * H[7]) * iw);
  A.f1 = (float)((H[3] - V0 * H[6]) * iw);
  A.f2 = (float)((H[4] - V0 * H[7]) * iw);
  A.k1 = (float)(H[6] * iw);
  A.k2 = (float)(H[7] * iw);
  A.sgn = w > 0.0 ? 1.0f : -1.0f;
  A.inv_w0 = (float)iw;
  A.u0s = (float)(U0 * P.s_inv_scale);
  A.v0s = (float)(V0 * P.s_inv_scale);
  double X0 = U0 + P.scr[0], Y0 = V0 + P.scr[1];
  bool finite = isfinite(X0) && isfinite(Y0) && w != 0.0;
  if (!finite || fabs(X0) > kFar || fabs(Y0) > kFar) {
    // the whole cell is (numerically) at infinity: nothing of it is covered
    A.bx = 0;
    A.by = 0;
    A.c0x = 0.0f;
    A.c0y = 0.0f;
    A.sgn = 0.0f;  // sgn * den > 0 never holds: every pixel is invalid
    A.touch = 0;
    A.ok = 0;
    return;
  }
  double fx = floor(X0), fy = floor(Y0);
  A.bx = (int32_t)fx;
  A.by = (int32_t)fy;
  A.c0x = (float)(X0 - fx);
  A.c0y = (float)(Y0 - fy);
  // Can any pixel of the cell reach the source?  The cell spans at most
  // 15 px per axis; its image lies within (|g1|+|g2|, |f1|+|f2|) * 15 of the
  // anchor's, grown by the projective denominator and by the source SIP
  // (bounded by a generous factor 2), plus the tap support and 8 px.
  // The SIP displacement and its slope at the anchor (only roughly needed):
  // with slope L, the cell's source image lies within (1 + 2L) times the
  // affine reach of the anchor while the slope stays below 1/2 over it.
  float fa, fau, fav, fb, fbu, fbv;
  if constexpr (SORD >= 0) {
    sip_f32_grad<SORD>(P.fsA, A.u0s, A.v0s, fa, fau, fav);
    sip_f32_grad<SORD>(P.fsB, A.u0s, A.v0s, fb, fbu, fbv);
  } else {
    sip_f32_grad_rt(P.fsA, P.s_order, A.u0s, A.v0s, fa, fau, fav);
    sip_f32_grad_rt(P.fsB, P.s_order, A.u0s, A.v0s, fb, fbu, fbv);
  }
  double L = (fabs((double)fau) + fabs((double)fav) + fabs((double)fbu) + fabs((double)fbv)) *
             P.s_inv_scale;
  double xs = X0 + (double)fa, ys = Y0 + (double)fb;
  // linear model of the cell's source positions (used to size the LDS box)
  {
    const float s_ = (float)P.s_inv_scale;
    const float apu = fau * s_, apv = fav * s_, bpu = fbu * s_, bpv = fbv * s_;
    A.jx[0] = (1.0f + apu) * A.g1 + apv * A.f1;
    A.jx[1] = (1.0f + apu) * A.g2 + apv * A.f2;
    A.jy[0] = bpu * A.g1 + (1.0f + bpv) * A.f1;
    A.jy[1] = bpu * A.g2 + (1.0f + bpv) * A.f2;
    A.sx0 = A.c0x + fa;
    A.sy0 = A.c0y + fb;
    // Rigorous distance of the cell's positions from that linear model:
    //  - projective denominator: |dU - g.d| <= |g.d| kap / (1 - kap),
    //    kap = max |k.d| over the cell;
    //  - SIP: second-order Taylor remainder, 1/2 B (|dU| + |dV|)^2 with B a
    //    bound on the second derivatives over the cell (scaled units);
    //  - 0.05 px for FP32 rounding of positions and of this bound.
    const float span = (float)(kCell - 1);
    const float kap = (fabsf(A.k1) + fabsf(A.k2)) * span;
    if (kap < 0.5f) {
      const float gu = (fabsf(A.g1) + fabsf(A.g2)) * span, gv = (fabsf(A.f1) + fabsf(A.f2)) * span;
      const float du_max = gu / (1.0f - kap), dv_max = gv / (1.0f - kap);
      const float eu = gu * kap / (1.0f - kap), ev = gv * kap / (1.0f - kap);
      const float R = fmaxf(fabsf(A.u0s), fabsf(A.v0s)) + (du_max + dv_max) * s_;
      const float d2 = (du_max + dv_max) * s_;
      const float r2a = 0.5f * sip_hess_bound<SORD>(P.fsA, P.s_order, R) * d2 * d2;
      const float r2b = 0.5f * sip_hess_bound<SORD>(P.fsB, P.s_order, R) * d2 * d2;
      A.ex = (1.0f + fabsf(apu)) * eu + fabsf(apv) * ev + r2a + 0.05f;
      A.ey = fabsf(bpu) * eu + (1.0f + fabsf(bpv)) * ev + r2b + 0.05f;
    } else {
      A.ex = 1.0e30f;
      A.ey = 1.0e30f;
    }
  }
  double kk = (fabs(H[6]) + fabs(H[7])) * fabs(iw) * 2.0 * kCell;
  // w > 0 at the anchor and |k . d| < 1/4 over the cell: w > 0 at every pixel
  A.ok = (w > 0.0 && kk < 0.5) ? 1 : 0;
  double mx = 2.0 * kCell * (fabs((double)A.g1) + fabs((double)A.g2)) * (1.0 + 2.0 * L) + 8.0 + support;
  double my = 2.0 * kCell * (fabs((double)A.f1) + fabs((double)A.f2)) * (1.0 + 2.0 * L) + 8.0 + support;
  bool outside = (xs < -mx) || (xs > (double)(P.src_w - 1) + mx) || (ys < -my) ||
                 (ys > (double)(P.src_h - 1) + my);
  // none can when the cell maps outside the source, or when w < 0 at the
  // anchor and, with kk < 1/2, everywhere in the cell (every direction is
  // behind the source tangent plane: no pixel has a position)
  const bool away = (w > 0.0 && kk < 0.5 && L < 0.25 && outside) || (w < 0.0 && kk < 0.5);
  A.touch = (away && P.t_order == 0) ? 0 : 1;
  if (P.src_h <= 0 || P.src_w <= 0) A.touch = 0;
}

// ------------------------------------------------------ wave reductions --

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = min(v, __shfl_xor(v, m, 64));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = max(v, __shfl_xor(v, m, 64));
  return v;
}
__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = fmaxf(v, __shfl_xor(v, m, 64));
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Sum over the wave, returned uniform: an inclusive scan within each row of
// 16 lanes (DPP row_shr 1, 2, 4, 8), then the row totals carried across the
// rows (DPP row_bcast 15 and 31), so lane 63 holds the total.  Plain VALU
// instructions (a shuffle tree would go through the LDS crossbar), in a
// fixed order.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float v) {
  const int s = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xf, false);
  return v + __builtin_bit_cast(float, s);
}
__device__ __forceinline__ float wave_sum_dpp(float v) {
  v = dpp_add<0x111, 0xf>(v);  // row_shr:1
  v = dpp_add<0x112, 0xf>(v);  // row_shr:2
  v = dpp_add<0x114, 0xf>(v);  // row_shr:4
  v = dpp_add<0x118, 0xf>(v);  // row_shr:8
  v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

// LDS row stride for a staged box of width bw: bw rounded up to 1 mod 4, so
// the 4 rows x 16 runs of 4 pixels a wave touches at once fall in distinct
// banks (rows shift the bank by 1, 2, 3 instead of a multiple of 4).
__host__ __device__ __forceinline__ int lds_pitch(int bw) { return bw + ((1 - bw) & 3); }

// Every image and table pointer the library hands a kernel is in global
// memory.  The compiler knows that for pointers passed as kernel arguments,
// not for pointers read from a frame table in memory, whose accesses it then
// emits as flat accesses (64-bit VGPR addresses, waits on both counters);
// this restores the address space.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *global_ptr(T *p) {
  return (__attribute__((address_space(1))) T *)p;
}

// Work-group index -> tile index, so that the ~n/8 consecutive (spatially
// adjacent) tiles land on the same XCD: work-groups are dealt round-robin
// over the 8 XCDs, each with its own L2, and neighbouring tiles share
// source halo rows.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  int per = n >> 3, rem = n & 7;
  int x = b & 7, k = b >> 3;
  return (x < rem) ? x * (per + 1) + k : rem * (per + 1) + (x - rem) * per + k;
}

// Keys cubic-convolution weights for taps i0-1 .. i0+2 at fraction t.
__device__ __forceinline__ void keys_weights(float t, float a, float w[4]) {
  float s = 1.0f - t;
  w[0] = a * t * s * s;                                  // W(1 + t) = a t (t-1)^2
  w[1] = fmaf(fmaf(a + 2.0f, t, -(a + 3.0f)), t * t, 1.0f);  // W(t)
  w[2] = fmaf(fmaf(a + 2.0f, s, -(a + 3.0f)), s * s, 1.0f);  // W(1 - t)
  w[3] = a * t * t * s;                                  // W(2 - t) = a t^2 (1-t)
}

// d/dx of the Keys weights (x = position, t its fraction).
__device__ __forceinline__ void keys_dweights(float t, float a, float d[4]) {
  float s = 1.0f - t;
  d[0] = a * s * (s - 2.0f * t);                              // d/dt [a t s^2]
  d[1] = t * fmaf(3.0f * (a + 2.0f), t, -2.0f * (a + 3.0f));  // W'(t)
  d[2] = -s * fmaf(3.0f * (a + 2.0f), s, -2.0f * (a + 3.0f)); // -W'(s)
  d[3] = a * t * (2.0f * s - t);                              // d/dt [a t^2 s]
}

}  // namespace dfr
