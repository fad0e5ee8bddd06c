// Certified local models of the position map (forward path, target
// without SIP).
//
// For a 32x32 cell of output pixels with centre (xc, yc), the source
// position of pixel (xc + a, yc + b), |a|, |b| <= 15.5, is written as
//     X = bx + sum_{i+j<=3} mx[a^i b^j] a^i b^j   (and Y likewise)
// plus a remainder bounded rigorously over the whole cell.  The model comes
// from Taylor-model arithmetic in FP64 (a degree-3 polynomial in (a, b) and
// an interval for everything it leaves out) applied to the two stages of
// section 3.2 in their composed form:
//   1. the projective step: dU = (g.d) / (1 + e), e = k.d linear in (a, b);
//      1/(1 + e) = 1 - e + e^2 - e^3 + e^4/(1 + e), |e| <= kap < 1/4;
//   2. the source SIP AP/BP re-expanded about the cell centre's (U, V)
//      (Taylor shift of the polynomial: exact up to rounding) and composed
//      with (dU, dV); terms of degree >= 4 in (dU, dV) go to the remainder.
// A cell is certified when the remainder is below kModelTol; the bound it
// reports adds the FP32 rounding of the stored coefficients.  Certification
// also proves the projective denominator positive over the cell (every
// pixel valid).
#pragma once

#include "common.hpp"

namespace dfr {

constexpr double kHalfCell = 0.5 * (kCell - 1);  // 15.5: |a|, |b| over a cell
constexpr double kModelTol = 1.0e-6;             // px: accepted model error
constexpr double kModelSlack = 1.0e-3;           // px: FP32 evaluation margin in box bounds

// Per-cell model (device table, 112 bytes).  Coefficient k of mx/my
// multiplies a^cm_i(k) b^cm_j(k); the layout groups powers of a so a row of
// pixels (fixed b) reduces to a cubic in a.
struct alignas(16) CellModel {
  float mx[10], my[10];  // source position minus (bx, by)
  float ex, ey;          // bound on |position - (constant + linear part)| over the cell
  int32_t bx, by;        // integer part of the source position at the cell centre
  float err;             // certified bound on |model - map| over the cell (px)
  int32_t certified;     // 1: truncation <= kModelTol and every pixel has a valid position
  float tie;             // nearest: FP32 positions this close to a rounding tie are decided in FP64
  int32_t pad_;
};
static_assert(sizeof(CellModel) == 112, "CellModel layout");

__host__ __device__ constexpr int cm_i(int k) { return k < 4 ? 0 : (k < 7 ? 1 : (k < 9 ? 2 : 3)); }
__host__ __device__ constexpr int cm_j(int k) { return k < 4 ? k : (k < 7 ? k - 4 : (k < 9 ? k - 7 : 0)); }
__host__ __device__ constexpr int cm_idx(int i, int j) {
  return i == 0 ? j : (i == 1 ? 4 + j : (i == 2 ? 7 + j : 9));
}

// Taylor model: degree-3 polynomial in (a, b) plus a bound r on the rest.
struct Tm3 {
  double c[10];
  double r;
};

__host__ __device__ inline void tm_zero(Tm3 &t) {
#pragma unroll
  for (int k = 0; k < 10; ++k) t.c[k] = 0.0;
  t.r = 0.0;
}

// Sum of |c| h^d over the terms of each degree d.
__host__ __device__ inline void tm_norms(const Tm3 &t, double n[4]) {
  const double h = kHalfCell;
  const double hp[4] = {1.0, h, h * h, h * h * h};
#pragma unroll
  for (int d = 0; d < 4; ++d) n[d] = 0.0;
#pragma unroll
  for (int k = 0; k < 10; ++k) n[cm_i(k) + cm_j(k)] += __builtin_fabs(t.c[k]) * hp[cm_i(k) + cm_j(k)];
}

// Bound on |t| over the cell.
__host__ __device__ inline double tm_bound(const Tm3 &t) {
  double n[4];
  tm_norms(t, n);
  return n[0] + n[1] + n[2] + n[3] + t.r;
}

// z = x * y: product terms of degree <= 3 kept, the others bounded.
__host__ __device__ inline void tm_mul(const Tm3 &x, const Tm3 &y, Tm3 &z) {
#pragma unroll
  for (int k = 0; k < 10; ++k) z.c[k] = 0.0;
#pragma unroll
  for (int kx = 0; kx < 10; ++kx)
#pragma unroll
    for (int ky = 0; ky < 10; ++ky) {
      const int i = cm_i(kx) + cm_i(ky), j = cm_j(kx) + cm_j(ky);
      if (i + j <= 3) z.c[cm_idx(i, j)] = __builtin_fma(x.c[kx], y.c[ky], z.c[cm_idx(i, j)]);
    }
  double nx[4], ny[4];
  tm_norms(x, nx);
  tm_norms(y, ny);
  double drop = 0.0;
#pragma unroll
  for (int d1 = 0; d1 < 4; ++d1)
#pragma unroll
    for (int d2 = 0; d2 < 4; ++d2)
      if (d1 + d2 >= 4) drop += nx[d1] * ny[d2];
  const double bx = nx[0] + nx[1] + nx[2] + nx[3], by = ny[0] + ny[1] + ny[2] + ny[3];
  z.r = drop + bx * y.r + by * x.r + x.r * y.r;
}

// z += s * x
__host__ __device__ inline void tm_axpy(double s, const Tm3 &x, Tm3 &z) {
#pragma unroll
  for (int k = 0; k < 10; ++k) z.c[k] = __builtin_fma(s, x.c[k], z.c[k]);
  z.r += __builtin_fabs(s) * x.r;
}

// Taylor coefficients of the SIP polynomial c (packed by tri9, order <= N,
// zero past its order) about (U0, V0): t[tri9(i, j)] multiplies dU^i dV^j.
// Repeated synthetic division along U for every power of V, then along V.
template <int N>
__host__ __device__ inline void sip_taylor(const double *__restrict__ c, double U0, double V0,
                                           double t[kMaxCoef]) {
#pragma unroll
  for (int k = 0; k < kMaxCoef; ++k) t[k] = 0.0;
#pragma unroll
  for (int p = 0; p <= N; ++p)
#pragma unroll
    for (int q = 0; p + q <= N; ++q) t[tri9(p, q)] = c[tri9(p, q)];
#pragma unroll
  for (int q = 0; q <= N; ++q) {
    const int m = N - q;
#pragma unroll
    for (int k = 0; k < m; ++k)
#pragma unroll
      for (int p = m - 1; p >= k; --p) t[tri9(p, q)] = __builtin_fma(U0, t[tri9(p + 1, q)], t[tri9(p, q)]);
  }
#pragma unroll
  for (int p = 0; p <= N; ++p) {
    const int m = N - p;
#pragma unroll
    for (int k = 0; k < m; ++k)
#pragma unroll
      for (int q = m - 1; q >= k; --q) t[tri9(p, q)] = __builtin_fma(V0, t[tri9(p, q + 1)], t[tri9(p, q)]);
  }
}

// Position model of cell (cx, cy) of the output grid.  SORD: source SIP
// order at compile time (< 0: any order up to kMaxOrder; the padded
// coefficients make both give the same model).
template <int SORD>
__host__ __device__ inline void cell_model(const FramePlan &P, int cx, int cy, CellModel &M) {
  constexpr int N = SORD >= 0 ? SORD : kMaxOrder;
  const double h = kHalfCell;
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    M.mx[k] = 0.0f;
    M.my[k] = 0.0f;
  }
  M.ex = M.ey = 0.0f;
  M.bx = M.by = 0;
  M.err = 1.0e30f;
  M.certified = 0;
  M.tie = 0.5f;
  M.pad_ = 0;
  if (P.t_order > 0) return;  // the target SIP is not modelled

  const double uc = (double)cx * kCell + h - P.tcr[0], vc = (double)cy * kCell + h - P.tcr[1];
  const double *H = P.H;
  const double pc = __builtin_fma(H[0], uc, __builtin_fma(H[1], vc, H[2]));
  const double qc = __builtin_fma(H[3], uc, __builtin_fma(H[4], vc, H[5]));
  const double wc = __builtin_fma(H[6], uc, __builtin_fma(H[7], vc, H[8]));
  if (!(wc > 0.0)) return;
  const double iw = 1.0 / wc;
  const double Uc = pc * iw, Vc = qc * iw;
  const double g1 = (H[0] - Uc * H[6]) * iw, g2 = (H[1] - Uc * H[7]) * iw;
  const double f1 = (H[3] - Vc * H[6]) * iw, f2 = (H[4] - Vc * H[7]) * iw;
  const double k1 = H[6] * iw, k2 = H[7] * iw;
  const double kap = (__builtin_fabs(k1) + __builtin_fabs(k2)) * h;
  if (!(kap < 0.25)) return;

  // 1 / (1 + e) as a Taylor model
  Tm3 eps, e2, e3, rho;
  tm_zero(eps);
  eps.c[cm_idx(1, 0)] = k1;
  eps.c[cm_idx(0, 1)] = k2;
  tm_mul(eps, eps, e2);
  tm_mul(e2, eps, e3);
#pragma unroll
  for (int k = 0; k < 10; ++k) rho.c[k] = e2.c[k] - eps.c[k] - e3.c[k];
  rho.c[0] += 1.0;
  rho.r = kap * kap * kap * kap / (1.0 - kap);

  Tm3 gd, fd, al, be;
  tm_zero(gd);
  tm_zero(fd);
  gd.c[cm_idx(1, 0)] = g1;
  gd.c[cm_idx(0, 1)] = g2;
  fd.c[cm_idx(1, 0)] = f1;
  fd.c[cm_idx(0, 1)] = f2;
  tm_mul(gd, rho, al);  // dU
  tm_mul(fd, rho, be);  // dV

  Tm3 X = al, Y = be;
  double sa0 = 0.0, sb0 = 0.0;
  if (N > 0 && P.s_order > 0) {
    double ta[kMaxCoef], tb[kMaxCoef];
    sip_taylor<N>(P.sA, Uc, Vc, ta);
    sip_taylor<N>(P.sB, Uc, Vc, tb);
    sa0 = ta[0];
    sb0 = tb[0];
    // degree 1..3 in (dU, dV): Taylor-model powers of al, be
    tm_axpy(ta[tri9(1, 0)], al, X);
    tm_axpy(ta[tri9(0, 1)], be, X);
    tm_axpy(tb[tri9(1, 0)], al, Y);
    tm_axpy(tb[tri9(0, 1)], be, Y);
    if (N >= 2) {
      Tm3 p2[3];  // al^2, al be, be^2
      tm_mul(al, al, p2[0]);
      tm_mul(al, be, p2[1]);
      tm_mul(be, be, p2[2]);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        tm_axpy(ta[tri9(2 - i, i)], p2[i], X);
        tm_axpy(tb[tri9(2 - i, i)], p2[i], Y);
      }
      if (N >= 3) {
        Tm3 p3;  // al^(3-i) be^i
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (i == 0)
            tm_mul(p2[0], al, p3);
          else
            tm_mul(p2[i - 1], be, p3);
          tm_axpy(ta[tri9(3 - i, i)], p3, X);
          tm_axpy(tb[tri9(3 - i, i)], p3, Y);
        }
      }
    }
    // degree >= 4 in (dU, dV): bounded term by term
    const double A = tm_bound(al), B = tm_bound(be);
    double apow[N + 1], bpow[N + 1];
    apow[0] = bpow[0] = 1.0;
#pragma unroll
    for (int i = 1; i <= N; ++i) {
      apow[i] = apow[i - 1] * A;
      bpow[i] = bpow[i - 1] * B;
    }
#pragma unroll
    for (int i = 0; i <= N; ++i)
#pragma unroll
      for (int j = 0; i + j <= N; ++j)
        if (i + j >= 4) {
          X.r += __builtin_fabs(ta[tri9(i, j)]) * apow[i] * bpow[j];
          Y.r += __builtin_fabs(tb[tri9(i, j)]) * apow[i] * bpow[j];
        }
  }

  const double X0 = Uc + sa0 + P.scr[0], Y0 = Vc + sb0 + P.scr[1];
  if (!(__builtin_fabs(X0) < kFar) || !(__builtin_fabs(Y0) < kFar)) return;  // also rejects NaN
  const double fx = __builtin_floor(X0), fy = __builtin_floor(Y0);
  M.bx = (int32_t)fx;
  M.by = (int32_t)fy;
  // constant terms of al, be are zero: the constant is the centre's position
  X.c[0] = X0 - fx;
  Y.c[0] = Y0 - fy;
  double rx = 0.0, ry = 0.0, nlx = 0.0, nly = 0.0;
  const double hp[4] = {1.0, h, h * h, h * h * h};
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    M.mx[k] = (float)X.c[k];
    M.my[k] = (float)Y.c[k];
    const double hd = hp[cm_i(k) + cm_j(k)];
    rx += __builtin_fabs((double)M.mx[k] - X.c[k]) * hd;
    ry += __builtin_fabs((double)M.my[k] - Y.c[k]) * hd;
    if (cm_i(k) + cm_j(k) >= 2) {
      nlx += __builtin_fabs((double)M.mx[k]) * hd;
      nly += __builtin_fabs((double)M.my[k]) * hd;
    }
  }
  // FP64 rounding of this construction, generously
  const double slack = 1.0e-12 * (1.0 + __builtin_fabs(Uc) + __builtin_fabs(Vc) + tm_bound(al) + tm_bound(be));
  const double tx = X.r + slack, ty = Y.r + slack;  // truncation of the map
  const double errx = tx + rx, erry = ty + ry;       // plus FP32 rounding of the coefficients
  const double err = __builtin_fmax(errx, erry);
  if (!(err < 1.0e6)) return;
  M.err = (float)(err * (1.0 + 1.0e-6));
  // The FP32 evaluation of the stored cubic (Horner's rule with fused
  // multiply-adds in b, then in a) is within gamma_6 * S of the cubic's exact
  // value, S = sum_k |m_k| h^(i+j) (the Horner bound gamma_n sum |c_j| |x|^j
  // for each level, composed), so an FP32 position is within
  // E = err + gamma_6 * S of the map; nearest decides the pixels within 2E of
  // a rounding tie in FP64.
  {
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int k = 0; k < 10; ++k) {
      const double hd = hp[cm_i(k) + cm_j(k)];
      sx += __builtin_fabs((double)M.mx[k]) * hd;
      sy += __builtin_fabs((double)M.my[k]) * hd;
    }
    const double u = 0x1p-24, g6 = 6.0 * u / (1.0 - 6.0 * u);
    const double t = 2.0 * (err + g6 * __builtin_fmax(sx, sy)) * (1.0 + 1.0e-6);
    M.tie = (float)__builtin_fmin(0.5, __builtin_fmax(t, 1.0e-6));  // >= 1e-6: 0.5f - tie rounds by < 3e-8
  }
  M.ex = (float)((nlx + errx + kModelSlack) * (1.0 + 1.0e-6));
  M.ey = (float)((nly + erry + kModelSlack) * (1.0 + 1.0e-6));
  // the coefficient rounding is the FP32 evaluation error every FP32 path has
  // (the anchored chain rounds its own coefficients alike); the tolerance
  // applies to what the cubic leaves out of the map
  M.certified = __builtin_fmax(tx, ty) <= kModelTol ? 1 : 0;
}

}  // namespace dfr
