// Per-pixel building blocks of the reprojection kernels (paper section 3.1:
// source positions by the two stages of section 3.2, interpolation,
// footprint normalisation): the FP32 position chain from a cell's FP64
// anchor, tap origins and interpolation weights, evaluation of a cell's
// cubic position model, streaming row stores and the FP64 rounding decision
// of nearest.  The forward tile body (forward_tile.hpp) and the backward
// kernel (backward.hip) are composed from them.
#pragma once

#include "cell_model.hpp"
#include "common.hpp"

namespace dfr {

constexpr int kRtOrder = -1;  // SORD value meaning "order read at run time"

template <int SORD>
__device__ __forceinline__ float sip_src(const float *__restrict__ c, int n, float x, float y) {
  if constexpr (SORD == kRtOrder) {
    return sip_f32_rt(c, n, x, y);
  } else {
    return sip_f32<SORD>(c, x, y);
  }
}

// Offsets of one pixel from its anchor, in FP32.
struct PixelGeom {
  float du, dv;   // SIP-corrected target offset from the anchor
  float r;        // 1 / (1 + k.d): ratio w_anchor / w_pixel
  float dU, dV;   // source intermediate offset from the anchor
  float us, vs;   // source intermediate / S_s (SIP arguments)
};

// The projective part of a pixel's position from its cell's anchor: the
// SIP-corrected target offset, the source intermediate offset and the SIP
// arguments (everything but the source SIP itself); `den` is 1 + k.d, whose
// sign against the anchor's tells whether the direction is in front of the
// source tangent plane.  TSIP compiles in the target SIP.
template <bool TSIP>
__device__ __forceinline__ void pixel_geom(const FramePlan &P, const Anchor &A, float tinv,
                                           float sinv, float dx, float dy, PixelGeom &g,
                                           float &den) {
  float du = dx, dv = dy;
  if (TSIP && P.t_order > 0) {
    float us = fmaf(dx, tinv, A.tus), vs = fmaf(dy, tinv, A.tvs);
    du = dx + (sip_f32_rt(P.ftA, P.t_order, us, vs) - A.ta0);
    dv = dy + (sip_f32_rt(P.ftB, P.t_order, us, vs) - A.tb0);
  }
  float nu = fmaf(A.g1, du, A.g2 * dv);
  float nv = fmaf(A.f1, du, A.f2 * dv);
  float r;
  if (P.series) {
    // |e| < 1e-3: 1/(1+e) = 1 - e + e^2 to a relative 1e-9
    const float e = fmaf(A.k1, du, A.k2 * dv);
    den = 1.0f + e;
    r = fmaf(e, e - 1.0f, 1.0f);
  } else {
    den = fmaf(A.k1, du, fmaf(A.k2, dv, 1.0f));
    r = __builtin_amdgcn_rcpf(den);
  }
  g.du = du;
  g.dv = dv;
  g.r = r;
  g.dU = nu * r;
  g.dV = nv * r;
  g.us = fmaf(g.dU, sinv, A.u0s);
  g.vs = fmaf(g.dV, sinv, A.v0s);
}

// FP32 source position of the pixel at offset (dx, dy) from its anchor,
// relative to (A.bx, A.by).  Returns false for directions on or behind the
// source tangent plane.
template <int SORD, bool TSIP>
__device__ __forceinline__ bool pixel_position(const FramePlan &P, const Anchor &A, float tinv,
                                               float sinv, float dx, float dy, float &rx,
                                               float &ry, PixelGeom *geom = nullptr) {
  PixelGeom g;
  float den;
  pixel_geom<TSIP>(P, A, tinv, sinv, dx, dy, g, den);
  float ax = sip_src<SORD>(P.fsA, P.s_order, g.us, g.vs);
  float ay = sip_src<SORD>(P.fsB, P.s_order, g.us, g.vs);
  rx = (A.c0x + g.dU) + ax;
  ry = (A.c0y + g.dV) + ay;
  if (geom) *geom = g;
  return (A.sgn * den > 0.0f) && (fabsf(rx) < 1.0e7f) && (fabsf(ry) < 1.0e7f);
}

template <int INTERP>
struct TapSupport {
  static constexpr int lo = INTERP == DFR_BICUBIC ? 1 : 0;  // taps left/up of floor
  static constexpr int hi = INTERP == DFR_NEAREST ? 0 : (INTERP == DFR_BILINEAR ? 1 : 2);
};

// Output stores are streaming (non-temporal): the output is written once
// and never read back by the kernel, so it should not evict the source
// footprint other tiles still read from L2 and the last-level cache.
__device__ __forceinline__ void store_run(float *__restrict__ base, int64_t off, int x, int out_w,
                                          bool vec, const float v[kRun]) {
  typedef float f4v __attribute__((ext_vector_type(4)));
  auto *g = global_ptr(base) + off;
  if (vec && x + kRun <= out_w) {
    __builtin_nontemporal_store((f4v){v[0], v[1], v[2], v[3]},
                                (__attribute__((address_space(1))) f4v *)g);
  } else {
#pragma unroll
    for (int e = 0; e < kRun; ++e)
      if (x + e < out_w) __builtin_nontemporal_store(v[e], g + e);
  }
}

__device__ __forceinline__ bool vector_stores_ok(const FramePlan &P, const TileGeom &G) {
  return ((G.out_w & (kRun - 1)) == 0) && ((reinterpret_cast<uintptr_t>(P.out) & 15) == 0) &&
         (P.fp == nullptr || (reinterpret_cast<uintptr_t>(P.fp) & 15) == 0);
}

// Nearest: the FP64 rounding decision for a pixel whose FP32 position lies
// within reach of its FP32 error of a tie (rare).  Writes the rounded position relative to
// (bx, by); returns false if the pixel has no source position.
template <int SORD, bool TSIP>
__device__ __forceinline__ bool nearest_exact(const FramePlan &P, int x, int y, int bx,
                                                       int by, float &px, float &py,
                                                       double &xs, double &ys) {
  bool ok = position_f64_ct<SORD, TSIP>(P, (double)x, (double)y, xs, ys) && fabs(xs - bx) < 1.0e7 &&
            fabs(ys - by) < 1.0e7;
  if (ok) {
    px = (float)(rint(xs) - (double)bx);
    py = (float)(rint(ys) - (double)by);
  }
  return ok;
}

// ------------------------------------------------ shared by the forward --
//
// Interpolation, store and position helpers of the forward kernels
// (forward_tile.hpp): the interior formulas below are the ones every path
// uses, so results agree bit for bit wherever all taps are inside.

// Values of one pixel's in-image taps combined the same way on every path
// (so all paths agree bit for bit where all taps are inside the source).
template <int INTERP>
struct Taps;

template <>
struct Taps<DFR_BILINEAR> {
  template <typename Fetch>
  __device__ static __forceinline__ float interior(int i0, int j0, float t, float s, const Fetch &f) {
    float v00 = f(i0, j0), v01 = f(i0 + 1, j0), v10 = f(i0, j0 + 1), v11 = f(i0 + 1, j0 + 1);
    float top = fmaf(t, v01 - v00, v00);
    float bot = fmaf(t, v11 - v10, v10);
    return fmaf(s, bot - top, top);
  }
};

template <>
struct Taps<DFR_BICUBIC> {
  template <typename Fetch>
  __device__ static __forceinline__ float interior(int i0, int j0, const float wx[4],
                                                   const float wy[4], const Fetch &f) {
    float S = 0.0f;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      float row = wx[0] * f(i0, j0 + l);
      row = fmaf(wx[1], f(i0 + 1, j0 + l), row);
      row = fmaf(wx[2], f(i0 + 2, j0 + l), row);
      row = fmaf(wx[3], f(i0 + 3, j0 + l), row);
      S = fmaf(wy[l], row, S);
    }
    return S;
  }
};

// General interpolation: taps outside the source are dropped (zero padding)
// and the value is normalised by the footprint; identical to the interior
// formula where every tap is inside.  `fetch` receives source coordinates.
template <int INTERP, typename Fetch>
__device__ __forceinline__ void interp_general(int i0, int j0, float t, float s, int W, int H,
                                               float a, const Fetch &fetch, float &out,
                                               float &fp) {
  if constexpr (INTERP == DFR_NEAREST) {
    bool in = ((unsigned)i0 < (unsigned)W) && ((unsigned)j0 < (unsigned)H);
    out = in ? fetch(i0, j0) : 0.0f;
    fp = in ? 1.0f : 0.0f;
  } else if constexpr (INTERP == DFR_BILINEAR) {
    bool ix0 = (unsigned)i0 < (unsigned)W, ix1 = (unsigned)(i0 + 1) < (unsigned)W;
    bool iy0 = (unsigned)j0 < (unsigned)H, iy1 = (unsigned)(j0 + 1) < (unsigned)H;
    if (ix0 && ix1 && iy0 && iy1) {
      out = Taps<DFR_BILINEAR>::interior(i0, j0, t, s, fetch);
      fp = 1.0f;
      return;
    }
    float wx0 = ix0 ? 1.0f - t : 0.0f, wx1 = ix1 ? t : 0.0f;
    float wy0 = iy0 ? 1.0f - s : 0.0f, wy1 = iy1 ? s : 0.0f;
    float v00 = (ix0 && iy0) ? fetch(i0, j0) : 0.0f;
    float v01 = (ix1 && iy0) ? fetch(i0 + 1, j0) : 0.0f;
    float v10 = (ix0 && iy1) ? fetch(i0, j0 + 1) : 0.0f;
    float v11 = (ix1 && iy1) ? fetch(i0 + 1, j0 + 1) : 0.0f;
    float S = fmaf(wy0, fmaf(wx0, v00, wx1 * v01), wy1 * fmaf(wx0, v10, wx1 * v11));
    float F = (wx0 + wx1) * (wy0 + wy1);
    out = F > 0.0f ? S * __builtin_amdgcn_rcpf(F) : 0.0f;
    fp = F > 0.0f ? F : 0.0f;
  } else {
    float wx[4], wy[4];
    keys_weights(t, a, wx);
    keys_weights(s, a, wy);
    bool inx[4], iny[4];
    bool all_in = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      inx[k] = (unsigned)(i0 + k) < (unsigned)W;
      iny[k] = (unsigned)(j0 + k) < (unsigned)H;
      all_in = all_in && inx[k] && iny[k];
    }
    if (all_in) {
      out = Taps<DFR_BICUBIC>::interior(i0, j0, wx, wy, fetch);
      fp = 1.0f;
      return;
    }
    float Fx = 0.0f, Fy = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      wx[k] = inx[k] ? wx[k] : 0.0f;
      wy[k] = iny[k] ? wy[k] : 0.0f;
      Fx += wx[k];
      Fy += wy[k];
    }
    float S = 0.0f;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      float row = 0.0f;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        float v = (inx[k] && iny[l]) ? fetch(i0 + k, j0 + l) : 0.0f;
        row = fmaf(wx[k], v, row);
      }
      S = fmaf(wy[l], row, S);
    }
    float F = Fx * Fy;
    out = F > 0.0f ? S * __builtin_amdgcn_rcpf(F) : 0.0f;
    fp = F > 0.0f ? F : 0.0f;
  }
}

// First tap and fractions of a position (relative to an integer base).
template <int INTERP>
__device__ __forceinline__ void tap_origin(float r, int base, int &i0, float &t) {
  if constexpr (INTERP == DFR_NEAREST) {
    i0 = base + (int)rintf(r);
    t = 0.0f;
  } else {
    float f = floorf(r);
    t = r - f;
    i0 = base + (int)f - TapSupport<INTERP>::lo;
  }
}

// A row of a cell model: the cubic in a at fixed b, four coefficients per
// axis (Horner in b, once per row).
struct ModelRow {
  float x0, x1, x2, x3, y0, y1, y2, y3;
};

__device__ __forceinline__ void model_row(const CellModel &M, float b, ModelRow &R) {
  R.x0 = fmaf(fmaf(fmaf(M.mx[3], b, M.mx[2]), b, M.mx[1]), b, M.mx[0]);
  R.x1 = fmaf(fmaf(M.mx[6], b, M.mx[5]), b, M.mx[4]);
  R.x2 = fmaf(M.mx[8], b, M.mx[7]);
  R.x3 = M.mx[9];
  R.y0 = fmaf(fmaf(fmaf(M.my[3], b, M.my[2]), b, M.my[1]), b, M.my[0]);
  R.y1 = fmaf(fmaf(M.my[6], b, M.my[5]), b, M.my[4]);
  R.y2 = fmaf(M.my[8], b, M.my[7]);
  R.y3 = M.my[9];
}

// Source position (relative to the model's base) of the pixel at column
// offset a from the cell centre.
__device__ __forceinline__ void model_at(const ModelRow &R, float a, float &px, float &py) {
  px = fmaf(fmaf(fmaf(R.x3, a, R.x2), a, R.x1), a, R.x0);
  py = fmaf(fmaf(fmaf(R.y3, a, R.y2), a, R.y1), a, R.y0);
}

// The model's position (relative to its base) at offsets (a, b) from the
// cell centre, evaluated in FP64 from the stored coefficients: within
// M.err of the map (the bound covers the coefficients' FP32 rounding), with
// an evaluation error far below that.
__device__ __forceinline__ double model_f64(const float m[10], double a, double b) {
  const double c0 = fma(fma(fma((double)m[3], b, (double)m[2]), b, (double)m[1]), b, (double)m[0]);
  const double c1 = fma(fma((double)m[6], b, (double)m[5]), b, (double)m[4]);
  const double c2 = fma((double)m[8], b, (double)m[7]);
  return fma(fma(fma((double)m[9], a, c2), a, c1), a, c0);
}

// Debug output: the FP64 source position of output pixel (x, y) as the
// kernel used it (NaN where invalid); only for pixels inside the output.
__device__ __forceinline__ void debug_position(const TileGeom &G, int x, int y, bool ok,
                                               bool exact, double dbx, double dby, int bx, int by,
                                               float px, float py) {
  if (y >= G.out_h || x >= G.out_w) return;
  double2 d;
  if (!ok) {
    d.x = __builtin_nan("");
    d.y = d.x;
  } else if (exact) {
    d.x = dbx;
    d.y = dby;
  } else {
    d.x = (double)bx + (double)px;
    d.y = (double)by + (double)py;
  }
  reinterpret_cast<double2 *>(G.debug)[(int64_t)y * G.out_w + x] = d;
}

}  // namespace dfr
