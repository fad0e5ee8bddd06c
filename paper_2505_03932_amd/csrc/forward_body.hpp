// Reprojection of one output tile (paper section 3.1: source positions by
// the two stages of section 3.2, interpolation, footprint normalisation).
//
// A tile is (kRun << txt_log2) x ((kThreads >> txt_log2) * NP) output
// pixels.  Thread (tx, ty) owns NP runs of kRun consecutive pixels in rows
// ty, ty + RP, ..., so every wave store covers contiguous row segments.
//
// Two schedules share the per-pixel position code:
//   * tile_anchors / tile_positions / stage_box (used by the backward
//     kernel): anchors, then positions with the exact bounding box of all
//     in-image taps (wave min/max reductions + LDS atomics), then a
//     synchronous copy of that box into LDS;
//   * forward_tile: anchors and a sampled source box in parallel, the box
//     staged by asynchronous DMA while the positions are computed (see the
//     comment above forward_tile).
#pragma once

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

// FP32 source position of the pixel at offset (dx, dy) from its anchor,
// relative to (A.bx, A.by).  Returns false for directions on or behind the
// source tangent plane.  TSIP compiles in the target SIP.
template <int SORD, bool TSIP>
__device__ __forceinline__ bool pixel_position(const FramePlan &P, const Anchor &A, float tinv,
                                               float sinv, float dx, float dy, float &rx,
                                               float &ry, PixelGeom *geom = nullptr) {
  float du = dx, dv = dy;
  if (TSIP && P.t_order > 0) {
    float us = fmaf(dx, tinv, A.tus), vs = fmaf(dy, tinv, A.tvs);
    du = dx + (sip_f32_rt(P.ftA, P.t_order, us, vs) - A.ta0);
    dv = dy + (sip_f32_rt(P.ftB, P.t_order, us, vs) - A.tb0);
  }
  float nu = fmaf(A.g1, du, A.g2 * dv);
  float nv = fmaf(A.f1, du, A.f2 * dv);
  float den, r;
  if (P.series) {
    // |e| < 1e-3: 1/(1+e) = 1 - e + e^2 to a relative 1e-9
    const float e = fmaf(A.k1, du, A.k2 * dv);
    den = 1.0f + e;
    r = fmaf(e, e - 1.0f, 1.0f);
  } else {
    den = fmaf(A.k1, du, fmaf(A.k2, dv, 1.0f));
    r = __builtin_amdgcn_rcpf(den);
  }
  float dU = nu * r, dV = nv * r;
  float us = fmaf(dU, sinv, A.u0s), vs = fmaf(dV, sinv, A.v0s);
  float ax = sip_src<SORD>(P.fsA, P.s_order, us, vs);
  float ay = sip_src<SORD>(P.fsB, P.s_order, us, vs);
  rx = (A.c0x + dU) + ax;
  ry = (A.c0y + dV) + ay;
  if (geom) {
    geom->du = du;
    geom->dv = dv;
    geom->r = r;
    geom->dU = dU;
    geom->dV = dV;
    geom->us = us;
    geom->vs = vs;
  }
  return (A.sgn * den > 0.0f) && (fabsf(rx) < 1.0e7f) && (fabsf(ry) < 1.0e7f);
}

// LDS scratch of a tile kernel besides the dynamic source tile.
struct TileShared {
  Anchor anchor[kMaxAnchors];
  int box[4];     // imin, imax, jmin, jmax of the source box
  int touch;      // any anchor cell can reach the source
  int item;       // batch: work item handed to this work-group
  int cells_ok;   // forward: every anchor cell has valid positions throughout
  int box_ok;     // forward: the anchors' linear models give a usable box
};

template <int INTERP>
struct TapSupport {
  static constexpr int lo = INTERP == DFR_BICUBIC ? 1 : 0;  // taps left/up of floor
  static constexpr int hi = INTERP == DFR_NEAREST ? 0 : (INTERP == DFR_BILINEAR ? 1 : 2);
};

// Geometry of a tile and of the calling thread inside it.
struct TileCtx {
  int x0, y0;    // tile origin (output pixels)
  int RP;        // rows per pass
  int cx0, cy0;  // first anchor cell
  int ncx;       // anchor cells per tile row
  int ty;        // thread row in the tile
  int xr;        // first output column of the thread's runs
};

// Phase 1.  Returns false when no pixel of the tile can reach the source
// (and skipping is allowed): the caller then only writes "uncovered".
template <int INTERP, int SORD, bool TSIP, int NP>
__device__ __forceinline__ bool tile_anchors(const FramePlan &P, const TileGeom &G, int tile,
                                             TileShared &sh, TileCtx &c) {
  const int tid = threadIdx.x;
  const int lg = G.txt_log2;
  const int TW = kRun << lg;
  c.RP = kThreads >> lg;
  const int TH = c.RP * NP;
  const int trow = tile / G.tiles_x;
  c.x0 = (tile - trow * G.tiles_x) * TW;
  c.y0 = trow * TH;
  c.cx0 = c.x0 / kCell;
  c.ncx = TW / kCell;
  c.cy0 = c.y0 / kCell;
  const int ncy = TH >= kCell ? TH / kCell : 1;
  const int nA = c.ncx * ncy;
  c.ty = tid >> lg;
  c.xr = c.x0 + (tid & ((1 << lg) - 1)) * kRun;
  if (tid < 64) {
    int t = 0;
    if (tid < nA) {
      int cy = c.cy0 + tid / c.ncx, cx = c.cx0 + tid % c.ncx;
      compute_anchor<SORD, TSIP>(P, cx * kCell, cy * kCell, TapSupport<INTERP>::hi, sh.anchor[tid]);
      t = sh.anchor[tid].touch;
    }
    unsigned long long any = __ballot(t != 0);
    if (tid == 0) {
      sh.touch = any != 0ull;
      sh.box[0] = 0x7fffffff;
      sh.box[1] = -0x7fffffff;
      sh.box[2] = 0x7fffffff;
      sh.box[3] = -0x7fffffff;
    }
  }
  __syncthreads();
  return sh.touch || !G.allow_skip;
}

template <int NP>
struct TilePos {
  float rx[NP][kRun], ry[NP][kRun];
  int abx[NP], aby[NP];  // anchor base of each run
  int aidx[NP];          // anchor index of each run
  unsigned valid;        // bit k*kRun+e: pixel (run k, element e) has a position
  int bi0, bi1, bj0, bj1;
  bool empty;            // no pixel of the tile has a tap inside the source
};

// Phases 2 and 3 (ends with a barrier; the box is then known to all).
template <int INTERP, int SORD, bool TSIP, int NP>
__device__ __forceinline__ void tile_positions(const FramePlan &P, const TileGeom &G,
                                               TileShared &sh, const TileCtx &c,
                                               TilePos<NP> &T) {
  constexpr int SLO = TapSupport<INTERP>::lo, SHI = TapSupport<INTERP>::hi;
  const int W = P.src_w, Hs = P.src_h;
  const float tinv = (float)P.t_inv_scale, sinv = (float)P.s_inv_scale;
  int imin = 0x7fffffff, imax = -0x7fffffff, jmin = 0x7fffffff, jmax = -0x7fffffff;
  T.valid = 0u;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int y = c.y0 + c.ty + k * c.RP;
    const int a = ((y >> kCellLog2) - c.cy0) * c.ncx + ((c.xr >> kCellLog2) - c.cx0);
    const Anchor &A = sh.anchor[a];
    T.aidx[k] = a;
    T.abx[k] = A.bx;
    T.aby[k] = A.by;
    const float dy = (float)(y & (kCell - 1));
#pragma unroll
    for (int e = 0; e < kRun; ++e) {
      const int x = c.xr + e;
      const float dx = (float)((c.xr & (kCell - 1)) + e);
      float px, py;
      bool ok = pixel_position<SORD, TSIP>(P, A, tinv, sinv, dx, dy, px, py);
      ok = ok && (y < G.out_h) && (x < G.out_w);
      double dbx = 0.0, dby = 0.0;
      bool exact = false;
      if constexpr (INTERP == DFR_NEAREST) {
        // a rounding decision within reach of the FP32 error: decide in FP64
        float tx_ = px - floorf(px), ty_ = py - floorf(py);
        if (ok && (fabsf(tx_ - 0.5f) < 1e-4f || fabsf(ty_ - 0.5f) < 1e-4f)) {
          double xs, ys;
          ok = position_f64_ct<SORD, TSIP>(P, (double)x, (double)y, xs, ys) && fabs(xs - A.bx) < 1.0e7 &&
               fabs(ys - A.by) < 1.0e7;
          if (ok) {
            px = (float)(rint(xs) - (double)A.bx);
            py = (float)(rint(ys) - (double)A.by);
            exact = true;
            dbx = xs;
            dby = ys;
          }
        }
      }
      T.rx[k][e] = px;
      T.ry[k][e] = py;
      if (G.debug && y < G.out_h && x < G.out_w) {
        double2 d;
        if (!ok) {
          d.x = __builtin_nan("");
          d.y = d.x;
        } else if (exact) {
          d.x = dbx;
          d.y = dby;
        } else {
          d.x = (double)A.bx + (double)px;
          d.y = (double)A.by + (double)py;
        }
        reinterpret_cast<double2 *>(G.debug)[(int64_t)y * G.out_w + x] = d;
      }
      if (ok) {
        int ic, jc;
        if constexpr (INTERP == DFR_NEAREST) {
          ic = A.bx + (int)rintf(px);
          jc = A.by + (int)rintf(py);
        } else {
          ic = A.bx + (int)floorf(px);
          jc = A.by + (int)floorf(py);
        }
        int ilo = ic - SLO, ihi = ic + SHI, jlo = jc - SLO, jhi = jc + SHI;
        if (ihi >= 0 && ilo < W && jhi >= 0 && jlo < Hs) {
          imin = min(imin, max(ilo, 0));
          imax = max(imax, min(ihi, W - 1));
          jmin = min(jmin, max(jlo, 0));
          jmax = max(jmax, min(jhi, Hs - 1));
        }
        T.valid |= 1u << (k * kRun + e);
      }
    }
  }
  imin = wave_min(imin);
  imax = wave_max(imax);
  jmin = wave_min(jmin);
  jmax = wave_max(jmax);
  if ((threadIdx.x & 63) == 0 && imin <= imax) {
    atomicMin(&sh.box[0], imin);
    atomicMax(&sh.box[1], imax);
    atomicMin(&sh.box[2], jmin);
    atomicMax(&sh.box[3], jmax);
  }
  __syncthreads();
  T.bi0 = sh.box[0];
  T.bi1 = sh.box[1];
  T.bj0 = sh.box[2];
  T.bj1 = sh.box[3];
  T.empty = T.bi0 > T.bi1;
  if (T.empty) T.valid = 0u;  // no tap inside the source: every pixel is uncovered
}

// Phase 4: copy the box [bi0, bi1] x [bj0, bj1] of the source into LDS (row
// stride bw) with one wave per row and consecutive lanes on consecutive
// columns.  The caller synchronises.
__device__ __forceinline__ void stage_box(const FramePlan &P, int bi0, int bj0, int bw, int bh,
                                          float *__restrict__ lds) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const float *__restrict__ s0 = P.src + (int64_t)bj0 * P.pitch + bi0;
  for (int r = wave; r < bh; r += kThreads / 64) {
    const float *__restrict__ sr = s0 + (int64_t)r * P.pitch;
    float *__restrict__ lr = lds + r * bw;
    for (int col = lane; col < bw; col += 64) lr[col] = sr[col];
  }
}

__device__ __forceinline__ void store_run(float *__restrict__ base, int64_t off, int x, int out_w,
                                          bool vec, const float v[kRun]) {
  if (vec && x + kRun <= out_w) {
    *reinterpret_cast<float4 *>(base + off) = make_float4(v[0], v[1], v[2], v[3]);
  } else {
#pragma unroll
    for (int e = 0; e < kRun; ++e)
      if (x + e < out_w) base[off + e] = v[e];
  }
}

__device__ __forceinline__ bool vector_stores_ok(const FramePlan &P, const TileGeom &G) {
  return ((G.out_w & (kRun - 1)) == 0) && ((reinterpret_cast<uintptr_t>(P.out) & 15) == 0) &&
         (P.fp == nullptr || (reinterpret_cast<uintptr_t>(P.fp) & 15) == 0);
}

// Nearest: the FP64 rounding decision for a pixel whose FP32 position lies
// within 1e-4 px of a tie (rare).  Writes the rounded position relative to
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

// -------------------------------------------------------------- forward --
//
// The forward tile runs a different schedule from the one above, built so
// that the source staging overlaps the position arithmetic:
//   1. wave 0: the FP64 anchors of the tile's cells; wave 1, at the same
//      time: FP64 source positions at 9 points of the tile (corners, edge
//      midpoints, centre) giving the tile's source box, grown by the tap
//      support and 2 px;
//   2. the box is staged into LDS with asynchronous global->LDS DMA loads
//      (gfx950 global_load_lds_dword), row by row;
//   3. meanwhile every pixel's FP32 position is computed;
//   4. wait for the DMA, then gather.  A tile whose box lies inside the
//      source, whose cells all have valid positions and which lies inside the
//      output takes an unmasked path (footprint exactly 1); every pixel is
//      still checked against the box and a wave with any pixel outside it
//      takes the general (masked, global-fallback) path, so the box is only
//      a performance hint.

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

// Stage rows [bj0, bj0+bh) x columns [bi0, bi0+bw) of the source into LDS
// (row stride bw) with asynchronous DMA: one wave per row, 64 columns per
// instruction, lanes past the row end masked off.
__device__ __forceinline__ void dma_box(const FramePlan &P, int bi0, int bj0, int bw, int bh,
                                        float *__restrict__ lds) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const float *__restrict__ s0 = P.src + (int64_t)bj0 * P.pitch + bi0;
#pragma unroll 1
  for (int r = wave; r < bh; r += kThreads / 64) {
    const float *sr = s0 + (int64_t)r * P.pitch;
#pragma unroll 1
    for (int c0 = 0; c0 < bw; c0 += 64) {
      if (c0 + lane < bw)
        __builtin_amdgcn_global_load_lds(sr + c0 + lane, lds + r * bw + c0, 4, 0, 0);
    }
  }
}

// The target SIP is compiled only into the run-time-order variant (the
// launcher uses it whenever the target WCS has A/B).
template <int INTERP, int SORD, int NP>
__device__ __forceinline__ void forward_tile(const FramePlan &P, const TileGeom &G, int tile,
                                             float *__restrict__ lds, TileShared &sh) {
  constexpr bool TSIP = SORD == kRtOrder;
  const int tid = threadIdx.x, wave = tid >> 6;
  const int lg = G.txt_log2;
  const int TW = kRun << lg, RP = kThreads >> lg, TH = RP * NP;
  const int trow = tile / G.tiles_x;
  const int x0 = (tile - trow * G.tiles_x) * TW, y0 = trow * TH;
  const int cx0 = x0 / kCell, ncx = TW / kCell, cy0 = y0 / kCell;
  const int nA = ncx * (TH >= kCell ? TH / kCell : 1);
  const int ty = tid >> lg, xr = x0 + (tid & ((1 << lg) - 1)) * kRun;
  const int W = P.src_w, Hs = P.src_h;

  // ---- 1. anchors (FP64) and, from their linear models, the source box
  if (wave == 0) {
    constexpr int lo = TapSupport<INTERP>::lo + 2, hi = TapSupport<INTERP>::hi + 2;
    int t = 0, okc = 1;
    int imn = 0x3fffffff, imx = -0x3fffffff, jmn = 0x3fffffff, jmx = -0x3fffffff;
    if (tid < nA) {
      const int cy = cy0 + tid / ncx, cx = cx0 + tid % ncx;
      const int xa = cx * kCell, ya = cy * kCell;
      Anchor &A = sh.anchor[tid];
      compute_anchor<SORD, TSIP>(P, xa, ya, TapSupport<INTERP>::hi, A);
      t = A.touch;
      okc = A.ok;
      // the part of the cell inside the tile and the output, as offsets
      const float ux = (float)(min(xa + kCell, min(x0 + TW, G.out_w)) - 1 - xa);
      const float vy0 = (float)(max(ya, y0) - ya);
      const float vy1 = (float)(min(ya + kCell, min(y0 + TH, G.out_h)) - 1 - ya);
      // extremes of the linear model over that rectangle, grown by the
      // rigorous bound on the model's error, relative to (bx, by)
      const float mx = A.ex, my = A.ey;
      const float x_a = A.sx0 + fminf(0.0f, A.jx[0] * ux) + fminf(A.jx[1] * vy0, A.jx[1] * vy1) - mx;
      const float x_b = A.sx0 + fmaxf(0.0f, A.jx[0] * ux) + fmaxf(A.jx[1] * vy0, A.jx[1] * vy1) + mx;
      const float y_a = A.sy0 + fminf(0.0f, A.jy[0] * ux) + fminf(A.jy[1] * vy0, A.jy[1] * vy1) - my;
      const float y_b = A.sy0 + fmaxf(0.0f, A.jy[0] * ux) + fmaxf(A.jy[1] * vy0, A.jy[1] * vy1) + my;
      if (okc && fabsf(x_a) < 1.0e7f && fabsf(x_b) < 1.0e7f && fabsf(y_a) < 1.0e7f &&
          fabsf(y_b) < 1.0e7f) {
        imn = A.bx + (int)floorf(x_a) - lo;
        imx = A.bx + (int)floorf(x_b) + hi;
        jmn = A.by + (int)floorf(y_a) - lo;
        jmx = A.by + (int)floorf(y_b) + hi;
      } else {
        okc = 0;
      }
    }
#pragma unroll
    for (int m = kMaxAnchors / 2; m >= 1; m >>= 1) {
      imn = min(imn, __shfl_xor(imn, m, 64));
      imx = max(imx, __shfl_xor(imx, m, 64));
      jmn = min(jmn, __shfl_xor(jmn, m, 64));
      jmx = max(jmx, __shfl_xor(jmx, m, 64));
    }
    const unsigned long long any = __ballot(t != 0), bad = __ballot(okc == 0);
    if (tid == 0) {
      sh.touch = any != 0ull;
      sh.cells_ok = bad == 0ull;
      sh.box_ok = bad == 0ull;
      sh.box[0] = imn;
      sh.box[1] = imx;
      sh.box[2] = jmn;
      sh.box[3] = jmx;
    }
  }
  __syncthreads();

  const bool vec = vector_stores_ok(P, G);
  const float miss = G.nan_outside ? __builtin_nanf("") : 0.0f;
  if (!sh.touch && G.allow_skip) {
    float zo[kRun], zf[kRun];
#pragma unroll
    for (int e = 0; e < kRun; ++e) {
      zo[e] = miss;
      zf[e] = 0.0f;
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      int y = y0 + ty + k * RP;
      if (y >= G.out_h || xr >= G.out_w) continue;
      int64_t off = (int64_t)y * G.out_w + xr;
      store_run(P.out, off, xr, G.out_w, vec, zo);
      if (P.fp) store_run(P.fp, off, xr, G.out_w, vec, zf);
    }
    return;
  }

  // ---- 2. stage the box (asynchronous)
  const int bu0 = sh.box[0], bu1 = sh.box[1], bu2 = sh.box[2], bu3 = sh.box[3];
  const int bi0 = max(bu0, 0), bi1 = min(bu1, W - 1), bj0 = max(bu2, 0), bj1 = min(bu3, Hs - 1);
  const bool box_ok = sh.box_ok && bi0 <= bi1 && bj0 <= bj1;
  const int bw = box_ok ? bi1 - bi0 + 1 : 0, bh = box_ok ? bj1 - bj0 + 1 : 0;
  const bool use_lds = box_ok && (int64_t)bw * bh <= (int64_t)G.lds_cap;
  const bool interior = use_lds && sh.cells_ok && P.t_order == 0 && bu0 == bi0 && bu1 == bi1 &&
                        bu2 == bj0 && bu3 == bj1 && x0 + TW <= G.out_w && y0 + TH <= G.out_h;
  if (use_lds) dma_box(P, bi0, bj0, bw, bh, lds);

  // ---- 3. positions (FP32 offsets from the anchors)
  const float tinv = (float)P.t_inv_scale, sinv = (float)P.s_inv_scale;
  float rx[NP][kRun], ry[NP][kRun];
  int abx[NP], aby[NP];
  unsigned valid = 0u;
  if (interior && !G.debug) {
    // every cell is valid throughout and the tile lies inside the output
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const int y = y0 + ty + k * RP;
      const Anchor &A = sh.anchor[((y >> kCellLog2) - cy0) * ncx + ((xr >> kCellLog2) - cx0)];
      abx[k] = A.bx - bi0;
      aby[k] = A.by - bj0;
      const float dy = (float)(y & (kCell - 1));
#pragma unroll
      for (int e = 0; e < kRun; ++e) {
        float px, py;
        pixel_position<SORD, TSIP>(P, A, tinv, sinv, (float)((xr & (kCell - 1)) + e), dy, px, py);
        if constexpr (INTERP == DFR_NEAREST) {
          // a rounding decision within reach of the FP32 error: decide in FP64
          float tx_ = px - floorf(px), ty_ = py - floorf(py);
          if (fabsf(tx_ - 0.5f) < 1e-4f || fabsf(ty_ - 0.5f) < 1e-4f) {
            double xs, ys;
            nearest_exact<SORD, TSIP>(P, xr + e, y, A.bx, A.by, px, py, xs, ys);
          }
        }
        rx[k][e] = px;
        ry[k][e] = py;
      }
    }
    valid = ~0u;
  } else {
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const int y = y0 + ty + k * RP;
      const Anchor &A = sh.anchor[((y >> kCellLog2) - cy0) * ncx + ((xr >> kCellLog2) - cx0)];
      abx[k] = A.bx - bi0;
      aby[k] = A.by - bj0;
      const float dy = (float)(y & (kCell - 1));
#pragma unroll
      for (int e = 0; e < kRun; ++e) {
        const int x = xr + e;
        float px, py;
        bool ok = pixel_position<SORD, TSIP>(P, A, tinv, sinv, (float)((xr & (kCell - 1)) + e), dy,
                                       px, py);
        ok = ok && (y < G.out_h) && (x < G.out_w);
        double dbx = 0.0, dby = 0.0;
        bool exact = false;
        if constexpr (INTERP == DFR_NEAREST) {
          // a rounding decision within reach of the FP32 error: decide in FP64
          float tx_ = px - floorf(px), ty_ = py - floorf(py);
          if (ok && (fabsf(tx_ - 0.5f) < 1e-4f || fabsf(ty_ - 0.5f) < 1e-4f)) {
            ok = nearest_exact<SORD, TSIP>(P, x, y, A.bx, A.by, px, py, dbx, dby);
            exact = ok;
          }
        }
        rx[k][e] = px;
        ry[k][e] = py;
        if (G.debug && y < G.out_h && x < G.out_w) {
          double2 d;
          if (!ok) {
            d.x = __builtin_nan("");
            d.y = d.x;
          } else if (exact) {
            d.x = dbx;
            d.y = dby;
          } else {
            d.x = (double)A.bx + (double)px;
            d.y = (double)A.by + (double)py;
          }
          reinterpret_cast<double2 *>(G.debug)[(int64_t)y * G.out_w + x] = d;
        }
        if (ok) valid |= 1u << (k * kRun + e);
      }
    }
  }

  // ---- 4. gather
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  constexpr int SPAN = TapSupport<INTERP>::lo + TapSupport<INTERP>::hi;
  // Interior tiles need no per-pixel check: the box holds every tap by the
  // rigorous margin of the anchors' linear models.
  const bool fast = interior && valid == ~0u;
  const float a = G.cubic_a;
  if (fast) {
    // box-relative tap coordinates: unmasked LDS reads from one base address
    // per pixel, footprint exactly 1
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const int y = y0 + ty + k * RP;
      float o[kRun], f[kRun];
#pragma unroll
      for (int e = 0; e < kRun; ++e) {
        int i0, j0;
        float t_, s_;
        tap_origin<INTERP>(rx[k][e], abx[k], i0, t_);
        tap_origin<INTERP>(ry[k][e], aby[k], j0, s_);
        // i0, j0 >= 0 inside the box: one 24-bit multiply-add per pixel
        const float *__restrict__ b = lds + __umul24(j0, bw) + i0;
        auto fl = [&](int i, int j) -> float { return b[j * bw + i]; };
        if constexpr (INTERP == DFR_NEAREST) {
          o[e] = b[0];
        } else if constexpr (INTERP == DFR_BILINEAR) {
          o[e] = Taps<DFR_BILINEAR>::interior(0, 0, t_, s_, fl);
        } else {
          float wx[4], wy[4];
          keys_weights(t_, a, wx);
          keys_weights(s_, a, wy);
          o[e] = Taps<DFR_BICUBIC>::interior(0, 0, wx, wy, fl);
        }
        f[e] = 1.0f;
      }
      const int64_t off = (int64_t)y * G.out_w + xr;
      store_run(P.out, off, xr, G.out_w, vec, o);
      if (P.fp) store_run(P.fp, off, xr, G.out_w, vec, f);
    }
    return;
  }
  // general path: source coordinates, zero padding, footprint normalisation;
  // taps come from LDS when the pixel's in-image taps are inside the box
  auto fl = [&](int i, int j) -> float { return lds[__umul24(j - bj0, bw) + (i - bi0)]; };
  auto fg = [&](int i, int j) -> float { return P.src[(int64_t)j * P.pitch + i]; };
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int y = y0 + ty + k * RP;
    if (y >= G.out_h || xr >= G.out_w) continue;
    float o[kRun], f[kRun];
#pragma unroll
    for (int e = 0; e < kRun; ++e) {
      o[e] = miss;
      f[e] = 0.0f;
      if (valid & (1u << (k * kRun + e))) {
        int i0, j0;
        float t_, s_;
        tap_origin<INTERP>(rx[k][e], abx[k] + bi0, i0, t_);
        tap_origin<INTERP>(ry[k][e], aby[k] + bj0, j0, s_);
        const bool in_lds = use_lds && max(i0, 0) >= bi0 && min(i0 + SPAN, W - 1) <= bi1 &&
                            max(j0, 0) >= bj0 && min(j0 + SPAN, Hs - 1) <= bj1;
        float ov, fv;
        if (in_lds)
          interp_general<INTERP>(i0, j0, t_, s_, W, Hs, a, fl, ov, fv);
        else
          interp_general<INTERP>(i0, j0, t_, s_, W, Hs, a, fg, ov, fv);
        if (fv > 0.0f) {
          o[e] = ov;
          f[e] = fv;
        }
      }
    }
    const int64_t off = (int64_t)y * G.out_w + xr;
    store_run(P.out, off, xr, G.out_w, vec, o);
    if (P.fp) store_run(P.fp, off, xr, G.out_w, vec, f);
  }
}

}  // namespace dfr
