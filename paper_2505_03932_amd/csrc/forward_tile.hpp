// Forward reprojection of one output tile per work-group (section 3.1 for
// every pixel: the two stages of section 3.2 give the source position, then
// interpolation and footprint normalisation).
//
// A tile is (kRun << txt_log2) x ((kThreads >> txt_log2) * NP) output
// pixels.  Thread (tx, ty) owns NP runs of kRun consecutive pixels in rows
// ty, ty + RP, ..., so every wave store covers contiguous row segments.
//   1. wave 0: per cell of the tile (32x32 output pixels) its certified
//      position model (cell_model.hpp) from the model table, else its FP64
//      anchor; from them a rigorous source box, grown by the tap support;
//   2. the box is staged into LDS with asynchronous global->LDS DMA loads
//      (gfx950 global_load_lds_dword), row by row, by all waves;
//   3. meanwhile every pixel's FP32 source position is computed;
//   4. wait for the DMA, then gather.  A tile whose box lies inside the
//      source, whose cells all have valid positions and which lies inside the
//      output is gathered without per-pixel checks (footprint exactly 1);
//      others take the general path (zero padding, footprint normalisation,
//      global fetches for taps outside the box).
// Positions depend only on the pixel's cell (its model or anchor), never on
// the tile shape, so every tile shape, the batch and the coadd give identical
// per-pixel results.  A sink takes them (stores, or the coadd's sums).
#pragma once

#include "forward_body.hpp"

namespace dfr {

// LDS of a forward work-group besides the staged source box.
struct FwdShared {
  union CellSlot {
    Anchor anchor;
    CellModel model;
  } cell[kMaxAnchors];
  int kind[kMaxAnchors];  // 1: cell[i].model, 0: cell[i].anchor
  int box[4];             // imin, imax, jmin, jmax of the source box
  int touch;              // some cell can reach the source
  int cells_ok;           // every cell has valid positions throughout
  int box_ok;             // the box is finite
  int all_model;          // every cell has a model
  int item;               // batch: work item handed to this work-group
};

// Stage rows [bj0, bj0+bh) x columns [bi0, bi0+bw) of the source into LDS
// (row stride lp) with asynchronous DMA: one wave per row, 64 columns per
// instruction, lanes past the row end masked off.
__device__ __forceinline__ void dma_box(const FramePlan &P, int bi0, int bj0, int bw, int bh,
                                        int lp, float *__restrict__ lds) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const auto *__restrict__ s0 = global_ptr(P.src) + (int64_t)bj0 * P.pitch + bi0;
#pragma unroll 1
  for (int r = wave; r < bh; r += kThreads / 64) {
    const auto *sr = s0 + (int64_t)r * P.pitch;
#pragma unroll 1
    for (int c0 = 0; c0 < bw; c0 += 64) {
      if (c0 + lane < bw)
        __builtin_amdgcn_global_load_lds(sr + c0 + lane, lds + r * lp + c0, 4, 0, 0);
    }
  }
}

// A tile no pixel of which reaches the source: output "uncovered" (0, or
// NaN with nan_outside) and footprint 0.
template <int NP>
__device__ __forceinline__ void tile_uncovered(const FramePlan &P, const TileGeom &G, int tile) {
  const int lg = G.txt_log2;
  const int TW = kRun << lg, RP = kThreads >> lg, TH = RP * NP;
  const int trow = tile / G.tiles_x;
  const int x0 = (tile - trow * G.tiles_x) * TW, y0 = trow * TH;
  const int ty = threadIdx.x >> lg, xr = x0 + (threadIdx.x & ((1 << lg) - 1)) * kRun;
  const bool vec = vector_stores_ok(P, G);
  const float miss = G.nan_outside ? __builtin_nanf("") : 0.0f;
  float zo[kRun], zf[kRun];
#pragma unroll
  for (int e = 0; e < kRun; ++e) {
    zo[e] = miss;
    zf[e] = 0.0f;
  }
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int y = y0 + ty + k * RP;
    if (y >= G.out_h || xr >= G.out_w) continue;
    const int64_t off = (int64_t)y * G.out_w + xr;
    store_run(P.out, off, xr, G.out_w, vec, zo);
    if (P.fp) store_run(P.fp, off, xr, G.out_w, vec, zf);
  }
}

// Whether tile `tile` lies outside the frame's reach box (cells that may
// reach the source, recorded by the batch model prepass): then it is
// uncovered without looking at its cells.
template <int NP>
__device__ __forceinline__ bool tile_out_of_reach(const FramePlan &P, const TileGeom &G, int tile) {
  if (P.reach == nullptr) return false;
  using ConstI = const __attribute__((address_space(4))) int32_t;
  ConstI *r = (ConstI *)P.reach;
  const int r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
  if (r1 == 0) return true;  // no cell of the frame reaches its source
  const int lg = G.txt_log2;
  const int TW = kRun << lg, TH = (kThreads >> lg) * NP;
  const int trow = tile / G.tiles_x;
  const int x0 = (tile - trow * G.tiles_x) * TW, y0 = trow * TH;
  const int cx0 = x0 >> kCellLog2, cx1 = (x0 + TW - 1) >> kCellLog2;
  const int cy0 = y0 >> kCellLog2, cy1 = (y0 + TH - 1) >> kCellLog2;
  return cx1 < kReachBig - r0 || cx0 >= r1 || cy1 < kReachBig - r2 || cy0 >= r3;
}

// Where the results of a forward tile go.  StoreSink writes each pixel's
// value and footprint to the frame's outputs (dfr_reproject, the batch);
// StackSink adds out * F and F of every covered pixel to per-thread
// accumulators (the coadd), so the per-pixel arithmetic is the same code
// either way.
struct StoreSink {
  // nearest: pixels whose rounding is decided in FP64 are stored first with
  // the FP32 decision and overwritten by pixel() after the gather
  static constexpr bool kDeferTies = true;
  __device__ __forceinline__ void pixel(const FramePlan &P, const TileGeom &G, int y, int x,
                                        float o, float f) {
    const int64_t off = (int64_t)y * G.out_w + x;
    __builtin_nontemporal_store(o, global_ptr(P.out) + off);
    if (P.fp) __builtin_nontemporal_store(f, global_ptr(P.fp) + off);
  }
  template <int NP>
  __device__ __forceinline__ void uncovered(const FramePlan &P, const TileGeom &G, int tile) {
    tile_uncovered<NP>(P, G, tile);
  }
  // run k of the thread (output row y, columns xr ..); `full`: every
  // footprint is exactly 1
  __device__ __forceinline__ void row(const FramePlan &P, const TileGeom &G, int k, int y,
                                      int xr, bool vec, bool full, const float o[kRun],
                                      const float f[kRun]) {
    const int64_t off = (int64_t)y * G.out_w + xr;
    store_run(P.out, off, xr, G.out_w, vec, o);
    if (P.fp) store_run(P.fp, off, xr, G.out_w, vec, f);
  }
};

template <int NP>
struct StackSink {
  static constexpr bool kDeferTies = false;  // sums cannot be corrected afterwards
  float s[NP][kRun];  // sum of out * F
  float w[NP][kRun];  // sum of F
  template <int NP_>
  __device__ __forceinline__ void uncovered(const FramePlan &, const TileGeom &, int) {}
  __device__ __forceinline__ void row(const FramePlan &, const TileGeom &, int k, int, int, bool,
                                      bool full, const float o[kRun], const float f[kRun]) {
#pragma unroll
    for (int e = 0; e < kRun; ++e) {
      if (full) {
        s[k][e] += o[e];  // F = 1: out * F is out exactly
        w[k][e] += 1.0f;
      } else if (f[e] > 0.0f) {
        s[k][e] = fmaf(o[e], f[e], s[k][e]);
        w[k][e] += f[e];
      }
    }
  }
};

// Writes into the frame's window (cropped batch): P.out and P.fp are
// [crop h][crop w] arrays of the target pixels x0 .. x0+w-1, y0 .. y0+h-1;
// pixels of the tile outside the window are not stored.
struct CropSink {
  static constexpr bool kDeferTies = true;
  __device__ __forceinline__ void pixel(const FramePlan &P, const TileGeom &G, int y, int x,
                                        float o, float f) {
    const int cx = P.crop[0], cy = P.crop[1], cw = P.crop[2], ch = P.crop[3];
    if (y < cy || y >= cy + ch || x < cx || x >= cx + cw) return;
    const int64_t off = (int64_t)(y - cy) * cw + (x - cx);
    __builtin_nontemporal_store(o, global_ptr(P.out) + off);
    if (P.fp) __builtin_nontemporal_store(f, global_ptr(P.fp) + off);
  }
  template <int NP>
  __device__ __forceinline__ void uncovered(const FramePlan &P, const TileGeom &G, int tile);
  __device__ __forceinline__ void row(const FramePlan &P, const TileGeom &G, int, int y, int xr,
                                      bool, bool, const float o[kRun], const float f[kRun]) {
    const int cx = P.crop[0], cy = P.crop[1], cw = P.crop[2], ch = P.crop[3];
    if (y < cy || y >= cy + ch || xr + kRun <= cx || xr >= cx + cw) return;
    const int rx = xr - cx;
    const int64_t off = (int64_t)(y - cy) * cw + rx;
    const bool vec = rx >= 0 && rx + kRun <= cw && ((rx | cw) & (kRun - 1)) == 0 &&
                     ((reinterpret_cast<uintptr_t>(P.out) & 15) == 0) &&
                     (P.fp == nullptr || (reinterpret_cast<uintptr_t>(P.fp) & 15) == 0);
    if (vec) {
      store_run(P.out, off, 0, kRun, true, o);
      if (P.fp) store_run(P.fp, off, 0, kRun, true, f);
      return;
    }
#pragma unroll
    for (int e = 0; e < kRun; ++e) {
      if (rx + e < 0 || rx + e >= cw) continue;
      __builtin_nontemporal_store(o[e], global_ptr(P.out) + off + e);
      if (P.fp) __builtin_nontemporal_store(f[e], global_ptr(P.fp) + off + e);
    }
  }
};

// Placement of a tile in the output and of this thread's runs in the tile.
struct TileXY {
  int TW, RP, TH;   // tile width and height; rows between a thread's runs
  int x0, y0;       // first output pixel of the tile
  int cx0, cy0;     // first cell of the tile
  int ncx, nA;      // cells per tile row, cells of the tile
  int ty, xr;       // this thread's first row (in the tile) and first column
};

template <int NP>
__device__ __forceinline__ TileXY tile_xy(const TileGeom &G, int tile) {
  TileXY T;
  const int lg = G.txt_log2;
  T.TW = kRun << lg;
  T.RP = kThreads >> lg;
  T.TH = T.RP * NP;
  const int trow = tile / G.tiles_x;
  T.x0 = (tile - trow * G.tiles_x) * T.TW;
  T.y0 = trow * T.TH;
  T.cx0 = T.x0 / kCell;
  T.ncx = T.TW / kCell;
  T.cy0 = T.y0 / kCell;
  T.nA = T.ncx * (T.TH >= kCell ? T.TH / kCell : 1);
  T.ty = threadIdx.x >> lg;
  T.xr = T.x0 + (threadIdx.x & ((1 << lg) - 1)) * kRun;
  return T;
}

// Index of cell i of the tile in the frame's model table.
__device__ __forceinline__ int64_t tile_cell_index(const TileGeom &G, const TileXY &T, int i) {
  const int cy = T.cy0 + i / T.ncx, cx = T.cx0 + i % T.ncx;
  return (int64_t)cy * ((G.out_w + kCell - 1) >> kCellLog2) + cx;
}

// Phase 1, run by wave 0: per cell of the tile its certified model from the
// model table, else its FP64 anchor; from them the rigorous source box and
// the tile's flags, into sh.
// The target SIP is compiled only into the run-time-order variant (the
// launcher uses it whenever the target WCS has A/B).
template <int INTERP, int SORD, int NP>
__device__ __forceinline__ void tile_cells(const FramePlan &P, const TileGeom &G, const TileXY &T,
                                           FwdShared &sh) {
  constexpr bool TSIP = SORD == kRtOrder;
  const int tid = threadIdx.x;
  const int W = P.src_w, Hs = P.src_h;
  int t = 0, okc = 1, kind = 0;
  int imn = 0x3fffffff, imx = -0x3fffffff, jmn = 0x3fffffff, jmx = -0x3fffffff;
  if (tid < T.nA) {
    const int cy = T.cy0 + tid / T.ncx, cx = T.cx0 + tid % T.ncx;
    const int xa = cx * kCell, ya = cy * kCell;
    if (xa >= G.out_w || ya >= G.out_h) {
      // a cell of a ragged edge tile wholly outside the output: none of its
      // pixels is computed, it has no model-table entry and adds nothing to
      // the box (its sh.cell slot is never read for a valid pixel)
      kind = 1;
    } else if (P.models) {
      const CellModel *Mg = P.models + tile_cell_index(G, T, tid);
      typedef unsigned u4v __attribute__((ext_vector_type(4)));
#pragma unroll
      for (int part = 0; part < (int)(sizeof(CellModel) / 16); ++part)
        reinterpret_cast<u4v *>(&sh.cell[tid].model)[part] =
            global_ptr(reinterpret_cast<const u4v *>(Mg))[part];
      kind = sh.cell[tid].model.certified;
      if (kind) {
        // the model covers every pixel of the cell: the box needs only the
        // tap support (+1 px kept as a guard)
        constexpr int lo = TapSupport<INTERP>::lo + 1, hi = TapSupport<INTERP>::hi + 1;
        const CellModel &M = sh.cell[tid].model;
        // the part of the cell inside the tile and the output, as offsets
        // from the cell centre; extremes of the linear part there, grown
        // by the bound on the rest
        const float h = (float)kHalfCell;
        const float a0 = (float)(max(xa, T.x0) - xa) - h;
        const float a1 = (float)(min(xa + kCell, min(T.x0 + T.TW, G.out_w)) - 1 - xa) - h;
        const float b0 = (float)(max(ya, T.y0) - ya) - h;
        const float b1 = (float)(min(ya + kCell, min(T.y0 + T.TH, G.out_h)) - 1 - ya) - h;
        const float xl = M.mx[0] + fminf(M.mx[4] * a0, M.mx[4] * a1) + fminf(M.mx[1] * b0, M.mx[1] * b1) - M.ex;
        const float xh = M.mx[0] + fmaxf(M.mx[4] * a0, M.mx[4] * a1) + fmaxf(M.mx[1] * b0, M.mx[1] * b1) + M.ex;
        const float yl = M.my[0] + fminf(M.my[4] * a0, M.my[4] * a1) + fminf(M.my[1] * b0, M.my[1] * b1) - M.ey;
        const float yh = M.my[0] + fmaxf(M.my[4] * a0, M.my[4] * a1) + fmaxf(M.my[1] * b0, M.my[1] * b1) + M.ey;
        imn = M.bx + (int)floorf(xl) - lo;
        imx = M.bx + (int)floorf(xh) + hi;
        jmn = M.by + (int)floorf(yl) - lo;
        jmx = M.by + (int)floorf(yh) + hi;
        t = (imx >= 0 && imn <= W - 1 && jmx >= 0 && jmn <= Hs - 1) ? 1 : 0;
      }
    }
    if (!kind) {
      // no certified model: the cell's FP64 anchor and linear-model bound
      constexpr int lo = TapSupport<INTERP>::lo + 2, hi = TapSupport<INTERP>::hi + 2;
      Anchor &A = sh.cell[tid].anchor;
      compute_anchor<SORD, TSIP>(P, xa, ya, TapSupport<INTERP>::hi, A);
      t = A.touch;
      okc = A.ok;
      // the part of the cell inside the tile and the output, as offsets
      const float ux = (float)(min(xa + kCell, min(T.x0 + T.TW, G.out_w)) - 1 - xa);
      const float vy0 = (float)(max(ya, T.y0) - ya);
      const float vy1 = (float)(min(ya + kCell, min(T.y0 + T.TH, G.out_h)) - 1 - ya);
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
    sh.kind[tid] = kind;
  }
#pragma unroll
  for (int m = kMaxAnchors / 2; m >= 1; m >>= 1) {
    imn = min(imn, __shfl_xor(imn, m, 64));
    imx = max(imx, __shfl_xor(imx, m, 64));
    jmn = min(jmn, __shfl_xor(jmn, m, 64));
    jmx = max(jmx, __shfl_xor(jmx, m, 64));
  }
  const unsigned long long any = __ballot(t != 0), bad = __ballot(okc == 0),
                           anch = __ballot(tid < T.nA && kind == 0);
  if (tid == 0) {
    sh.touch = any != 0ull;
    sh.cells_ok = bad == 0ull;
    sh.box_ok = bad == 0ull;
    sh.all_model = anch == 0ull;
    sh.box[0] = imn;
    sh.box[1] = imx;
    sh.box[2] = jmn;
    sh.box[3] = jmx;
  }
}

// The staged source box of a tile (phase 2), from the flags tile_cells set.
struct TileBox {
  int bi0, bi1, bj0, bj1;  // the box clamped to the source
  int bw, bh, lp;          // its size and LDS row stride
  bool use_lds;            // staged (fits the LDS budget)
  bool interior;           // no per-pixel checks needed
  bool all_model;          // every cell has a certified model
  bool touch;              // some cell can reach the source
};

template <int NP>
__device__ __forceinline__ TileBox tile_box(const FramePlan &P, const TileGeom &G,
                                            const TileXY &T, const FwdShared &sh, int lds_cap) {
  TileBox B;
  const int W = P.src_w, Hs = P.src_h;
  const int bu0 = sh.box[0], bu1 = sh.box[1], bu2 = sh.box[2], bu3 = sh.box[3];
  B.bi0 = max(bu0, 0);
  B.bi1 = min(bu1, W - 1);
  B.bj0 = max(bu2, 0);
  B.bj1 = min(bu3, Hs - 1);
  const bool box_ok = sh.box_ok && B.bi0 <= B.bi1 && B.bj0 <= B.bj1;
  B.bw = box_ok ? B.bi1 - B.bi0 + 1 : 0;
  B.bh = box_ok ? B.bj1 - B.bj0 + 1 : 0;
  B.lp = lds_pitch(B.bw);  // padded row stride (bank spread)
  B.use_lds = box_ok && (int64_t)B.lp * B.bh <= (int64_t)lds_cap;
  B.interior = B.use_lds && sh.cells_ok && P.t_order == 0 && bu0 == B.bi0 && bu1 == B.bi1 &&
               bu2 == B.bj0 && bu3 == B.bj1 && T.x0 + T.TW <= G.out_w && T.y0 + T.TH <= G.out_h;
  B.all_model = sh.all_model;
  B.touch = sh.touch;
  return B;
}

// FP32 source positions of a thread's pixels relative to the box.
template <int NP>
struct FwdPos {
  float rx[NP][kRun], ry[NP][kRun];
  int abx[NP], aby[NP];  // cell base position minus the box origin, per run
  unsigned valid;        // bit k * kRun + e: pixel (k, e) has a position
  unsigned tie;          // nearest, deferred: pixel (k, e) needs the FP64 decision
};

// Nearest: whether the FP32 position (px, py) lies closer to a rounding tie
// than 0.5 - lim on either axis (x - rint(x) is exact in FP32).
__device__ __forceinline__ bool near_tie(float px, float py, float lim) {
  return fmaxf(fabsf(px - rintf(px)), fabsf(py - rintf(py))) > lim;
}

// FP32 positions of the anchored chain: within 1e-4 px of a tie they are
// decided in FP64 (at least 5x that chain's FP32 error).
constexpr float kAnchorTieLim = 0.4999f;

// Phase 3: every pixel's position from its cell's model or anchor (sh.cell).
// Nearest: a pixel whose FP32 position lies within reach of its FP32 error
// of a rounding tie (the model's rigorous M.tie, or 1e-4 px for an anchored
// cell) is decided from an FP64 position, here (DEFER false) or after the
// gather by nearest_ties (DEFER true: only a bit is kept here, so the FP64
// chain's registers are not live across the tile's main work).
template <int INTERP, int SORD, int NP, bool DEFER>
__device__ __forceinline__ void tile_positions(const FramePlan &P, const TileGeom &G,
                                               const TileXY &T, const FwdShared &sh,
                                               const TileBox &B, FwdPos<NP> &R) {
  constexpr bool TSIP = SORD == kRtOrder;
  const float tinv = (float)P.t_inv_scale, sinv = (float)P.s_inv_scale;
  const float hc = (float)kHalfCell;
  const int xr = T.xr;
  R.valid = 0u;
  R.tie = 0u;
  if (B.all_model && B.interior && !G.debug) {
    // certified cubic models throughout, tile inside the output: every pixel
    // is valid
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const int y = T.y0 + T.ty + k * T.RP;
      const CellModel &M = sh.cell[((y >> kCellLog2) - T.cy0) * T.ncx + ((xr >> kCellLog2) - T.cx0)].model;
      R.abx[k] = M.bx - B.bi0;
      R.aby[k] = M.by - B.bj0;
      const float lim = 0.5f - M.tie;
      ModelRow Rw;
      model_row(M, (float)(y & (kCell - 1)) - hc, Rw);
      const float a0 = (float)(xr & (kCell - 1)) - hc;
#pragma unroll
      for (int e = 0; e < kRun; ++e) {
        float px, py;
        model_at(Rw, a0 + (float)e, px, py);
        if constexpr (INTERP == DFR_NEAREST) {
          // a rounding decision within reach of the FP32 error: decide in FP64
          if (near_tie(px, py, lim)) {
            if constexpr (DEFER) {
              R.tie |= 1u << (k * kRun + e);
            } else {
              double xs, ys;
              nearest_exact<SORD, TSIP>(P, xr + e, y, M.bx, M.by, px, py, xs, ys);
            }
          }
        }
        R.rx[k][e] = px;
        R.ry[k][e] = py;
      }
    }
    R.valid = ~0u;
  } else {
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const int y = T.y0 + T.ty + k * T.RP;
      const int ci = ((y >> kCellLog2) - T.cy0) * T.ncx + ((xr >> kCellLog2) - T.cx0);
      const bool mk = sh.kind[ci] != 0;
      const Anchor &A = sh.cell[ci].anchor;
      const CellModel &M = sh.cell[ci].model;
      const int bx = mk ? M.bx : A.bx, by = mk ? M.by : A.by;
      R.abx[k] = bx - B.bi0;
      R.aby[k] = by - B.bj0;
      const float lim = mk ? 0.5f - M.tie : kAnchorTieLim;
      ModelRow Rw;
      if (mk) model_row(M, (float)(y & (kCell - 1)) - hc, Rw);
      const float dy = (float)(y & (kCell - 1));
      const float a0 = (float)(xr & (kCell - 1)) - hc;
#pragma unroll
      for (int e = 0; e < kRun; ++e) {
        const int x = xr + e;
        float px, py;
        bool ok;
        if (mk) {
          model_at(Rw, a0 + (float)e, px, py);
          ok = true;
        } else {
          ok = pixel_position<SORD, TSIP>(P, A, tinv, sinv, (float)((xr & (kCell - 1)) + e), dy,
                                          px, py);
        }
        ok = ok && (y < G.out_h) && (x < G.out_w);
        double dbx = 0.0, dby = 0.0;
        bool exact = false;
        if constexpr (INTERP == DFR_NEAREST) {
          // a rounding decision within reach of the FP32 error: decide in FP64
          if (ok && near_tie(px, py, lim)) {
            if constexpr (DEFER) {
              R.tie |= 1u << (k * kRun + e);
            } else {
              ok = nearest_exact<SORD, TSIP>(P, x, y, bx, by, px, py, dbx, dby);
              exact = ok;
            }
          }
        }
        R.rx[k][e] = px;
        R.ry[k][e] = py;
        if (G.debug) debug_position(G, x, y, ok, exact, dbx, dby, bx, by, px, py);
        if (ok) R.valid |= 1u << (k * kRun + e);
      }
    }
  }
}

// Phase 4: interpolation from the staged box (the caller has waited for its
// DMA and synchronised), results to the sink.
template <int INTERP, int NP, class Sink>
__device__ __forceinline__ void tile_gather(const FramePlan &P, const TileGeom &G,
                                            const TileXY &T, const TileBox &B,
                                            const float *__restrict__ lds, const FwdPos<NP> &R,
                                            Sink &sink) {
  constexpr int SPAN = TapSupport<INTERP>::lo + TapSupport<INTERP>::hi;
  const int W = P.src_w, Hs = P.src_h;
  const int xr = T.xr, lp = B.lp;
  const bool vec = vector_stores_ok(P, G);
  const float miss = G.nan_outside ? __builtin_nanf("") : 0.0f;
  // Interior tiles need no per-pixel check: the box holds every tap by the
  // rigorous margin of the cells' models.
  const bool fast = B.interior && R.valid == ~0u;
  const float a = G.cubic_a;
  if (fast) {
    // box-relative tap coordinates: unmasked LDS reads from one base address
    // per pixel, footprint exactly 1
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const int y = T.y0 + T.ty + k * T.RP;
      float o[kRun], f[kRun];
#pragma unroll
      for (int e = 0; e < kRun; ++e) {
        int i0, j0;
        float t_, s_;
        tap_origin<INTERP>(R.rx[k][e], R.abx[k], i0, t_);
        tap_origin<INTERP>(R.ry[k][e], R.aby[k], j0, s_);
        // i0, j0 >= 0 inside the box: one 24-bit multiply-add per pixel
        const float *__restrict__ b = lds + __umul24(j0, lp) + i0;
        auto fl = [&](int i, int j) -> float { return b[j * lp + i]; };
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
      sink.row(P, G, k, y, xr, vec, true, o, f);
    }
    return;
  }
  // general path: source coordinates, zero padding, footprint normalisation;
  // taps come from LDS when the pixel's in-image taps are inside the box
  const int bi0 = B.bi0, bi1 = B.bi1, bj0 = B.bj0, bj1 = B.bj1;
  auto fl = [&](int i, int j) -> float { return lds[__umul24(j - bj0, lp) + (i - bi0)]; };
  auto fg = [&](int i, int j) -> float { return global_ptr(P.src)[(int64_t)j * P.pitch + i]; };
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int y = T.y0 + T.ty + k * T.RP;
    if (y >= G.out_h || xr >= G.out_w) continue;
    float o[kRun], f[kRun];
#pragma unroll
    for (int e = 0; e < kRun; ++e) {
      o[e] = miss;
      f[e] = 0.0f;
      if (R.valid & (1u << (k * kRun + e))) {
        int i0, j0;
        float t_, s_;
        tap_origin<INTERP>(R.rx[k][e], R.abx[k] + bi0, i0, t_);
        tap_origin<INTERP>(R.ry[k][e], R.aby[k] + bj0, j0, s_);
        const bool in_lds = B.use_lds && max(i0, 0) >= bi0 && min(i0 + SPAN, W - 1) <= bi1 &&
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
    sink.row(P, G, k, y, xr, vec, false, o, f);
  }
}

// A tile of a cropped frame no pixel of which reaches the source.
template <int NP>
__device__ __forceinline__ void CropSink::uncovered(const FramePlan &P, const TileGeom &G,
                                                    int tile) {
  const TileXY T = tile_xy<NP>(G, tile);
  const float miss = G.nan_outside ? __builtin_nanf("") : 0.0f;
  float zo[kRun], zf[kRun];
#pragma unroll
  for (int e = 0; e < kRun; ++e) {
    zo[e] = miss;
    zf[e] = 0.0f;
  }
#pragma unroll
  for (int k = 0; k < NP; ++k) row(P, G, k, T.y0 + T.ty + k * T.RP, T.xr, false, false, zo, zf);
}

// Nearest, after the gather: the pixels flagged in `tie` (bit k * kRun + e
// for pixel e of run k) are rounded from an FP64 position and stored again,
// with that position for the debug output.  In a cell with a certified
// model the model is evaluated in FP64 first: it lies within M.err of the
// map, so where both coordinates are farther than M.err + 1e-9 px from a
// rounding tie it decides exactly as the FP64 chain would (whose own error
// is far below 1e-9 px); only the rest take the full FP64 chain.  A wave's vector
// stores are performed in the order it issues them, so the correction is
// the last write to its address without waiting for the earlier stores; the
// source value comes from the staged box (still intact: the group has not
// passed its next barrier), so no vector-memory load has to wait behind
// those stores either (on this architecture one counter covers loads and
// stores).  It runs at the end of the tile, where little else is live, so
// the FP64 chain adds no registers to the tile's main work.
template <int SORD, int NP, class Sink>
__device__ __forceinline__ void nearest_ties(const FramePlan &P, const TileGeom &G,
                                             const TileXY &T, const FwdShared &sh,
                                             const TileBox &B, const float *__restrict__ lds,
                                             unsigned tie, Sink &sink) {
  constexpr bool TSIP = SORD == kRtOrder;
  const float miss = G.nan_outside ? __builtin_nanf("") : 0.0f;
  while (tie) {
    const int bit = __builtin_ctz(tie);
    tie &= tie - 1u;
    const int k = bit / kRun, e = bit % kRun;
    const int y = T.y0 + T.ty + k * T.RP, x = T.xr + e;
    const int ci = ((y >> kCellLog2) - T.cy0) * T.ncx + ((T.xr >> kCellLog2) - T.cx0);
    const bool mk = sh.kind[ci] != 0;
    const int bx = mk ? sh.cell[ci].model.bx : sh.cell[ci].anchor.bx;
    const int by = mk ? sh.cell[ci].model.by : sh.cell[ci].anchor.by;
    float px = 0.0f, py = 0.0f;
    double xs = 0.0, ys = 0.0;
    bool decided = false;
    if (mk) {
      const CellModel &M = sh.cell[ci].model;
      const double a = (double)(x & (kCell - 1)) - kHalfCell;
      const double b = (double)(y & (kCell - 1)) - kHalfCell;
      const double mxv = model_f64(M.mx, a, b), myv = model_f64(M.my, a, b);
      const double tol = (double)M.err + 1.0e-9;
      if (fabs(mxv - floor(mxv) - 0.5) > tol && fabs(myv - floor(myv) - 0.5) > tol) {
        px = (float)rint(mxv);
        py = (float)rint(myv);
        xs = (double)bx + mxv;
        ys = (double)by + myv;
        decided = true;
      }
    }
    const bool ok = decided || nearest_exact<SORD, TSIP>(P, x, y, bx, by, px, py, xs, ys);
    float o = miss, f = 0.0f;
    if (ok) {
      const int i = bx + (int)px, j = by + (int)py;
      if ((unsigned)i < (unsigned)P.src_w && (unsigned)j < (unsigned)P.src_h) {
        if (B.use_lds && i >= B.bi0 && i <= B.bi1 && j >= B.bj0 && j <= B.bj1)
          o = lds[__umul24(j - B.bj0, B.lp) + (i - B.bi0)];
        else
          o = global_ptr(P.src)[(int64_t)j * P.pitch + i];
        f = 1.0f;
      }
    }
    if (G.debug) debug_position(G, x, y, ok, true, xs, ys, bx, by, px, py);
    sink.pixel(P, G, y, x, o, f);
  }
}

// One tile of one frame: the four phases in order.
template <int INTERP, int SORD, int NP, class Sink>
__device__ __forceinline__ void forward_tile(const FramePlan &P, const TileGeom &G, int tile,
                                             float *__restrict__ lds, FwdShared &sh, Sink &sink) {
  constexpr bool kDefer = INTERP == DFR_NEAREST && Sink::kDeferTies;
  const TileXY T = tile_xy<NP>(G, tile);
  if ((threadIdx.x >> 6) == 0) tile_cells<INTERP, SORD, NP>(P, G, T, sh);
  __syncthreads();
  if (!sh.touch && G.allow_skip) {
    sink.template uncovered<NP>(P, G, tile);
    return;
  }
  const TileBox B = tile_box<NP>(P, G, T, sh, G.lds_cap);
  if (B.use_lds) dma_box(P, B.bi0, B.bj0, B.bw, B.bh, B.lp, lds);
  FwdPos<NP> R;
  tile_positions<INTERP, SORD, NP, kDefer>(P, G, T, sh, B, R);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  tile_gather<INTERP, NP>(P, G, T, B, lds, R, sink);
  if constexpr (kDefer) {
    if (R.tie) nearest_ties<SORD, NP>(P, G, T, sh, B, lds, R.tie, sink);
  }
}

}  // namespace dfr
