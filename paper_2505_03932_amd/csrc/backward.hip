// Backward pass of the FP32 reprojection (not in the paper: it turns the
// reprojection into a differentiable step so WCS alignment can be refined
// by gradient descent on image residuals).
//
// For a loss L with g = dL/dout:
//   dL/dsrc_k = sum_p g_p w_kp / F_p       -- adjoint of the interpolation, a
//                                            scatter-add of contributions
//                                            rounded to a fixed grid and
//                                            summed exactly in 64-bit
//                                            integers (in an LDS copy of the
//                                            tile's source box, then one
//                                            global atomic per touched source
//                                            pixel), so the result does not
//                                            depend on the order of the adds;
//   dL/dpos_p  = g_p (dS/dpos - out dF/dpos) / F
// and through the map pos = (U, V) + SIP(U, V) + CRPIX - 1 with
// (U, V) = (p/w, q/w), (p, q, w) = H t:
//   dL/dH_1j = sum a t_j / w,  dL/dH_2j = sum b t_j / w,
//   dL/dH_3j = -sum (a U + b V) t_j / w,
// a = dL/dU, b = dL/dV; plus dL/dCRPIX and the AP/BP monomial sums.  These
// are reduced per wave, then per work-group into FP64 partials, then in a
// fixed order (deterministic), and chained to CRVAL and CD on the device
// with the FP64 Jacobian dH/d(CRVAL, CD) composed on the host.
#include "forward_body.hpp"
#include "launch.hpp"

namespace dfr {

// ---- tile set-up of the backward kernel (anchors, exact tap box, staging)

// LDS scratch of a tile kernel besides the dynamic source tile.
struct TileShared {
  Anchor anchor[kMaxAnchors];
  int box[4];     // imin, imax, jmin, jmax of the source box
  int touch;      // any anchor cell can reach the source
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

// A backward tile works from its cells' FP64 anchors (the WCS gradient
// needs the projective intermediates of every pixel), computes every
// pixel's position and the exact box of its in-image taps, and copies that
// box into LDS.
//
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
__device__ __forceinline__ void anchor_positions(const FramePlan &P, const TileGeom &G,
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
                                          int lp, float *__restrict__ lds) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const auto *__restrict__ s0 = global_ptr(P.src) + (int64_t)bj0 * P.pitch + bi0;
  for (int r = wave; r < bh; r += kThreads / 64) {
    const auto *__restrict__ sr = s0 + (int64_t)r * P.pitch;
    float *__restrict__ lr = lds + r * lp;
    for (int col = lane; col < bw; col += 64) lr[col] = sr[col];
  }
}

// ---- per-pixel adjoint

// FLAT: the taps come from a staged box through `flat` (index(i, j), then
// value(idx) and add(idx, v) at idx + l * pitch + k), used where every tap
// is inside the source: no per-tap test, one address per row.  The same
// arithmetic in the same order as the general loop, so the same bits.
template <int INTERP, bool FLAT, typename Fetch, typename Scatter, typename Flat>
__device__ __forceinline__ bool interp_backward(int bx, int by, float rx, float ry, int W, int H,
                                                float a, float g, const Fetch &fetch,
                                                const Scatter &scatter, const Flat &flat,
                                                float &gx, float &gy) {
  gx = 0.0f;
  gy = 0.0f;
  if constexpr (INTERP == DFR_NEAREST) {
    int i = bx + (int)rintf(rx), j = by + (int)rintf(ry);
    bool in = ((unsigned)i < (unsigned)W) && ((unsigned)j < (unsigned)H);
    if (in) scatter(0, 0, i, j, flat.scaled(g));
    return in;
  } else {
    constexpr int NT = INTERP == DFR_BILINEAR ? 2 : 4;
    float fx = floorf(rx), fy = floorf(ry);
    float t = rx - fx, s = ry - fy;
    int i0 = bx + (int)fx - (NT == 4 ? 1 : 0), j0 = by + (int)fy - (NT == 4 ? 1 : 0);
    float wx[4], wy[4], dx[4], dy[4];
    if constexpr (NT == 2) {
      wx[0] = 1.0f - t; wx[1] = t; dx[0] = -1.0f; dx[1] = 1.0f;
      wy[0] = 1.0f - s; wy[1] = s; dy[0] = -1.0f; dy[1] = 1.0f;
    } else {
      keys_weights(t, a, wx);
      keys_weights(s, a, wy);
      keys_dweights(t, a, dx);
      keys_dweights(s, a, dy);
    }
    if constexpr (FLAT) {
      if (W >= NT && H >= NT && (unsigned)i0 <= (unsigned)(W - NT) &&
          (unsigned)j0 <= (unsigned)(H - NT)) {
        const int base = flat.index(i0, j0);
        const float gs = flat.scaled(g);
        float gw[NT];
#pragma unroll
        for (int k = 0; k < NT; ++k) gw[k] = gs * wx[k];
        float S = 0.0f, Sx = 0.0f, Sy = 0.0f;
#pragma unroll
        for (int l = 0; l < NT; ++l) {
          const int rb = base + l * flat.pitch();
          float row = 0.0f, rowd = 0.0f;
#pragma unroll
          for (int k = 0; k < NT; ++k) {
            const float v = flat.value(rb + k);
            row = fmaf(wx[k], v, row);
            rowd = fmaf(dx[k], v, rowd);
            flat.add_scaled(rb + k, gw[k] * wy[l]);
          }
          S = fmaf(wy[l], row, S);
          Sx = fmaf(wy[l], rowd, Sx);
          Sy = fmaf(dy[l], row, Sy);
        }
        gx = g * Sx;
        gy = g * Sy;
        return true;
      }
    }
    bool inx[NT], iny[NT];
    bool all_in = true;
    float Fx = 0.0f, Fy = 0.0f, dFx = 0.0f, dFy = 0.0f;
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      inx[k] = (unsigned)(i0 + k) < (unsigned)W;
      iny[k] = (unsigned)(j0 + k) < (unsigned)H;
      all_in = all_in && inx[k] && iny[k];
      wx[k] = inx[k] ? wx[k] : 0.0f;
      dx[k] = inx[k] ? dx[k] : 0.0f;
      wy[k] = iny[k] ? wy[k] : 0.0f;
      dy[k] = iny[k] ? dy[k] : 0.0f;
      Fx += wx[k];
      Fy += wy[k];
      dFx += dx[k];
      dFy += dy[k];
    }
    float F = all_in ? 1.0f : Fx * Fy;
    if (!(F > 0.0f)) return false;
    float iF = all_in ? 1.0f : __builtin_amdgcn_rcpf(F);
    float c = g * iF;
    const float cs = flat.scaled(c);  // the source adjoint's contributions, times 2^Q
    // Where taps leave the source, d out = (dS - out dF) / F cancels the
    // level of the values; taking every value relative to one in-bounds tap
    // (exact: the in-bounds taps form a product set, so both dS and out dF
    // move by vr dF) leaves a rounding relative to the local contrast
    // instead.  Interior pixels use vr = 0.
    float vr = 0.0f;
    if (!all_in) {
      int kr = 0, lr = 0;
#pragma unroll
      for (int k = NT - 1; k >= 0; --k) {
        if (inx[k]) kr = k;
        if (iny[k]) lr = k;
      }
      vr = fetch(i0 + kr, j0 + lr);  // F > 0: some tap is in bounds on each axis
    }
    float S = 0.0f, Sx = 0.0f, Sy = 0.0f;
#pragma unroll
    for (int l = 0; l < NT; ++l) {
      float row = 0.0f, rowd = 0.0f;
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        if (inx[k] && iny[l]) {
          float v = fetch(i0 + k, j0 + l) - vr;
          row = fmaf(wx[k], v, row);
          rowd = fmaf(dx[k], v, rowd);
          scatter(k, l, i0 + k, j0 + l, cs * wx[k] * wy[l]);
        }
      }
      S = fmaf(wy[l], row, S);
      Sx = fmaf(wy[l], rowd, Sx);
      Sy = fmaf(dy[l], row, Sy);
    }
    float out = S * iF;
    float Fdx = all_in ? 0.0f : dFx * Fy, Fdy = all_in ? 0.0f : Fx * dFy;
    gx = g * (Sx - out * Fdx) * iF;
    gy = g * (Sy - out * Fdy) * iF;
    return true;
  }
}

// Source adjoint: every contribution v = g w / F is rounded to a
// multiple of 2^-Q (Q fixed per call from max |g|: 2^-Q = 2^-30 max |g|,
// rounded to a power of two) and the multiples are summed in 64-bit
// integers.  Integer sums do not depend on the order or the grouping of
// the additions, so the result is the same bits for every run and every
// tile shape; 64-bit LDS integer adds are also much faster here than
// ds_add_f32 on contended addresses (measured: 148 against 382 us per
// 2048^2 bicubic backward with one add per tap).  The rounding (at most
// 2^-31 max |g| per contribution) stays far below an FP32 sum's; where
// every tap is inside the source |v| 2^Q < 2^31, one 32-bit conversion;
// |v| beyond 2^32 max |g| (footprints below ~2.3e-10 at frame edges)
// saturates at +-2^62.
constexpr int kDetBits = 30;
__device__ __forceinline__ double det_scale(const int *__restrict__ gmax_bits) {
  const float m = __int_as_float(*gmax_bits);
  return m > 0.0f ? ldexp(1.0, kDetBits - ilogbf(m)) : 1.0;
}

// The same scale as an exponent: 2^Q.
__device__ __forceinline__ int det_exponent(const int *__restrict__ gmax_bits) {
  const float m = __int_as_float(*gmax_bits);
  return m > 0.0f ? kDetBits - ilogbf(m) : 0;
}

// An FP32 integer of at most 63 bits as a 64-bit integer, split exactly
// into 32-bit halves.
__device__ __forceinline__ unsigned long long det_int(float y) {
  const double d = (double)y;
  const double hi = floor(d * 0x1p-32);
  const double lo = fma(hi, -0x1p32, d);
  return ((unsigned long long)(unsigned)(int)hi << 32) | (unsigned long long)(unsigned)lo;
}

// A contribution already scaled by 2^Q (formed as (g/F 2^Q) wx wy: the
// scaling of g/F is exact), rounded to the nearest integer in FP32 and
// saturated at +-2^62.
__device__ __forceinline__ unsigned long long det_quant(float y) {
  return det_int(rintf(__builtin_amdgcn_fmed3f(y, -0x1p62f, 0x1p62f)));
}

// A pixel's taps in the staged box and, for the source adjoint, its 64-bit
// integer accumulation copy (same index, same row stride).  On this path
// every tap is inside the source (F = 1): |g| 2^Q < 2^31 and |wx wy| <= 1,
// and each rounded product is at most |g| 2^Q, so a contribution is an
// integer below 2^31 in magnitude: one 32-bit conversion, no saturation.
// The contributions are formed exactly as on the general path, so a pixel
// gives the same integers on either.
template <bool SRC>
struct BwdFlat {
  const float *vals;
  unsigned long long *qacc;
  int lp, bi0, bj0, Q;
  __device__ int index(int i, int j) const { return (j - bj0) * lp + (i - bi0); }
  __device__ int pitch() const { return lp; }
  __device__ float value(int idx) const { return vals[idx]; }
  __device__ float scaled(float g) const { return ldexpf(g, Q); }
  // y = (g 2^Q wx) wy
  __device__ void add_scaled(int idx, float y) const {
    if constexpr (SRC)
      atomicAdd(&qacc[idx], (unsigned long long)(long long)(int)rintf(y));
  }
};

// The two halves of a lane-swap pair summed: permlane32 (lanes 0-31 get
// a(i) + a(i + 32), lanes 32-63 get b(i - 32) + b(i)) or permlane16 (rows
// 0 and 2 of 16 lanes get a's pairs of rows 0+1 and 2+3, rows 1 and 3 get
// b's).  The empty asm makes the swap's two results opaque: without it
// this compiler folds r[0] + r[1] into r[0] + r[0].
template <bool ROWS16>
__device__ __forceinline__ float swap_sum(float a, float b) {
  const auto r = ROWS16 ? __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, a),
                                                           __builtin_bit_cast(unsigned, b),
                                                           false, false)
                        : __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, a),
                                                           __builtin_bit_cast(unsigned, b),
                                                           false, false);
  unsigned r0 = r[0], r1 = r[1];
  asm volatile("" : "+v"(r0), "+v"(r1));
  return __builtin_bit_cast(float, r0) + __builtin_bit_cast(float, r1);
}

// SRC: the source gradient is wanted (its integer sums go to gq,
// [src_h][src_w] dense; bwd_finish_kernel converts them); without it the
// kernel carries no scatter code at all.
template <int INTERP, int SORD, int NP, bool TSIP, bool SRC>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(NP == 1 ? 5 : 1)))
void reproject_bwd(FramePlan P, TileGeom G,
                                                          const float *__restrict__ gout,
                                                          double *__restrict__ partials,
                                                          unsigned long long *__restrict__ gq,
                                                          const int *__restrict__ gmax_bits) {
  constexpr int NC = (SORD + 1) * (SORD + 2) / 2;
  constexpr int NS = 11 + 2 * NC;
  extern __shared__ float lds[];
  __shared__ TileShared sh;
  __shared__ float wsum[kThreads / 64][NS];
  const int tile = xcd_tile(blockIdx.x, G.n_tiles);
  const int tid = threadIdx.x;
  float acc[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) acc[s] = 0.0f;

  TileCtx c;
  if (tile_anchors<INTERP, SORD, TSIP, NP>(P, G, tile, sh, c)) {
    TilePos<NP> T;
    anchor_positions<INTERP, SORD, TSIP, NP>(P, G, sh, c, T);
    const int bw = T.empty ? 0 : T.bi1 - T.bi0 + 1;
    const int bh = T.empty ? 0 : T.bj1 - T.bj0 + 1;
    const int lp = lds_pitch(bw);  // padded row stride (bank spread)
    constexpr bool want_src = SRC;
    const int qs = SRC ? det_exponent(gmax_bits) : 0;
    // LDS: the staged box, then the 64-bit integer accumulation box (8-byte
    // aligned, two floats per entry)
    const int lp_acc = 2 * lp;
    const bool use_lds = !T.empty && (want_src ? 3 : 1) * (int64_t)lp * bh + 2 <=
                                         (int64_t)G.lds_cap;
    float *vals = lds;
    float *gacc = lds + (use_lds ? ((lp * bh + 1) & ~1) : 0);
    unsigned long long *qacc = reinterpret_cast<unsigned long long *>(gacc);
    if (use_lds) {
      stage_box(P, T.bi0, T.bj0, bw, bh, lp, vals);
      if (want_src)
        for (int i = tid; i < lp_acc * bh; i += kThreads) gacc[i] = 0.0f;
    }
    __syncthreads();
    const int W = P.src_w, Hs = P.src_h;
    const int bi0 = T.bi0, bj0 = T.bj0;
    auto fetch_lds = [&](int i, int j) -> float { return vals[(j - bj0) * lp + (i - bi0)]; };
    auto fetch_glb = [&](int i, int j) -> float { return P.src[(int64_t)j * P.pitch + i]; };
    auto scat_lds = [&](int, int, int i, int j, float v) {
      if (want_src) atomicAdd(&qacc[(j - bj0) * lp + (i - bi0)], det_quant(v));
    };
    auto scat_glb = [&](int, int, int i, int j, float v) {
      if (want_src) atomicAdd(&gq[(int64_t)j * W + i], det_quant(v));
    };
    const BwdFlat<SRC> flat{vals, qacc, lp, bi0, bj0, qs};
    const float tinv = (float)P.t_inv_scale, sinv = (float)P.s_inv_scale;
    const float S_s = (float)P.s_scale;
    // Every tap's contribution is quantised and added on its own (64-bit
    // integer LDS adds are cheap; summing a run's taps in a register window
    // first measured slower, the window's registers costing occupancy).
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const int y = c.y0 + c.ty + k * c.RP;
      // the run's interpolant gradients; the WCS terms are formed from them
      // after the run's scatter, so the scatter's and the WCS sums'
      // registers are not live together
      float gxs[kRun], gys[kRun];
      unsigned covm = 0u;
#pragma unroll
      for (int e = 0; e < kRun; ++e) {
        gxs[e] = 0.0f;
        gys[e] = 0.0f;
        if (!(T.valid & (1u << (k * kRun + e)))) continue;
        const int x = c.xr + e;
        const float g = gout[(int64_t)y * G.out_w + x];
        if (g == 0.0f) continue;
        float gx, gy;
        bool cov;
        if (use_lds)
          cov = interp_backward<INTERP, true>(T.abx[k], T.aby[k], T.rx[k][e], T.ry[k][e], W, Hs,
                                              G.cubic_a, g, fetch_lds, scat_lds, flat, gx, gy);
        else
          cov = interp_backward<INTERP, false>(T.abx[k], T.aby[k], T.rx[k][e], T.ry[k][e], W,
                                               Hs, G.cubic_a, g, fetch_glb, scat_glb, flat, gx,
                                               gy);
        if (cov) {
          gxs[e] = gx;
          gys[e] = gy;
          covm |= 1u << e;
        }
      }
      if constexpr (INTERP != DFR_NEAREST) {
        // the WCS terms of the run's covered pixels, in pixel order
        const Anchor &A = sh.anchor[T.aidx[k]];
#pragma unroll
        for (int e = 0; e < kRun; ++e) {
          if (!(covm & (1u << e))) continue;
          const float gx = gxs[e], gy = gys[e];
          // the projective intermediates of the pixel (its position is known)
          PixelGeom pg;
          float den;
          pixel_geom<TSIP>(P, A, tinv, sinv, (float)((c.xr & (kCell - 1)) + e),
                           (float)(y & (kCell - 1)), pg, den);
          float fa, fau, fav, fb, fbu, fbv;
          sip_f32_grad<SORD>(P.fsA, pg.us, pg.vs, fa, fau, fav);
          sip_f32_grad<SORD>(P.fsB, pg.us, pg.vs, fb, fbu, fbv);
          const float da = gx * fmaf(fau, sinv, 1.0f) + gy * (fbu * sinv);  // dL/dU
          const float db = gx * (fav * sinv) + gy * fmaf(fbv, sinv, 1.0f);  // dL/dV
          const float U = pg.us * S_s, V = pg.vs * S_s;
          const float iw = A.inv_w0 * pg.r;
          const float t0 = A.tu0 + pg.du, t1 = A.tv0 + pg.dv;
          const float a1 = da * iw, b1 = db * iw, c1 = -(da * U + db * V) * iw;
          acc[0] = fmaf(a1, t0, acc[0]);
          acc[1] = fmaf(a1, t1, acc[1]);
          acc[2] += a1;
          acc[3] = fmaf(b1, t0, acc[3]);
          acc[4] = fmaf(b1, t1, acc[4]);
          acc[5] += b1;
          acc[6] = fmaf(c1, t0, acc[6]);
          acc[7] = fmaf(c1, t1, acc[7]);
          acc[8] += c1;
          acc[9] += gx;
          acc[10] += gy;
          if constexpr (SORD > 0) {
            float up = 1.0f;
#pragma unroll
            for (int p = 0; p <= SORD; ++p) {
              float m = up;
#pragma unroll
              for (int q = 0; p + q <= SORD; ++q) {
                acc[11 + tri_n(SORD, p, q)] = fmaf(gx, m, acc[11 + tri_n(SORD, p, q)]);
                acc[11 + NC + tri_n(SORD, p, q)] = fmaf(gy, m, acc[11 + NC + tri_n(SORD, p, q)]);
                m *= pg.vs;
              }
              up *= pg.us;
            }
          }
        }
      }
    }
    __syncthreads();
    if (SRC && use_lds) {
      const int wave = tid >> 6, lane = tid & 63;
      for (int r = wave; r < bh; r += kThreads / 64)
        for (int col = lane; col < bw; col += 64) {
          const unsigned long long q = qacc[r * lp + col];
          if (q != 0ull) atomicAdd(&gq[(int64_t)(bj0 + r) * W + bi0 + col], q);
        }
    }
  }
  // per-wave, then per-group sums of the WCS terms (skipped tiles give 0):
  // a transposing butterfly halves the number of live sums at each lane
  // exchange (lanes i, i + 32, then rows 0/1 and 2/3 of 16 lanes), so each
  // row of the wave ends with a quarter of the sums, which DPP shifts
  // reduce within the row (lane 15 holds the row's total).  Fixed order.
  {
    constexpr int NSP = NS <= 16 ? 16 : (NS <= 32 ? 32 : 64);
    constexpr int H = NSP / 2, Q = NSP / 4;
    static_assert(NS <= 64, "WCS sums per wave");
    float x[H];
#pragma unroll
    for (int s = 0; s < H; ++s) {
      // lanes 0-31: sum s over lanes i and i + 32; lanes 32-63: sum s + H
      x[s] = swap_sum<false>(acc[s], s + H < NS ? acc[s + H] : 0.0f);
    }
    float y[Q];
#pragma unroll
    for (int s = 0; s < Q; ++s) {
      // row 0: sum s, row 1: s + Q, row 2: s + H, row 3: s + H + Q
      float v = swap_sum<true>(x[s], x[s + Q]);
      v = dpp_add<0x111, 0xf>(v);  // row_shr:1
      v = dpp_add<0x112, 0xf>(v);  // row_shr:2
      v = dpp_add<0x114, 0xf>(v);  // row_shr:4
      y[s] = dpp_add<0x118, 0xf>(v);  // row_shr:8
    }
    const int lane = tid & 63, row = lane >> 4;
    if ((lane & 15) == 15) {
      const int off = row == 0 ? 0 : (row == 1 ? Q : (row == 2 ? H : H + Q));
#pragma unroll
      for (int s = 0; s < Q; ++s)
        if (s + off < NS) wsum[tid >> 6][s + off] = y[s];
    }
  }
  __syncthreads();
  if (tid < NS) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) t += (double)wsum[w][tid];
    partials[(int64_t)tid * G.n_tiles + tile] = t;  // column-major: one column per sum
  }
}

using BwdKernel = void (*)(FramePlan, TileGeom, const float *, double *, unsigned long long *,
                          const int *);

template <int INTERP, int NP, bool TSIP, bool SRC>
static BwdKernel bwd_sord(int sord) {
  switch (sord) {
    case 0: return reproject_bwd<INTERP, 0, NP, TSIP, SRC>;
    case 1: return reproject_bwd<INTERP, 1, NP, TSIP, SRC>;
    case 2: return reproject_bwd<INTERP, 2, NP, TSIP, SRC>;
    case 3: return reproject_bwd<INTERP, 3, NP, TSIP, SRC>;
    case 4: return reproject_bwd<INTERP, 4, NP, TSIP, SRC>;
    default: return reproject_bwd<INTERP, 5, NP, TSIP, SRC>;
  }
}

// The backward kernel runs 1 or 2 rows per thread (the host picks such
// tiles); the target SIP is compiled in only where the target has one.
template <int INTERP>
static BwdKernel bwd_pick(int np, int sord, bool tsip, bool src) {
  if (src) {
    if (tsip) return np == 1 ? bwd_sord<INTERP, 1, true, true>(sord) : bwd_sord<INTERP, 2, true, true>(sord);
    return np == 1 ? bwd_sord<INTERP, 1, false, true>(sord) : bwd_sord<INTERP, 2, false, true>(sord);
  }
  if (tsip) return np == 1 ? bwd_sord<INTERP, 1, true, false>(sord) : bwd_sord<INTERP, 2, true, false>(sord);
  return np == 1 ? bwd_sord<INTERP, 1, false, false>(sord) : bwd_sord<INTERP, 2, false, false>(sord);
}

hipError_t launch_backward(const FramePlan &P, const TileGeom &G, int interp, int np,
                           const float *grad_out, double *partials, unsigned long long *src_acc,
                           const int *gmax_bits, hipStream_t stream) {
  if (G.n_tiles <= 0) return hipSuccess;
  const bool tsip = P.t_order > 0;
  const bool src = src_acc != nullptr;
  BwdKernel k = interp == DFR_NEAREST    ? bwd_pick<DFR_NEAREST>(np, P.s_order, tsip, src)
                : interp == DFR_BILINEAR ? bwd_pick<DFR_BILINEAR>(np, P.s_order, tsip, src)
                                         : bwd_pick<DFR_BICUBIC>(np, P.s_order, tsip, src);
  size_t lds = (size_t)G.lds_cap * sizeof(float);
  hipLaunchKernelGGL(k, dim3(G.n_tiles), dim3(kThreads), lds, stream, P, G, grad_out, partials,
                     src_acc, gmax_bits);
  return hipGetLastError();
}

// Before the backward kernel, for the source adjoint, in one launch: the
// 64-bit integer image is zeroed and max |g| over the output gradient is
// folded into *gmax as the bits of a non-negative float (their integer
// order is the float order, so atomicMax gives the same result in any
// order).  *gmax is 0 on entry; *gmax_next, the slot the next call uses, is
// zeroed here (the previous call's kernels, which read it, have finished).
__global__ __launch_bounds__(256) void det_prepare_kernel(const float *__restrict__ g, int64_t n,
                                                          unsigned long long *__restrict__ q,
                                                          int64_t nq, int *__restrict__ gmax,
                                                          int *__restrict__ gmax_next) {
  __shared__ float wm[4];
  const int64_t stride = (int64_t)gridDim.x * 256;
  const int64_t i0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i0 == 0) *gmax_next = 0;
  // the image is 16-byte aligned (a 256-byte aligned workspace offset)
  typedef unsigned long long u2v __attribute__((ext_vector_type(2)));
#pragma unroll 4
  for (int64_t i = i0; i < nq / 2; i += stride) reinterpret_cast<u2v *>(q)[i] = u2v{0ull, 0ull};
  if (i0 == 0 && (nq & 1)) q[nq - 1] = 0ull;
  float m = 0.0f;
  // 16-byte loads where the gradient is aligned, then the tail
  typedef float f4v __attribute__((ext_vector_type(4)));
  const int64_t n4 = (reinterpret_cast<uintptr_t>(g) & 15) == 0 ? n / 4 : 0;
#pragma unroll 4
  for (int64_t i = i0; i < n4; i += stride) {
    const f4v v = reinterpret_cast<const f4v *>(g)[i];
    m = fmaxf(fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y))), fmaxf(fabsf(v.z), fabsf(v.w)));
  }
  for (int64_t i = 4 * n4 + i0; i < n; i += stride) m = fmaxf(m, fabsf(g[i]));
  m = wave_max_f(m);
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]));
    // one atomic per block, few blocks: atomics on one address serialise
    if (m > 0.0f) atomicMax(gmax, __float_as_int(m));
  }
}

hipError_t launch_det_prepare(const float *grad_out, int64_t n, unsigned long long *q, int64_t nq,
                              int *gmax, int *gmax_next, hipStream_t stream) {
  const int64_t work = std::max<int64_t>(n / 4, nq / 2);
  hipLaunchKernelGGL(det_prepare_kernel,
                     dim3((unsigned)std::min<int64_t>(512, std::max<int64_t>(1, (work + 255) / 256))),
                     dim3(256), 0, stream, grad_out, n, q, nq, gmax, gmax_next);
  return hipGetLastError();
}

// Column c of the partials ([ns][n_blocks], column-major), summed by one
// block in a fixed order (256 strided partial sums, then a tree); the
// result is in sm[0].
__device__ __forceinline__ void column_sum(const FinishArgs &A, int c, double *sm) {
  const int tid = threadIdx.x;
  double a = 0.0;
  const double *col = A.partials + (int64_t)c * A.n_blocks;
#pragma unroll 4
  for (int k = tid; k < A.n_blocks; k += 256) a += col[k];
  sm[tid] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) sm[tid] += sm[tid + w];
    __syncthreads();
  }
}

// After the backward kernel, in one launch with no block depending on
// another.  With WCS gradients (nr = ns - 10 blocks): block 0 sums the nine
// dH and two CRPIX columns and applies the chain rule to CRVAL, CRPIX and CD
// (dH/dtheta), and writes the AP/BP entries of the square layouts that lie
// above their order (zero); block 1 + k sums SIP column 11 + k and writes its
// entry, scaled by S^(p+q) (A.col_entry / A.col_deg; -1: a padded column).
// The remaining blocks convert rows of the integer sums to grad_src =
// q 2^-Q.  Grad entries follow dfr_wcs_grad_size: CRVAL(2), CRPIX(2), CD(4),
// AP, BP.
__global__ __launch_bounds__(256) void bwd_finish_kernel(FinishArgs A) {
  __shared__ double sm[11 * 256];
  __shared__ double tot[11];
  const int b = blockIdx.x, tid = threadIdx.x;
  if (b >= A.nr) {
    const double inv = 1.0 / det_scale(A.gmax);
    const int nc = (int)gridDim.x - A.nr;
    for (int64_t r = b - A.nr; r < A.h; r += nc) {
      const unsigned long long *qr = A.q + r * A.w;
      float *gr = A.gsrc + r * A.gpitch;
      for (int64_t c = tid; c < A.w; c += 256) gr[c] = (float)((double)(long long)qr[c] * inv);
    }
    return;
  }
  if (b > 0) {
    const int k = b - 1;
    column_sum(A, 11 + k, sm);
    if (tid == 0 && A.col_entry[k] >= 0) {
      double sc = 1.0;
      for (int i = 0; i < A.col_deg[k]; ++i) sc *= A.S;
      A.grad_wcs[A.col_entry[k]] = sm[0] * sc;
    }
    return;
  }
  // the 11 leading columns side by side (one load of each per row, so
  // eleven are in flight together), then 11 trees side by side
  double a[11];
#pragma unroll
  for (int c = 0; c < 11; ++c) a[c] = 0.0;
  const int64_t nb = A.n_blocks;
#pragma unroll 2
  for (int k = tid; k < A.n_blocks; k += 256) {
#pragma unroll
    for (int c = 0; c < 11; ++c) a[c] += A.partials[c * nb + k];
  }
#pragma unroll
  for (int c = 0; c < 11; ++c) sm[c * 256 + tid] = a[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
#pragma unroll
      for (int c = 0; c < 11; ++c) sm[c * 256 + tid] += sm[c * 256 + tid + w];
    }
    __syncthreads();
  }
  if (tid < 11) tot[tid] = sm[tid * 256];
  __syncthreads();
  if (tid < 8) {
    if (tid < 2 || tid >= 4) {
      // CRVAL_k (tid < 2) or CD_kl (tid = 4 + kl) through dH/dtheta
      const int row = tid < 2 ? tid : 2 + (tid - 4);
      double g = 0.0;
      for (int i = 0; i < 9; ++i) g += tot[i] * A.J.dh[row * 9 + i];
      A.grad_wcs[tid] = g;
    } else {
      A.grad_wcs[tid] = tot[9 + (tid - 2)];  // CRPIX
    }
  }
  for (int t = tid; t < A.n_above; t += 256) A.grad_wcs[A.above[t]] = 0.0;
}

hipError_t launch_backward_finish(const FinishArgs &A, hipStream_t stream) {
  const int nc = A.q ? (int)std::min<int64_t>(2048, A.h) : 0;
  if (A.nr + nc == 0) return hipSuccess;
  hipLaunchKernelGGL(bwd_finish_kernel, dim3(A.nr + nc), dim3(256), 0, stream, A);
  return hipGetLastError();
}

// ------------------------------------------------------ alignment loss

__global__ __launch_bounds__(256) void sq_residual_kernel(const float *__restrict__ out,
                                                          const float *__restrict__ ref,
                                                          const float *__restrict__ mask,
                                                          int64_t n, double *__restrict__ partials,
                                                          float *__restrict__ gout) {
  __shared__ double ws[4];
  double acc = 0.0;
  // four elements per step with 16-byte loads and stores when every buffer
  // is 16-byte aligned; element by element otherwise and for the tail
  typedef float f4v __attribute__((ext_vector_type(4)));
  const bool vec = ((reinterpret_cast<uintptr_t>(out) | reinterpret_cast<uintptr_t>(ref) |
                     reinterpret_cast<uintptr_t>(mask) | reinterpret_cast<uintptr_t>(gout)) &
                    15) == 0;
  const int64_t n4 = vec ? n / 4 : 0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += stride) {
    const f4v o = reinterpret_cast<const f4v *>(out)[i];
    const f4v r0 = reinterpret_cast<const f4v *>(ref)[i];
    const f4v m = mask ? reinterpret_cast<const f4v *>(mask)[i] : (f4v){1.0f, 1.0f, 1.0f, 1.0f};
    const f4v r = o - r0;
    acc += (double)m.x * (double)r.x * (double)r.x;
    acc += (double)m.y * (double)r.y * (double)r.y;
    acc += (double)m.z * (double)r.z * (double)r.z;
    acc += (double)m.w * (double)r.w * (double)r.w;
    if (gout) reinterpret_cast<f4v *>(gout)[i] = 2.0f * m * r;
  }
  for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    float r = out[i] - ref[i];
    float m = mask ? mask[i] : 1.0f;
    acc += (double)m * (double)r * (double)r;
    if (gout) gout[i] = 2.0f * m * r;
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

__global__ __launch_bounds__(256) void sum_partials_kernel(const double *__restrict__ partials,
                                                           int n, double *__restrict__ loss) {
  __shared__ double sm[256];
  double a = 0.0;
  for (int b = threadIdx.x; b < n; b += 256) a += partials[b];
  sm[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = sm[0];
}

hipError_t launch_sq_residual(const float *out, const float *ref, const float *mask, int64_t n,
                              double *partials, int n_blocks, double *loss, float *grad_out,
                              hipStream_t stream) {
  hipLaunchKernelGGL(sq_residual_kernel, dim3(n_blocks), dim3(256), 0, stream, out, ref, mask, n,
                     partials, grad_out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, stream, partials, n_blocks,
                     loss);
  return hipGetLastError();
}

}  // namespace dfr
