// Host-side launch helpers shared by the translation units of libdfr.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace dfr {

// Tile shapes: id 1..kTileCount.  id-1 = li*3 + ni with threads-per-row
// 8 << li (tile width 32 << li px) and NP = 1 << ni rows per thread.
constexpr int kTileCount = 12;
constexpr int kDefaultTile = 5;  // 64 x 32
constexpr int kCoaddTile = 5;    // coadd default

// Untuned default tile of the forward kernels (single image, plan, batch),
// measured on the 6000x4000 SIP-3 frame: 128 x 16 for nearest and bilinear,
// 32 x 64 for bicubic.
inline int forward_default_tile(int interp) { return interp == DFR_BICUBIC ? 2 : 8; }
// The backward's, measured on the 2048^2 bicubic and 6000x4000 bilinear
// cases: 64 x 16 (one row per thread) for bicubic with the source gradient
// (its LDS adds), else 64 x 32.
inline int backward_default_tile(int interp, bool src_grad) {
  return interp == DFR_BICUBIC && src_grad ? 4 : kDefaultTile;
}

struct TileShape {
  int txt_log2;  // threads per tile row, log2
  int np;        // rows per thread
  int width, height;
};

inline bool tile_shape(int id, TileShape &s) {
  if (id < 1 || id > kTileCount) return false;
  int li = (id - 1) / 3, ni = (id - 1) % 3;
  s.txt_log2 = 3 + li;
  s.np = 1 << ni;
  s.width = kRun << s.txt_log2;
  s.height = (kThreads >> s.txt_log2) * s.np;
  return true;
}

// Extra per-frame data the FP64 comparison forms need (trig form: the
// explicit two-stage formulas of section 3.2).
struct TrigPlan {
  double tcd[4];     // target CD (deg/px)
  double scdi[4];    // inverse of the source CD (px/deg)
  double tcrval[2];  // target (RA, Dec) in radians
  double scrval[2];  // source (RA, Dec) in radians
};

hipError_t launch_forward_f32(const FramePlan &P, const TileGeom &G, int interp, int np,
                              hipStream_t stream);
// Per-cell position models of the output grid (ncx x ncy cells of 32x32).
hipError_t launch_cell_models(const FramePlan &P, int ncx, int ncy, CellModel *out,
                              hipStream_t stream);
// Kernel (plans, ncx, ncells, total, out) modelling every cell of every
// frame of a batch; sord as for the batch kernel.
const void *cell_models_batch_ptr(int sord);
hipError_t launch_forward_f64(const FramePlan &P, const TrigPlan &T, const TileGeom &G,
                              int interp, bool trig, hipStream_t stream);
hipError_t launch_batch_f32(const FramePlan *plans_dev, int n_frames, int max_sord,
                            const TileGeom &G, int interp, int np, int *counter,
                            int grid, hipStream_t stream);
const void *batch_kernel_ptr(int interp, int np, int sord);
// The batch into per-frame windows (FramePlan crop, item0, tile0, ntx):
// `total` items over the frames, persistent grid as the batch.
hipError_t launch_batch_cropped(const FramePlan *plans_dev, int n_frames, int total, int max_sord,
                                const TileGeom &G, int interp, int np, int *counter, int grid,
                                hipStream_t stream);
// Coadd of a frame table: one work-group per target tile (G.n_tiles).
hipError_t launch_coadd_f32(const FramePlan *plans_dev, int n_frames, int max_sord,
                            const TileGeom &G, int interp, int np, const CoaddOut &C,
                            hipStream_t stream);
const void *zero_i32_kernel_ptr();
int batch_blocks_per_cu(int interp, int np, int sord, int lds_bytes);
// Number of per-tile FP64 partial sums the backward kernel produces for a
// source SIP order (9 for H, 2 for CRPIX, AP and BP monomial sums).
inline int backward_sums(int s_order) { return 11 + (s_order + 1) * (s_order + 2); }

struct WcsJacobian {
  double dh[54];  // dH_i / d theta_k at [k * 9 + i], theta = CRVAL1..2, CD1_1..CD2_2
};

// src_acc non-null: the source adjoint too, as integer sums into src_acc
// [src_h][src_w] (zeroed by launch_det_prepare), quantised with the scale
// from max|g| in gmax_bits; launch_backward_finish then writes grad_src.
hipError_t launch_backward(const FramePlan &P, const TileGeom &G, int interp, int np,
                           const float *grad_out, double *partials, unsigned long long *src_acc,
                           const int *gmax_bits, hipStream_t stream);
// Zero q[0 .. nq) and *gmax_next, and fold max |g| into *gmax (which must
// start at 0).
hipError_t launch_det_prepare(const float *grad_out, int64_t n, unsigned long long *q, int64_t nq,
                              int *gmax, int *gmax_next, hipStream_t stream);
// What follows the backward kernel: the WCS partials reduced and chained
// into grad_wcs (nr = ns - 10 blocks when grad_wcs is wanted, else 0), and
// the integer sums q (if non-null) converted into grad_src with the scale
// from *gmax.
constexpr int kBwdMaxOrder = 5;  // highest source SIP order the backward takes
constexpr int kBwdSipCols = (kBwdMaxOrder + 1) * (kBwdMaxOrder + 2);  // AP and BP
constexpr int kBwdSipEntries = 2 * (kBwdMaxOrder + 1) * (kBwdMaxOrder + 1);
struct FinishArgs {
  const double *partials;
  int n_blocks, ns, nr;
  WcsJacobian J;
  double S;
  double *grad_wcs;
  int col_entry[kBwdSipCols];   // grad entry of SIP column 11 + k, or -1
  int col_deg[kBwdSipCols];     // its p + q
  int above[kBwdSipEntries];    // grad entries above their polynomial's order
  int n_above;
  const unsigned long long *q;
  int64_t h, w;
  float *gsrc;
  int64_t gpitch;
  const int *gmax;
};
hipError_t launch_backward_finish(const FinishArgs &args, hipStream_t stream);
hipError_t launch_zero_i32(int *p, int64_t n, hipStream_t stream);
hipError_t launch_sq_residual(const float *out, const float *ref, const float *mask, int64_t n,
                              double *partials, int n_blocks, double *loss, float *grad_out,
                              hipStream_t stream);

}  // namespace dfr
