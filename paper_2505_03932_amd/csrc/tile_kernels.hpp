// The tiled forward kernels (single image, persistent batch, coadd) as
// templates; each interpolation is instantiated in its own translation unit
// (tiles_nearest.hip, tiles_bilinear.hip, tiles_bicubic.hip) so the library
// builds in parallel.
#pragma once

#include "forward_tile.hpp"
#include "launch.hpp"

namespace dfr {

template <int INTERP, int SORD, int NP>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(NP >= 4 ? 4 : (INTERP == DFR_BICUBIC ? 6 : 8))))
void reproject_tiles(FramePlan P, TileGeom G) {
  extern __shared__ float lds[];
  __shared__ FwdShared sh;
  StoreSink sink;
  forward_tile<INTERP, SORD, NP>(P, G, xcd_tile(blockIdx.x, G.n_tiles), lds, sh, sink);
}

constexpr int kBatchChunk = 16;  // (frame, tile) items claimed per atomic

// Batched reprojection: many source frames of uneven sizes onto one target
// grid in one persistent launch (the paper's stacking use case, section 1).
// Work items are (frame, tile) pairs handed out by an atomic counter, so
// frames of very different coverage balance across the whole chip; each
// item runs exactly the single-image tile body, so every frame's result is
// bit-identical to a single-image call.
template <int INTERP, int SORD, int NP>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(NP >= 4 ? 4 : 5)))
void reproject_batch(const FramePlan *__restrict__ plans, int n_frames, TileGeom G,
                     int *__restrict__ counter) {
  extern __shared__ float lds[];
  __shared__ FwdShared sh;
  const int total = n_frames * G.n_tiles;
  // thread 0 claims kBatchChunk consecutive items per atomic (one counter
  // round trip per chunk, not per item) and hands them out one by one
  int next = 0, end = 0;
  while (true) {
    if (threadIdx.x == 0) {
      if (next >= end) {
        next = atomicAdd(counter, kBatchChunk);
        end = next + kBatchChunk;
      }
      sh.item = next++;
    }
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(sh.item);
    if (item >= total) break;  // every wave sees the same item: the group leaves together
    const int frame = item / G.n_tiles;
    // read the frame table through the constant address space: it is not
    // written during the launch, so its fields can be scalar (SGPR) loads
    using ConstPlan = const __attribute__((address_space(4))) FramePlan;
    ConstPlan *cp = (ConstPlan *)(plans + frame);
    const FramePlan &P = *(const FramePlan *)cp;
    const int tile = item - frame * G.n_tiles;
    StoreSink sink;
    if (tile_out_of_reach<NP>(P, G, tile))
      tile_uncovered<NP>(P, G, tile);  // most of a frame that covers part of the grid
    else
      forward_tile<INTERP, SORD, NP>(P, G, tile, lds, sh, sink);
    __syncthreads();
  }
}

// The batch into per-frame windows of the target grid (cropped outputs):
// frame i has items item0 .. item0 + (tiles of its window) - 1, the tiles of
// the global tile grid that meet its window, so every pixel is computed
// exactly as in the full batch; only the window's pixels are stored.
template <int INTERP, int SORD, int NP>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(NP >= 4 ? 4 : 5)))
void reproject_batch_cropped(const FramePlan *__restrict__ plans, int n_frames, int total,
                             TileGeom G, int *__restrict__ counter) {
  extern __shared__ float lds[];
  __shared__ FwdShared sh;
  using ConstPlan = const __attribute__((address_space(4))) FramePlan;
  int next = 0, end = 0;
  while (true) {
    if (threadIdx.x == 0) {
      if (next >= end) {
        next = atomicAdd(counter, kBatchChunk);
        end = next + kBatchChunk;
      }
      sh.item = next++;
    }
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(sh.item);
    if (item >= total) break;  // uniform: the group leaves together
    // the last frame whose first item is <= item (frames without items share
    // the next frame's item0 and are passed over)
    int lo = 0, hi = n_frames - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (((ConstPlan *)(plans + mid))->item0 <= item)
        lo = mid;
      else
        hi = mid - 1;
    }
    const FramePlan &P = *(const FramePlan *)((ConstPlan *)(plans + lo));
    const int k = item - P.item0;
    const int tile = (P.tile0[1] + k / P.ntx) * G.tiles_x + P.tile0[0] + k % P.ntx;
    CropSink sink;
    if (tile_out_of_reach<NP>(P, G, tile))
      sink.uncovered<NP>(P, G, tile);
    else
      forward_tile<INTERP, SORD, NP>(P, G, tile, lds, sh, sink);
    __syncthreads();
  }
}

// Coadd (stacking) of many frames onto one target grid, the paper's
// motivating use (section 1): per target pixel the sums over the frames of
// out * F and of F, and their ratio.  One work-group owns one target tile for
// the whole stack and visits the frames in index order, so the sums stay in
// registers, every output pixel is written once, and the result is
// deterministic (no atomics).  Each frame's per-pixel out and F are exactly
// those of a single-image call.
template <int INTERP, int SORD, int NP>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(NP >= 4 ? 3 : 4)))  // room for the sums
void coadd_tiles(const FramePlan *__restrict__ plans, int n_frames, TileGeom G, CoaddOut C) {
  extern __shared__ float lds[];
  __shared__ FwdShared sh;
  // Work per tile follows the stack's depth there, which varies across the
  // target (deep in the middle, zero at the edges): consecutive blocks, which
  // the dispatcher deals round-robin to the XCDs, take consecutive tiles, so
  // every XCD gets a share of each region (contiguous per-XCD bands would
  // leave the XCDs holding the edges idle).
  const int tile = blockIdx.x;
  const int lg = G.txt_log2;
  const int TW = kRun << lg, RP = kThreads >> lg, TH = RP * NP;
  const int trow = tile / G.tiles_x;
  const int x0 = (tile - trow * G.tiles_x) * TW, y0 = trow * TH;
  const int ty = threadIdx.x >> lg, xr = x0 + (threadIdx.x & ((1 << lg) - 1)) * kRun;
  StackSink<NP> acc;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int y = y0 + ty + k * RP;
    const int64_t off = (int64_t)y * G.out_w + xr;
#pragma unroll
    for (int e = 0; e < kRun; ++e) {
      const bool in = C.accumulate && y < G.out_h && xr + e < G.out_w;
      acc.s[k][e] = in ? C.sum_wf[off + e] : 0.0f;
      acc.w[k][e] = in ? C.sum_f[off + e] : 0.0f;
    }
  }
  using ConstPlan = const __attribute__((address_space(4))) FramePlan;
#pragma unroll 1
  for (int i = 0; i < n_frames; ++i) {
    const FramePlan &P = *(const FramePlan *)((ConstPlan *)(plans + i));
    if (tile_out_of_reach<NP>(P, G, tile)) continue;  // uniform over the group
    forward_tile<INTERP, SORD, NP>(P, G, tile, lds, sh, acc);
    __syncthreads();  // LDS and the per-tile state are reused by the next frame
  }
  const bool vec = ((G.out_w & (kRun - 1)) == 0) &&
                   (((reinterpret_cast<uintptr_t>(C.sum_wf) | reinterpret_cast<uintptr_t>(C.sum_f) |
                      reinterpret_cast<uintptr_t>(C.coadd)) & 15) == 0);
  const float miss = G.nan_outside ? __builtin_nanf("") : 0.0f;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int y = y0 + ty + k * RP;
    if (y >= G.out_h || xr >= G.out_w) continue;
    const int64_t off = (int64_t)y * G.out_w + xr;
    store_run(C.sum_wf, off, xr, G.out_w, vec, acc.s[k]);
    store_run(C.sum_f, off, xr, G.out_w, vec, acc.w[k]);
    if (C.coadd) {
      float q[kRun];
#pragma unroll
      for (int e = 0; e < kRun; ++e) q[e] = acc.w[k][e] > 0.0f ? acc.s[k][e] / acc.w[k][e] : miss;
      store_run(C.coadd, off, xr, G.out_w, vec, q);
    }
  }
}

// Source SIP orders 0..5 have compile-time kernels; higher orders, and any
// target with SIP A/B (sord < 0 here), use the run-time-order kernel.
template <template <int, int, int> class K, int INTERP, int NP>
const void *pick_sord(int sord) {
  switch (sord) {
    case 0: return K<INTERP, 0, NP>::ptr();
    case 1: return K<INTERP, 1, NP>::ptr();
    case 2: return K<INTERP, 2, NP>::ptr();
    case 3: return K<INTERP, 3, NP>::ptr();
    case 4: return K<INTERP, 4, NP>::ptr();
    case 5: return K<INTERP, 5, NP>::ptr();
    default: return K<INTERP, kRtOrder, NP>::ptr();
  }
}

template <int INTERP, int SORD, int NP>
struct TileK {
  static const void *ptr() { return reinterpret_cast<const void *>(reproject_tiles<INTERP, SORD, NP>); }
};
template <int INTERP, int SORD, int NP>
struct BatchK {
  static const void *ptr() { return reinterpret_cast<const void *>(reproject_batch<INTERP, SORD, NP>); }
};

template <int INTERP, int SORD, int NP>
struct CropK {
  static const void *ptr() { return reinterpret_cast<const void *>(reproject_batch_cropped<INTERP, SORD, NP>); }
};
template <int INTERP, int SORD, int NP>
struct CoaddK {
  static const void *ptr() { return reinterpret_cast<const void *>(coadd_tiles<INTERP, SORD, NP>); }
};

// Kernel for (rows per thread, source SIP order) of one interpolation.
template <int INTERP>
const void *tile_kernel_for(int np, int sord) {
  switch (np) {
    case 1: return pick_sord<TileK, INTERP, 1>(sord);
    case 2: return pick_sord<TileK, INTERP, 2>(sord);
    default: return pick_sord<TileK, INTERP, 4>(sord);
  }
}

template <int INTERP>
const void *batch_kernel_for(int np, int sord) {
  switch (np) {
    case 1: return pick_sord<BatchK, INTERP, 1>(sord);
    case 2: return pick_sord<BatchK, INTERP, 2>(sord);
    default: return pick_sord<BatchK, INTERP, 4>(sord);
  }
}

template <int INTERP>
const void *crop_kernel_for(int np, int sord) {
  switch (np) {
    case 1: return pick_sord<CropK, INTERP, 1>(sord);
    case 2: return pick_sord<CropK, INTERP, 2>(sord);
    default: return pick_sord<CropK, INTERP, 4>(sord);
  }
}

template <int INTERP>
const void *coadd_kernel_for(int np, int sord) {
  switch (np) {
    case 1: return pick_sord<CoaddK, INTERP, 1>(sord);
    case 2: return pick_sord<CoaddK, INTERP, 2>(sord);
    default: return pick_sord<CoaddK, INTERP, 4>(sord);
  }
}

extern template const void *tile_kernel_for<DFR_NEAREST>(int, int);
extern template const void *tile_kernel_for<DFR_BILINEAR>(int, int);
extern template const void *tile_kernel_for<DFR_BICUBIC>(int, int);
extern template const void *batch_kernel_for<DFR_NEAREST>(int, int);
extern template const void *batch_kernel_for<DFR_BILINEAR>(int, int);
extern template const void *batch_kernel_for<DFR_BICUBIC>(int, int);
extern template const void *crop_kernel_for<DFR_NEAREST>(int, int);
extern template const void *crop_kernel_for<DFR_BILINEAR>(int, int);
extern template const void *crop_kernel_for<DFR_BICUBIC>(int, int);
extern template const void *coadd_kernel_for<DFR_NEAREST>(int, int);
extern template const void *coadd_kernel_for<DFR_BILINEAR>(int, int);
extern template const void *coadd_kernel_for<DFR_BICUBIC>(int, int);

}  // namespace dfr
