// Batched reprojection: many source frames of uneven sizes onto one target
// grid in one persistent launch (the paper's stacking use case, section 1).
// Work items are (frame, tile) pairs handed out by an atomic counter, so
// frames of very different coverage balance across the whole chip; each
// item runs exactly the single-image tile body, so every frame's result is
// bit-identical to a single-image call.
#include "forward_body.hpp"
#include "launch.hpp"

namespace dfr {

template <int INTERP, int SORD, int NP>
__global__ __launch_bounds__(kThreads) void reproject_batch(const FramePlan *__restrict__ plans,
                                                             int n_frames, TileGeom G,
                                                             int *__restrict__ counter) {
  extern __shared__ float lds[];
  __shared__ TileShared sh;
  const int total = n_frames * G.n_tiles;
  while (true) {
    if (threadIdx.x == 0) sh.item = atomicAdd(counter, 1);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(sh.item);
    if (item >= total) break;  // every wave sees the same item: the group leaves together
    const int frame = item / G.n_tiles;
    forward_tile<INTERP, SORD, NP>(plans[frame], G, item - frame * G.n_tiles, lds, sh);
    __syncthreads();
  }
}

using BatchKernel = void (*)(const FramePlan *, int, TileGeom, int *);

template <int INTERP, int NP>
static BatchKernel batch_sord(int sord) {
  switch (sord) {
    case 0: return reproject_batch<INTERP, 0, NP>;
    case 1: return reproject_batch<INTERP, 1, NP>;
    case 2: return reproject_batch<INTERP, 2, NP>;
    case 3: return reproject_batch<INTERP, 3, NP>;
    case 4: return reproject_batch<INTERP, 4, NP>;
    case 5: return reproject_batch<INTERP, 5, NP>;
    default: return reproject_batch<INTERP, kRtOrder, NP>;
  }
}

template <int INTERP>
static BatchKernel batch_np(int np, int sord) {
  switch (np) {
    case 1: return batch_sord<INTERP, 1>(sord);
    case 2: return batch_sord<INTERP, 2>(sord);
    default: return batch_sord<INTERP, 4>(sord);
  }
}

const void *batch_kernel_ptr(int interp, int np, int sord) {
  BatchKernel k = interp == DFR_NEAREST    ? batch_np<DFR_NEAREST>(np, sord)
                  : interp == DFR_BILINEAR ? batch_np<DFR_BILINEAR>(np, sord)
                                           : batch_np<DFR_BICUBIC>(np, sord);
  return reinterpret_cast<const void *>(k);
}

int batch_blocks_per_cu(int interp, int np, int sord, int lds_bytes) {
  int n = 0;
  const void *k = batch_kernel_ptr(interp, np, sord);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, kThreads, lds_bytes) != hipSuccess ||
      n < 1)
    n = 1;
  return n;
}

hipError_t launch_batch_f32(const FramePlan *plans_dev, int n_frames, int max_sord,
                            const TileGeom &G, int interp, int np, int *counter, int grid,
                            hipStream_t stream) {
  hipError_t e = launch_zero_i32(counter, 1, stream);
  if (e != hipSuccess) return e;
  BatchKernel k = reinterpret_cast<BatchKernel>(const_cast<void *>(batch_kernel_ptr(interp, np, max_sord)));
  size_t lds = (size_t)G.lds_cap * sizeof(float);
  hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), lds, stream, plans_dev, n_frames, G, counter);
  return hipGetLastError();
}

}  // namespace dfr
