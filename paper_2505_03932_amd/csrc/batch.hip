// Launch helpers of the persistent batch and the coadd kernels (defined in
// tile_kernels.hpp).
#include "tile_kernels.hpp"

namespace dfr {

using BatchKernel = void (*)(const FramePlan *, int, TileGeom, int *);

const void *batch_kernel_ptr(int interp, int np, int sord) {
  return interp == DFR_NEAREST    ? batch_kernel_for<DFR_NEAREST>(np, sord)
         : interp == DFR_BILINEAR ? batch_kernel_for<DFR_BILINEAR>(np, sord)
                                  : batch_kernel_for<DFR_BICUBIC>(np, sord);
}

const void *crop_kernel_ptr(int interp, int np, int sord) {
  return interp == DFR_NEAREST    ? crop_kernel_for<DFR_NEAREST>(np, sord)
         : interp == DFR_BILINEAR ? crop_kernel_for<DFR_BILINEAR>(np, sord)
                                  : crop_kernel_for<DFR_BICUBIC>(np, sord);
}

const void *coadd_kernel_ptr(int interp, int np, int sord) {
  return interp == DFR_NEAREST    ? coadd_kernel_for<DFR_NEAREST>(np, sord)
         : interp == DFR_BILINEAR ? coadd_kernel_for<DFR_BILINEAR>(np, sord)
                                  : coadd_kernel_for<DFR_BICUBIC>(np, sord);
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

hipError_t launch_batch_cropped(const FramePlan *plans_dev, int n_frames, int total, int max_sord,
                                const TileGeom &G, int interp, int np, int *counter, int grid,
                                hipStream_t stream) {
  hipError_t e = launch_zero_i32(counter, 1, stream);
  if (e != hipSuccess) return e;
  using CropKernel = void (*)(const FramePlan *, int, int, TileGeom, int *);
  CropKernel k = reinterpret_cast<CropKernel>(const_cast<void *>(crop_kernel_ptr(interp, np, max_sord)));
  size_t lds = (size_t)G.lds_cap * sizeof(float);
  hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), lds, stream, plans_dev, n_frames, total, G,
                     counter);
  return hipGetLastError();
}

hipError_t launch_coadd_f32(const FramePlan *plans_dev, int n_frames, int max_sord,
                            const TileGeom &G, int interp, int np, const CoaddOut &C,
                            hipStream_t stream) {
  using CoaddKernel = void (*)(const FramePlan *, int, TileGeom, CoaddOut);
  CoaddKernel k = reinterpret_cast<CoaddKernel>(const_cast<void *>(coadd_kernel_ptr(interp, np, max_sord)));
  size_t lds = (size_t)G.lds_cap * sizeof(float);
  hipLaunchKernelGGL(k, dim3(G.n_tiles), dim3(kThreads), lds, stream, plans_dev, n_frames, G, C);
  return hipGetLastError();
}

}  // namespace dfr
