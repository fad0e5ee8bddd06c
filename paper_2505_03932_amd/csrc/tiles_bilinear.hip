// Tiled forward, batch and coadd kernels, bilinear interpolation.
#include "tile_kernels.hpp"

namespace dfr {
template const void *tile_kernel_for<DFR_BILINEAR>(int, int);
template const void *batch_kernel_for<DFR_BILINEAR>(int, int);
template const void *coadd_kernel_for<DFR_BILINEAR>(int, int);
template const void *crop_kernel_for<DFR_BILINEAR>(int, int);
}  // namespace dfr
