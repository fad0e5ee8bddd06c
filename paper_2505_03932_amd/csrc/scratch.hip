// Fixed device scratch of the allocation-free entry point
// (dfr_reproject_noalloc): a file-scope device array that every GPU the
// library runs on holds from the library's load to the end of the process.
// In host code the array's name is only a stand-in for the symbol; its
// device address differs per GPU and is looked up once per device with
// hipGetSymbolAddress, and only that address is ever handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "scratch.hpp"

namespace dfr {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_addr[kMaxDevices];  // device address of `scratch`, per device id

}  // namespace

hipError_t scratch_address(void **ptr) {
  *ptr = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mutex);
  if (g_scratch_addr[dev] == nullptr) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    g_scratch_addr[dev] = p;
  }
  *ptr = g_scratch_addr[dev];
  return hipSuccess;
}

}  // namespace dfr
