// qedx_scratch.hip -- the fixed device scratch of the allocation-free
// gradient entry point (qed_eval_grad_noalloc).
//
// A file-scope device array: every GPU the library runs on holds its own
// copy, allocated with the code object and kept until the process ends.  In
// host code the array's name is only a stand-in, not a device address, so
// the address is resolved once per device with hipGetSymbolAddress (with
// that device current) and cached; kernels receive that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "qedx_scratch.hpp"

namespace {

__device__ __align__(256) unsigned char scratch[qedx_rt::kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

}  // namespace

namespace qedx_rt {

hipError_t scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_addr[dev] = p;
  }
  *out = g_addr[dev];
  return hipSuccess;
}

}  // namespace qedx_rt
