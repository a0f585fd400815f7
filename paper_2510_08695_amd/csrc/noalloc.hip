// Static device scratch of bpdc_decode_noalloc: the entry point for callers
// that cannot allocate device memory (code under HIP graph capture, serving
// loops that must not call hipMalloc).  The array is a file-scope __device__
// symbol, so every device the library's code object is loaded on holds its own
// copy until the process ends.  In host code the array's name is only a
// host-side stand-in; the device address of each device's copy is looked up
// once per device with hipGetSymbolAddress (that device current) and cached.
#include <mutex>

#include "bpdc.h"
#include "internal.h"

namespace bpdc {

namespace {

static __device__ __align__(256) unsigned char scratch[BPDC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch(int device, void** ptr) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[device] = p;
  }
  *ptr = g_ptr[device];
  return hipSuccess;
}

}  // namespace bpdc
