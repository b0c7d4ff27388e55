// sfft_noalloc.hip -- the static device scratch of sfft_exec_noalloc and its
// per-device set-up.  The array is a file-scope __device__ object: every GPU
// the library runs on holds its own copy at its own address for the life of
// the process.  In host code the array's name is only a host-side stand-in,
// so the device address of each copy is taken once per device with
// hipGetSymbolAddress and kept; host code uses that address, never the name.
#include <mutex>
#include <vector>

#include "sfft_internal.h"

namespace sfft {

namespace {

__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
char *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

// Device address of the current device's scratch (set up on the first call
// on that device: address taken, twiddle table written at its start).
hipError_t noalloc_scratch(int device, char **base) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    std::vector<float2> tw(kFftMax);
    host_twiddles(tw.data());
    e = hipMemcpy(ptr, tw.data(), sizeof(float2) * kFftMax, hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = (char *)ptr;
  }
  *base = g_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace sfft
