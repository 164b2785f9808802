// Scratch of the allocation-free energy entry point (tmop_energy_noalloc):
// one file-scope device array per GPU, so that the call needs no device
// allocation.  The array's name is a host-side stand-in in host code; its
// device address comes from hipGetSymbolAddress, taken once per device with
// that device current and cached here, and only that address is handed to
// kernels and copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "tmop_internal.h"

namespace tmop {

static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_addr[MAX_DEVICES] = {};
}  // namespace

int noalloc_scratch(int device, double** out) {
  if (!out || device < 0 || device >= MAX_DEVICES) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    if (!p) return (int)hipErrorInvalidSymbol;
    g_addr[device] = static_cast<double*>(p);
  }
  *out = g_addr[device];
  return 0;
}

}  // namespace tmop
