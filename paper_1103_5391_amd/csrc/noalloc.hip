// Device scratch owned by the library for its allocation-free entry point: one array per GPU, in
// the code object's zero-initialised data, held from the library's load on that GPU until the
// process ends.  Host code never passes the array's name to a kernel (in host code it is a
// stand-in, not a device address): the address is resolved once per device with
// hipGetSymbolAddress, with that device current, and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.hpp"

namespace dmrg {

namespace {

static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_addr[kMaxDevices];   // device address of `scratch` per device, once resolved

}  // namespace

// The scratch array of the current device (resolved on the first call for that device).
hipError_t noalloc_scratch(double** out) {
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_addr[dev] = static_cast<double*>(p);
    }
    *out = g_addr[dev];
    return hipSuccess;
}

}  // namespace dmrg
