// The library-held workspace of bcf_decode_noalloc: one array per GPU, in
// device memory the code object reserves, so that decoding needs no
// allocation by the library or the caller.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.hpp"

namespace bcf {

static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];       // the array's device address on each device, once looked up

}  // namespace

hipError_t noalloc_workspace(void **ptr)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        // once per device, with that device current: in host code `scratch`
        // names a host-side stand-in, so its device address comes from the runtime
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = p;
    }
    *ptr = g_ptr[dev];
    return hipSuccess;
}

}  // namespace bcf
