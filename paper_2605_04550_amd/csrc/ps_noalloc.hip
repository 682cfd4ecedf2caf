// The fixed device scratch of ps_eval_points_noalloc: a file-scope device array, so that the
// call needs no allocation.  Each GPU that loads the library holds its own copy until the
// process ends; host code reaches it only through the address hipGetSymbolAddress returns
// for the current device (the array's name is a host-side stand-in, not a device address).
#include "ps_internal.h"

#include <mutex>

namespace ps {

namespace {

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void *g_ptr[kMaxDevices] = {};

}  // namespace

// Address of the current device's scratch (looked up once per device), or the HIP error.
hipError_t noalloc_scratch(void **ptr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_lock);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = p;
    }
    *ptr = g_ptr[dev];
    return hipSuccess;
}

}  // namespace ps
