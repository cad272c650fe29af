// Static device scratch of the allocation-free evaluation
// (mdet_eval_walkers_noalloc): the per-call work buffers of one evaluation
// carved out of one file-scope device array instead of hipMalloc.
//
// Every GPU the library runs on holds its own copy of `scratch` (kNoallocBytes)
// from the time the code object is loaded on it until the process ends.  In
// host code the array's name is only a host-side stand-in: its device address
// is looked up once per device with hipGetSymbolAddress, with that device
// current, and only that address is ever handed to kernels.

#include <hip/hip_runtime.h>

#include <mutex>

#include "mdet_internal.h"

namespace mdet {

namespace {

__device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void *g_ptr[kMaxDevices] = {nullptr};

}  // namespace

hipError_t noalloc_scratch(int device, void **ptr) {
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (g_ptr[device] == nullptr) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (p == nullptr) return hipErrorInvalidSymbol;
        g_ptr[device] = p;
    }
    *ptr = g_ptr[device];
    return hipSuccess;
}

}  // namespace mdet
