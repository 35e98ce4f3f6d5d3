// Device scratch of the no-allocation entry point (xf_probabilities_noalloc):
// a fixed array in the code object, resolved to a device address once per
// device.  Each device that runs the library holds its own copy until the
// process ends; every call on that device shares it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "xf_internal.h"

namespace xf {
namespace {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch(int device, void **ptr) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[device]) {
        // the caller has made `device` current; the host-side name of the
        // array is not a device address, only what this returns is
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_addr[device] = p;
    }
    *ptr = g_addr[device];
    return hipSuccess;
}

}  // namespace xf
