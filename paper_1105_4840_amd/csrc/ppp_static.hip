// The allocation-free entry point: ppp_run with its workspace in a device
// array the library holds for the life of the process, for callers that cannot
// allocate device memory.
//
// `scratch` below is a file-scope device array.  In host code its name is a
// host-side stand-in, not a device address, so it is never passed to a kernel
// or a copy: on its first call on a device (that device current) the entry
// point asks the runtime for the array's address on that device with
// hipGetSymbolAddress and keeps it per device; every later use goes through
// that pointer.  Each GPU holds its own copy of the array at its own address.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "ppp.h"
#include "ppp_internal_api.hpp"

static __device__ __align__(256) char scratch[PPP_STATIC_WORKSPACE_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void *g_scratch[kMaxDevices] = {};

// The array's address on the current device, looked up once per device.
ppp_status scratch_on_current_device(ppp_handle *h, void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        ppp::set_error(h, "no current HIP device (or more than 64 devices)");
        return PPP_E_DEVICE;
    }
    std::lock_guard<std::mutex> lock(g_lock);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            ppp::set_error(h, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return PPP_E_DEVICE;
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return PPP_OK;
}

}  // namespace

extern "C" {

ppp_status ppp_run_static(ppp_handle *h, void *hip_stream) {
    if (!h) return PPP_E_INVALID_ARG;
    void *ws = nullptr;
    ppp_status s = scratch_on_current_device(h, &ws);
    if (s != PPP_OK) return s;
    return ppp::run_without_allocation(h, ws, (size_t)PPP_STATIC_WORKSPACE_BYTES, hip_stream);
}

}  // extern "C"
