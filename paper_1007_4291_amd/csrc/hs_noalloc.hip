// Scratch memory of the allocation-free sweep application (sweep_apply_noalloc): one statically
// allocated device array per GPU, created when the library's code object is loaded on that GPU and
// held until the process ends.  Host code never uses the array's name as a device address: the
// address is looked up with hipGetSymbolAddress once per device, with that device current, and every
// kernel argument and copy uses that address.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "../../include/helmsweep.h"
#include "hs_kernels.h"

namespace hs {

namespace {

__device__ __align__(256) unsigned char scratch[HELM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices];
std::mutex g_scratch_mu;
thread_local char g_scratch_msg[256];

}  // namespace

void* noalloc_scratch() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        snprintf(g_scratch_msg, sizeof(g_scratch_msg), "hipGetDevice: %s", hipGetErrorString(e));
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        snprintf(g_scratch_msg, sizeof(g_scratch_msg), "device %d beyond the %d the scratch table covers", dev,
                 kMaxDevices);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            snprintf(g_scratch_msg, sizeof(g_scratch_msg), "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                     hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

const char* noalloc_error() { return g_scratch_msg; }

}  // namespace hs
