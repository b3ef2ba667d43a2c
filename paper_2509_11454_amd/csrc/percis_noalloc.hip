// Device scratch of the no-allocation sampling call: one file-scope array
// per GPU, sized once for the library, never freed before the process ends.
//
// Host code never uses the array's name as an address: each device's copy
// lives at its own device address, which noalloc_scratch() takes from
// hipGetSymbolAddress once per device (with that device current) and keeps.
#include <mutex>

#include "percis_host.h"

namespace percis {

constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kNoAllocMaxDevices];

int noalloc_scratch(percis_ctx* c, void** out) {
    *out = nullptr;
    if (c->device < 0 || c->device >= kNoAllocMaxDevices)
        return fail(c, PERCIS_E_DEVICE, "device %d: the no-allocation scratch covers devices 0..%d", c->device,
                    kNoAllocMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[c->device]) {
        HIPCHK(c, hipSetDevice(c->device));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(c, PERCIS_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", c->device,
                        hipGetErrorString(e));
        g_scratch_ptr[c->device] = p;
    }
    *out = g_scratch_ptr[c->device];
    return PERCIS_OK;
}

}  // namespace percis
