// The library's fixed device scratch array, for callers that cannot allocate
// device memory (bd_query_batch_noalloc).
//
// `scratch` is a file-scope device array: every device the library runs on
// holds its own copy, at its own address, from the time the code object is
// loaded there until the process ends. In host code the name `scratch` is a
// host-side stand-in and never a device address, so host code only ever uses
// the address hipGetSymbolAddress returns for the current device, resolved
// once per device and kept here.
#include <hip/hip_runtime.h>

#include <mutex>

#include "probewalk.h"
#include "pw_internal.hpp"

static __device__ __align__(256) unsigned char scratch[pw::kScratchBytes];

namespace pw {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_resolve_mu;
void* g_scratch[kMaxDevices] = {};
std::mutex g_device_mu[kMaxDevices];

}  // namespace

int scratch_acquire(int device, void** base, std::unique_lock<std::mutex>* held)
{
    if (device < 0 || device >= kMaxDevices) return BD_E_INVALID;
    {
        std::lock_guard<std::mutex> lk(g_resolve_mu);
        if (!g_scratch[device]) {
            int cur = -1;
            if (hipGetDevice(&cur) != hipSuccess) {
                (void)hipGetLastError();
                return BD_E_HIP;
            }
            if (cur != device) return BD_E_INVALID;  // resolved with that device current
            void* p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
                (void)hipGetLastError();
                return BD_E_HIP;
            }
            g_scratch[device] = p;
        }
    }
    *held = std::unique_lock<std::mutex>(g_device_mu[device]);
    *base = g_scratch[device];
    return BD_OK;
}

}  // namespace pw
