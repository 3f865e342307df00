// Library-held device scratch for the entry points that allocate nothing
// (tfim_measure_triples_noalloc): a file-scope device array that every GPU
// the library runs on holds until the process ends.
//
// In host code the array's name stands for a host-side shadow, not a device
// address, so it is never passed to a kernel or a copy: its device address
// is looked up once per device, with that device current, and kept.
#include <mutex>

#include "tfim_internal.h"

namespace tfim {
namespace {

// 64 MiB: the int8 G/2 digit planes of 16 configurations at L = 24 with six
// replicas (2 R (64 ceil(L/8)^2)^2 = 3.98 MB each).
constexpr size_t kScratchBytes = (size_t)64 << 20;

__device__ __align__(256) int8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void* g_addr[kMaxDevices] = {};

}  // namespace

hipError_t static_scratch(int device, void** ptr, size_t* bytes) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> hold(g_lock);
    if (!g_addr[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        const hipError_t e2 = cur != device ? hipSetDevice(cur) : hipSuccess;
        if (e != hipSuccess) return e;
        if (e2 != hipSuccess) return e2;
        g_addr[device] = p;
    }
    *ptr = g_addr[device];
    *bytes = kScratchBytes;
    return hipSuccess;
}

}  // namespace tfim
