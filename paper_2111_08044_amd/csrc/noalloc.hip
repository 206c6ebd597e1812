// Static device scratch of the entry points that allocate nothing.
//
// `scratch` is a file-scope device array: every GPU the library runs on holds
// its own copy for the life of the process, at its own address.  In host code
// the name is only a host-side stand-in, so the device address is looked up
// once per device (with that device current) and kept in g_ptr; host code
// uses only that pointer.  Every call on one GPU shares that GPU's copy and
// finds the previous call's contents in it: calls that overlap on one GPU
// race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "noalloc.h"

namespace {

constexpr size_t kScratchBytes = size_t(4) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

namespace fl {

size_t scratch_bytes() { return kScratchBytes; }

hipError_t scratch_init(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[dev]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = p;
    return hipSuccess;
}

void* scratch_ptr(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_ptr[dev];
}

}  // namespace fl
