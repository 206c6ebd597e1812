// The static device scratch used by the entry points that allocate nothing
// (noalloc.hip): kScratchBytes per device, looked up per device.
#pragma once
#include <hip/hip_runtime.h>

#include <stddef.h>

namespace fl {

// Capacity of the scratch in bytes.
size_t scratch_bytes();
// Look up the calling thread's current device's copy of the scratch (once
// per device; later calls return at once).  dev must be the current device.
hipError_t scratch_init(int dev);
// The device address found by scratch_init for dev, or NULL before it.
void* scratch_ptr(int dev);

}  // namespace fl
