// Fixed device scratch of the forward entry point that allocates nothing
// (morlet_forward_noalloc): the scan's workspace lives in a file-scope device array.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

#include "morlet.h"

namespace mk {

// Size of the array (each device that runs the library holds one copy until the process ends).
constexpr size_t kScratchBytes = MORLET_NOALLOC_SCRATCH_BYTES;

// Resolve the array's address on `device`, which must be the current device; once per device,
// later calls return at once. Thread-safe.
hipError_t scratch_setup(int device);
// The address resolved for `device`, or nullptr before a successful scratch_setup.
void* scratch_ptr(int device);

}  // namespace mk
