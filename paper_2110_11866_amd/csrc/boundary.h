// Edge extension of a single signal (Sec. II: beyond [0, N-1] the signal is zero or the value
// on the edge): the forward scans a padded copy and keeps the central outputs.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mk {

// xe[m] = x[clamp(m - P, 0, N - 1)] for m in [0, N + 2P), as float32 (x of the given dtype).
hipError_t launch_edge_extend(const void* x, int dtype, int64_t N, int64_t P, float* xe, hipStream_t s);

}  // namespace mk
