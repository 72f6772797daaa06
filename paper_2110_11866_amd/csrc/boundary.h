// Edge extension of a single signal (Sec. II: beyond [0, N-1] the signal is zero or the value
// on the edge): the forward scans a padded copy and keeps the central outputs.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mk {

// xe[m] = x[clamp(m - P, 0, N - 1)] for m in [0, N + 2P), as float32 (x of the given dtype).
hipError_t launch_edge_extend(const void* x, int dtype, int64_t N, int64_t P, float* xe, hipStream_t s);

// The backward of the extension. ge[m] = g[m - P] inside [P, P + N), zero elsewhere, for
// m in [0, N + 2P) (elements of esize 4 or 8 bytes): the cotangent of the padded outputs.
hipError_t launch_pad_center(const void* g, int esize, int64_t N, int64_t P, void* ge, hipStream_t s);
// gx[j] = gxe[P + j], plus the sums of gxe over [0, P) into gx[0] and over [P + N, N + 2P) into
// gx[N - 1] (the transpose of the edge extension), summed in a fixed order.
hipError_t launch_edge_fold(const float* gxe, int64_t N, int64_t P, float* gx, hipStream_t s);

// out[n] = in[N - 1 - n] (float32): the time reversal R, for the transpose R A R of a real-tap
// "same" convolution A.
hipError_t launch_reverse(const float* in, float* out, int64_t N, hipStream_t s);

}  // namespace mk
