// Transposes between an interleaved complex image and two real planes, for the separable 2-D
// Gabor filter (complex row pass, then real column scans of the real and imaginary parts).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mk {

// Plane 0 of P (C x R float32, row-major) gets the real parts and plane 1 (the next R C
// floats) the imaginary parts of the transposed R x C row-major complex64 matrix Z:
// P[c R + r] = Re Z[r][c], P[R C + c R + r] = Im Z[r][c]. P holds 2 R C floats.
hipError_t launch_transpose_c2p(const float2* Z, float* P, int64_t R, int64_t C, hipStream_t s);

// The inverse: Z[r][c] = (plane 0 [c][r], plane 1 [c][r]) for two C x R float32 planes.
hipError_t launch_transpose_p2c(const float* P, float2* Z, int64_t R, int64_t C, hipStream_t s);

}  // namespace mk
