// Backward of the multiplication method: the transposes of the remodulation and the
// demodulation around the three-row Gaussian adjoint (multiply.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mk {

// g (3N float32) from gW (complex64 N), the transpose of W = ce (e^{i xi n}(g0 + i g1) - kappa g2)
hipError_t launch_mm_remodulate_t(const float2* gW, float* g, int64_t N, double xi, double ce, double cek,
                                  hipStream_t s);
// gx (float32 N) from gu (3N float32), the transpose of u = [x cos(xi m), -x sin(xi m), x]
hipError_t launch_mm_demodulate_t(const float* gu, float* gx, int64_t N, double xi, hipStream_t s);

}  // namespace mk
