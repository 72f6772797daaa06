// Edge extension kernel (see boundary.h): one coalesced pass writing the padded float32 copy.
#include "boundary.h"

#include <algorithm>

#include "scan_common.h"

namespace mk {
namespace {

constexpr int kEdThreads = 256;

__global__ __launch_bounds__(kEdThreads) void edge_extend_kernel(const void* x, int dtype, int64_t N, int64_t P,
                                                                  float* xe) {
  const int64_t Ne = N + 2 * P;
  const int64_t stride = (int64_t)gridDim.x * kEdThreads;
  for (int64_t m = (int64_t)blockIdx.x * kEdThreads + threadIdx.x; m < Ne; m += stride) {
    const int64_t j = m - P < 0 ? 0 : (m - P >= N ? N - 1 : m - P);
    xe[m] = load1(x, dtype, j);
  }
}

}  // namespace

hipError_t launch_edge_extend(const void* x, int dtype, int64_t N, int64_t P, float* xe, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  const int64_t Ne = N + 2 * P;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((Ne + kEdThreads - 1) / kEdThreads, 8192));
  hipLaunchKernelGGL(edge_extend_kernel, dim3((unsigned)blocks), dim3(kEdThreads), 0, s, x, dtype, N, P, xe);
  return hipGetLastError();
}

}  // namespace mk
