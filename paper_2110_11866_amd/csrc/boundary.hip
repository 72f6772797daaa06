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

__global__ __launch_bounds__(kEdThreads) void pad_center_kernel(const void* g, int esize, int64_t N, int64_t P,
                                                                 void* ge) {
  const int64_t Ne = N + 2 * P;
  const int64_t stride = (int64_t)gridDim.x * kEdThreads;
  for (int64_t m = (int64_t)blockIdx.x * kEdThreads + threadIdx.x; m < Ne; m += stride) {
    const bool in = m >= P && m < P + N;
    if (esize == 8)
      static_cast<uint64_t*>(ge)[m] = in ? static_cast<const uint64_t*>(g)[m - P] : 0ull;
    else
      static_cast<uint32_t*>(ge)[m] = in ? static_cast<const uint32_t*>(g)[m - P] : 0u;
  }
}

// interior copy by every block; block 0 also forms the two edge sums (fixed order: per-thread
// strided partials, then a fixed tree) and writes gx[0] and gx[N - 1]
__global__ __launch_bounds__(kEdThreads) void edge_fold_kernel(const float* gxe, int64_t N, int64_t P, float* gx) {
  const int64_t stride = (int64_t)gridDim.x * kEdThreads;
  for (int64_t j = (int64_t)blockIdx.x * kEdThreads + threadIdx.x; j < N; j += stride)
    if (j != 0 && j != N - 1) gx[j] = gxe[P + j];
  if (blockIdx.x != 0) return;
  __shared__ double red[2][kEdThreads];
  double lo = 0.0, hi = 0.0;
  for (int64_t m = threadIdx.x; m < P; m += kEdThreads) {
    lo += (double)gxe[m];
    hi += (double)gxe[P + N + m];
  }
  red[0][threadIdx.x] = lo;
  red[1][threadIdx.x] = hi;
  __syncthreads();
  for (int off = kEdThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      red[0][threadIdx.x] += red[0][threadIdx.x + off];
      red[1][threadIdx.x] += red[1][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (N == 1) {
      gx[0] = (float)((double)gxe[P] + red[0][0] + red[1][0]);
    } else {
      gx[0] = (float)((double)gxe[P] + red[0][0]);
      gx[N - 1] = (float)((double)gxe[P + N - 1] + red[1][0]);
    }
  }
}

__global__ __launch_bounds__(kEdThreads) void reverse_kernel(const float* in, float* out, int64_t N) {
  const int64_t stride = (int64_t)gridDim.x * kEdThreads;
  for (int64_t n = (int64_t)blockIdx.x * kEdThreads + threadIdx.x; n < N; n += stride) out[n] = in[N - 1 - n];
}

}  // namespace

hipError_t launch_reverse(const float* in, float* out, int64_t N, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((N + kEdThreads - 1) / kEdThreads, 8192));
  hipLaunchKernelGGL(reverse_kernel, dim3((unsigned)blocks), dim3(kEdThreads), 0, s, in, out, N);
  return hipGetLastError();
}

hipError_t launch_pad_center(const void* g, int esize, int64_t N, int64_t P, void* ge, hipStream_t s) {
  const int64_t Ne = N + 2 * P;
  if (Ne <= 0) return hipSuccess;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((Ne + kEdThreads - 1) / kEdThreads, 8192));
  hipLaunchKernelGGL(pad_center_kernel, dim3((unsigned)blocks), dim3(kEdThreads), 0, s, g, esize, N, P, ge);
  return hipGetLastError();
}

hipError_t launch_edge_fold(const float* gxe, int64_t N, int64_t P, float* gx, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((N + kEdThreads - 1) / kEdThreads, 8192));
  hipLaunchKernelGGL(edge_fold_kernel, dim3((unsigned)blocks), dim3(kEdThreads), 0, s, gxe, N, P, gx);
  return hipGetLastError();
}

hipError_t launch_edge_extend(const void* x, int dtype, int64_t N, int64_t P, float* xe, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  const int64_t Ne = N + 2 * P;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((Ne + kEdThreads - 1) / kEdThreads, 8192));
  hipLaunchKernelGGL(edge_extend_kernel, dim3((unsigned)blocks), dim3(kEdThreads), 0, s, x, dtype, N, P, xe);
  return hipGetLastError();
}

}  // namespace mk
