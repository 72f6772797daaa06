// Transpose for separable 2-D filtering of images: the lines of an image are filtered
// independently (Sec. IV), rows by one batched scan launch over the H rows, columns by a
// second over the W rows of the transposed image. out[c][r] = in[r][c] for an R x C row-major
// float32 matrix, through 64 x 64 LDS tiles (row pitch 65, so the transposed reads hit 64
// different banks); both the loads and the stores are row-contiguous across a wave.
#include <hip/hip_runtime.h>

#include "launch.h"

namespace mk {
namespace {

constexpr int kTpTile = 64;
constexpr int kTpThreads = 256;   // 64 x 4

__global__ __launch_bounds__(kTpThreads) void transpose_kernel(const float* in, float* out, int64_t R, int64_t C,
                                                                 int64_t nbc) {
  __shared__ float t[kTpTile][kTpTile + 1];
  const int64_t b = blockIdx.x;
  const int64_t r0 = (b / nbc) * kTpTile, c0 = (b % nbc) * kTpTile;
  const int tx = threadIdx.x & (kTpTile - 1), ty = threadIdx.x / kTpTile;
  for (int i = ty; i < kTpTile; i += kTpThreads / kTpTile) {
    const int64_t r = r0 + i, c = c0 + tx;
    if (r < R && c < C) t[i][tx] = in[r * C + c];
  }
  __syncthreads();
  for (int i = ty; i < kTpTile; i += kTpThreads / kTpTile) {
    const int64_t c = c0 + i, r = r0 + tx;
    if (c < C && r < R) out[c * R + r] = t[tx][i];
  }
}

}  // namespace

hipError_t launch_transpose(const float* in, float* out, int64_t R, int64_t C, hipStream_t s) {
  if (R <= 0 || C <= 0) return hipSuccess;
  const int64_t nbr = (R + kTpTile - 1) / kTpTile, nbc = (C + kTpTile - 1) / kTpTile;
  if (nbr * nbc > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)(nbr * nbc)), dim3(kTpThreads), 0, s, in, out, R, C, nbc);
  return hipGetLastError();
}

}  // namespace mk
