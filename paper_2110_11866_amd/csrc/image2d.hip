// Transposes for separable 2-D filtering of images: the lines of an image are filtered
// independently (Sec. IV), rows by one batched scan launch over the H rows, columns by a
// second over the W rows of the transposed image. out[c][r] = in[r][c] for an R x C row-major
// float32 matrix, through 64 x 64 LDS tiles (row pitch 65, so the transposed reads hit 64
// different banks); both the loads and the stores are row-contiguous across a wave.
#include <hip/hip_runtime.h>

#include "image2d.h"
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

// Complex image to two planes, in tiles of 32 rows x 64 columns (16.6 KB of LDS, so up to eight
// blocks per CU keep loads in flight). Loads: each wave reads 64 consecutive 8-byte words of a
// row of Z. Stores: each half wave writes 32 consecutive floats (one 128-byte line) of a row of
// a plane. The LDS row pitch 65 puts the transposed reads of a half wave in 32 banks.
constexpr int kCpRows = 32;

__global__ __launch_bounds__(kTpThreads) void transpose_c2p_kernel(const float2* in, float* out, int64_t R, int64_t C,
                                                                     int64_t nbc) {
  __shared__ float tr[kCpRows][kTpTile + 1], ti[kCpRows][kTpTile + 1];
  const int64_t b = blockIdx.x;
  const int64_t r0 = (b / nbc) * kCpRows, c0 = (b % nbc) * kTpTile;
  const int tx = threadIdx.x & (kTpTile - 1), ty = threadIdx.x / kTpTile;
  for (int i = ty; i < kCpRows; i += kTpThreads / kTpTile) {
    const int64_t r = r0 + i, c = c0 + tx;
    if (r < R && c < C) {
      const float2 v = in[r * C + c];
      tr[i][tx] = v.x;
      ti[i][tx] = v.y;
    }
  }
  __syncthreads();
  const int64_t plane = R * C;
  const int lane = threadIdx.x & (kCpRows - 1), row = threadIdx.x / kCpRows;   // row: 0..7
  for (int k = row; k < kTpTile; k += kTpThreads / kCpRows) {
    const int64_t c = c0 + k, r = r0 + lane;
    if (c < C && r < R) {
      out[c * R + r] = tr[lane][k];
      out[plane + c * R + r] = ti[lane][k];
    }
  }
}

// Two planes back to the complex image, tiles of 32 rows x 64 columns of Z: each half wave
// reads 32 consecutive floats of a plane row, each wave writes 64 consecutive 8-byte words of
// a row of Z. LDS [column][row] with pitch 33.
__global__ __launch_bounds__(kTpThreads) void transpose_p2c_kernel(const float* in, float2* out, int64_t R, int64_t C,
                                                                     int64_t nbc) {
  __shared__ float tr[kTpTile][kCpRows + 1], ti[kTpTile][kCpRows + 1];
  const int64_t b = blockIdx.x;
  const int64_t r0 = (b / nbc) * kCpRows, c0 = (b % nbc) * kTpTile;
  const int64_t plane = R * C;
  const int lane = threadIdx.x & (kCpRows - 1), row = threadIdx.x / kCpRows;
  for (int k = row; k < kTpTile; k += kTpThreads / kCpRows) {
    const int64_t c = c0 + k, r = r0 + lane;
    if (c < C && r < R) {
      tr[k][lane] = in[c * R + r];
      ti[k][lane] = in[plane + c * R + r];
    }
  }
  __syncthreads();
  const int tx = threadIdx.x & (kTpTile - 1), ty = threadIdx.x / kTpTile;
  for (int i = ty; i < kCpRows; i += kTpThreads / kTpTile) {
    const int64_t r = r0 + i, c = c0 + tx;
    if (r < R && c < C) out[r * C + c] = make_float2(tr[tx][i], ti[tx][i]);
  }
}

}  // namespace

hipError_t launch_transpose_c2p(const float2* Z, float* P, int64_t R, int64_t C, hipStream_t s) {
  if (R <= 0 || C <= 0) return hipSuccess;
  const int64_t nbr = (R + kCpRows - 1) / kCpRows, nbc = (C + kTpTile - 1) / kTpTile;
  if (nbr * nbc > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(transpose_c2p_kernel, dim3((unsigned)(nbr * nbc)), dim3(kTpThreads), 0, s, Z, P, R, C, nbc);
  return hipGetLastError();
}

hipError_t launch_transpose_p2c(const float* P, float2* Z, int64_t R, int64_t C, hipStream_t s) {
  if (R <= 0 || C <= 0) return hipSuccess;
  const int64_t nbr = (R + kCpRows - 1) / kCpRows, nbc = (C + kTpTile - 1) / kTpTile;
  if (nbr * nbc > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(transpose_p2c_kernel, dim3((unsigned)(nbr * nbc)), dim3(kTpThreads), 0, s, P, Z, R, C, nbc);
  return hipGetLastError();
}

hipError_t launch_transpose(const float* in, float* out, int64_t R, int64_t C, hipStream_t s) {
  if (R <= 0 || C <= 0) return hipSuccess;
  const int64_t nbr = (R + kTpTile - 1) / kTpTile, nbc = (C + kTpTile - 1) / kTpTile;
  if (nbr * nbc > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)(nbr * nbc)), dim3(kTpThreads), 0, s, in, out, R, C, nbc);
  return hipGetLastError();
}

}  // namespace mk
