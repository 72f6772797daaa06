// Baseline (gfx950): the truncated direct convolution W[n] = sum_{|k|<=H} h[k] x[n-k] with the
// exact complex taps h (the conventional method of Sec. V-B uses H = 3 sigma), x zero outside
// [0, N). Not part of the SFT/ASFT path: it is the comparison the benchmark times.
//
// One block computes 256 x 4 consecutive outputs over one slab of the taps; the slab's taps
// are swept in chunks of 1024 staged in LDS together with the signal segment they touch. Each
// thread keeps a sliding window of four signal samples in registers, so a tap costs one
// broadcast tap read, a quarter of a signal read and 8 FMAs. With several slabs (short
// signals, long windows: too few output blocks to fill the chip) each slab writes a partial
// output and a second kernel adds the slabs in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "launch.h"

namespace mk {
namespace {

constexpr int kDcThreads = 256;
constexpr int kDcOut = 4;                          // outputs per thread
constexpr int kDcTile = kDcThreads * kDcOut;       // outputs per block
constexpr int kDcChunk = 1024;                     // taps per LDS chunk

__device__ __forceinline__ float dc_load(const void* x, int dtype, int64_t i, int64_t N) {
  if (i < 0 || i >= N) return 0.f;
  if (dtype == 0) return static_cast<const float*>(x)[i];
  const unsigned short h = static_cast<const unsigned short*>(x)[i];
  return dtype == 1 ? (float)__builtin_bit_cast(_Float16, h) : __uint_as_float((uint32_t)h << 16);
}

// slab blockIdx.y covers tap chunks [y cps, min((y + 1) cps, nchunks)); its partial goes to
// out + y N
__global__ __launch_bounds__(kDcThreads) void direct_conv_kernel(const void* x, int dtype, int64_t N,
                                                                  const float2* taps, int64_t H, int64_t cps,
                                                                  float2* out) {
  // seg[s] = x[nb - k0 - kDcChunk + 1 + s], s in [0, kDcTile + kDcChunk + 4)
  __shared__ float seg[kDcTile + kDcChunk + 4];
  __shared__ float2 tp[kDcChunk];
  const int tid = threadIdx.x;
  const int64_t nb = (int64_t)blockIdx.x * kDcTile;
  const int64_t ntaps = 2 * H + 1;
  const int64_t c_lo = (int64_t)blockIdx.y * cps * kDcChunk;
  const int64_t c_hi = std::min<int64_t>(ntaps, c_lo + cps * kDcChunk);
  float accr[kDcOut], acci[kDcOut];
#pragma unroll
  for (int i = 0; i < kDcOut; ++i) { accr[i] = 0.f; acci[i] = 0.f; }
  for (int64_t c0 = c_lo; c0 < c_hi; c0 += kDcChunk) {
    const int64_t k0 = c0 - H;                     // first tap offset k of this chunk
    const int nt = (int)std::min<int64_t>(kDcChunk, c_hi - c0);
    __syncthreads();
    for (int s = tid; s < kDcChunk; s += kDcThreads) tp[s] = s < nt ? taps[c0 + s] : make_float2(0.f, 0.f);
    const int64_t base = nb - k0 - kDcChunk + 1;   // x index of seg[0]
    for (int s = tid; s < kDcTile + kDcChunk + 4; s += kDcThreads) seg[s] = dc_load(x, dtype, base + s, N);
    __syncthreads();
    // output n = nb + o (o = kDcOut tid + i), tap k = k0 + t: x[n - k] = seg[o - t + kDcChunk - 1]
    const int o = kDcOut * tid;
    float win[kDcOut];
#pragma unroll
    for (int i = 0; i < kDcOut; ++i) win[i] = seg[o + i + kDcChunk - 1];
    for (int t = 0; t < nt; ++t) {
      const float2 h = tp[t];
#pragma unroll
      for (int i = 0; i < kDcOut; ++i) {
        accr[i] = fmaf(h.x, win[i], accr[i]);
        acci[i] = fmaf(h.y, win[i], acci[i]);
      }
#pragma unroll
      for (int i = kDcOut - 1; i > 0; --i) win[i] = win[i - 1];
      if (t + 1 < nt) win[0] = seg[o + kDcChunk - 2 - t];
    }
  }
  float2* W = out + (int64_t)blockIdx.y * N;
#pragma unroll
  for (int i = 0; i < kDcOut; ++i) {
    const int64_t n = nb + kDcOut * tid + i;
    if (n < N) W[n] = make_float2(accr[i], acci[i]);
  }
}

__global__ __launch_bounds__(256) void direct_sum_kernel(const float2* part, int slabs, int64_t N, float2* W) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += stride) {
    float2 a = part[n];
    for (int s = 1; s < slabs; ++s) {
      const float2 b = part[(int64_t)s * N + n];
      a.x += b.x;
      a.y += b.y;
    }
    W[n] = a;
  }
}

}  // namespace

int direct_conv_slabs(int64_t N, int64_t H, int num_cus) {
  const int64_t blocks = (N + kDcTile - 1) / kDcTile;
  const int64_t nchunks = (2 * H + 1 + kDcChunk - 1) / kDcChunk;
  const int64_t want = (4 * (int64_t)num_cus + blocks - 1) / std::max<int64_t>(blocks, 1);
  return (int)std::max<int64_t>(1, std::min<int64_t>({want, nchunks, 64}));
}

hipError_t launch_direct_conv(const void* x, int dtype, int64_t N, const float2* taps, int64_t H, int slabs,
                              float2* part, float2* W, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  const int64_t blocks = (N + kDcTile - 1) / kDcTile;
  const int64_t nchunks = (2 * H + 1 + kDcChunk - 1) / kDcChunk;
  const int64_t cps = (nchunks + slabs - 1) / slabs;
  const int used = (int)((nchunks + cps - 1) / cps);   // slabs that hold at least one chunk
  hipLaunchKernelGGL(direct_conv_kernel, dim3((unsigned)blocks, (unsigned)used), dim3(kDcThreads), 0, s, x, dtype, N,
                     taps, H, cps, used > 1 ? part : W);
  if (used > 1) {
    const unsigned sb = (unsigned)std::min<int64_t>((N + 255) / 256, 4096);
    hipLaunchKernelGGL(direct_sum_kernel, dim3(sb), dim3(256), 0, s, part, used, N, W);
  }
  return hipGetLastError();
}

}  // namespace mk
