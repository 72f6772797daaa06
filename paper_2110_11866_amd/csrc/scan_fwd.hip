// Dispatch of the forward scan kernels and the workspace fill kernel.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "launch.h"

namespace mk {

using KernelFn = void (*)(ScanLaunch);
KernelFn select_fwd_k1(int R, int wide, int kind);
KernelFn select_fwd_k2(int R, int wide, int kind);
KernelFn select_fwd_k3(int R, int wide, int kind);
KernelFn select_fwd_k4(int R, int wide, int kind);
KernelFn select_fwd_k5(int R, int wide, int kind);
KernelFn select_fwd_k6(int R, int wide, int kind);
KernelFn select_fwd_k7(int R, int wide, int kind);
KernelFn select_fwd_k8(int R, int wide, int kind);
KernelFn select_fwd_k9(int R, int wide, int kind);
KernelFn select_fwd_k10(int R, int wide, int kind);
KernelFn select_fwd_k11(int R, int wide, int kind);
KernelFn select_fwd_k12(int R, int wide, int kind);

namespace {

__global__ void zero_fill_kernel(uint4* p, size_t n16, unsigned char* tail, size_t ntail) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

KernelFn select_kernel(int K, int R, int wide, int kind) {
  switch (K) {
    case 1: return select_fwd_k1(R, wide, kind);
    case 2: return select_fwd_k2(R, wide, kind);
    case 3: return select_fwd_k3(R, wide, kind);
    case 4: return select_fwd_k4(R, wide, kind);
    case 5: return select_fwd_k5(R, wide, kind);
    case 6: return select_fwd_k6(R, wide, kind);
    case 7: return select_fwd_k7(R, wide, kind);
    case 8: return select_fwd_k8(R, wide, kind);
    case 9: return select_fwd_k9(R, wide, kind);
    case 10: return select_fwd_k10(R, wide, kind);
    case 11: return select_fwd_k11(R, wide, kind);
    case 12: return select_fwd_k12(R, wide, kind);
    default: return nullptr;
  }
}

}  // namespace

hipError_t launch_scan_forward(const ScanLaunch& a, hipStream_t s) {
  KernelFn fn = select_kernel(a.K, a.R, a.wide, a.kind);
  if (!fn) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fn, dim3(a.grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

int scan_forward_occupancy(int K, int R, int wide, int kind) {
  KernelFn fn = select_kernel(K, R, wide, kind);
  if (!fn) return 0;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(fn), kThreads, 0) != hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

hipError_t launch_zero_fill(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  const size_t n16 = bytes / 16, ntail = bytes % 16;
  const unsigned int blocks = (unsigned int)std::min<size_t>((n16 + 255) / 256 + 1, 4096);
  hipLaunchKernelGGL(zero_fill_kernel, dim3(blocks), dim3(256), 0, s, static_cast<uint4*>(p), n16,
                     static_cast<unsigned char*>(p) + n16 * 16, ntail);
  return hipGetLastError();
}

}  // namespace mk
