// Carrier kernels of the Morlet transform by the multiplication method (Sec. III-B).
//
// The method's sum over the real frequencies xi + beta p of the envelope's Fourier terms is the
// carrier times the fitted envelope, sum_p a'_p e^{i (xi + beta p) k} = e^{i xi k} G_hat[k], so
//   x_M[n] = C' [ e^{i xi n} (G_hat * u)[n] - kappa (G_hat * x)[n] ],   u[m] = e^{-i xi m} x[m].
// The three real Gaussian smoothings (Re u, Im u, x) run as three rows of one scan launch;
// these two elementwise kernels form the rows before it and combine them after it. The
// phase xi m is formed and reduced in float64 (sincos of the float64 product), so it stays
// exact to float32 for any index.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "launch.h"
#include "multiply.h"
#include "scan_common.h"

namespace mk {
namespace {

constexpr int kMmThreads = 256;

// u[m] = x[m] cos(xi m), u[N + m] = -x[m] sin(xi m), u[2N + m] = x[m]
__global__ __launch_bounds__(kMmThreads) void mm_demodulate_kernel(const void* x, int dtype, float* u, int64_t N,
                                                                     double xi) {
  const int64_t stride = (int64_t)gridDim.x * kMmThreads;
  for (int64_t m = (int64_t)blockIdx.x * kMmThreads + threadIdx.x; m < N; m += stride) {
    const float v = load1(x, dtype, m);
    double s, c;
    sincos(xi * (double)m, &s, &c);
    u[m] = (float)((double)v * c);
    u[N + m] = (float)(-(double)v * s);
    u[2 * N + m] = v;
  }
}

// W[n] = ce (e^{i xi n} (g[n] + i g[N + n]) - kappa g[2N + n])
__global__ __launch_bounds__(kMmThreads) void mm_remodulate_kernel(const float* g, float2* W, int64_t N, double xi,
                                                                     double ce, double cek) {
  const int64_t stride = (int64_t)gridDim.x * kMmThreads;
  for (int64_t n = (int64_t)blockIdx.x * kMmThreads + threadIdx.x; n < N; n += stride) {
    double s, c;
    sincos(xi * (double)n, &s, &c);
    const double gc = g[n], gs = g[N + n], gx = g[2 * N + n];
    W[n] = make_float2((float)(ce * (c * gc - s * gs) - cek * gx), (float)(ce * (s * gc + c * gs)));
  }
}

// Transposes for the backward (real loss, gW = dLoss/dRe W + i dLoss/dIm W):
//   g[n] = ce (gWr cos + gWi sin), g[N + n] = ce (gWi cos - gWr sin), g[2N + n] = -ce kappa gWr
__global__ __launch_bounds__(kMmThreads) void mm_remodulate_t_kernel(const float2* gW, float* g, int64_t N, double xi,
                                                                       double ce, double cek) {
  const int64_t stride = (int64_t)gridDim.x * kMmThreads;
  for (int64_t n = (int64_t)blockIdx.x * kMmThreads + threadIdx.x; n < N; n += stride) {
    double s, c;
    sincos(xi * (double)n, &s, &c);
    const double gr = gW[n].x, gi = gW[n].y;
    g[n] = (float)(ce * (gr * c + gi * s));
    g[N + n] = (float)(ce * (gi * c - gr * s));
    g[2 * N + n] = (float)(-cek * gr);
  }
}

//   gx[m] = cos(xi m) gu[m] - sin(xi m) gu[N + m] + gu[2N + m]
__global__ __launch_bounds__(kMmThreads) void mm_demodulate_t_kernel(const float* gu, float* gx, int64_t N, double xi) {
  const int64_t stride = (int64_t)gridDim.x * kMmThreads;
  for (int64_t m = (int64_t)blockIdx.x * kMmThreads + threadIdx.x; m < N; m += stride) {
    double s, c;
    sincos(xi * (double)m, &s, &c);
    gx[m] = (float)(c * (double)gu[m] - s * (double)gu[N + m] + (double)gu[2 * N + m]);
  }
}

int mm_grid(int64_t N) {
  const int64_t blocks = (N + kMmThreads - 1) / kMmThreads;
  return (int)std::max<int64_t>(1, std::min<int64_t>(blocks, 8192));
}

}  // namespace

hipError_t launch_mm_demodulate(const void* x, int dtype, float* u, int64_t N, double xi, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(mm_demodulate_kernel, dim3(mm_grid(N)), dim3(kMmThreads), 0, s, x, dtype, u, N, xi);
  return hipGetLastError();
}

hipError_t launch_mm_remodulate(const float* g, float2* W, int64_t N, double xi, double ce, double cek,
                                hipStream_t s) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(mm_remodulate_kernel, dim3(mm_grid(N)), dim3(kMmThreads), 0, s, g, W, N, xi, ce, cek);
  return hipGetLastError();
}

hipError_t launch_mm_remodulate_t(const float2* gW, float* g, int64_t N, double xi, double ce, double cek,
                                  hipStream_t s) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(mm_remodulate_t_kernel, dim3(mm_grid(N)), dim3(kMmThreads), 0, s, gW, g, N, xi, ce, cek);
  return hipGetLastError();
}

hipError_t launch_mm_demodulate_t(const float* gu, float* gx, int64_t N, double xi, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(mm_demodulate_t_kernel, dim3(mm_grid(N)), dim3(kMmThreads), 0, s, gu, gx, N, xi);
  return hipGetLastError();
}

}  // namespace mk
