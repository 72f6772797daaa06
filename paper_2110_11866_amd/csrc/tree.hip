// The paper's own GPU route (Sec. IV), built as a comparison path beside the scan: for each
// order p the window sum S_p[n] = sum_{j=n-L}^{n+L} x[j] e^{i beta p j} by binary doubling
// (Algorithm 1: g_{r+1}[n] = g_r[n] + g_r[n + 2^r], and h <- g_r[n] + h[n + 2^r] for every set
// bit r of the window length 2L + 1), then Z_p[n] = e^{-i beta p n} S_p[n] and the K-term
// combination. O(N K log L) work in log2(2L + 1) levels.
//
// Layout: per term a planar array of M = N + 2L complex float32 positions, f_p[m] =
// x[m - L] e^{i beta p (m - L)} (zero outside the signal). The paper does three levels per
// pass in 16 x 8 shared-memory blocks and rearranges the array between passes; here the first
// nine levels run in one pass through 1024-position LDS tiles (with a 511-position halo), and
// each further level is one coalesced pass over global memory (g and h ping-pong between two
// buffers each). Phases use the exact index (p j) mod 2L, as the scan's tables do.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "launch.h"
#include "scan_common.h"

namespace mk {
namespace {

constexpr int kTrThreads = 256;
constexpr int kTrTile = 1024;                 // positions per block in the LDS pass
constexpr int kTrMaxLow = 9;                  // levels done in LDS
constexpr int kTrSpan = kTrTile + (1 << kTrMaxLow);
constexpr int kTrPer = (kTrSpan + kTrThreads - 1) / kTrThreads;

// e^{i pi idx / L} for the exact index idx = (p j) mod 2L
__device__ __forceinline__ float2 tr_phase(int64_t p, int64_t j, int64_t L) {
  int64_t idx = (p * j) % (2 * L);
  if (idx < 0) idx += 2 * L;
  double s, c;
  sincospi((double)idx / (double)L, &s, &c);
  return make_float2((float)c, (float)s);
}

// Levels 0..nlow-1 of term blockIdx.y for positions [t0, t0 + kTrTile) of f.
__global__ __launch_bounds__(kTrThreads) void tree_low_kernel(const void* x, int dtype, int64_t N, int64_t L,
                                                              int P_S, int64_t M, int64_t Lw, int nlow, float2* G,
                                                              float2* H) {
  __shared__ float2 sg[kTrSpan], sh[kTrSpan];
  const int tid = threadIdx.x;
  const int64_t t0 = (int64_t)blockIdx.x * kTrTile;
  const int64_t p = P_S + (int64_t)blockIdx.y;
  const int span = kTrTile + (1 << nlow);
  for (int i = tid; i < span; i += kTrThreads) {
    const int64_t m = t0 + i, j = m - L;
    float2 v = make_float2(0.f, 0.f);
    if (m < M && j >= 0 && j < N) {
      const float xv = load1(x, dtype, j);
      const float2 e = tr_phase(p, j, L);
      v = make_float2(xv * e.x, xv * e.y);
    }
    sg[i] = v;
    sh[i] = make_float2(0.f, 0.f);
  }
  __syncthreads();
  for (int r = 0; r < nlow; ++r) {
    const int s = 1 << r;
    const bool bit = (Lw >> r) & 1;
    float2 ng[kTrPer], nh[kTrPer];
#pragma unroll
    for (int q = 0; q < kTrPer; ++q) {
      const int i = tid + q * kTrThreads;
      if (i + s < span) {   // entries whose reads stay in the tile (the rest are never used)
        const float2 a = sg[i], b = sg[i + s];
        ng[q] = make_float2(a.x + b.x, a.y + b.y);
        if (bit) {
          const float2 c = sh[i + s];
          nh[q] = make_float2(a.x + c.x, a.y + c.y);
        } else {
          nh[q] = sh[i];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kTrPer; ++q) {
      const int i = tid + q * kTrThreads;
      if (i + s < span) {
        sg[i] = ng[q];
        sh[i] = nh[q];
      }
    }
    __syncthreads();
  }
  float2* Gp = G + (int64_t)blockIdx.y * M;
  float2* Hp = H + (int64_t)blockIdx.y * M;
  for (int i = tid; i < kTrTile; i += kTrThreads) {
    const int64_t m = t0 + i;
    if (m < M) {
      Gp[m] = sg[i];
      Hp[m] = sh[i];
    }
  }
}

// One level r >= nlow over all terms: g' = g[m] + g[m + s]; h' = g[m] + h[m + s] if the bit is set
// (reads past M are zero, as f is). On the last level g' is not needed.
__global__ __launch_bounds__(kTrThreads) void tree_level_kernel(const float2* Gi, const float2* Hi, float2* Go,
                                                                float2* Ho, int64_t M, int K, int64_t s, int bit,
                                                                int last) {
  const int64_t total = M * K;
  const int64_t stride = (int64_t)gridDim.x * kTrThreads;
  for (int64_t e = (int64_t)blockIdx.x * kTrThreads + threadIdx.x; e < total; e += stride) {
    const int64_t m = e % M;
    const float2 a = Gi[e];
    const bool in = m + s < M;
    if (!last) {
      const float2 b = in ? Gi[e + s] : make_float2(0.f, 0.f);
      Go[e] = make_float2(a.x + b.x, a.y + b.y);
    }
    if (bit) {
      const float2 c = in ? Hi[e + s] : make_float2(0.f, 0.f);
      Ho[e] = make_float2(a.x + c.x, a.y + c.y);
    }
  }
}

// W[n] = sum_t cc_t Re Z_t[n] - i sc_t Im Z_t[n], Z_t[n] = e^{-i beta p n} S_t[n], p = P_S + t
// (real output: the real part only).
__global__ __launch_bounds__(kTrThreads) void tree_combine_kernel(const float2* Hs, int64_t M, int64_t N, int64_t L,
                                                                  int P_S, TreeCoef c, int real_out, void* W) {
  const int64_t stride = (int64_t)gridDim.x * kTrThreads;
  for (int64_t n = (int64_t)blockIdx.x * kTrThreads + threadIdx.x; n < N; n += stride) {
    double re = 0.0, im = 0.0;
    for (int t = 0; t < c.K; ++t) {
      const float2 S = Hs[(int64_t)t * M + n];
      const float2 e = tr_phase(P_S + t, n, L);   // Z = conj(e) S
      const double zr = (double)e.x * S.x + (double)e.y * S.y;
      const double zi = (double)e.x * S.y - (double)e.y * S.x;
      re += c.cc[t] * zr;
      im -= c.sc[t] * zi;
    }
    if (real_out) static_cast<float*>(W)[n] = (float)re;
    else static_cast<float2*>(W)[n] = make_float2((float)re, (float)im);
  }
}

int tr_grid(int64_t n) {
  const int64_t blocks = (n + kTrThreads - 1) / kTrThreads;
  return (int)std::max<int64_t>(1, std::min<int64_t>(blocks, 8192));
}

}  // namespace

hipError_t launch_tree(const void* x, int dtype, int64_t N, int64_t L, int K, int P_S, const TreeCoef& coef,
                       int real_out, float2* buf, void* W, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  const int64_t M = N + 2 * L, Lw = 2 * L + 1;
  int R = 0;
  while ((Lw >> R) > 0) ++R;
  const int nlow = std::min(R, kTrMaxLow);
  float2* G[2] = {buf, buf + (int64_t)K * M};
  float2* H[2] = {buf + 2 * (int64_t)K * M, buf + 3 * (int64_t)K * M};
  const int64_t ntile = (M + kTrTile - 1) / kTrTile;
  if (ntile > 0x7fffffff || K > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(tree_low_kernel, dim3((unsigned)ntile, (unsigned)K), dim3(kTrThreads), 0, s, x, dtype, N, L, P_S,
                     M, Lw, nlow, G[0], H[0]);
  hipError_t e = hipGetLastError();
  int gc = 0, hc = 0;
  for (int r = nlow; r < R && e == hipSuccess; ++r) {
    const int bit = (int)((Lw >> r) & 1);
    const int last = r == R - 1;
    hipLaunchKernelGGL(tree_level_kernel, dim3(tr_grid(M * K)), dim3(kTrThreads), 0, s, G[gc], H[hc], G[gc ^ 1],
                       H[hc ^ 1], M, K, (int64_t)1 << r, bit, last);
    e = hipGetLastError();
    gc ^= 1;
    if (bit) hc ^= 1;
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(tree_combine_kernel, dim3(tr_grid(N)), dim3(kTrThreads), 0, s, H[hc], M, N, L, P_S, coef,
                     real_out, W);
  return hipGetLastError();
}

}  // namespace mk
