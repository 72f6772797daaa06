// Dispatch of the scan kernels, the gradient finalize and scale-sum kernels and the
// workspace fill kernel.
#include <hip/hip_runtime.h>

#include <atomic>

#include <algorithm>

#include "launch.h"
#include "scan_common.h"

namespace mk {

using KernelFn = void (*)(ScanLaunch);
// Selectors of the per-(K, R) instantiation sets, one object each (scan_inst.hip).
using SelectFn = KernelFn (*)(int var, int acc, int kind, int mom, int dt);
#define MK_DECL_R(K) \
  KernelFn select_scan_k##K##_r4(int, int, int, int, int); KernelFn select_scan_k##K##_r8(int, int, int, int, int); \
  KernelFn select_scan_k##K##_r16(int, int, int, int, int); KernelFn select_scan_k##K##_r32(int, int, int, int, int);
MK_DECL_R(1) MK_DECL_R(2) MK_DECL_R(3) MK_DECL_R(4) MK_DECL_R(5) MK_DECL_R(6)
MK_DECL_R(7) MK_DECL_R(8) MK_DECL_R(9) MK_DECL_R(10) MK_DECL_R(11) MK_DECL_R(12)
#undef MK_DECL_R

namespace {

// index of a supported tile shape: R = 4, 8, 16, 32 -> 0..3, else -1
int r_index(int R) { return R == 4 ? 0 : R == 8 ? 1 : R == 16 ? 2 : R == 32 ? 3 : -1; }

KernelFn select_kernel(int K, int R, int var, int acc, int kind, int mom, int dt) {
#define MK_ROW(K) {select_scan_k##K##_r4, select_scan_k##K##_r8, select_scan_k##K##_r16, select_scan_k##K##_r32}
  static const SelectFn table[kMaxTerms][4] = {MK_ROW(1), MK_ROW(2), MK_ROW(3), MK_ROW(4),  MK_ROW(5),  MK_ROW(6),
                                               MK_ROW(7), MK_ROW(8), MK_ROW(9), MK_ROW(10), MK_ROW(11), MK_ROW(12)};
#undef MK_ROW
  const int ri = r_index(R);
  if (K < 1 || K > kMaxTerms || ri < 0) return nullptr;
  return table[K - 1][ri](var, acc, kind, mom, dt);
}

__global__ void zero_fill_kernel(uint4* p, size_t n16, unsigned char* tail, size_t ntail) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

// One block per scale. The per-tile partial sums of the gradient pass are summed in a fixed
// order (tile k of the scale goes to thread k mod 256, then a fixed tree), then turned into
// dLoss/dsigma and dLoss/dxi:
//   dL/dm_p = sgn_p (e^{aL} S1_p + e^{-aL} Sx),  dL/dl_p = sgn_p e^{aL} S2_p   (chain rule
//   through the fitted coefficients, Jacobian rows from the plan), plus for ASFT the output
//   scale (n0^2/sigma^3 Re Q), the carrier phase (-n0 Im Q) and the decay
//   dL/dalpha = sum_p sgn_p [m_p (e^{aL} (L S1_p + S3_p) - L e^{-aL} Sx) + l_p e^{aL} (L S2_p + S4_p)],
//   dalpha/dsigma = -2 n0 / sigma^3.
// Per-row sums of the tile partials (block r = row r): a row's tiles are consecutive, so its
// partials are one contiguous [ntiles][NRED] block; thread (g, q) = (tid / NRED, tid % NRED)
// adds value q of tiles g, g + G, ... (G = 256 / NRED groups, coalesced reads), and the G
// group sums are added in order.
__global__ __launch_bounds__(256) void pg_rows_kernel(ScanLaunch P, int K, double* rowpart) {
  const int r = blockIdx.x, tid = threadIdx.x;
  const int NRED = 4 * K + 3, G = 256 / NRED, g = tid / NRED, q = tid % NRED;
  __shared__ double red[256];
  const Row row = P.nrows == 1 ? P.row0 : P.rows[r];
  double acc = 0.0;
  if (g < G)
    for (int64_t t = g; t < row.ntiles; t += G) acc += P.partials[(size_t)(row.tile0 + t) * NRED + q];
  red[tid] = acc;
  __syncthreads();
  if (tid < NRED) {
    double sum = 0.0;
    for (int h = 0; h < G; ++h) sum += red[h * NRED + tid];
    rowpart[(size_t)r * NRED + tid] = sum;
  }
}

__global__ __launch_bounds__(256) void pg_finalize_kernel(ScanLaunch P, int K, const double* rowpart,
                                                          double* gparams) {
  const int s = blockIdx.x, tid = threadIdx.x;
  const int NRED = 4 * K + 3;
  __shared__ double tot[4 * kMaxTerms + 3];
  // the scale's rows: b S + s for every signal b of a batched launch (rows are signal-major,
  // one block per scale), or the only row; summed in signal order
  const int S = gridDim.x;
  const int nb = P.nrows == 1 ? 1 : P.nrows / S;
  if (tid < NRED) {
    double sum = 0.0;
    for (int b = 0; b < nb; ++b) sum += rowpart[((size_t)b * S + s) * NRED + tid];
    tot[tid] = sum;
  }
  __syncthreads();
  if (tid == 0) {
    const TabLayout lay{K, P.R};
    const double* td = reinterpret_cast<const double*>(P.tabs + (int64_t)s * P.tab_stride + P.f32_bytes);
    const double up = td[lay.sUP()], dn = td[lay.sDN()], LL = td[lay.sLL()];
    const double* S = tot;
    const double Sx = S[4 * K], Qr = S[4 * K + 1], Qi = S[4 * K + 2];
    double ds = td[lay.sDSIG()] * Qr, dx = -td[lay.sDXI()] * Qi, dal = 0.0;
    for (int t = 0; t < K; ++t) {
      const double sg = td[lay.rSGN() * K + t];
      const double gm = sg * (up * S[t] + dn * Sx), gl = sg * up * S[K + t];
      ds += td[lay.rJ(0) * K + t] * gm + td[lay.rJ(2) * K + t] * gl;
      dx += td[lay.rJ(1) * K + t] * gm + td[lay.rJ(3) * K + t] * gl;
      const double cc = td[lay.rCC() * K + t], sc = td[lay.rSC() * K + t];
      dal += sg * (cc * (up * (LL * S[t] + S[2 * K + t]) - LL * dn * Sx) + sc * up * (LL * S[K + t] + S[3 * K + t]));
    }
    ds += td[lay.sDALPHA()] * dal;
    gparams[2 * s] = ds;
    gparams[2 * s + 1] = dx;
  }
}

// out[x_off_b + n] = sum_s part[S x_off_b + s len_b + n]: the adjoints of one signal's
// scales summed in scale order. Row b S is scale 0 of signal b.
// Four consecutive outputs per thread. Where the four lie in one signal and every scale's run of
// them, and the four outputs, are 16-byte aligned (N a multiple of 4), each scale is one 16-byte load; otherwise the
// elements are summed one by one. Either way every output adds its S terms in scale order, so
// the result does not depend on the path.
__global__ __launch_bounds__(256) void sum_scales_kernel(const float* part, float* out, const Row* rows, int B, int S,
                                                         int64_t total) {
  auto signal_of = [&](int64_t e) {   // last signal with x_off <= e
    int lo = 0, hi = B - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (rows[(int64_t)mid * S].x_off <= e) lo = mid; else hi = mid - 1;
    }
    return lo;
  };
  const bool aligned = ((reinterpret_cast<uintptr_t>(part) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
  for (int64_t e0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; e0 < total; e0 += stride) {
    const Row r0 = rows[(int64_t)signal_of(e0) * S];
    const int64_t n = e0 - r0.x_off;
    const int64_t base = (int64_t)S * r0.x_off + n;
    if (aligned && n + 4 <= r0.N && e0 + 4 <= total && (base & 3) == 0 && (r0.N & 3) == 0) {
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
      for (int s = 0; s < S; ++s) {
        const float4 v = *reinterpret_cast<const float4*>(part + base + (int64_t)s * r0.N);
        acc.x += v.x; acc.y += v.y; acc.z += v.z; acc.w += v.w;
      }
      *reinterpret_cast<float4*>(out + e0) = acc;
    } else {
      for (int64_t e = e0; e < e0 + 4 && e < total; ++e) {
        const Row r = rows[(int64_t)signal_of(e) * S];
        const int64_t m = e - r.x_off;
        float acc = 0.f;
        for (int s = 0; s < S; ++s) acc += part[(int64_t)S * r.x_off + (int64_t)s * r.N + m];
        out[e] = acc;
      }
    }
  }
}

// Segments schedule, between its two passes (one block per row): the segment sums have left in
// segstate[s] the state A_s at the end of segment s from a zero state at its start. The state
// at the start of the row's segment s is
//   S_0 = 0,  S_{s+1} = c S_s + A_s,  c = a^{T len} (per term; every segment but the last, which
// precedes none, has len tiles of T positions),
// written over A_s. In rounds of 1024 segments, four consecutive ones per thread (their loads in
// flight together): each thread folds its four (Horner with c), the folds are scanned across the
// wave with C = c^4 (Hillis-Steele, the constant squared per level, C^lane formed from the same
// squares), the four wave totals are chained in order through LDS, and each thread writes the
// incoming states of its four from its exclusive prefix; the state after the round carries into
// the next. Float64 throughout, a fixed order, so the result does not depend on timing. One wave
// per SIMD leaves the registers for all K terms at once (without spills up to K = 6).
template <int K>
__global__ __launch_bounds__(256) void seg_combine_kernel(ScanLaunch P) {
  constexpr int NW = 4, NT = NW * 64, Q = 4;
  __shared__ double s_tot[NW][2 * K];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int rr = blockIdx.x;   // one block per row
  const Row row = P.nrows == 1 ? P.row0 : P.rows[rr];
  const TabLayout lay{K, P.R};
  const Tab<true> tabd{(cptr<double>)(P.tabs + (int64_t)row.scale * P.tab_stride + P.f32_bytes), K};
  const int len = P.seg_len;
  auto cmul = [](double ar, double ai, double br, double bi, double& outr, double& outi) {
    outr = ar * br - ai * bi;
    outi = ar * bi + ai * br;
  };
  double cr[K], ci[K];
#pragma unroll
  for (int t = 0; t < K; ++t) {
    if (len <= kLookback) {
      cr[t] = tabd.re(lay.eLB(len), t);
      ci[t] = tabd.im(lay.eLB(len), t);
    } else {   // a^{T len} = a^{64 T (len / 64)} a^{T (len mod 64)}
      cmul(tabd.re(lay.eLB2(len / kLookback), t), tabd.im(lay.eLB2(len / kLookback), t),
           tabd.re(lay.eLB(len % kLookback), t), tabd.im(lay.eLB(len % kLookback), t), cr[t], ci[t]);
    }
  }
  const int64_t n = P.seg_start[rr + 1] - P.seg_start[rr];
  double* st = P.segstate + (int64_t)P.seg_start[rr] * 2 * K;
  double carry_r[K], carry_i[K];   // the state entering the round
#pragma unroll
  for (int t = 0; t < K; ++t) { carry_r[t] = 0; carry_i[t] = 0; }
  for (int64_t base = 0; base < n; base += (int64_t)Q * NT) {
    const int64_t k0 = base + (int64_t)Q * tid;
    double ar[Q][K], ai[Q][K];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int t = 0; t < K; ++t) {
        ar[q][t] = k0 + q < n ? st[(k0 + q) * 2 * K + 2 * t] : 0.0;
        ai[q][t] = k0 + q < n ? st[(k0 + q) * 2 * K + 2 * t + 1] : 0.0;
      }
    // the fold of the four, then the inclusive scan over the wave; pw = C^(2^d), pl = C^lane
    double gr[K], gi[K], pwr[K], pwi[K], plr[K], pli[K];
#pragma unroll
    for (int t = 0; t < K; ++t) {
      gr[t] = 0;
      gi[t] = 0;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        double vr, vi;
        cmul(cr[t], ci[t], gr[t], gi[t], vr, vi);
        gr[t] = vr + ar[q][t];
        gi[t] = vi + ai[q][t];
      }
      double c2r, c2i;
      cmul(cr[t], ci[t], cr[t], ci[t], c2r, c2i);
      cmul(c2r, c2i, c2r, c2i, pwr[t], pwi[t]);
      plr[t] = 1;
      pli[t] = 0;
    }
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      const int sh = 1 << d;
#pragma unroll
      for (int t = 0; t < K; ++t) {
        const double ur = __shfl_up(gr[t], sh, 64), ui = __shfl_up(gi[t], sh, 64);
        double vr, vi;
        if (lane >= sh) {
          cmul(pwr[t], pwi[t], ur, ui, vr, vi);
          gr[t] += vr;
          gi[t] += vi;
        }
        if (lane & sh) {
          cmul(plr[t], pli[t], pwr[t], pwi[t], vr, vi);
          plr[t] = vr;
          pli[t] = vi;
        }
        cmul(pwr[t], pwi[t], pwr[t], pwi[t], vr, vi);
        pwr[t] = vr;
        pwi[t] = vi;
      }
    }
    // pw is now C^64, the step across one wave
    if (lane == 63) {
#pragma unroll
      for (int t = 0; t < K; ++t) { s_tot[wid][2 * t] = gr[t]; s_tot[wid][2 * t + 1] = gi[t]; }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < K; ++t) {
      // Y: the state entering each wave in turn, from the round's carry; the one entering this
      // thread's wave is kept, the one after the last wave is the next round's carry
      double yr = carry_r[t], yi = carry_i[t], wr = 0, wi = 0;
#pragma unroll
      for (int v = 0; v < NW; ++v) {
        if (v == wid) { wr = yr; wi = yi; }
        double vr, vi;
        cmul(pwr[t], pwi[t], yr, yi, vr, vi);
        yr = vr + s_tot[v][2 * t];
        yi = vi + s_tot[v][2 * t + 1];
      }
      carry_r[t] = yr;
      carry_i[t] = yi;
      // the thread's incoming state: the wave-exclusive prefix plus C^lane times the wave's entry
      const double er = __shfl_up(gr[t], 1, 64), ei = __shfl_up(gi[t], 1, 64);
      double vr, vi;
      cmul(plr[t], pli[t], wr, wi, vr, vi);
      double sr = (lane > 0 ? er : 0.0) + vr, si = (lane > 0 ? ei : 0.0) + vi;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        if (k0 + q < n) {
          st[(k0 + q) * 2 * K + 2 * t] = sr;
          st[(k0 + q) * 2 * K + 2 * t + 1] = si;
        }
        cmul(cr[t], ci[t], sr, si, vr, vi);
        sr = vr + ar[q][t];
        si = vi + ai[q][t];
      }
    }
    __syncthreads();   // s_tot is rewritten by the next round
  }
}

hipError_t launch_seg_combine(const ScanLaunch& a, hipStream_t s) {
  switch (a.K) {
#define MK_SEG(K) \
  case K: hipLaunchKernelGGL(seg_combine_kernel<K>, dim3(a.nrows), dim3(256), 0, s, a); break;
    MK_SEG(1) MK_SEG(2) MK_SEG(3) MK_SEG(4) MK_SEG(5) MK_SEG(6) MK_SEG(7) MK_SEG(8) MK_SEG(9) MK_SEG(10)
    MK_SEG(11) MK_SEG(12)
#undef MK_SEG
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_scan(const ScanLaunch& a, int variant, int mom, hipStream_t s) {
  KernelFn fn = select_kernel(a.K, a.R, variant, a.acc, a.kind, mom, variant == kVarAdjoint ? 0 : a.dtype);
  if (!fn) return hipErrorInvalidValue;
  if (a.nseg > 0) {
    if (variant != kVarForward || !a.serial || a.nrows < 1 || a.nrows > kQueues || !a.segstate || a.seg_len < 1 ||
        a.seg_len > kLookback * kLookback || a.seg_start[0] != 0 || a.seg_start[a.nrows] != a.nseg)
      return hipErrorInvalidValue;
    KernelFn sum = select_kernel(a.K, a.R, kVarSegSum, 0, 0, 0, a.dtype);
    if (!sum || a.nseg > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(sum, dim3((unsigned)a.nseg), dim3(kThreads), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_seg_combine(a, s);
    if (e != hipSuccess) return e;
    ScanLaunch b = a;
    b.seg_mode = 1;
    hipLaunchKernelGGL(fn, dim3(b.grid), dim3(kThreads), 0, s, b);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(fn, dim3(a.grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

int scan_occupancy(int K, int R, int variant, int acc, int kind, int mom, int dtype) {
  // resident blocks per CU of one kernel instantiation; queried once per instantiation (every
  // device this library runs on is a gfx950) and kept, so launches make no runtime query
  static std::atomic<int> cache[kMaxTerms + 1][4][3][4][4][2][3];
  if (K < 1 || K > kMaxTerms || r_index(R) < 0 || variant < 0 || variant > 2 || acc < 0 || acc > 3 ||
      kind < 0 || kind > 3 || mom < 0 || mom > 1 || dtype < 0 || dtype > 2)
    return 0;
  std::atomic<int>& slot = cache[K][r_index(R)][variant][acc][kind][mom][variant == kVarAdjoint ? 0 : dtype];
  const int known = slot.load(std::memory_order_relaxed);
  if (known > 0) return known;
  KernelFn fn = select_kernel(K, R, variant, acc, kind, mom, variant == kVarAdjoint ? 0 : dtype);
  if (!fn) return 0;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(fn), kThreads, 0) != hipSuccess)
    return 1;
  n = n > 0 ? n : 1;
  slot.store(n, std::memory_order_relaxed);
  return n;
}

hipError_t launch_scan_forward(const ScanLaunch& a, hipStream_t s) { return launch_scan(a, kVarForward, 0, s); }

int scan_forward_occupancy(int K, int R, int acc, int kind) { return scan_occupancy(K, R, kVarForward, acc, kind, 0, 0); }

hipError_t launch_pg_finalize(const ScanLaunch& a, int nscales, double* rowpart, double* gparams, hipStream_t s) {
  hipLaunchKernelGGL(pg_rows_kernel, dim3(a.nrows), dim3(256), 0, s, a, a.K, rowpart);
  hipLaunchKernelGGL(pg_finalize_kernel, dim3(nscales), dim3(256), 0, s, a, a.K,
                     static_cast<const double*>(rowpart), gparams);
  return hipGetLastError();
}

hipError_t launch_sum_scales(const float* part, float* out, const Row* rows, int B, int S, int64_t total,
                             hipStream_t s) {
  if (total <= 0) return hipSuccess;
  const unsigned int blocks = (unsigned int)std::min<int64_t>((total + 1023) / 1024, 8192);
  hipLaunchKernelGGL(sum_scales_kernel, dim3(blocks), dim3(256), 0, s, part, out, rows, B, S, total);
  return hipGetLastError();
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
