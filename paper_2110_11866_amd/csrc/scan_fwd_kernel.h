// Forward kernel (gfx950): K-term SFT / ASFT of one or many scan rows, one fused pass.
//
// What is computed (per row, per term p = P_S + i, a = e^{-alpha} e^{-i beta p}):
//   the windowed kernel integral of eq. kernelInt written in its demodulated form,
//     v_p[j] = sum_{q=j-2L+1}^{j} a^{j-q} x[q]                   (2L window, eq. iir12K / aiir12K)
//   obtained as one prefix scan of the differenced input (eq. kernelIntZenka: the window
//   difference is taken on the input, before the scan)
//     v_p[j] = a v_p[j-1] + dx[j],   dx[j] = x[j] - a^{2L} x[j-2L],  a^{2L} = e^{-2 alpha L},
//   then the SFT / ASFT component (eqs. sfiir12K, asfiir12K with the prefactor e^{+alpha L})
//     c_p - i s_p = (-1)^p (e^{alpha L} v_p[j] + e^{-alpha L} x[j-2L]),   j = n - n0 + L,
//   and the K-term combination of Sec. III-A (Morlet) or eq. GsSFT / GsASFT (Gaussian).
//   Multiplying v_p by e^{i beta p j} gives the modulated kernel integral u_(2L)[j] of
//   eqs. kernel..kernelInter; carrying the demodulated state makes every constant a power
//   of a at a fixed distance, identical for all tiles.
//
// How (one block = one tile of T = 256 R scan positions, persistent grid, ticketed tiles):
//   1. each thread loads R consecutive x[j] and x[j-2L] and forms dx (coalesced runs);
//   2. chunk sums B_p = sum_r a^{R-1-r} dx[r] (the thread's contribution to the state);
//   3. inclusive scan of the chunk sums across the wavefront (6 shuffle levels, constants
//      a^{R 2^d});
//   4. wave 0 forms the tile aggregate in float64, publishes it, and resolves the tile's
//      exclusive prefix by a deterministic decoupled look-back: the aggregates of the
//      earlier tiles of its 64-tile group plus the inclusive prefix of the previous
//      group's last tile, combined in a fixed order (flags read lane-parallel, float64
//      payloads, agent-scope atomics that bypass the per-XCD L2, so tiles on different
//      XCDs see each other's states);
//   5. each thread rotates its carry in, runs the R-step recurrence and combines the K
//      terms into the output, staged through LDS for coalesced complex64 / float32 stores.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "launch.h"

namespace mk {
namespace {

// ------------------------------------------------------------ coherent tile-state access
__device__ __forceinline__ void st_u64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_u64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_f64(double* p, double v) {
  st_u64(reinterpret_cast<uint64_t*>(p), (uint64_t)__double_as_longlong(v));
}
__device__ __forceinline__ double ld_f64(const double* p) {
  return __longlong_as_double((long long)ld_u64(reinterpret_cast<const uint64_t*>(p)));
}
// s_waitcnt vmcnt(0): wait for all of this wave's vector memory operations.
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }
__device__ __forceinline__ void release_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  wait_vmem();
}
__device__ __forceinline__ void acquire_order() {
  wait_vmem();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

struct TileState {
  unsigned char* b;
  int K;
  __device__ uint64_t* flag() const { return reinterpret_cast<uint64_t*>(b); }
  __device__ double* agg(int i, int c) const { return reinterpret_cast<double*>(b + 8) + 2 * i + c; }
  __device__ double* inc(int i, int c) const { return reinterpret_cast<double*>(b + 8) + 2 * K + 2 * i + c; }
};

// ------------------------------------------------------------ input loads
__device__ __forceinline__ float cvt_f16(unsigned short h) {
  return (float)__builtin_bit_cast(_Float16, h);
}
__device__ __forceinline__ float cvt_bf16(unsigned short h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float load1(const void* base, int dtype, int64_t j) {
  if (dtype == 0) return static_cast<const float*>(base)[j];
  const unsigned short h = static_cast<const unsigned short*>(base)[j];
  return dtype == 1 ? cvt_f16(h) : cvt_bf16(h);
}

// v[r] = x[j + r] for r < R, zero outside [0, N).
template <int R>
__device__ __forceinline__ void load_run(const void* base, int dtype, int64_t j, int64_t N, float (&v)[R]) {
  if (j >= 0 && j + R <= N) {
    if (dtype == 0) {
      const float* p = static_cast<const float*>(base) + j;
      if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {
#pragma unroll
        for (int r = 0; r < R; r += 4) {
          const float4 q = *reinterpret_cast<const float4*>(p + r);
          v[r] = q.x; v[r + 1] = q.y; v[r + 2] = q.z; v[r + 3] = q.w;
        }
      } else if ((reinterpret_cast<uintptr_t>(p) & 7) == 0) {
#pragma unroll
        for (int r = 0; r < R; r += 2) {
          const float2 q = *reinterpret_cast<const float2*>(p + r);
          v[r] = q.x; v[r + 1] = q.y;
        }
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = p[r];
      }
    } else {
      const unsigned short* p = static_cast<const unsigned short*>(base) + j;
      if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {
#pragma unroll
        for (int r = 0; r < R; r += 8) {
          const uint4 q = *reinterpret_cast<const uint4*>(p + r);
          const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
          for (int h = 0; h < 4; ++h) {
            const unsigned short lo = (unsigned short)(w[h] & 0xffffu), hi = (unsigned short)(w[h] >> 16);
            v[r + 2 * h] = dtype == 1 ? cvt_f16(lo) : cvt_bf16(lo);
            v[r + 2 * h + 1] = dtype == 1 ? cvt_f16(hi) : cvt_bf16(hi);
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = dtype == 1 ? cvt_f16(p[r]) : cvt_bf16(p[r]);
      }
    }
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t q = j + r;
      v[r] = (q >= 0 && q < N) ? load1(base, dtype, q) : 0.0f;
    }
  }
}

// ------------------------------------------------------------ constant table access
// Table reads go through the constant address space: uniform indices become scalar loads
// into SGPRs instead of occupying vector registers.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

template <bool WIDE>
struct Tab {
  using T = typename std::conditional<WIDE, double, float>::type;
  cptr<T> p;
  int K;
  __device__ T re(int e, int i) const { return p[(2 * e) * K + i]; }
  __device__ T im(int e, int i) const { return p[(2 * e + 1) * K + i]; }
  __device__ T row(int rrow, int i) const { return p[rrow * K + i]; }
  __device__ T scalar(int s) const { return p[s]; }
};

template <int K, int R, bool WIDE, bool GAUSS>
__global__ __launch_bounds__(kThreads) void scan_forward_kernel(ScanLaunch P) {
  using acc_t = typename std::conditional<WIDE, double, float>::type;
  constexpr int T = R * kThreads;
  constexpr int LSTR = GAUSS ? (R + 1) : (2 * R + 2);  // padded per-lane stride of the staging buffer

  __shared__ uint32_t s_tile;
  __shared__ double s_wagg[kWaves][2 * K];
  __shared__ double s_xw[kWaves][2 * K];
  __shared__ float s_stage[kWaves][64 * LSTR];

  WsHeader* hdr = static_cast<WsHeader*>(P.ws);
  unsigned char* states = static_cast<unsigned char*>(P.ws) + sizeof(WsHeader);
  const size_t sbytes = tile_state_bytes(K);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const uint64_t epoch = ld_u64(&hdr->epoch);
  const uint64_t tag = (epoch + 1) << 2;
  const TabLayout lay{K, R};
  const int esz = P.dtype == 0 ? 4 : 2;

  for (;;) {
    if (tid == 0) s_tile = atomicAdd(&hdr->ticket, 1u);
    __syncthreads();
    const uint32_t tile = __builtin_amdgcn_readfirstlane(s_tile);
    if ((int64_t)tile >= P.ntiles) break;
    Row row = P.row0;
    if (P.nrows != 1) {
      const cptr<Row> rp = (cptr<Row>)P.rows + __builtin_amdgcn_readfirstlane(((cptr<int32_t>)P.tile_row)[tile]);
      row.x_off = rp->x_off; row.w_off = rp->w_off; row.N = rp->N; row.L = rp->L;
      row.jout0 = rp->jout0; row.jend = rp->jend; row.tile0 = rp->tile0;
      row.scale = rp->scale; row.ntiles = rp->ntiles;
    }

    const int64_t ti = (int64_t)tile - row.tile0;
    const int64_t jt = ti * T;
    const int64_t j0 = jt + (int64_t)tid * R;
    const unsigned char* tb = P.tabs + (int64_t)row.scale * P.tab_stride;
    const Tab<WIDE> tab{(cptr<acc_t>)(WIDE ? tb + P.f32_bytes : tb), K};
    const Tab<true> tabd{(cptr<double>)(tb + P.f32_bytes), K};
    const void* xs = static_cast<const char*>(P.x) + row.x_off * esz;

    // 1. differenced input dx[j] = x[j] - a^{2L} x[j-2L] (zero past the row's scan range)
    float xa[R], xb[R];
    load_run<R>(xs, P.dtype, j0, row.N, xa);
    load_run<R>(xs, P.dtype, j0 - 2 * row.L, row.N, xb);
    const acc_t Dw = tab.scalar(lay.sD());
    acc_t dx[R];
#pragma unroll
    for (int r = 0; r < R; ++r)
      dx[r] = (j0 + r < row.jend) ? (acc_t)xa[r] - Dw * (acc_t)xb[r] : (acc_t)0;

    // 2. chunk sums B_i = sum_r a_i^{R-1-r} dx[r]
    acc_t br[K], bi[K];
#pragma unroll
    for (int i = 0; i < K; ++i) { br[i] = 0; bi[i] = 0; }
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int i = 0; i < K; ++i) {
        br[i] = fma(tab.re(lay.eP1(r), i), dx[r], br[i]);
        bi[i] = fma(tab.im(lay.eP1(r), i), dx[r], bi[i]);
      }
    }

    // 3. inclusive scan over the wave: S_l = sum_{m <= l} a^{R (l - m)} B_m
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      const int off = 1 << d;
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const acc_t ur = __shfl_up(br[i], off, 64), ui = __shfl_up(bi[i], off, 64);
        if (lane >= off) {
          const acc_t cr = tab.re(lay.eTR(d), i), ci = tab.im(lay.eTR(d), i);
          br[i] = fma(cr, ur, fma(-ci, ui, br[i]));
          bi[i] = fma(cr, ui, fma(ci, ur, bi[i]));
        }
      }
    }
    // lane-exclusive state E_l = S_{l-1}; the wave's aggregate goes to LDS
    acc_t er[K], ei[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      er[i] = __shfl_up(br[i], 1, 64);
      ei[i] = __shfl_up(bi[i], 1, 64);
      if (lane == 0) { er[i] = 0; ei[i] = 0; }
    }
    if (lane == 63) {
#pragma unroll
      for (int i = 0; i < K; ++i) { s_wagg[wid][2 * i] = (double)br[i]; s_wagg[wid][2 * i + 1] = (double)bi[i]; }
    }
    __syncthreads();

    // 4. tile aggregate, decoupled look-back and per-wave carries (wave 0; lane i = term i)
    if (wid == 0) {
      double Ar = 0, Ai = 0;
      if (lane < K) {
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
          const double cr = tabd.re(lay.eWV(kWaves - 1 - w), lane), ci = tabd.im(lay.eWV(kWaves - 1 - w), lane);
          const double wr = s_wagg[w][2 * lane], wi = s_wagg[w][2 * lane + 1];
          Ar += cr * wr - ci * wi;
          Ai += cr * wi + ci * wr;
        }
      }
      const TileState st{states + (size_t)tile * sbytes, K};
      // Deterministic look-back: tiles are grouped by 64 within the row. Tile i combines,
      // in a fixed order, the aggregates of the earlier tiles of its group and the inclusive
      // prefix of the previous group's last tile, so the float64 sums never depend on timing.
      const int64_t grp0 = (ti / kLookback) * kLookback;      // first tile of the group (row-relative)
      const int dd = (int)(ti - grp0);                        // aggregates to combine
      const bool group_last = (ti % kLookback) == kLookback - 1;
      if (lane < K) { st_f64(st.agg(lane, 0), Ar); st_f64(st.agg(lane, 1), Ai); }
      release_order();
      if (lane == 0) st_u64(st.flag(), tag | kAggregate);
      double Pr = 0, Pi = 0;
      if (ti > 0) {
        for (;;) {
          bool ok = true;
          if (lane < dd || (lane == dd && grp0 > 0)) {
            const uint64_t f = ld_u64(TileState{states + (size_t)((int64_t)tile - 1 - lane) * sbytes, K}.flag());
            const int status = ((f & ~3ull) == tag) ? (int)(f & 3ull) : 0;
            ok = (lane < dd) ? (status >= 1) : (status == 2);
          }
          if (__ballot(!ok) == 0) break;
          __builtin_amdgcn_s_sleep(1);
        }
        acquire_order();
        if (lane < K) {
          const int kmax = grp0 > 0 ? dd : dd - 1;
          for (int k = 0; k <= kmax; ++k) {
            const TileState sk{states + (size_t)((int64_t)tile - 1 - k) * sbytes, K};
            double vr, vi;
            if (k < dd) { vr = ld_f64(sk.agg(lane, 0)); vi = ld_f64(sk.agg(lane, 1)); }
            else { vr = ld_f64(sk.inc(lane, 0)); vi = ld_f64(sk.inc(lane, 1)); }
            const double cr = tabd.re(lay.eLB(k), lane), ci = tabd.im(lay.eLB(k), lane);
            Pr += cr * vr - ci * vi;
            Pi += cr * vi + ci * vr;
          }
        }
      }
      if (group_last) {
        if (lane < K) {
          const double cr = tabd.re(lay.eWV(kWaves), lane), ci = tabd.im(lay.eWV(kWaves), lane);  // a^T
          st_f64(st.inc(lane, 0), cr * Pr - ci * Pi + Ar);
          st_f64(st.inc(lane, 1), cr * Pi + ci * Pr + Ai);
        }
        release_order();
        if (lane == 0) st_u64(st.flag(), tag | kInclusive);
      }
      if (lane < K) {
        double Er = 0, Ei = 0;
        const double ar = tabd.re(lay.eWV(1), lane), ai = tabd.im(lay.eWV(1), lane);
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
          const double cr = tabd.re(lay.eWV(w), lane), ci = tabd.im(lay.eWV(w), lane);
          s_xw[w][2 * lane] = Er + cr * Pr - ci * Pi;
          s_xw[w][2 * lane + 1] = Ei + cr * Pi + ci * Pr;
          const double wr = s_wagg[w][2 * lane], wi = s_wagg[w][2 * lane + 1];
          const double nr = ar * Er - ai * Ei + wr, ni = ar * Ei + ai * Er + wi;
          Er = nr; Ei = ni;
        }
      }
    }
    __syncthreads();

    // 5. thread carry (state just before the thread's first position), recurrence, output
    const bool has_out = (jt + T > row.jout0) && (row.jout0 + row.N > jt);
    if (has_out) {
      acc_t vr[K], vi[K];
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const acc_t xr = (acc_t)s_xw[wid][2 * i], xi = (acc_t)s_xw[wid][2 * i + 1];
        const acc_t cr = tab.re(lay.eLANE(lane), i), ci = tab.im(lay.eLANE(lane), i);
        vr[i] = fma(cr, xr, fma(-ci, xi, er[i]));
        vi[i] = fma(cr, xi, fma(ci, xr, ei[i]));
      }
      const acc_t cx = tab.scalar(lay.sCX());
      const acc_t gre = tab.scalar(lay.sGre()), gim = tab.scalar(lay.sGim());
      float* stg = &s_stage[wid][lane * LSTR];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        acc_t A = cx * (acc_t)xb[r], B = 0;
#pragma unroll
        for (int i = 0; i < K; ++i) {
          const acc_t ar = tab.re(lay.eA(), i), ai = tab.im(lay.eA(), i);
          const acc_t nr = fma(ar, vr[i], fma(-ai, vi[i], dx[r]));
          const acc_t ni = fma(ar, vi[i], ai * vr[i]);
          vr[i] = nr;
          vi[i] = ni;
          A = fma(tab.row(lay.rMW(), i), nr, A);
          if (!GAUSS) B = fma(tab.row(lay.rLW(), i), ni, B);
        }
        if (GAUSS) {
          stg[r] = (float)(gre * A);
        } else {
          stg[2 * r] = (float)(gre * A + gim * B);
          stg[2 * r + 1] = (float)(gim * A - gre * B);
        }
      }
      __syncthreads();
      const int64_t jw = jt + (int64_t)wid * 64 * R;
      const float* sw = &s_stage[wid][0];
      if (GAUSS) {
        float* y = static_cast<float*>(P.out) + row.w_off;
#pragma unroll
        for (int s = 0; s < R; ++s) {
          const int e = s * 64 + lane;
          const int64_t n = jw + e - row.jout0;
          if (n >= 0 && n < row.N) y[n] = sw[(e / R) * LSTR + (e % R)];
        }
      } else {
        float2* W = static_cast<float2*>(P.out) + row.w_off;
#pragma unroll
        for (int s = 0; s < R; ++s) {
          const int e = s * 64 + lane;
          const int64_t n = jw + e - row.jout0;
          const float* q = sw + (e / R) * LSTR + 2 * (e % R);
          if (n >= 0 && n < row.N) W[n] = make_float2(q[0], q[1]);
        }
      }
    }
    __syncthreads();
  }

  // last block of the launch re-arms the workspace for the next launch
  if (tid == 0) {
    const uint32_t d = atomicAdd(&hdr->done, 1u);
    if (d == gridDim.x - 1) {
      __hip_atomic_store(&hdr->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&hdr->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      st_u64(&hdr->epoch, epoch + 1);
    }
  }
}

}  // namespace

using KernelFn = void (*)(ScanLaunch);

// One instantiation set per K, defined in scan_fwd_k<K>.hip.
template <int K, int R>
KernelFn pick_fwd(int wide, int kind) {
  if (wide) return kind ? (KernelFn)scan_forward_kernel<K, R, true, true> : (KernelFn)scan_forward_kernel<K, R, true, false>;
  return kind ? (KernelFn)scan_forward_kernel<K, R, false, true> : (KernelFn)scan_forward_kernel<K, R, false, false>;
}

}  // namespace mk
