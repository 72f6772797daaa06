// Scan kernels (gfx950): the K-term SFT / ASFT kernel integral of one or many scan rows,
// in three variants that share the tile scan and the look-back.
//
// What is scanned (per row, per term p = P_S + t, a = e^{-alpha} e^{-i beta p}):
//   the windowed kernel integral of eq. kernelInt in its demodulated form,
//     v_p[j] = sum_{q=j-2L+1}^{j} a^{j-q} y[q]                   (2L window, eq. iir12K / aiir12K)
//   obtained as one prefix scan of the differenced input (eq. kernelIntZenka: the window
//   difference is taken on the input, before the scan)
//     v_p[j] = a v_p[j-1] + dy[j],   dy[j] = y[j] - a^{2L} y[j-2L],  a^{2L} = e^{-2 alpha L},
//   and the SFT / ASFT component (eqs. sfiir12K, asfiir12K with the prefactor e^{+alpha L})
//     c_p - i s_p = (-1)^p (e^{alpha L} v_p[j] + e^{-alpha L} y[j-2L]),   j = n - n0 + L.
//   Multiplying v_p by e^{i beta p j} gives the modulated kernel integral u_(2L)[j] of
//   eqs. kernel..kernelInter; carrying the demodulated state makes every constant a power
//   of a at a fixed distance, the same for every tile.
//
// Variants:
//   kFwd : y = x; output the K-term combination of Sec. III-A (Morlet, complex64) or
//          eq. GsSFT / GsASFT (Gaussian, float32).
//   kAdj : the transposed operator for a real loss. With W = h * x (taps h[k] on [-L, L],
//          output shift n0) and cotangent g = dLoss/dRe W + i dLoss/dIm W,
//            dLoss/dx[j] = Re sum_k conj(h[k]) g[j + n0 + k];
//          on the time-reversed cotangent g'[m] = g[N-1-m] this is the same scan with the
//          conjugate kernel (l -> -l) and the conjugate output factor, run on the two real
//          streams Re g' and Im g' (one stream for the Gaussian), real output written back
//          reversed. So the adjoint is again a causal, decaying scan.
//   kPg  : forward scan of x whose per-position components are reduced against g instead
//          of stored: per tile, sum_n Re u Re v_p, sum_n Im u Im v_p, sum_n Re u y[j-2L]
//          and sum_n u (A - iB) with u = conj(g) G; with MOM (ASFT) it also carries
//          w_p = d v_p / d alpha (w = a w - a v + 2L a^{2L} y[j-2L]) for the sigma gradient.
//
// How (one block = one tile of T = 256 R scan positions, persistent grid, ticketed tiles):
//   1. each thread loads R consecutive inputs at j and j-2L and forms dy (coalesced runs);
//   2. chunk sums B = sum_r a^{R-1-r} dy[r] (the thread's contribution to the state), in
//      float64 like everything else that propagates along the row;
//   3. inclusive scan of the chunk sums within each 16-lane row of the wavefront (4 DPP
//      levels, constants a^{R 2^d}, float64); the four row totals combine through LDS into
//      the wave aggregate and, once the wave's incoming state is known, into each row's
//      incoming state;
//   4. wave 0 forms the tile aggregate in float64, publishes it, and resolves the tile's
//      exclusive prefix by a deterministic decoupled look-back: the aggregates of the
//      earlier tiles of its 64-tile group plus the inclusive prefix of the previous
//      group's last tile, gathered one predecessor per lane and summed by a fixed butterfly
//      (agent-scope atomics that bypass the per-XCD L2, so tiles on different XCDs see each
//      other's states);
//   5. each thread rotates its carry in and runs the R-step recurrence; its R outputs go to
//      an LDS stage from which the wave writes its 64 R consecutive outputs with consecutive
//      lanes on consecutive 16-byte words (kFwd, kAdj), or they are reduced per tile into
//      float64 partials (kPg).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "launch.h"
#include "scan_common.h"

namespace mk {
namespace {

enum { kFwd = 0, kAdj = 1, kPg = 2, kSegSum = 3 };

// The matrix-core evaluation of the per-thread run (below) computes the same outputs as the
// vector-ALU recurrence with a third fewer vector instructions, but on the ragged scalogram it
// measured 1.70 ms per launch against 1.58 ms: the kernel is bound by the latency of its per-tile
// dependency chain, not by vector issue, and the run's operand loads lengthen that chain. Off
// until the chain is shortened.
constexpr bool kMatrixRun = false;

// four floats as a clang vector (what the nontemporal-store builtin takes); outputs are
// written once and never re-read by the kernel, so they bypass the cache hierarchy's reuse
typedef float v4f __attribute__((ext_vector_type(4)));

// row_shr:n DPP move within 16-lane rows (dpp_ctrl 0x110 + n); bound_ctrl: lanes whose source
// lies outside the row read zero
template <typename T>
__device__ __forceinline__ T dpp_row_shr(T v, int sh) {
  switch (sh) {
    case 1: return __builtin_amdgcn_update_dpp((T)0, v, 0x111, 0xF, 0xF, true);
    case 2: return __builtin_amdgcn_update_dpp((T)0, v, 0x112, 0xF, 0xF, true);
    case 4: return __builtin_amdgcn_update_dpp((T)0, v, 0x114, 0xF, 0xF, true);
    default: return __builtin_amdgcn_update_dpp((T)0, v, 0x118, 0xF, 0xF, true);
  }
}

// complex multiply-add helpers on (re, im) pairs
template <typename T>
__device__ __forceinline__ void cmac(T& zr, T& zi, T cr, T ci, T xr, T xi) {  // z += c x
  zr = fma(cr, xr, fma(-ci, xi, zr));
  zi = fma(cr, xi, fma(ci, xr, zi));
}

// KIND: 0 Morlet (complex64 out); 1 real output from the cosine components (Gaussian
// smoothing, its second differential); 2 real output from the sine components (the
// Gaussian's first differential, forward only); 3 real output from both components (the
// differentials by the attenuated transform, forward only)
// ACC: arithmetic of the scan (the library's morlet_accum values)
//   kAccF32   : float32 for the per-thread work (chunk sums, 16-lane wave scan, recurrence,
//               combination); float64 only for the carries between rows of a wave, waves and
//               tiles (forward and adjoint).
//   kAccF64   : float64 scan state, carries and combination.
//   kAccMixed : float64 chunk sums and wave scan, float32 recurrence and combination.
//   kAccKahan : the per-thread work of kAccF32 (chunk sums, wave scan, recurrence, combination)
//               compensated: float-float arithmetic (ff.h) from error-free float32 transforms;
//               float64 only for the carries, as in kAccF32 (forward only).
template <int VAR, int K, int R, int ACC, int KIND, bool MOM, int DT>
// Occupancy: the float32-state forward scans fit four waves per SIMD (at most 128 VGPRs). The
// gradient pass runs three up to K = 5: its LDS at R = 16 (41 KB per block) leaves no room for a
// fourth, and at K = 5 the few float64 registers it spills cost less than the third wave gains
// (about 40 us of a 450 us pass at 64 x 32768 x 16 scales); at K = 6 it would spill 65. The rest
// leave the register count to the compiler.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(
    (VAR == kFwd && (ACC == kAccF32 || (ACC == kAccMixed && R <= 16))) ? 4
    : (VAR == kPg && K <= 5)                                            ? 3
                                                                        : 1))) void scan_kernel(ScanLaunch P) {
  constexpr bool WIDE = ACC == kAccF64;
  constexpr bool F32T = ACC == kAccF32;                  // float32 tile scan
  constexpr bool KAHAN = ACC == kAccKahan;               // compensated float32 tile scan
  static_assert(!KAHAN || VAR == kFwd, "the compensated tile scan is built for the forward");
  static_assert(!F32T || VAR != kPg, "the float32 tile scan is not built for the gradient pass");
  // recurrence and combination; chunk sums and wave scan
  using acc_t = typename std::conditional<WIDE, double, typename std::conditional<KAHAN, ff, float>::type>::type;
  using sc_t = typename std::conditional<F32T, float, typename std::conditional<KAHAN, ff, double>::type>::type;
  constexpr int T = R * kThreads;
  constexpr bool GAUSS = KIND != 0;                      // real output
  constexpr bool SINE = KIND == 2;
  constexpr bool MIXED = KIND == 3;
  static_assert(!(SINE || MIXED) || VAR == kFwd, "sine-component output only in the forward scan");
  constexpr int NS = (VAR == kAdj && !GAUSS) ? 2 : 1;   // real input streams
  constexpr int KS = (NS == 2 || MOM) ? 2 * K : K;      // complex states per position
  constexpr int NRED = 4 * K + 3;                        // kPg partial sums per tile
  static_assert(!(MOM && VAR != kPg), "moment states only in the gradient pass");

  __shared__ uint32_t s_tile;
  __shared__ double s_wagg[2][kWaves][2 * KS];   // wave aggregates (two buffers: row-serial tiles alternate)
  __shared__ double s_c[2][2 * KS];              // row-serial: the block's state before its next tile
  __shared__ double s_rt[kWaves][4][2 * KS];     // per wave: totals of its four 16-lane rows, then
                                                 // the state at the start of rows 1..3
  __shared__ double s_xw[kWaves][2 * KS];
  __shared__ double s_e[kWaves][2 * KS];
  __shared__ double s_p[2 * KS];
  __shared__ double s_lb[2 * KS];                // look-back: a state vector on its way through Op
  // row-serial schedule: the row's constants of the block-level combination (a^{16 R k}, k < 4,
  // and a^{64 R w}, w <= kWaves, per term), copied from the table when a block takes a row, so the
  // chain of combination steps reads LDS instead of waiting on memory at each step. Up to K = 5
  // (the copy then fits beside the stash without costing a block per CU).
  constexpr bool KCACHE = !MOM && K <= 5;
  __shared__ double s_k[KCACHE ? 9 : 1][2 * K];
  __shared__ double s_red[(VAR == kPg) ? kWaves * NRED : 1];
  // Per-wave LDS slab, each thread's slots padded by 16 bytes. Forward and adjoint: the
  // thread's R input pairs (y[j], y[j-2L]; per stream for the adjoint's two) stashed by step 2
  // for step 5, which then overwrites them with the outputs (every pair is read before its
  // slot is written).
  constexpr bool kCplxOut = VAR == kFwd && !GAUSS;
  // R = 32: the adjoint's pairs would take 132 KB (one block per CU), the gradient pass's 66 KB
  constexpr bool kStash = VAR == kFwd || (VAR != kFwd && R <= 16);
  constexpr int kSub = R < 16 ? R : 16;                     // positions per thread per store round
  static_assert(R % kSub == 0, "R must be a multiple of the store sub-run");
  constexpr int kStride = (kStash ? 2 * NS * R : kSub * (kCplxOut ? 2 : 1)) + 4;   // floats per thread
  // Morlet forward, R = 16, float32 recurrence: each thread's run of 16 positions is evaluated as
  // one linear map on the matrix cores (v_mfma_f32_16x16x4_f32), outputs = Tc dy + Cc S + Y y
  // per component (the run matrices of the table's fourth section), instead of 16 steps of the
  // K-term recurrence and combination on the vector ALUs. The stash then holds the run's input
  // differences dy (16 floats) and the thread's state S before the run (2K floats, zero-padded
  // to a multiple of 4); y[j - 2L] is read again from the input (a cache hit).
  constexpr int NKB_C = (2 * K + 3) / 4;   // k-blocks of four state components
  constexpr bool MFMA = kMatrixRun && VAR == kFwd && KIND == 0 && R == 16 && (F32T || ACC == kAccMixed) && NS == 1 &&
                        16 + 4 * NKB_C <= kStride;
  __shared__ __align__(16) float s_out[kWaves][(VAR == kPg && !kStash) ? 4 : 64 * kStride];

  WsHeader* hdr = static_cast<WsHeader*>(P.ws);
  unsigned char* states = static_cast<unsigned char*>(P.ws) + sizeof(WsHeader);
  const size_t sbytes = tile_state_bytes(KS);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const uint64_t epoch = ld_u64(&hdr->epoch);
  const uint64_t tag = (epoch + 1) << 2;
  const TabLayout lay{K, R};

  auto load_row = [&](int32_t r, Row& row) {
    const cptr<Row> rp = (cptr<Row>)P.rows + __builtin_amdgcn_readfirstlane(r);
    row.x_off = rp->x_off; row.w_off = rp->w_off; row.N = rp->N; row.L = rp->L;
    row.jout0 = rp->jout0; row.jend = rp->jend; row.tile0 = rp->tile0;
    row.scale = rp->scale; row.ntiles = rp->ntiles;
  };

  // Two schedules. Tiles: a block claims its next tile only when it is ready to start it
  // (a tile claimed early would hold back the look-back of every later tile of its group)
  // and resolves the tile's incoming state by the look-back. Row-serial: a block claims a
  // whole row (longest rows first) and runs its tiles in order, carrying the state in LDS.
  Row row = P.row0;
  int64_t ti = 0, row_left = 0;
  // row-serial: the block starts on its own XCD's queue and moves on to the next queue only
  // when that one is empty (thread 0 keeps the count of queues it has left behind)
  int qdone = 0;
  for (;;) {
    uint32_t tile;
    if (P.serial) {
      if (row_left == 0) {
        // the next row (rows schedule: from the queues) or segment (segments schedule: one row,
        // through the ticket)
        if (tid == 0) {
          uint32_t r = (uint32_t)P.nrows;
          if (P.seg_mode != 0) {
            r = atomicAdd(&hdr->ticket, 1u);
          } else {
            for (; qdone < kQueues; ++qdone) {
              const int q = (int)((blockIdx.x + (unsigned)qdone) % kQueues);
              const uint32_t k = atomicAdd(&hdr->qticket[q], 1u);
              if ((int64_t)k < (int64_t)(P.qstart[q + 1] - P.qstart[q])) {
                r = (uint32_t)P.qstart[q] + k;
                break;
              }
            }
          }
          s_tile = r;
        }
        __syncthreads();
        const uint32_t r = __builtin_amdgcn_readfirstlane(s_tile);
        __syncthreads();   // every wave has read s_tile before thread 0 may claim again
        if (P.seg_mode != 0) {
          if ((int64_t)r >= P.nseg) break;
          int q = 0;   // the segment's row
          while (q + 1 < P.nrows && (int32_t)r >= P.seg_start[q + 1]) ++q;
          if (P.nrows != 1) load_row(q, row);
          ti = (int64_t)((int32_t)r - P.seg_start[q]) * P.seg_len;
          row_left = row.ntiles - ti < P.seg_len ? row.ntiles - ti : P.seg_len;
          // the state the segment starts from
          if (tid < 2 * KS) s_c[ti & 1][tid] = P.segstate[(int64_t)r * 2 * KS + tid];
        } else {
          if ((int64_t)r >= P.nrows) break;
          load_row(((cptr<int32_t>)P.row_order)[r], row);
          ti = 0;
          row_left = row.ntiles;
        }
        if constexpr (KCACHE) {
          const cptr<double> td = (cptr<double>)(P.tabs + (int64_t)row.scale * P.tab_stride + P.f32_bytes);
          if (tid < 9 * K) {
            const int slot = tid / K, t = tid % K;
            const int e = slot < 4 ? lay.eLANE(16 * slot) : lay.eWV(slot - 4);
            s_k[slot][2 * t] = td[(2 * e) * K + t];
            s_k[slot][2 * t + 1] = td[(2 * e + 1) * K + t];
          }
        }
        if (KCACHE || P.seg_mode != 0) __syncthreads();
        if (row_left == 0) continue;
      } else {
        ++ti;
      }
      --row_left;
      tile = (uint32_t)(row.tile0 + ti);
    } else {
      if (tid == 0) s_tile = atomicAdd(&hdr->ticket, 1u);
      __syncthreads();
      tile = __builtin_amdgcn_readfirstlane(s_tile);
      if ((int64_t)tile >= P.ntiles) break;
      if (P.nrows != 1) load_row(((cptr<int32_t>)P.tile_row)[tile], row);
      ti = (int64_t)tile - row.tile0;
    }
    const int par = P.serial ? (int)(ti & 1) : 0;
    const int64_t jt = ti * T;
    const int64_t j0 = jt + (int64_t)tid * R;
    // a wave whose positions all lie at or past jend (only in a row's last tile) feeds no output
    // and no later state: it skips its loads, chunk sums and outputs (its sums stay zero)
    const bool wave_dead = jt + (int64_t)__builtin_amdgcn_readfirstlane(wid) * 64 * R >= row.jend;
    const unsigned char* tb = P.tabs + (int64_t)row.scale * P.tab_stride;
    const TabT<acc_t> tab = tab_view<acc_t>(tb, P.f32_bytes, lay);
    const Tab<true> tabd{(cptr<double>)(tb + P.f32_bytes), K};
    const TabT<sc_t> tabs = tab_view<sc_t>(tb, P.f32_bytes, lay);   // chunk sums, wave scan
    const int mo = lay.nComplex();   // offset of the moment entries d a^d

    // 1. inputs, four positions at a time: y[j..j+3] and y[j-2L..j-2L+3] (zero outside the
    //    signal). Passes over the thread's R positions run as rolled loops over these quads,
    //    so register use does not grow with R.
    auto load_quad = [&](int64_t j, float (&ya)[NS][4], float (&yb)[NS][4]) {
      if constexpr (VAR == kAdj) {
        if constexpr (GAUSS) {
          const float* g = static_cast<const float*>(P.x) + row.w_off;
          load4_rev(g, j, row.N, ya[0]);
          load4_rev(g, j - 2 * row.L, row.N, yb[0]);
        } else {
          const float2* g = static_cast<const float2*>(P.x) + row.w_off;
          load4_rev_c(g, j, row.N, ya[0], ya[NS - 1]);
          load4_rev_c(g, j - 2 * row.L, row.N, yb[0], yb[NS - 1]);
        }
      } else {
        const void* xs = static_cast<const char*>(P.x) + row.x_off * (DT == 0 ? 4 : 2);
        load4(xs, DT, j, row.N, ya[0]);
        load4(xs, DT, j - 2 * row.L, row.N, yb[0]);
      }
    };
    // the same without bounds checks, for threads whose whole run (and trailing run) lies
    // inside the signal with 16-byte (f32) / 8-byte (16-bit) aligned quads
    auto load_quad_fast = [&](int64_t j, float (&ya)[NS][4], float (&yb)[NS][4]) {
      if constexpr (VAR == kAdj) {
        if constexpr (GAUSS) {
          const float* g = static_cast<const float*>(P.x) + row.w_off;
          ld4_rev_fast(g, row.N, j, ya[0]);
          ld4_rev_fast(g, row.N, j - 2 * row.L, yb[0]);
        } else {
          const float2* g = static_cast<const float2*>(P.x) + row.w_off;
          ld4c_rev_fast(g, row.N, j, ya[0], ya[NS - 1]);
          ld4c_rev_fast(g, row.N, j - 2 * row.L, yb[0], yb[NS - 1]);
        }
      } else {
        const void* xs = static_cast<const char*>(P.x) + row.x_off * (DT == 0 ? 4 : 2);
        ld4_fast<DT>(xs, j, ya[0]);
        ld4_fast<DT>(xs, j - 2 * row.L, yb[0]);
      }
    };
    // Positions past jend in a wave that also holds earlier positions are scanned like the
    // others: they produce no output and their state is never carried further, so their inputs
    // need no masking (in the gradient pass the cotangent is zero there).
    bool fast_in = (j0 - 2 * row.L >= 0) && (j0 + R <= row.N);
    {
      if constexpr (VAR == kAdj) {
        const char* g = static_cast<const char*>(P.x) + row.w_off * (GAUSS ? 4 : 8);
        const int64_t e = GAUSS ? 4 : 8;
        fast_in = fast_in && ((reinterpret_cast<uintptr_t>(g + (row.N - j0 - R) * e) & 15) == 0) &&
                  ((reinterpret_cast<uintptr_t>(g + (row.N - j0 + 2 * row.L - R) * e) & 15) == 0);
      } else {
        const char* xs = static_cast<const char*>(P.x) + row.x_off * (DT == 0 ? 4 : 2);
        const uintptr_t m = DT == 0 ? 15 : 7;
        const int64_t e = DT == 0 ? 4 : 2;
        fast_in = fast_in && ((reinterpret_cast<uintptr_t>(xs + j0 * e) & m) == 0) &&
                  ((reinterpret_cast<uintptr_t>(xs + (j0 - 2 * row.L) * e) & m) == 0);
      }
    }
    const acc_t Dw = tab.scalar(lay.sD());

    // 2. chunk sums: the recurrence run from a zero state over the thread's R positions,
    //    B = sum_r a^{R-1-r} dy[r], in Horner form, in sc_t: float32 in the float32 mode,
    //    float64 in the others. The sums over rows of a wave, waves and tiles (aggregates,
    //    carries) are float64 in every mode, so float32 rounding never accumulates along the
    //    row: each thread starts from a rounded float64 carry and runs R steps. On gfx950 a
    //    float64 FMA issues at the rate of an unpacked float32 FMA; the float32 mode saves the
    //    conversions and half the DPP moves of the wave scan.
    //    State i = s K + t: stream s, term t; with MOM, state K + t is the alpha-derivative of
    //    state t: w <- a (w - v) + ddy, ddy = d dy / d alpha = 2L a^{2L} y[j-2L].
    sc_t br[KS], bi[KS];
#pragma unroll
    for (int i = 0; i < KS; ++i) { br[i] = 0; bi[i] = 0; }
    {
      const sc_t Dd = tabs.scalar(lay.sD());
      auto step1 = [&](int q, const float (&ya)[NS][4], const float (&yb)[NS][4]) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const sc_t ddy = MOM ? (sc_t)(2 * row.L) * Dd * (sc_t)yb[0][r] : (sc_t)0;
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            const sc_t dyd = (sc_t)ya[s][r] - Dd * (sc_t)yb[s][r];
#pragma unroll
            for (int t = 0; t < K; ++t) {
              const int i = s * K + t;
              const sc_t ar = tabs.re(lay.eA(), t), ai = tabs.im(lay.eA(), t);
              const sc_t pr = br[i], pi = bi[i];
              br[i] = fma(ar, pr, fma(-ai, pi, dyd));
              bi[i] = fma(ar, pi, ai * pr);
              if (MOM && s == 0) {
                const sc_t wr = br[K + t] - pr, wi = bi[K + t] - pi;
                br[K + t] = fma(ar, wr, fma(-ai, wi, ddy));
                bi[K + t] = fma(ar, wi, ai * wr);
              }
            }
          }
        }
      };
      float* stash = &s_out[wid][0] + lane * kStride;
      auto keep = [&](int q, const float (&ya)[NS][4], const float (&yb)[NS][4]) {
        if constexpr (MFMA) {
          float d[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) d[r] = (float)((sc_t)ya[0][r] - Dd * (sc_t)yb[0][r]);
          *reinterpret_cast<float4*>(stash + 4 * q) = make_float4(d[0], d[1], d[2], d[3]);
        } else if constexpr (kStash && NS == 1) {
          *reinterpret_cast<float4*>(stash + 8 * q) = make_float4(ya[0][0], yb[0][0], ya[0][1], yb[0][1]);
          *reinterpret_cast<float4*>(stash + 8 * q + 4) = make_float4(ya[0][2], yb[0][2], ya[0][3], yb[0][3]);
        } else if constexpr (kStash) {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            *reinterpret_cast<float4*>(stash + 16 * q + 4 * r) = make_float4(ya[0][r], ya[1][r], yb[0][r], yb[1][r]);
        }
      };
      if (wave_dead) {
        // nothing to load or sum
      } else if (fast_in && NS == 1 && !MOM) {
        // every position of the run is in range: form all R differences first, then per term
        // a Horner pass four positions at a time, B <- a^4 B + (a^3 dy_0 + a^2 dy_1 + a dy_2 + dy_3)
        sc_t dyd[R];
#pragma unroll
        for (int q = 0; q < R / 4; ++q) {
          float ya[NS][4], yb[NS][4];
          load_quad_fast(j0 + 4 * q, ya, yb);
          if constexpr (!MFMA) keep(q, ya, yb);
#pragma unroll
          for (int r = 0; r < 4; ++r) dyd[4 * q + r] = (sc_t)ya[0][r] - Dd * (sc_t)yb[0][r];
          if constexpr (MFMA)
            *reinterpret_cast<float4*>(stash + 4 * q) = make_float4((float)dyd[4 * q], (float)dyd[4 * q + 1],
                                                                    (float)dyd[4 * q + 2], (float)dyd[4 * q + 3]);
        }
#pragma unroll
        for (int t = 0; t < K; ++t) {
          // the term's own contiguous block (one scalar load): a^1 .. a^4
          const int hc = lay.vHC(t);
          const sc_t a1r = tabs.scalar(hc), a1i = tabs.scalar(hc + 1);
          const sc_t a2r = tabs.scalar(hc + 2), a2i = tabs.scalar(hc + 3);
          const sc_t a3r = tabs.scalar(hc + 4), a3i = tabs.scalar(hc + 5);
          const sc_t a4r = tabs.scalar(hc + 6), a4i = tabs.scalar(hc + 7);
          sc_t Br = 0, Bi = 0;
#pragma unroll
          for (int q = 0; q < R / 4; ++q) {
            const sc_t d0 = dyd[4 * q], d1 = dyd[4 * q + 1], d2 = dyd[4 * q + 2], d3 = dyd[4 * q + 3];
            const sc_t cr = fma(a3r, d0, fma(a2r, d1, fma(a1r, d2, d3)));
            const sc_t ci = fma(a3i, d0, fma(a2i, d1, a1i * d2));
            if (q == 0) {
              Br = cr;
              Bi = ci;
            } else {
              const sc_t nr = fma(a4r, Br, fma(-a4i, Bi, cr));
              Bi = fma(a4r, Bi, fma(a4i, Br, ci));
              Br = nr;
            }
          }
          br[t] = Br;
          bi[t] = Bi;
          __builtin_amdgcn_sched_barrier(0);   // one term's constants live at a time (SGPR budget)
        }
      } else if (fast_in) {
#pragma unroll
        for (int q = 0; q < R / 4; ++q) {
          float ya[NS][4], yb[NS][4];
          load_quad_fast(j0 + 4 * q, ya, yb);
          keep(q, ya, yb);
          step1(q, ya, yb);
        }
      } else {
#pragma unroll 1
        for (int q = 0; q < R / 4; ++q) {
          float ya[NS][4], yb[NS][4];
          load_quad(j0 + 4 * q, ya, yb);
          keep(q, ya, yb);
          step1(q, ya, yb);
        }
      }
    }

    // state `lane` of Op(d) v for a vector v held in LDS (entry e holds a^d, mo + e holds d a^d);
    // whole state vectors pass through LDS so a moment state can read its base
    auto op_lds = [&](int e, const double* v, double& outr, double& outi) {
      const int t = lane % K;
      outr = 0; outi = 0;
      cmac(outr, outi, tabd.re(e, t), tabd.im(e, t), v[2 * lane], v[2 * lane + 1]);
      if (MOM && lane >= K) cmac(outr, outi, -tabd.re(mo + e, t), -tabd.im(mo + e, t), v[2 * t], v[2 * t + 1]);
    };
    // the same with the constant of slot `slot` of the row's LDS copy (row-serial schedule)
    auto op_c = [&](int slot, int e, const double* v, double& outr, double& outi) {
      if constexpr (KCACHE) {
        if (P.serial) {
          const int t = lane % K;
          outr = 0; outi = 0;
          cmac(outr, outi, s_k[slot][2 * t], s_k[slot][2 * t + 1], v[2 * lane], v[2 * lane + 1]);
          return;
        }
      }
      op_lds(e, v, outr, outi);
    };

    // 3. inclusive scan within each row of 16 lanes: S_l = sum_{m <= l, same row} Op(R (l - m)) B_m,
    //    where Op(d) multiplies a state by a^d (and, for a moment state, subtracts d a^d times
    //    its base). Row shifts are DPP moves, lanes shifted in from outside the row read zero.
    //    Then the row-exclusive prefix E_l (S shifted by one lane) stays in registers and the
    //    four row totals go to LDS.
    auto row_shr = [](sc_t v, int sh) -> sc_t {
      if constexpr (KAHAN) {
        return ff(dpp_row_shr(v.h, sh), dpp_row_shr(v.l, sh));
      } else {
        return dpp_row_shr(v, sh);
      }
    };
    // one state (with its moment partner) at a time, so only its shifted copies are live
#pragma unroll
    for (int d = 0; d < 4; ++d) {
#pragma unroll
      for (int i = 0; i < (MOM ? K : KS); ++i) {
        const int t = i % K;
        const sc_t ar = tabs.re(lay.eTR(d), t), ai = tabs.im(lay.eTR(d), t);
        const sc_t ur = row_shr(br[i], 1 << d), ui = row_shr(bi[i], 1 << d);
        if constexpr (MOM) {
          const sc_t wr = row_shr(br[K + i], 1 << d), wi = row_shr(bi[K + i], 1 << d);
          cmac(br[K + i], bi[K + i], ar, ai, wr, wi);
          cmac(br[K + i], bi[K + i], -tabd.re(mo + lay.eTR(d), t), -tabd.im(mo + lay.eTR(d), t), ur, ui);
        }
        cmac(br[i], bi[i], ar, ai, ur, ui);
      }
    }
    sc_t er[KS], ei[KS];
#pragma unroll
    for (int i = 0; i < KS; ++i) { er[i] = row_shr(br[i], 1); ei[i] = row_shr(bi[i], 1); }
    const int rw = lane >> 4;   // row of the lane within its wave
    if ((lane & 15) == 15) {
#pragma unroll
      for (int i = 0; i < KS; ++i) { s_rt[wid][rw][2 * i] = (double)br[i]; s_rt[wid][rw][2 * i + 1] = (double)bi[i]; }
    }
    wave_lds_sync();
    // wave aggregate: sum_r Op(16 R (3 - r)) T_r (lane i owns state i)
    if (lane < KS) {
      double Ar = 0, Ai = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double cr, ci;
        op_c(3 - r, lay.eLANE(16 * (3 - r)), &s_rt[wid][r][0], cr, ci);
        Ar += cr; Ai += ci;
      }
      s_wagg[par][wid][2 * lane] = Ar;
      s_wagg[par][wid][2 * lane + 1] = Ai;
    }
    __syncthreads();
    if (P.serial) {
      // 4'. row-serial: P = the block's running state (zero at the row's start). Every wave
      //     forms its own carry X_w = E_w + Op(64 R w) P, E_0 = 0, E_{w+1} = Op(64 R) E_w + agg_w
      //     (lane i owns state i, the E_w vector lives in the wave's own s_e slot); wave 0
      //     advances the running state to Op(T) P + A, A = sum_w Op(64 R (W-1-w)) agg_w.
      const double* cin = &s_c[ti & 1][0];
      if constexpr (!MOM) {
        // without moment states Op acts on each state alone, so lane i forms its state of
        // E_w = sum_{k < w} Op(64 R k) agg_{w-1-k} directly, the terms independent of each other
        if (lane < KS) {
          double er = 0, ei = 0;
          for (int k = 0; k < wid; ++k) {
            double cr, ci;
            op_c(4 + k, lay.eWV(k), &s_wagg[par][wid - 1 - k][0], cr, ci);
            er += cr;
            ei += ci;
          }
          double cr = 0, ci = 0;
          if (ti > 0) op_c(4 + wid, lay.eWV(wid), cin, cr, ci);
          s_xw[wid][2 * lane] = er + cr;
          s_xw[wid][2 * lane + 1] = ei + ci;
        }
      } else {
        if (lane < KS) { s_e[wid][2 * lane] = 0; s_e[wid][2 * lane + 1] = 0; }
        wave_lds_sync();
        for (int w = 0; w < wid; ++w) {
          double cr = 0, ci = 0;
          if (lane < KS) op_c(5, lay.eWV(1), &s_e[wid][0], cr, ci);
          wave_lds_sync();
          if (lane < KS) {
            s_e[wid][2 * lane] = cr + s_wagg[par][w][2 * lane];
            s_e[wid][2 * lane + 1] = ci + s_wagg[par][w][2 * lane + 1];
          }
          wave_lds_sync();
        }
        if (lane < KS) {
          double cr = 0, ci = 0;
          if (ti > 0) op_c(4 + wid, lay.eWV(wid), cin, cr, ci);
          s_xw[wid][2 * lane] = s_e[wid][2 * lane] + cr;
          s_xw[wid][2 * lane + 1] = s_e[wid][2 * lane + 1] + ci;
        }
      }
      if (wid == 0 && lane < KS) {
        double Ar = 0, Ai = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
          double cr, ci;
          op_c(4 + kWaves - 1 - w, lay.eWV(kWaves - 1 - w), &s_wagg[par][w][0], cr, ci);
          Ar += cr; Ai += ci;
        }
        double cr = 0, ci = 0;
        if (ti > 0) op_c(4 + kWaves, lay.eWV(kWaves), cin, cr, ci);
        s_c[(ti + 1) & 1][2 * lane] = cr + Ar;
        s_c[(ti + 1) & 1][2 * lane + 1] = ci + Ai;
      }
      wave_lds_sync();
    } else if (wid == 0) {
      // 4. tile aggregate, deterministic look-back and per-wave carries (wave 0; lane i owns
      //    state i)
      double Ar = 0, Ai = 0;
      if (lane < KS) {
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
          double cr, ci;
          op_lds(lay.eWV(kWaves - 1 - w), &s_wagg[0][w][0], cr, ci);
          Ar += cr; Ai += ci;
        }
      }
      const TileState st{states + (size_t)tile * sbytes, KS};
      // Three fixed levels within the row, so the float64 sums never depend on timing:
      // tiles in groups of 64, groups in super-groups of 64. The exclusive prefix of tile ti
      // (group g, position dd in it, position gd of g in its super-group) is
      //   P = S1 + Op(T dd) Z,  S1 = sum_{k<dd} Op(T k) A_{ti-1-k}   (its group's earlier tiles)
      //   Z = sum_{k<gd} Op(64 T k) GA_{g-1-k} + Op(64 T gd) I      (state at the end of group g-1)
      // with A the tile aggregates, GA the group aggregates (published by each group's last
      // tile as soon as its own group is known) and I the inclusive prefix published by the
      // last tile of the previous super-group: the only serial chain is one link per
      // 4096 tiles.
      const int64_t g = ti / kLookback;
      const int dd = (int)(ti - g * kLookback);
      const int64_t sg0 = (g / kLookback) * kLookback;   // first group of the super-group
      const int gd = (int)(g - sg0);
      const bool group_last = dd == kLookback - 1;
      const bool super_last = group_last && gd == kLookback - 1;
      if (lane < KS) { st_f64(st.agg(lane, 0), Ar); st_f64(st.agg(lane, 1), Ai); }
      release_order();
      if (lane == 0) st_u64(st.flag(), tag | kAggregate);
      auto status_of = [&](int64_t rel) {   // status of the tile rel places before this one
        const uint64_t f = ld_u64(TileState{states + (size_t)((int64_t)tile - rel) * sbytes, KS}.flag());
        return ((f & ~3ull) == tag) ? (int)(f & 3ull) : 0;
      };
      // lane k's weighted contribution to state i from the state vector v of one predecessor
      // (e: weight entry; the moment variant also reads the base state t of the same vector)
      auto contrib = [&](int i, int e, const TileState& sk, int which, double& cr, double& ci) {
        const int t = i % K;
        auto ptr = [&](int s, int c) { return which == 0 ? sk.agg(s, c) : which == 1 ? sk.gag(s, c) : sk.inc(s, c); };
        cmac(cr, ci, tabd.re(e, t), tabd.im(e, t), ld_f64(ptr(i, 0)), ld_f64(ptr(i, 1)));
        if (MOM && i >= K) cmac(cr, ci, -tabd.re(mo + e, t), -tabd.im(mo + e, t), ld_f64(ptr(t, 0)), ld_f64(ptr(t, 1)));
      };
      // phase 1: the earlier tiles of the group
      double S1r = 0, S1i = 0;
      if (dd > 0) {
        for (;;) {
          const bool ok = lane >= dd || status_of(1 + lane) >= 1;
          if (__ballot(!ok) == 0) break;
          __builtin_amdgcn_s_sleep(1);
        }
        acquire_order();
        // lanes past the last predecessor point at the nearest one (never read)
        const TileState sk{states + (size_t)((int64_t)tile - 1 - (lane < dd ? lane : 0)) * sbytes, KS};
#pragma unroll
        for (int i = 0; i < KS; ++i) {
          double cr = 0, ci = 0;
          if (lane < dd) contrib(i, lay.eLB(lane), sk, 0, cr, ci);
#pragma unroll
          for (int off = 32; off >= 1; off >>= 1) { cr += __shfl_xor(cr, off, 64); ci += __shfl_xor(ci, off, 64); }
          if (lane == i) { S1r = cr; S1i = ci; }
        }
      }
      if (group_last && !super_last) {
        // group aggregate GA = Op(T) S1 + A, independent of everything before the group
        if (lane < KS) { s_lb[2 * lane] = S1r; s_lb[2 * lane + 1] = S1i; }
        wave_lds_sync();
        if (lane < KS) {
          double cr, ci;
          op_lds(lay.eWV(kWaves), s_lb, cr, ci);
          st_f64(st.gag(lane, 0), cr + Ar);
          st_f64(st.gag(lane, 1), ci + Ai);
        }
        release_order();
        if (lane == 0) st_u64(st.flag(), tag | kGroup);
      }
      // phase 2: the state at the end of the previous group
      double Pr = S1r, Pi = S1i;
      if (g > 0) {
        const bool has_inc = sg0 > 0;
        for (;;) {
          bool ok = true;
          if (lane < gd) ok = status_of(ti - (kLookback * (g - 1 - lane) + kLookback - 1)) == (int)kGroup;
          else if (lane == gd && has_inc) ok = status_of(ti - (kLookback * sg0 - 1)) == (int)kInclusive;
          if (__ballot(!ok) == 0) break;
          __builtin_amdgcn_s_sleep(1);
        }
        acquire_order();
        const int64_t rel = lane < gd ? ti - (kLookback * (g - 1 - lane) + kLookback - 1)
                            : has_inc ? ti - (kLookback * sg0 - 1) : 1;   // 1: never read
        const TileState sk{states + (size_t)((int64_t)tile - rel) * sbytes, KS};
        double Zr = 0, Zi = 0;
#pragma unroll
        for (int i = 0; i < KS; ++i) {
          double cr = 0, ci = 0;
          if (lane < gd) contrib(i, lay.eLB2(lane), sk, 1, cr, ci);
          else if (lane == gd && has_inc) contrib(i, lay.eLB2(gd), sk, 2, cr, ci);
#pragma unroll
          for (int off = 32; off >= 1; off >>= 1) { cr += __shfl_xor(cr, off, 64); ci += __shfl_xor(ci, off, 64); }
          if (lane == i) { Zr = cr; Zi = ci; }
        }
        // P = S1 + Op(T dd) Z
        if (lane < KS) { s_lb[2 * lane] = Zr; s_lb[2 * lane + 1] = Zi; }
        wave_lds_sync();
        if (lane < KS) {
          double cr, ci;
          op_lds(lay.eLB(dd), s_lb, cr, ci);
          Pr += cr;
          Pi += ci;
        }
      }
      if (lane < KS) { s_p[2 * lane] = Pr; s_p[2 * lane + 1] = Pi; }
      wave_lds_sync();
      if (super_last) {
        if (lane < KS) {   // inclusive = Op(T) P + A
          double cr, ci;
          op_lds(lay.eWV(kWaves), s_p, cr, ci);
          st_f64(st.inc(lane, 0), cr + Ar);
          st_f64(st.inc(lane, 1), ci + Ai);
        }
        release_order();
        if (lane == 0) st_u64(st.flag(), tag | kInclusive);
      }
      // per-wave carries: X_w = E_w + Op(64 R w) P, E_0 = 0, E_{w+1} = Op(64 R) E_w + agg_w
      if (lane < KS) { s_e[0][2 * lane] = 0; s_e[0][2 * lane + 1] = 0; }
      wave_lds_sync();
#pragma unroll
      for (int w = 0; w < kWaves; ++w) {
        if (lane < KS) {
          double cr, ci;
          op_lds(lay.eWV(w), s_p, cr, ci);
          s_xw[w][2 * lane] = s_e[w][2 * lane] + cr;
          s_xw[w][2 * lane + 1] = s_e[w][2 * lane + 1] + ci;
          if (w + 1 < kWaves) {
            op_lds(lay.eWV(1), &s_e[w][0], cr, ci);
            s_e[w + 1][2 * lane] = cr + s_wagg[0][w][2 * lane];
            s_e[w + 1][2 * lane + 1] = ci + s_wagg[0][w][2 * lane + 1];
          }
        }
        wave_lds_sync();
      }
    }
    if (!P.serial) __syncthreads();

    // 5. thread carry (state just before the thread's first position): E_l + Op(R (l mod 16)) Z_r
    //    with Z_r the state at the start of row r: Z_0 = X_w, Z_{r+1} = Op(16 R) Z_r + T_r.
    //    Row-serial tiles: s_rt and s_xw belong to the wave, which reaches its next step 3
    //    only after this one.
    const bool has_out = (jt + T > row.jout0) && (row.jout0 + row.N > jt);
    if (has_out) {
      // the thread's carry constants a^{R (l mod 16)}, requested before the chain of row states
      // (where the registers allow: up to K = 5)
      [[maybe_unused]] double kcr[K], kci[K];
      if constexpr (KCACHE) {
        const int e = lay.eLANE(lane & 15);
#pragma unroll
        for (int t = 0; t < K; ++t) { kcr[t] = tabd.re(e, t); kci[t] = tabd.im(e, t); }
      }
      // Z_{r+1} overwrites T_r in place (each lane rewrites only its own state of it)
      if constexpr (!MOM && KCACHE) {
        // each state on its own: lane i carries its Z in registers, one LDS round at the end
        if (P.serial && lane < KS) {
          const double ar = s_k[1][2 * (lane % K)], ai = s_k[1][2 * (lane % K) + 1];
          double zr = s_xw[wid][2 * lane], zi = s_xw[wid][2 * lane + 1];
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            double cr = 0, ci = 0;
            cmac(cr, ci, ar, ai, zr, zi);
            zr = s_rt[wid][r][2 * lane] + cr;
            zi = s_rt[wid][r][2 * lane + 1] + ci;
            s_rt[wid][r][2 * lane] = zr;
            s_rt[wid][r][2 * lane + 1] = zi;
          }
        }
      }
      if (!(!MOM && KCACHE) || !P.serial) {
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          if (lane < KS) {
            double cr, ci;
            op_c(1, lay.eLANE(16), r == 0 ? &s_xw[wid][0] : &s_rt[wid][r - 1][0], cr, ci);
            s_rt[wid][r][2 * lane] += cr;
            s_rt[wid][r][2 * lane + 1] += ci;
          }
          wave_lds_sync();
        }
      } else {
        wave_lds_sync();
      }
      const double* z = rw == 0 ? &s_xw[wid][0] : &s_rt[wid][rw - 1][0];
      const int e = lay.eLANE(lane & 15);
      acc_t vr[KS], vi[KS];
#pragma unroll
      for (int i = 0; i < KS; ++i) {
        const int t = i % K;
        double cr = (double)er[i], ci = (double)ei[i];
        if constexpr (KCACHE) cmac(cr, ci, kcr[t], kci[t], z[2 * i], z[2 * i + 1]);
        else cmac(cr, ci, tabd.re(e, t), tabd.im(e, t), z[2 * i], z[2 * i + 1]);
        if (MOM && i >= K) cmac(cr, ci, -tabd.re(mo + e, t), -tabd.im(mo + e, t), z[2 * t], z[2 * t + 1]);
        vr[i] = (acc_t)cr;
        vi[i] = (acc_t)ci;
      }
      const acc_t cx = tab.scalar(lay.sCX());
      const acc_t gre = tab.scalar(lay.sGre()), gim = tab.scalar(lay.sGim());
      const int64_t nb = j0 - row.jout0;   // output index of the thread's first position
      // store sub-run u: element e (0 <= e < 64 kSub) is lane e / kSub's position
      // kSub u + e % kSub, output nw + (e / kSub) R + kSub u + e % kSub. Lane l handles
      // e = G l + 64 G i (G = 2 complex or 4 real per 16-byte word; G = 1 when not whole or
      // unaligned), so one base address per lane plus a fixed stride per i.
      auto flush = [&](int u) {
        wave_lds_sync();
        constexpr int C = kCplxOut ? 2 : 1;                 // floats per output
        const int64_t nw = jt + (int64_t)wid * 64 * R - row.jout0;   // output of the wave's first position
        const bool whole = nw >= 0 && nw + 64 * R <= row.N;
        const float* sw = &s_out[wid][0] + (kStash ? kSub * u : 0) * C;
        const int64_t n0u = nw + kSub * u;                  // output of lane 0's first element
        if constexpr (VAR == kFwd && !GAUSS) {
          float2* W = static_cast<float2*>(P.out) + row.w_off;
          if (whole && (reinterpret_cast<uintptr_t>(W + nw) & 15) == 0) {
            constexpr int LPR = kSub / 2;                   // lanes per sub-run
            const float* sp = sw + (lane / LPR) * kStride + 2 * (lane % LPR) * C;
            float2* wp = W + n0u + (int64_t)(lane / LPR) * R + 2 * (lane % LPR);
#pragma unroll
            for (int i = 0; i < kSub / 2; ++i)
              __builtin_nontemporal_store(*reinterpret_cast<const v4f*>(sp + i * (64 / LPR) * kStride),
                                          reinterpret_cast<v4f*>(wp + (int64_t)i * (64 / LPR) * R));
          } else {
            const float* sp = sw + (lane / kSub) * kStride + (lane % kSub) * C;
            const int64_t nl = n0u + (int64_t)(lane / kSub) * R + (lane % kSub);
#pragma unroll 1
            for (int i = 0; i < kSub; ++i) {
              const int64_t n = nl + (int64_t)i * (64 / kSub) * R;
              if (n >= 0 && n < row.N) W[n] = *reinterpret_cast<const float2*>(sp + i * (64 / kSub) * kStride);
            }
          }
        } else {
          float* Y = static_cast<float*>(P.out) + row.w_off;
          // forward (Gaussian): Y[n]; adjoint: written time-reversed, Y[N - 1 - n]
          constexpr bool rev = VAR == kAdj;
          if (whole && (reinterpret_cast<uintptr_t>(rev ? Y + (row.N - 4 - nw) : Y + nw) & 15) == 0) {
            constexpr int LPR = kSub / 4;
            const float* sp = sw + (lane / LPR) * kStride + 4 * (lane % LPR);
            const int64_t nl = n0u + (int64_t)(lane / LPR) * R + 4 * (lane % LPR);
            float* yp = rev ? Y + (row.N - 4 - nl) : Y + nl;
#pragma unroll
            for (int i = 0; i < kSub / 4; ++i) {
              const v4f v = *reinterpret_cast<const v4f*>(sp + i * (64 / LPR) * kStride);
              if constexpr (rev) __builtin_nontemporal_store(v.wzyx, reinterpret_cast<v4f*>(yp - (int64_t)i * (64 / LPR) * R));
              else __builtin_nontemporal_store(v, reinterpret_cast<v4f*>(yp + (int64_t)i * (64 / LPR) * R));
            }
          } else {
            const float* sp = sw + (lane / kSub) * kStride + (lane % kSub);
            const int64_t nl = n0u + (int64_t)(lane / kSub) * R + (lane % kSub);
#pragma unroll 1
            for (int i = 0; i < kSub; ++i) {
              const int64_t n = nl + (int64_t)i * (64 / kSub) * R;
              if (n >= 0 && n < row.N) Y[rev ? row.N - 1 - n : n] = sp[i * (64 / kSub) * kStride];
            }
          }
        }
        // the next sub-run's stage writes stay behind this one's reads
        __builtin_amdgcn_wave_barrier();
      };

      if constexpr (VAR == kPg) {
        // reductions against the cotangent at the output positions n = j - jout0:
        // S1_t = sum Re u Re v_t, S2_t = sum Im u Im v_t (S3, S4 the same for the alpha
        // derivative states), Sx = sum Re u y[j-2L], Q = sum u (A - iB), u = conj(g) G
        acc_t sv_re[K], sv_im[K], sw_re[K], sw_im[K], s_xb = 0, q_re = 0, q_im = 0;
#pragma unroll
        for (int t = 0; t < K; ++t) { sv_re[t] = 0; sv_im[t] = 0; sw_re[t] = 0; sw_im[t] = 0; }
#pragma unroll 1
        for (int q = 0; q < (wave_dead ? 0 : R / 4); ++q) {
          float ya[NS][4], yb[NS][4], gr[4], gi[4];
          if constexpr (kStash) {
            const float* stg = &s_out[wid][0] + lane * kStride;
            const float4 v0 = *reinterpret_cast<const float4*>(stg + 8 * q);
            const float4 v1 = *reinterpret_cast<const float4*>(stg + 8 * q + 4);
            ya[0][0] = v0.x; yb[0][0] = v0.y; ya[0][1] = v0.z; yb[0][1] = v0.w;
            ya[0][2] = v1.x; yb[0][2] = v1.y; ya[0][3] = v1.z; yb[0][3] = v1.w;
          } else {
            load_quad(j0 + 4 * q, ya, yb);
          }
          if constexpr (GAUSS) {
            load4_f32(static_cast<const float*>(P.g) + row.w_off, nb + 4 * q, row.N, gr);
#pragma unroll
            for (int r = 0; r < 4; ++r) gi[r] = 0.f;
          } else {
            load4_c(static_cast<const float2*>(P.g) + row.w_off, nb + 4 * q, row.N, gr, gi);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const acc_t dyr = (acc_t)ya[0][r] - Dw * (acc_t)yb[0][r];
            const acc_t ybr = (acc_t)yb[0][r];
            const acc_t ur = (acc_t)gr[r] * gre + (acc_t)gi[r] * gim;
            const acc_t ui = (acc_t)gr[r] * gim - (acc_t)gi[r] * gre;
            const acc_t ddy = MOM ? (acc_t)(2 * row.L) * Dw * ybr : (acc_t)0;
            acc_t A = cx * ybr, B = 0;
#pragma unroll
            for (int t = 0; t < K; ++t) {
              const acc_t ar = tab.re(lay.eA(), t), ai = tab.im(lay.eA(), t);
              const acc_t pr = vr[t], pi = vi[t];
              const acc_t nr = fma(ar, pr, fma(-ai, pi, dyr));
              const acc_t ni = fma(ar, pi, ai * pr);
              vr[t] = nr;
              vi[t] = ni;
              if constexpr (MOM) {   // w = a (w - v_prev) + ddy
                const acc_t wr = vr[K + t] - pr, wi = vi[K + t] - pi;
                vr[K + t] = fma(ar, wr, fma(-ai, wi, ddy));
                vi[K + t] = fma(ar, wi, ai * wr);
                sw_re[t] = fma(ur, vr[K + t], sw_re[t]);
                sw_im[t] = fma(ui, vi[K + t], sw_im[t]);
              }
              sv_re[t] = fma(ur, nr, sv_re[t]);
              sv_im[t] = fma(ui, ni, sv_im[t]);
              A = fma(tab.row(lay.rMW(), t), nr, A);
              if (!GAUSS) B = fma(tab.row(lay.rLW(), t), ni, B);
            }
            s_xb = fma(ur, ybr, s_xb);
            q_re = fma(ur, A, fma(ui, B, q_re));
            q_im = fma(ui, A, fma(-ur, B, q_im));
          }
        }
        // block reduction of the 4K + 3 partial sums in float64, fixed order
        double red[NRED];
#pragma unroll
        for (int t = 0; t < K; ++t) {
          red[t] = (double)sv_re[t]; red[K + t] = (double)sv_im[t];
          red[2 * K + t] = (double)sw_re[t]; red[3 * K + t] = (double)sw_im[t];
        }
        red[4 * K] = (double)s_xb; red[4 * K + 1] = (double)q_re; red[4 * K + 2] = (double)q_im;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
          for (int q = 0; q < NRED; ++q) red[q] += __shfl_xor(red[q], off, 64);
        if (lane == 0)
#pragma unroll
          for (int q = 0; q < NRED; ++q) s_red[wid * NRED + q] = red[q];
        __syncthreads();
        if (tid < NRED) {
          double sacc = 0;
#pragma unroll
          for (int w = 0; w < kWaves; ++w) sacc += s_red[w * NRED + tid];
          P.partials[(size_t)tile * NRED + tid] = sacc;
        }
      } else if constexpr (MFMA) {
        // The run of thread c (positions j0(c) + r, r < 16) as a 16 x 16 x 4 product per group of
        // 16 threads: D[r][c'] = sum_k A[r][k] B[k][c'] with c = 16 g + c'. Lane l supplies
        // A[l % 16][l / 16] and B[l / 16][l % 16] of each k-block and receives D[4 (l / 16) + v][l % 16],
        // v < 4. The k-blocks' K index is permuted so that lane l supplies, for the Toeplitz part,
        // the input differences dy[4 (l / 16) + kb] of its chunk (kb = 0..3: one 16-byte LDS read)
        // and, for the state part, components NKB_C (l / 16) + kb; its results are the outputs
        // r = 4 (l / 16) + v of chunk c, i.e. four consecutive positions.
        if (!wave_dead) {
          float* slot = &s_out[wid][0] + lane * kStride;
          {
            float st[4 * NKB_C];
#pragma unroll
            for (int k = 0; k < 4 * NKB_C; ++k) st[k] = k < 2 * K ? (float)((k & 1) ? vi[k >> 1] : vr[k >> 1]) : 0.0f;
#pragma unroll
            for (int k = 0; k < NKB_C; ++k)
              *reinterpret_cast<float4*>(slot + 16 + 4 * k) = make_float4(st[4 * k], st[4 * k + 1], st[4 * k + 2], st[4 * k + 3]);
          }
          // the lane's operands from memory: its run-matrix entries and y[j - 2L] of the four
          // chunks it computes (one request each, all in flight together)
          const int i16 = lane & 15, q = lane >> 4;
          const float* tm = reinterpret_cast<const float*>(tb + lay.mfmaOff());
          const float4 m_tre = *reinterpret_cast<const float4*>(tm + lay.mTre() + 16 * i16 + 4 * q);
          const float4 m_tim = *reinterpret_cast<const float4*>(tm + lay.mTim() + 16 * i16 + 4 * q);
          float m_cre[NKB_C], m_cim[NKB_C], m_y[4][4];
#pragma unroll
          for (int kb = 0; kb < NKB_C; ++kb) {
            m_cre[kb] = tm[lay.mCre() + lay.mCW() * i16 + NKB_C * q + kb];
            m_cim[kb] = tm[lay.mCim() + lay.mCW() * i16 + NKB_C * q + kb];
          }
          {
            const void* xs = static_cast<const char*>(P.x) + row.x_off * (DT == 0 ? 4 : 2);
#pragma unroll
            for (int g = 0; g < 4; ++g)
              load4(xs, DT, jt + (int64_t)(wid * 64 + 16 * g + i16) * R + 4 * q - 2 * row.L, row.N, m_y[g]);
          }
          wave_lds_sync();
          const float yre = (float)(gre * cx), yim = (float)(gim * cx);
          // two groups at a time: four independent accumulation chains keep the matrix core busy
#pragma unroll
          for (int gp = 0; gp < 4; gp += 2) {
            float* sl[2];
            float4 d4[2];
            float sc[2][NKB_C];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              sl[h] = &s_out[wid][0] + (16 * (gp + h) + i16) * kStride;
              d4[h] = *reinterpret_cast<const float4*>(sl[h] + 4 * q);
#pragma unroll
              for (int kb = 0; kb < NKB_C; ++kb) sc[h][kb] = sl[h][16 + NKB_C * q + kb];
            }
            v4f dre[2], dim[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              dre[h] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
              dim[h] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
            }
            const float tr[4] = {m_tre.x, m_tre.y, m_tre.z, m_tre.w}, ti[4] = {m_tim.x, m_tim.y, m_tim.z, m_tim.w};
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
              const float dv[2] = {kb == 0 ? d4[0].x : kb == 1 ? d4[0].y : kb == 2 ? d4[0].z : d4[0].w,
                                   kb == 0 ? d4[1].x : kb == 1 ? d4[1].y : kb == 2 ? d4[1].z : d4[1].w};
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                dre[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(tr[kb], dv[h], dre[h], 0, 0, 0);
                dim[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(ti[kb], dv[h], dim[h], 0, 0, 0);
              }
            }
#pragma unroll
            for (int kb = 0; kb < NKB_C; ++kb) {
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                dre[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(m_cre[kb], sc[h][kb], dre[h], 0, 0, 0);
                dim[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(m_cim[kb], sc[h][kb], dim[h], 0, 0, 0);
              }
            }
            // outputs r = 4 q + v of each chunk go to floats 2 r, 2 r + 1 of its slot (read above by
            // this group only, before these writes)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const float* y = m_y[gp + h];
              *reinterpret_cast<float4*>(sl[h] + 8 * q) =
                  make_float4(fmaf(yre, y[0], dre[h][0]), fmaf(yim, y[0], dim[h][0]), fmaf(yre, y[1], dre[h][1]),
                              fmaf(yim, y[1], dim[h][1]));
              *reinterpret_cast<float4*>(sl[h] + 8 * q + 4) =
                  make_float4(fmaf(yre, y[2], dre[h][2]), fmaf(yim, y[2], dim[h][2]), fmaf(yre, y[3], dre[h][3]),
                              fmaf(yim, y[3], dim[h][3]));
            }
          }
          flush(0);
        }
      } else {
        // outputs n = j - jout0, in sub-runs of kSub positions per thread: each thread writes
        // a sub-run to the wave's LDS stage, then the wave stores the 64 sub-runs with
        // consecutive lanes on consecutive 16-byte words (every line written whole by one
        // instruction), instead of each lane writing its own run R positions from its
        // neighbour's
        float* stg = &s_out[wid][0] + lane * kStride;
        auto step2 = [&](int q, const float (&ya)[NS][4], const float (&yb)[NS][4]) {
          float o0[4], o1[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            acc_t A[NS], B[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
              const acc_t dyr = (acc_t)ya[s][r] - Dw * (acc_t)yb[s][r];
              A[s] = SINE ? (acc_t)0 : cx * (acc_t)yb[s][r];
              B[s] = 0;
#pragma unroll
              for (int t = 0; t < K; ++t) {
                const int i = s * K + t;
                const acc_t ar = tab.re(lay.eA(), t), ai = tab.im(lay.eA(), t);
                const acc_t nr = fma(ar, vr[i], fma(-ai, vi[i], dyr));
                const acc_t ni = fma(ar, vi[i], ai * vr[i]);
                vr[i] = nr;
                vi[i] = ni;
                if (!SINE) A[s] = fma(tab.row(lay.rMW(), t), nr, A[s]);
                if (!GAUSS || SINE || MIXED) B[s] = fma(tab.row(lay.rLW(), t), ni, B[s]);
              }
            }
            if constexpr (VAR == kFwd && !GAUSS) {
              o0[r] = (float)(gre * A[0] + gim * B[0]);
              o1[r] = (float)(gim * A[0] - gre * B[0]);
            } else if constexpr (SINE) {
              // sum_p b_p s_p with s_p = -(-1)^p e^{alpha L} Im v_p (the y[j-2L] term is real)
              o0[r] = (float)(-gre * B[0]);
            } else if constexpr (MIXED) {
              // sum_p cc_p c_p + sc_p s_p
              o0[r] = (float)(gre * (A[0] - B[0]));
            } else if constexpr (VAR == kFwd || GAUSS) {
              o0[r] = (float)(gre * A[0]);
            } else {
              // Re[conj(G) W_c(Re g')] - Im[conj(G) W_c(Im g')], W_c(y) = A(y) + i B(y)
              o0[r] = (float)(gre * (A[0] - B[NS - 1]) + gim * (B[0] + A[NS - 1]));
            }
          }
          // slot of the quad's outputs: sub-run relative (stage) or the whole run (stash)
          const int qs = kStash ? q : q % (kSub / 4);
          if constexpr (kCplxOut) {
            *reinterpret_cast<float4*>(stg + 8 * qs) = make_float4(o0[0], o1[0], o0[1], o1[1]);
            *reinterpret_cast<float4*>(stg + 8 * qs + 4) = make_float4(o0[2], o1[2], o0[3], o1[3]);
          } else {
            // a real output of position p goes to float p, inside the stash of position
            // p / (2 NS), which an earlier quad (or this one, before writing) has read
            *reinterpret_cast<float4*>(stg + 4 * qs) = make_float4(o0[0], o0[1], o0[2], o0[3]);
          }
        };
        // fast_in differs between the lanes of a wave, so each sub-run's quads run on either
        // path and the wave reconverges before the cooperative store
#pragma unroll
        for (int u = 0; u < R / kSub; ++u) {
          if (wave_dead) break;
          if constexpr (kStash) {
#pragma unroll
            for (int q = u * (kSub / 4); q < (u + 1) * (kSub / 4); ++q) {
              float ya[NS][4], yb[NS][4];
              if constexpr (NS == 1) {
                const float4 v0 = *reinterpret_cast<const float4*>(stg + 8 * q);
                const float4 v1 = *reinterpret_cast<const float4*>(stg + 8 * q + 4);
                ya[0][0] = v0.x; yb[0][0] = v0.y; ya[0][1] = v0.z; yb[0][1] = v0.w;
                ya[0][2] = v1.x; yb[0][2] = v1.y; ya[0][3] = v1.z; yb[0][3] = v1.w;
              } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                  const float4 v = *reinterpret_cast<const float4*>(stg + 16 * q + 4 * r);
                  ya[0][r] = v.x; ya[NS - 1][r] = v.y; yb[0][r] = v.z; yb[NS - 1][r] = v.w;
                }
              }
              step2(q, ya, yb);
              __builtin_amdgcn_sched_barrier(0);   // keep each quad's LDS reads with its compute
            }
          } else if (fast_in) {
#pragma unroll
            for (int q = u * (kSub / 4); q < (u + 1) * (kSub / 4); ++q) {
              float ya[NS][4], yb[NS][4];
              load_quad_fast(j0 + 4 * q, ya, yb);
              step2(q, ya, yb);
            }
          } else {
#pragma unroll 1
            for (int q = u * (kSub / 4); q < (u + 1) * (kSub / 4); ++q) {
              float ya[NS][4], yb[NS][4];
              load_quad(j0 + 4 * q, ya, yb);
              step2(q, ya, yb);
            }
          }
          flush(u);
        }
      }
    } else if constexpr (VAR == kPg) {
      if (tid < NRED) P.partials[(size_t)tile * NRED + tid] = 0.0;
    }
    // Tiles: the next claim reuses s_tile and the LDS vectors. Row-serial: the alternating
    // buffers and the barrier after the next tile's wave aggregates keep the waves at most
    // one tile apart, which is all the sharing needs.
    if (!P.serial) __syncthreads();
  }

  // last block of the launch re-arms the workspace for the next launch
  if (tid == 0) {
    const uint32_t d = atomicAdd(&hdr->done, 1u);
    if (d == gridDim.x - 1) {
      __hip_atomic_store(&hdr->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      for (int q = 0; q < kQueues; ++q) __hip_atomic_store(&hdr->qticket[q], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&hdr->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      st_u64(&hdr->epoch, epoch + 1);
    }
  }
}

// Segments schedule, first pass: the state at the end of every segment from a zero state at its
// start,
//   A_s = sum_{j in segment s} a^{e_s - 1 - j} dy[j]   (e_s: the segment's end position),
// the same quantity the rows schedule carries from tile to tile, here without the scan inside the
// tiles: thread c of the block forms its chunk sum B_{t,c} over positions [jt + R c, jt + R c + R)
// of every tile t of the segment (in float64, by the same Horner steps as the scan), folds them
// over the tiles, Acc <- a^T Acc + B, weights the fold by a^{R (255 - c)} (its distance to a tile's
// end), and the block adds the 256 weighted states in a fixed order. One block per segment; no
// block waits on another.
template <int K, int R, int DT>
__global__ __launch_bounds__(kThreads) void seg_sum_kernel(ScanLaunch P) {
  constexpr int T = R * kThreads;
  __shared__ double s_sum[kWaves][2 * K];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int64_t s = blockIdx.x;
  int rr = 0;   // the segment's row
  while (rr + 1 < P.nrows && s >= P.seg_start[rr + 1]) ++rr;
  Row row = P.row0;
  if (P.nrows != 1) {
    const cptr<Row> rp = (cptr<Row>)P.rows + rr;
    row.x_off = rp->x_off; row.w_off = rp->w_off; row.N = rp->N; row.L = rp->L;
    row.jout0 = rp->jout0; row.jend = rp->jend; row.tile0 = rp->tile0;
    row.scale = rp->scale; row.ntiles = rp->ntiles;
  }
  const TabLayout lay{K, R};
  const unsigned char* tb = P.tabs + (int64_t)row.scale * P.tab_stride;
  const TabT<double> tab{(cptr<double>)(tb + P.f32_bytes), K};
  const double D = tab.scalar(lay.sD());
  const void* xs = static_cast<const char*>(P.x) + row.x_off * (DT == 0 ? 4 : 2);
  const int64_t t0 = (s - P.seg_start[rr]) * P.seg_len;
  const int64_t t1 = t0 + P.seg_len < row.ntiles ? t0 + P.seg_len : row.ntiles;
  double ar[K], ai[K];
#pragma unroll
  for (int t = 0; t < K; ++t) { ar[t] = 0; ai[t] = 0; }
  for (int64_t ti = t0; ti < t1; ++ti) {
    const int64_t j0 = ti * T + (int64_t)tid * R;
    double dy[R];
    const bool fast = (j0 - 2 * row.L >= 0) && (j0 + R <= row.N) &&
                      ((reinterpret_cast<uintptr_t>(static_cast<const char*>(xs) + (j0 - 2 * row.L) * (DT == 0 ? 4 : 2)) |
                        reinterpret_cast<uintptr_t>(static_cast<const char*>(xs) + j0 * (DT == 0 ? 4 : 2))) &
                       (DT == 0 ? 15 : 7)) == 0;
#pragma unroll
    for (int q = 0; q < R / 4; ++q) {
      float ya[4], yb[4];
      if (fast) {
        ld4_fast<DT>(xs, j0 + 4 * q, ya);
        ld4_fast<DT>(xs, j0 + 4 * q - 2 * row.L, yb);
      } else {
        load4(xs, DT, j0 + 4 * q, row.N, ya);
        load4(xs, DT, j0 + 4 * q - 2 * row.L, row.N, yb);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) dy[4 * q + r] = fma(-D, (double)yb[r], (double)ya[r]);
    }
#pragma unroll
    for (int t = 0; t < K; ++t) {
      // B = sum_r a^{R-1-r} dy[r], four positions per Horner step (a^1 .. a^4 of the term's block)
      const int hc = lay.vHC(t);
      const double a1r = tab.scalar(hc), a1i = tab.scalar(hc + 1), a2r = tab.scalar(hc + 2), a2i = tab.scalar(hc + 3);
      const double a3r = tab.scalar(hc + 4), a3i = tab.scalar(hc + 5), a4r = tab.scalar(hc + 6), a4i = tab.scalar(hc + 7);
      double Br = 0, Bi = 0;
#pragma unroll
      for (int q = 0; q < R / 4; ++q) {
        const double d0 = dy[4 * q], d1 = dy[4 * q + 1], d2 = dy[4 * q + 2], d3 = dy[4 * q + 3];
        const double cr = fma(a3r, d0, fma(a2r, d1, fma(a1r, d2, d3)));
        const double ci = fma(a3i, d0, fma(a2i, d1, a1i * d2));
        if (q == 0) {
          Br = cr;
          Bi = ci;
        } else {
          const double nr = fma(a4r, Br, fma(-a4i, Bi, cr));
          Bi = fma(a4r, Bi, fma(a4i, Br, ci));
          Br = nr;
        }
      }
      // Acc <- a^T Acc + B
      const double cr = tab.re(lay.eWV(kWaves), t), ci = tab.im(lay.eWV(kWaves), t);
      const double nr = fma(cr, ar[t], fma(-ci, ai[t], Br));
      ai[t] = fma(cr, ai[t], fma(ci, ar[t], Bi));
      ar[t] = nr;
    }
  }
  // weight a^{R (255 - c)} = a^{64 R (3 - w)} a^{R (63 - l)}, then the block sum
#pragma unroll
  for (int t = 0; t < K; ++t) {
    const double pr = tab.re(lay.eWV(kWaves - 1 - wid), t), pi = tab.im(lay.eWV(kWaves - 1 - wid), t);
    const double qr = tab.re(lay.eLANE(63 - lane), t), qi = tab.im(lay.eLANE(63 - lane), t);
    const double wr = pr * qr - pi * qi, wi = pr * qi + pi * qr;
    double vr = wr * ar[t] - wi * ai[t], vi = wr * ai[t] + wi * ar[t];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) { vr += __shfl_xor(vr, off, 64); vi += __shfl_xor(vi, off, 64); }
    if (lane == 0) { s_sum[wid][2 * t] = vr; s_sum[wid][2 * t + 1] = vi; }
  }
  __syncthreads();
  if (tid < 2 * K) {
    double v = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) v += s_sum[w][tid];
    P.segstate[s * 2 * K + tid] = v;
  }
}

}  // namespace

using KernelFn = void (*)(ScanLaunch);

// One instantiation set per K, defined in scan_k<K>.hip.
template <int K, int R>
KernelFn pick_scan(int var, int acc, int gauss, int mom, int dt) {
  static_assert(R % 4 == 0, "R must be a multiple of 4");
#define MK_PICK(V, A, G, M, D) \
  if (var == V && acc == A && gauss == G && mom == M && dt == D) return (KernelFn)scan_kernel<V, K, R, A, G, M, D>;
#define MK_PICK_DT(V, A, G, M) MK_PICK(V, A, G, M, 0) MK_PICK(V, A, G, M, 1) MK_PICK(V, A, G, M, 2)
#define MK_PICK_FWD(A) MK_PICK_DT(kFwd, A, 0, 0) MK_PICK_DT(kFwd, A, 1, 0) MK_PICK_DT(kFwd, A, 2, 0) MK_PICK_DT(kFwd, A, 3, 0)
  MK_PICK_FWD(kAccF32) MK_PICK_FWD(kAccF64) MK_PICK_FWD(kAccMixed)
  // the compensated scan (a precision reference): Morlet and Gaussian smoothing, one tile shape
  if constexpr (R == 16) { MK_PICK_DT(kFwd, kAccKahan, 0, 0) MK_PICK_DT(kFwd, kAccKahan, 1, 0) }
  MK_PICK(kAdj, kAccMixed, 0, 0, 0) MK_PICK(kAdj, kAccMixed, 1, 0, 0) MK_PICK(kAdj, kAccF64, 0, 0, 0) MK_PICK(kAdj, kAccF64, 1, 0, 0)
  MK_PICK(kAdj, kAccF32, 0, 0, 0) MK_PICK(kAdj, kAccF32, 1, 0, 0)
  MK_PICK_DT(kPg, kAccF64, 0, 0) MK_PICK_DT(kPg, kAccF64, 1, 0) MK_PICK_DT(kPg, kAccF64, 0, 1) MK_PICK_DT(kPg, kAccF64, 1, 1)
  // the segments schedule's pass without outputs (one per input type)
  if (var == kSegSum) return dt == 0 ? (KernelFn)seg_sum_kernel<K, R, 0> : dt == 1 ? (KernelFn)seg_sum_kernel<K, R, 1>
                              : dt == 2 ? (KernelFn)seg_sum_kernel<K, R, 2> : nullptr;
#undef MK_PICK_FWD
#undef MK_PICK_DT
#undef MK_PICK
  return nullptr;
}

}  // namespace mk
