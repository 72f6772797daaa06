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
//   2. chunk sums B = sum_r a^{R-1-r} dy[r] (the thread's contribution to the state);
//   3. inclusive scan of the chunk sums across the wavefront (6 shuffle levels, constants
//      a^{R 2^d});
//   4. wave 0 forms the tile aggregate in float64, publishes it, and resolves the tile's
//      exclusive prefix by a deterministic decoupled look-back: the aggregates of the
//      earlier tiles of its 64-tile group plus the inclusive prefix of the previous
//      group's last tile, gathered one predecessor per lane and summed by a fixed butterfly
//      (agent-scope atomics that bypass the per-XCD L2, so tiles on different XCDs see each
//      other's states);
//   5. each thread rotates its carry in, runs the R-step recurrence and produces its
//      outputs, staged through LDS for coalesced stores (kFwd, kAdj) or reduced per tile
//      into float64 partials (kPg).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "launch.h"
#include "scan_common.h"

namespace mk {
namespace {

enum { kFwd = 0, kAdj = 1, kPg = 2 };

// complex multiply-add helpers on (re, im) pairs
template <typename T>
__device__ __forceinline__ void cmac(T& zr, T& zi, T cr, T ci, T xr, T xi) {  // z += c x
  zr = fma(cr, xr, fma(-ci, xi, zr));
  zi = fma(cr, xi, fma(ci, xr, zi));
}

template <int VAR, int K, int R, bool WIDE, bool GAUSS, bool MOM>
__global__ __launch_bounds__(kThreads) void scan_kernel(ScanLaunch P) {
  using acc_t = typename std::conditional<WIDE, double, float>::type;
  constexpr int T = R * kThreads;
  constexpr int NS = (VAR == kAdj && !GAUSS) ? 2 : 1;   // real input streams
  constexpr int KS = (NS == 2 || MOM) ? 2 * K : K;      // complex states per position
  constexpr int LSTR = (VAR == kFwd && !GAUSS) ? (2 * R + 2) : (R + 1);
  constexpr int NRED = 4 * K + 3;                        // kPg partial sums per tile
  static_assert(!(MOM && VAR != kPg), "moment states only in the gradient pass");

  __shared__ uint32_t s_tile;
  __shared__ double s_wagg[kWaves][2 * KS];
  __shared__ double s_xw[kWaves][2 * KS];
  __shared__ double s_e[kWaves][2 * KS];
  __shared__ double s_p[2 * KS];
  __shared__ float s_stage[(VAR == kPg) ? 1 : kWaves * 64 * LSTR];
  __shared__ double s_red[(VAR == kPg) ? kWaves * NRED : 1];

  WsHeader* hdr = static_cast<WsHeader*>(P.ws);
  unsigned char* states = static_cast<unsigned char*>(P.ws) + sizeof(WsHeader);
  const size_t sbytes = tile_state_bytes(KS);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const uint64_t epoch = ld_u64(&hdr->epoch);
  const uint64_t tag = (epoch + 1) << 2;
  const TabLayout lay{K, R};
  const int esz = P.dtype == 0 ? 4 : 2;

  // A block claims its next tile only when it is ready to start it: a tile claimed early
  // would hold back the look-back of every later tile of its group.
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
    const int mo = lay.nComplex();   // offset of the moment entries d a^d

    // 1. differenced inputs dy[j] = y[j] - a^{2L} y[j-2L] (zero past the row's scan range)
    float ya[NS][R], yb[NS][R];
    if constexpr (VAR == kAdj) {
      if constexpr (GAUSS) {
        const float* g = static_cast<const float*>(P.x) + row.w_off;
        load_run_rev<R>(g, j0, row.N, ya[0]);
        load_run_rev<R>(g, j0 - 2 * row.L, row.N, yb[0]);
      } else {
        const float2* g = static_cast<const float2*>(P.x) + row.w_off;
        load_run_rev_c<R>(g, j0, row.N, ya[0], ya[NS - 1]);
        load_run_rev_c<R>(g, j0 - 2 * row.L, row.N, yb[0], yb[NS - 1]);
      }
    } else {
      const void* xs = static_cast<const char*>(P.x) + row.x_off * esz;
      load_run<R>(xs, P.dtype, j0, row.N, ya[0]);
      load_run<R>(xs, P.dtype, j0 - 2 * row.L, row.N, yb[0]);
    }
    const acc_t Dw = tab.scalar(lay.sD());
    acc_t dy[NS][R];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int r = 0; r < R; ++r)
        dy[s][r] = (j0 + r < row.jend) ? (acc_t)ya[s][r] - Dw * (acc_t)yb[s][r] : (acc_t)0;

    // 2. chunk sums. State i = s K + t: stream s, term t; with MOM, state K + t is the
    //    alpha-derivative of state t: B_w = sum_r a^m ddy[r] - m a^m dy[r], m = R-1-r,
    //    ddy = d dy / d alpha = 2L a^{2L} y[j-2L].
    acc_t br[KS], bi[KS];
#pragma unroll
    for (int i = 0; i < KS; ++i) { br[i] = 0; bi[i] = 0; }
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
#pragma unroll
        for (int t = 0; t < K; ++t) {
          br[s * K + t] = fma(tab.re(lay.eP1(r), t), dy[s][r], br[s * K + t]);
          bi[s * K + t] = fma(tab.im(lay.eP1(r), t), dy[s][r], bi[s * K + t]);
        }
      }
      if constexpr (MOM) {
        const acc_t ddy = (j0 + r < row.jend) ? (acc_t)(2 * row.L) * Dw * (acc_t)yb[0][r] : (acc_t)0;
#pragma unroll
        for (int t = 0; t < K; ++t) {
          br[K + t] = fma(tab.re(lay.eP1(r), t), ddy, fma(-tab.re(mo + lay.eP1(r), t), dy[0][r], br[K + t]));
          bi[K + t] = fma(tab.im(lay.eP1(r), t), ddy, fma(-tab.im(mo + lay.eP1(r), t), dy[0][r], bi[K + t]));
        }
      }
    }

    // 3. inclusive scan over the wave: S_l = sum_{m <= l} Op(R (l - m)) B_m, where Op(d)
    //    multiplies a state by a^d (and, for a moment state, subtracts d a^d times its base)
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      const int off = 1 << d;
      acc_t ur[KS], ui[KS];
#pragma unroll
      for (int i = 0; i < KS; ++i) { ur[i] = __shfl_up(br[i], off, 64); ui[i] = __shfl_up(bi[i], off, 64); }
      if (lane >= off) {
#pragma unroll
        for (int i = 0; i < KS; ++i) {
          const int t = i % K;
          cmac(br[i], bi[i], tab.re(lay.eTR(d), t), tab.im(lay.eTR(d), t), ur[i], ui[i]);
          if (MOM && i >= K) cmac(br[i], bi[i], -tab.re(mo + lay.eTR(d), t), -tab.im(mo + lay.eTR(d), t), ur[t], ui[t]);
        }
      }
    }
    acc_t er[KS], ei[KS];
#pragma unroll
    for (int i = 0; i < KS; ++i) {
      er[i] = __shfl_up(br[i], 1, 64);
      ei[i] = __shfl_up(bi[i], 1, 64);
      if (lane == 0) { er[i] = 0; ei[i] = 0; }
    }
    if (lane == 63) {
#pragma unroll
      for (int i = 0; i < KS; ++i) { s_wagg[wid][2 * i] = (double)br[i]; s_wagg[wid][2 * i + 1] = (double)bi[i]; }
    }
    __syncthreads();

    // 4. tile aggregate, deterministic look-back and per-wave carries (wave 0; lane i owns
    //    state i; whole state vectors pass through LDS so a moment state can read its base)
    if (wid == 0) {
      // state `lane` of Op(d) v for a vector v held in LDS (entry e holds a^d, mo + e holds d a^d)
      auto op_lds = [&](int e, const double* v, double& outr, double& outi) {
        const int t = lane % K;
        outr = 0; outi = 0;
        cmac(outr, outi, tabd.re(e, t), tabd.im(e, t), v[2 * lane], v[2 * lane + 1]);
        if (MOM && lane >= K) cmac(outr, outi, -tabd.re(mo + e, t), -tabd.im(mo + e, t), v[2 * t], v[2 * t + 1]);
      };
      double Ar = 0, Ai = 0;
      if (lane < KS) {
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
          double cr, ci;
          op_lds(lay.eWV(kWaves - 1 - w), &s_wagg[w][0], cr, ci);
          Ar += cr; Ai += ci;
        }
      }
      const TileState st{states + (size_t)tile * sbytes, KS};
      // Tiles are grouped by 64 within the row. Tile i combines, in a fixed order, the
      // aggregates of the earlier tiles of its group and the inclusive prefix of the previous
      // group's last tile, so the float64 sums never depend on timing.
      const int64_t grp0 = (ti / kLookback) * kLookback;
      const int dd = (int)(ti - grp0);
      const bool group_last = (ti % kLookback) == kLookback - 1;
      if (lane < KS) { st_f64(st.agg(lane, 0), Ar); st_f64(st.agg(lane, 1), Ai); }
      release_order();
      if (lane == 0) st_u64(st.flag(), tag | kAggregate);
      double Pr = 0, Pi = 0;
      if (ti > 0) {
        for (;;) {
          bool ok = true;
          if (lane < dd || (lane == dd && grp0 > 0)) {
            const uint64_t f = ld_u64(TileState{states + (size_t)((int64_t)tile - 1 - lane) * sbytes, KS}.flag());
            const int status = ((f & ~3ull) == tag) ? (int)(f & 3ull) : 0;
            ok = (lane < dd) ? (status >= 1) : (status == 2);
          }
          if (__ballot(!ok) == 0) break;
          __builtin_amdgcn_s_sleep(1);
        }
        acquire_order();
        // lane k takes predecessor k's contribution Op(T k) v_k, one state at a time; a fixed
        // butterfly sums them (lanes past the last predecessor contribute exact zeros, so the
        // order never varies)
        const int kmax = grp0 > 0 ? dd : dd - 1;
        const TileState sk{states + (size_t)((int64_t)tile - 1 - lane) * sbytes, KS};
        const bool agg_lane = lane < dd;
#pragma unroll
        for (int i = 0; i < KS; ++i) {
          const int t = i % K;
          double cr = 0, ci = 0;
          if (lane <= kmax) {
            const double vr = ld_f64(agg_lane ? sk.agg(i, 0) : sk.inc(i, 0));
            const double vi = ld_f64(agg_lane ? sk.agg(i, 1) : sk.inc(i, 1));
            cmac(cr, ci, tabd.re(lay.eLB(lane), t), tabd.im(lay.eLB(lane), t), vr, vi);
            if (MOM && i >= K) {
              const double ur = ld_f64(agg_lane ? sk.agg(t, 0) : sk.inc(t, 0));
              const double ui = ld_f64(agg_lane ? sk.agg(t, 1) : sk.inc(t, 1));
              cmac(cr, ci, -tabd.re(mo + lay.eLB(lane), t), -tabd.im(mo + lay.eLB(lane), t), ur, ui);
            }
          }
#pragma unroll
          for (int off = 32; off >= 1; off >>= 1) { cr += __shfl_xor(cr, off, 64); ci += __shfl_xor(ci, off, 64); }
          if (lane == i) { Pr = cr; Pi = ci; }
        }
      }
      if (lane < KS) { s_p[2 * lane] = Pr; s_p[2 * lane + 1] = Pi; }
      wave_lds_sync();
      if (group_last) {
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
            s_e[w + 1][2 * lane] = cr + s_wagg[w][2 * lane];
            s_e[w + 1][2 * lane + 1] = ci + s_wagg[w][2 * lane + 1];
          }
        }
        wave_lds_sync();
      }
    }
    __syncthreads();

    // 5. thread carry (state just before the thread's first position): Op(R lane) X_w + E_l
    const bool has_out = (jt + T > row.jout0) && (row.jout0 + row.N > jt);
    if (has_out) {
      acc_t vr[KS], vi[KS];
#pragma unroll
      for (int i = 0; i < KS; ++i) {
        const int t = i % K;
        vr[i] = er[i];
        vi[i] = ei[i];
        cmac(vr[i], vi[i], tab.re(lay.eLANE(lane), t), tab.im(lay.eLANE(lane), t), (acc_t)s_xw[wid][2 * i],
             (acc_t)s_xw[wid][2 * i + 1]);
        if (MOM && i >= K)
          cmac(vr[i], vi[i], -tab.re(mo + lay.eLANE(lane), t), -tab.im(mo + lay.eLANE(lane), t),
               (acc_t)s_xw[wid][2 * t], (acc_t)s_xw[wid][2 * t + 1]);
      }
      const acc_t cx = tab.scalar(lay.sCX());
      const acc_t gre = tab.scalar(lay.sGre()), gim = tab.scalar(lay.sGim());

      if constexpr (VAR == kPg) {
        // reductions against the cotangent at the output positions n = j - jout0
        float gr[R], gi[R];
        const int64_t n0v = j0 - row.jout0;
        if constexpr (GAUSS) {
          load_run_f32<R>(static_cast<const float*>(P.g) + row.w_off, n0v, row.N, gr);
#pragma unroll
          for (int r = 0; r < R; ++r) gi[r] = 0.f;
        } else {
          load_run_c<R>(static_cast<const float2*>(P.g) + row.w_off, n0v, row.N, gr, gi);
        }
        acc_t sv_re[K], sv_im[K], sw_re[K], sw_im[K], s_xb = 0, q_re = 0, q_im = 0;
#pragma unroll
        for (int t = 0; t < K; ++t) { sv_re[t] = 0; sv_im[t] = 0; sw_re[t] = 0; sw_im[t] = 0; }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          // u = conj(g) G (positions past the row read g = 0)
          const acc_t ur = (acc_t)gr[r] * gre + (acc_t)gi[r] * gim;
          const acc_t ui = (acc_t)gr[r] * gim - (acc_t)gi[r] * gre;
          const acc_t ddy = MOM ? (acc_t)(2 * row.L) * Dw * (acc_t)yb[0][r] : (acc_t)0;
          acc_t A = cx * (acc_t)yb[0][r], B = 0;
#pragma unroll
          for (int t = 0; t < K; ++t) {
            const acc_t ar = tab.re(lay.eA(), t), ai = tab.im(lay.eA(), t);
            const acc_t pr = vr[t], pi = vi[t];
            const acc_t nr = fma(ar, pr, fma(-ai, pi, dy[0][r]));
            const acc_t ni = fma(ar, pi, ai * pr);
            vr[t] = nr; vi[t] = ni;
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
          s_xb = fma(ur, (acc_t)yb[0][r], s_xb);
          q_re = fma(ur, A, fma(ui, B, q_re));
          q_im = fma(ui, A, fma(-ur, B, q_im));
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
      } else {
        float* stg = &s_stage[(wid * 64 + lane) * LSTR];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          acc_t A[NS], B[NS];
#pragma unroll
          for (int s = 0; s < NS; ++s) { A[s] = cx * (acc_t)yb[s][r]; B[s] = 0; }
#pragma unroll
          for (int s = 0; s < NS; ++s) {
#pragma unroll
            for (int t = 0; t < K; ++t) {
              const int i = s * K + t;
              const acc_t ar = tab.re(lay.eA(), t), ai = tab.im(lay.eA(), t);
              const acc_t nr = fma(ar, vr[i], fma(-ai, vi[i], dy[s][r]));
              const acc_t ni = fma(ar, vi[i], ai * vr[i]);
              vr[i] = nr;
              vi[i] = ni;
              A[s] = fma(tab.row(lay.rMW(), t), nr, A[s]);
              if (!GAUSS) B[s] = fma(tab.row(lay.rLW(), t), ni, B[s]);
            }
          }
          if constexpr (VAR == kFwd) {
            if (GAUSS) {
              stg[r] = (float)(gre * A[0]);
            } else {
              stg[2 * r] = (float)(gre * A[0] + gim * B[0]);
              stg[2 * r + 1] = (float)(gim * A[0] - gre * B[0]);
            }
          } else {
            // Re[conj(G) W_c(Re g')] - Im[conj(G) W_c(Im g')], W_c(y) = A(y) + i B(y)
            if (GAUSS) stg[r] = (float)(gre * A[0]);
            else stg[r] = (float)(gre * (A[0] - B[NS - 1]) + gim * (B[0] + A[NS - 1]));
          }
        }
        __syncthreads();
        const int64_t jw = jt + (int64_t)wid * 64 * R;
        const float* sw = &s_stage[wid * 64 * LSTR];
        if constexpr (VAR == kFwd && !GAUSS) {
          float2* W = static_cast<float2*>(P.out) + row.w_off;
#pragma unroll
          for (int s = 0; s < R; ++s) {
            const int e = s * 64 + lane;
            const int64_t n = jw + e - row.jout0;
            const float* q = sw + (e / R) * LSTR + 2 * (e % R);
            if (n >= 0 && n < row.N) W[n] = make_float2(q[0], q[1]);
          }
        } else {
          float* y = static_cast<float*>(P.out) + row.w_off;
#pragma unroll
          for (int s = 0; s < R; ++s) {
            const int e = s * 64 + lane;
            const int64_t n = jw + e - row.jout0;
            if (n >= 0 && n < row.N) y[VAR == kAdj ? row.N - 1 - n : n] = sw[(e / R) * LSTR + (e % R)];
          }
        }
      }
    } else if constexpr (VAR == kPg) {
      if (tid < NRED) P.partials[(size_t)tile * NRED + tid] = 0.0;
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

// One instantiation set per K, defined in scan_k<K>.hip.
template <int K, int R>
KernelFn pick_scan(int var, int wide, int gauss, int mom) {
#define MK_PICK(V, W, G, M) \
  if (var == V && wide == W && gauss == G && mom == M) return (KernelFn)scan_kernel<V, K, R, W, G, M>;
  MK_PICK(kFwd, 0, 0, 0) MK_PICK(kFwd, 0, 1, 0) MK_PICK(kFwd, 1, 0, 0) MK_PICK(kFwd, 1, 1, 0)
  MK_PICK(kAdj, 0, 0, 0) MK_PICK(kAdj, 0, 1, 0) MK_PICK(kAdj, 1, 0, 0) MK_PICK(kAdj, 1, 1, 0)
  MK_PICK(kPg, 1, 0, 0) MK_PICK(kPg, 1, 1, 0) MK_PICK(kPg, 1, 0, 1) MK_PICK(kPg, 1, 1, 1)
#undef MK_PICK
  return nullptr;
}

}  // namespace mk
