// Internal layouts shared by the host plan code and the gfx950 kernels: the per-scale
// constant table, the scan rows, the workspace header and the per-tile look-back state.
#pragma once
#include <stdint.h>
#include <stddef.h>

#if defined(__HIP__)
#define MK_HD __host__ __device__
#else
#define MK_HD
#endif

namespace mk {

constexpr int kWave = 64;        // gfx950 wavefront
constexpr int kThreads = 256;    // threads per block of the scan kernels
constexpr int kWaves = kThreads / kWave;
constexpr int kMaxTerms = 12;
constexpr int kLookback = 64;    // predecessors inspected per look-back step (one per lane)
// Row queues of the row-serial schedule: one per XCD of the chip (workgroups are dispatched to
// the XCDs round-robin, block b to XCD b mod 8), so the rows of one signal, which read the same
// input, run behind one XCD's L2. A queue that runs dry sends its blocks on to the next one.
constexpr int kQueues = 8;

// ---------------------------------------------------------------------------------
// Per-scale constant table. Every constant is a power of the per-term rotation
//   a_p = e^{-alpha} e^{-i beta p}
// at a fixed distance, so the same table serves every tile of every row that uses
// the scale. Complex entry e, term i is stored as re at [(2e) K + i], im at
// [(2e+1) K + i]; the K values of one entry are contiguous (one scalar load).
// The table exists three times: float32 entries, then float64 entries, then the float32
// remainders (float64 entry minus float32 entry, rounded) for float-float arithmetic; a fourth
// section holds the run matrices of the matrix-core recurrence (below).
// ---------------------------------------------------------------------------------
struct TabLayout {
  int K, R;
  // complex entries: powers a_p^d at the distances the kernels need
  MK_HD int eA() const { return 0; }                    // a_p
  MK_HD int eP1(int r) const { return 1 + r; }          // a_p^{R-1-r}, r in [0, R): chunk sum weights
  MK_HD int eTR(int d) const { return 1 + R + d; }      // a_p^{R 2^d}, d in [0, 6): wave scan
  MK_HD int eLANE(int l) const { return 7 + R + l; }    // a_p^{R l}, l in [0, 64): per-lane carry phase
  MK_HD int eWV(int w) const { return 71 + R + w; }     // a_p^{64 R w}, w in [0, kWaves]: per-wave carry; w = kWaves gives a^T
  MK_HD int eLB(int k) const { return 72 + R + kWaves + k; }  // a_p^{T k}, k in [0, 64]: look-back weights
  MK_HD int eLB2(int k) const { return 137 + R + kWaves + k; }  // a_p^{64 T k}, k in [0, 64]: group weights
  MK_HD int nComplex() const { return 137 + R + kWaves + 65; }
  // entry nComplex() + e holds d a_p^d for the distance d of entry e (alpha-derivative)
  MK_HD int nComplexAll() const { return 2 * nComplex(); }
  // real K-rows, after the complex ones (row index in units of K values)
  MK_HD int rMW() const { return 2 * nComplexAll(); }      // (-1)^p m_p e^{alpha L}
  MK_HD int rLW() const { return 2 * nComplexAll() + 1; }  // (-1)^p l_p e^{alpha L}
  MK_HD int rSGN() const { return 2 * nComplexAll() + 2; } // (-1)^p
  MK_HD int rCC() const { return 2 * nComplexAll() + 3; }  // m_p (a_p for the Gaussian)
  MK_HD int rSC() const { return 2 * nComplexAll() + 4; }  // l_p
  MK_HD int rJ(int q) const { return 2 * nComplexAll() + 5 + q; }  // Jacobian rows: dcc/dsigma, dcc/dxi, dsc/dsigma, dsc/dxi
  MK_HD int nKRows() const { return 2 * nComplexAll() + 9; }
  // scalars, after the K-rows
  MK_HD int sCX() const { return nKRows() * K + 0; }    // sum_p (-1)^p m_p e^{-alpha L}
  MK_HD int sD() const { return nKRows() * K + 1; }     // e^{-2 alpha L}: trailing-edge weight
  MK_HD int sGre() const { return nKRows() * K + 2; }   // output factor e^{i xi n0} e^{-n0^2/(2 sigma^2)}
  MK_HD int sGim() const { return nKRows() * K + 3; }
  MK_HD int sUP() const { return nKRows() * K + 4; }    // e^{alpha L}
  MK_HD int sDN() const { return nKRows() * K + 5; }    // e^{-alpha L}
  MK_HD int sLL() const { return nKRows() * K + 6; }    // L
  MK_HD int sDSIG() const { return nKRows() * K + 7; }  // d log(output scale) / d sigma = n0^2 / sigma^3 (ASFT)
  MK_HD int sDXI() const { return nKRows() * K + 8; }   // d arg(output factor) / d xi = n0 (ASFT Morlet)
  MK_HD int sDALPHA() const { return nKRows() * K + 9; }  // d alpha / d sigma = -2 n0 / sigma^3 (ASFT)
  // per-term blocks (term t at vHC(t), 64-byte aligned): a_p^1, a_p^2, a_p^3, a_p^4 as
  // (re, im) pairs, the constants of the four-position Horner step of the chunk sums
  MK_HD int vHC(int t) const { return (nKRows() * K + 10 + 7) / 8 * 8 + 8 * t; }
  MK_HD int nValues() const { return vHC(K); }
  MK_HD size_t f32Bytes() const { return ((size_t)nValues() * 4 + 255) / 256 * 256; }
  MK_HD size_t f64Bytes() const { return ((size_t)nValues() * 8 + 255) / 256 * 256; }
  // Fourth section (float32): the run of kRun = 16 positions as one linear map, for the matrix
  // cores. Output o[r] (r < 16) of a run with input differences dy[r'] and state S before the
  // run is, per output component (real part, imaginary part),
  //   o[r] = sum_{r' <= r} Tc[r][r'] dy[r'] + sum_k Cc[r][k] S[k] + Y y[r - 2L]
  // with S[2t] = Re v_t, S[2t + 1] = Im v_t. Tre, Tim: 16 x 16 row-major; Cre, Cim: 16 x mCW()
  // row-major (the state components padded with zero columns to a multiple of 4).
  static constexpr int kRun = 16;
  MK_HD int mCW() const { return 4 * ((2 * K + 3) / 4); }
  MK_HD size_t mfmaOff() const { return 2 * f32Bytes() + f64Bytes(); }
  MK_HD int mTre() const { return 0; }
  MK_HD int mTim() const { return kRun * kRun; }
  MK_HD int mCre() const { return 2 * kRun * kRun; }
  MK_HD int mCim() const { return 2 * kRun * kRun + kRun * mCW(); }
  MK_HD size_t mfmaBytes() const { return (((size_t)2 * kRun * kRun + (size_t)2 * kRun * mCW()) * 4 + 255) / 256 * 256; }
  MK_HD size_t bytes() const { return 2 * f32Bytes() + f64Bytes() + mfmaBytes(); }
};

// One scan row: one signal filtered at one scale. Scan positions j = 0 .. jend-1;
// position j produces output n = j - jout0 when 0 <= n < N.
struct Row {
  int64_t x_off;     // element offset of the signal in the input array
  int64_t w_off;     // element offset of the output row (complex or real elements)
  int64_t N;         // signal length
  int64_t L;         // window half width
  int64_t jout0;     // L - n0
  int64_t jend;      // N + L - n0
  int64_t tile0;     // index of the row's first tile in the launch
  int32_t scale;     // table index
  int32_t ntiles;
};

// Workspace: a header followed by the tile states.
struct WsHeader {
  uint32_t ticket;   // next tile to claim
  uint32_t done;     // blocks finished in the current launch
  uint64_t epoch;    // launches completed on this workspace; tags the tile flags
  uint32_t qticket[kQueues];   // row-serial schedule: next row of each queue
  uint64_t pad[2];
};
static_assert(sizeof(WsHeader) == 64, "header size");

// Tile state: flag word, then K complex float64 aggregates, then K complex inclusive
// prefixes. flag = (epoch + 1) << 2 | status.
// tile status: aggregate published; inclusive prefix published (last tile of a super-group);
// group aggregate published (last tile of any other group)
enum : uint64_t { kEmpty = 0, kAggregate = 1, kInclusive = 2, kGroup = 3 };
// flag, then K complex float64 each: aggregate, inclusive prefix, group aggregate
MK_HD inline size_t tile_state_bytes(int K) { return ((size_t)(8 + 48 * K) + 63) / 64 * 64; }

inline size_t workspace_bytes(int K, int64_t ntiles) {
  return sizeof(WsHeader) + tile_state_bytes(K) * (size_t)(ntiles > 0 ? ntiles : 0);
}

// Per-tile partial sums of the parameter-gradient pass: 4K + 3 doubles.
inline int pg_partials(int K) { return 4 * K + 3; }

}  // namespace mk
