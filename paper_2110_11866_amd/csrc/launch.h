// Launch descriptors between the C ABI layer and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "layout.h"

namespace mk {

// Scan arithmetic: float32 tile scan with float64 carries, float64 throughout, float64 chunk
// sums and wave scan with a float32 recurrence, the float32 tile scan in compensated
// (float-float) arithmetic.
enum ScanAcc { kAccF32 = 0, kAccF64 = 1, kAccMixed = 2, kAccKahan = 3 };

struct ScanLaunch {
  int K, R, acc, kind;          // acc: ScanAcc; kind: 0 Morlet (complex64 out), 1 Gaussian (float32 out)
  const void* x;                // signal(s)
  int dtype;                    // 0 f32, 1 f16, 2 bf16
  void* out;                    // complex64 or float32
  Row row0;                     // the only row when nrows == 1
  const Row* rows;              // device rows when nrows > 1
  int nrows;
  const int32_t* tile_row;      // device: row of every tile when nrows > 1
  const int32_t* row_order;     // device: row-serial schedule, the rows of queue q at
                                // [qstart[q], qstart[q + 1]), each queue longest rows first
  int32_t qstart[kQueues + 1];
  int serial;                   // 1: blocks take whole rows (no look-back); 0: tiles + look-back
  int64_t ntiles;
  const unsigned char* tabs;    // device constant tables, one per scale
  int64_t tab_stride;
  int64_t f32_bytes;            // offset of the float64 half of a table
  void* ws;                     // workspace (header + tile states)
  int grid;                     // persistent grid size
  const void* g;                // gradient pass: cotangent at the outputs (complex64 or float32)
  double* partials;             // gradient pass: per-tile float64 partial sums
  // Segments schedule (forward, at most kQueues rows): each row's tiles in segments of seg_len
  // tiles (its last one shorter), the segments of row r numbered [seg_start[r], seg_start[r + 1]).
  // seg_mode 1 (set for the launch with outputs): blocks take segments through the ticket and run
  // each segment's tiles in order from the state segstate holds for it.
  int seg_mode;
  int seg_len;
  int64_t nseg;                 // 0: not this schedule
  int32_t seg_start[kQueues + 1];
  double* segstate;             // device [nseg][2 K] float64 (re, im per term), in the workspace
};

enum ScanVariant { kVarForward = 0, kVarAdjoint = 1, kVarParamGrad = 2, kVarSegSum = 3 };

// Launch a scan variant (forward, adjoint, parameter-gradient pass; mom: carry the
// alpha-derivative states for the ASFT sigma gradient). A forward launch under the segments
// schedule (nseg > 0) is three launches: the segment sums (one block per segment, each
// segment's end state from a zero start), their combination into incoming states, and the scan
// with outputs over the segments.
hipError_t launch_scan(const ScanLaunch& a, int variant, int mom, hipStream_t s);
int scan_occupancy(int K, int R, int variant, int acc, int kind, int mom, int dtype);
// Sum per-tile partials into d/dsigma, d/dxi per scale: per-row sums into rowpart
// [nrows][4K+3] (one block per row), then one block per scale over its rows.
hipError_t launch_pg_finalize(const ScanLaunch& a, int nscales, double* rowpart, double* gparams, hipStream_t s);
// out[b][n] = sum_s part[b][s][n] over the signals of a batched adjoint.
hipError_t launch_sum_scales(const float* part, float* out, const Row* rows, int B, int S, int64_t total,
                             hipStream_t s);

// Truncated direct convolution with exact taps h[k], k in [-H, H] (the benchmark's baseline).
// Number of tap slabs for N outputs and half width H on a device with num_cus compute units;
// with more than one slab the launch needs a partial buffer of slabs x N complex64.
int direct_conv_slabs(int64_t N, int64_t H, int num_cus);
hipError_t launch_direct_conv(const void* x, int dtype, int64_t N, const float2* taps, int64_t H, int slabs,
                              float2* part, float2* W, hipStream_t s);

hipError_t launch_scan_forward(const ScanLaunch& a, hipStream_t s);
// Resident blocks per CU of the forward kernel for this configuration (0 if unsupported).
int scan_forward_occupancy(int K, int R, int acc, int kind);
hipError_t launch_zero_fill(void* p, size_t bytes, hipStream_t s);

// Multiplication method (Sec. III-B), around a three-row Gaussian scan: u = [x cos(xi m),
// -x sin(xi m), x] (float32, 3N), and W[n] = ce (e^{i xi n} (g[n] + i g[N + n]) - kappa g[2N + n])
// with cek = ce kappa, from the rows' smoothings g (3N).
hipError_t launch_mm_demodulate(const void* x, int dtype, float* u, int64_t N, double xi, hipStream_t s);
hipError_t launch_mm_remodulate(const float* g, float2* W, int64_t N, double xi, double ce, double cek,
                                hipStream_t s);

// out[c][r] = in[r][c] for an R x C row-major float32 matrix (separable 2-D filtering).
hipError_t launch_transpose(const float* in, float* out, int64_t R, int64_t C, hipStream_t s);

// The paper's sliding-sum route (comparison path): K-term combination weights, and the
// launches over a buffer of 4 K (N + 2L) complex float32 (g and h, two of each).
struct TreeCoef {
  int K;
  double cc[kMaxTerms], sc[kMaxTerms];
};
hipError_t launch_tree(const void* x, int dtype, int64_t N, int64_t L, int K, int P_S, const TreeCoef& coef,
                       int real_out, float2* buf, void* W, hipStream_t s);

}  // namespace mk
