/*
 * morlet.h - C ABI of the MI355X (gfx950) library for the Morlet wavelet transform and
 * Gaussian smoothing computed by the sliding Fourier transform (SFT) and the attenuated
 * SFT (ASFT) evaluated as kernel integrals (Yamashita & Wakahara, arXiv 2110.11866).
 *
 * Problem statement (Sec. II, Sec. III): a real signal x[n], n = 0..N-1, zero outside
 * that interval, is filtered by a kernel on the window [-L, L] (the paper calls the half
 * width K; here K is the number of Fourier terms):
 *
 *   Morlet, direct method (Sec. III-A):
 *     psi_hat[k] = sum_{p=P_S}^{P_S+K-1} m_p cos(beta p k) + i l_p sin(beta p k),  beta = pi/L,
 *     with m, l fitted to the dilated Morlet wavelet by minimum squared error (eq. mmse);
 *     SFT : W[n] = sum_{k=-L}^{L} psi_hat[k] x[n-k]
 *     ASFT: W[n] = e^{i xi n0} e^{-n0^2/(2 sigma^2)} sum_{k=-L}^{L} e^{-alpha k} psi_hat[k] x[n-n0-k],
 *           alpha = n0 / sigma^2 (eqs. acp, asfiir12K, siftGauss, GsASFT; the weight decays
 *           for older samples and the output is read n0 samples earlier);
 *   Gaussian (eqs. aproGauss, GsSFT, GsASFT): the same with orders 0..K-1 and the fitted
 *     Gaussian G_hat[k] = sum_p a_p cos(beta p k); the result is real.
 *
 * The library never forms the 2L+1 taps on the device. Each term is a kernel integral
 * (eqs. kernel..kernelInter) evaluated by one fused prefix-scan kernel per call.
 *
 * Conventions for every call below
 *  - Host vs device: plan handles and the arrays documented "host" live in host memory;
 *    x, W, y, gW, gx, gparams and the workspace are device pointers on the device that
 *    was current when the plan was created.
 *  - Layout: real arrays are contiguous; complex arrays are interleaved (re, im) float32
 *    pairs (complex64), contiguous, 8-byte aligned.
 *  - Ownership: the caller owns every array it passes. A plan owns its host data and a
 *    small device table allocated when it is created; morlet_destroy frees both.
 *  - Streams: every launch goes on the given hipStream_t (passed as void*, NULL = the
 *    default stream). Calls are asynchronous and allocate nothing, so they may be
 *    captured in a HIP graph.
 *  - Workspace: forward and backward calls need a device workspace of at least the size
 *    that morlet_workspace_size returns, zero-filled once before its first use
 *    (morlet_workspace_init, or any zero fill). After that it needs no clearing: calls
 *    leave it ready for the next call. Calls that overlap in time must not share one.
 *  - Errors: invalid arguments are reported synchronously, before anything is launched,
 *    with no side effect. A failed HIP launch returns MORLET_ERR_HIP. Asynchronous faults
 *    show up at the caller's next synchronisation. morlet_last_error() returns a message
 *    for the calling thread's last failure.
 *  - Diagnostics: with the environment variable MORLET_LOG set (not "0"), plan creation, the
 *    term chooser and the autotuner print their choices (window, lowest order, kernel error,
 *    tile shape) on stderr.
 */
#ifndef MORLET_H_
#define MORLET_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct morlet_plan_s* morlet_plan_t;

typedef enum {
  MORLET_OK = 0,
  MORLET_ERR_INVALID_ARG = 1,
  MORLET_ERR_UNSUPPORTED = 2,
  MORLET_ERR_ALLOC = 3,
  MORLET_ERR_WORKSPACE = 4,
  MORLET_ERR_HIP = 5
} morlet_status;

/* Storage type of the input signal; arithmetic is float32 (or float64, see below). */
typedef enum { MORLET_F32 = 0, MORLET_F16 = 1, MORLET_BF16 = 2 } morlet_dtype;

/* Transform: plain SFT (Sec. II-A/B) or attenuated SFT (Sec. II-D/E). */
typedef enum { MORLET_SCAN_SFT = 0, MORLET_SCAN_ASFT = 1 } morlet_scan;

/* Scan arithmetic. Inputs and outputs stay 32-bit (16-bit inputs are widened) in every mode.
 *   MORLET_ACC_AUTO  (default): MORLET_ACC_F32 for the attenuated transform, MORLET_ACC_MIXED for
 *                    plain SFT. Without attenuation (|a_p| = 1) the scan state never forgets, so
 *                    the rounding of every tile's float32 aggregate would stay in the state to the
 *                    row's end (a random walk over the row's tiles); with it each aggregate's
 *                    rounding decays by e^{-alpha T} per tile of T positions (Sec. II-D).
 *   MORLET_ACC_F32 : float32 for everything a thread computes - the chunk sums of its positions,
 *                    the 16-lane wave scan, the recurrence and the K-term combination; float64
 *                    only for the carries between the 16-lane rows of a wave, between waves and
 *                    between tiles (the decoupled look-back). Backward calls run the mixed scan
 *                    in this mode.
 *   MORLET_ACC_F64 : float64 scan state, carries and K-term combination (a reference mode).
 *   MORLET_ACC_MIXED: float64 chunk sums and wave scan, float32 recurrence and combination.
 *   MORLET_ACC_KAHAN: the float32 tile scan compensated: every sum and product a thread forms
 *                    (chunk sums, wave scan, recurrence, K-term combination) is carried as an
 *                    unevaluated float32 pair by error-free transformations (TwoSum, FMA-based
 *                    TwoProduct), the constants as float32 pairs too; carries float64 as in
 *                    MORLET_ACC_F32. A precision reference: Morlet and Gaussian smoothing plans
 *                    (not the differentials), R = 16 only (morlet_plan_set_tile returns
 *                    MORLET_ERR_UNSUPPORTED for other tiles), several times the float32 scan's
 *                    cost; backward calls run the mixed scan. */
typedef enum {
  MORLET_ACC_F32 = 0,
  MORLET_ACC_F64 = 1,
  MORLET_ACC_MIXED = 2,
  MORLET_ACC_AUTO = 3,
  MORLET_ACC_KAHAN = 4
} morlet_accum;

/* Maximum number of Fourier terms a plan may use. */
#define MORLET_MAX_TERMS 12

/* Create a Morlet plan for signals of length N (Sec. III-A, direct method).
 *   sigma > 0   : dilation of the wavelet (standard deviation of its Gaussian), samples
 *   xi    > 0   : carrier in rad/sample (the dimensionless carrier is xi*sigma)
 *   K           : number of Fourier terms, 1..MORLET_MAX_TERMS
 *   L           : window half width, K <= L <= 2^30; or 0 to choose the L of smallest
 *                 kernel error on the grid L = round(c sigma), c = 1.50, 1.52, ..., 5.00
 *                 (Sec. V-A chooses the window by minimum error)
 * The lowest order P_S is the one of smallest kernel relative RMSE (Sec. V-A, Fig. MSE2)
 * among 0..min(L-K+1, ceil(xi L / pi) + K); ties go to the smallest P_S.
 * Defaults: SFT, float32 accumulation, n0 = max(1, round(sigma/8)) for ASFT.
 * N >= 0 (N = 0 makes every call a no-op). Allocates the plan's device table on the
 * current device. Errors: MORLET_ERR_INVALID_ARG, MORLET_ERR_ALLOC, MORLET_ERR_HIP. */
morlet_status morlet_plan(morlet_plan_t* out, int64_t N, double sigma, double xi, int32_t K,
                          int64_t L);

/* Create a Gaussian-smoothing plan (eq. aproGauss, orders 0..K-1; eq. GsSFT / GsASFT).
 * Same argument rules as morlet_plan without xi; K <= L + 1. */
morlet_status morlet_plan_gauss(morlet_plan_t* out, int64_t N, double sigma, int32_t K,
                                int64_t L);

/* Create a plan for the Gaussian's differentials applied to the signal (Sec. II-A):
 *   order 1: x_GD[n]  = sum_{p=1}^{K} b_p s_p[n],   G_D[k]  = -2 gamma k G[k] ~ sum b_p sin(beta p k)
 *   order 2: x_GDD[n] = sum_{p=0}^{K-1} d_p c_p[n], G_DD[k] = (4 gamma^2 k^2 - 2 gamma) G[k]
 *                                                          ~ sum d_p cos(beta p k)
 * gamma = 1/(2 sigma^2), b and d by MMSE on [-L, L] (eq. mmse). Run with gauss_smooth
 * (float32 output). Same argument rules as morlet_plan_gauss, with K <= L for order 1;
 * L = 0 takes the window of the Gaussian fit with the same top order (Table 1 uses one
 * beta for G, G_D and G_DD). gauss_smooth_backward gives dLoss/dx (gparams must be null,
 * else MORLET_ERR_UNSUPPORTED): the taps are real, so the transpose is R A R with R the time
 * reversal, i.e. the plan's own forward of the reversed cotangent, reversed; with edge
 * extension the same over the padded row, folded onto the ends (workspace:
 * morlet_backward_workspace_size). morlet_plan_info reports b as sin_coef
 * (order 1) or d as cos_coef (order 2); P_S is 1 or 0.
 * After morlet_plan_set(..., MORLET_SCAN_ASFT, n0, ...) the plan is refitted for the
 * attenuated transform (eqs. siftGauss, gddAsft): the K terms become orders 0..K-1 (P_S = 0)
 * with both components, a_p, b_p, d_p the fits of G (orders 0..K-1), G_D (sines 1..K-1) and
 * G_DD (cosines 0..K-1), alpha = n0 / sigma^2, s = e^{-n0^2/(2 sigma^2)}:
 *   order 1: x_GD[n]  = s sum_p (-alpha a_p) ct_p[n-n0] + b_p st_p[n-n0]
 *   order 2: x_GDD[n] = s sum_p (d_p + alpha^2 a_p) ct_p[n-n0] - 2 alpha b_p st_p[n-n0]
 * and morlet_plan_info reports those two weight vectors as cos_coef and sin_coef, and as
 * kernel_relrmse the error of the attenuated taps against G_D[k + n0] (G_DD[k + n0]) on
 * [-L, L]. Setting SFT again restores the SFT fit.
 * Errors: MORLET_ERR_INVALID_ARG (also for an order other than 1 or 2), MORLET_ERR_ALLOC,
 * MORLET_ERR_HIP. */
morlet_status morlet_plan_gauss_deriv(morlet_plan_t* out, int64_t N, double sigma, int32_t K, int64_t L,
                                      int32_t order);

/* Create a plan for the Morlet wavelet transform by the multiplication method (Sec. III-B):
 * the wavelet's Gaussian envelope is fitted with the cosines of orders 0..P_M on [-L, L]
 * (eq. aproGauss, K = P_M + 1 terms) and the carrier multiplies it,
 *   psi_hat_M[k] = C' (e^{i xi k} - kappa_xi) G_hat[k],  C' = C_xi / (pi^{1/4} sqrt(sigma)) / sqrt(gamma/pi),
 * which is the paper's sum over the real frequencies omega_p = xi + beta p, p = -P_M..P_M.
 * Evaluated as x_M[n] = C' [e^{i xi n} (G_hat * u)[n] - kappa_xi (G_hat * x)[n]] with
 * u[m] = e^{-i xi m} x[m]: a demodulation kernel, one scan launch over three rows (Re u, Im u,
 * x) and a remodulation kernel. Run with morlet_forward (complex64 out); the workspace holds
 * the scan's tile states and 6 N float32 (morlet_workspace_size). morlet_plan_set selects
 * SFT/ASFT (ASFT: the smoothings are read n0 earlier and scaled by e^{-n0^2/(2 sigma^2)}; only
 * the carrier part takes the phase e^{i xi n0}, so the result approximates psi[k + n0]
 * exactly) and the accumulation precision; morlet_plan_set_tile, _set_schedule and
 * _autotune apply. morlet_plan_info reports a_p as cos_coef (sin_coef zero), P_S = 0 and the
 * error of psi_hat_M against psi on [-L, L] as kernel_relrmse. L = 0 takes the error-optimal
 * window of the Gaussian fit. morlet_backward gives dLoss/dx (gparams must be null: parameter
 * gradients return MORLET_ERR_UNSUPPORTED): the transposes of the remodulation and the
 * demodulation around the three rows' adjoint scan; workspace: morlet_backward_workspace_size.
 * Errors: MORLET_ERR_INVALID_ARG (N < 0 or N > 2^38, sigma or xi not finite and > 0,
 * P_M < 0 or P_M + 1 > MORLET_MAX_TERMS, 0 < L < P_M), MORLET_ERR_ALLOC, MORLET_ERR_HIP. */
morlet_status morlet_plan_multiply(morlet_plan_t* out, int64_t N, double sigma, double xi, int32_t P_M,
                                   int64_t L);

/* Create a plan for separable 2-D Gaussian smoothing of an H x W image (row-major, x along a
 * row): the lines of an image are filtered independently (Sec. IV), so
 *   y = G_y *_columns (G_x *_rows img),
 * each axis by eq. aproGauss with orders 0..K-1 on its own window [-L_x, L_x], [-L_y, L_y]
 * (0: the error-optimal window of the fit), zero outside the image. Evaluated as one scan
 * launch over the H rows, a transpose, one scan launch over the W rows of the transposed
 * image and a transpose back. morlet_plan_set (SFT/ASFT with one n0 for both axes, 0 = each
 * axis's default; accumulation), _set_tile and _set_schedule apply to both axes; autotune
 * and the 1-D backward calls return MORLET_ERR_UNSUPPORTED (gauss_smooth2d_backward is the
 * image's backward); morlet_plan_info returns
 * MORLET_ERR_INVALID_ARG (use morlet_image_axis_info). Errors: MORLET_ERR_INVALID_ARG (H or
 * W < 0 or > 2^24, H W > 2^36, sigma not finite and > 0, K outside [1, MORLET_MAX_TERMS],
 * 0 < L < K - 1), MORLET_ERR_UNSUPPORTED (more than 2^31 tiles on an axis),
 * MORLET_ERR_ALLOC, MORLET_ERR_HIP. */
morlet_status morlet_plan_gauss2d(morlet_plan_t* out, int64_t H, int64_t W, double sigma_y, double sigma_x,
                                  int32_t K, int64_t L_y, int64_t L_x);

/* 2-D smoothing: x (device, H x W elements of dtype, row-major) -> y (device float32, H x W).
 * The workspace (morlet_workspace_size, zero-filled once) holds the larger axis's tile states
 * and two H x W float32 buffers. Stream-ordered, no allocation or synchronization. Errors as
 * gauss_smooth; MORLET_ERR_INVALID_ARG for a plan that is not an image plan. */
morlet_status gauss_smooth2d(morlet_plan_t plan, const void* x, morlet_dtype dtype, float* y, void* ws,
                             size_t ws_bytes, void* stream);

/* Backward of the 2-D smoothing for a real loss: gy = dLoss/dy (device float32, H x W) ->
 * gx = dLoss/dx (device float32, H x W, overwritten). The smoothing is linear, so gx is its
 * transpose applied to gy: a transpose, the adjoint scan over the W column lines, a transpose,
 * the adjoint scan over the H row lines. Workspace: morlet_backward_workspace_size (zero-filled
 * once; it is not the forward's). Errors as gauss_smooth2d. */
morlet_status gauss_smooth2d_backward(morlet_plan_t plan, const float* gy, float* gx, void* ws, size_t ws_bytes,
                                      void* stream);

/* The same backward with the width gradients: gx = dLoss/dx as gauss_smooth2d_backward, and
 * gparams (device, 2 doubles) = {dLoss/dsigma_y, dLoss/dsigma_x}, each axis's fitted
 * coefficients differentiated with its window, terms and shift frozen (as for the 1-D plans).
 * x is the forward's input (device, H x W of dtype). It recomputes the row pass and runs each
 * axis's adjoint and gradient pass: the columns of S_x x against the transposed cotangent, then
 * x against the rows' cotangent. Workspace: morlet_backward_workspace_size (zero-filled once).
 * Errors: a Gabor or non-image plan MORLET_ERR_INVALID_ARG; an empty image or unknown dtype
 * MORLET_ERR_UNSUPPORTED; otherwise as gauss_smooth2d_backward. */
morlet_status gauss_smooth2d_grad(morlet_plan_t plan, const void* x, morlet_dtype dtype, const float* gy, float* gx,
                                  double* gparams, void* ws, size_t ws_bytes, void* stream);

/* Create a plan for the separable 2-D Gabor filter of a real H x W image (row-major, x along
 * a row; Sec. IV filters the lines of an image independently): the Morlet transform of every
 * row (sigma_x, xi in rad/sample, K_x terms, window L_x: the direct method of Sec. III-A, rules
 * as morlet_plan), then the Gaussian smoothing of every column of its real and imaginary parts
 * (sigma_y, K_y terms, window L_y: rules as morlet_plan_gauss). L = 0 selects the error-optimal
 * window per axis. y[r][c] = sum_{i,j} G_y[i] psi_x[j] x[r - i][c - j] (ASFT: each axis's
 * attenuated taps, read n0 of that axis later). morlet_plan_set, morlet_plan_set_tile and
 * morlet_plan_set_schedule apply to both axes. H, W in [0, 2^24], H W <= 2^35. The backward
 * (dLoss/dx) is gabor2d_backward; gauss_smooth2d_backward refuses a Gabor plan. */
morlet_status morlet_plan_gabor2d(morlet_plan_t* out, int64_t H, int64_t W, double sigma_x, double xi, int32_t K_x,
                                  int64_t L_x, double sigma_y, int32_t K_y, int64_t L_y);

/* 2-D Gabor filter: x (device, H x W elements of dtype, row-major) -> y (device complex64
 * [re, im] pairs, H x W, row-major). Four launches on the stream: the batched Morlet scan of
 * the H rows into the workspace, a transpose into the real and imaginary planes, one Gaussian
 * scan over their 2W column lines, a transpose back into y. Workspace: morlet_workspace_size
 * (zero-filled once): the tile states and two H W complex64 buffers. Errors: a non-Gabor plan
 * is MORLET_ERR_INVALID_ARG; otherwise as gauss_smooth2d. */
morlet_status gabor2d(morlet_plan_t plan, const void* x, morlet_dtype dtype, void* y, void* ws, size_t ws_bytes,
                      void* stream);

/* Backward of the 2-D Gabor filter for a real loss: gW = dLoss/dRe y + i dLoss/dIm y (device
 * complex64, H x W) -> gx = dLoss/dx (device float32, H x W, overwritten). The transposes of
 * the two passes in reverse order: gW into its real and imaginary planes, the Gaussian adjoint
 * over the 2W column lines, back to complex64, the batched Morlet adjoint over the H rows
 * (per-line adjoints as morlet_backward); gabor2d_grad adds the parameter gradients. Workspace:
 * morlet_backward_workspace_size (zero-filled once; not the forward's). Errors: a non-Gabor
 * plan is MORLET_ERR_INVALID_ARG; a short workspace MORLET_ERR_WORKSPACE. */
morlet_status gabor2d_backward(morlet_plan_t plan, const void* gW, float* gx, void* ws, size_t ws_bytes,
                               void* stream);

/* The same backward with the parameter gradients: gx as gabor2d_backward, and gparams (device,
 * 3 doubles) = {dLoss/dsigma_y, dLoss/dsigma_x, dLoss/dxi}, each axis's fitted coefficients
 * differentiated with its window, terms and shift frozen (as for the 1-D plans). x is the
 * forward's input (device, H x W of dtype). It recomputes the row pass, runs the column pass's
 * adjoint and gradient over the 2W planar column lines, then the row pass's over the H rows.
 * Workspace: morlet_backward_workspace_size (zero-filled once). Errors: a non-Gabor plan
 * MORLET_ERR_INVALID_ARG; an empty image or unknown dtype MORLET_ERR_UNSUPPORTED; otherwise as
 * gabor2d_backward. */
morlet_status gabor2d_grad(morlet_plan_t plan, const void* x, morlet_dtype dtype, const void* gW, float* gx,
                           double* gparams, void* ws, size_t ws_bytes, void* stream);

/* Per-axis parameters of an image plan: axis 0 filters along x (the rows), axis 1 along y.
 * L: window half width; n0: ASFT shift in use (0 for SFT); cos_coef[K of that axis]: a_p (the
 * Gaussian) or m_p (the Morlet rows of a Gabor plan); kernel_relrmse: error of the fitted
 * kernel on [-L, L]. Outputs are nullable. */
morlet_status morlet_image_axis_info(morlet_plan_t plan, int32_t axis, int64_t* L, int64_t* n0, double* cos_coef,
                                     double* kernel_relrmse);

/* Select SFT or ASFT, the ASFT shift n0 (0 = default; 1 <= n0 <= L otherwise) and the
 * accumulation precision. Rebuilds the device table (synchronously). */
morlet_status morlet_plan_set(morlet_plan_t plan, morlet_scan mode, int64_t n0,
                              morlet_accum accum);

/* Tile shape of the scan kernels: R consecutive samples per thread (4, 8, 16 or 32; 256
 * threads per block, so a tile covers 256 R scan positions). Default 16. Small R gives short
 * inputs more tiles (more blocks in flight, less serial work per thread); large R amortises
 * the per-tile carries over more samples. Changes the workspace size; rebuilds the device
 * tables synchronously. Results do not depend on R beyond float32 rounding.
 * Errors: MORLET_ERR_UNSUPPORTED for another R or when a batched plan would exceed 2^31
 * tiles (the plan keeps its tile shape). */
morlet_status morlet_plan_set_tile(morlet_plan_t plan, int32_t R);

/* How a single signal is extended beyond [0, N-1] (Sec. II: zero, or the value on the edge).
 * MORLET_BOUNDARY_ZERO (default). MORLET_BOUNDARY_EDGE: x[j] = x[0] for j < 0 and x[N-1] for
 * j >= N; the forward (morlet_forward, gauss_smooth) pads the signal by 2L edge copies per
 * side in the workspace, scans N + 4L samples and copies the central N outputs (the workspace
 * grows accordingly: query morlet_workspace_size after setting). Host-only, no device work.
 * The backward calls (morlet_backward, gauss_smooth_backward) take the extension's transpose:
 * the adjoint of the padded row folded back (the padded ends' gradients summed onto x[0] and
 * x[N-1]) and the parameter gradients over the padded signal; morlet_backward_workspace_size
 * covers them (it also serves the forward).
 * Errors: MORLET_ERR_INVALID_ARG (unknown value), MORLET_ERR_UNSUPPORTED (scalogram,
 * multiplication-method and image plans). With edge extension morlet_direct_forward and
 * morlet_tree_forward return MORLET_ERR_UNSUPPORTED. */
typedef enum { MORLET_BOUNDARY_ZERO = 0, MORLET_BOUNDARY_EDGE = 1 } morlet_boundary;
morlet_status morlet_plan_set_boundary(morlet_plan_t plan, morlet_boundary boundary);

/* How a plan's forward launch distributes its rows (signal x scale) over the persistent
 * blocks. MORLET_SCHED_TILES: blocks take single tiles in row order and resolve each
 * tile's incoming state with the decoupled look-back. MORLET_SCHED_ROWS (plans of several
 * rows): a block takes a whole row (longest rows first) and carries the state from tile to
 * tile itself, so no block waits on another. MORLET_SCHED_SEGMENTS (launches of at most eight
 * rows: single-signal plans, the multiplication method's three rows, small scalograms): every
 * row is cut into segments of equal tile counts, about two per resident block over all rows; a
 * first launch forms every segment's end state from a zero start (one block per segment,
 * without outputs), a second (one block per row) turns those into each segment's incoming
 * state, and a third runs the segments with outputs, each block carrying the state through its
 * segment's tiles as in the rows schedule (the input is read twice; no block waits on another).
 * For more rows it acts as AUTO. MORLET_SCHED_AUTO (default): rows when the longest row has no
 * more tiles than one block's share of all tiles; else segments for at most eight rows with at
 * least two tiles per resident block; else tiles. The schedules are deterministic; they differ
 * only in the float64 rounding of the carried states. The adjoint and gradient passes use tiles
 * or rows. Host-only, no device work. */
typedef enum {
  MORLET_SCHED_AUTO = 0,
  MORLET_SCHED_TILES = 1,
  MORLET_SCHED_ROWS = 2,
  MORLET_SCHED_SEGMENTS = 3
} morlet_schedule;
morlet_status morlet_plan_set_schedule(morlet_plan_t plan, morlet_schedule schedule);

/* Segments schedule: tiles per segment, 1..4096, or 0 (default) for the automatic length
 * max(ceil(tiles / (2 x resident blocks)), ceil(longest row's tiles / 1024)). The length sets
 * the float64 rounding of the carried states, not the result otherwise. Host-only;
 * MORLET_ERR_INVALID_ARG outside [0, 4096]. */
morlet_status morlet_plan_set_segments(morlet_plan_t plan, int32_t tiles_per_segment);

/* Autotuner: times this plan's forward launch on the caller's input x (device, dtype) for each
 * tile shape (R = 16, 32, 8, 4, in that order; a shape the plan cannot take is skipped) and,
 * each schedule the plan can take (tiles; rows for several rows; segments for at most eight
 * rows): one warm-up launch, then `reps` launches
 * (1..1000) timed with HIP events on `stream`; keeps the fastest (ties: the earlier
 * candidate) as the plan's tile shape and schedule. out (device) receives the
 * trial outputs: any buffer of the forward's output size, overwritten. A setup call: it
 * allocates and frees its own workspace and events, rebuilds the tables synchronously and
 * synchronizes the stream, so it must not run under graph capture. R_out, schedule_out
 * (nullable) report the choice (MORLET_SCHED_TILES, _ROWS or _SEGMENTS). Errors as
 * morlet_forward, MORLET_ERR_ALLOC if the trial workspace cannot be allocated; on error the
 * plan keeps its tile shape and schedule.
 * Persisted choices: when the environment variable MORLET_TUNE_CACHE names a file, a choice
 * is appended to it as one text line (key, R, schedule, time per launch), the key made of the
 * device architecture and the launch shape (plan kind, mode, accumulation, dtype, K, batch
 * shape, total scan positions and largest window in powers of two); a later call whose key is in
 * the file applies the recorded choice without timing (the last line for a key wins). */
morlet_status morlet_plan_autotune(morlet_plan_t plan, const void* x, morlet_dtype dtype, void* out, int32_t reps,
                                   int32_t* R_out, int32_t* schedule_out, void* stream);

/* Refit a single-signal Morlet or Gaussian-smoothing plan at new parameters sigma (and xi, in
 * rad/sample, for Morlet; ignored for Gaussian), keeping its window L, lowest order P_S, terms K,
 * ASFT shift n0, mode, accumulation, tile shape and boundary: the MMSE fit of Sec. III-A (eq.
 * mmse; eq. aproGauss for the Gaussian) and its Jacobian are recomputed on the host at the frozen
 * orders, and the constant table (which also depends on alpha = n0/sigma^2) is copied into the
 * plan's existing device table with hipMemcpyAsync on `stream`, so launches queued on that stream
 * before the call use the old coefficients and later ones the new. For training loops that update
 * sigma and xi every step (the parameter gradients treat L, P_S and n0 as frozen): no device
 * allocation. The first call allocates a pinned host staging copy of the table and an event (kept
 * until morlet_destroy); each call waits on that event for the previous upload to have read the
 * staging copy. Host work and an event wait: not for use under graph capture. Launches on other
 * streams are not ordered with the upload. Errors: MORLET_ERR_INVALID_ARG (null plan, sigma or xi
 * not finite and > 0), MORLET_ERR_UNSUPPORTED (scalogram, image, multiplication-method and
 * differential plans), MORLET_ERR_ALLOC, MORLET_ERR_HIP. */
morlet_status morlet_plan_refit(morlet_plan_t plan, double sigma, double xi, void* stream);

/* Plan parameters (host outputs; any pointer may be NULL).
 *   cos_coef[K]: m_p (Morlet) or a_p (Gaussian); sin_coef[K]: l_p (0 for Gaussian);
 *   jac[4*K]: d(cos_coef)/dsigma, d(cos_coef)/dxi, d(sin_coef)/dsigma, d(sin_coef)/dxi
 *             for the frozen (L, P_S, K), each K long;
 *   kernel_relrmse: ||fit - kernel|| / ||kernel|| on [-L, L]. */
morlet_status morlet_plan_info(morlet_plan_t plan, int64_t* L, int32_t* P_S, int64_t* n0,
                               double* alpha, double* cos_coef, double* sin_coef, double* jac,
                               double* kernel_relrmse);

/* The forward without allocation, for callers that cannot allocate device memory or must not
 * call hipMalloc (code under HIP graph capture, tight serving loops, harnesses that forbid it):
 * morlet_forward on a single-signal Morlet plan, or morlet_scalogram_forward on a scalogram
 * plan, with the scan's workspace taken from a fixed device array inside the library
 * (MORLET_NOALLOC_SCRATCH_BYTES = 8 MiB; each device the library runs on holds one copy until the
 * process ends). x, W, dtype and stream as for those calls. Each call first clears the part of
 * the array its launch reads as its start state (header and tile flags) with a fill kernel on
 * the stream, then launches the scan; the array keeps the last call's contents. Calls that
 * overlap in time on one device share the array and race: order them (one stream, or events).
 * Allocates nothing and synchronises nothing; the array's address is resolved once per device
 * when the first plan is created there (or on the first call). Takes zero-extension plans
 * only, not the multiplication method. Errors: as morlet_forward / morlet_scalogram_forward
 * (MORLET_ERR_INVALID_ARG for a plan that is not a Morlet plan, MORLET_ERR_UNSUPPORTED for edge
 * extension, multiplication-method and image plans); MORLET_ERR_WORKSPACE, with nothing
 * launched, when the launch needs more than the array: the row-serial schedule of a scalogram
 * needs 64 bytes, the tiles schedule 64 bytes plus one tile state per tile of 256 R positions
 * (256 bytes at K <= 5, 640 at K = 12), so a single signal of up to about 2^27 samples at K = 5,
 * R = 16; the segments schedule (the automatic choice for long single signals) 64 bytes plus
 * 16 K bytes per segment (about two segments per resident block); MORLET_ERR_HIP if the
 * array's address cannot be resolved or a launch fails. */
#define MORLET_NOALLOC_SCRATCH_BYTES (8u << 20)
morlet_status morlet_forward_noalloc(morlet_plan_t plan, const void* x, morlet_dtype dtype, void* W, void* stream);

/* Number of terms for an accuracy target (the tuner's choice of K and L): for K = 1, 2, ...,
 * MORLET_MAX_TERMS, the window of smallest kernel error (the L = 0 rule of morlet_plan) and its
 * fit's relative RMSE on [-L, L] (Sec. V-A chooses the window by minimum error; the error falls
 * with the number of terms, Table 1); returns the first K whose error is at most target, with
 * that L and error. Host only (no device). Errors: MORLET_ERR_INVALID_ARG (sigma, xi or target
 * not finite and > 0, null outputs), MORLET_ERR_UNSUPPORTED when no K up to MORLET_MAX_TERMS
 * reaches the target (the outputs then hold the most accurate K). */
morlet_status morlet_choose_terms(double sigma, double xi, double target_relrmse, int32_t* K, int64_t* L,
                                  double* relrmse);
/* The same for Gaussian smoothing (orders 0..K-1, eq. aproGauss). */
morlet_status morlet_choose_terms_gauss(double sigma, double target_relrmse, int32_t* K, int64_t* L, double* relrmse);

/* Test hook for callers' error paths: the nth following launch setup of any entry point
 * (1 = the next) fails with `status` (one of the MORLET_ERR_ codes) instead of launching; later
 * ones run normally. A call whose first launch is the failing one launches nothing; a call of
 * several launches may stop after earlier ones, as it would on a real launch failure. nth = 0
 * disarms. Process-wide. Errors: MORLET_ERR_INVALID_ARG (nth < 0, or a status that is not an
 * error code). */
morlet_status morlet_inject_failure(morlet_status status, int32_t nth);

/* Device workspace bytes needed by forward/backward calls on this plan. */
morlet_status morlet_workspace_size(morlet_plan_t plan, size_t* bytes);

/* Zero-fill a workspace on the stream (needed once, before its first use). */
morlet_status morlet_workspace_init(void* ws, size_t ws_bytes, void* stream);

/* Morlet transform: W[n], n = 0..N-1, complex64 (device), from x (device, N elements of
 * the given dtype). Returns MORLET_ERR_INVALID_ARG for a Gaussian plan or NULL pointers,
 * MORLET_ERR_WORKSPACE if ws_bytes is too small. */
morlet_status morlet_forward(morlet_plan_t plan, const void* x, morlet_dtype dtype, void* W,
                             void* ws, size_t ws_bytes, void* stream);

/* Gaussian smoothing: y[n] float32 (device). Needs a Gaussian plan. */
morlet_status gauss_smooth(morlet_plan_t plan, const void* x, morlet_dtype dtype, float* y,
                           void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------------------
 * Batched ragged scalogram: B signals of lengths lengths[b] (host int64[B], >= 0),
 * packed back to back in one input array, each transformed at S scales (host
 * sigmas[S], xis[S] in rad/sample) with the Morlet direct method (Sec. III-A), K terms.
 * Every scale gets its own window, lowest order and fit:
 *   L_over_sigma = 0 : error-optimal window per scale (the rule of morlet_plan with L = 0)
 *   L_over_sigma > 0 : L_s = ceil(L_over_sigma * sigma_s) (at least K)
 * Output layout (complex64, device): W_packed[S * off_b + s * len_b + n] is scale s of
 * signal b at sample n, off_b = sum_{i<b} len_i (signal-major, then scale, then sample).
 * One persistent launch processes every (signal, scale, tile) work item.
 * morlet_plan_set applies to every scale; its n0 (if > 0) is clamped to each L_s, and
 * n0 = 0 selects max(1, round(sigma_s/8)) per scale. Destroy with morlet_destroy.
 * ------------------------------------------------------------------------------------ */
morlet_status morlet_scalogram_plan(morlet_plan_t* out, int32_t B, const int64_t* lengths, int32_t S,
                                    const double* sigmas, const double* xis, int32_t K, double L_over_sigma);

/* Parameters of scale s of a scalogram plan (outputs as in morlet_plan_info). */
morlet_status morlet_scalogram_scale_info(morlet_plan_t plan, int32_t s, int64_t* L, int32_t* P_S, int64_t* n0,
                                          double* alpha, double* cos_coef, double* sin_coef, double* jac,
                                          double* kernel_relrmse);

/* Scalogram forward: x_packed (device, sum(lengths) elements of dtype) -> W_packed
 * (device complex64, S * sum(lengths) elements). Workspace rules as above. */
morlet_status morlet_scalogram_forward(morlet_plan_t plan, const void* x_packed, morlet_dtype dtype,
                                       void* W_packed, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------------------
 * Differentiation (no counterpart in the paper). For a real loss of W and its cotangent
 *   gW = dLoss/dRe W + i dLoss/dIm W            (complex64 [N], PyTorch's convention)
 * the backward call writes
 *   gx[j] = dLoss/dx[j] = Re sum_k conj(h[k]) gW[j + n0 + k]    (float32 [N], overwritten)
 * where h are the taps of the transform (psi_hat for SFT, e^{i xi n0} e^{-n0^2/(2 sigma^2)}
 * e^{-alpha k} psi_hat[k] for ASFT), computed as the same scan run on the time-reversed
 * cotangent with the conjugate kernel; and, if gparams is not NULL (device float64),
 *   gparams[0] = dLoss/dsigma, gparams[1] = dLoss/dxi
 * with the window L, the order P_S and the shift n0 held fixed. The sigma and xi dependence
 * goes through the fitted coefficients (the plan's Jacobian), and for ASFT also through
 * alpha = n0/sigma^2 (a scan of the alpha-derivative states), the output scale and the
 * carrier phase. x is the forward input (needed only when gparams is not NULL). The
 * gradient pass scans and accumulates in float64 (the chain rule through the fitted
 * coefficients cancels its per-term sums by orders of magnitude); the sums are taken in a
 * fixed order, so repeated calls give identical bits.
 * Workspace: morlet_backward_workspace_size bytes (zero-filled once, as above).
 * ------------------------------------------------------------------------------------ */
morlet_status morlet_backward_workspace_size(morlet_plan_t plan, size_t* bytes);

morlet_status morlet_backward(morlet_plan_t plan, const void* x, morlet_dtype dtype, const void* gW, float* gx,
                              double* gparams, void* ws, size_t ws_bytes, void* stream);

/* Gaussian smoothing backward: gy float32 [N] is dLoss/dy; gparams[0] = dLoss/dsigma,
 * gparams[1] = 0. On a differential plan (morlet_plan_gauss_deriv) only dLoss/dx is built:
 * gparams must be NULL (else MORLET_ERR_UNSUPPORTED); x is unused. */
morlet_status gauss_smooth_backward(morlet_plan_t plan, const void* x, morlet_dtype dtype, const float* gy,
                                    float* gx, double* gparams, void* ws, size_t ws_bytes, void* stream);

/* Scalogram backward: gW_packed as W_packed; gx_packed float32 [sum lengths] gets the sum
 * over scales of each scale's adjoint (summed in scale order); gparams (device float64
 * [S][2], nullable) gets dLoss/dsigma_s and dLoss/dxi_s summed over the signals. */
morlet_status morlet_scalogram_backward(morlet_plan_t plan, const void* x_packed, morlet_dtype dtype,
                                        const void* gW_packed, float* gx_packed, double* gparams, void* ws,
                                        size_t ws_bytes, void* stream);

/* Baseline for comparison (Sec. V-B, the "conventional method"): the truncated direct
 * convolution W[n] = sum_{|k|<=H} psi[k] x[n-k] with the exact Morlet taps of the plan's
 * sigma and xi (not the K-term fit), H = half_width (0 = the plan's L; the paper's method
 * uses H = ceil(3 sigma)). W complex64 [N] (device). O(N H) work. The first call for a given
 * H allocates and uploads the taps (synchronously), plus a partial-output buffer of up to 64 N
 * complex64 when the taps are split into slabs to fill the device (few outputs, many taps);
 * later calls allocate nothing. Needs a single-signal Morlet plan. */
morlet_status morlet_direct_forward(morlet_plan_t plan, const void* x, morlet_dtype dtype, void* W,
                                    int64_t half_width, void* stream);

/* Comparison path: the paper's own GPU route (Sec. IV). Per order p the window sum of
 * x[j] e^{i beta p j} over [n - L, n + L] by binary doubling (Algorithm 1), then demodulation
 * and the K-term combination: the same SFT result as morlet_forward / gauss_smooth (SFT
 * mode only) by another summation order, O(N K log L) work in log2(2L + 1) levels (the first
 * nine in one LDS pass, one global pass per further level). For single-signal Morlet plans
 * (out: complex64 [N]) and Gaussian smoothing plans (out: float32 [N]). The workspace
 * (morlet_tree_workspace_size: 4 K (N + 2L) complex float32, no initialisation needed)
 * belongs to the caller. Errors: MORLET_ERR_INVALID_ARG (other plan kinds, null pointers),
 * MORLET_ERR_UNSUPPORTED (ASFT mode, unknown dtype), MORLET_ERR_WORKSPACE, MORLET_ERR_HIP. */
morlet_status morlet_tree_workspace_size(morlet_plan_t plan, size_t* bytes);
morlet_status morlet_tree_forward(morlet_plan_t plan, const void* x, morlet_dtype dtype, void* out, void* ws,
                                  size_t ws_bytes, void* stream);

/* Destroy a plan (NULL is ignored). Not stream-ordered: no call using it may be pending. */
void morlet_destroy(morlet_plan_t plan);

/* Message for the calling thread's last failed call ("" if none). */
const char* morlet_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MORLET_H_ */
