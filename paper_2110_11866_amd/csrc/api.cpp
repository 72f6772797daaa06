// C ABI entry points (include/morlet.h): argument checks, plan construction, launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <limits>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "../../include/morlet.h"
#include "boundary.h"
#include "image2d.h"
#include "launch.h"
#include "multiply.h"
#include "noalloc.h"
#include "plan_internal.h"

namespace {

thread_local std::string g_err;

morlet_status fail(morlet_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// MORLET_LOG set (to anything but "0"): plan diagnostics on stderr
bool log_on() {
  static const bool on = [] {
    const char* v = std::getenv("MORLET_LOG");
    return v && *v && std::strcmp(v, "0") != 0;
  }();
  return on;
}

// morlet_inject_failure: the armed launch setup (counting down) fails with the armed status
std::atomic<int> g_inject_after{0};
std::atomic<int> g_inject_status{0};
morlet_status injected() {
  if (g_inject_after.load(std::memory_order_relaxed) <= 0) return MORLET_OK;
  if (g_inject_after.fetch_sub(1, std::memory_order_relaxed) != 1) return MORLET_OK;
  return fail((morlet_status)g_inject_status.load(std::memory_order_relaxed), "injected failure (morlet_inject_failure)");
}

int64_t default_n0(double sigma, int64_t L) {
  int64_t n0 = (int64_t)std::llround(sigma / 8.0);
  if (n0 < 1) n0 = 1;
  if (n0 > L) n0 = L;
  return n0;
}

int64_t tiles_for(int64_t jend, int R) {
  const int64_t T = (int64_t)R * mk::kThreads;
  return jend <= 0 ? 0 : (jend + T - 1) / T;
}

// Device table upload; a plan built without a usable HIP device keeps d_tab == nullptr and
// every launch on it reports MORLET_ERR_HIP.
morlet_status upload_table(morlet_plan_s* p) {
  if (p->d_tab == nullptr) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
      (void)hipGetLastError();
      return MORLET_OK;
    }
    p->device = dev;
    // set-up of the fixed scratch behind morlet_forward_noalloc, once per device (its failure
    // only disables that entry point, which retries the set-up itself)
    (void)mk::scratch_setup(dev);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
      p->num_cus = cus;
    if (hipMalloc(&p->d_tab, p->h_tab.size()) != hipSuccess) {
      (void)hipGetLastError();
      p->d_tab = nullptr;
      return fail(MORLET_ERR_ALLOC, "hipMalloc of the plan table failed");
    }
    p->tab_bytes = p->h_tab.size();
  }
  if (hipMemcpy(p->d_tab, p->h_tab.data(), p->h_tab.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return fail(MORLET_ERR_HIP, "hipMemcpy of the plan table failed");
  }
  return MORLET_OK;
}

morlet_status finish_plan(morlet_plan_s* p, morlet_plan_t* out) {
  mk::jacobian(p);
  p->n0_asft = default_n0(p->sigma, p->L);
  p->R = 16;
  std::string err;
  mk::build_table(p, &err);
  const morlet_status s = upload_table(p);
  if (s != MORLET_OK) {
    delete p;
    return s;
  }
  if (log_on())
    std::fprintf(stderr, "morlet: plan %s N=%lld sigma=%.6g xi=%.6g K=%d L=%lld P_S=%d relrmse=%.3e\n",
                 p->kind == 0 ? "morlet" : "gauss", (long long)p->N, p->sigma, p->xi, p->K, (long long)p->L, p->P_S,
                 p->relrmse);
  *out = p;
  return MORLET_OK;
}

morlet_status check_common(int64_t N, double sigma, int32_t K, int64_t L) {
  if (N < 0) return fail(MORLET_ERR_INVALID_ARG, "N must be >= 0");
  if (N > ((int64_t)1 << 40)) return fail(MORLET_ERR_INVALID_ARG, "N must be <= 2^40");
  if (!finite_pos(sigma)) return fail(MORLET_ERR_INVALID_ARG, "sigma must be finite and > 0");
  if (K < 1 || K > MORLET_MAX_TERMS) return fail(MORLET_ERR_INVALID_ARG, "K must be in [1, MORLET_MAX_TERMS]");
  if (L < 0 || L > ((int64_t)1 << 30)) return fail(MORLET_ERR_INVALID_ARG, "L must be 0 or in [K, 2^30]");
  return MORLET_OK;
}


// ---------------------------------------------------------------- batched ragged plans
// Row queues of the row-serial schedule, one per XCD. A block that takes a row runs all of its
// tiles, so within a queue the long rows come first (they must start early for the blocks to
// finish together). The rows of one signal read the same input: they go to one queue, so one
// XCD's L2 fetches the signal and its S rows share it. Signals are dealt to the queues longest
// first, each to the queue with the least work so far; with fewer than 4 signals per queue the
// rows are dealt one by one instead (a single long signal's scales are spread over the chip).
void build_row_queues(morlet_plan_s* p) {
  const int nq = mk::kQueues;
  const int64_t nrows = (int64_t)p->rows.size();
  const int S = p->S > 0 ? p->S : 1;
  const bool by_signal = (int64_t)p->B >= 4 * nq && nrows == (int64_t)p->B * S;
  const int64_t ngroups = by_signal ? p->B : nrows;
  auto group_rows = [&](int64_t g, int64_t& r0, int64_t& nr) {
    r0 = by_signal ? g * S : g;
    nr = by_signal ? S : 1;
  };
  std::vector<int64_t> work(ngroups, 0);
  for (int64_t g = 0; g < ngroups; ++g) {
    int64_t r0, nr;
    group_rows(g, r0, nr);
    for (int64_t r = r0; r < r0 + nr; ++r) work[g] += p->rows[r].ntiles;
  }
  std::vector<int64_t> order(ngroups);
  for (int64_t g = 0; g < ngroups; ++g) order[g] = g;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return work[a] > work[b]; });
  std::vector<std::vector<int32_t>> q(nq);
  std::vector<int64_t> load(nq, 0);
  for (int64_t g : order) {
    int best = 0;
    for (int i = 1; i < nq; ++i)
      if (load[i] < load[best]) best = i;
    load[best] += work[g];
    int64_t r0, nr;
    group_rows(g, r0, nr);
    for (int64_t r = r0; r < r0 + nr; ++r) q[best].push_back((int32_t)r);
  }
  p->row_order.clear();
  p->max_row_tiles = 0;
  for (int i = 0; i < nq; ++i) {
    // whole signals: in the order they were dealt (most work first), each signal's rows
    // together, longest first, so that the blocks running at once on the queue's XCD share few
    // signals and find them in its L2; single rows: longest first
    if (by_signal) {   // the queue holds whole signals, S consecutive rows each
      for (size_t k = 0; k + (size_t)S <= q[i].size(); k += (size_t)S)
        std::stable_sort(q[i].begin() + k, q[i].begin() + k + S,
                         [&](int32_t a, int32_t b) { return p->rows[a].ntiles > p->rows[b].ntiles; });
    } else {
      std::stable_sort(q[i].begin(), q[i].end(),
                       [&](int32_t a, int32_t b) { return p->rows[a].ntiles > p->rows[b].ntiles; });
    }
    p->qstart[i] = (int32_t)p->row_order.size();
    p->row_order.insert(p->row_order.end(), q[i].begin(), q[i].end());
    for (int32_t r : q[i]) p->max_row_tiles = std::max<int64_t>(p->max_row_tiles, p->rows[r].ntiles);
  }
  p->qstart[nq] = (int32_t)p->row_order.size();
}

// Rows are signal-major: row b*S + s filters signal b at scale s. The output of row (b, s)
// starts at S * offset_b + s * len_b (layout [signal][scale][n]).
void build_rows(morlet_plan_s* p) {
  p->rows.clear();
  p->tile_row.clear();
  int64_t tile0 = 0, tmax = 0;
  for (int b = 0; b < p->B; ++b) {
    for (int s = 0; s < p->S; ++s) {
      const ScaleParams& sp = p->scales[s];
      const int64_t n0 = p->mode == 1 ? sp.n0_asft : 0;
      mk::Row r{};
      r.x_off = p->offsets[b];
      r.w_off = (int64_t)p->S * p->offsets[b] + (int64_t)s * p->lengths[b];
      r.N = p->lengths[b];
      r.L = sp.L;
      r.jout0 = sp.L - n0;
      r.jend = p->lengths[b] + sp.L - n0;
      r.tile0 = tile0;
      r.scale = s;
      const int64_t nt = p->lengths[b] == 0 ? 0 : tiles_for(r.jend, p->R);
      r.ntiles = (int32_t)nt;
      for (int64_t t = 0; t < nt; ++t) p->tile_row.push_back((int32_t)p->rows.size());
      tile0 += nt;
      tmax += p->lengths[b] == 0 ? 0 : tiles_for(p->lengths[b] + sp.L, p->R);
      p->rows.push_back(r);
    }
  }
  p->ntiles = tile0;
  p->ntiles_max = tmax;
  build_row_queues(p);
}

void build_batched_tables(morlet_plan_s* p) {
  const mk::TabLayout lay{p->K, p->R};
  const size_t tb = lay.bytes();
  p->h_tab.assign(tb * p->S, 0);
  for (int s = 0; s < p->S; ++s) {
    const ScaleParams& sp = p->scales[s];
    mk::fill_table(p->h_tab.data() + tb * s, p->kind, p->K, p->R, sp.L, sp.P_S, sp.sigma, sp.xi, p->mode,
                   p->mode == 1 ? sp.n0_asft : 0, sp.cc, sp.sc, sp.jac);
  }
}

morlet_status upload_batched(morlet_plan_s* p) {
  morlet_status s = upload_table(p);
  if (s != MORLET_OK || !p->d_tab) return s;
  const size_t rb = p->rows.size() * sizeof(mk::Row), tb = p->tile_row.size() * sizeof(int32_t);
  const size_t ob = p->row_order.size() * sizeof(int32_t);
  const size_t need = rb + tb + ob + 16;
  if (p->d_rows && p->rows_bytes < need) {
    (void)hipFree(p->d_rows);
    p->d_rows = nullptr;
  }
  if (!p->d_rows) {
    if (hipMalloc(&p->d_rows, need) != hipSuccess) {
      (void)hipGetLastError();
      p->d_rows = nullptr;
      return fail(MORLET_ERR_ALLOC, "hipMalloc of the row table failed");
    }
    p->rows_bytes = need;
  }
  if ((rb && hipMemcpy(p->d_rows, p->rows.data(), rb, hipMemcpyHostToDevice) != hipSuccess) ||
      (tb && hipMemcpy(static_cast<char*>(p->d_rows) + rb, p->tile_row.data(), tb, hipMemcpyHostToDevice) != hipSuccess) ||
      (ob && hipMemcpy(static_cast<char*>(p->d_rows) + rb + tb, p->row_order.data(), ob, hipMemcpyHostToDevice) !=
                 hipSuccess)) {
    (void)hipGetLastError();
    return fail(MORLET_ERR_HIP, "hipMemcpy of the row table failed");
  }
  return MORLET_OK;
}

// A batched Gaussian plan over B rows of equal length (one scale, orders 0..K-1 on [-L, L],
// L = 0: the fit's error-optimal window): the scan behind the multiplication method and the
// two axes of an image plan. On error the plan is left for the caller to destroy.
morlet_status init_gauss_rows(morlet_plan_s* p, int B, int64_t len, double sigma, int K, int64_t L) {
  p->kind = 1;
  p->sigma = sigma;
  p->K = K;
  p->L = L ? L : mk::select_L(sigma, 0.0, K, true);
  p->P_S = 0;
  std::vector<double> g, none;
  mk::gauss_taps(sigma, p->L, g);
  const mk::Fit f = mk::fit_orders(g, none, p->L, 0, K);
  p->cc = f.cc;
  p->sc.assign(K, 0.0);
  p->relrmse = f.relrmse;
  mk::jacobian(p);   // d a / d sigma, for the parameter gradients of image plans
  p->batched = true;
  p->B = B;
  p->S = 1;
  p->N = (int64_t)B * len;
  p->R = 16;
  p->lengths.assign(B, len);
  p->offsets.resize(B);
  for (int b = 0; b < B; ++b) p->offsets[b] = (int64_t)b * len;
  ScaleParams sp;
  sp.sigma = sigma;
  sp.xi = 0.0;
  sp.L = p->L;
  sp.P_S = 0;
  sp.n0_asft = default_n0(sigma, p->L);
  sp.cc = f.cc;
  sp.sc.assign(K, 0.0);
  sp.jac = p->jac;
  sp.relrmse = f.relrmse;
  p->scales = {sp};
  p->n0_asft = sp.n0_asft;
  build_rows(p);
  if (p->ntiles > ((int64_t)1 << 31)) return fail(MORLET_ERR_UNSUPPORTED, "too many tiles");
  build_batched_tables(p);
  return upload_batched(p);
}

// B Morlet rows of one length at one scale (the row pass of the 2-D Gabor filter): the same
// fit as morlet_plan, rows laid out back to back.
morlet_status init_morlet_rows(morlet_plan_s* p, int B, int64_t len, double sigma, double xi, int K, int64_t L) {
  p->kind = 0;
  p->sigma = sigma;
  p->xi = xi;
  p->K = K;
  p->L = L ? L : mk::select_L(sigma, xi, K, false);
  p->P_S = mk::select_ps(sigma, xi, K, p->L, nullptr);
  std::vector<double> re, im;
  mk::morlet_taps(sigma, xi, p->L, re, im);
  const mk::Fit f = mk::fit_orders(re, im, p->L, p->P_S, K);
  p->cc = f.cc;
  p->sc = f.sc;
  p->relrmse = f.relrmse;
  mk::jacobian(p);
  p->batched = true;
  p->B = B;
  p->S = 1;
  p->N = (int64_t)B * len;
  p->R = 16;
  p->lengths.assign(B, len);
  p->offsets.resize(B);
  for (int b = 0; b < B; ++b) p->offsets[b] = (int64_t)b * len;
  ScaleParams sp;
  sp.sigma = sigma;
  sp.xi = xi;
  sp.L = p->L;
  sp.P_S = p->P_S;
  sp.n0_asft = default_n0(sigma, p->L);
  sp.cc = p->cc;
  sp.sc = p->sc;
  sp.jac = p->jac;
  sp.relrmse = p->relrmse;
  if (!std::isfinite(sp.relrmse)) return fail(MORLET_ERR_INVALID_ARG, "fit failed");
  p->scales = {sp};
  p->n0_asft = sp.n0_asft;
  build_rows(p);
  if (p->ntiles > ((int64_t)1 << 31)) return fail(MORLET_ERR_UNSUPPORTED, "too many tiles");
  build_batched_tables(p);
  return upload_batched(p);
}

// Fill the launch descriptor for this plan (rows, tables, tiles, workspace, grid).
// recompute = true: a forward pass recomputed inside a gradient call; under the default
// accumulation it runs the mixed scan (float64 chunk sums), whose rounding stays below what the
// float64 gradient reductions resolve.
morlet_status make_launch(morlet_plan_t plan, mk::ScanLaunch& a, void* ws, int variant, int mom, int dtype,
                          bool recompute = false) {
  if (const morlet_status inj = injected(); inj != MORLET_OK) return inj;
  const int64_t jend = plan->N + plan->L - plan->n0;
  const int64_t ntiles = plan->batched ? plan->ntiles : tiles_for(jend, plan->R);
  a = mk::ScanLaunch{};
  a.K = plan->K;
  a.R = plan->R;
  // the gradient pass always accumulates in float64: the chain rule through the fitted
  // coefficients cancels the per-term sums by orders of magnitude; the adjoint runs the float64
  // scan, the float32 tile scan under ASFT (whose attenuation bounds what float32 rounding
  // leaves in the state, as in the forward), else the mixed scan
  const int accum = plan->accum == MORLET_ACC_AUTO
                        ? (plan->mode == 1 && !recompute ? MORLET_ACC_F32 : MORLET_ACC_MIXED)
                        : plan->accum;
  a.acc = variant == mk::kVarParamGrad ? mk::kAccF64
          : variant == mk::kVarAdjoint ? (accum == MORLET_ACC_F64                            ? mk::kAccF64
                                          : (accum == MORLET_ACC_F32 && plan->mode == 1) ? mk::kAccF32
                                                                                          : mk::kAccMixed)
          : accum == MORLET_ACC_KAHAN  ? mk::kAccKahan
                                       : accum;
  // differentials: 2 real output from the sines (SFT, first), 1 from the cosines (SFT,
  // second), 3 from both (ASFT)
  a.kind = plan->deriv == 0 ? plan->kind : plan->mode == MORLET_SCAN_ASFT ? 3 : plan->deriv == 1 ? 2 : 1;
  a.row0.x_off = 0;
  a.row0.w_off = 0;
  a.row0.N = plan->N;
  a.row0.L = plan->L;
  a.row0.jout0 = plan->L - plan->n0;
  a.row0.jend = jend;
  a.row0.tile0 = 0;
  a.row0.scale = 0;
  a.row0.ntiles = (int32_t)ntiles;
  a.nrows = 1;
  if (plan->batched) {
    if (!plan->d_rows) return fail(MORLET_ERR_HIP, "plan has no device row table");
    a.rows = static_cast<const mk::Row*>(plan->d_rows);
    a.tile_row = reinterpret_cast<const int32_t*>(static_cast<const char*>(plan->d_rows) +
                                                  plan->rows.size() * sizeof(mk::Row));
    a.row_order = reinterpret_cast<const int32_t*>(static_cast<const char*>(plan->d_rows) +
                                                   plan->rows.size() * sizeof(mk::Row) +
                                                   plan->tile_row.size() * sizeof(int32_t));
    a.nrows = (int)plan->rows.size();
    for (int q = 0; q <= mk::kQueues; ++q) a.qstart[q] = plan->qstart[q];
    if (a.nrows == 1) a.row0 = plan->rows[0];
  }
  a.ntiles = ntiles;
  a.tabs = static_cast<const unsigned char*>(plan->d_tab);
  a.tab_stride = (int64_t)mk::TabLayout{plan->K, plan->R}.bytes();
  a.f32_bytes = (int64_t)mk::TabLayout{plan->K, plan->R}.f32Bytes();
  a.ws = ws;
  a.dtype = dtype;
  const int occ = mk::scan_occupancy(a.K, a.R, variant, a.acc, a.kind, mom, dtype);
  if (occ <= 0) return fail(MORLET_ERR_UNSUPPORTED, "no kernel for this configuration");
  const int64_t cap = (int64_t)occ * plan->num_cus;
  a.grid = (int)(ntiles < cap ? ntiles : cap);
  // Row-serial schedule when the longest row is no more than one block's share of the tiles:
  // every block then runs whole rows, longest first, carrying the state from tile to tile
  // in LDS, and no tile waits on another block.
  a.serial = 0;
  if (plan->batched && a.nrows > 1 && plan->row_serial != 0 && !(plan->row_serial == 2 && a.nrows <= mk::kQueues)) {
    const int64_t share = (ntiles + cap - 1) / cap;
    if (plan->row_serial == 1 || plan->max_row_tiles <= share) {
      a.serial = 1;
      a.grid = (int)(a.nrows < cap ? a.nrows : cap);
    }
  }
  // Segments schedule for a forward launch of at most eight rows that the rows schedule did not
  // take: chosen, or automatic when the launch has at least two tiles per resident block. About
  // two segments per block over all rows (the ticket balances them), at most 64 x 64 tiles each
  // (the reach of the table's look-back weights), every row cut on its own. The segment states
  // sit in the workspace after its header (within what the tiles schedule needs).
  a.nseg = 0;
  if (variant == mk::kVarForward && !a.serial && a.nrows >= 1 && a.nrows <= mk::kQueues && ntiles >= 2 &&
      (plan->row_serial == 2 || (plan->row_serial == -1 && ntiles >= 2 * cap))) {
    // automatic length: about two segments per resident block, and at most 1024 segments per row
    // (one round of the combination, which runs on one CU per row)
    int64_t len = plan->seg_tiles;
    if (len <= 0) {
      int64_t longest = 0;
      for (int r = 0; r < a.nrows; ++r)
        longest = std::max<int64_t>(longest, a.nrows == 1 ? a.row0.ntiles : (int64_t)plan->rows[r].ntiles);
      len = std::max<int64_t>((ntiles + 2 * cap - 1) / (2 * cap), (longest + 1023) / 1024);
    }
    if (len > (int64_t)mk::kLookback * mk::kLookback) len = (int64_t)mk::kLookback * mk::kLookback;
    int64_t nseg = 0;
    a.seg_start[0] = 0;
    for (int r = 0; r < a.nrows; ++r) {
      const int64_t nt = a.nrows == 1 ? a.row0.ntiles : (int64_t)plan->rows[r].ntiles;
      nseg += (nt + len - 1) / len;
      a.seg_start[r + 1] = (int32_t)std::min<int64_t>(nseg, INT32_MAX);
    }
    if (nseg > 0 && nseg <= INT32_MAX) {
      a.seg_len = (int)len;
      a.nseg = nseg;
      a.serial = 1;
      a.grid = (int)(a.nseg < cap ? a.nseg : cap);
      a.segstate = reinterpret_cast<double*>(static_cast<unsigned char*>(ws) + sizeof(mk::WsHeader));
    }
  }
  return MORLET_OK;
}

// Workspace bytes a forward launch reads and writes: the header; the tiles schedule adds a tile
// state per tile, the segments schedule a float64 state vector per segment.
size_t launch_ws_bytes(const mk::ScanLaunch& a, int K, int64_t ntiles) {
  if (a.nseg > 0) return sizeof(mk::WsHeader) + (size_t)a.nseg * 2 * (size_t)K * sizeof(double);
  return a.serial ? sizeof(mk::WsHeader) : mk::workspace_bytes(K, ntiles);
}

int64_t plan_ntiles_max(morlet_plan_t plan) {
  return plan->batched ? plan->ntiles_max : tiles_for(plan->N + plan->L, plan->R);
}

// Backward workspace: header + tile states (2K complex states) | per-tile partials |
// (batched) per-scale adjoint scratch [S][sum lengths] float32.
struct BwdLayout {
  size_t states_end, partials_off, scratch_off, rowpart_off, total;
};
BwdLayout bwd_layout(morlet_plan_t plan) {
  const int64_t nt = plan_ntiles_max(plan);
  BwdLayout b;
  b.states_end = mk::workspace_bytes(2 * plan->K, nt);
  b.partials_off = (b.states_end + 255) / 256 * 256;
  const size_t pbytes = (size_t)nt * mk::pg_partials(plan->K) * sizeof(double);
  b.scratch_off = (b.partials_off + pbytes + 255) / 256 * 256;
  const size_t sbytes = plan->batched ? (size_t)plan->S * (size_t)plan->N * sizeof(float) : 0;
  b.rowpart_off = (b.scratch_off + sbytes + 255) / 256 * 256;
  const size_t nrows = plan->batched ? plan->rows.size() : 1;
  b.total = b.rowpart_off + nrows * mk::pg_partials(plan->K) * sizeof(double);
  return b;
}

// Workspace of a single-signal forward with edge extension: the tile states of the padded
// row, the padded float32 signal (N + 4L) and its outputs (N + 4L), each 256-byte aligned.
struct EdgeLayout {
  size_t x_off, out_off, total;
};
EdgeLayout edge_layout(morlet_plan_t plan) {
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const int64_t Ne = plan->N + 4 * plan->L;
  const size_t esize = plan->kind == 0 ? 8 : 4;
  EdgeLayout e;
  e.x_off = up(mk::workspace_bytes(plan->K, tiles_for(Ne + plan->L, plan->R)));
  e.out_off = up(e.x_off + (size_t)Ne * sizeof(float));
  e.total = e.out_off + (size_t)Ne * esize;
  return e;
}

// Edge extension (Sec. II): every output reads at most 2L samples outside [0, N-1], so the
// signal is padded by 2L edge copies on each side, scanned as one zero-extended row of
// N + 4L samples, and the central N outputs are copied out.
morlet_status run_edge(morlet_plan_t plan, const void* x, int dtype, void* out, void* ws, size_t ws_bytes,
                       void* stream) {
  if (plan->N == 0) return MORLET_OK;
  if (!x || !out || !ws) return fail(MORLET_ERR_INVALID_ARG, "null x, output or workspace pointer");
  const EdgeLayout e = edge_layout(plan);
  if (ws_bytes < e.total) return fail(MORLET_ERR_WORKSPACE, "workspace too small");
  if (!plan->d_tab) return fail(MORLET_ERR_HIP, "plan has no device table (created without a HIP device)");
  const int64_t P = 2 * plan->L, Ne = plan->N + 2 * P;
  const int64_t jend = Ne + plan->L - plan->n0;
  const int64_t ntiles = tiles_for(jend, plan->R);
  if (ntiles > ((int64_t)1 << 31)) return fail(MORLET_ERR_UNSUPPORTED, "too many tiles");
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* wsb = static_cast<unsigned char*>(ws);
  float* xe = reinterpret_cast<float*>(wsb + e.x_off);
  unsigned char* oe = wsb + e.out_off;
  hipError_t err = mk::launch_edge_extend(x, dtype, plan->N, P, xe, s);
  if (err != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(err));
  mk::ScanLaunch a;
  const morlet_status st = make_launch(plan, a, ws, mk::kVarForward, 0, 0);
  if (st != MORLET_OK) return st;
  a.row0.N = Ne;
  a.row0.jend = jend;
  a.row0.ntiles = (int32_t)ntiles;
  a.ntiles = ntiles;
  const int occ = mk::scan_occupancy(a.K, a.R, mk::kVarForward, a.acc, a.kind, 0, 0);
  const int64_t cap = (int64_t)(occ > 0 ? occ : 1) * plan->num_cus;
  a.grid = (int)(ntiles < cap ? ntiles : cap);
  a.x = xe;
  a.dtype = 0;
  a.out = oe;
  err = mk::launch_scan(a, mk::kVarForward, 0, s);
  const size_t esize = plan->kind == 0 ? 8 : 4;
  if (err == hipSuccess)
    err = hipMemcpyAsync(out, oe + (size_t)P * esize, (size_t)plan->N * esize, hipMemcpyDeviceToDevice, s);
  if (err != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(err));
  return MORLET_OK;
}

morlet_status run_scan(morlet_plan_t plan, const void* x, int dtype, void* out, void* ws, size_t ws_bytes,
                       void* stream, int want_kind, bool want_batched = false) {
  if (!plan) return fail(MORLET_ERR_INVALID_ARG, "null plan");
  if (plan->image2d) return fail(MORLET_ERR_INVALID_ARG, "an image plan runs with gauss_smooth2d or gabor2d");
  if (plan->kind != want_kind)
    return fail(MORLET_ERR_INVALID_ARG, want_kind == 0 ? "morlet_forward needs a Morlet plan"
                                                       : "gauss_smooth needs a Gaussian plan");
  if (dtype < 0 || dtype > 2) return fail(MORLET_ERR_UNSUPPORTED, "unknown dtype");
  if (want_batched != plan->batched)
    return fail(MORLET_ERR_INVALID_ARG, want_batched ? "needs a scalogram plan" : "needs a single-signal plan");
  if (plan->boundary == 1) return run_edge(plan, x, dtype, out, ws, ws_bytes, stream);
  const int64_t ntiles = plan->batched ? plan->ntiles : tiles_for(plan->N + plan->L - plan->n0, plan->R);
  if (plan->N == 0 || ntiles == 0) return MORLET_OK;
  if (!x || !out || !ws) return fail(MORLET_ERR_INVALID_ARG, "null x, output or workspace pointer");
  if (ntiles > ((int64_t)1 << 31)) return fail(MORLET_ERR_UNSUPPORTED, "too many tiles");
  if (ws_bytes < mk::workspace_bytes(plan->K, ntiles)) return fail(MORLET_ERR_WORKSPACE, "workspace too small");
  if (!plan->d_tab) return fail(MORLET_ERR_HIP, "plan has no device table (created without a HIP device)");
  mk::ScanLaunch a;
  morlet_status st = make_launch(plan, a, ws, mk::kVarForward, 0, dtype);
  if (st != MORLET_OK) return st;
  a.x = x;
  a.dtype = dtype;
  a.out = out;
  const hipError_t e = mk::launch_scan(a, mk::kVarForward, 0, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  return MORLET_OK;
}

// Workspace of a multiplication-method plan: the three-row scan's tile states, then the rows'
// inputs u (3N float32) and their smoothings g (3N float32), each 256-byte aligned.
struct MultLayout {
  size_t u_off, g_off, total;
};
MultLayout mult_layout(morlet_plan_t plan) {
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  MultLayout m;
  m.u_off = up(mk::workspace_bytes(plan->K, plan->ntiles_max));
  m.g_off = up(m.u_off + 3 * (size_t)plan->mult_N * sizeof(float));
  m.total = m.g_off + 3 * (size_t)plan->mult_N * sizeof(float);
  return m;
}

// Multiplication method (Sec. III-B): demodulate, three-row Gaussian scan, remodulate.
morlet_status run_multiply(morlet_plan_t plan, const void* x, int dtype, void* W, void* ws, size_t ws_bytes,
                           void* stream) {
  if (dtype < 0 || dtype > 2) return fail(MORLET_ERR_UNSUPPORTED, "unknown dtype");
  const int64_t N = plan->mult_N;
  if (N == 0) return MORLET_OK;
  if (!x || !W || !ws) return fail(MORLET_ERR_INVALID_ARG, "null x, output or workspace pointer");
  if (plan->ntiles > ((int64_t)1 << 31)) return fail(MORLET_ERR_UNSUPPORTED, "too many tiles");
  const MultLayout m = mult_layout(plan);
  if (ws_bytes < m.total) return fail(MORLET_ERR_WORKSPACE, "workspace too small");
  if (!plan->d_tab) return fail(MORLET_ERR_HIP, "plan has no device table (created without a HIP device)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* wsb = static_cast<unsigned char*>(ws);
  float* u = reinterpret_cast<float*>(wsb + m.u_off);
  float* g = reinterpret_cast<float*>(wsb + m.g_off);
  hipError_t e = mk::launch_mm_demodulate(x, dtype, u, N, plan->xi, s);
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  mk::ScanLaunch a;
  const morlet_status st = make_launch(plan, a, ws, mk::kVarForward, 0, 0);
  if (st != MORLET_OK) return st;
  a.x = u;
  a.dtype = 0;
  a.out = g;
  e = mk::launch_scan(a, mk::kVarForward, 0, s);
  if (e == hipSuccess)
    e = mk::launch_mm_remodulate(g, static_cast<float2*>(W), N, plan->xi, plan->mult_ce,
                                 plan->mult_ce * plan->mult_kappa, s);
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  return MORLET_OK;
}

// Workspace of an image plan: the larger of the two axes' tile states, then two H x W float32
// buffers (the row pass's output, the transposed image).
struct ImageLayout {
  size_t a_off, b_off, total;
};
ImageLayout image_layout(morlet_plan_t plan) {
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t px = (size_t)plan->img_H * (size_t)plan->img_W * sizeof(float);
  ImageLayout m;
  m.a_off = up(std::max(mk::workspace_bytes(plan->K, plan->axis[0]->ntiles_max),
                        mk::workspace_bytes(plan->K, plan->axis[1]->ntiles_max)));
  m.b_off = up(m.a_off + px);
  m.total = m.b_off + px;
  return m;
}

// Separable 2-D Gaussian smoothing: rows (x -> A), transpose (A -> B), rows of the transposed
// image (B -> A), transpose back (A -> y). Both scans share the workspace's tile states: they
// run in stream order and each launch re-arms the header for the next.
// Workspace of a 2-D Gabor plan: the larger axis's tile states, then two buffers of H W
// complex64 (the row pass's output, then the two real planes of its transpose).
ImageLayout gabor_layout(morlet_plan_t plan) {
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t px = (size_t)plan->img_H * (size_t)plan->img_W * 2 * sizeof(float);
  ImageLayout m;
  m.a_off = up(std::max(mk::workspace_bytes(plan->axis[0]->K, plan->axis[0]->ntiles_max),
                        mk::workspace_bytes(plan->axis[1]->K, plan->axis[1]->ntiles_max)));
  m.b_off = up(m.a_off + px);
  m.total = m.b_off + px;
  return m;
}

// Separable 2-D Gabor filter (Sec. IV: lines filtered independently): the Morlet transform of
// the H rows (one batched launch, complex64 out), a transpose into the real and imaginary
// planes (W x H each), one Gaussian launch over their 2W rows, a transpose back to complex64.
morlet_status run_gabor2d(morlet_plan_t plan, const void* x, int dtype, void* y, void* ws, size_t ws_bytes,
                          void* stream) {
  if (dtype < 0 || dtype > 2) return fail(MORLET_ERR_UNSUPPORTED, "unknown dtype");
  const int64_t H = plan->img_H, W = plan->img_W;
  if (H == 0 || W == 0) return MORLET_OK;
  if (!x || !y || !ws) return fail(MORLET_ERR_INVALID_ARG, "null x, output or workspace pointer");
  const ImageLayout m = gabor_layout(plan);
  if (ws_bytes < m.total) return fail(MORLET_ERR_WORKSPACE, "workspace too small");
  if (!plan->axis[0]->d_tab || !plan->axis[1]->d_tab)
    return fail(MORLET_ERR_HIP, "plan has no device table (created without a HIP device)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* wsb = static_cast<unsigned char*>(ws);
  float2* Z = reinterpret_cast<float2*>(wsb + m.a_off);
  float* P = reinterpret_cast<float*>(wsb + m.b_off);
  mk::ScanLaunch a;
  morlet_status st = make_launch(plan->axis[0], a, ws, mk::kVarForward, 0, dtype);
  if (st != MORLET_OK) return st;
  a.x = x;
  a.dtype = dtype;
  a.out = Z;
  hipError_t e = mk::launch_scan(a, mk::kVarForward, 0, s);
  if (e == hipSuccess) e = mk::launch_transpose_c2p(Z, P, H, W, s);
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  st = make_launch(plan->axis[1], a, ws, mk::kVarForward, 0, 0);
  if (st != MORLET_OK) return st;
  float* G = reinterpret_cast<float*>(Z);   // the 2W smoothed column lines, planar
  a.x = P;
  a.dtype = 0;
  a.out = G;
  e = mk::launch_scan(a, mk::kVarForward, 0, s);
  if (e == hipSuccess) e = mk::launch_transpose_p2c(G, static_cast<float2*>(y), H, W, s);
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  return MORLET_OK;
}

morlet_status run_image2d(morlet_plan_t plan, const void* x, int dtype, float* y, void* ws, size_t ws_bytes,
                          void* stream) {
  if (dtype < 0 || dtype > 2) return fail(MORLET_ERR_UNSUPPORTED, "unknown dtype");
  const int64_t H = plan->img_H, W = plan->img_W;
  if (H == 0 || W == 0) return MORLET_OK;
  if (!x || !y || !ws) return fail(MORLET_ERR_INVALID_ARG, "null x, output or workspace pointer");
  const ImageLayout m = image_layout(plan);
  if (ws_bytes < m.total) return fail(MORLET_ERR_WORKSPACE, "workspace too small");
  if (!plan->axis[0]->d_tab || !plan->axis[1]->d_tab)
    return fail(MORLET_ERR_HIP, "plan has no device table (created without a HIP device)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* wsb = static_cast<unsigned char*>(ws);
  float* A = reinterpret_cast<float*>(wsb + m.a_off);
  float* B = reinterpret_cast<float*>(wsb + m.b_off);
  mk::ScanLaunch a;
  morlet_status st = make_launch(plan->axis[0], a, ws, mk::kVarForward, 0, dtype);
  if (st != MORLET_OK) return st;
  a.x = x;
  a.dtype = dtype;
  a.out = A;
  hipError_t e = mk::launch_scan(a, mk::kVarForward, 0, s);
  if (e == hipSuccess) e = mk::launch_transpose(A, B, H, W, s);
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  st = make_launch(plan->axis[1], a, ws, mk::kVarForward, 0, 0);
  if (st != MORLET_OK) return st;
  a.x = B;
  a.dtype = 0;
  a.out = A;
  e = mk::launch_scan(a, mk::kVarForward, 0, s);
  if (e == hipSuccess) e = mk::launch_transpose(A, y, W, H, s);
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  return MORLET_OK;
}

// Backward workspace of a single signal with edge extension: the states, partials and row
// partials for the padded row (N + 4L), then the padded signal, the padded cotangent and the
// padded row's adjoint, each 256-byte aligned.
struct EdgeBwdLayout {
  size_t partials_off, rowpart_off, x_off, g_off, gx_off, total;
};
EdgeBwdLayout edge_bwd_layout(morlet_plan_t plan) {
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const int64_t Ne = plan->N + 4 * plan->L;
  const int64_t nt = tiles_for(Ne + plan->L, plan->R);
  const size_t nred = (size_t)mk::pg_partials(plan->K) * sizeof(double);
  const size_t esize = plan->kind == 0 ? 8 : 4;
  EdgeBwdLayout b;
  b.partials_off = up(mk::workspace_bytes(2 * plan->K, nt));
  b.rowpart_off = up(b.partials_off + (size_t)nt * nred);
  b.x_off = up(b.rowpart_off + nred);
  b.g_off = up(b.x_off + (size_t)Ne * sizeof(float));
  b.gx_off = up(b.g_off + (size_t)Ne * esize);
  b.total = b.gx_off + (size_t)Ne * sizeof(float);
  return b;
}

// The launch of a single-signal plan moved onto its padded row of Ne samples.
void pad_launch(morlet_plan_t plan, mk::ScanLaunch& a, int64_t Ne, int variant, int mom, int dtype) {
  const int64_t jend = Ne + plan->L - plan->n0;
  const int64_t ntiles = tiles_for(jend, plan->R);
  a.row0.N = Ne;
  a.row0.jend = jend;
  a.row0.ntiles = (int32_t)ntiles;
  a.ntiles = ntiles;
  const int occ = mk::scan_occupancy(a.K, a.R, variant, a.acc, a.kind, mom, dtype);
  const int64_t cap = (int64_t)(occ > 0 ? occ : 1) * plan->num_cus;
  a.grid = (int)(ntiles < cap ? ntiles : cap);
}

// Backward with edge extension: the forward is W = C A E x (E the extension, A the scan of the
// padded row, C the central crop), so dLoss/dx = E^T A^T C^T g: the cotangent zero-padded, the
// adjoint of the padded row, and the fold of the padded ends onto x[0] and x[N-1]; the
// parameter gradients come from the gradient pass over (E x, C^T g).
morlet_status run_backward_edge(morlet_plan_t plan, const void* x, int dtype, const void* g, float* gx,
                                double* gparams, void* ws, size_t ws_bytes, void* stream) {
  if (plan->N == 0) {
    if (gparams) return fail(MORLET_ERR_UNSUPPORTED, "parameter gradients of an empty signal are not computed");
    return MORLET_OK;
  }
  if (!g || !gx || !ws || (gparams && !x)) return fail(MORLET_ERR_INVALID_ARG, "null pointer");
  const EdgeBwdLayout b = edge_bwd_layout(plan);
  if (ws_bytes < b.total) return fail(MORLET_ERR_WORKSPACE, "workspace too small for the backward pass");
  if (!plan->d_tab) return fail(MORLET_ERR_HIP, "plan has no device table (created without a HIP device)");
  const int64_t P = 2 * plan->L, Ne = plan->N + 2 * P;
  if (tiles_for(Ne + plan->L, plan->R) > ((int64_t)1 << 31)) return fail(MORLET_ERR_UNSUPPORTED, "too many tiles");
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* wsb = static_cast<unsigned char*>(ws);
  float* xe = reinterpret_cast<float*>(wsb + b.x_off);
  void* ge = wsb + b.g_off;
  float* gxe = reinterpret_cast<float*>(wsb + b.gx_off);
  hipError_t e = mk::launch_pad_center(g, plan->kind == 0 ? 8 : 4, plan->N, P, ge, s);
  mk::ScanLaunch a;
  morlet_status st = make_launch(plan, a, ws, mk::kVarAdjoint, 0, 0);
  if (st != MORLET_OK) return st;
  pad_launch(plan, a, Ne, mk::kVarAdjoint, 0, 0);
  a.x = ge;
  a.dtype = 0;
  a.out = gxe;
  if (e == hipSuccess) e = mk::launch_scan(a, mk::kVarAdjoint, 0, s);
  if (e == hipSuccess) e = mk::launch_edge_fold(gxe, plan->N, P, gx, s);
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  if (!gparams) return MORLET_OK;
  const int mom = plan->mode == 1 ? 1 : 0;
  e = mk::launch_edge_extend(x, dtype, plan->N, P, xe, s);
  st = make_launch(plan, a, ws, mk::kVarParamGrad, mom, 0);
  if (st != MORLET_OK) return st;
  pad_launch(plan, a, Ne, mk::kVarParamGrad, mom, 0);
  a.x = xe;
  a.dtype = 0;
  a.g = ge;
  a.partials = reinterpret_cast<double*>(wsb + b.partials_off);
  if (e == hipSuccess) e = mk::launch_scan(a, mk::kVarParamGrad, mom, s);
  if (e == hipSuccess)
    e = mk::launch_pg_finalize(a, 1, reinterpret_cast<double*>(wsb + b.rowpart_off), gparams, s);
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  return MORLET_OK;
}

// Backward workspace of a multiplication-method plan: the three-row plan's backward workspace
// (header first), then the rows' cotangents and their adjoints (3N float32 each).
struct MultBwdLayout {
  size_t g_off, gu_off, total;
};
MultBwdLayout mult_bwd_layout(morlet_plan_t plan) {
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  MultBwdLayout m;
  m.g_off = up(bwd_layout(plan).total);
  m.gu_off = up(m.g_off + 3 * (size_t)plan->mult_N * sizeof(float));
  m.total = m.gu_off + 3 * (size_t)plan->mult_N * sizeof(float);
  return m;
}

// dLoss/dx of the multiplication method: the transpose of the remodulation (three row
// cotangents), the adjoint scan of the three Gaussian rows (one scale, so each row's adjoint is
// written straight to its place), the transpose of the demodulation.
morlet_status run_multiply_backward(morlet_plan_t plan, const void* gW, float* gx, void* ws, size_t ws_bytes,
                                    void* stream) {
  const int64_t N = plan->mult_N;
  if (N == 0) return MORLET_OK;
  if (!gW || !gx || !ws) return fail(MORLET_ERR_INVALID_ARG, "null pointer");
  if (plan->ntiles > ((int64_t)1 << 31)) return fail(MORLET_ERR_UNSUPPORTED, "too many tiles");
  const MultBwdLayout m = mult_bwd_layout(plan);
  if (ws_bytes < m.total) return fail(MORLET_ERR_WORKSPACE, "workspace too small for the backward pass");
  if (!plan->d_tab) return fail(MORLET_ERR_HIP, "plan has no device table (created without a HIP device)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* wsb = static_cast<unsigned char*>(ws);
  float* g3 = reinterpret_cast<float*>(wsb + m.g_off);
  float* gu3 = reinterpret_cast<float*>(wsb + m.gu_off);
  hipError_t e = mk::launch_mm_remodulate_t(static_cast<const float2*>(gW), g3, N, plan->xi, plan->mult_ce,
                                            plan->mult_ce * plan->mult_kappa, s);
  mk::ScanLaunch a;
  const morlet_status st = make_launch(plan, a, ws, mk::kVarAdjoint, 0, 0);
  if (st != MORLET_OK) return st;
  a.x = g3;
  a.dtype = 0;
  a.out = gu3;
  if (e == hipSuccess) e = mk::launch_scan(a, mk::kVarAdjoint, 0, s);
  if (e == hipSuccess) e = mk::launch_mm_demodulate_t(gu3, gx, N, plan->xi, s);
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  return MORLET_OK;
}
// Backward of a differential plan (dLoss/dx). The taps are real and the map of the zero-extended
// signal is an N x N Toeplitz matrix A (y[n] = sum_k h[k] x[n - n0 - k]); every square
// Toeplitz matrix is persymmetric, so A^T = R A R with R the time reversal: gx = R A R gy, the
// plan's own forward of the reversed cotangent, reversed. With edge extension the forward is
// C A_e E (E the extension to Ne = N + 4L samples, A_e the Toeplitz map of the padded row, C the
// central crop), so gx = E^T R A_e R C^T gy: the cotangent zero-padded and reversed, the forward
// over the padded row, reversed, and the padded ends folded onto x[0] and x[N-1].
// Workspace: the forward's tile states, then two float32 buffers of the row's length.
struct DerivBwdLayout {
  int64_t Ne, ntiles;
  size_t a_off, b_off, total;
};
DerivBwdLayout deriv_bwd_layout(morlet_plan_t plan) {
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  DerivBwdLayout m;
  m.Ne = plan->boundary == 1 ? plan->N + 4 * plan->L : plan->N;
  m.ntiles = tiles_for(m.Ne + plan->L - plan->n0, plan->R);
  m.a_off = up(mk::workspace_bytes(plan->K, m.ntiles));
  m.b_off = up(m.a_off + (size_t)m.Ne * sizeof(float));
  m.total = m.b_off + (size_t)m.Ne * sizeof(float);
  return m;
}

morlet_status run_deriv_backward(morlet_plan_t plan, const float* gy, float* gx, void* ws, size_t ws_bytes,
                                 void* stream) {
  if (plan->N == 0) return MORLET_OK;
  if (!gy || !gx || !ws) return fail(MORLET_ERR_INVALID_ARG, "null pointer");
  const DerivBwdLayout m = deriv_bwd_layout(plan);
  if (ws_bytes < m.total) return fail(MORLET_ERR_WORKSPACE, "workspace too small for the backward pass");
  if (!plan->d_tab) return fail(MORLET_ERR_HIP, "plan has no device table (created without a HIP device)");
  if (m.ntiles > ((int64_t)1 << 31)) return fail(MORLET_ERR_UNSUPPORTED, "too many tiles");
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* wsb = static_cast<unsigned char*>(ws);
  float* A = reinterpret_cast<float*>(wsb + m.a_off);
  float* B = reinterpret_cast<float*>(wsb + m.b_off);
  const bool edge = plan->boundary == 1;
  const int64_t P = 2 * plan->L;
  hipError_t e = hipSuccess;
  if (edge) {
    e = mk::launch_pad_center(gy, 4, plan->N, P, A, s);   // C^T gy
    if (e == hipSuccess) e = mk::launch_reverse(A, B, m.Ne, s);
  } else {
    e = mk::launch_reverse(gy, B, m.Ne, s);
  }
  mk::ScanLaunch a;
  const morlet_status st = make_launch(plan, a, ws, mk::kVarForward, 0, 0);
  if (st != MORLET_OK) return st;
  if (edge) pad_launch(plan, a, m.Ne, mk::kVarForward, 0, 0);
  a.x = B;
  a.dtype = 0;
  a.out = A;
  if (e == hipSuccess) e = mk::launch_scan(a, mk::kVarForward, 0, s);
  if (edge) {
    if (e == hipSuccess) e = mk::launch_reverse(A, B, m.Ne, s);
    if (e == hipSuccess) e = mk::launch_edge_fold(B, plan->N, P, gx, s);   // E^T
  } else if (e == hipSuccess) {
    e = mk::launch_reverse(A, gx, m.Ne, s);
  }
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  return MORLET_OK;
}

morlet_status run_backward(morlet_plan_t plan, const void* x, int dtype, const void* g, float* gx, double* gparams,
                           void* ws, size_t ws_bytes, void* stream, int want_kind, bool want_batched) {
  if (!plan) return fail(MORLET_ERR_INVALID_ARG, "null plan");
  if (plan->multiply) {
    if (want_kind != 0 || want_batched) return fail(MORLET_ERR_INVALID_ARG, "plan kind does not match the call");
    if (gparams) return fail(MORLET_ERR_UNSUPPORTED, "parameter gradients are not built for the multiplication method");
    return run_multiply_backward(plan, g, gx, ws, ws_bytes, stream);
  }
  if (plan->image2d) return fail(MORLET_ERR_UNSUPPORTED, "no backward pass for image plans");
  if (plan->kind != want_kind) return fail(MORLET_ERR_INVALID_ARG, "plan kind does not match the call");
  if (plan->deriv != 0) {
    if (gparams) return fail(MORLET_ERR_UNSUPPORTED, "parameter gradients are not built for differential plans");
    return run_deriv_backward(plan, static_cast<const float*>(g), gx, ws, ws_bytes, stream);
  }
  if (want_batched != plan->batched)
    return fail(MORLET_ERR_INVALID_ARG, want_batched ? "needs a scalogram plan" : "needs a single-signal plan");
  if (dtype < 0 || dtype > 2) return fail(MORLET_ERR_UNSUPPORTED, "unknown dtype");
  if (plan->boundary == 1) return run_backward_edge(plan, x, dtype, g, gx, gparams, ws, ws_bytes, stream);
  const int64_t ntiles = plan->batched ? plan->ntiles : tiles_for(plan->N + plan->L - plan->n0, plan->R);
  if (plan->N == 0 || ntiles == 0) {
    if (gparams) return fail(MORLET_ERR_UNSUPPORTED, "parameter gradients of an empty signal are not computed");
    return MORLET_OK;
  }
  if (!g || !gx || !ws || (gparams && !x)) return fail(MORLET_ERR_INVALID_ARG, "null pointer");
  if (ntiles > ((int64_t)1 << 31)) return fail(MORLET_ERR_UNSUPPORTED, "too many tiles");
  const BwdLayout L = bwd_layout(plan);
  if (ws_bytes < L.total) return fail(MORLET_ERR_WORKSPACE, "workspace too small for the backward pass");
  if (!plan->d_tab) return fail(MORLET_ERR_HIP, "plan has no device table (created without a HIP device)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* wsb = static_cast<unsigned char*>(ws);
  // 1. adjoint: dLoss/dx (per scale into the scratch for batched plans, then summed)
  mk::ScanLaunch a;
  morlet_status st = make_launch(plan, a, ws, mk::kVarAdjoint, 0, 0);
  if (st != MORLET_OK) return st;
  a.x = g;
  a.dtype = 0;
  a.out = plan->batched ? static_cast<void*>(wsb + L.scratch_off) : static_cast<void*>(gx);
  hipError_t e = mk::launch_scan(a, mk::kVarAdjoint, 0, s);
  if (e == hipSuccess && plan->batched)
    e = mk::launch_sum_scales(reinterpret_cast<const float*>(wsb + L.scratch_off), gx, a.rows, plan->B, plan->S,
                              plan->N, s);
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  if (!gparams) return MORLET_OK;
  // 2. parameter gradients: forward scan of x reduced against g, then the finalize kernel
  const int mom = plan->mode == 1 ? 1 : 0;
  st = make_launch(plan, a, ws, mk::kVarParamGrad, mom, dtype);
  if (st != MORLET_OK) return st;
  a.x = x;
  a.dtype = dtype;
  a.g = g;
  a.partials = reinterpret_cast<double*>(wsb + L.partials_off);
  e = mk::launch_scan(a, mk::kVarParamGrad, mom, s);
  if (e == hipSuccess)
    e = mk::launch_pg_finalize(a, plan->batched ? plan->S : 1, reinterpret_cast<double*>(wsb + L.rowpart_off),
                               gparams, s);
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  return MORLET_OK;
}


// Backward of an image plan (dLoss/dx for y = T S_y T S_x x, T the transpose, S the line
// smoothings): gx = S_x^T T S_y^T T gy, the batched adjoint of each axis between transposes.
// Workspace: the larger of the two axes' backward workspaces first (its header at offset 0, where
// every launch on this workspace keeps it), then two H x W float32 buffers.
struct ImageBwdLayout {
  size_t axis_bytes, a_off, b_off, c_off = 0, gp_off = 0, total;
};
ImageBwdLayout image_bwd_layout(morlet_plan_t plan) {
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t px = (size_t)plan->img_H * (size_t)plan->img_W * sizeof(float);
  ImageBwdLayout m;
  m.axis_bytes = std::max(bwd_layout(plan->axis[0]).total, bwd_layout(plan->axis[1]).total);
  m.a_off = up(m.axis_bytes);
  m.b_off = up(m.a_off + px);
  m.c_off = up(m.b_off + px);              // third buffer and the per-axis gradients: the
  m.gp_off = up(m.c_off + px);             // parameter-gradient path only
  m.total = m.gp_off + 4 * sizeof(double);
  return m;
}

morlet_status run_image2d_backward(morlet_plan_t plan, const float* gy, float* gx, void* ws, size_t ws_bytes,
                                   void* stream) {
  const int64_t H = plan->img_H, W = plan->img_W;
  if (H == 0 || W == 0) return MORLET_OK;
  if (!gy || !gx || !ws) return fail(MORLET_ERR_INVALID_ARG, "null pointer");
  const ImageBwdLayout m = image_bwd_layout(plan);
  if (ws_bytes < m.total) return fail(MORLET_ERR_WORKSPACE, "workspace too small for the backward pass");
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* wsb = static_cast<unsigned char*>(ws);
  float* A = reinterpret_cast<float*>(wsb + m.a_off);
  float* B = reinterpret_cast<float*>(wsb + m.b_off);
  void* aw = ws;
  const size_t aw_bytes = m.axis_bytes;
  hipError_t e = mk::launch_transpose(gy, A, H, W, s);   // W x H: the column lines' cotangents
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  morlet_status st = run_backward(plan->axis[1], nullptr, 0, A, B, nullptr, aw, aw_bytes, stream, 1, true);
  if (st != MORLET_OK) return st;
  e = mk::launch_transpose(B, A, W, H, s);                // H x W: the row lines' cotangents
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  return run_backward(plan->axis[0], nullptr, 0, A, gx, nullptr, aw, aw_bytes, stream, 1, true);
}

// dLoss/dx and the width gradients of the 2-D smoothing y = T S_y T S_x x. The column pass sees
// the columns of y1 = S_x x with cotangent T gy; the row pass sees x with cotangent
// g1 = T S_y^T T gy. Each axis's batched backward gives its adjoint and its dLoss/dsigma in one
// call (the plan's coefficients frozen, as for the 1-D plans).
morlet_status run_image2d_grad(morlet_plan_t plan, const void* x, int dtype, const float* gy, float* gx,
                               double* gparams, void* ws, size_t ws_bytes, void* stream) {
  if (dtype < 0 || dtype > 2) return fail(MORLET_ERR_UNSUPPORTED, "unknown dtype");
  const int64_t H = plan->img_H, W = plan->img_W;
  if (H == 0 || W == 0) return fail(MORLET_ERR_UNSUPPORTED, "parameter gradients of an empty image are not computed");
  if (!x || !gy || !gx || !gparams || !ws) return fail(MORLET_ERR_INVALID_ARG, "null pointer");
  const ImageBwdLayout m = image_bwd_layout(plan);
  if (ws_bytes < m.total) return fail(MORLET_ERR_WORKSPACE, "workspace too small for the backward pass");
  if (!plan->axis[0]->d_tab || !plan->axis[1]->d_tab)
    return fail(MORLET_ERR_HIP, "plan has no device table (created without a HIP device)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* wsb = static_cast<unsigned char*>(ws);
  float* A = reinterpret_cast<float*>(wsb + m.a_off);
  float* B = reinterpret_cast<float*>(wsb + m.b_off);
  float* C = reinterpret_cast<float*>(wsb + m.c_off);
  double* gp = reinterpret_cast<double*>(wsb + m.gp_off);
  mk::ScanLaunch a;
  morlet_status st = make_launch(plan->axis[0], a, ws, mk::kVarForward, 0, dtype, true);
  if (st != MORLET_OK) return st;
  a.x = x;
  a.dtype = dtype;
  a.out = A;                                                   // y1 = S_x x (H x W)
  hipError_t e = mk::launch_scan(a, mk::kVarForward, 0, s);
  if (e == hipSuccess) e = mk::launch_transpose(A, B, H, W, s);  // its columns (W x H)
  if (e == hipSuccess) e = mk::launch_transpose(gy, C, H, W, s); // their cotangents (W x H)
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  st = run_backward(plan->axis[1], B, 0, C, A, gp, ws, m.axis_bytes, stream, 1, true);
  if (st != MORLET_OK) return st;
  e = mk::launch_transpose(A, B, W, H, s);                       // g1 (H x W)
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  st = run_backward(plan->axis[0], x, dtype, B, gx, gp + 2, ws, m.axis_bytes, stream, 1, true);
  if (st != MORLET_OK) return st;
  e = hipMemcpyAsync(gparams, gp, sizeof(double), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(gparams + 1, gp + 2, sizeof(double), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("copy failed: ") + hipGetErrorString(e));
  return MORLET_OK;
}

// Backward of the 2-D Gabor filter for a real loss (gW = dLoss/dRe y + i dLoss/dIm y, H x W
// complex64): the column pass's transpose on both planes, then the row pass's. gW to planes
// (W x H each), the Gaussian adjoint over the 2W column lines, back to complex64 (H x W), the
// Morlet adjoint over the H rows. Workspace: the larger axis's backward workspace, then two
// buffers of H W complex64.
ImageBwdLayout gabor_bwd_layout(morlet_plan_t plan) {
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t px = (size_t)plan->img_H * (size_t)plan->img_W * 2 * sizeof(float);
  ImageBwdLayout m;
  m.axis_bytes = std::max(bwd_layout(plan->axis[0]).total, bwd_layout(plan->axis[1]).total);
  m.a_off = up(m.axis_bytes);
  m.b_off = up(m.a_off + px);
  m.c_off = up(m.b_off + px);              // third buffer and the per-axis gradients: the
  m.gp_off = up(m.c_off + px);             // parameter-gradient path only
  m.total = m.gp_off + 4 * sizeof(double);
  return m;
}

morlet_status run_gabor2d_backward(morlet_plan_t plan, const void* gW, float* gx, void* ws, size_t ws_bytes,
                                   void* stream) {
  const int64_t H = plan->img_H, W = plan->img_W;
  if (H == 0 || W == 0) return MORLET_OK;
  if (!gW || !gx || !ws) return fail(MORLET_ERR_INVALID_ARG, "null pointer");
  const ImageBwdLayout m = gabor_bwd_layout(plan);
  if (ws_bytes < m.total) return fail(MORLET_ERR_WORKSPACE, "workspace too small for the backward pass");
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* wsb = static_cast<unsigned char*>(ws);
  float* A = reinterpret_cast<float*>(wsb + m.a_off);
  float* B = reinterpret_cast<float*>(wsb + m.b_off);
  hipError_t e = mk::launch_transpose_c2p(static_cast<const float2*>(gW), B, H, W, s);
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  morlet_status st = run_backward(plan->axis[1], nullptr, 0, B, A, nullptr, ws, m.axis_bytes, stream, 1, true);
  if (st != MORLET_OK) return st;
  e = mk::launch_transpose_p2c(A, reinterpret_cast<float2*>(B), H, W, s);   // the rows' complex cotangent
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  return run_backward(plan->axis[0], nullptr, 0, B, gx, nullptr, ws, m.axis_bytes, stream, 0, true);
}

// dLoss/dx with the parameter gradients of the 2-D Gabor filter: the row pass recomputed, its
// planes against the cotangent's planes for the column pass (dLoss/dsigma_y over the 2W
// column lines of one scale), then x against the rows' complex cotangent for the row pass
// (dLoss/dsigma_x, dLoss/dxi). gparams = {dsigma_y, dsigma_x, dxi}.
morlet_status run_gabor2d_grad(morlet_plan_t plan, const void* x, int dtype, const void* gW, float* gx,
                               double* gparams, void* ws, size_t ws_bytes, void* stream) {
  if (dtype < 0 || dtype > 2) return fail(MORLET_ERR_UNSUPPORTED, "unknown dtype");
  const int64_t H = plan->img_H, W = plan->img_W;
  if (H == 0 || W == 0) return fail(MORLET_ERR_UNSUPPORTED, "parameter gradients of an empty image are not computed");
  if (!x || !gW || !gx || !gparams || !ws) return fail(MORLET_ERR_INVALID_ARG, "null pointer");
  const ImageBwdLayout m = gabor_bwd_layout(plan);
  if (ws_bytes < m.total) return fail(MORLET_ERR_WORKSPACE, "workspace too small for the backward pass");
  if (!plan->axis[0]->d_tab || !plan->axis[1]->d_tab)
    return fail(MORLET_ERR_HIP, "plan has no device table (created without a HIP device)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* wsb = static_cast<unsigned char*>(ws);
  float* A = reinterpret_cast<float*>(wsb + m.a_off);
  float* B = reinterpret_cast<float*>(wsb + m.b_off);
  float* C = reinterpret_cast<float*>(wsb + m.c_off);
  double* gp = reinterpret_cast<double*>(wsb + m.gp_off);
  mk::ScanLaunch a;
  morlet_status st = make_launch(plan->axis[0], a, ws, mk::kVarForward, 0, dtype, true);
  if (st != MORLET_OK) return st;
  a.x = x;
  a.dtype = dtype;
  a.out = A;                                                            // y1 = rows' transform
  hipError_t e = mk::launch_scan(a, mk::kVarForward, 0, s);
  if (e == hipSuccess) e = mk::launch_transpose_c2p(reinterpret_cast<const float2*>(A), B, H, W, s);
  if (e == hipSuccess) e = mk::launch_transpose_c2p(static_cast<const float2*>(gW), C, H, W, s);
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  st = run_backward(plan->axis[1], B, 0, C, A, gp, ws, m.axis_bytes, stream, 1, true);
  if (st != MORLET_OK) return st;
  e = mk::launch_transpose_p2c(A, reinterpret_cast<float2*>(B), H, W, s);   // the rows' cotangent
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  st = run_backward(plan->axis[0], x, dtype, B, gx, gp + 2, ws, m.axis_bytes, stream, 0, true);
  if (st != MORLET_OK) return st;
  e = hipMemcpyAsync(gparams, gp, sizeof(double), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(gparams + 1, gp + 2, 2 * sizeof(double), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("copy failed: ") + hipGetErrorString(e));
  return MORLET_OK;
}
}  // namespace

namespace {

// Persisted autotuning (MORLET_TUNE_CACHE names a text file): one line per tuned plan shape,
// "<key>\t<R>\t<rows>", the key made of the device's architecture and everything the launch
// shape depends on (kind, mode, accumulation, input type, terms, batch shape and the sizes in
// powers of two).
std::mutex g_tune_mu;

std::string tune_key(morlet_plan_t plan, int dtype) {
  static std::string arch = [] {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
      (void)hipGetLastError();
      return std::string("unknown");
    }
    return std::string(prop.gcnArchName);
  }();
  int64_t positions = 0, maxL = plan->L;
  if (plan->batched) {
    for (const mk::Row& r : plan->rows) positions += r.jend;
    for (const ScaleParams& sp : plan->scales) maxL = std::max(maxL, sp.L);
  } else {
    positions = plan->N + plan->L;
  }
  auto lg = [](int64_t v) { int b = 0; while (v > 1) { v >>= 1; ++b; } return b; };
  std::ostringstream k;
  k << "arch=" << arch << " kind=" << plan->kind << " deriv=" << plan->deriv << " mult=" << (plan->multiply ? 1 : 0)
    << " mode=" << plan->mode << " accum=" << plan->accum << " dtype=" << dtype << " K=" << plan->K
    << " batched=" << (plan->batched ? 1 : 0) << " B=" << plan->B << " S=" << plan->S << " lgpos=" << lg(positions)
    << " lgL=" << lg(maxL + 1);
  return k.str();
}

bool tune_lookup(const std::string& key, int& R, int& rows) {
  const char* path = std::getenv("MORLET_TUNE_CACHE");
  if (!path || !*path) return false;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  std::ifstream in(path);
  std::string line;
  bool found = false;
  while (std::getline(in, line)) {   // the last entry for a key wins
    const size_t t1 = line.find('\t');
    if (t1 == std::string::npos || line.compare(0, t1, key) != 0 || t1 != key.size()) continue;
    int r = 0, w = 0;
    if (std::sscanf(line.c_str() + t1 + 1, "%d\t%d", &r, &w) == 2 && (r == 4 || r == 8 || r == 16 || r == 32)) {
      R = r;
      rows = w ? 1 : 0;
      found = true;
    }
  }
  return found;
}

void tune_store(const std::string& key, int R, int rows, float ms) {
  const char* path = std::getenv("MORLET_TUNE_CACHE");
  if (!path || !*path) return;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  std::ofstream out(path, std::ios::app);
  out << key << '\t' << R << '\t' << rows << '\t' << ms << '\n';
}

}  // namespace

extern "C" {

morlet_status morlet_plan(morlet_plan_t* out, int64_t N, double sigma, double xi, int32_t K, int64_t L) {
  if (!out) return fail(MORLET_ERR_INVALID_ARG, "null output handle");
  morlet_status s = check_common(N, sigma, K, L);
  if (s != MORLET_OK) return s;
  if (!finite_pos(xi)) return fail(MORLET_ERR_INVALID_ARG, "xi must be finite and > 0");
  if (L != 0 && L < K) return fail(MORLET_ERR_INVALID_ARG, "L must be >= K");
  auto* p = new (std::nothrow) morlet_plan_s;
  if (!p) return fail(MORLET_ERR_ALLOC, "out of host memory");
  p->kind = 0;
  p->N = N;
  p->sigma = sigma;
  p->xi = xi;
  p->K = K;
  p->L = L ? L : mk::select_L(sigma, xi, K, false);
  double err = 0;
  p->P_S = mk::select_ps(sigma, xi, K, p->L, &err);
  std::vector<double> re, im;
  mk::morlet_taps(sigma, xi, p->L, re, im);
  const mk::Fit f = mk::fit_orders(re, im, p->L, p->P_S, K);
  p->cc = f.cc;
  p->sc = f.sc;
  p->relrmse = f.relrmse;
  return finish_plan(p, out);
}

morlet_status morlet_plan_gauss(morlet_plan_t* out, int64_t N, double sigma, int32_t K, int64_t L) {
  if (!out) return fail(MORLET_ERR_INVALID_ARG, "null output handle");
  morlet_status s = check_common(N, sigma, K, L);
  if (s != MORLET_OK) return s;
  if (L != 0 && L + 1 < K) return fail(MORLET_ERR_INVALID_ARG, "L must be >= K - 1");
  auto* p = new (std::nothrow) morlet_plan_s;
  if (!p) return fail(MORLET_ERR_ALLOC, "out of host memory");
  p->kind = 1;
  p->N = N;
  p->sigma = sigma;
  p->xi = 0.0;
  p->K = K;
  p->L = L ? L : mk::select_L(sigma, 0.0, K, true);
  p->P_S = 0;
  std::vector<double> g, none;
  mk::gauss_taps(sigma, p->L, g);
  const mk::Fit f = mk::fit_orders(g, none, p->L, 0, K);
  p->cc = f.cc;
  p->sc = f.sc;
  p->relrmse = f.relrmse;
  return finish_plan(p, out);
}

// Coefficients of a differential plan for its scan mode (Sec. II).
// SFT: the sines 1..K of G_D (order 1) or the cosines 0..K-1 of G_DD (order 2).
// ASFT (eqs. siftGauss, gddAsft): orders 0..K-1 with both components. The attenuation moves
// the Gaussian by n0, G[k + n0] = s e^{-alpha k} G[k] (alpha = n0 / sigma^2, s = e^{-n0^2 /
// (2 sigma^2)}), so G_D[k + n0] = s e^{-alpha k} (G_D - alpha G)[k] and G_DD[k + n0] =
// s e^{-alpha k} (G_DD - 2 alpha G_D + alpha^2 G)[k]; with G ~ sum a_p cos, G_D ~ sum b_p sin
// and G_DD ~ sum d_p cos the weights of c_p and s_p are
//   order 1: cc = -alpha a, sc = b;   order 2: cc = d + alpha^2 a, sc = -2 alpha b.
// The scale s is the output factor the table already carries for every ASFT plan.
static void fit_deriv(morlet_plan_s* p) {
  const int K = p->K;
  const int64_t L = p->L;
  std::vector<double> g, none;
  if (p->mode != MORLET_SCAN_ASFT) {
    mk::gauss_taps(p->sigma, L, g, p->deriv);
    mk::Fit f;
    if (p->deriv == 1) {
      const std::vector<double> zero(g.size(), 0.0);
      f = mk::fit_orders(zero, g, L, 1, K);   // odd target: sine components 1..K
    } else {
      f = mk::fit_orders(g, none, L, 0, K);   // even target: cosine components 0..K-1
    }
    p->P_S = p->deriv == 1 ? 1 : 0;
    p->cc = f.cc;
    p->sc = f.sc;
    p->relrmse = f.relrmse;
    return;
  }
  const double alpha = (double)p->n0 / (p->sigma * p->sigma);
  mk::gauss_taps(p->sigma, L, g, 0);
  const std::vector<double> a = mk::fit_orders(g, none, L, 0, K).cc;
  std::vector<double> b(K, 0.0);
  if (K > 1) {
    std::vector<double> gd;
    mk::gauss_taps(p->sigma, L, gd, 1);
    const std::vector<double> zero(gd.size(), 0.0);
    const std::vector<double> bs = mk::fit_orders(zero, gd, L, 1, K - 1).sc;
    for (int i = 0; i < K - 1; ++i) b[i + 1] = bs[i];
  }
  p->P_S = 0;
  p->cc.assign(K, 0.0);
  p->sc.assign(K, 0.0);
  if (p->deriv == 1) {
    for (int i = 0; i < K; ++i) {
      p->cc[i] = -alpha * a[i];
      p->sc[i] = b[i];
    }
  } else {
    std::vector<double> gdd;
    mk::gauss_taps(p->sigma, L, gdd, 2);
    const std::vector<double> d = mk::fit_orders(gdd, none, L, 0, K).cc;
    for (int i = 0; i < K; ++i) {
      p->cc[i] = d[i] + alpha * alpha * a[i];
      p->sc[i] = -2.0 * alpha * b[i];
    }
  }
  // relative RMSE of the attenuated taps against the shifted differential on [-L, L]
  const double s = std::exp(-(double)p->n0 * (double)p->n0 / (2.0 * p->sigma * p->sigma));
  const double kPi = 3.14159265358979323846;
  const double gamma = 1.0 / (2.0 * p->sigma * p->sigma), norm = std::sqrt(gamma / kPi);
  double num = 0.0, den = 0.0;
  for (int64_t k = -L; k <= L; ++k) {
    double h = 0.0;
    for (int i = 0; i < K; ++i) {
      const double ph = kPi * (double)((i * k) % (2 * L)) / (double)L;
      h += p->cc[i] * std::cos(ph) + p->sc[i] * std::sin(ph);
    }
    h *= s * std::exp(-alpha * (double)k);
    const double u = (double)(k + p->n0), G = norm * std::exp(-gamma * u * u);
    const double t = p->deriv == 1 ? -2.0 * gamma * u * G : (4.0 * gamma * gamma * u * u - 2.0 * gamma) * G;
    num += (h - t) * (h - t);
    den += t * t;
  }
  p->relrmse = den > 0.0 ? std::sqrt(num / den) : 0.0;
}

morlet_status morlet_plan_gauss_deriv(morlet_plan_t* out, int64_t N, double sigma, int32_t K, int64_t L,
                                      int32_t order) {
  if (!out) return fail(MORLET_ERR_INVALID_ARG, "null output handle");
  if (order != 1 && order != 2) return fail(MORLET_ERR_INVALID_ARG, "order must be 1 or 2");
  morlet_status s = check_common(N, sigma, K, L);
  if (s != MORLET_OK) return s;
  if (L != 0 && (order == 1 ? L < K : L + 1 < K))
    return fail(MORLET_ERR_INVALID_ARG, order == 1 ? "L must be >= K" : "L must be >= K - 1");
  auto* p = new (std::nothrow) morlet_plan_s;
  if (!p) return fail(MORLET_ERR_ALLOC, "out of host memory");
  p->kind = 1;
  p->deriv = order;
  p->N = N;
  p->sigma = sigma;
  p->xi = 0.0;
  p->K = K;
  // L = 0: the window of the Gaussian fit with the same top order (orders 0..K for the first
  // differential's sines 1..K, 0..K-1 for the second's cosines)
  p->L = L ? L : mk::select_L(sigma, 0.0, order == 1 ? K + 1 : K, true);
  fit_deriv(p);
  return finish_plan(p, out);
}

morlet_status morlet_plan_multiply(morlet_plan_t* out, int64_t N, double sigma, double xi, int32_t P_M, int64_t L) {
  if (!out) return fail(MORLET_ERR_INVALID_ARG, "null output handle");
  if (P_M < 0 || P_M + 1 > MORLET_MAX_TERMS) return fail(MORLET_ERR_INVALID_ARG, "P_M must be in [0, MORLET_MAX_TERMS - 1]");
  const int K = P_M + 1;
  morlet_status s = check_common(N, sigma, K, L);
  if (s != MORLET_OK) return s;
  if (N > ((int64_t)1 << 38)) return fail(MORLET_ERR_INVALID_ARG, "N must be <= 2^38 for the multiplication method");
  if (!finite_pos(xi)) return fail(MORLET_ERR_INVALID_ARG, "xi must be finite and > 0");
  if (L != 0 && L + 1 < K) return fail(MORLET_ERR_INVALID_ARG, "L must be >= P_M");
  auto* p = new (std::nothrow) morlet_plan_s;
  if (!p) return fail(MORLET_ERR_ALLOC, "out of host memory");
  p->multiply = true;
  p->mult_N = N;
  p->xi = xi;
  // the scan runs in Gaussian form over three rows (Re u, Im u, x)
  s = init_gauss_rows(p, 3, N, sigma, K, L);
  if (s != MORLET_OK) {
    morlet_destroy(p);
    return s;
  }
  const double xi0 = xi * sigma, gamma = 1.0 / (2.0 * sigma * sigma), kPi = 3.14159265358979323846;
  const double C = 1.0 / std::sqrt(1.0 + std::exp(-xi0 * xi0) - 2.0 * std::exp(-0.75 * xi0 * xi0));
  p->mult_kappa = std::exp(-0.5 * xi0 * xi0);
  p->mult_ce = C / (std::pow(kPi, 0.25) * std::sqrt(sigma)) / std::sqrt(gamma / kPi);
  // error of psi_hat_M[k] = ce (e^{i xi k} - kappa) G_hat[k] against the wavelet on [-L, L]
  {
    std::vector<double> re, im;
    mk::morlet_taps(sigma, xi, p->L, re, im);
    double num = 0.0, den = 0.0;
    for (int64_t k = -p->L; k <= p->L; ++k) {
      double gh = 0.0;
      for (int i = 0; i < K; ++i) gh += p->cc[i] * std::cos(kPi * (double)((i * k) % (2 * p->L)) / (double)p->L);
      const double hr = p->mult_ce * (std::cos(xi * (double)k) - p->mult_kappa) * gh;
      const double hi = p->mult_ce * std::sin(xi * (double)k) * gh;
      const double dr = hr - re[p->L + k], di = hi - im[p->L + k];
      num += dr * dr + di * di;
      den += re[p->L + k] * re[p->L + k] + im[p->L + k] * im[p->L + k];
    }
    p->relrmse = den > 0.0 ? std::sqrt(num / den) : 0.0;
  }
  *out = p;
  return MORLET_OK;
}

morlet_status morlet_plan_gauss2d(morlet_plan_t* out, int64_t H, int64_t W, double sigma_y, double sigma_x,
                                  int32_t K, int64_t L_y, int64_t L_x) {
  if (!out) return fail(MORLET_ERR_INVALID_ARG, "null output handle");
  if (H < 0 || W < 0 || H > ((int64_t)1 << 24) || W > ((int64_t)1 << 24) || H * W > ((int64_t)1 << 36))
    return fail(MORLET_ERR_INVALID_ARG, "H, W must be in [0, 2^24] with H W <= 2^36");
  morlet_status s = check_common(W, sigma_x, K, L_x);
  if (s == MORLET_OK) s = check_common(H, sigma_y, K, L_y);
  if (s != MORLET_OK) return s;
  if ((L_x != 0 && L_x + 1 < K) || (L_y != 0 && L_y + 1 < K)) return fail(MORLET_ERR_INVALID_ARG, "L must be >= K - 1");
  auto* p = new (std::nothrow) morlet_plan_s;
  auto* ax = new (std::nothrow) morlet_plan_s;
  auto* ay = new (std::nothrow) morlet_plan_s;
  if (!p || !ax || !ay) {
    delete p;
    delete ax;
    delete ay;
    return fail(MORLET_ERR_ALLOC, "out of host memory");
  }
  p->kind = 1;
  p->image2d = true;
  p->img_H = H;
  p->img_W = W;
  p->K = K;
  p->N = H * W;
  p->axis[0] = ax;
  p->axis[1] = ay;
  // an empty image has no lines to filter on either axis
  const bool empty = H == 0 || W == 0;
  s = init_gauss_rows(ax, empty ? 0 : (int)H, W, sigma_x, K, L_x);
  if (s == MORLET_OK) s = init_gauss_rows(ay, empty ? 0 : (int)W, H, sigma_y, K, L_y);
  if (s != MORLET_OK) {
    morlet_destroy(p);
    return s;
  }
  *out = p;
  return MORLET_OK;
}

morlet_status gauss_smooth2d(morlet_plan_t plan, const void* x, morlet_dtype dtype, float* y, void* ws,
                             size_t ws_bytes, void* stream) {
  if (!plan || !plan->image2d || plan->gabor)
    return fail(MORLET_ERR_INVALID_ARG, "gauss_smooth2d needs a Gaussian image plan");
  return run_image2d(plan, x, (int)dtype, y, ws, ws_bytes, stream);
}

morlet_status gauss_smooth2d_backward(morlet_plan_t plan, const float* gy, float* gx, void* ws, size_t ws_bytes,
                                      void* stream) {
  if (!plan || !plan->image2d) return fail(MORLET_ERR_INVALID_ARG, "gauss_smooth2d_backward needs an image plan");
  if (plan->gabor) return fail(MORLET_ERR_INVALID_ARG, "a Gabor image plan runs with gabor2d_backward");
  return run_image2d_backward(plan, gy, gx, ws, ws_bytes, stream);
}

morlet_status morlet_plan_gabor2d(morlet_plan_t* out, int64_t H, int64_t W, double sigma_x, double xi, int32_t K_x,
                                  int64_t L_x, double sigma_y, int32_t K_y, int64_t L_y) {
  if (!out) return fail(MORLET_ERR_INVALID_ARG, "null output handle");
  if (H < 0 || W < 0 || H > ((int64_t)1 << 24) || W > ((int64_t)1 << 24) || H * W > ((int64_t)1 << 35))
    return fail(MORLET_ERR_INVALID_ARG, "H, W must be in [0, 2^24] with H W <= 2^35");
  morlet_status s = check_common(W, sigma_x, K_x, L_x);
  if (s == MORLET_OK) s = check_common(H, sigma_y, K_y, L_y);
  if (s != MORLET_OK) return s;
  if (!finite_pos(xi)) return fail(MORLET_ERR_INVALID_ARG, "xi must be finite and > 0");
  if (L_x != 0 && L_x < K_x) return fail(MORLET_ERR_INVALID_ARG, "L_x must be >= K_x");
  if (L_y != 0 && L_y + 1 < K_y) return fail(MORLET_ERR_INVALID_ARG, "L_y must be >= K_y - 1");
  auto* p = new (std::nothrow) morlet_plan_s;
  auto* ax = new (std::nothrow) morlet_plan_s;
  auto* ay = new (std::nothrow) morlet_plan_s;
  if (!p || !ax || !ay) {
    delete p;
    delete ax;
    delete ay;
    return fail(MORLET_ERR_ALLOC, "out of host memory");
  }
  p->kind = 0;
  p->image2d = true;
  p->gabor = true;
  p->img_H = H;
  p->img_W = W;
  p->K = std::max(K_x, K_y);
  p->N = H * W;
  p->axis[0] = ax;
  p->axis[1] = ay;
  const bool empty = H == 0 || W == 0;
  s = init_morlet_rows(ax, empty ? 0 : (int)H, W, sigma_x, xi, K_x, L_x);
  if (s == MORLET_OK) s = init_gauss_rows(ay, empty ? 0 : (int)(2 * W), H, sigma_y, K_y, L_y);
  if (s != MORLET_OK) {
    morlet_destroy(p);
    return s;
  }
  *out = p;
  return MORLET_OK;
}

morlet_status gabor2d(morlet_plan_t plan, const void* x, morlet_dtype dtype, void* y, void* ws, size_t ws_bytes,
                      void* stream) {
  if (!plan || !plan->image2d || !plan->gabor) return fail(MORLET_ERR_INVALID_ARG, "gabor2d needs a Gabor image plan");
  return run_gabor2d(plan, x, (int)dtype, y, ws, ws_bytes, stream);
}

morlet_status gauss_smooth2d_grad(morlet_plan_t plan, const void* x, morlet_dtype dtype, const float* gy, float* gx,
                                  double* gparams, void* ws, size_t ws_bytes, void* stream) {
  if (!plan || !plan->image2d || plan->gabor)
    return fail(MORLET_ERR_INVALID_ARG, "gauss_smooth2d_grad needs a Gaussian image plan");
  return run_image2d_grad(plan, x, (int)dtype, gy, gx, gparams, ws, ws_bytes, stream);
}

morlet_status gabor2d_grad(morlet_plan_t plan, const void* x, morlet_dtype dtype, const void* gW, float* gx,
                           double* gparams, void* ws, size_t ws_bytes, void* stream) {
  if (!plan || !plan->image2d || !plan->gabor)
    return fail(MORLET_ERR_INVALID_ARG, "gabor2d_grad needs a Gabor image plan");
  return run_gabor2d_grad(plan, x, (int)dtype, gW, gx, gparams, ws, ws_bytes, stream);
}

morlet_status gabor2d_backward(morlet_plan_t plan, const void* gW, float* gx, void* ws, size_t ws_bytes, void* stream) {
  if (!plan || !plan->image2d || !plan->gabor)
    return fail(MORLET_ERR_INVALID_ARG, "gabor2d_backward needs a Gabor image plan");
  return run_gabor2d_backward(plan, gW, gx, ws, ws_bytes, stream);
}

morlet_status morlet_image_axis_info(morlet_plan_t plan, int32_t axis, int64_t* L, int64_t* n0, double* cos_coef,
                                     double* kernel_relrmse) {
  if (!plan || !plan->image2d) return fail(MORLET_ERR_INVALID_ARG, "needs an image plan");
  if (axis != 0 && axis != 1) return fail(MORLET_ERR_INVALID_ARG, "axis must be 0 (x, along rows) or 1 (y)");
  const morlet_plan_s* a = plan->axis[axis];
  const ScaleParams& sp = a->scales[0];
  if (L) *L = sp.L;
  if (n0) *n0 = a->mode == 1 ? sp.n0_asft : 0;
  if (cos_coef) std::memcpy(cos_coef, sp.cc.data(), sizeof(double) * a->K);
  if (kernel_relrmse) *kernel_relrmse = sp.relrmse;
  return MORLET_OK;
}

morlet_status morlet_plan_set(morlet_plan_t plan, morlet_scan mode, int64_t n0, morlet_accum accum) {
  if (!plan) return fail(MORLET_ERR_INVALID_ARG, "null plan");
  if (plan->image2d) {
    morlet_status st = morlet_plan_set(plan->axis[0], mode, n0, accum);
    if (st == MORLET_OK) st = morlet_plan_set(plan->axis[1], mode, n0, accum);
    if (st == MORLET_OK) {
      plan->mode = (int)mode;
      plan->accum = (int)accum;
    }
    return st;
  }
  if (mode != MORLET_SCAN_SFT && mode != MORLET_SCAN_ASFT) return fail(MORLET_ERR_UNSUPPORTED, "unknown scan mode");
  if (accum != MORLET_ACC_F32 && accum != MORLET_ACC_F64 && accum != MORLET_ACC_MIXED && accum != MORLET_ACC_AUTO &&
      accum != MORLET_ACC_KAHAN)
    return fail(MORLET_ERR_UNSUPPORTED, "unknown accumulation mode");
  if (accum == MORLET_ACC_KAHAN && (plan->deriv != 0 || plan->R != 16))
    return fail(MORLET_ERR_UNSUPPORTED, "the compensated scan takes Morlet and Gaussian smoothing plans at R = 16");
  if (n0 < 0 || (!plan->batched && n0 > plan->L))
    return fail(MORLET_ERR_INVALID_ARG, "n0 must be 0 (default) or in [1, L]");
  plan->mode = (int)mode;
  plan->accum = (int)accum;
  if (plan->batched) {
    for (ScaleParams& sp : plan->scales)
      sp.n0_asft = n0 > 0 ? std::min<int64_t>(n0, sp.L) : default_n0(sp.sigma, sp.L);
    build_rows(plan);
    build_batched_tables(plan);
    if (plan->d_tab) return upload_batched(plan);
    return MORLET_OK;
  }
  if (n0 > 0) plan->n0_asft = n0;
  plan->n0 = (mode == MORLET_SCAN_ASFT) ? plan->n0_asft : 0;
  if (plan->deriv != 0) fit_deriv(plan);   // the term set and weights follow the mode
  std::string err;
  mk::build_table(plan, &err);
  if (plan->d_tab) return upload_table(plan);
  return MORLET_OK;
}

morlet_status morlet_plan_set_boundary(morlet_plan_t plan, morlet_boundary boundary) {
  if (!plan) return fail(MORLET_ERR_INVALID_ARG, "null plan");
  if (boundary != MORLET_BOUNDARY_ZERO && boundary != MORLET_BOUNDARY_EDGE)
    return fail(MORLET_ERR_INVALID_ARG, "unknown boundary");
  if (plan->batched || plan->multiply || plan->image2d)
    return fail(MORLET_ERR_UNSUPPORTED, "edge extension is built for single-signal plans");
  plan->boundary = (int)boundary;
  return MORLET_OK;
}

morlet_status morlet_plan_set_schedule(morlet_plan_t plan, morlet_schedule schedule) {
  if (!plan) return fail(MORLET_ERR_INVALID_ARG, "null plan");
  if (plan->image2d) {
    const morlet_status st = morlet_plan_set_schedule(plan->axis[0], schedule);
    return st == MORLET_OK ? morlet_plan_set_schedule(plan->axis[1], schedule) : st;
  }
  switch (schedule) {
    case MORLET_SCHED_AUTO: plan->row_serial = -1; return MORLET_OK;
    case MORLET_SCHED_TILES: plan->row_serial = 0; return MORLET_OK;
    case MORLET_SCHED_ROWS: plan->row_serial = 1; return MORLET_OK;
    case MORLET_SCHED_SEGMENTS: plan->row_serial = 2; return MORLET_OK;
  }
  return fail(MORLET_ERR_INVALID_ARG, "unknown schedule");
}

morlet_status morlet_plan_set_segments(morlet_plan_t plan, int32_t tiles_per_segment) {
  if (!plan) return fail(MORLET_ERR_INVALID_ARG, "null plan");
  if (tiles_per_segment < 0 || tiles_per_segment > mk::kLookback * mk::kLookback)
    return fail(MORLET_ERR_INVALID_ARG, "tiles per segment must be in [0, 4096]");
  if (plan->image2d) {
    plan->axis[0]->seg_tiles = tiles_per_segment;
    plan->axis[1]->seg_tiles = tiles_per_segment;
  }
  plan->seg_tiles = tiles_per_segment;
  return MORLET_OK;
}

morlet_status morlet_plan_set_tile(morlet_plan_t plan, int32_t R) {
  if (!plan) return fail(MORLET_ERR_INVALID_ARG, "null plan");
  if (plan->image2d) {
    // both axes or neither: a shape the second axis cannot take restores the first
    const int oldR = plan->axis[0]->R;
    morlet_status st = morlet_plan_set_tile(plan->axis[0], R);
    if (st == MORLET_OK) {
      st = morlet_plan_set_tile(plan->axis[1], R);
      if (st != MORLET_OK) (void)morlet_plan_set_tile(plan->axis[0], oldR);
    }
    if (st == MORLET_OK) plan->R = R;
    return st;
  }
  if (R != 4 && R != 8 && R != 16 && R != 32) return fail(MORLET_ERR_UNSUPPORTED, "R must be 4, 8, 16 or 32");
  if (plan->accum == MORLET_ACC_KAHAN && R != 16)
    return fail(MORLET_ERR_UNSUPPORTED, "the compensated scan is built for R = 16 only");
  if (R == plan->R) return MORLET_OK;
  const int oldR = plan->R;
  plan->R = R;
  if (plan->batched) {
    build_rows(plan);
    if (plan->ntiles > ((int64_t)1 << 31)) {
      plan->R = oldR;
      build_rows(plan);
      return fail(MORLET_ERR_UNSUPPORTED, "too many tiles");
    }
    build_batched_tables(plan);
    if (plan->d_tab) {
      // the table size depends on R: reallocate
      (void)hipFree(plan->d_tab);
      plan->d_tab = nullptr;
      return upload_batched(plan);
    }
    return MORLET_OK;
  }
  std::string err;
  mk::build_table(plan, &err);
  if (plan->d_tab) {
    (void)hipFree(plan->d_tab);
    plan->d_tab = nullptr;
    return upload_table(plan);
  }
  return MORLET_OK;
}

morlet_status morlet_plan_info(morlet_plan_t plan, int64_t* L, int32_t* P_S, int64_t* n0, double* alpha,
                               double* cos_coef, double* sin_coef, double* jac, double* kernel_relrmse) {
  if (!plan) return fail(MORLET_ERR_INVALID_ARG, "null plan");
  if (plan->batched && !plan->multiply)
    return fail(MORLET_ERR_INVALID_ARG, "use morlet_scalogram_scale_info for a scalogram plan");
  if (plan->image2d) return fail(MORLET_ERR_INVALID_ARG, "use morlet_image_axis_info for an image plan");
  // a multiplication-method plan keeps its shift with its one scale
  const int64_t n0v = plan->multiply ? (plan->mode == 1 ? plan->scales[0].n0_asft : 0) : plan->n0;
  if (L) *L = plan->L;
  if (P_S) *P_S = plan->P_S;
  if (n0) *n0 = n0v;
  if (alpha) *alpha = plan->mode == 1 ? (double)n0v / (plan->sigma * plan->sigma) : 0.0;
  if (cos_coef) std::memcpy(cos_coef, plan->cc.data(), sizeof(double) * plan->K);
  if (sin_coef) std::memcpy(sin_coef, plan->sc.data(), sizeof(double) * plan->K);
  if (jac) std::memcpy(jac, plan->jac.data(), sizeof(double) * 4 * plan->K);
  if (kernel_relrmse) *kernel_relrmse = plan->relrmse;
  return MORLET_OK;
}

// the schedule of a plan's row_serial value (-1 automatic, 0 tiles, 1 rows, 2 segments)
int32_t sched_of(int rows) {
  return rows == 1 ? MORLET_SCHED_ROWS : rows == 2 ? MORLET_SCHED_SEGMENTS : rows == 0 ? MORLET_SCHED_TILES : MORLET_SCHED_AUTO;
}

morlet_status morlet_plan_autotune(morlet_plan_t plan, const void* x, morlet_dtype dtype, void* out, int32_t reps,
                                   int32_t* R_out, int32_t* schedule_out, void* stream) {
  if (!plan) return fail(MORLET_ERR_INVALID_ARG, "null plan");
  if (plan->image2d) return fail(MORLET_ERR_UNSUPPORTED, "autotune does not take image plans");
  if (reps < 1 || reps > 1000) return fail(MORLET_ERR_INVALID_ARG, "reps must be in [1, 1000]");
  if ((int)dtype < 0 || (int)dtype > 2) return fail(MORLET_ERR_UNSUPPORTED, "unknown dtype");
  if (!plan->d_tab) return fail(MORLET_ERR_HIP, "plan has no device table (created without a HIP device)");
  const std::string key = tune_key(plan, (int)dtype);
  {
    int cR = 0, cRows = 0;
    if (tune_lookup(key, cR, cRows)) {
      const int R0 = plan->R;
      morlet_status st = morlet_plan_set_tile(plan, cR);
      if (st == MORLET_OK) {
        plan->row_serial = cRows;
        if (R_out) *R_out = cR;
        if (schedule_out) *schedule_out = sched_of(cRows);
        if (log_on()) std::fprintf(stderr, "morlet: autotune cache hit %s -> R=%d rows=%d\n", key.c_str(), cR, cRows);
        return MORLET_OK;
      }
      (void)morlet_plan_set_tile(plan, R0);   // a stale entry: tune again
    }
  }
  const int oldR = plan->R, oldSched = plan->row_serial;
  // schedules: tiles, whole rows (several rows), segments (at most eight rows)
  const size_t nrows = plan->batched ? plan->rows.size() : 1;
  struct Cand { int R, rows; };
  std::vector<Cand> cands;
  // one workspace serves every candidate: the largest of their sizes. A tile shape the plan
  // cannot take (too many tiles for a batched plan) is left out; ties go to the earlier
  // candidate, so the default shape comes first.
  size_t need = 0;
  for (int R : {16, 32, 8, 4}) {
    morlet_status st = morlet_plan_set_tile(plan, R);
    size_t b = 0;
    if (st == MORLET_ERR_UNSUPPORTED) continue;
    if (st == MORLET_OK) st = morlet_workspace_size(plan, &b);
    if (st != MORLET_OK) {
      (void)morlet_plan_set_tile(plan, oldR);
      return st;
    }
    need = std::max(need, b);
    cands.push_back({R, 0});
    if (nrows > 1) cands.push_back({R, 1});
    if (nrows <= (size_t)mk::kQueues) cands.push_back({R, 2});
  }
  if (cands.empty()) {
    (void)morlet_plan_set_tile(plan, oldR);
    return fail(MORLET_ERR_UNSUPPORTED, "autotune: no tile shape fits this plan");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  void* ws = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipMalloc(&ws, need) != hipSuccess || hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipGetLastError();
    if (ws) (void)hipFree(ws);
    if (e0) (void)hipEventDestroy(e0);
    (void)morlet_plan_set_tile(plan, oldR);
    return fail(MORLET_ERR_ALLOC, "autotune: workspace or event allocation failed");
  }
  morlet_status st = MORLET_OK;
  size_t best = 0;
  float best_ms = 0.f;
  for (size_t c = 0; c < cands.size() && st == MORLET_OK; ++c) {
    st = morlet_plan_set_tile(plan, cands[c].R);
    plan->row_serial = cands[c].rows;
    if (st == MORLET_OK) st = morlet_workspace_init(ws, need, stream);
    auto trial = [&]() {
      return plan->multiply ? run_multiply(plan, x, (int)dtype, out, ws, need, stream)
                            : run_scan(plan, x, (int)dtype, out, ws, need, stream, plan->kind, plan->batched);
    };
    if (st == MORLET_OK) st = trial();
    if (st != MORLET_OK) break;
    if (hipEventRecord(e0, s) != hipSuccess) { st = fail(MORLET_ERR_HIP, "autotune: event record failed"); break; }
    for (int r = 0; r < reps && st == MORLET_OK; ++r) st = trial();
    float ms = 0.f;
    if (st == MORLET_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      st = fail(MORLET_ERR_HIP, "autotune: event timing failed");
    if (st == MORLET_OK && (c == 0 || ms < best_ms)) {
      best_ms = ms;
      best = c;
    }
  }
  (void)hipStreamSynchronize(s);
  (void)hipFree(ws);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != MORLET_OK) {
    (void)morlet_plan_set_tile(plan, oldR);
    plan->row_serial = oldSched;
    return st;
  }
  st = morlet_plan_set_tile(plan, cands[best].R);
  plan->row_serial = cands[best].rows;
  if (st == MORLET_OK) {
    tune_store(key, cands[best].R, cands[best].rows, best_ms / (float)reps);
    if (log_on())
      std::fprintf(stderr, "morlet: autotune %s -> R=%d rows=%d (%.4f ms)\n", key.c_str(), cands[best].R,
                   cands[best].rows, best_ms / (float)reps);
  }
  if (R_out) *R_out = cands[best].R;
  if (schedule_out) *schedule_out = sched_of(cands[best].rows);
  return st;
}

morlet_status morlet_workspace_size(morlet_plan_t plan, size_t* bytes) {
  if (!plan || !bytes) return fail(MORLET_ERR_INVALID_ARG, "null plan or output");
  // sized for the longest scan range over every n0 the plan may use (n0 = 0)
  if (plan->image2d) {
    *bytes = plan->gabor ? gabor_layout(plan).total : image_layout(plan).total;
    return MORLET_OK;
  }
  if (plan->boundary == 1) {
    *bytes = edge_layout(plan).total;
    return MORLET_OK;
  }
  *bytes = plan->multiply ? mult_layout(plan).total
                          : mk::workspace_bytes(plan->K, plan->batched ? plan->ntiles_max : tiles_for(plan->N + plan->L, plan->R));
  return MORLET_OK;
}

morlet_status morlet_workspace_init(void* ws, size_t ws_bytes, void* stream) {
  if (!ws && ws_bytes) return fail(MORLET_ERR_INVALID_ARG, "null workspace");
  const hipError_t e = mk::launch_zero_fill(ws, ws_bytes, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  return MORLET_OK;
}

morlet_status morlet_forward(morlet_plan_t plan, const void* x, morlet_dtype dtype, void* W, void* ws,
                             size_t ws_bytes, void* stream) {
  if (plan && plan->multiply) return run_multiply(plan, x, (int)dtype, W, ws, ws_bytes, stream);
  return run_scan(plan, x, (int)dtype, W, ws, ws_bytes, stream, 0, false);
}

morlet_status gauss_smooth(morlet_plan_t plan, const void* x, morlet_dtype dtype, float* y, void* ws,
                           size_t ws_bytes, void* stream) {
  return run_scan(plan, x, (int)dtype, y, ws, ws_bytes, stream, 1, false);
}

morlet_status morlet_scalogram_plan(morlet_plan_t* out, int32_t B, const int64_t* lengths, int32_t S,
                                    const double* sigmas, const double* xis, int32_t K, double L_over_sigma) {
  if (!out) return fail(MORLET_ERR_INVALID_ARG, "null output handle");
  if (B < 1 || S < 1) return fail(MORLET_ERR_INVALID_ARG, "B and S must be >= 1");
  if (!lengths || !sigmas || !xis) return fail(MORLET_ERR_INVALID_ARG, "null lengths, sigmas or xis");
  if (K < 1 || K > MORLET_MAX_TERMS) return fail(MORLET_ERR_INVALID_ARG, "K must be in [1, MORLET_MAX_TERMS]");
  if (!(L_over_sigma >= 0.0) || !std::isfinite(L_over_sigma))
    return fail(MORLET_ERR_INVALID_ARG, "L_over_sigma must be 0 or a finite positive ratio");
  int64_t total = 0;
  for (int b = 0; b < B; ++b) {
    if (lengths[b] < 0 || lengths[b] > ((int64_t)1 << 40)) return fail(MORLET_ERR_INVALID_ARG, "bad signal length");
    total += lengths[b];
  }
  for (int s = 0; s < S; ++s) {
    if (!finite_pos(sigmas[s]) || !finite_pos(xis[s])) return fail(MORLET_ERR_INVALID_ARG, "bad sigma or xi");
    if (L_over_sigma > 0 && std::ceil(L_over_sigma * sigmas[s]) > (double)((int64_t)1 << 30))
      return fail(MORLET_ERR_INVALID_ARG, "window too large");
  }
  auto* p = new (std::nothrow) morlet_plan_s;
  if (!p) return fail(MORLET_ERR_ALLOC, "out of host memory");
  p->kind = 0;
  p->batched = true;
  p->B = B;
  p->S = S;
  p->K = K;
  p->N = total;
  p->R = 16;
  p->lengths.assign(lengths, lengths + B);
  p->offsets.resize(B);
  int64_t off = 0;
  for (int b = 0; b < B; ++b) { p->offsets[b] = off; off += lengths[b]; }
  p->scales.resize(S);
  bool bad = false;
  auto work = [&](int s) {
    ScaleParams& sp = p->scales[s];
    sp.sigma = sigmas[s];
    sp.xi = xis[s];
    sp.L = L_over_sigma > 0 ? (int64_t)std::ceil(L_over_sigma * sp.sigma) : mk::select_L(sp.sigma, sp.xi, K, false);
    if (sp.L < K) sp.L = K;
    sp.P_S = mk::select_ps(sp.sigma, sp.xi, K, sp.L, nullptr);
    std::vector<double> re, im;
    mk::morlet_taps(sp.sigma, sp.xi, sp.L, re, im);
    const mk::Fit f = mk::fit_orders(re, im, sp.L, sp.P_S, K);
    sp.cc = f.cc;
    sp.sc = f.sc;
    sp.relrmse = f.relrmse;
    morlet_plan_s tmp;
    tmp.kind = 0; tmp.sigma = sp.sigma; tmp.xi = sp.xi; tmp.K = K; tmp.L = sp.L; tmp.P_S = sp.P_S;
    mk::jacobian(&tmp);
    sp.jac = tmp.jac;
    sp.n0_asft = default_n0(sp.sigma, sp.L);
    if (!std::isfinite(sp.relrmse)) bad = true;
  };
  {
    const int nth = (int)std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t)
      th.emplace_back([&, t] { for (int s = t; s < S; s += nth) work(s); });
    for (auto& t : th) t.join();
  }
  if (bad) {
    delete p;
    return fail(MORLET_ERR_INVALID_ARG, "fit failed for some scale");
  }
  build_rows(p);
  if (p->ntiles > ((int64_t)1 << 31)) {
    delete p;
    return fail(MORLET_ERR_UNSUPPORTED, "too many tiles");
  }
  build_batched_tables(p);
  const morlet_status s = upload_batched(p);
  if (s != MORLET_OK) {
    morlet_destroy(p);
    return s;
  }
  if (log_on()) {
    std::fprintf(stderr, "morlet: scalogram B=%d S=%d K=%d rows=%zu tiles=%lld\n", p->B, p->S, p->K, p->rows.size(),
                 (long long)p->ntiles);
    for (int q = 0; q < p->S; ++q)
      std::fprintf(stderr, "morlet:   scale %d sigma=%.6g xi=%.6g L=%lld P_S=%d relrmse=%.3e\n", q, p->scales[q].sigma,
                   p->scales[q].xi, (long long)p->scales[q].L, p->scales[q].P_S, p->scales[q].relrmse);
  }
  *out = p;
  return MORLET_OK;
}

morlet_status morlet_scalogram_scale_info(morlet_plan_t plan, int32_t s, int64_t* L, int32_t* P_S, int64_t* n0,
                                          double* alpha, double* cos_coef, double* sin_coef, double* jac,
                                          double* kernel_relrmse) {
  if (!plan || !plan->batched) return fail(MORLET_ERR_INVALID_ARG, "needs a scalogram plan");
  if (s < 0 || s >= plan->S) return fail(MORLET_ERR_INVALID_ARG, "scale index out of range");
  const ScaleParams& sp = plan->scales[s];
  const int64_t n0v = plan->mode == 1 ? sp.n0_asft : 0;
  if (L) *L = sp.L;
  if (P_S) *P_S = sp.P_S;
  if (n0) *n0 = n0v;
  if (alpha) *alpha = (double)n0v / (sp.sigma * sp.sigma);
  if (cos_coef) std::memcpy(cos_coef, sp.cc.data(), sizeof(double) * plan->K);
  if (sin_coef) std::memcpy(sin_coef, sp.sc.data(), sizeof(double) * plan->K);
  if (jac) std::memcpy(jac, sp.jac.data(), sizeof(double) * 4 * plan->K);
  if (kernel_relrmse) *kernel_relrmse = sp.relrmse;
  return MORLET_OK;
}

morlet_status morlet_scalogram_forward(morlet_plan_t plan, const void* x_packed, morlet_dtype dtype,
                                       void* W_packed, void* ws, size_t ws_bytes, void* stream) {
  return run_scan(plan, x_packed, (int)dtype, W_packed, ws, ws_bytes, stream, 0, true);
}

morlet_status morlet_plan_refit(morlet_plan_t plan, double sigma, double xi, void* stream) {
  if (!plan) return fail(MORLET_ERR_INVALID_ARG, "null plan");
  if (plan->batched || plan->image2d || plan->multiply || plan->deriv != 0)
    return fail(MORLET_ERR_UNSUPPORTED, "refit takes single-signal Morlet and Gaussian smoothing plans");
  if (!finite_pos(sigma)) return fail(MORLET_ERR_INVALID_ARG, "sigma must be finite and > 0");
  if (plan->kind == 0 && !finite_pos(xi)) return fail(MORLET_ERR_INVALID_ARG, "xi must be finite and > 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the previous refit's upload must have left the staging buffer before it is rewritten
  if (plan->stage_event && hipEventSynchronize(static_cast<hipEvent_t>(plan->stage_event)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(MORLET_ERR_HIP, "waiting for the previous table upload failed");
  }
  plan->sigma = sigma;
  std::vector<double> re, im;
  if (plan->kind == 0) {
    plan->xi = xi;
    mk::morlet_taps(sigma, xi, plan->L, re, im);
  } else {
    mk::gauss_taps(sigma, plan->L, re);
  }
  const mk::Fit f = mk::fit_orders(re, im, plan->L, plan->P_S, plan->K);
  plan->cc = f.cc;
  plan->sc = f.sc;
  plan->relrmse = f.relrmse;
  mk::jacobian(plan);
  plan->direct_H = -1;   // the direct-convolution baseline's taps follow sigma and xi
  std::string err;
  mk::build_table(plan, &err);
  if (!plan->d_tab) return MORLET_OK;   // no HIP device: host-side plan only
  if (plan->h_tab.size() != plan->tab_bytes) return fail(MORLET_ERR_HIP, "table size changed");
  if (plan->h_stage && plan->stage_bytes != plan->tab_bytes) {   // the tile shape changed the table
    (void)hipHostFree(plan->h_stage);
    plan->h_stage = nullptr;
  }
  if (!plan->h_stage) {
    if (hipHostMalloc(&plan->h_stage, plan->tab_bytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      plan->h_stage = nullptr;
      return fail(MORLET_ERR_ALLOC, "hipHostMalloc of the staging table failed");
    }
    plan->stage_bytes = plan->tab_bytes;
  }
  if (!plan->stage_event) {
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      return fail(MORLET_ERR_HIP, "hipEventCreate failed");
    }
    plan->stage_event = ev;
  }
  std::memcpy(plan->h_stage, plan->h_tab.data(), plan->tab_bytes);
  hipError_t e = hipMemcpyAsync(plan->d_tab, plan->h_stage, plan->tab_bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(static_cast<hipEvent_t>(plan->stage_event), s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(MORLET_ERR_HIP, std::string("table upload failed: ") + hipGetErrorString(e));
  }
  return MORLET_OK;
}

void morlet_destroy(morlet_plan_t plan) {
  if (!plan) return;
  morlet_destroy(plan->axis[0]);
  morlet_destroy(plan->axis[1]);
  if (plan->stage_event) {
    (void)hipEventSynchronize(static_cast<hipEvent_t>(plan->stage_event));
    (void)hipEventDestroy(static_cast<hipEvent_t>(plan->stage_event));
  }
  if (plan->h_stage) (void)hipHostFree(plan->h_stage);
  if (plan->d_tab) (void)hipFree(plan->d_tab);
  if (plan->d_rows) (void)hipFree(plan->d_rows);
  if (plan->d_direct) (void)hipFree(plan->d_direct);
  delete plan;
}

// ---------------------------------------------------------------- forward without allocation
// The scan's workspace taken from the library's fixed device array (noalloc.hip): for callers
// that cannot allocate. Only plans whose forward needs nothing but the scan's workspace.
morlet_status morlet_forward_noalloc(morlet_plan_t plan, const void* x, morlet_dtype dtype, void* W, void* stream) {
  if (!plan) return fail(MORLET_ERR_INVALID_ARG, "null plan");
  if (plan->image2d || plan->multiply || plan->boundary == 1)
    return fail(MORLET_ERR_UNSUPPORTED, "no-allocation forward: image, multiplication-method and edge-extension "
                                        "plans need more than the scan's workspace");
  if (plan->kind != 0) return fail(MORLET_ERR_INVALID_ARG, "morlet_forward_noalloc needs a Morlet plan");
  if ((int)dtype < 0 || (int)dtype > 2) return fail(MORLET_ERR_UNSUPPORTED, "unknown dtype");
  const int64_t ntiles = plan->batched ? plan->ntiles : tiles_for(plan->N + plan->L - plan->n0, plan->R);
  if (plan->N == 0 || ntiles == 0) return MORLET_OK;
  if (!x || !W) return fail(MORLET_ERR_INVALID_ARG, "null x or output pointer");
  if (ntiles > ((int64_t)1 << 31)) return fail(MORLET_ERR_UNSUPPORTED, "too many tiles");
  if (!plan->d_tab) return fail(MORLET_ERR_HIP, "plan has no device table (created without a HIP device)");
  void* ws = mk::scratch_ptr(plan->device);
  if (!ws) {
    // set-up missed at plan creation (or failed): resolve it now, on the plan's device
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != plan->device) {
      (void)hipGetLastError();
      return fail(MORLET_ERR_INVALID_ARG, "the plan's device is not the current device");
    }
    const hipError_t e = mk::scratch_setup(plan->device);
    if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("scratch set-up failed: ") + hipGetErrorString(e));
    ws = mk::scratch_ptr(plan->device);
  }
  mk::ScanLaunch a;
  morlet_status st = make_launch(plan, a, ws, mk::kVarForward, 0, (int)dtype);
  if (st != MORLET_OK) return st;
  const size_t need = launch_ws_bytes(a, plan->K, ntiles);
  if (need > mk::kScratchBytes)
    return fail(MORLET_ERR_WORKSPACE, "the launch needs " + std::to_string(need) +
                                          " bytes of workspace, more than the fixed scratch of " +
                                          std::to_string(mk::kScratchBytes) + " bytes");
  a.x = x;
  a.dtype = (int)dtype;
  a.out = W;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // every call clears what the launch reads as its start state (header and tile flags): the
  // array keeps the previous call's contents, which may come from a plan of another shape
  hipError_t e = mk::launch_zero_fill(ws, need, s);
  if (e == hipSuccess) e = mk::launch_scan(a, mk::kVarForward, 0, s);
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  return MORLET_OK;
}

morlet_status morlet_backward_workspace_size(morlet_plan_t plan, size_t* bytes) {
  if (!plan || !bytes) return fail(MORLET_ERR_INVALID_ARG, "null plan or output");
  if (plan->image2d) {
    *bytes = plan->gabor ? gabor_bwd_layout(plan).total : image_bwd_layout(plan).total;
    return MORLET_OK;
  }
  if (plan->multiply) {
    *bytes = std::max(mult_bwd_layout(plan).total, mult_layout(plan).total);
    return MORLET_OK;
  }
  if (plan->deriv != 0) {
    *bytes = deriv_bwd_layout(plan).total;
    return MORLET_OK;
  }
  *bytes = plan->boundary == 1 ? std::max(edge_bwd_layout(plan).total, edge_layout(plan).total) : bwd_layout(plan).total;
  return MORLET_OK;
}

morlet_status morlet_backward(morlet_plan_t plan, const void* x, morlet_dtype dtype, const void* gW, float* gx,
                              double* gparams, void* ws, size_t ws_bytes, void* stream) {
  return run_backward(plan, x, (int)dtype, gW, gx, gparams, ws, ws_bytes, stream, 0, false);
}

morlet_status gauss_smooth_backward(morlet_plan_t plan, const void* x, morlet_dtype dtype, const float* gy,
                                    float* gx, double* gparams, void* ws, size_t ws_bytes, void* stream) {
  return run_backward(plan, x, (int)dtype, gy, gx, gparams, ws, ws_bytes, stream, 1, false);
}

morlet_status morlet_scalogram_backward(morlet_plan_t plan, const void* x_packed, morlet_dtype dtype,
                                        const void* gW_packed, float* gx_packed, double* gparams, void* ws,
                                        size_t ws_bytes, void* stream) {
  return run_backward(plan, x_packed, (int)dtype, gW_packed, gx_packed, gparams, ws, ws_bytes, stream, 0, true);
}

static bool tree_plan_ok(morlet_plan_t plan) {
  return plan && !plan->batched && !plan->multiply && !plan->image2d && plan->deriv == 0 &&
         (plan->kind == 0 || plan->kind == 1) && plan->boundary == 0;
}

morlet_status morlet_tree_workspace_size(morlet_plan_t plan, size_t* bytes) {
  if (!bytes) return fail(MORLET_ERR_INVALID_ARG, "null output");
  if (!tree_plan_ok(plan)) return fail(MORLET_ERR_INVALID_ARG, "needs a single-signal Morlet or Gaussian smoothing plan");
  *bytes = 4 * (size_t)plan->K * (size_t)(plan->N + 2 * plan->L) * sizeof(float2);
  return MORLET_OK;
}

morlet_status morlet_tree_forward(morlet_plan_t plan, const void* x, morlet_dtype dtype, void* out, void* ws,
                                  size_t ws_bytes, void* stream) {
  if (!tree_plan_ok(plan)) return fail(MORLET_ERR_INVALID_ARG, "needs a single-signal Morlet or Gaussian smoothing plan");
  if (plan->mode != MORLET_SCAN_SFT) return fail(MORLET_ERR_UNSUPPORTED, "the sliding-sum route is the SFT form");
  if ((int)dtype < 0 || (int)dtype > 2) return fail(MORLET_ERR_UNSUPPORTED, "unknown dtype");
  if (plan->N == 0) return MORLET_OK;
  if (!x || !out || !ws) return fail(MORLET_ERR_INVALID_ARG, "null x, output or workspace pointer");
  size_t need = 0;
  (void)morlet_tree_workspace_size(plan, &need);
  if (ws_bytes < need) return fail(MORLET_ERR_WORKSPACE, "workspace too small");
  mk::TreeCoef c{};
  c.K = plan->K;
  for (int t = 0; t < plan->K; ++t) {
    c.cc[t] = plan->cc[t];
    c.sc[t] = plan->sc[t];
  }
  const hipError_t e = mk::launch_tree(x, (int)dtype, plan->N, plan->L, plan->K, plan->P_S, c, plan->kind == 1 ? 1 : 0,
                                       static_cast<float2*>(ws), out, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  return MORLET_OK;
}

morlet_status morlet_direct_forward(morlet_plan_t plan, const void* x, morlet_dtype dtype, void* W,
                                    int64_t half_width, void* stream) {
  if (!plan || plan->batched || plan->kind != 0) return fail(MORLET_ERR_INVALID_ARG, "needs a single-signal Morlet plan");
  if (plan->boundary != 0) return fail(MORLET_ERR_UNSUPPORTED, "the direct-convolution baseline extends by zeros only");
  if ((int)dtype < 0 || (int)dtype > 2) return fail(MORLET_ERR_UNSUPPORTED, "unknown dtype");
  if (half_width < 0 || half_width > ((int64_t)1 << 30)) return fail(MORLET_ERR_INVALID_ARG, "bad half width");
  if (plan->N == 0) return MORLET_OK;
  if (!x || !W) return fail(MORLET_ERR_INVALID_ARG, "null pointer");
  const int64_t H = half_width ? half_width : plan->L;
  const int slabs = mk::direct_conv_slabs(plan->N, H, plan->num_cus);
  const size_t tap_bytes = ((size_t)(2 * H + 1) * 8 + 255) / 256 * 256;
  if (plan->direct_H != H) {
    std::vector<double> re, im;
    mk::morlet_taps(plan->sigma, plan->xi, H, re, im);
    std::vector<float> h(2 * (2 * H + 1));
    for (int64_t k = 0; k < 2 * H + 1; ++k) { h[2 * k] = (float)re[k]; h[2 * k + 1] = (float)im[k]; }
    if (plan->d_direct) { (void)hipFree(plan->d_direct); plan->d_direct = nullptr; }
    plan->direct_H = -1;
    // taps, then the slab partials (slabs x N complex64) when the taps are split
    const size_t bytes = tap_bytes + (slabs > 1 ? (size_t)slabs * (size_t)plan->N * 8 : 0);
    if (hipMalloc(&plan->d_direct, bytes) != hipSuccess) {
      (void)hipGetLastError();
      plan->d_direct = nullptr;
      return fail(MORLET_ERR_ALLOC, "hipMalloc of the direct taps failed");
    }
    if (hipMemcpy(plan->d_direct, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipGetLastError();
      return fail(MORLET_ERR_HIP, "hipMemcpy of the direct taps failed");
    }
    plan->direct_H = H;
  }
  float2* part = reinterpret_cast<float2*>(static_cast<char*>(plan->d_direct) + tap_bytes);
  const hipError_t e = mk::launch_direct_conv(x, (int)dtype, plan->N, static_cast<const float2*>(plan->d_direct), H,
                                              slabs, part, static_cast<float2*>(W), static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  return MORLET_OK;
}

morlet_status morlet_inject_failure(morlet_status status, int32_t nth) {
  if (nth < 0) return fail(MORLET_ERR_INVALID_ARG, "nth must be >= 0");
  if (nth > 0 && (status == MORLET_OK || (int)status < 0 || (int)status > (int)MORLET_ERR_HIP))
    return fail(MORLET_ERR_INVALID_ARG, "status must be one of the MORLET_ERR_ codes");
  g_inject_status.store((int)status, std::memory_order_relaxed);
  g_inject_after.store(nth, std::memory_order_relaxed);
  return MORLET_OK;
}

static morlet_status choose_terms(double sigma, double xi, bool gauss, double target, int32_t* K, int64_t* L,
                                  double* relrmse) {
  if (!finite_pos(sigma) || (!gauss && !finite_pos(xi))) return fail(MORLET_ERR_INVALID_ARG, "sigma and xi must be finite and > 0");
  if (!finite_pos(target)) return fail(MORLET_ERR_INVALID_ARG, "target must be finite and > 0");
  if (!K || !L || !relrmse) return fail(MORLET_ERR_INVALID_ARG, "null output");
  int bestK = 0;
  int64_t bestL = 0;
  double best = std::numeric_limits<double>::infinity();
  for (int k = 1; k <= MORLET_MAX_TERMS; ++k) {
    const int64_t l = mk::select_L(sigma, gauss ? 0.0 : xi, k, gauss);
    const double e = mk::err_at_L(sigma, gauss ? 0.0 : xi, k, l, gauss);
    if (log_on()) std::fprintf(stderr, "morlet: choose_terms sigma=%.6g K=%d L=%lld relrmse=%.3e\n", sigma, k, (long long)l, e);
    if (e < best) {
      best = e;
      bestK = k;
      bestL = l;
    }
    if (e <= target) {
      *K = k;
      *L = l;
      *relrmse = e;
      return MORLET_OK;
    }
  }
  *K = bestK;
  *L = bestL;
  *relrmse = best;
  return fail(MORLET_ERR_UNSUPPORTED, "no number of terms up to MORLET_MAX_TERMS reaches the target");
}

morlet_status morlet_choose_terms(double sigma, double xi, double target_relrmse, int32_t* K, int64_t* L,
                                  double* relrmse) {
  return choose_terms(sigma, xi, false, target_relrmse, K, L, relrmse);
}

morlet_status morlet_choose_terms_gauss(double sigma, double target_relrmse, int32_t* K, int64_t* L, double* relrmse) {
  return choose_terms(sigma, 0.0, true, target_relrmse, K, L, relrmse);
}

const char* morlet_last_error(void) { return g_err.c_str(); }

}  // extern "C"
