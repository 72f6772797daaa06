// C ABI entry points (include/morlet.h): argument checks, plan construction, launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "../../include/morlet.h"
#include "launch.h"
#include "plan_internal.h"

namespace {

thread_local std::string g_err;

morlet_status fail(morlet_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

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

morlet_status run_scan(morlet_plan_t plan, const void* x, int dtype, void* out, void* ws, size_t ws_bytes,
                       void* stream, int want_kind) {
  if (!plan) return fail(MORLET_ERR_INVALID_ARG, "null plan");
  if (plan->kind != want_kind)
    return fail(MORLET_ERR_INVALID_ARG, want_kind == 0 ? "morlet_forward needs a Morlet plan"
                                                       : "gauss_smooth needs a Gaussian plan");
  if (dtype < 0 || dtype > 2) return fail(MORLET_ERR_UNSUPPORTED, "unknown dtype");
  if (plan->N == 0) return MORLET_OK;
  if (!x || !out || !ws) return fail(MORLET_ERR_INVALID_ARG, "null x, output or workspace pointer");
  const int64_t jend = plan->N + plan->L - plan->n0;
  const int64_t ntiles = tiles_for(jend, plan->R);
  if (ntiles > ((int64_t)1 << 31)) return fail(MORLET_ERR_UNSUPPORTED, "too many tiles");
  if (ws_bytes < mk::workspace_bytes(plan->K, ntiles)) return fail(MORLET_ERR_WORKSPACE, "workspace too small");
  if (!plan->d_tab) return fail(MORLET_ERR_HIP, "plan has no device table (created without a HIP device)");
  mk::ScanLaunch a{};
  a.K = plan->K;
  a.R = plan->R;
  a.wide = plan->accum;
  a.kind = plan->kind;
  a.x = x;
  a.dtype = dtype;
  a.out = out;
  a.row0.x_off = 0;
  a.row0.w_off = 0;
  a.row0.N = plan->N;
  a.row0.L = plan->L;
  a.row0.jout0 = plan->L - plan->n0;
  a.row0.jend = jend;
  a.row0.tile0 = 0;
  a.row0.scale = 0;
  a.row0.ntiles = (int32_t)ntiles;
  a.rows = nullptr;
  a.nrows = 1;
  a.tile_row = nullptr;
  a.ntiles = ntiles;
  a.tabs = static_cast<const unsigned char*>(plan->d_tab);
  a.tab_stride = (int64_t)plan->tab_bytes;
  a.f32_bytes = (int64_t)mk::TabLayout{plan->K, plan->R}.f32Bytes();
  a.ws = ws;
  const int occ = mk::scan_forward_occupancy(a.K, a.R, a.wide, a.kind);
  if (occ <= 0) return fail(MORLET_ERR_UNSUPPORTED, "no kernel for this configuration");
  const int64_t cap = (int64_t)occ * plan->num_cus;
  a.grid = (int)(ntiles < cap ? ntiles : cap);
  const hipError_t e = mk::launch_scan_forward(a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(MORLET_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
  return MORLET_OK;
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

morlet_status morlet_plan_set(morlet_plan_t plan, morlet_scan mode, int64_t n0, morlet_accum accum) {
  if (!plan) return fail(MORLET_ERR_INVALID_ARG, "null plan");
  if (mode != MORLET_SCAN_SFT && mode != MORLET_SCAN_ASFT) return fail(MORLET_ERR_UNSUPPORTED, "unknown scan mode");
  if (accum != MORLET_ACC_F32 && accum != MORLET_ACC_COMPENSATED)
    return fail(MORLET_ERR_UNSUPPORTED, "unknown accumulation mode");
  if (n0 < 0 || n0 > plan->L) return fail(MORLET_ERR_INVALID_ARG, "n0 must be 0 (default) or in [1, L]");
  plan->mode = (int)mode;
  plan->accum = (int)accum;
  if (n0 > 0) plan->n0_asft = n0;
  plan->n0 = (mode == MORLET_SCAN_ASFT) ? plan->n0_asft : 0;
  std::string err;
  mk::build_table(plan, &err);
  if (plan->d_tab) return upload_table(plan);
  return MORLET_OK;
}

morlet_status morlet_plan_info(morlet_plan_t plan, int64_t* L, int32_t* P_S, int64_t* n0, double* alpha,
                               double* cos_coef, double* sin_coef, double* jac, double* kernel_relrmse) {
  if (!plan) return fail(MORLET_ERR_INVALID_ARG, "null plan");
  if (L) *L = plan->L;
  if (P_S) *P_S = plan->P_S;
  if (n0) *n0 = plan->n0;
  if (alpha) *alpha = plan->mode == 1 ? (double)plan->n0 / (plan->sigma * plan->sigma) : 0.0;
  if (cos_coef) std::memcpy(cos_coef, plan->cc.data(), sizeof(double) * plan->K);
  if (sin_coef) std::memcpy(sin_coef, plan->sc.data(), sizeof(double) * plan->K);
  if (jac) std::memcpy(jac, plan->jac.data(), sizeof(double) * 4 * plan->K);
  if (kernel_relrmse) *kernel_relrmse = plan->relrmse;
  return MORLET_OK;
}

morlet_status morlet_workspace_size(morlet_plan_t plan, size_t* bytes) {
  if (!plan || !bytes) return fail(MORLET_ERR_INVALID_ARG, "null plan or output");
  // sized for the longest scan range over every n0 the plan may use (n0 = 0)
  *bytes = mk::workspace_bytes(plan->K, tiles_for(plan->N + plan->L, plan->R));
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
  return run_scan(plan, x, (int)dtype, W, ws, ws_bytes, stream, 0);
}

morlet_status gauss_smooth(morlet_plan_t plan, const void* x, morlet_dtype dtype, float* y, void* ws,
                           size_t ws_bytes, void* stream) {
  return run_scan(plan, x, (int)dtype, y, ws, ws_bytes, stream, 1);
}

void morlet_destroy(morlet_plan_t plan) {
  if (!plan) return;
  if (plan->d_tab) (void)hipFree(plan->d_tab);
  delete plan;
}

const char* morlet_last_error(void) { return g_err.c_str(); }

}  // extern "C"
