// Drives every host-side path of the C ABI that runs without a GPU (plan construction, fits,
// window and lowest-order searches, row queues of batched plans, setters, queries, workspace
// sizes, argument checks) for a build with the host sanitizers. Exit status 0 when every call
// returned what the header promises; any other status names the failing check.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "morlet.h"

static int g_fail = 0;
#define EXPECT(cond)                                                            \
  do {                                                                          \
    if (!(cond)) {                                                              \
      std::fprintf(stderr, "check failed at line %d: %s (%s)\n", __LINE__, #cond, \
                   morlet_last_error());                                        \
      ++g_fail;                                                                 \
    }                                                                           \
  } while (0)

static void query(morlet_plan_t p, int K) {
  int64_t L = 0, n0 = 0;
  int32_t ps = -1;
  double alpha = 0, rel = 0;
  std::vector<double> cc(K), sc(K), jac(4 * K);
  EXPECT(morlet_plan_info(p, &L, &ps, &n0, &alpha, cc.data(), sc.data(), jac.data(), &rel) == MORLET_OK);
  EXPECT(L >= 1 && ps >= 0 && std::isfinite(rel));
  size_t ws = 0, bws = 0;
  EXPECT(morlet_workspace_size(p, &ws) == MORLET_OK && ws > 0);
  EXPECT(morlet_backward_workspace_size(p, &bws) == MORLET_OK);
}

int main() {
  morlet_plan_t p = nullptr;
  // single-signal plans: fixed and error-optimal windows, every mode, tile and accumulation
  const double sig[] = {1.5, 16.0, 300.0, 8192.0};
  for (double s : sig) {
    for (int K : {1, 4, 6, 12}) {
      const int64_t L = (int64_t)std::ceil(4 * s) < K ? K : (int64_t)std::ceil(4 * s);
      if (morlet_plan(&p, 5000, s, 6.0 / s, K, L) != MORLET_OK) {
        EXPECT(K > L);
        continue;
      }
      query(p, K);
      EXPECT(morlet_plan_set(p, MORLET_SCAN_ASFT, 0, MORLET_ACC_F32) == MORLET_OK);
      for (int R : {4, 8, 16, 32}) EXPECT(morlet_plan_set_tile(p, R) == MORLET_OK);
      EXPECT(morlet_plan_set_tile(p, 16) == MORLET_OK);
      EXPECT(morlet_plan_set(p, MORLET_SCAN_SFT, 0, MORLET_ACC_KAHAN) == MORLET_OK);
      EXPECT(morlet_plan_set_tile(p, 32) == MORLET_ERR_UNSUPPORTED);
      EXPECT(morlet_plan_set(p, MORLET_SCAN_ASFT, 3, MORLET_ACC_AUTO) == MORLET_OK);
      EXPECT(morlet_plan_set_boundary(p, MORLET_BOUNDARY_EDGE) == MORLET_OK);
      query(p, K);
      EXPECT(morlet_plan_set_boundary(p, MORLET_BOUNDARY_ZERO) == MORLET_OK);
      EXPECT(morlet_plan_refit(p, s * 1.01, 6.0 / s, nullptr) == MORLET_OK);   // host refit (no device table)
      EXPECT(morlet_plan_refit(p, -1.0, 6.0 / s, nullptr) == MORLET_ERR_INVALID_ARG);
      query(p, K);
      EXPECT(morlet_forward(p, nullptr, MORLET_F32, nullptr, nullptr, 0, nullptr) != MORLET_OK);
      morlet_destroy(p);
    }
    EXPECT(morlet_plan(&p, 3000, s, 6.0 / s, 5, 0) == MORLET_OK);
    query(p, 5);
    morlet_destroy(p);
    EXPECT(morlet_plan_gauss(&p, 3000, s, 4, 0) == MORLET_OK);
    query(p, 4);
    morlet_destroy(p);
    for (int order : {1, 2}) {
      EXPECT(morlet_plan_gauss_deriv(&p, 3000, s, 5, 0, order) == MORLET_OK);
      EXPECT(morlet_plan_set(p, MORLET_SCAN_ASFT, 0, MORLET_ACC_F32) == MORLET_OK);
      query(p, 5);
      EXPECT(morlet_plan_set(p, MORLET_SCAN_ASFT, 0, MORLET_ACC_KAHAN) == MORLET_ERR_UNSUPPORTED);
      morlet_destroy(p);
    }
    EXPECT(morlet_plan_multiply(&p, 3000, s, 6.0 / s, 2, 0) == MORLET_OK);
    query(p, 3);
    morlet_destroy(p);
  }
  // argument errors: synchronous, no side effect
  EXPECT(morlet_plan(nullptr, 10, 1.0, 1.0, 2, 4) == MORLET_ERR_INVALID_ARG);
  EXPECT(morlet_plan(&p, -1, 1.0, 1.0, 2, 4) == MORLET_ERR_INVALID_ARG);
  EXPECT(morlet_plan(&p, 10, -1.0, 1.0, 2, 4) == MORLET_ERR_INVALID_ARG);
  EXPECT(morlet_plan(&p, 10, NAN, 1.0, 2, 4) == MORLET_ERR_INVALID_ARG);
  EXPECT(morlet_plan(&p, 10, 1.0, 1.0, 0, 4) == MORLET_ERR_INVALID_ARG);
  EXPECT(morlet_plan(&p, 10, 1.0, 1.0, 13, 40) == MORLET_ERR_INVALID_ARG);
  EXPECT(morlet_plan(&p, 10, 1.0, 1.0, 5, 4) == MORLET_ERR_INVALID_ARG);
  EXPECT(morlet_plan_gauss(&p, 10, 1.0, 9, 4) == MORLET_ERR_INVALID_ARG);
  // batched ragged plans: empty, one-sample and multi-tile signals, queues dealt per signal
  {
    std::vector<int64_t> lengths;
    for (int b = 0; b < 70; ++b) lengths.push_back(b % 7 == 0 ? 0 : (int64_t)(37 * b * b + 1));
    const double sg[] = {3.0, 10.0, 45.0, 300.0, 1500.0};
    double xi[5];
    for (int s = 0; s < 5; ++s) xi[s] = 6.0 / sg[s];
    EXPECT(morlet_scalogram_plan(&p, (int32_t)lengths.size(), lengths.data(), 5, sg, xi, 5, 0.0) == MORLET_OK);
    for (int s = 0; s < 5; ++s) {
      int64_t L = 0, n0 = 0;
      int32_t ps = 0;
      double a = 0, cc[5], sc[5], jac[20], rel = 0;
      EXPECT(morlet_scalogram_scale_info(p, s, &L, &ps, &n0, &a, cc, sc, jac, &rel) == MORLET_OK);
    }
    EXPECT(morlet_scalogram_scale_info(p, 5, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                       nullptr) == MORLET_ERR_INVALID_ARG);
    for (int R : {4, 8, 16, 32}) EXPECT(morlet_plan_set_tile(p, R) == MORLET_OK);
    EXPECT(morlet_plan_set_schedule(p, MORLET_SCHED_ROWS) == MORLET_OK);
    EXPECT(morlet_plan_set(p, MORLET_SCAN_ASFT, 0, MORLET_ACC_AUTO) == MORLET_OK);
    size_t ws = 0;
    EXPECT(morlet_workspace_size(p, &ws) == MORLET_OK);
    EXPECT(morlet_scalogram_forward(p, nullptr, MORLET_F32, nullptr, nullptr, 0, nullptr) != MORLET_OK);
    morlet_destroy(p);
    const int64_t none = 0;
    EXPECT(morlet_scalogram_plan(&p, 1, &none, 1, sg, xi, 5, 4.0) == MORLET_OK);
    morlet_destroy(p);
    EXPECT(morlet_scalogram_plan(&p, 0, lengths.data(), 5, sg, xi, 5, 0.0) == MORLET_ERR_INVALID_ARG);
  }
  // images
  EXPECT(morlet_plan_gauss2d(&p, 37, 300, 3.0, 8.0, 4, 0, 0) == MORLET_OK);
  {
    int64_t L = 0, n0 = 0;
    double cc[4], rel = 0;
    EXPECT(morlet_image_axis_info(p, 1, &L, &n0, cc, &rel) == MORLET_OK);
    EXPECT(morlet_image_axis_info(p, 2, &L, &n0, cc, &rel) == MORLET_ERR_INVALID_ARG);
  }
  size_t ws = 0;
  EXPECT(morlet_workspace_size(p, &ws) == MORLET_OK);
  morlet_destroy(p);
  EXPECT(morlet_plan_gabor2d(&p, 64, 48, 6.0, 1.0, 5, 0, 4.0, 4, 0) == MORLET_OK);
  EXPECT(morlet_workspace_size(p, &ws) == MORLET_OK);
  EXPECT(morlet_plan_set(p, MORLET_SCAN_ASFT, 0, MORLET_ACC_F32) == MORLET_OK);
  morlet_destroy(p);
  morlet_destroy(nullptr);
  // term chooser and the failure hook (host only)
  {
    int32_t K = 0;
    int64_t L = 0;
    double e = 0;
    EXPECT(morlet_choose_terms(16.0, 6.0 / 16.0, 1e-2, &K, &L, &e) == MORLET_OK && K >= 1 && e <= 1e-2);
    EXPECT(morlet_choose_terms_gauss(8.0, 1e-4, &K, &L, &e) == MORLET_OK && e <= 1e-4);
    EXPECT(morlet_choose_terms(16.0, 6.0 / 16.0, 1e-300, &K, &L, &e) == MORLET_ERR_UNSUPPORTED);
    EXPECT(morlet_choose_terms(16.0, 6.0 / 16.0, 1e-2, nullptr, &L, &e) == MORLET_ERR_INVALID_ARG);
    EXPECT(morlet_inject_failure(MORLET_ERR_HIP, -1) == MORLET_ERR_INVALID_ARG);
    EXPECT(morlet_inject_failure(MORLET_OK, 2) == MORLET_ERR_INVALID_ARG);
    EXPECT(morlet_inject_failure(MORLET_ERR_HIP, 0) == MORLET_OK);
  }
  if (g_fail) std::fprintf(stderr, "%d checks failed\n", g_fail);
  else std::printf("abi driver: all checks passed\n");
  return g_fail ? 1 : 0;
}
