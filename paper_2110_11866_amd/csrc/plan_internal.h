// Host-side plan object and the host math behind it (fits, order search, tables).
#pragma once
#include <stdint.h>
#include <string>
#include <vector>

#include "layout.h"

// One scale of a batched plan.
struct ScaleParams {
  double sigma = 0, xi = 0;
  int64_t L = 0;
  int P_S = 0;
  int64_t n0_asft = 0;
  std::vector<double> cc, sc, jac;
  double relrmse = 0;
};

struct morlet_plan_s {
  int kind = 0;           // 0 Morlet, 1 Gaussian family (real output)
  int deriv = 0;          // Gaussian family: 0 smoothing, 1 first differential (sine
                          // components 1..K), 2 second differential (cosine components 0..K-1)
  int64_t N = 0;
  double sigma = 0, xi = 0;
  int K = 0;
  int64_t L = 0;
  int P_S = 0;
  int mode = 0;           // 0 SFT, 1 ASFT
  int64_t n0 = 0;         // ASFT shift (0 for SFT)
  int64_t n0_asft = 0;    // shift used when ASFT is selected
  int accum = 3;          // morlet_accum: 0 float32 tile scan, 1 float64, 2 mixed, 3 by mode
  int boundary = 0;       // single signals: 0 zero extension, 1 edge values (Sec. II)
  std::vector<double> cc, sc;   // cos / sin coefficients (m, l) or (a, 0)
  std::vector<double> jac;      // [4K]: dcc/dsigma, dcc/dxi, dsc/dsigma, dsc/dxi
  double relrmse = 0;
  int R = 16;             // samples per thread
  int row_serial = -1;    // schedule: -1 automatic, 0 tiles with look-back, 1 whole rows, 2 segments
  int seg_tiles = 0;      // segments schedule: tiles per segment (0: about two segments per resident block)
  int device = 0;
  int num_cus = 256;
  void* d_tab = nullptr;  // device copy of the constant table
  size_t tab_bytes = 0;
  std::vector<unsigned char> h_tab;
  // morlet_plan_refit: pinned staging copy of the table for the stream-ordered upload, and the
  // event recorded after that upload (allocated by the first refit, kept until destroy)
  void* h_stage = nullptr;
  size_t stage_bytes = 0;
  void* stage_event = nullptr;            // hipEvent_t
  // batched ragged plans (B signals x S scales); empty for single-signal plans
  bool batched = false;
  int B = 0, S = 0;
  std::vector<int64_t> lengths, offsets;   // per signal (offsets: prefix sums of lengths)
  std::vector<ScaleParams> scales;
  std::vector<mk::Row> rows;               // B*S rows, signal-major
  std::vector<int32_t> tile_row;
  std::vector<int32_t> row_order;          // row-serial schedule: the row queues back to back
  int32_t qstart[mk::kQueues + 1] = {0};   // queue q is row_order[qstart[q] .. qstart[q + 1])
  int64_t max_row_tiles = 0;
  int64_t ntiles = 0, ntiles_max = 0;
  void* d_rows = nullptr;                  // device rows, then tile_row, then row_order
  size_t rows_bytes = 0;
  // exact taps of the direct-convolution baseline (uploaded on its first call)
  void* d_direct = nullptr;
  int64_t direct_H = -1;
  // Morlet by the multiplication method (Sec. III-B): a batched Gaussian plan over three rows
  // of the signal's length (the demodulated signal's real and imaginary parts, and the signal),
  // the carrier applied around the scan
  bool multiply = false;
  int64_t mult_N = 0;                  // signal length
  double mult_ce = 0, mult_kappa = 0;  // C_xi / (pi^(1/4) sqrt(sigma)) / sqrt(gamma / pi), kappa_xi
  // separable 2-D Gaussian smoothing of an H x W image (Sec. IV: lines filtered independently):
  // axis[0] is a batched Gaussian plan over the H rows (length W), axis[1] one over the W rows
  // of the transposed image (length H); this plan owns both
  bool image2d = false;
  bool gabor = false;   // image plan: Morlet rows (axis 0) then Gaussian columns of both parts
  int64_t img_H = 0, img_W = 0;
  morlet_plan_s* axis[2] = {nullptr, nullptr};
};

namespace mk {

struct Fit {
  std::vector<double> cc, sc;
  double relrmse;
};

// Kernel samples on k = -L..L (index k + L).
void morlet_taps(double sigma, double xi, int64_t L, std::vector<double>& re, std::vector<double>& im);
// G[k] (deriv 0), G_D[k] (1) or G_DD[k] (2) for k = -L..L (Sec. II)
void gauss_taps(double sigma, int64_t L, std::vector<double>& g, int deriv = 0);

// MMSE fit of the given real targets on orders P_S..P_S+K-1 (cos part to `even`,
// sin part to `odd`); relrmse against the combined complex target.
Fit fit_orders(const std::vector<double>& tre, const std::vector<double>& tim, int64_t L, int P_S, int K);

int select_ps(double sigma, double xi, int K, int64_t L, double* best_err);
int64_t select_L(double sigma, double xi, int K, bool gauss);
// kernel relRMSE of the K-term fit on [-L, L] (Morlet: at the best lowest order)
double err_at_L(double sigma, double xi, int K, int64_t L, bool gauss);

void jacobian(morlet_plan_s* p);
// Fill p->h_tab for the plan's current mode and R; returns false on bad parameters.
bool build_table(morlet_plan_s* p, std::string* err);
// Fill one table for arbitrary parameters (used by the scalogram plans as well).
void fill_table(unsigned char* dst, int kind, int K, int R, int64_t L, int P_S, double sigma, double xi,
                int mode, int64_t n0, const std::vector<double>& cc, const std::vector<double>& sc,
                const std::vector<double>& jac);

}  // namespace mk
