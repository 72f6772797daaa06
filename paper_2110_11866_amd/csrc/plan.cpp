// Host plan math: kernel samples, minimum-squared-error Fourier fits (eq. mmse), the
// lowest-order search of the direct method (Sec. III-A, Sec. V-A), the window choice,
// coefficient Jacobians and the per-scale constant tables of the scan kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

#include "plan_internal.h"

namespace mk {

namespace {

const double kPi = 3.14159265358979323846;

struct MorletConsts {
  double C, kappa, A;
};

MorletConsts morlet_consts(double sigma, double xi) {
  const double x0 = xi * sigma;  // dimensionless carrier
  MorletConsts c;
  c.C = 1.0 / std::sqrt(1.0 + std::exp(-x0 * x0) - 2.0 * std::exp(-0.75 * x0 * x0));
  c.kappa = std::exp(-0.5 * x0 * x0);
  c.A = c.C / (std::pow(kPi, 0.25) * std::sqrt(sigma));
  return c;
}

// Projections of a target y[k] (k = -L..L, index k + L) on cos(beta p k) and sin(beta p k)
// for p = p_lo..p_hi, with the angle reduced exactly: beta p k = pi ((p k) mod 2L) / L.
// Uses y[k] cos + y[-k] cos = (y[k] + y[-k]) cos (and the odd counterpart for sin).
void project(const std::vector<double>& y, int64_t L, int p_lo, int p_hi, std::vector<double>& bc,
             std::vector<double>& bs) {
  const int n = p_hi - p_lo + 1;
  bc.assign(n, 0.0);
  bs.assign(n, 0.0);
  const int64_t twoL = 2 * L;
  for (int i = 0; i < n; ++i) {
    const int64_t p = p_lo + i;
    double sc = y[L], ss = 0.0;  // k = 0 term
    int64_t m = 0;
    for (int64_t k = 1; k <= L; ++k) {
      m += p;
      if (m >= twoL) m -= twoL * (m / twoL);
      const double ang = kPi * (double)m / (double)L;
      sc += (y[L + k] + y[L - k]) * std::cos(ang);
      ss += (y[L + k] - y[L - k]) * std::sin(ang);
    }
    bc[i] = sc;
    bs[i] = ss;
  }
}

double sumsq(const std::vector<double>& v) {
  double s = 0;
  for (double x : v) s += x * x;
  return s;
}

// Normal equations of the fit. Over k = -L..L the cosines of orders 0..L have Gram matrix
// diag(d) + s s^T with d_p = 2L for p in {0, L} (L otherwise) and s_p = (-1)^p, because the
// end point k = L repeats k = -L of the 2L-periodic grid; the sines of orders 1..L-1 are
// orthogonal with squared norm L and vanish for p in {0, L}.
void solve_cos(const std::vector<double>& b, int64_t L, int P_S, std::vector<double>& c) {
  const int K = (int)b.size();
  std::vector<double> db(K), ds(K);
  double sdb = 0, sds = 0;
  for (int i = 0; i < K; ++i) {
    const int64_t p = P_S + i;
    const double d = (p == 0 || p == L) ? 2.0 * (double)L : (double)L;
    const double s = (p & 1) ? -1.0 : 1.0;
    db[i] = b[i] / d;
    ds[i] = s / d;
    sdb += s * db[i];
    sds += s * ds[i];
  }
  c.resize(K);
  const double f = sdb / (1.0 + sds);
  for (int i = 0; i < K; ++i) c[i] = db[i] - ds[i] * f;
}

void solve_sin(const std::vector<double>& b, int64_t L, int P_S, std::vector<double>& c) {
  const int K = (int)b.size();
  c.assign(K, 0.0);
  for (int i = 0; i < K; ++i) {
    const int64_t p = P_S + i;
    if (p >= 1 && p <= L - 1) c[i] = b[i] / (double)L;
  }
}

double kterm_relrmse(const std::vector<double>& tre, const std::vector<double>& tim, int64_t L, int P_S,
                     const std::vector<double>& cc, const std::vector<double>& sc) {
  const int K = (int)cc.size();
  double num = 0, den = 0;
  for (int64_t k = -L; k <= L; ++k) {
    double fr = 0, fi = 0;
    for (int i = 0; i < K; ++i) {
      const int64_t p = P_S + i;
      int64_t m = (p * k) % (2 * L);
      if (m < 0) m += 2 * L;
      const double ang = kPi * (double)m / (double)L;
      fr += cc[i] * std::cos(ang);
      fi += sc[i] * std::sin(ang);
    }
    const double er = fr - tre[L + k], ei = fi - (tim.empty() ? 0.0 : tim[L + k]);
    num += er * er + ei * ei;
    den += tre[L + k] * tre[L + k] + (tim.empty() ? 0.0 : tim[L + k] * tim[L + k]);
  }
  return std::sqrt(num / den);
}

int ps_hi(double xi, int K, int64_t L) {
  const int64_t carrier = (int64_t)std::ceil(xi * (double)L / kPi);
  const int64_t hi = std::min<int64_t>(L - K + 1, carrier + K);
  return (int)std::max<int64_t>(hi, 0);
}

// Residual^2 of the fit on orders P_S..P_S+K-1 from the projections (index p - p_lo).
double residual2(const std::vector<double>& bc_all, const std::vector<double>& bs_all, int p_lo, int P_S,
                 int K, int64_t L, double yy) {
  std::vector<double> bc(bc_all.begin() + (P_S - p_lo), bc_all.begin() + (P_S - p_lo) + K);
  std::vector<double> bs(bs_all.begin() + (P_S - p_lo), bs_all.begin() + (P_S - p_lo) + K);
  std::vector<double> c, s;
  solve_cos(bc, L, P_S, c);
  solve_sin(bs, L, P_S, s);
  double r = yy;
  for (int i = 0; i < K; ++i) r -= c[i] * bc[i] + s[i] * bs[i];
  return r;
}

}  // namespace

void morlet_taps(double sigma, double xi, int64_t L, std::vector<double>& re, std::vector<double>& im) {
  const MorletConsts mc = morlet_consts(sigma, xi);
  re.resize(2 * L + 1);
  im.resize(2 * L + 1);
  for (int64_t k = -L; k <= L; ++k) {
    const double kk = (double)k;
    const double env = mc.A * std::exp(-kk * kk / (2.0 * sigma * sigma));
    re[L + k] = env * (std::cos(xi * kk) - mc.kappa);
    im[L + k] = env * std::sin(xi * kk);
  }
}

void gauss_taps(double sigma, int64_t L, std::vector<double>& g, int deriv) {
  const double gamma = 1.0 / (2.0 * sigma * sigma);
  const double a = std::sqrt(gamma / kPi);
  g.resize(2 * L + 1);
  for (int64_t k = -L; k <= L; ++k) {
    const double kk = (double)k, G = a * std::exp(-gamma * kk * kk);
    // G, G_D = (-2 gamma k) G, G_DD = (4 gamma^2 k^2 - 2 gamma) G (Sec. II)
    g[L + k] = deriv == 0 ? G : deriv == 1 ? -2.0 * gamma * kk * G : (4.0 * gamma * gamma * kk * kk - 2.0 * gamma) * G;
  }
}

Fit fit_orders(const std::vector<double>& tre, const std::vector<double>& tim, int64_t L, int P_S, int K) {
  std::vector<double> bc, bs, bc2, bs2;
  project(tre, L, P_S, P_S + K - 1, bc, bs2);
  Fit f;
  solve_cos(bc, L, P_S, f.cc);
  if (!tim.empty()) {
    project(tim, L, P_S, P_S + K - 1, bc2, bs);
    solve_sin(bs, L, P_S, f.sc);
  } else {
    f.sc.assign(K, 0.0);
  }
  f.relrmse = kterm_relrmse(tre, tim, L, P_S, f.cc, f.sc);
  return f;
}

int select_ps(double sigma, double xi, int K, int64_t L, double* best_err) {
  std::vector<double> re, im;
  morlet_taps(sigma, xi, L, re, im);
  const int hi = ps_hi(xi, K, L);
  std::vector<double> bc, bs_unused, bc_unused, bs;
  project(re, L, 0, hi + K - 1, bc, bs_unused);
  project(im, L, 0, hi + K - 1, bc_unused, bs);
  const double yy = sumsq(re) + sumsq(im);
  int best = 0;
  double best_r = std::numeric_limits<double>::infinity();
  for (int ps = 0; ps <= hi; ++ps) {
    const double r = std::sqrt(std::max(residual2(bc, bs, 0, ps, K, L, yy), 0.0) / yy);
    if (r < best_r * (1.0 - 1e-12)) {
      best_r = r;
      best = ps;
    }
  }
  if (best_err) *best_err = best_r;
  return best;
}

double err_at_L(double sigma, double xi, int K, int64_t L, bool gauss) {
  if (gauss) {
    std::vector<double> g, none;
    gauss_taps(sigma, L, g);
    std::vector<double> bc, bs;
    project(g, L, 0, K - 1, bc, bs);
    return std::sqrt(std::max(residual2(bc, std::vector<double>(K, 0.0), 0, 0, K, L, sumsq(g)), 0.0) / sumsq(g));
  }
  double e = 0;
  select_ps(sigma, xi, K, L, &e);
  return e;
}

int64_t select_L(double sigma, double xi, int K, bool gauss) {
  // Grid L = round(c sigma), c = 1.50, 1.52, ..., 5.00, searched coarse to fine: every
  // fifth grid point first, then the grid points within 0.10 of the best coarse one.
  auto L_of = [&](int ci) {
    int64_t L = (int64_t)std::llround((1.5 + 0.02 * ci) * sigma);
    return std::max<int64_t>(L, std::max(K, 1));
  };
  int best_ci = 0;
  double best = std::numeric_limits<double>::infinity();
  for (int ci = 0; ci <= 175; ci += 5) {
    const double e = err_at_L(sigma, xi, K, L_of(ci), gauss);
    if (e < best * (1.0 - 1e-12)) {
      best = e;
      best_ci = ci;
    }
  }
  const int c0 = best_ci;
  for (int ci = std::max(0, c0 - 5); ci <= std::min(175, c0 + 5); ++ci) {
    if (ci % 5 == 0) continue;
    const double e = err_at_L(sigma, xi, K, L_of(ci), gauss);
    if (e < best * (1.0 - 1e-12) || (e <= best && ci < best_ci)) {
      best = e;
      best_ci = ci;
    }
  }
  return L_of(best_ci);
}

void jacobian(morlet_plan_s* p) {
  const int K = p->K;
  const int64_t L = p->L;
  p->jac.assign(4 * K, 0.0);
  if (p->deriv != 0) return;   // differential smoothing has no parameter gradients
  std::vector<double> ds_re(2 * L + 1), ds_im(2 * L + 1), dx_re(2 * L + 1), dx_im(2 * L + 1);
  if (p->kind == 0) {
    // d psi / d sigma and d psi / d xi by the product rule on
    //   psi = A(x0) sigma^{-1/2} E (e^{i xi k} - kappa(x0)),  x0 = xi sigma,
    //   A = C(x0) pi^{-1/4}, C = D^{-1/2}, D = 1 + e^{-x0^2} - 2 e^{-3 x0^2/4}, kappa = e^{-x0^2/2}.
    const double sigma = p->sigma, xi = p->xi, x0 = xi * sigma;
    const MorletConsts mc = morlet_consts(sigma, xi);
    const double D = 1.0 + std::exp(-x0 * x0) - 2.0 * std::exp(-0.75 * x0 * x0);
    const double dD = -2.0 * x0 * std::exp(-x0 * x0) + 3.0 * x0 * std::exp(-0.75 * x0 * x0);
    const double dA = (-0.5 * std::pow(D, -1.5) * dD) / std::pow(kPi, 0.25);  // dA/dx0
    const double A = mc.C / std::pow(kPi, 0.25);
    const double dkappa = -x0 * mc.kappa;  // dkappa/dx0
    const double s = 1.0 / std::sqrt(sigma), dsig_s = -0.5 * std::pow(sigma, -1.5);
    for (int64_t k = -L; k <= L; ++k) {
      const double kk = (double)k;
      const double E = std::exp(-kk * kk / (2.0 * sigma * sigma));
      const double dE = E * kk * kk / (sigma * sigma * sigma);
      const double cr = std::cos(xi * kk) - mc.kappa, ci = std::sin(xi * kk);
      // sigma: A and kappa move through x0 (dx0/dsigma = xi), plus sigma^{-1/2} and E
      const double gs = dA * xi * s * E + A * dsig_s * E + A * s * dE;
      ds_re[L + k] = gs * cr + A * s * E * (-dkappa * xi);
      ds_im[L + k] = gs * ci;
      // xi: A and kappa move through x0 (dx0/dxi = sigma); the carrier gives i k e^{i xi k}
      const double gx = dA * sigma * s * E;
      dx_re[L + k] = gx * cr + A * s * E * (-kk * std::sin(xi * kk) - dkappa * sigma);
      dx_im[L + k] = gx * ci + A * s * E * (kk * std::cos(xi * kk));
    }
  } else {
    // Gaussian: dG/dsigma = G (k^2/sigma^3 - 1/sigma); no xi
    std::vector<double> g;
    gauss_taps(p->sigma, L, g);
    for (int64_t k = -L; k <= L; ++k) {
      const double kk = (double)k;
      ds_re[L + k] = g[L + k] * (kk * kk / (p->sigma * p->sigma * p->sigma) - 1.0 / p->sigma);
      ds_im[L + k] = 0.0;
      dx_re[L + k] = 0.0;
      dx_im[L + k] = 0.0;
    }
  }
  const int P_S = p->P_S;
  std::vector<double> bc, bs, c;
  const std::vector<double>* srcs[4] = {&ds_re, &dx_re, &ds_im, &dx_im};
  for (int t = 0; t < 4; ++t) {
    project(*srcs[t], L, P_S, P_S + K - 1, bc, bs);
    if (t < 2) solve_cos(bc, L, P_S, c);
    else if (p->kind == 0) solve_sin(bs, L, P_S, c);
    else c.assign(K, 0.0);
    for (int i = 0; i < K; ++i) p->jac[t * K + i] = c[i];
  }
}

namespace {
// a_p^m = e^{-alpha m} e^{-i beta p m}, angle reduced exactly
inline void apow(int64_t p, int64_t m, int64_t L, double alpha, double& re, double& im) {
  int64_t r = (p % (2 * L)) * (m % (2 * L)) % (2 * L);
  const double ang = -kPi * (double)r / (double)L;
  const double mag = std::exp(-alpha * (double)m);
  re = mag * std::cos(ang);
  im = mag * std::sin(ang);
}
}  // namespace

void fill_table(unsigned char* dst, int kind, int K, int R, int64_t L, int P_S, double sigma, double xi,
                int mode, int64_t n0, const std::vector<double>& cc, const std::vector<double>& sc,
                const std::vector<double>& jac) {
  TabLayout lay{K, R};
  std::memset(dst, 0, lay.bytes());
  float* tf = (float*)dst;
  double* td = (double*)(dst + lay.f32Bytes());
  const double alpha = (mode == 1) ? (double)n0 / (sigma * sigma) : 0.0;
  const int64_t T = (int64_t)R * kThreads;
  const int mo = lay.nComplex();
  // entry e gets a^d, entry mo + e gets d a^d
  auto put = [&](int e, int i, int64_t p, int64_t d) {
    double re, im;
    apow(p, d, L, alpha, re, im);
    const double dd = (double)d;
    tf[(2 * e) * K + i] = (float)re;
    tf[(2 * e + 1) * K + i] = (float)im;
    td[(2 * e) * K + i] = re;
    td[(2 * e + 1) * K + i] = im;
    tf[(2 * (mo + e)) * K + i] = (float)(dd * re);
    tf[(2 * (mo + e) + 1) * K + i] = (float)(dd * im);
    td[(2 * (mo + e)) * K + i] = dd * re;
    td[(2 * (mo + e) + 1) * K + i] = dd * im;
  };
  auto putrow = [&](int row, int i, double v) {
    tf[row * K + i] = (float)v;
    td[row * K + i] = v;
  };
  double cx = 0;
  for (int i = 0; i < K; ++i) {
    const int64_t p = P_S + i;
    put(lay.eA(), i, p, 1);
    for (int r = 0; r < R; ++r) put(lay.eP1(r), i, p, R - 1 - r);
    for (int d = 0; d < 6; ++d) put(lay.eTR(d), i, p, (int64_t)R << d);
    for (int l = 0; l < 64; ++l) put(lay.eLANE(l), i, p, (int64_t)R * l);
    for (int w = 0; w <= kWaves; ++w) put(lay.eWV(w), i, p, (int64_t)64 * R * w);
    for (int k = 0; k <= 64; ++k) put(lay.eLB(k), i, p, T * k);
    for (int k = 0; k <= 64; ++k) put(lay.eLB2(k), i, p, 64 * T * k);
    const double sgn = (p & 1) ? -1.0 : 1.0;
    const double up = std::exp(alpha * (double)L), dn = std::exp(-alpha * (double)L);
    putrow(lay.rMW(), i, sgn * cc[i] * up);
    putrow(lay.rLW(), i, sgn * sc[i] * up);
    putrow(lay.rSGN(), i, sgn);
    putrow(lay.rCC(), i, cc[i]);
    putrow(lay.rSC(), i, sc[i]);
    for (int q = 0; q < 4; ++q) putrow(lay.rJ(q), i, jac.size() == (size_t)4 * K ? jac[q * K + i] : 0.0);
    for (int k = 1; k <= 4; ++k) {
      double re, im;
      apow(p, k, L, alpha, re, im);
      const int v = lay.vHC(i) + 2 * (k - 1);
      tf[v] = (float)re;
      tf[v + 1] = (float)im;
      td[v] = re;
      td[v + 1] = im;
    }
    cx += sgn * cc[i] * dn;
  }
  const double D = std::exp(-2.0 * alpha * (double)L);
  double gre = 1.0, gim = 0.0, dsig = 0.0, dxi = 0.0, dalpha = 0.0;
  if (mode == 1) {
    const double s = std::exp(-(double)n0 * (double)n0 / (2.0 * sigma * sigma));
    if (kind == 0) {
      gre = s * std::cos(xi * (double)n0);
      gim = s * std::sin(xi * (double)n0);
      dxi = (double)n0;
    } else {
      gre = s;
    }
    dsig = (double)n0 * (double)n0 / (sigma * sigma * sigma);
    dalpha = -2.0 * (double)n0 / (sigma * sigma * sigma);
  }
  const double sv[10] = {cx, D, gre, gim, std::exp(alpha * (double)L), std::exp(-alpha * (double)L), (double)L,
                         dsig, dxi, dalpha};
  const int so[10] = {lay.sCX(), lay.sD(), lay.sGre(), lay.sGim(), lay.sUP(), lay.sDN(), lay.sLL(), lay.sDSIG(),
                      lay.sDXI(), lay.sDALPHA()};
  for (int q = 0; q < 10; ++q) {
    tf[so[q]] = (float)sv[q];
    td[so[q]] = sv[q];
  }
  // float32 remainders of every entry, for float-float arithmetic
  float* tl = (float*)(dst + lay.f32Bytes() + lay.f64Bytes());
  for (int v = 0; v < lay.nValues(); ++v) tl[v] = (float)(td[v] - (double)tf[v]);
  // run matrices of the matrix-core recurrence (Morlet output): with v_t after r + 1 steps
  //   v_t[r] = a_t^{r+1} S_t + sum_{r' <= r} a_t^{r - r'} dy[r'],
  //   o_re = gre A + gim B, o_im = gim A - gre B, A = cx y + sum_t mw_t Re v_t, B = sum_t lw_t Im v_t
  if (kind == 0) {
    float* tm = (float*)(dst + lay.mfmaOff());
    const int RN = TabLayout::kRun, CW = lay.mCW();
    std::vector<double> Tre(RN * RN, 0.0), Tim(RN * RN, 0.0), Cre(RN * CW, 0.0), Cim(RN * CW, 0.0);
    for (int i = 0; i < K; ++i) {
      const int64_t p = P_S + i;
      const double mw = td[lay.rMW() * K + i], lw = td[lay.rLW() * K + i];
      for (int r = 0; r < RN; ++r) {
        for (int rp = 0; rp <= r; ++rp) {
          double re, im;
          apow(p, r - rp, L, alpha, re, im);
          Tre[RN * r + rp] += gre * mw * re + gim * lw * im;
          Tim[RN * r + rp] += gim * mw * re - gre * lw * im;
        }
        double re, im;
        apow(p, r + 1, L, alpha, re, im);
        Cre[CW * r + 2 * i] = gre * mw * re + gim * lw * im;
        Cre[CW * r + 2 * i + 1] = -gre * mw * im + gim * lw * re;
        Cim[CW * r + 2 * i] = gim * mw * re - gre * lw * im;
        Cim[CW * r + 2 * i + 1] = -gim * mw * im - gre * lw * re;
      }
    }
    for (int v = 0; v < RN * RN; ++v) {
      tm[lay.mTre() + v] = (float)Tre[v];
      tm[lay.mTim() + v] = (float)Tim[v];
    }
    for (int v = 0; v < RN * CW; ++v) {
      tm[lay.mCre() + v] = (float)Cre[v];
      tm[lay.mCim() + v] = (float)Cim[v];
    }
  }
}

bool build_table(morlet_plan_s* p, std::string* err) {
  TabLayout lay{p->K, p->R};
  p->h_tab.assign(lay.bytes(), 0);
  fill_table(p->h_tab.data(), p->kind, p->K, p->R, p->L, p->P_S, p->sigma, p->xi, p->mode, p->n0, p->cc, p->sc,
             p->jac);
  (void)err;
  return true;
}

}  // namespace mk
