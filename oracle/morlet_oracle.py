"""FP64 CPU oracle for the Morlet wavelet transform and Gaussian smoothing by
SFT / ASFT evaluated as kernel integrals (Yamashita & Wakahara, arXiv 2110.11866).

TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this module. The product path never calls it, and it
shares no code with the HIP library (it does not import the package, and the
package does not import it).

Everything here is plain numpy/scipy in float64, written to be checked against
the paper by eye. Notation follows the paper with one renaming, because the
paper uses K for the half width of the summation window while the library API
uses K for the number of Fourier terms:

    L      half width of the window [-L, L]         (the paper's K)
    beta   pi / L                                   (Sec. II-A, "Let beta = pi/K")
    K      number of Fourier terms                  (the paper's P+1 for the
                                                     Gaussian, P_D for Morlet)
    P_S    lowest Fourier order of the direct method (Sec. III-A)
    gamma  1 / (2 sigma^2)                          (Sec. II)
    n0     ASFT output shift, alpha = 2 gamma n0 = n0 / sigma^2  (eq. siftGauss)

Readings of passages that are garbled or ambiguous in the paper (all of them
are listed, with evidence, in the design notes of the repository):
  * the dilated discrete Morlet wavelet carries C_xi / (pi^(1/4) sqrt(sigma))
    and the sample index n in the carrier (Sec. III, discrete psi);
  * xi is given in rad/sample; the dimensionless xi of the continuous wavelet
    is xi0 = xi * sigma and feeds C_xi and kappa_xi;
  * ASFT uses the causal weight e^{-alpha k} for k >= 0 (older samples decay,
    as the text under eq. asp says), so the extraction prefactor is e^{+alpha L}
    and the output is read n0 samples earlier (eqs. asfiir12K, GsASFT);
  * the Morlet ASFT formula of Sec. III-A is completed with the carrier phase
    e^{i xi n0} that the shift of eq. siftGauss introduces;
  * x is zero outside [0, N-1] (one of the two extensions Sec. II names);
  * the multiplication method (Sec. III-B) multiplies the carrier by the fit of
    the wavelet's own envelope e^{-n^2/(2 sigma^2)}, i.e. the a_p of eq.
    aproGauss divided by sqrt(gamma/pi), its kappa term is subtracted, and in
    ASFT form only the carrier part takes the phase e^{i xi n0}.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from functools import partial

import numpy as np
from scipy.signal import fftconvolve, lfilter

__all__ = [
    "gaussian", "gaussian_d1", "gaussian_d2", "fit_gauss_d1", "fit_gauss_d2", "plan_gauss_deriv",
    "kterm_gauss_deriv",
    "morlet", "Plan", "plan_morlet", "plan_gauss", "fit_morlet", "fit_gauss",
    "select_PS", "select_PS_full", "default_n0", "kterm_morlet", "kterm_gauss", "asft_kernel", "kernel_relrmse",
    "conv_same", "conv_same_at", "phase", "sft_component", "asft_component",
    "forward", "forward_direct", "adjoint", "param_grads", "dpsi_dtheta",
    "plan_multiply", "kterm_multiply", "freq_component", "gauss_smooth_2d", "gabor_2d", "gabor_2d_adjoint", "sliding_sum", "forward_tree",
    "forward_edge",
]


# --------------------------------------------------------------------------
# Kernels (Sec. II: Gaussian; Sec. III: Morlet wavelet)
# --------------------------------------------------------------------------
def gaussian(sigma: float, k: np.ndarray) -> np.ndarray:
    """G[k] = sqrt(gamma/pi) exp(-gamma k^2), gamma = 1/(2 sigma^2) (Sec. II).

    Not renormalised on the integers."""
    gamma = 1.0 / (2.0 * sigma * sigma)
    k = np.asarray(k, dtype=np.float64)
    return math.sqrt(gamma / math.pi) * np.exp(-gamma * k * k)


def gaussian_d1(sigma: float, k: np.ndarray) -> np.ndarray:
    """G_D[k] = (-2 gamma k) G[k], the first differential of the Gaussian (Sec. II)."""
    gamma = 1.0 / (2.0 * sigma * sigma)
    k = np.asarray(k, dtype=np.float64)
    return -2.0 * gamma * k * gaussian(sigma, k)


def gaussian_d2(sigma: float, k: np.ndarray) -> np.ndarray:
    """G_DD[k] = (4 gamma^2 k^2 - 2 gamma) G[k], the second differential (Sec. II)."""
    gamma = 1.0 / (2.0 * sigma * sigma)
    k = np.asarray(k, dtype=np.float64)
    return (4.0 * gamma * gamma * k * k - 2.0 * gamma) * gaussian(sigma, k)


def _morlet_consts(xi0: float) -> tuple[float, float]:
    """C_xi and kappa_xi of the mother wavelet (Sec. III)."""
    C = (1.0 + math.exp(-xi0 * xi0) - 2.0 * math.exp(-0.75 * xi0 * xi0)) ** -0.5
    kappa = math.exp(-0.5 * xi0 * xi0)
    return C, kappa


def morlet(sigma: float, xi: float, k: np.ndarray) -> np.ndarray:
    """Dilated discrete Morlet wavelet psi_{sigma,xi}[k] (Sec. III).

    psi[k] = C/(pi^(1/4) sqrt(sigma)) e^{-k^2/(2 sigma^2)} (e^{i xi k} - kappa),
    xi in rad/sample, xi0 = xi*sigma the dimensionless carrier."""
    xi0 = xi * sigma
    C, kappa = _morlet_consts(xi0)
    k = np.asarray(k, dtype=np.float64)
    env = C / (math.pi ** 0.25 * math.sqrt(sigma)) * np.exp(-k * k / (2.0 * sigma * sigma))
    return env * (np.exp(1j * xi * k) - kappa)


def dpsi_dtheta(sigma: float, xi: float, k: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Analytic partial derivatives d psi / d sigma and d psi / d xi of morlet().

    Written out from the product rule on the Sec. III formula with xi0 = xi*sigma:
      psi = A(xi0) sigma^{-1/2} E(k, sigma) (e^{i xi k} - kappa(xi0)),
      A = C(xi0) pi^{-1/4},  E = exp(-k^2 / (2 sigma^2)).
    """
    k = np.asarray(k, dtype=np.float64)
    xi0 = xi * sigma
    C, kappa = _morlet_consts(xi0)
    # dC/dxi0 from C = D^{-1/2}, D = 1 + e^{-xi0^2} - 2 e^{-3 xi0^2 / 4}
    dD = -2.0 * xi0 * math.exp(-xi0 * xi0) + 3.0 * xi0 * math.exp(-0.75 * xi0 * xi0)
    D = 1.0 + math.exp(-xi0 * xi0) - 2.0 * math.exp(-0.75 * xi0 * xi0)
    dC = -0.5 * D ** -1.5 * dD
    dkappa = -xi0 * kappa
    A = C / math.pi ** 0.25
    dA = dC / math.pi ** 0.25
    E = np.exp(-k * k / (2.0 * sigma * sigma))
    dE_dsigma = E * (k * k / sigma ** 3)
    car = np.exp(1j * xi * k) - kappa
    s = sigma ** -0.5
    ds = -0.5 * sigma ** -1.5
    # d/dsigma: xi0 depends on sigma (dxi0/dsigma = xi); the carrier e^{i xi k} does not.
    d_sigma = (dA * xi) * s * E * car + A * ds * E * car + A * s * dE_dsigma * car \
        + A * s * E * (-dkappa * xi)
    # d/dxi: xi0 depends on xi (dxi0/dxi = sigma); the carrier gives i k e^{i xi k}.
    d_xi = (dA * sigma) * s * E * car + A * s * E * (1j * k * np.exp(1j * xi * k) - dkappa * sigma)
    return d_sigma, d_xi


# --------------------------------------------------------------------------
# Plan: the truncated Fourier fits (eqs. aproGauss, mmse; Sec. III-A)
# --------------------------------------------------------------------------
@dataclass
class Plan:
    kind: str                 # "morlet", "gauss", "gd1", "gd2" (Gaussian differentials) or
                              # "mult" (Morlet by the multiplication method)
    sigma: float
    xi: float                 # rad/sample (0 for the Gaussian)
    K: int                    # number of Fourier terms
    L: int                    # window half width
    P_S: int                  # lowest order (0 for the Gaussian)
    mode: str = "sft"         # "sft" or "asft"
    n0: int = 0               # ASFT shift
    cos_coef: np.ndarray = field(default_factory=lambda: np.zeros(0))  # m_p or a_p
    sin_coef: np.ndarray = field(default_factory=lambda: np.zeros(0))  # l_p (zeros for Gauss)

    @property
    def beta(self) -> float:
        return math.pi / self.L

    @property
    def orders(self) -> np.ndarray:
        return np.arange(self.P_S, self.P_S + self.K)

    @property
    def alpha(self) -> float:
        return self.n0 / (self.sigma * self.sigma) if self.mode == "asft" else 0.0


def _basis(L: int, orders: np.ndarray) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """k = -L..L and the columns cos(beta p k), sin(beta p k) (eqs. cp, sp)."""
    k = np.arange(-L, L + 1, dtype=np.float64)
    # exact argument reduction: beta p k = pi * ((p k) mod 2L) / L
    pk = np.mod(np.outer(k.astype(np.int64), orders.astype(np.int64)), 2 * L).astype(np.float64)
    ang = math.pi * pk / L
    return k, np.cos(ang), np.sin(ang)


def _lstsq(B: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Minimum-squared-error coefficients (eq. mmse), columns that vanish on the
    integer grid (sin of order 0 or L) get coefficient 0."""
    coef = np.zeros(B.shape[1])
    keep = np.linalg.norm(B, axis=0) > 1e-9 * math.sqrt(B.shape[0])
    if keep.any():
        coef[keep] = np.linalg.lstsq(B[:, keep], y, rcond=None)[0]
    return coef


def fit_morlet(sigma: float, xi: float, K: int, L: int, P_S: int) -> tuple[np.ndarray, np.ndarray]:
    """Direct method (Sec. III-A): psi[k] ~ sum_p m_p cos(beta p k) + i l_p sin(beta p k)
    for p = P_S..P_S+K-1 on k in [-L, L]; m and l by MMSE, fitted to Re and Im
    separately (the two parts of the squared error decouple)."""
    orders = np.arange(P_S, P_S + K)
    k, Bc, Bs = _basis(L, orders)
    psi = morlet(sigma, xi, k)
    return _lstsq(Bc, psi.real), _lstsq(Bs, psi.imag)


def fit_gauss(sigma: float, K: int, L: int) -> np.ndarray:
    """eq. aproGauss with orders 0..K-1, coefficients a_p by MMSE (eq. mmse)."""
    k, Bc, _ = _basis(L, np.arange(K))
    return _lstsq(Bc, gaussian(sigma, k))


def fit_gauss_d1(sigma: float, K: int, L: int) -> np.ndarray:
    """G_D[k] ~ sum_{p=1}^{K} b_p sin(beta p k) on [-L, L], b by MMSE (Sec. II-A, eq. mmse):
    the odd differential takes the sine components of orders 1..K."""
    k, _, Bs = _basis(L, np.arange(1, K + 1))
    return _lstsq(Bs, gaussian_d1(sigma, k))


def fit_gauss_d2(sigma: float, K: int, L: int) -> np.ndarray:
    """G_DD[k] ~ sum_{p=0}^{K-1} d_p cos(beta p k) on [-L, L], d by MMSE (Sec. II-A)."""
    k, Bc, _ = _basis(L, np.arange(K))
    return _lstsq(Bc, gaussian_d2(sigma, k))


def _ps_range(xi: float, K: int, L: int) -> range:
    """Candidate lowest orders. Orders alias modulo 2L, so P_S + K - 1 <= L.
    The carrier sits at order xi L / pi; windows that start more than K orders
    above it only lose carrier energy, so the search stops there."""
    hi = min(L - K + 1, int(math.ceil(xi * L / math.pi)) + K)
    return range(0, max(hi, 0) + 1)


def kernel_relrmse(approx: np.ndarray, exact: np.ndarray) -> float:
    return float(np.linalg.norm(approx - exact) / np.linalg.norm(exact))


def _argmin_PS(sigma: float, xi: float, K: int, L: int, candidates) -> int:
    k = np.arange(-L, L + 1, dtype=np.float64)
    psi = morlet(sigma, xi, k)
    best, best_err = 0, math.inf
    for ps in candidates:
        m, l = fit_morlet(sigma, xi, K, L, ps)
        err = kernel_relrmse(_kterm(m, l, ps, L), psi)
        if err < best_err * (1.0 - 1e-12):
            best, best_err = ps, err
    return best


def select_PS(sigma: float, xi: float, K: int, L: int) -> int:
    """P_S minimising the relative RMSE of the fitted wavelet on [-L, L]
    (Sec. V-A, the optimum P_S of Fig. MSE2); ties go to the smallest P_S.
    The search stops K orders above the carrier (see _ps_range); the tests pin
    this against select_PS_full, the argmin over every admissible order."""
    return _argmin_PS(sigma, xi, K, L, _ps_range(xi, K, L))


def select_PS_full(sigma: float, xi: float, K: int, L: int) -> int:
    """The same argmin over every admissible lowest order 0..L-K+1 (orders alias
    modulo 2L, so P_S + K - 1 <= L), with no cap at the carrier. O(L^2 K^2) work:
    meant for small windows."""
    return _argmin_PS(sigma, xi, K, L, range(0, max(L - K + 1, 0) + 1))


def default_n0(sigma: float) -> int:
    """Default ASFT shift max(1, round(sigma / 8)). The paper fixes no rule (it uses
    n0 = 10 at a window of 256); this reading rounds halves up (sigma = 20 gives 3)."""
    return max(1, int(math.floor(sigma / 8.0 + 0.5)))


def plan_morlet(sigma: float, xi: float, K: int, L: int, mode: str = "sft",
                n0: int | None = None, P_S: int | None = None) -> Plan:
    if P_S is None:
        P_S = select_PS(sigma, xi, K, L)
    m, l = fit_morlet(sigma, xi, K, L, P_S)
    if mode == "asft" and n0 is None:
        n0 = default_n0(sigma)
    return Plan("morlet", sigma, xi, K, L, P_S, mode, int(n0 or 0) if mode == "asft" else 0, m, l)


def plan_gauss(sigma: float, K: int, L: int, mode: str = "sft", n0: int | None = None) -> Plan:
    a = fit_gauss(sigma, K, L)
    if mode == "asft" and n0 is None:
        n0 = default_n0(sigma)
    return Plan("gauss", sigma, 0.0, K, L, 0, mode, int(n0 or 0) if mode == "asft" else 0,
                a, np.zeros(K))


def plan_gauss_deriv(sigma: float, K: int, L: int, order: int, mode: str = "sft",
                     n0: int | None = None) -> Plan:
    """Gaussian differential smoothing (Sec. II).

    SFT: order 1 is x_GD with the sine components of orders 1..K, order 2 is x_GDD with the
    cosine components of orders 0..K-1 (G_D is odd, G_DD even).

    ASFT (Sec. II-B, eqs. siftGauss and gddAsft): the K terms are orders 0..K-1 and both
    components are used. The attenuation e^{-alpha k} with alpha = n0 / sigma^2 moves the
    Gaussian by n0, G[k + n0] = s e^{-alpha k} G[k] with s = e^{-n0^2/(2 sigma^2)}, and
    differentiating that identity gives
        G_D[k + n0]  = s e^{-alpha k} (G_D[k] - alpha G[k]),
        G_DD[k + n0] = s e^{-alpha k} (G_DD[k] - 2 alpha G_D[k] + alpha^2 G[k]).
    With G ~ sum a_p cos, G_D ~ sum b_p sin (p >= 1) and G_DD ~ sum d_p cos on [-L, L] the
    result weights ct_p and st_p by
        order 1: cos_coef = -alpha a_p,          sin_coef = b_p
        order 2: cos_coef = d_p + alpha^2 a_p,   sin_coef = -2 alpha b_p
    (the scale s is applied to the sum, as for the smoothing itself)."""
    if order not in (1, 2):
        raise ValueError("order must be 1 or 2")
    kind = "gd1" if order == 1 else "gd2"
    if mode == "sft":
        if order == 1:
            return Plan(kind, sigma, 0.0, K, L, 1, "sft", 0, np.zeros(K), fit_gauss_d1(sigma, K, L))
        return Plan(kind, sigma, 0.0, K, L, 0, "sft", 0, fit_gauss_d2(sigma, K, L), np.zeros(K))
    if mode != "asft":
        raise ValueError("mode must be 'sft' or 'asft'")
    if n0 is None:
        n0 = default_n0(sigma)
    alpha = n0 / (sigma * sigma)
    a = fit_gauss(sigma, K, L)
    b = np.concatenate([[0.0], fit_gauss_d1(sigma, K - 1, L) if K > 1 else np.zeros(0)])
    if order == 1:
        cc, sc = -alpha * a, b
    else:
        cc, sc = fit_gauss_d2(sigma, K, L) + alpha * alpha * a, -2.0 * alpha * b
    return Plan(kind, sigma, 0.0, K, L, 0, "asft", int(n0), cc, sc)


def plan_multiply(sigma: float, xi: float, P_M: int, L: int, mode: str = "sft",
                  n0: int | None = None) -> Plan:
    """Morlet wavelet by the multiplication method (Sec. III-B): the Gaussian envelope fitted
    with the cosines of orders 0..P_M (K = P_M + 1 terms; cos_coef holds the a_p of eq.
    aproGauss), multiplied by the carrier."""
    a = fit_gauss(sigma, P_M + 1, L)
    if mode == "asft" and n0 is None:
        n0 = default_n0(sigma)
    return Plan("mult", sigma, xi, P_M + 1, L, 0, mode, int(n0 or 0) if mode == "asft" else 0,
                a, np.zeros(P_M + 1))


# --------------------------------------------------------------------------
# The K-term kernels as explicit taps (plain definitions the method equals)
# --------------------------------------------------------------------------
def _kterm(cos_coef, sin_coef, P_S, L) -> np.ndarray:
    orders = np.arange(P_S, P_S + len(cos_coef))
    _, Bc, Bs = _basis(L, orders)
    return Bc @ cos_coef + 1j * (Bs @ sin_coef)


def kterm_morlet(plan: Plan) -> np.ndarray:
    """psi_hat[k], k = -L..L (Sec. III-A)."""
    return _kterm(plan.cos_coef, plan.sin_coef, plan.P_S, plan.L)


def kterm_gauss(plan: Plan) -> np.ndarray:
    """G_hat[k], k = -L..L (eq. aproGauss); real."""
    return _kterm(plan.cos_coef, plan.sin_coef, plan.P_S, plan.L).real


def kterm_gauss_deriv(plan: Plan) -> np.ndarray:
    """G_D_hat[k] = sum_p b_p sin(beta p k) (order 1) or G_DD_hat[k] = sum_p d_p cos(beta p k)
    (order 2), k = -L..L (Sec. II-A); real. For an ASFT plan, the unattenuated
    sum_p cos_coef_p cos(beta p k) + sin_coef_p sin(beta p k) that asft_kernel() weights."""
    t = _kterm(plan.cos_coef, plan.sin_coef, plan.P_S, plan.L)
    if plan.mode == "asft":
        return t.real + t.imag
    return t.imag if plan.kind == "gd1" else t.real


def _mult_scale(plan: Plan) -> tuple[float, float]:
    """C_xi / (pi^(1/4) sqrt(sigma)) / sqrt(gamma/pi) (the envelope is G / sqrt(gamma/pi)) and
    kappa_xi, for the multiplication method."""
    C, kappa = _morlet_consts(plan.xi * plan.sigma)
    gamma = 1.0 / (2.0 * plan.sigma * plan.sigma)
    return C / (math.pi ** 0.25 * math.sqrt(plan.sigma)) / math.sqrt(gamma / math.pi), kappa


def kterm_multiply(plan: Plan) -> np.ndarray:
    """psi_hat_M[k] = C' (e^{i xi k} - kappa) G_hat[k], k = -L..L (Sec. III-B): the sum
    sum_{p=-P}^{P} a'_p e^{i omega_p k} with omega_p = xi + beta p equals e^{i xi k} G_hat[k]."""
    ce, kappa = _mult_scale(plan)
    k = np.arange(-plan.L, plan.L + 1, dtype=np.float64)
    return ce * (np.exp(1j * plan.xi * k) - kappa) * kterm_gauss(plan)


def asft_kernel(plan: Plan) -> np.ndarray:
    """Taps h[k], k = -L..L, of the ASFT result written as a plain convolution
    y[n] = sum_k h[k] x[n - n0 - k]:
      h[k] = e^{i xi n0} e^{-n0^2/(2 sigma^2)} e^{-alpha k} khat[k]
    (eqs. siftGauss and GsASFT, Sec. III-A; alpha^2/(4 gamma) = n0^2/(2 sigma^2))."""
    k = np.arange(-plan.L, plan.L + 1, dtype=np.float64)
    if plan.kind == "mult":
        # only the carrier part is shifted: ce s e^{-alpha k} (e^{i xi (k + n0)} - kappa) G_hat[k]
        ce, kappa = _mult_scale(plan)
        scale = math.exp(-plan.n0 ** 2 / (2.0 * plan.sigma ** 2))
        return (ce * scale * np.exp(-plan.alpha * k) * (np.exp(1j * plan.xi * (k + plan.n0)) - kappa)
                * kterm_gauss(plan))
    if plan.kind == "morlet":
        base = kterm_morlet(plan)
    elif plan.kind == "gauss":
        base = kterm_gauss(plan).astype(np.complex128)
    else:
        base = kterm_gauss_deriv(plan).astype(np.complex128)
    scale = math.exp(-plan.n0 ** 2 / (2.0 * plan.sigma ** 2))
    ph = np.exp(1j * plan.xi * plan.n0) if plan.kind == "morlet" else 1.0
    return ph * scale * np.exp(-plan.alpha * k) * base


# --------------------------------------------------------------------------
# Plain convolution, x zero outside [0, N-1] (eqs. xG..xGDD)
# --------------------------------------------------------------------------
FFT_CONV_MIN = 1 << 24   # N * (2L + 1) above which the full convolution is taken by FFT


def conv_same(x: np.ndarray, h: np.ndarray, L: int, shift: int = 0) -> np.ndarray:
    """y[n] = sum_{k=-L}^{L} h[k] x[n - shift - k], n = 0..N-1 (x real or complex).

    The full linear convolution is a library primitive: np.convolve (direct sums) for small
    sizes, scipy's FFT convolution for large ones (same sums, rounding ~1e-15 of the
    largest term)."""
    x = np.asarray(x)
    x = x.astype(np.complex128 if np.iscomplexobj(x) else np.float64)
    N = x.shape[0]
    if N == 0:
        return np.zeros(0, dtype=np.result_type(h, x, np.float64))
    if N * len(h) >= FFT_CONV_MIN:
        full = fftconvolve(x, h)
    else:
        full = np.convolve(x, h)        # full[i] = sum_k h[k+L] x[i - (k+L)]
    idx = np.arange(N) - shift + L      # index of n - shift in 'full'
    out = np.zeros(N, dtype=full.dtype)
    ok = (idx >= 0) & (idx < full.shape[0])
    out[ok] = full[idx[ok]]
    return out


def conv_same_at(x: np.ndarray, h: np.ndarray, L: int, ns: np.ndarray, shift: int = 0) -> np.ndarray:
    """conv_same evaluated only at the outputs ns, one direct sum per output."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    out = np.zeros(len(ns), dtype=np.result_type(h, np.float64))
    k = np.arange(-L, L + 1)
    for i, n in enumerate(ns):
        j = n - shift - k
        ok = (j >= 0) & (j < N)
        out[i] = np.sum(h[ok] * x[j[ok]])
    return out


# --------------------------------------------------------------------------
# Kernel integral (Sec. II-B) and its attenuated version (Sec. II-D)
# --------------------------------------------------------------------------
def phase(p: int, j: np.ndarray, L: int) -> np.ndarray:
    """e^{i beta p j}, with the argument reduced exactly: beta p j = pi ((p j) mod 2L) / L."""
    r = np.mod(np.asarray(j, dtype=np.int64) * int(p), 2 * L).astype(np.float64)
    return np.exp(1j * math.pi * r / L)


def sft_component(x: np.ndarray, p: int, L: int) -> np.ndarray:
    """Z_p[n] = c_p[n] - i s_p[n] = sum_{k=-L}^{L} x[n-k] e^{-i beta p k} (eqs. cp, sp)
    computed the paper's way:
      u[n]   = u[n-1] + x[n] e^{i beta p n}               (eqs. kernel, kernelZenka)
      u_w[n] = u[n] - u[n-2L-1]                           (eqs. kernelInt, kernelInter)
      c_p[n] - i s_p[n] = e^{-i beta p n} u_w[n+L]        (SFT from the kernel integral)
    with x zero outside [0, N-1], so u is held constant beyond N-1 and is 0 below 0."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    j = np.arange(N)
    u = np.cumsum(x * phase(p, j, L))               # u[0..N-1]

    def U(idx):                                      # u extended: 0 below 0, held above N-1
        idx = np.asarray(idx)
        out = np.zeros(idx.shape, dtype=np.complex128)
        pos = idx >= 0
        out[pos] = u[np.minimum(idx[pos], N - 1)]
        return out

    n = np.arange(N)
    uw = U(n + L) - U(n - L - 1)
    return np.conj(phase(p, n, L)) * uw


def asft_component(x: np.ndarray, p: int, L: int, alpha: float, q: np.ndarray) -> np.ndarray:
    """Attenuated component Zt_p[q] = sum_{k=-L}^{L} x[q-k] e^{-alpha k} e^{-i beta p k}
    (eqs. acp, asp with the causal weight) computed by the attenuated kernel integral:
      ut[j] = e^{-alpha} ut[j-1] + x[j] e^{i beta p j}      (eq. iir1A, modulated frame)
      Zt[q] = e^{alpha L} e^{-i beta p q} (ut[q+L] - e^{-alpha(2L+1)} ut[q-L-1])
    (eq. aiir12K with the prefactor of eq. asfiir12K). Beyond N-1 the input is
    zero, so ut keeps decaying: ut[j] = ut[N-1] e^{-alpha (j-N+1)}; below 0 it is 0.
    Evaluated at the requested positions q (any integers)."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    j = np.arange(N)
    ut = lfilter([1.0], [1.0, -math.exp(-alpha)], x * phase(p, j, L))

    def U(idx):
        idx = np.asarray(idx)
        out = np.zeros(idx.shape, dtype=np.complex128)
        inr = (idx >= 0) & (idx < N)
        out[inr] = ut[idx[inr]]
        hi = idx >= N
        out[hi] = ut[N - 1] * np.exp(-alpha * (idx[hi] - (N - 1)))
        return out

    q = np.asarray(q, dtype=np.int64)
    diff = U(q + L) - math.exp(-alpha * (2 * L + 1)) * U(q - L - 1)
    return math.exp(alpha * L) * np.conj(phase(p, q, L)) * diff


def freq_component(x: np.ndarray, omega: float, L: int, alpha: float, q: np.ndarray) -> np.ndarray:
    """Component at a real frequency (Sec. III-B), Z(omega)[q] = c(omega)[q] - i s(omega)[q]
    = sum_{k=-L}^{L} x[q-k] e^{-alpha k} e^{-i omega k} (alpha = 0: SFT), by the kernel integral
    of asft_component() with the phase e^{i omega j} evaluated in float64."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    j = np.arange(N)
    ut = lfilter([1.0], [1.0, -math.exp(-alpha)], x * np.exp(1j * omega * j))

    def U(idx):
        idx = np.asarray(idx)
        out = np.zeros(idx.shape, dtype=np.complex128)
        inr = (idx >= 0) & (idx < N)
        out[inr] = ut[idx[inr]]
        hi = idx >= N
        out[hi] = ut[N - 1] * np.exp(-alpha * (idx[hi] - (N - 1)))
        return out

    q = np.asarray(q, dtype=np.int64)
    diff = U(q + L) - math.exp(-alpha * (2 * L + 1)) * U(q - L - 1)
    return math.exp(alpha * L) * np.exp(-1j * omega * q) * diff


def _forward_multiply(x: np.ndarray, plan: Plan) -> np.ndarray:
    """x_M[n] = C' [ sum_{p=-P}^{P} a'_p (c(omega_p) + i s(omega_p)) - kappa sum_{p=0}^{P} a_p c_p ]
    with a'_0 = a_0, a'_{+-p} = a_p / 2 and omega_p = xi + beta p (Sec. III-B). For real x,
    c(omega) + i s(omega) = conj Z(omega). ASFT: the components are the attenuated ones read at
    n - n0, the sum is scaled by e^{-n0^2/(2 sigma^2)} and the carrier sum by e^{i xi n0}."""
    N = x.shape[0]
    if N == 0:
        return np.zeros(0, dtype=np.complex128)
    q = np.arange(N) - plan.n0
    P = plan.K - 1
    a = plan.cos_coef
    carrier = np.zeros(N, dtype=np.complex128)
    for p in range(-P, P + 1):
        ap = a[0] if p == 0 else 0.5 * a[abs(p)]
        carrier += ap * np.conj(freq_component(x, plan.xi + plan.beta * p, plan.L, plan.alpha, q))
    gauss = np.zeros(N)
    for p in range(P + 1):
        if plan.mode == "sft":
            Z = sft_component(x, p, plan.L)
        else:
            Z = asft_component(x, p, plan.L, plan.alpha, q)
        gauss += a[p] * Z.real
    ce, kappa = _mult_scale(plan)
    if plan.mode == "asft":
        s = math.exp(-plan.n0 ** 2 / (2.0 * plan.sigma ** 2))
        return ce * s * (np.exp(1j * plan.xi * plan.n0) * carrier - kappa * gauss)
    return ce * (carrier - kappa * gauss)


def forward(x: np.ndarray, plan: Plan) -> np.ndarray:
    """Method result.

    Morlet, SFT:  x_M[n] = sum_p m_p c_p[n] + i l_p s_p[n]            (Sec. III-A)
    Morlet, ASFT: x_M[n] = e^{i xi n0} e^{-n0^2/(2 sigma^2)}
                           sum_p m_p ct_p[n-n0] + i l_p st_p[n-n0]
    Gauss,  SFT:  x_G[n] = sum_p a_p c_p[n]                            (eq. GsSFT)
    Gauss,  ASFT: x_G[n] = e^{-n0^2/(2 sigma^2)} sum_p a_p ct_p[n-n0]  (eq. GsASFT)
    GD,     SFT:  x_GD[n] = sum_{p=1}^{K} b_p s_p[n]                 (Sec. II-A)
    GDD,    SFT:  x_GDD[n] = sum_{p=0}^{K-1} d_p c_p[n]              (Sec. II-A)
    GD/GDD, ASFT: e^{-n0^2/(2 sigma^2)} sum_{p=0}^{K-1} cos_coef_p ct_p[n-n0]
                                                 + sin_coef_p st_p[n-n0]  (eq. gddAsft)
    Mult:         _forward_multiply (Sec. III-B)
    with c - i s = Z, so c = Re Z and s = -Im Z."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    if plan.kind == "mult":
        return _forward_multiply(x, plan)
    if plan.kind in ("gd1", "gd2"):
        out = np.zeros(N)
        for i, p in enumerate(plan.orders):
            if N == 0:
                break
            if plan.mode == "sft":
                Z = sft_component(x, int(p), plan.L)
                out += plan.sin_coef[i] * (-Z.imag) if plan.kind == "gd1" else plan.cos_coef[i] * Z.real
            else:
                Zt = asft_component(x, int(p), plan.L, plan.alpha, np.arange(N) - plan.n0)
                out += plan.cos_coef[i] * Zt.real + plan.sin_coef[i] * (-Zt.imag)
        if plan.mode == "asft":
            out *= math.exp(-plan.n0 ** 2 / (2.0 * plan.sigma ** 2))
        return out
    acc = np.zeros(N, dtype=np.complex128)
    if N == 0:
        return acc if plan.kind == "morlet" else acc.real
    for i, p in enumerate(plan.orders):
        if plan.mode == "sft":
            Z = sft_component(x, int(p), plan.L)
        else:
            Z = asft_component(x, int(p), plan.L, plan.alpha, np.arange(N) - plan.n0)
        acc += plan.cos_coef[i] * Z.real - 1j * plan.sin_coef[i] * Z.imag
    if plan.mode == "asft":
        acc *= math.exp(-plan.n0 ** 2 / (2.0 * plan.sigma ** 2))
        if plan.kind == "morlet":
            acc *= np.exp(1j * plan.xi * plan.n0)
    return acc if plan.kind == "morlet" else acc.real


def forward_direct(x: np.ndarray, sigma: float, xi: float | None, L: int, deriv: int = 0) -> np.ndarray:
    """Truncated direct convolution with the exact kernel on [-L, L] (eqs. xG..xGDD; the
    comparison method of Sec. V-B uses the window [-3 sigma, 3 sigma]). deriv = 1, 2 take
    the Gaussian's first and second differentials."""
    k = np.arange(-L, L + 1)
    if xi is not None:
        h = morlet(sigma, xi, k)
    else:
        h = (gaussian, gaussian_d1, gaussian_d2)[deriv](sigma, k)
    return conv_same(x, h, L)


# --------------------------------------------------------------------------
# Differentiation (no counterpart in the paper; derived from the forward map)
# --------------------------------------------------------------------------
def _taps_and_shift(plan: Plan) -> tuple[np.ndarray, int]:
    if plan.mode == "asft":
        return asft_kernel(plan), plan.n0
    if plan.kind == "mult":
        return kterm_multiply(plan), 0
    if plan.kind in ("gd1", "gd2"):
        return kterm_gauss_deriv(plan), 0
    base = kterm_morlet(plan) if plan.kind == "morlet" else kterm_gauss(plan)
    return base, 0


def adjoint(g: np.ndarray, plan: Plan) -> np.ndarray:
    """Transpose of the real-input forward map W = A x for a real-valued loss.

    With W[n] = sum_k h[k] x[n - s - k] and g = dLoss/dRe W + i dLoss/dIm W,
      dLoss/dx[j] = Re sum_n conj(g[n]) h[n - s - j] = Re sum_k conj(h[k]) g[j + s + k].
    Written as a plain sum over the taps."""
    h, s = _taps_and_shift(plan)
    g = np.asarray(g, dtype=np.complex128)
    # sum_k conj(h[k]) g[j + s + k] = sum_k' conj(h[-k']) g[(j + s) - k']: a convolution with
    # the reversed conjugate taps, read s samples later
    return conv_same(g, np.conj(np.asarray(h)[::-1]), plan.L, shift=-s).real


def _jacobian(plan: Plan) -> np.ndarray:
    """d(cos_coef, sin_coef)/d(sigma, xi) for the frozen basis (L, P_S, K fixed):
    the MMSE coefficients are linear in the target, c = pinv(B) target, so
    dc/dtheta = pinv(B) dtarget/dtheta. Returns array [2K, 2] (rows: m then l)."""
    k, Bc, Bs = _basis(plan.L, plan.orders)
    if plan.kind == "morlet":
        ds, dx = dpsi_dtheta(plan.sigma, plan.xi, k)
        cols = []
        for d in (ds, dx):
            cols.append(np.concatenate([_lstsq(Bc, d.real), _lstsq(Bs, d.imag)]))
        return np.stack(cols, axis=1)
    # Gaussian: dG/dsigma = G (k^2/sigma^3 - 1/sigma); no xi
    G = gaussian(plan.sigma, k)
    dG = G * (k * k / plan.sigma ** 3 - 1.0 / plan.sigma)
    return np.stack([np.concatenate([_lstsq(Bc, dG), np.zeros(plan.K)]),
                     np.zeros(2 * plan.K)], axis=1)


def param_grads(x: np.ndarray, g: np.ndarray, plan: Plan) -> np.ndarray:
    """[dLoss/dsigma, dLoss/dxi] with (L, P_S, n0, K) frozen, for a real loss with
    complex cotangent g = dLoss/dRe W + i dLoss/dIm W:
        dLoss/dtheta = Re sum_n conj(g[n]) dW[n]/dtheta,
    where W is a plain convolution whose taps depend on theta through the fitted
    coefficients and, for ASFT, through alpha = n0/sigma^2, the scale
    e^{-n0^2/(2 sigma^2)} and the phase e^{i xi n0}."""
    J = _jacobian(plan)
    K, L = plan.K, plan.L
    k = np.arange(-L, L + 1, dtype=np.float64)
    g = np.asarray(g, dtype=np.complex128)
    out = np.zeros(2)
    for t in range(2):
        dcos, dsin = J[:K, t], J[K:, t]
        dbase = _kterm(dcos, dsin, plan.P_S, L)
        if plan.kind == "gauss":
            dbase = dbase.real.astype(np.complex128)
        if plan.mode == "asft":
            base = kterm_morlet(plan) if plan.kind == "morlet" else kterm_gauss(plan).astype(np.complex128)
            n0, sig = plan.n0, plan.sigma
            scale = math.exp(-n0 ** 2 / (2 * sig ** 2))
            ph = np.exp(1j * plan.xi * n0) if plan.kind == "morlet" else 1.0
            att = np.exp(-plan.alpha * k)
            dh = ph * scale * att * dbase
            if t == 0:   # sigma also moves alpha = n0/sigma^2 and the scale
                dalpha = -2.0 * n0 / sig ** 3
                dscale = scale * (n0 ** 2 / sig ** 3)
                dh = dh + ph * dscale * att * base + ph * scale * (-k * dalpha) * att * base
            elif plan.kind == "morlet":   # xi moves the phase
                dh = dh + (1j * n0) * ph * scale * att * base
            dW = conv_same(x, dh, L, shift=n0)
        else:
            dW = conv_same(x, dbase, L)
            if plan.kind == "gauss":
                dW = dW.real
        out[t] = np.sum((np.conj(g) * dW).real)
    return out


# --------------------------------------------------------------------------
# Images: separable 2-D Gaussian smoothing (Sec. IV: the lines of an image are filtered
# independently, rows then columns)
# --------------------------------------------------------------------------
def _lines(fn, items, map_lines):
    return list(map_lines(fn, items)) if map_lines is not None else [fn(v) for v in items]


def gauss_smooth_2d(img: np.ndarray, plan_x: Plan, plan_y: Plan, map_lines=None) -> np.ndarray:
    """y = G_y *_columns (G_x *_rows img) for an H x W image (row-major, x along a row), each
    line by forward() with the axis's plan. map_lines(fn, lines), if given, applies fn to every
    line (the lines are independent, so a caller may spread them over processes)."""
    img = np.asarray(img, dtype=np.float64)
    H, W = img.shape
    if H == 0 or W == 0:
        return np.zeros((H, W))
    rows = np.stack(_lines(partial(forward, plan=plan_x), list(img), map_lines))
    cols = _lines(partial(forward, plan=plan_y), list(np.ascontiguousarray(rows.T)), map_lines)
    return np.stack(cols, axis=1)


def gabor_2d(img: np.ndarray, plan_x: Plan, plan_y: Plan, map_lines=None) -> np.ndarray:
    """Separable 2-D Gabor filter of a real H x W image: the Morlet transform of every row
    (plan_x, complex), then the Gaussian smoothing of every column of its real and imaginary
    parts (plan_y), the lines filtered independently (Sec. IV). map_lines as for
    gauss_smooth_2d."""
    img = np.asarray(img, dtype=np.float64)
    H, W = img.shape
    if H == 0 or W == 0:
        return np.zeros((H, W), dtype=np.complex128)
    rows = np.stack(_lines(partial(forward, plan=plan_x), list(img), map_lines))
    cT = np.ascontiguousarray(rows.T)
    re = _lines(partial(forward, plan=plan_y), list(cT.real.copy()), map_lines)
    im = _lines(partial(forward, plan=plan_y), list(cT.imag.copy()), map_lines)
    return np.stack(re, axis=1) + 1j * np.stack(im, axis=1)


def gabor_2d_adjoint(g: np.ndarray, plan_x: Plan, plan_y: Plan) -> np.ndarray:
    """Transpose of gabor_2d for a real loss, g = dLoss/dRe y + i dLoss/dIm y (H x W): the
    column pass's adjoint on the real and imaginary parts of every column, then the row pass's
    adjoint (adjoint()) of every row's complex cotangent."""
    g = np.asarray(g, dtype=np.complex128)
    H, W = g.shape
    if H == 0 or W == 0:
        return np.zeros((H, W))
    cols = [adjoint(g[:, c].real, plan_y) + 1j * adjoint(g[:, c].imag, plan_y) for c in range(W)]
    g1 = np.stack(cols, axis=1)
    return np.stack([adjoint(g1[r], plan_x) for r in range(H)])


# --------------------------------------------------------------------------
# The paper's GPU route (Sec. IV): window sums by binary doubling (Algorithm 1)
# --------------------------------------------------------------------------
def sliding_sum(f: np.ndarray, Lw: int) -> np.ndarray:
    """h[n] = sum_{k=0}^{Lw-1} f[n+k] for every n, f zero past its end: the window sums
    that Algorithm 1 forms by binary doubling, taken here from their definition (a
    correlation with Lw ones; scipy's FFT convolution for long windows, a library
    primitive for the same sums)."""
    f = np.asarray(f)
    M = f.shape[0]
    if M == 0 or Lw <= 0:
        return np.zeros_like(f)
    ones = np.ones(Lw)
    if M * Lw <= (1 << 24):
        full = np.convolve(f, ones)            # full[i] = sum_{k=0}^{Lw-1} f[i-k]
    else:
        full = fftconvolve(f, ones)
    # h[n] = full[n + Lw - 1] (terms past the end of f are zero)
    out = np.zeros_like(f)
    src = full[Lw - 1:Lw - 1 + M]
    out[:src.shape[0]] = src
    return out


def forward_tree(x: np.ndarray, plan: Plan) -> np.ndarray:
    """SFT Morlet (or Gaussian) result by the route of Sec. IV: per order p the window sum
    S_p[n] = sum_{j=n-L}^{n+L} x[j] e^{i beta p j} by sliding_sum() of f_p[m] = x[m-L] e^{i beta p (m-L)},
    then Z_p[n] = e^{-i beta p n} S_p[n] and the K-term combination of forward()."""
    if plan.mode != "sft":
        raise ValueError("the sliding-sum route is the SFT form")
    x = np.asarray(x, dtype=np.float64)
    N, L = x.shape[0], plan.L
    acc = np.zeros(N, dtype=np.complex128)
    if N == 0:
        return acc if plan.kind == "morlet" else acc.real
    m = np.arange(N + 2 * L)
    j = m - L
    xm = np.where((j >= 0) & (j < N), np.concatenate([np.zeros(L), x, np.zeros(L)]), 0.0)
    for i, p in enumerate(plan.orders):
        h = sliding_sum(xm * phase(int(p), j, L), 2 * L + 1)[:N]
        Z = np.conj(phase(int(p), np.arange(N), L)) * h
        acc += plan.cos_coef[i] * Z.real - 1j * plan.sin_coef[i] * Z.imag
    return acc if plan.kind == "morlet" else acc.real


# --------------------------------------------------------------------------
# Edge extension (Sec. II: x beyond [0, N-1] is zero or the value on the edge)
# --------------------------------------------------------------------------
def forward_edge(x: np.ndarray, plan: Plan) -> np.ndarray:
    """forward() with x extended by its edge values instead of zeros: every output n reads
    x[n - n0 - k] for |k| <= L, i.e. at most 2L samples outside [0, N-1] on either side, so x is
    padded by 2L copies of x[0] and of x[N-1] and the central N outputs are kept."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    if N == 0:
        return forward(x, plan)
    P = 2 * plan.L
    return forward(np.pad(x, (P, P), mode="edge"), plan)[P:P + N]

