"""The C ABI without a GPU: the library loads, exports every symbol include/morlet.h
declares, builds plans whose coefficients match the oracle's independent fit, and rejects
bad arguments before anything is launched."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from oracle import morlet_oracle as O
from paper_2110_11866_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "morlet.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"^\s*#.*$", "", src, flags=re.M)   # preprocessor lines (macros are not symbols)
    return sorted(set(re.findall(r"\b(\w+)\s*\(", src)) - {"defined", "if", "return", "sizeof"})


def test_library_exports_every_declared_function():
    L = _abi.lib()
    names = _header_functions()
    assert "morlet_forward" in names and "gauss_smooth" in names
    for n in names:
        assert hasattr(L, n), n
        assert n in _abi.SIGNATURES, n


@pytest.mark.parametrize("sigma,K,L", [(16.0, 4, 64), (8192.0, 6, 32768), (37.5, 5, 100), (3.0, 7, 12)])
def test_plan_matches_oracle_fit(sigma, K, L):
    xi = 6.0 / sigma
    h = _abi.morlet_plan(1000, sigma, xi, K, L)
    try:
        info = _abi.morlet_plan_info(h, K)
    finally:
        _abi.morlet_destroy(h)
    p = O.plan_morlet(sigma, xi, K, L)
    assert info["P_S"] == p.P_S
    assert info["L"] == L
    scale = np.abs(p.cos_coef).max()
    assert np.allclose(info["cos_coef"], p.cos_coef, rtol=1e-10, atol=1e-12 * scale)
    assert np.allclose(info["sin_coef"], p.sin_coef, rtol=1e-10, atol=1e-12 * scale)
    k = np.arange(-L, L + 1)
    assert math.isclose(info["kernel_relrmse"], O.kernel_relrmse(O.kterm_morlet(p), O.morlet(sigma, xi, k)),
                        rel_tol=1e-9)


@pytest.mark.parametrize("xi0", [1.0, 2.0, 4.0, 10.0, 20.0])
def test_plan_PS_matches_oracle_over_xi(xi0):
    sigma, K, L = 60.0, 6, 180
    h = _abi.morlet_plan(10, sigma, xi0 / sigma, K, L)
    ps = _abi.morlet_plan_info(h, K)["P_S"]
    _abi.morlet_destroy(h)
    assert ps == O.select_PS(sigma, xi0 / sigma, K, L)


def test_gauss_plan_matches_oracle():
    for sigma, K, L in [(16.0, 4, 64), (100.0, 6, 350), (2.0, 3, 5)]:
        h = _abi.morlet_plan_gauss(100, sigma, K, L)
        info = _abi.morlet_plan_info(h, K)
        _abi.morlet_destroy(h)
        a = O.fit_gauss(sigma, K, L)
        assert np.allclose(info["cos_coef"], a, rtol=1e-10, atol=1e-14)
        assert np.allclose(info["sin_coef"], 0.0)


def test_differential_plans_match_oracle():
    for sigma, K, L in [(16.0, 4, 64), (60.0, 6, 256), (3.0, 5, 9)]:
        for order, fit in ((1, O.fit_gauss_d1), (2, O.fit_gauss_d2)):
            h = _abi.morlet_plan_gauss_deriv(100, sigma, K, L, order)
            info = _abi.morlet_plan_info(h, K)
            _abi.morlet_destroy(h)
            c = fit(sigma, K, L)
            got, zero = (info["sin_coef"], info["cos_coef"]) if order == 1 else (info["cos_coef"], info["sin_coef"])
            assert info["P_S"] == (1 if order == 1 else 0)
            assert np.allclose(got, c, rtol=1e-10, atol=1e-15), (order, got, c)
            assert np.allclose(zero, 0.0)


def test_differential_plan_errors():
    L = _abi.lib()
    h = ctypes.c_void_p()
    assert L.morlet_plan_gauss_deriv(ctypes.byref(h), 100, 4.0, 4, 16, 3) == _abi.MORLET_ERR_INVALID_ARG
    assert L.morlet_plan_gauss_deriv(ctypes.byref(h), 100, 4.0, 6, 5, 1) == _abi.MORLET_ERR_INVALID_ARG
    assert L.morlet_plan_gauss_deriv(ctypes.byref(h), 100, 4.0, 6, 5, 2) == _abi.MORLET_OK
    hp = h.value
    try:
        assert L.morlet_plan_set(hp, _abi.MORLET_SCAN_ASFT, 6, 0) == _abi.MORLET_ERR_INVALID_ARG   # n0 > L
        assert L.morlet_plan_set(hp, _abi.MORLET_SCAN_SFT, 0, 1) == _abi.MORLET_OK
        fake = 1 << 20
        # dLoss/dx only: parameter gradients are refused, a short workspace too
        assert L.gauss_smooth_backward(hp, fake, 0, fake, fake, fake, fake, 1 << 30, None) == _abi.MORLET_ERR_UNSUPPORTED
        assert L.gauss_smooth_backward(hp, fake, 0, fake, fake, None, fake, 100, None) == _abi.MORLET_ERR_WORKSPACE
        assert L.morlet_plan_set(hp, _abi.MORLET_SCAN_ASFT, 0, 0) == _abi.MORLET_OK
        assert L.gauss_smooth_backward(hp, fake, 0, fake, fake, fake, fake, 1 << 30, None) == _abi.MORLET_ERR_UNSUPPORTED
        assert L.gauss_smooth_backward(hp, fake, 0, fake, fake, None, fake, 100, None) == _abi.MORLET_ERR_WORKSPACE
        s0 = _abi.morlet_backward_workspace_size(hp)
        assert s0 >= 2 * 100 * 4
        assert L.morlet_plan_set_boundary(hp, 1) == _abi.MORLET_OK
        # edge extension: two buffers of the padded row (N + 4L float32 each) on top of the tile states
        assert _abi.morlet_backward_workspace_size(hp) >= s0 + 4 * 5 * 4
        assert L.gauss_smooth_backward(hp, fake, 0, fake, fake, None, fake, s0, None) == _abi.MORLET_ERR_WORKSPACE
        assert L.gauss_smooth_backward(hp, fake, 0, fake, fake, fake, fake, 1 << 30, None) == _abi.MORLET_ERR_UNSUPPORTED
    finally:
        _abi.morlet_destroy(hp)


def test_asft_differential_plans_match_oracle():
    # refit on morlet_plan_set(ASFT): orders 0..K-1, both weight vectors as eq. gddAsft gives
    # them, the reported error that of the attenuated taps against the shifted differential;
    # SFT again restores the SFT fit
    for sigma, K, L, n0 in [(16.0, 4, 64, 2), (60.0, 6, 256, 10), (3.0, 5, 9, 1), (40.0, 1, 120, 5)]:
        for order in (1, 2):
            h = _abi.morlet_plan_gauss_deriv(100, sigma, K, L, order)
            try:
                _abi.morlet_plan_set(h, _abi.MORLET_SCAN_ASFT, n0, 0)
                info = _abi.morlet_plan_info(h, K)
                pl = O.plan_gauss_deriv(sigma, K, L, order, mode="asft", n0=n0)
                assert info["P_S"] == 0 and info["n0"] == n0
                assert abs(info["alpha"] - n0 / sigma ** 2) < 1e-15
                scale = max(np.abs(pl.cos_coef).max(), np.abs(pl.sin_coef).max())
                assert np.allclose(info["cos_coef"], pl.cos_coef, rtol=1e-9, atol=1e-12 * scale), (order, sigma, K)
                assert np.allclose(info["sin_coef"], pl.sin_coef, rtol=1e-9, atol=1e-12 * scale), (order, sigma, K)
                k = np.arange(-L, L + 1)
                want = (O.gaussian_d1 if order == 1 else O.gaussian_d2)(sigma, k + n0)
                err = np.linalg.norm(O.asft_kernel(pl).real - want) / np.linalg.norm(want)
                assert abs(info["kernel_relrmse"] / err - 1) < 1e-8, (info["kernel_relrmse"], err)
                _abi.morlet_plan_set(h, _abi.MORLET_SCAN_SFT, 0, 0)
                info = _abi.morlet_plan_info(h, K)
                c = (O.fit_gauss_d1 if order == 1 else O.fit_gauss_d2)(sigma, K, L)
                assert info["P_S"] == (1 if order == 1 else 0)
                assert np.allclose(info["sin_coef"] if order == 1 else info["cos_coef"], c, rtol=1e-9,
                                   atol=1e-12 * np.abs(c).max())
            finally:
                _abi.morlet_destroy(h)


def test_jacobian_matches_oracle():
    sigma, xi, K, L = 8.0, 0.75, 5, 32
    h = _abi.morlet_plan(100, sigma, xi, K, L)
    jac = np.array(_abi.morlet_plan_info(h, K)["jac"]).reshape(4, K)
    _abi.morlet_destroy(h)
    J = O._jacobian(O.plan_morlet(sigma, xi, K, L))   # [2K, 2]: rows m then l, cols sigma, xi
    assert np.allclose(jac[0], J[:K, 0], rtol=1e-9, atol=1e-13)
    assert np.allclose(jac[1], J[:K, 1], rtol=1e-9, atol=1e-13)
    assert np.allclose(jac[2], J[K:, 0], rtol=1e-9, atol=1e-13)
    assert np.allclose(jac[3], J[K:, 1], rtol=1e-9, atol=1e-13)


def test_error_optimal_window_rule():
    # L = 0: the window of smallest kernel error on the grid round(c sigma), c = 1.50..5.00
    # step 0.02 (coarse step 0.10, then 0.02 around the best), recomputed with the oracle.
    sigma, K = 20.0, 5
    h = _abi.morlet_plan(10, sigma, 6 / sigma, K, 0)
    L = _abi.morlet_plan_info(h, K)["L"]
    _abi.morlet_destroy(h)

    def err(ci):
        Lc = max(int(round((1.5 + 0.02 * ci) * sigma)), K)
        ps = O.select_PS(sigma, 6 / sigma, K, Lc)
        m, l = O.fit_morlet(sigma, 6 / sigma, K, Lc, ps)
        k = np.arange(-Lc, Lc + 1)
        return O.kernel_relrmse(O._kterm(m, l, ps, Lc), O.morlet(sigma, 6 / sigma, k)), Lc

    coarse = min(range(0, 176, 5), key=lambda c: err(c)[0])
    fine = min(range(max(0, coarse - 5), min(175, coarse + 5) + 1), key=lambda c: (err(c)[0], c))
    assert L == err(fine)[1]


def test_invalid_arguments_rejected():
    h = ctypes.c_void_p()
    L = _abi.lib()
    assert L.morlet_plan(ctypes.byref(h), -1, 1.0, 1.0, 4, 64) == _abi.MORLET_ERR_INVALID_ARG
    assert L.morlet_plan(ctypes.byref(h), 10, 0.0, 1.0, 4, 64) == _abi.MORLET_ERR_INVALID_ARG
    assert L.morlet_plan(ctypes.byref(h), 10, float("nan"), 1.0, 4, 64) == _abi.MORLET_ERR_INVALID_ARG
    assert L.morlet_plan(ctypes.byref(h), 10, 4.0, -1.0, 4, 64) == _abi.MORLET_ERR_INVALID_ARG
    assert L.morlet_plan(ctypes.byref(h), 10, 4.0, 1.0, 0, 64) == _abi.MORLET_ERR_INVALID_ARG
    assert L.morlet_plan(ctypes.byref(h), 10, 4.0, 1.0, 13, 64) == _abi.MORLET_ERR_INVALID_ARG
    assert L.morlet_plan(ctypes.byref(h), 10, 4.0, 1.0, 6, 5) == _abi.MORLET_ERR_INVALID_ARG
    assert L.morlet_plan(None, 10, 4.0, 1.0, 4, 64) == _abi.MORLET_ERR_INVALID_ARG
    assert L.morlet_plan_gauss(ctypes.byref(h), 10, 4.0, 8, 5) == _abi.MORLET_ERR_INVALID_ARG
    assert "K" in _abi.morlet_last_error()


def test_call_errors_before_launch():
    L = _abi.lib()
    h = _abi.morlet_plan(4096, 16.0, 6 / 16, 4, 64)
    hg = _abi.morlet_plan_gauss(4096, 16.0, 4, 64)
    try:
        need = _abi.morlet_workspace_size(h)
        fake = 1 << 20   # never dereferenced: every call below fails its checks first
        assert L.morlet_forward(h, None, 0, fake, fake, need, None) == _abi.MORLET_ERR_INVALID_ARG
        assert L.morlet_forward(h, fake, 0, fake, fake, need - 1, None) == _abi.MORLET_ERR_WORKSPACE
        assert L.morlet_forward(h, fake, 7, fake, fake, need, None) == _abi.MORLET_ERR_UNSUPPORTED
        assert L.morlet_forward(hg, fake, 0, fake, fake, need, None) == _abi.MORLET_ERR_INVALID_ARG
        assert L.gauss_smooth(h, fake, 0, fake, fake, need, None) == _abi.MORLET_ERR_INVALID_ARG
        assert L.morlet_plan_set(h, 5, 0, 0) == _abi.MORLET_ERR_UNSUPPORTED
        assert L.morlet_plan_set(h, 1, 65, 0) == _abi.MORLET_ERR_INVALID_ARG
        assert L.morlet_plan_set(h, 1, 0, 9) == _abi.MORLET_ERR_UNSUPPORTED
        assert L.morlet_forward(None, fake, 0, fake, fake, need, None) == _abi.MORLET_ERR_INVALID_ARG
        assert L.morlet_plan_set_schedule(h, 4) == _abi.MORLET_ERR_INVALID_ARG
        assert L.morlet_plan_set_schedule(h, _abi.MORLET_SCHED_SEGMENTS) == _abi.MORLET_OK
        assert L.morlet_plan_set_segments(h, -1) == _abi.MORLET_ERR_INVALID_ARG
        assert L.morlet_plan_set_segments(h, 4097) == _abi.MORLET_ERR_INVALID_ARG
        assert L.morlet_plan_set_segments(h, 7) == _abi.MORLET_OK
        assert L.morlet_plan_set_schedule(None, 0) == _abi.MORLET_ERR_INVALID_ARG
        assert L.morlet_plan_set_schedule(h, _abi.MORLET_SCHED_ROWS) == _abi.MORLET_OK
        assert L.morlet_plan_autotune(h, fake, 0, fake, 0, None, None, None) == _abi.MORLET_ERR_INVALID_ARG
        assert L.morlet_plan_autotune(h, fake, 7, fake, 3, None, None, None) == _abi.MORLET_ERR_UNSUPPORTED
        assert L.morlet_plan_autotune(None, fake, 0, fake, 3, None, None, None) == _abi.MORLET_ERR_INVALID_ARG
    finally:
        _abi.morlet_destroy(h)
        _abi.morlet_destroy(hg)


def test_empty_signal_is_a_noop():
    h = _abi.morlet_plan(0, 16.0, 6 / 16, 4, 64)
    try:
        assert _abi.lib().morlet_forward(h, None, 0, None, None, 0, None) == _abi.MORLET_OK
    finally:
        _abi.morlet_destroy(h)


def test_asft_shift_and_alpha_reported():
    h = _abi.morlet_plan(100, 16.0, 6 / 16, 4, 64)
    try:
        _abi.morlet_plan_set(h, _abi.MORLET_SCAN_ASFT, 0, 0)
        info = _abi.morlet_plan_info(h, 4)
        assert info["n0"] == O.default_n0(16.0)
        assert math.isclose(info["alpha"], info["n0"] / 16.0 ** 2)
        _abi.morlet_plan_set(h, _abi.MORLET_SCAN_ASFT, 5, 0)
        assert _abi.morlet_plan_info(h, 4)["n0"] == 5
        _abi.morlet_plan_set(h, _abi.MORLET_SCAN_SFT, 0, 0)
        assert _abi.morlet_plan_info(h, 4)["n0"] == 0
    finally:
        _abi.morlet_destroy(h)


def test_plan_sweep_matches_oracle():
    # seeded sweep over sigma, xi0, K and the window: P_S and the fitted coefficients of the
    # library's host plan against the oracle's independent least-squares fit
    rng = np.random.default_rng(2024)
    for _ in range(40):
        sigma = float(np.exp(rng.uniform(np.log(1.5), np.log(3000.0))))
        K = int(rng.integers(1, 13))
        xi0 = float(rng.uniform(1.0, 8.0))
        L = max(K + 1, int(sigma * rng.uniform(1.5, 5.0)))
        h = _abi.morlet_plan(100, sigma, xi0 / sigma, K, L)
        info = _abi.morlet_plan_info(h, K)
        _abi.morlet_destroy(h)
        ps = O.select_PS(sigma, xi0 / sigma, K, L)
        assert info["P_S"] == ps, (sigma, K, xi0, L)
        m, l = O.fit_morlet(sigma, xi0 / sigma, K, L, ps)
        scale = max(np.abs(m).max(), np.abs(l).max())
        assert np.allclose(info["cos_coef"], m, rtol=1e-9, atol=1e-12 * scale), (sigma, K, xi0, L)
        assert np.allclose(info["sin_coef"], l, rtol=1e-9, atol=1e-12 * scale), (sigma, K, xi0, L)
        for order in (1, 2):
            Kd = min(K, L - 1) if order == 1 else K
            hd = _abi.morlet_plan_gauss_deriv(100, sigma, Kd, L, order)
            di = _abi.morlet_plan_info(hd, Kd)
            _abi.morlet_destroy(hd)
            c = (O.fit_gauss_d1 if order == 1 else O.fit_gauss_d2)(sigma, Kd, L)
            got = di["sin_coef"] if order == 1 else di["cos_coef"]
            assert np.allclose(got, c, rtol=1e-9, atol=1e-12 * np.abs(c).max()), (order, sigma, Kd, L)


def test_tile_shapes_and_workspace():
    # R in {4, 8, 16, 32}; the tile count (and the workspace's tile states) scales with 1/R
    L = _abi.lib()
    h = _abi.morlet_plan(100000, 50.0, 6.0 / 50.0, 5, 200)
    try:
        sizes = {}
        for R in (4, 8, 16, 32):
            assert L.morlet_plan_set_tile(h, R) == _abi.MORLET_OK
            sizes[R] = _abi.morlet_workspace_size(h)
        for R in (0, 2, 12, 64):
            assert L.morlet_plan_set_tile(h, R) == _abi.MORLET_ERR_UNSUPPORTED
        assert sizes[4] > sizes[8] > sizes[16] > sizes[32]
    finally:
        _abi.morlet_destroy(h)


def test_multiply_plan_matches_oracle():
    # envelope fit a_p (orders 0..P_M), window as the Gaussian fit's, and the reported kernel
    # error of psi_hat_M = C' (e^{i xi k} - kappa) G_hat against psi on [-L, L]
    for sigma, xi0, PM, L in [(16.0, 6.0, 3, 0), (60.0, 2.0, 2, 200), (300.0, 6.0, 4, 0)]:
        h = _abi.morlet_plan_multiply(1000, sigma, xi0 / sigma, PM, L)
        try:
            info = _abi.morlet_plan_info(h, PM + 1)
            _abi.morlet_plan_set(h, _abi.MORLET_SCAN_ASFT, 0, 0)
            ia = _abi.morlet_plan_info(h, PM + 1)
        finally:
            _abi.morlet_destroy(h)
        if L == 0:
            hg = _abi.morlet_plan_gauss(1000, sigma, PM + 1, 0)
            L = _abi.morlet_plan_info(hg, PM + 1)["L"]
            _abi.morlet_destroy(hg)
        assert info["L"] == L and info["P_S"] == 0 and info["n0"] == 0
        pl = O.plan_multiply(sigma, xi0 / sigma, PM, L)
        assert np.allclose(info["cos_coef"], pl.cos_coef, rtol=1e-10, atol=1e-14)
        assert np.allclose(info["sin_coef"], 0.0)
        k = np.arange(-L, L + 1)
        psi = O.morlet(sigma, xi0 / sigma, k)
        err = np.linalg.norm(O.kterm_multiply(pl) - psi) / np.linalg.norm(psi)
        assert abs(info["kernel_relrmse"] / err - 1) < 1e-8, (info["kernel_relrmse"], err)
        assert ia["n0"] == O.default_n0(sigma) and abs(ia["alpha"] - ia["n0"] / sigma ** 2) < 1e-15


def test_multiply_plan_errors_and_workspace():
    L = _abi.lib()
    h = ctypes.c_void_p()
    bad = [(100, 4.0, 0.5, -1, 0), (100, 4.0, 0.5, 12, 0), (100, 4.0, 0.0, 2, 0), (100, 4.0, 0.5, 3, 2),
           (-1, 4.0, 0.5, 2, 0), (100, -4.0, 0.5, 2, 0)]
    for args in bad:
        assert L.morlet_plan_multiply(ctypes.byref(h), *args) == _abi.MORLET_ERR_INVALID_ARG, args
    assert L.morlet_plan_multiply(ctypes.byref(h), 5000, 20.0, 0.3, 3, 0) == _abi.MORLET_OK
    hp = h.value
    try:
        assert _abi.morlet_workspace_size(hp) >= 6 * 5000 * 4
        fake = 1 << 20
        assert L.morlet_backward(hp, fake, 0, fake, fake, fake, fake, 1 << 30, None) == _abi.MORLET_ERR_UNSUPPORTED
        assert L.morlet_backward(hp, None, 0, fake, fake, None, fake, 100, None) == _abi.MORLET_ERR_WORKSPACE
        assert L.gauss_smooth_backward(hp, None, 0, fake, fake, None, fake, 1 << 30, None) == _abi.MORLET_ERR_INVALID_ARG
        assert _abi.morlet_backward_workspace_size(hp) >= max(_abi.morlet_workspace_size(hp), 6 * 5000 * 4)
        assert L.gauss_smooth(hp, fake, 0, fake, fake, 1 << 30, None) == _abi.MORLET_ERR_INVALID_ARG
        assert L.morlet_direct_forward(hp, fake, 0, fake, 0, None) == _abi.MORLET_ERR_INVALID_ARG
        assert L.morlet_forward(hp, fake, 0, fake, fake, 100, None) == _abi.MORLET_ERR_WORKSPACE
        assert L.morlet_forward(hp, fake, 5, fake, fake, 1 << 30, None) == _abi.MORLET_ERR_UNSUPPORTED
        for R in (4, 8, 16, 32):
            assert L.morlet_plan_set_tile(hp, R) == _abi.MORLET_OK
    finally:
        _abi.morlet_destroy(hp)


def test_image_plan_axes_match_oracle():
    # each axis is a Gaussian fit of its own sigma on its own window; defaults as the 1-D plans
    for H, W, sy, sx, K, Ly, Lx in [(300, 200, 4.0, 9.0, 4, 0, 0), (64, 4096, 20.0, 3.0, 5, 70, 12)]:
        h = _abi.morlet_plan_gauss2d(H, W, sy, sx, K, Ly, Lx)
        try:
            ix, iy = _abi.morlet_image_axis_info(h, 0, K), _abi.morlet_image_axis_info(h, 1, K)
            _abi.morlet_plan_set(h, _abi.MORLET_SCAN_ASFT, 0, 0)
            ax, ay = _abi.morlet_image_axis_info(h, 0, K), _abi.morlet_image_axis_info(h, 1, K)
        finally:
            _abi.morlet_destroy(h)
        for info, sigma, L in ((ix, sx, Lx), (iy, sy, Ly)):
            if L == 0:
                hg = _abi.morlet_plan_gauss(1000, sigma, K, 0)
                L = _abi.morlet_plan_info(hg, K)["L"]
                _abi.morlet_destroy(hg)
            assert info["L"] == L and info["n0"] == 0
            assert np.allclose(info["cos_coef"], O.fit_gauss(sigma, K, L), rtol=1e-10, atol=1e-14)
        assert ax["n0"] == O.default_n0(sx) and ay["n0"] == O.default_n0(sy)


def test_image_plan_errors_and_workspace():
    L = _abi.lib()
    h = ctypes.c_void_p()
    for args in [(-1, 10, 2.0, 2.0, 3, 0, 0), (10, 1 << 25, 2.0, 2.0, 3, 0, 0), (10, 10, 2.0, 2.0, 0, 0, 0),
                 (10, 10, -2.0, 2.0, 3, 0, 0), (10, 10, 2.0, 2.0, 5, 2, 0)]:
        assert L.morlet_plan_gauss2d(ctypes.byref(h), *args) == _abi.MORLET_ERR_INVALID_ARG, args
    assert L.morlet_plan_gauss2d(ctypes.byref(h), 120, 90, 3.0, 5.0, 4, 0, 0) == _abi.MORLET_OK
    hp = h.value
    try:
        assert _abi.morlet_workspace_size(hp) >= 2 * 120 * 90 * 4
        fake = 1 << 20
        assert L.gauss_smooth(hp, fake, 0, fake, fake, 1 << 30, None) == _abi.MORLET_ERR_INVALID_ARG
        assert L.morlet_forward(hp, fake, 0, fake, fake, 1 << 30, None) == _abi.MORLET_ERR_INVALID_ARG
        assert L.gauss_smooth_backward(hp, fake, 0, fake, fake, None, fake, 1 << 30, None) == _abi.MORLET_ERR_UNSUPPORTED
        assert L.morlet_plan_autotune(hp, fake, 0, fake, 3, None, None, None) == _abi.MORLET_ERR_UNSUPPORTED
        assert L.gauss_smooth2d(hp, fake, 0, fake, fake, 100, None) == _abi.MORLET_ERR_WORKSPACE
        assert L.morlet_image_axis_info(hp, 2, None, None, None, None) == _abi.MORLET_ERR_INVALID_ARG
        for R in (4, 8, 16, 32):
            assert L.morlet_plan_set_tile(hp, R) == _abi.MORLET_OK
    finally:
        _abi.morlet_destroy(hp)
    h1 = _abi.morlet_plan_gauss(100, 3.0, 4, 0)
    try:
        assert L.gauss_smooth2d(h1, 1 << 20, 0, 1 << 20, 1 << 20, 1 << 30, None) == _abi.MORLET_ERR_INVALID_ARG
    finally:
        _abi.morlet_destroy(h1)


def test_gabor_plan_errors_and_workspace():
    L = _abi.lib()
    h = ctypes.c_void_p()
    for args in [(-1, 10, 2.0, 1.0, 3, 0, 2.0, 3, 0), (10, 1 << 25, 2.0, 1.0, 3, 0, 2.0, 3, 0),
                 (10, 10, 2.0, 0.0, 3, 0, 2.0, 3, 0), (10, 10, 2.0, 1.0, 5, 4, 2.0, 3, 0),
                 (10, 10, 2.0, 1.0, 3, 0, -2.0, 3, 0), (10, 10, 2.0, 1.0, 3, 0, 2.0, 5, 2)]:
        assert L.morlet_plan_gabor2d(ctypes.byref(h), *args) == _abi.MORLET_ERR_INVALID_ARG, args
    hp = _abi.morlet_plan_gabor2d(120, 90, 3.0, 2.0, 5, 0, 4.0, 4, 0)
    hg = _abi.morlet_plan_gauss2d(120, 90, 3.0, 5.0, 4, 0, 0)
    fake = 1 << 20
    try:
        # two complex64 buffers of the image on top of the tile states
        assert _abi.morlet_workspace_size(hp) >= 2 * 120 * 90 * 8
        assert L.gabor2d(hp, fake, 0, fake, fake, 100, None) == _abi.MORLET_ERR_WORKSPACE
        assert L.gabor2d(hp, fake, 3, fake, fake, 1 << 30, None) == _abi.MORLET_ERR_UNSUPPORTED
        assert L.gabor2d(hg, fake, 0, fake, fake, 1 << 30, None) == _abi.MORLET_ERR_INVALID_ARG
        assert L.gauss_smooth2d(hp, fake, 0, fake, fake, 1 << 30, None) == _abi.MORLET_ERR_INVALID_ARG
        assert L.morlet_forward(hp, fake, 0, fake, fake, 1 << 30, None) == _abi.MORLET_ERR_INVALID_ARG
        assert L.gauss_smooth2d_backward(hp, fake, fake, fake, 1 << 30, None) == _abi.MORLET_ERR_INVALID_ARG
        assert L.gabor2d_backward(hg, fake, fake, fake, 1 << 30, None) == _abi.MORLET_ERR_INVALID_ARG
        assert L.gauss_smooth2d_grad(hp, fake, 0, fake, fake, fake, fake, 1 << 30, None) == _abi.MORLET_ERR_INVALID_ARG
        assert L.gabor2d_grad(hg, fake, 0, fake, fake, fake, fake, 1 << 30, None) == _abi.MORLET_ERR_INVALID_ARG
        assert L.gabor2d_grad(hp, fake, 3, fake, fake, fake, fake, 1 << 30, None) == _abi.MORLET_ERR_UNSUPPORTED
        assert L.gabor2d_grad(hp, fake, 0, fake, fake, fake, fake, 100, None) == _abi.MORLET_ERR_WORKSPACE
        assert L.gauss_smooth2d_grad(hg, fake, 3, fake, fake, fake, fake, 1 << 30, None) == _abi.MORLET_ERR_UNSUPPORTED
        assert L.gauss_smooth2d_grad(hg, fake, 0, fake, fake, None, fake, 1 << 30, None) == _abi.MORLET_ERR_INVALID_ARG
        assert L.gauss_smooth2d_grad(hg, fake, 0, fake, fake, fake, fake, 100, None) == _abi.MORLET_ERR_WORKSPACE
        assert _abi.morlet_backward_workspace_size(hp) >= 2 * 120 * 90 * 8
        assert L.gabor2d_backward(hp, fake, fake, fake, 2 * 120 * 90 * 8, None) == _abi.MORLET_ERR_WORKSPACE
        assert L.morlet_plan_set_boundary(hp, 1) == _abi.MORLET_ERR_UNSUPPORTED
        # axis 0 carries the Morlet fit (K_x = 5 coefficients), axis 1 the Gaussian (K_y = 4)
        ix = _abi.morlet_image_axis_info(hp, 0, 5)
        iy = _abi.morlet_image_axis_info(hp, 1, 4)
        assert ix["L"] >= 5 and iy["L"] >= 3 and ix["kernel_relrmse"] < 0.5 and iy["kernel_relrmse"] < 0.1
        for R in (4, 8, 32, 16):
            assert L.morlet_plan_set_tile(hp, R) == _abi.MORLET_OK
        assert L.morlet_plan_set(hp, _abi.MORLET_SCAN_ASFT, 0, 0) == _abi.MORLET_OK
        assert _abi.morlet_image_axis_info(hp, 0, 5)["n0"] >= 1
        h0 = _abi.morlet_plan_gabor2d(0, 90, 3.0, 2.0, 5, 0, 4.0, 4, 0)
        try:
            assert L.gabor2d(h0, None, 0, None, None, 0, None) == _abi.MORLET_OK   # empty: nothing to do
        finally:
            _abi.morlet_destroy(h0)
    finally:
        _abi.morlet_destroy(hp)
        _abi.morlet_destroy(hg)


def test_tree_path_errors_and_workspace():
    L = _abi.lib()
    h = _abi.morlet_plan(5000, 20.0, 0.3, 5, 80)
    hg = _abi.morlet_plan_gauss(5000, 20.0, 4, 80)
    hd = _abi.morlet_plan_gauss_deriv(5000, 20.0, 4, 80, 1)
    hs = _abi.morlet_scalogram_plan([100, 200], [4.0, 8.0], [1.5, 0.75], 4, 0.0)
    fake = 1 << 20
    try:
        assert _abi.morlet_tree_workspace_size(h) == 4 * 5 * (5000 + 160) * 8
        assert _abi.morlet_tree_workspace_size(hg) == 4 * 4 * (5000 + 160) * 8
        n = ctypes.c_size_t()
        for bad in (hd, hs):
            assert L.morlet_tree_workspace_size(bad, ctypes.byref(n)) == _abi.MORLET_ERR_INVALID_ARG
            assert L.morlet_tree_forward(bad, fake, 0, fake, fake, 1 << 30, None) == _abi.MORLET_ERR_INVALID_ARG
        assert L.morlet_tree_forward(h, fake, 0, fake, fake, 100, None) == _abi.MORLET_ERR_WORKSPACE
        assert L.morlet_tree_forward(h, fake, 7, fake, fake, 1 << 30, None) == _abi.MORLET_ERR_UNSUPPORTED
        _abi.morlet_plan_set(h, _abi.MORLET_SCAN_ASFT, 0, 0)
        assert L.morlet_tree_forward(h, fake, 0, fake, fake, 1 << 30, None) == _abi.MORLET_ERR_UNSUPPORTED
    finally:
        for x in (h, hg, hd, hs):
            _abi.morlet_destroy(x)


def test_empty_inputs_of_the_newer_paths():
    # N = 0 (or an empty image) is a no-op that succeeds before any pointer is looked at
    L = _abi.lib()
    hm = _abi.morlet_plan_multiply(0, 10.0, 0.6, 2, 0)
    hi = _abi.morlet_plan_gauss2d(0, 50, 3.0, 3.0, 4, 0, 0)
    hj = _abi.morlet_plan_gauss2d(40, 0, 3.0, 3.0, 4, 0, 0)
    ht = _abi.morlet_plan(0, 10.0, 0.6, 4, 40)
    hd = _abi.morlet_plan_gauss_deriv(0, 10.0, 4, 40, 1)
    try:
        assert L.morlet_forward(hm, None, 0, None, None, 0, None) == _abi.MORLET_OK
        assert L.gauss_smooth2d(hi, None, 0, None, None, 0, None) == _abi.MORLET_OK
        assert L.gauss_smooth2d(hj, None, 0, None, None, 0, None) == _abi.MORLET_OK
        assert L.morlet_tree_forward(ht, None, 0, None, None, 0, None) == _abi.MORLET_OK
        _abi.morlet_plan_set(hd, _abi.MORLET_SCAN_ASFT, 0, 0)
        assert L.gauss_smooth(hd, None, 0, None, None, 0, None) == _abi.MORLET_OK
    finally:
        for h in (hm, hi, hj, ht, hd):
            _abi.morlet_destroy(h)


def test_edge_boundary_setting():
    L = _abi.lib()
    h = _abi.morlet_plan(1000, 20.0, 0.3, 5, 80)
    hs = _abi.morlet_scalogram_plan([100, 200], [4.0, 8.0], [1.5, 0.75], 4, 0.0)
    hm = _abi.morlet_plan_multiply(1000, 20.0, 0.3, 2, 0)
    hd = _abi.morlet_plan_gauss_deriv(1000, 20.0, 4, 80, 2)
    fake = 1 << 20
    try:
        base = _abi.morlet_workspace_size(h)
        _abi.morlet_plan_set_boundary(h, _abi.MORLET_BOUNDARY_EDGE)
        assert _abi.morlet_workspace_size(h) >= base + (1000 + 4 * 80) * (4 + 8)
        assert L.morlet_plan_set_boundary(h, 5) == _abi.MORLET_ERR_INVALID_ARG
        assert L.morlet_backward(h, fake, 0, fake, fake, None, fake, 100, None) == _abi.MORLET_ERR_WORKSPACE
        bw = _abi.morlet_backward_workspace_size(h)
        assert bw >= (1000 + 4 * 80) * (4 + 8 + 4) and bw >= _abi.morlet_workspace_size(h)
        assert L.morlet_direct_forward(h, fake, 0, fake, 0, None) == _abi.MORLET_ERR_UNSUPPORTED
        assert L.morlet_tree_forward(h, fake, 0, fake, fake, 1 << 30, None) != _abi.MORLET_OK
        assert L.morlet_forward(h, fake, 0, fake, fake, 100, None) == _abi.MORLET_ERR_WORKSPACE
        for bad in (hs, hm):
            assert L.morlet_plan_set_boundary(bad, _abi.MORLET_BOUNDARY_EDGE) == _abi.MORLET_ERR_UNSUPPORTED
        assert L.morlet_plan_set_boundary(hd, _abi.MORLET_BOUNDARY_EDGE) == _abi.MORLET_OK
        _abi.morlet_plan_set_boundary(h, _abi.MORLET_BOUNDARY_ZERO)
        assert _abi.morlet_workspace_size(h) == base
    finally:
        for x in (h, hs, hm, hd):
            _abi.morlet_destroy(x)


def test_image_backward_workspace_keeps_the_header_first():
    # forward and backward share a workspace: the backward's own scan workspace (with the header)
    # comes first, and the backward size also covers the forward
    h = _abi.morlet_plan_gauss2d(120, 90, 3.0, 5.0, 4, 0, 0)
    try:
        fw, bw = _abi.morlet_workspace_size(h), _abi.morlet_backward_workspace_size(h)
        assert bw >= fw and bw >= 2 * 120 * 90 * 4
        L = _abi.lib()
        assert L.gauss_smooth2d_backward(h, 1 << 20, 1 << 20, 1 << 20, 100, None) == _abi.MORLET_ERR_WORKSPACE
    finally:
        _abi.morlet_destroy(h)


@pytest.mark.parametrize("which", ["scalogram", "differentiation"])
def test_workload_scales_lowest_order_chosen_by_oracle(which):
    # every scale of the batched workloads (32 scales 4..4096 of the ragged scalogram, 16
    # scales 8..2048 of the differentiation batch), K = 5, error-optimal windows: at the
    # library's window the oracle picks the lowest order itself (argmin of the fitted
    # wavelet's error, Sec. III-A), and for windows of at most 700 also over the full range
    # 0..L-K+1; both must equal the library's choice, and the fits must agree
    s = np.arange(32 if which == "scalogram" else 16, dtype=np.float64)
    sigmas = 4.0 * 1024.0 ** (s / 31) if which == "scalogram" else 8.0 * 256.0 ** (s / 15)
    xis = 6.0 / sigmas
    hs = _abi.morlet_scalogram_plan([1000, 3000], list(sigmas), list(xis), 5, 0.0)
    try:
        infos = [_abi.morlet_scalogram_scale_info(hs, i, 5) for i in range(len(sigmas))]
    finally:
        _abi.morlet_destroy(hs)
    for sg, xi, info in zip(sigmas, xis, infos):
        L = info["L"]
        ps = O.select_PS(float(sg), float(xi), 5, L)
        assert ps == info["P_S"], (sg, L, ps, info["P_S"])
        if L <= 700:
            assert O.select_PS_full(float(sg), float(xi), 5, L) == ps, (sg, L)
        m, l = O.fit_morlet(float(sg), float(xi), 5, L, ps)
        scale = max(np.abs(m).max(), np.abs(l).max())
        assert np.allclose(info["cos_coef"], m, rtol=1e-9, atol=1e-12 * scale), (sg, L)
        assert np.allclose(info["sin_coef"], l, rtol=1e-9, atol=1e-12 * scale), (sg, L)


def _oracle_err(sigma, xi, K, L, gauss):
    k = np.arange(-L, L + 1)
    if gauss:
        return O.kernel_relrmse(O.kterm_gauss(O.plan_gauss(sigma, K, L)), O.gaussian(sigma, k))
    return O.kernel_relrmse(O.kterm_morlet(O.plan_morlet(sigma, xi, K, L)), O.morlet(sigma, xi, k))


@pytest.mark.parametrize("sigma,target,gauss", [(16.0, 1e-2, False), (40.0, 1e-3, False), (300.0, 3e-2, False),
                                                (8.0, 1e-4, True), (64.0, 1e-6, True), (12.0, 5e-3, False)])
def test_choose_terms_is_fewest_reaching_target(sigma, target, gauss):
    # the chooser's error is the oracle's at the same (K, L); it reaches the target; one term
    # fewer, at that count's own error-optimal window, does not
    xi = 6.0 / sigma
    K, L, e = _abi.morlet_choose_terms(sigma, xi, target, gauss=gauss)
    assert 1 <= K <= _abi.MORLET_MAX_TERMS
    # the library forms the residual from the normal equations (|g|^2 minus the projection), whose
    # relative precision is a few ulps of |g|^2 over residual^2: 1e-7 at an error of 4e-5
    assert math.isclose(e, _oracle_err(sigma, xi, K, L, gauss), rel_tol=max(1e-9, 1e-15 / e ** 2))
    assert e <= target
    if K > 1:
        h = _abi.morlet_plan_gauss(100, sigma, K - 1, 0) if gauss else _abi.morlet_plan(100, sigma, xi, K - 1, 0)
        try:
            L1 = _abi.morlet_plan_info(h, K - 1)["L"]
        finally:
            _abi.morlet_destroy(h)
        assert _oracle_err(sigma, xi, K - 1, L1, gauss) > target


def test_choose_terms_reports_best_when_unreachable():
    K, L, e = _abi.morlet_choose_terms(16.0, 6.0 / 16.0, 1e-30, strict=False)
    assert K >= 1 and e > 1e-30
    with pytest.raises(_abi.MorletError) as ex:
        _abi.morlet_choose_terms(16.0, 6.0 / 16.0, 1e-30)
    assert ex.value.status == _abi.MORLET_ERR_UNSUPPORTED
    with pytest.raises(_abi.MorletError):
        _abi.morlet_choose_terms(-1.0, 1.0, 1e-3)
    with pytest.raises(_abi.MorletError):
        _abi.morlet_inject_failure(_abi.MORLET_OK, 1)
    _abi.morlet_inject_failure(_abi.MORLET_ERR_HIP, 0)   # disarmed
