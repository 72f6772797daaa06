"""Seeded synthetic inputs shaped like the workloads the method is measured on.

This module only draws random numbers and lays them out; it holds none of the
transform's arithmetic, so both the HIP path's tests and the CPU oracle can take
their inputs from it. The paper names no dataset and does not describe its test
signals (Sec. V-B times one signal of N = 102400 samples at sigma = 8192), so
every recipe below is a stand-in with the stated distribution and seed.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "small_signal", "paper_scale_signal", "ragged_scalogram", "precision_stress_signal",
    "differentiation_batch", "morlet_xi",
]


def morlet_xi(sigma: float, xi0: float = 6.0) -> float:
    """Carrier in rad/sample for a dimensionless carrier xi0 (xi0 = 6 throughout)."""
    return xi0 / sigma


def small_signal(N: int = 1024, seed: int = 1) -> np.ndarray:
    """i.i.d. N(0, 1), float64. Small single transform: sigma = 16, K = 4, L = 64."""
    return np.random.default_rng(seed).standard_normal(N)


def paper_scale_signal(N: int = 102400, seed: int = 2) -> np.ndarray:
    """Sum of three unit-amplitude sinusoids, frequencies U[0.001, 0.2] cycles/sample
    and phases U[0, 2 pi), plus N(0, 0.1^2) noise; float32. sigma = 8192."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.001, 0.2, size=3)
    ph = rng.uniform(0.0, 2.0 * math.pi, size=3)
    n = np.arange(N, dtype=np.float64)
    x = np.zeros(N)
    for i in range(3):
        x += np.sin(2.0 * math.pi * f[i] * n + ph[i])
    x += 0.1 * rng.standard_normal(N)
    return x.astype(np.float32)


def _pink(rng: np.random.Generator, n: int) -> np.ndarray:
    """White N(0,1) shaped to a 1/f power spectrum (amplitude f^{-1/2}, DC removed),
    rescaled to unit variance."""
    w = rng.standard_normal(n)
    F = np.fft.rfft(w)
    f = np.fft.rfftfreq(n)
    F[0] = 0.0
    F[1:] /= np.sqrt(f[1:])
    x = np.fft.irfft(F, n)
    s = x.std()
    return x / s if s > 0 else x


def ragged_scalogram(B: int = 256, S: int = 32, lo: int = 4096, hi: int = 262144,
                     seed: int = 3):
    """Batched ragged scalogram: B signal lengths log-uniform in [lo, hi], pink
    noise, float32, packed back to back; S scales sigma_s = 4 * 1024^{s/(S-1)}.

    Returns (x_packed float32, lengths int64[B], sigmas float64[S], xis float64[S])."""
    rng = np.random.default_rng(seed)
    lengths = np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), size=B))).astype(np.int64)
    parts = [_pink(rng, int(n)) for n in lengths]
    x = np.concatenate(parts).astype(np.float32) if parts else np.zeros(0, np.float32)
    s = np.arange(S, dtype=np.float64)
    sigmas = 4.0 * 1024.0 ** (s / max(S - 1, 1))
    xis = np.array([morlet_xi(v) for v in sigmas])
    return x, lengths, sigmas, xis


def precision_stress_signal(N: int = 1 << 22, seed: int = 1234) -> np.ndarray:
    """Random walk plus white noise: cumsum(N(0,1)) + N(0,1), float64 (callers
    store it as float16 / bfloat16; the range stays well inside float16)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.standard_normal(N)) + rng.standard_normal(N)


def differentiation_batch(B: int = 64, N: int = 32768, S: int = 16, seed: int = 5):
    """Batch of i.i.d. N(0,1) float32 signals [B][N], S scales sigma_s = 8 * 256^{s/(S-1)},
    and loss weights w ~ U[0, 1] of shape [S][N] shared over the batch.

    Returns (x, sigmas, xis, w)."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((B, N)).astype(np.float32)
    s = np.arange(S, dtype=np.float64)
    sigmas = 8.0 * 256.0 ** (s / max(S - 1, 1))
    xis = np.array([morlet_xi(v) for v in sigmas])
    w = rng.uniform(0.0, 1.0, size=(S, N)).astype(np.float32)
    return x, sigmas, xis, w
