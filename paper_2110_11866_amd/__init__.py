"""MI355X (gfx950) Morlet wavelet transform and Gaussian smoothing by SFT / ASFT kernel
integrals (Yamashita & Wakahara, arXiv 2110.11866).

The compute path is libmorlet.so (include/morlet.h), hand-written HIP for gfx950.
This package only marshals PyTorch tensors (device memory, current stream) into its C ABI;
if the library is missing every call raises.
"""
from __future__ import annotations

import torch

from . import _abi
from ._abi import (MORLET_ACC_COMPENSATED, MORLET_ACC_F32, MORLET_BF16, MORLET_F16, MORLET_F32,
                   MORLET_SCAN_ASFT, MORLET_SCAN_SFT, MorletError)

__all__ = ["MorletPlan", "GaussPlan", "MorletError", "torch_dtype_code"]

_DT = {torch.float32: MORLET_F32, torch.float16: MORLET_F16, torch.bfloat16: MORLET_BF16}
_MODE = {"sft": MORLET_SCAN_SFT, "asft": MORLET_SCAN_ASFT}
_ACC = {"f32": MORLET_ACC_F32, "compensated": MORLET_ACC_COMPENSATED}


def torch_dtype_code(dt: torch.dtype) -> int:
    if dt not in _DT:
        raise TypeError(f"unsupported signal dtype {dt}; use float32, float16 or bfloat16")
    return _DT[dt]


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


class _PlanBase:
    kind = ""

    def __init__(self, handle: int, N: int, K: int):
        self.handle = handle
        self.N = N
        self.K = K
        self._ws = None

    def set(self, mode: str = "sft", n0: int = 0, accum: str = "f32") -> "_PlanBase":
        _abi.morlet_plan_set(self.handle, _MODE[mode], int(n0), _ACC[accum])
        return self

    def info(self) -> dict:
        return _abi.morlet_plan_info(self.handle, self.K)

    def workspace_bytes(self) -> int:
        return _abi.morlet_workspace_size(self.handle)

    def workspace(self, device) -> torch.Tensor:
        """A zero-filled workspace owned by the plan (allocated on first use)."""
        need = self.workspace_bytes()
        if self._ws is None or self._ws.numel() < need or self._ws.device != torch.device(device):
            self._ws = torch.zeros(max(need, 64), dtype=torch.uint8, device=device)
        return self._ws

    def _check_x(self, x: torch.Tensor) -> None:
        if not x.is_cuda:
            raise ValueError("x must be a device tensor")
        if x.dim() != 1 or x.numel() != self.N or not x.is_contiguous():
            raise ValueError(f"x must be a contiguous 1-D tensor of {self.N} samples")

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                _abi.morlet_destroy(h)
            except Exception:
                pass
            self.handle = None


class MorletPlan(_PlanBase):
    """Morlet transform, direct method (Sec. III-A): W = psi_hat * x, K Fourier terms on
    the window [-L, L] (L = 0: error-optimal window), xi in rad/sample."""

    kind = "morlet"

    def __init__(self, N: int, sigma: float, xi: float, K: int, L: int = 0, mode: str = "sft",
                 n0: int = 0, accum: str = "f32"):
        super().__init__(_abi.morlet_plan(int(N), float(sigma), float(xi), int(K), int(L)), int(N), int(K))
        self.sigma, self.xi = float(sigma), float(xi)
        if mode != "sft" or n0 or accum != "f32":
            self.set(mode, n0, accum)

    def forward(self, x: torch.Tensor, out: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
        self._check_x(x)
        if out is None:
            out = torch.empty(self.N, dtype=torch.complex64, device=x.device)
        if out.dtype != torch.complex64 or out.numel() != self.N or not out.is_contiguous():
            raise ValueError("out must be a contiguous complex64 tensor of N elements")
        w = self.workspace(x.device) if ws is None else ws
        _abi.morlet_forward(self.handle, x.data_ptr(), torch_dtype_code(x.dtype), out.data_ptr(), w.data_ptr(),
                            w.numel(), _stream())
        return out


class GaussPlan(_PlanBase):
    """Gaussian smoothing (eqs. aproGauss, GsSFT, GsASFT): orders 0..K-1 on [-L, L]."""

    kind = "gauss"

    def __init__(self, N: int, sigma: float, K: int, L: int = 0, mode: str = "sft", n0: int = 0,
                 accum: str = "f32"):
        super().__init__(_abi.morlet_plan_gauss(int(N), float(sigma), int(K), int(L)), int(N), int(K))
        self.sigma = float(sigma)
        if mode != "sft" or n0 or accum != "f32":
            self.set(mode, n0, accum)

    def forward(self, x: torch.Tensor, out: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
        self._check_x(x)
        if out is None:
            out = torch.empty(self.N, dtype=torch.float32, device=x.device)
        if out.dtype != torch.float32 or out.numel() != self.N or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 tensor of N elements")
        w = self.workspace(x.device) if ws is None else ws
        _abi.gauss_smooth(self.handle, x.data_ptr(), torch_dtype_code(x.dtype), out.data_ptr(), w.data_ptr(),
                          w.numel(), _stream())
        return out
