"""MI355X (gfx950) Morlet wavelet transform and Gaussian smoothing by SFT / ASFT kernel
integrals (Yamashita & Wakahara, arXiv 2110.11866).

The compute path is libmorlet.so (include/morlet.h), hand-written HIP for gfx950.
This package only marshals PyTorch tensors (device memory, current stream) into its C ABI;
if the library is missing every call raises.
"""
from __future__ import annotations

import torch

from . import _abi
from ._abi import (MORLET_ACC_AUTO, MORLET_ACC_F32, MORLET_ACC_F64, MORLET_ACC_KAHAN, MORLET_ACC_MIXED, MORLET_BF16, MORLET_F16, MORLET_F32,
                   MORLET_SCAN_ASFT, MORLET_SCAN_SFT, MorletError)

def choose_terms(sigma: float, xi: float | None, target_relrmse: float) -> dict:
    """Fewest Fourier terms K (with its error-optimal window L) whose fitted kernel reaches the
    relative RMSE target; xi=None for Gaussian smoothing. Host-side (morlet_choose_terms)."""
    K, L, e = _abi.morlet_choose_terms(float(sigma), float(xi or 0.0), float(target_relrmse), gauss=xi is None)
    return {"K": K, "L": L, "kernel_relrmse": e}


__all__ = ["choose_terms", "MorletPlan", "MultiplyPlan", "GaussPlan", "GaussDerivPlan", "Gauss2DPlan", "Gabor2DPlan", "ScalogramPlan", "MorletError", "torch_dtype_code", "morlet_transform",
           "MorletTransform"]

_DT = {torch.float32: MORLET_F32, torch.float16: MORLET_F16, torch.bfloat16: MORLET_BF16}
_MODE = {"sft": MORLET_SCAN_SFT, "asft": MORLET_SCAN_ASFT}
_ACC = {"auto": MORLET_ACC_AUTO, "f32": MORLET_ACC_F32, "f64": MORLET_ACC_F64, "mixed": MORLET_ACC_MIXED,
        "kahan": MORLET_ACC_KAHAN}


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

    def set(self, mode: str = "sft", n0: int = 0, accum: str = "auto") -> "_PlanBase":
        _abi.morlet_plan_set(self.handle, _MODE[mode], int(n0), _ACC[accum])
        return self

    def set_boundary(self, boundary: str) -> "_PlanBase":
        """Extension of a single signal beyond [0, N-1]: "zero" (default) or "edge" (Sec. II)."""
        code = {"zero": _abi.MORLET_BOUNDARY_ZERO, "edge": _abi.MORLET_BOUNDARY_EDGE}
        if boundary not in code:
            raise ValueError("boundary must be zero or edge")
        _abi.morlet_plan_set_boundary(self.handle, code[boundary])
        self._ws = None
        return self

    def set_tile(self, R: int) -> "_PlanBase":
        """Samples per thread of the scan kernels (4, 8, 16 or 32)."""
        _abi.morlet_plan_set_tile(self.handle, int(R))
        self._ws = None
        return self

    def set_schedule(self, schedule: str) -> "_PlanBase":
        """Forward launch schedule: "auto", "tiles" (look-back between tiles), "rows" (a block
        runs whole rows; several rows) or "segments" (one long row in segments: a pass for
        the segment states, then a pass with outputs)."""
        code = {"auto": _abi.MORLET_SCHED_AUTO, "tiles": _abi.MORLET_SCHED_TILES, "rows": _abi.MORLET_SCHED_ROWS,
                "segments": _abi.MORLET_SCHED_SEGMENTS}
        if schedule not in code:
            raise ValueError("schedule must be auto, tiles, rows or segments")
        _abi.morlet_plan_set_schedule(self.handle, code[schedule])
        return self

    def set_segments(self, tiles: int) -> "_PlanBase":
        """Segments schedule: tiles per segment (0: automatic)."""
        _abi.morlet_plan_set_segments(self.handle, int(tiles))
        return self

    def info(self) -> dict:
        return _abi.morlet_plan_info(self.handle, self.K)

    def refit(self, sigma: float, xi: float = 0.0) -> "_PlanBase":
        """Refit the coefficients at new sigma (and xi, Morlet plans) with the window, lowest
        order, ASFT shift and tile shape kept, into the plan's own device table on the
        current stream (morlet_plan_refit; single-signal Morlet and Gaussian plans)."""
        _abi.morlet_plan_refit(self.handle, float(sigma), float(xi), _stream() if torch.cuda.is_available() else 0)
        self.sigma = float(sigma)
        if self.kind == "morlet":
            self.xi = float(xi)
        return self

    def _out_like(self, x: torch.Tensor) -> torch.Tensor:
        n = self.S * self.N if self.kind == "scalogram" else self.N
        return torch.empty(n, dtype=torch.float32 if self.kind == "gauss" else torch.complex64, device=x.device)

    def autotune(self, x: torch.Tensor, reps: int = 5) -> dict:
        """Time the forward on x for each tile shape (and schedule, for scalograms) and keep
        the fastest; returns {"R": 4 | 8 | 16 | 32, "schedule": "tiles" | "rows" | "segments"}."""
        self._check_x(x)
        out = self._out_like(x)
        R, sched = _abi.morlet_plan_autotune(self.handle, x.data_ptr(), torch_dtype_code(x.dtype), out.data_ptr(),
                                             int(reps), _stream())
        self._ws = None
        names = {_abi.MORLET_SCHED_ROWS: "rows", _abi.MORLET_SCHED_SEGMENTS: "segments"}
        return {"R": R, "schedule": names.get(sched, "tiles")}

    def workspace_bytes(self) -> int:
        return _abi.morlet_workspace_size(self.handle)

    def tree(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Comparison path: the same SFT result by the paper's sliding-sum route (Sec. IV,
        Algorithm 1), single-signal Morlet and Gaussian smoothing plans in SFT mode."""
        self._check_x(x)
        if out is None:
            out = self._out_like(x)
        need = _abi.morlet_tree_workspace_size(self.handle)
        tw = getattr(self, "_tree_ws", None)
        if tw is None or tw.numel() < need or tw.device != x.device:
            tw = self._tree_ws = torch.empty(max(need, 64), dtype=torch.uint8, device=x.device)
        _abi.morlet_tree_forward(self.handle, x.data_ptr(), torch_dtype_code(x.dtype), out.data_ptr(), tw.data_ptr(),
                                 tw.numel(), _stream())
        return out

    def backward_workspace_bytes(self) -> int:
        return _abi.morlet_backward_workspace_size(self.handle)

    def workspace(self, device, backward: bool = False) -> torch.Tensor:
        """A zero-filled workspace owned by the plan (allocated on first use); the backward
        size also serves the forward."""
        need = self.backward_workspace_bytes() if backward else self.workspace_bytes()
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


def _bwd_common(plan, fn, x, g, want_params, nparams):
    if not g.is_cuda or not g.is_contiguous():
        raise ValueError("the cotangent must be a contiguous device tensor")
    w = plan.workspace(g.device, backward=True)
    gx = torch.empty(plan.N, dtype=torch.float32, device=g.device)
    gp = torch.empty(nparams, dtype=torch.float64, device=g.device) if want_params else None
    xp = x.data_ptr() if x is not None else None
    dt = torch_dtype_code(x.dtype) if x is not None else 0
    fn(plan.handle, xp, dt, g.data_ptr(), gx.data_ptr(), gp.data_ptr() if gp is not None else None,
       w.data_ptr(), w.numel(), _stream())
    return gx, gp


class MorletPlan(_PlanBase):
    """Morlet transform, direct method (Sec. III-A): W = psi_hat * x, K Fourier terms on
    the window [-L, L] (L = 0: error-optimal window), xi in rad/sample."""

    kind = "morlet"

    def __init__(self, N: int, sigma: float, xi: float, K: int, L: int = 0, mode: str = "sft",
                 n0: int = 0, accum: str = "auto"):
        super().__init__(_abi.morlet_plan(int(N), float(sigma), float(xi), int(K), int(L)), int(N), int(K))
        self.sigma, self.xi = float(sigma), float(xi)
        if mode != "sft" or n0 or accum != "auto":
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

    def direct(self, x: torch.Tensor, half_width: int = 0, out: torch.Tensor | None = None) -> torch.Tensor:
        """Baseline: truncated direct convolution with the exact wavelet on [-H, H]
        (H = half_width, 0 = the plan's L)."""
        self._check_x(x)
        if out is None:
            out = torch.empty(self.N, dtype=torch.complex64, device=x.device)
        _abi.morlet_direct_forward(self.handle, x.data_ptr(), torch_dtype_code(x.dtype), out.data_ptr(),
                                   int(half_width), _stream())
        return out

    def backward(self, x: torch.Tensor | None, gW: torch.Tensor, want_params: bool = True):
        """(dLoss/dx float32 [N], [dLoss/dsigma, dLoss/dxi] float64 or None) for the cotangent
        gW = dLoss/dRe W + i dLoss/dIm W (complex64 [N])."""
        if gW.dtype != torch.complex64 or gW.numel() != self.N:
            raise ValueError("gW must be complex64 of N elements")
        if want_params:
            self._check_x(x)
        return _bwd_common(self, _abi.morlet_backward, x if want_params else None, gW, want_params, 2)


class MultiplyPlan(MorletPlan):
    """Morlet transform by the multiplication method (Sec. III-B): the Gaussian envelope
    fitted with the cosines of orders 0..P_M (K = P_M + 1 terms) times the carrier, evaluated
    as three Gaussian smoothings (demodulated real and imaginary parts, and the signal) in one
    scan launch between a demodulation and a remodulation kernel. The backward gives dLoss/dx."""

    kind = "morlet"

    def __init__(self, N: int, sigma: float, xi: float, P_M: int, L: int = 0, mode: str = "sft",
                 n0: int = 0, accum: str = "auto"):
        _PlanBase.__init__(self, _abi.morlet_plan_multiply(int(N), float(sigma), float(xi), int(P_M), int(L)),
                           int(N), int(P_M) + 1)
        self.sigma, self.xi, self.P_M = float(sigma), float(xi), int(P_M)
        if mode != "sft" or n0 or accum != "auto":
            self.set(mode, n0, accum)

    def direct(self, *args, **kwargs):
        raise NotImplementedError("the direct-convolution baseline needs a direct-method plan")

    def backward(self, x: torch.Tensor | None, gW: torch.Tensor, want_params: bool = False):
        """(dLoss/dx float32 [N], None) for the cotangent gW (complex64 [N]); parameter
        gradients are not built for the multiplication method."""
        if want_params:
            raise NotImplementedError("parameter gradients are not built for the multiplication method")
        if gW.dtype != torch.complex64 or gW.numel() != self.N:
            raise ValueError("gW must be complex64 of N elements")
        return _bwd_common(self, _abi.morlet_backward, None, gW, False, 2)


class GaussPlan(_PlanBase):
    """Gaussian smoothing (eqs. aproGauss, GsSFT, GsASFT): orders 0..K-1 on [-L, L]."""

    kind = "gauss"

    def __init__(self, N: int, sigma: float, K: int, L: int = 0, mode: str = "sft", n0: int = 0,
                 accum: str = "auto"):
        super().__init__(_abi.morlet_plan_gauss(int(N), float(sigma), int(K), int(L)), int(N), int(K))
        self.sigma = float(sigma)
        if mode != "sft" or n0 or accum != "auto":
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

    def backward(self, x: torch.Tensor | None, gy: torch.Tensor, want_params: bool = True):
        if gy.dtype != torch.float32 or gy.numel() != self.N:
            raise ValueError("gy must be float32 of N elements")
        if want_params:
            self._check_x(x)
        return _bwd_common(self, _abi.gauss_smooth_backward, x if want_params else None, gy, want_params, 2)


class GaussDerivPlan(GaussPlan):
    """The Gaussian's differentials applied to the signal (Sec. II); the backward gives dLoss/dx.
    SFT: order 1 gives x_GD (sine components 1..K), order 2 gives x_GDD (cosine components
    0..K-1). ASFT (eq. gddAsft): orders 0..K-1 with both components, shifted by n0."""

    def __init__(self, N: int, sigma: float, K: int, L: int = 0, order: int = 1, mode: str = "sft",
                 n0: int = 0, accum: str = "auto"):
        _PlanBase.__init__(self, _abi.morlet_plan_gauss_deriv(int(N), float(sigma), int(K), int(L), int(order)),
                           int(N), int(K))
        self.sigma = float(sigma)
        self.order = int(order)
        if mode != "sft" or n0 or accum != "auto":
            self.set(mode, n0, accum)

    def backward(self, x: torch.Tensor | None, gy: torch.Tensor, want_params: bool = False):
        """(dLoss/dx float32 [N], None) for gy = dLoss/dy (float32 [N]): the plan's forward of the
        reversed cotangent, reversed; parameter gradients are not built for differentials."""
        if want_params:
            raise NotImplementedError("parameter gradients are not built for differential plans")
        if gy.dtype != torch.float32 or gy.numel() != self.N:
            raise ValueError("gy must be float32 of N elements")
        return _bwd_common(self, _abi.gauss_smooth_backward, None, gy, False, 2)


class Gauss2DPlan(_PlanBase):
    """Separable 2-D Gaussian smoothing of an H x W image (row-major, x along a row): the
    lines are filtered independently (Sec. IV), rows then columns, each axis with K cosine
    terms on its own window (0: error-optimal). The backward gives dLoss/dx."""

    kind = "image"

    def __init__(self, H: int, W: int, sigma_y: float, sigma_x: float, K: int, L_y: int = 0, L_x: int = 0,
                 mode: str = "sft", n0: int = 0, accum: str = "auto"):
        h = _abi.morlet_plan_gauss2d(int(H), int(W), float(sigma_y), float(sigma_x), int(K), int(L_y), int(L_x))
        super().__init__(h, int(H) * int(W), int(K))
        self.H, self.W = int(H), int(W)
        self.sigma_y, self.sigma_x = float(sigma_y), float(sigma_x)
        if mode != "sft" or n0 or accum != "auto":
            self.set(mode, n0, accum)

    def info(self) -> dict:
        raise TypeError("use axis_info(0) (x, along rows) or axis_info(1) (y) for an image plan")

    def axis_info(self, axis: int) -> dict:
        return _abi.morlet_image_axis_info(self.handle, int(axis), self.K)

    def _check_x(self, x: torch.Tensor) -> None:
        if not x.is_cuda:
            raise ValueError("x must be a device tensor")
        if x.numel() != self.N or not x.is_contiguous():
            raise ValueError(f"x must be a contiguous tensor of {self.H} x {self.W} pixels")

    def forward(self, x: torch.Tensor, out: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
        self._check_x(x)
        if out is None:
            out = torch.empty((self.H, self.W), dtype=torch.float32, device=x.device)
        if out.dtype != torch.float32 or out.numel() != self.N or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 tensor of H x W elements")
        w = self.workspace(x.device) if ws is None else ws
        _abi.gauss_smooth2d(self.handle, x.data_ptr(), torch_dtype_code(x.dtype), out.data_ptr(), w.data_ptr(),
                            w.numel(), _stream())
        return out

    def autotune(self, *args, **kwargs):
        raise NotImplementedError("autotune does not take image plans")

    def backward(self, gy: torch.Tensor) -> torch.Tensor:
        """dLoss/dx (float32, H x W) for gy = dLoss/dy (float32, H x W)."""
        if not gy.is_cuda or gy.dtype != torch.float32 or gy.numel() != self.N or not gy.is_contiguous():
            raise ValueError("gy must be a contiguous float32 device tensor of H x W elements")
        w = self.workspace(gy.device, backward=True)
        gx = torch.empty((self.H, self.W), dtype=torch.float32, device=gy.device)
        _abi.gauss_smooth2d_backward(self.handle, gy.data_ptr(), gx.data_ptr(), w.data_ptr(), w.numel(), _stream())
        return gx

    def grad(self, x: torch.Tensor, gy: torch.Tensor):
        """(dLoss/dx float32 H x W, float64 [dLoss/dsigma_y, dLoss/dsigma_x]) for the forward
        input x and gy = dLoss/dy (float32, H x W); the fitted coefficients are differentiated
        with each axis's window, terms and shift frozen."""
        self._check_x(x)
        if not gy.is_cuda or gy.dtype != torch.float32 or gy.numel() != self.N or not gy.is_contiguous():
            raise ValueError("gy must be a contiguous float32 device tensor of H x W elements")
        w = self.workspace(gy.device, backward=True)
        gx = torch.empty((self.H, self.W), dtype=torch.float32, device=gy.device)
        gp = torch.empty(2, dtype=torch.float64, device=gy.device)
        _abi.gauss_smooth2d_grad(self.handle, x.data_ptr(), torch_dtype_code(x.dtype), gy.data_ptr(), gx.data_ptr(),
                                 gp.data_ptr(), w.data_ptr(), w.numel(), _stream())
        return gx, gp


class Gabor2DPlan(_PlanBase):
    """Separable 2-D Gabor filter of a real H x W image (row-major, x along a row): the Morlet
    transform of every row (sigma_x, xi in rad/sample, K_x terms), then the Gaussian smoothing
    of every column of its real and imaginary parts (sigma_y, K_y terms); windows 0 are
    error-optimal. Complex64 output; the backward gives dLoss/dx."""

    kind = "gabor"

    def __init__(self, H: int, W: int, sigma_x: float, xi: float, K_x: int, sigma_y: float, K_y: int,
                 L_x: int = 0, L_y: int = 0, mode: str = "sft", n0: int = 0, accum: str = "auto"):
        h = _abi.morlet_plan_gabor2d(int(H), int(W), float(sigma_x), float(xi), int(K_x), int(L_x), float(sigma_y),
                                     int(K_y), int(L_y))
        super().__init__(h, int(H) * int(W), max(int(K_x), int(K_y)))
        self.H, self.W = int(H), int(W)
        self.K_x, self.K_y = int(K_x), int(K_y)
        self.sigma_x, self.xi, self.sigma_y = float(sigma_x), float(xi), float(sigma_y)
        if mode != "sft" or n0 or accum != "auto":
            self.set(mode, n0, accum)

    def info(self) -> dict:
        raise TypeError("use axis_info(0) (Morlet rows) or axis_info(1) (Gaussian columns) for an image plan")

    def axis_info(self, axis: int) -> dict:
        return _abi.morlet_image_axis_info(self.handle, int(axis), self.K_x if int(axis) == 0 else self.K_y)

    def forward(self, x: torch.Tensor, out: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
        if not x.is_cuda:
            raise ValueError("x must be a device tensor")
        if x.numel() != self.N or not x.is_contiguous():
            raise ValueError(f"x must be a contiguous tensor of {self.H} x {self.W} pixels")
        if out is None:
            out = torch.empty((self.H, self.W), dtype=torch.complex64, device=x.device)
        if out.dtype != torch.complex64 or out.numel() != self.N or not out.is_contiguous():
            raise ValueError("out must be a contiguous complex64 tensor of H x W elements")
        w = self.workspace(x.device) if ws is None else ws
        _abi.gabor2d(self.handle, x.data_ptr(), torch_dtype_code(x.dtype), out.data_ptr(), w.data_ptr(), w.numel(),
                     _stream())
        return out

    def autotune(self, *args, **kwargs):
        raise NotImplementedError("autotune does not take image plans")

    def backward(self, gW: torch.Tensor) -> torch.Tensor:
        """dLoss/dx (float32, H x W) for gW = dLoss/dRe y + i dLoss/dIm y (complex64, H x W)."""
        if not gW.is_cuda or gW.dtype != torch.complex64 or gW.numel() != self.N or not gW.is_contiguous():
            raise ValueError("gW must be a contiguous complex64 device tensor of H x W elements")
        w = self.workspace(gW.device, backward=True)
        gx = torch.empty((self.H, self.W), dtype=torch.float32, device=gW.device)
        _abi.gabor2d_backward(self.handle, gW.data_ptr(), gx.data_ptr(), w.data_ptr(), w.numel(), _stream())
        return gx

    def grad(self, x: torch.Tensor, gW: torch.Tensor):
        """(dLoss/dx float32 H x W, float64 [dLoss/dsigma_y, dLoss/dsigma_x, dLoss/dxi]) for the
        forward input x and gW (complex64, H x W), each axis's plan frozen."""
        if not x.is_cuda or x.numel() != self.N or not x.is_contiguous():
            raise ValueError(f"x must be a contiguous device tensor of {self.H} x {self.W} pixels")
        if not gW.is_cuda or gW.dtype != torch.complex64 or gW.numel() != self.N or not gW.is_contiguous():
            raise ValueError("gW must be a contiguous complex64 device tensor of H x W elements")
        w = self.workspace(gW.device, backward=True)
        gx = torch.empty((self.H, self.W), dtype=torch.float32, device=gW.device)
        gp = torch.empty(3, dtype=torch.float64, device=gW.device)
        _abi.gabor2d_grad(self.handle, x.data_ptr(), torch_dtype_code(x.dtype), gW.data_ptr(), gx.data_ptr(),
                          gp.data_ptr(), w.data_ptr(), w.numel(), _stream())
        return gx, gp


class ScalogramPlan(_PlanBase):
    """Batched ragged scalogram: B packed signals x S scales, one persistent launch.
    Output [signal][scale][n] packed: scale s of signal b starts at S*off_b + s*len_b."""

    kind = "scalogram"

    def __init__(self, lengths, sigmas, xis, K: int, L_over_sigma: float = 0.0, mode: str = "sft",
                 n0: int = 0, accum: str = "auto"):
        lengths = [int(v) for v in lengths]
        h = _abi.morlet_scalogram_plan(lengths, list(sigmas), list(xis), int(K), float(L_over_sigma))
        super().__init__(h, int(sum(lengths)), int(K))
        self.lengths = lengths
        self.S = len(sigmas)
        self.sigmas, self.xis = [float(v) for v in sigmas], [float(v) for v in xis]
        if mode != "sft" or n0 or accum != "auto":
            self.set(mode, n0, accum)

    def info(self) -> dict:
        raise TypeError("use scale_info(s) for a scalogram plan")

    def scale_info(self, s: int) -> dict:
        return _abi.morlet_scalogram_scale_info(self.handle, int(s), self.K)

    def out_offset(self, b: int, s: int) -> int:
        return self.S * sum(self.lengths[:b]) + s * self.lengths[b]

    def forward(self, x: torch.Tensor, out: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
        self._check_x(x)
        total = self.S * self.N
        if out is None:
            out = torch.empty(total, dtype=torch.complex64, device=x.device)
        if out.dtype != torch.complex64 or out.numel() != total or not out.is_contiguous():
            raise ValueError("out must be a contiguous complex64 tensor of S * sum(lengths) elements")
        w = self.workspace(x.device) if ws is None else ws
        _abi.morlet_scalogram_forward(self.handle, x.data_ptr(), torch_dtype_code(x.dtype), out.data_ptr(),
                                      w.data_ptr(), w.numel(), _stream())
        return out

    def backward(self, x: torch.Tensor | None, gW: torch.Tensor, want_params: bool = True):
        """(dLoss/dx float32 [sum lengths], dLoss/d(sigma_s, xi_s) float64 [S, 2] or None)."""
        if gW.dtype != torch.complex64 or gW.numel() != self.S * self.N:
            raise ValueError("gW must be complex64 of S * sum(lengths) elements")
        if want_params:
            self._check_x(x)
        gx, gp = _bwd_common(self, _abi.morlet_scalogram_backward, x if want_params else None, gW, want_params,
                             2 * self.S)
        return gx, (gp.view(self.S, 2) if gp is not None else None)


class _MorletFn(torch.autograd.Function):
    """W = psi_hat * x through the library; gradients for x, sigma and xi from its backward
    kernels (window, lowest order and ASFT shift frozen by the plan)."""

    @staticmethod
    def forward(ctx, x, sigma, xi, plan):
        ctx.plan = plan
        # the parameter gradients come back in the parameters' own dtypes (float64 for the
        # layer's parameters), never rounded through float32 on the way
        ctx.param_dtypes = tuple(v.dtype if torch.is_tensor(v) else torch.float64 for v in (sigma, xi))
        ctx.save_for_backward(x)
        return plan.forward(x.contiguous())

    @staticmethod
    def backward(ctx, gW):
        (x,) = ctx.saved_tensors
        want_p = bool(ctx.needs_input_grad[1] or ctx.needs_input_grad[2])
        gx, gp = ctx.plan.backward(x.contiguous(), gW.contiguous().to(torch.complex64), want_params=want_p)
        gs = gxi = None
        if want_p:
            gs = gp[0].to(ctx.param_dtypes[0]) if ctx.needs_input_grad[1] else None
            gxi = gp[1].to(ctx.param_dtypes[1]) if ctx.needs_input_grad[2] else None
        return (gx.to(x.dtype) if ctx.needs_input_grad[0] else None), gs, gxi, None


def morlet_transform(x: torch.Tensor, sigma: torch.Tensor, xi: torch.Tensor, plan: "MorletPlan") -> torch.Tensor:
    """Differentiable Morlet transform of a 1-D device signal with a plan built at (sigma, xi)."""
    return _MorletFn.apply(x, sigma, xi, plan)


class MorletTransform(torch.nn.Module):
    """Morlet transform layer with learnable sigma and xi (rad/sample). The plan (window L,
    lowest order P_S, ASFT shift n0) is chosen once at construction and kept fixed, as the
    parameter gradients assume; whenever sigma or xi change the coefficients are refitted
    into the plan's existing device table on the current stream (morlet_plan_refit: no
    device allocation per step)."""

    def __init__(self, N: int, sigma: float, xi: float, K: int, L: int = 0, mode: str = "sft", n0: int = 0,
                 accum: str = "auto"):
        super().__init__()
        self.sigma = torch.nn.Parameter(torch.tensor(float(sigma), dtype=torch.float64))
        self.xi = torch.nn.Parameter(torch.tensor(float(xi), dtype=torch.float64))
        base = MorletPlan(N, sigma, xi, K, L, mode=mode, n0=n0, accum=accum)
        info = base.info()
        self._cfg = dict(N=N, K=K, L=info["L"], mode=mode, n0=info["n0"], accum=accum, P_S=info["P_S"])
        self._plan, self._key = base, (float(sigma), float(xi))

    def plan(self) -> MorletPlan:
        key = (float(self.sigma.detach()), float(self.xi.detach()))
        if key != self._key:
            self._plan.refit(key[0], key[1])
            self._key = key
        return self._plan

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        return _MorletFn.apply(x, self.sigma, self.xi, self.plan())
