"""ctypes binding of libmorlet.so (include/morlet.h): the same entry points, argument
marshalling only. Device memory and streams come from PyTorch; every step of the
transform runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmorlet.so")

MORLET_OK = 0
MORLET_ERR_INVALID_ARG = 1
MORLET_ERR_UNSUPPORTED = 2
MORLET_ERR_ALLOC = 3
MORLET_ERR_WORKSPACE = 4
MORLET_ERR_HIP = 5

MORLET_F32, MORLET_F16, MORLET_BF16 = 0, 1, 2
MORLET_SCAN_SFT, MORLET_SCAN_ASFT = 0, 1
MORLET_ACC_F32, MORLET_ACC_F64, MORLET_ACC_MIXED, MORLET_ACC_AUTO, MORLET_ACC_KAHAN = 0, 1, 2, 3, 4
MORLET_MAX_TERMS = 12

# every symbol include/morlet.h declares, with (restype, argtypes)
_i64, _i32, _dbl, _vp, _sz = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
_P = ctypes.POINTER
SIGNATURES = {
    "morlet_plan": (ctypes.c_int, [_P(_vp), _i64, _dbl, _dbl, _i32, _i64]),
    "morlet_plan_gauss": (ctypes.c_int, [_P(_vp), _i64, _dbl, _i32, _i64]),
    "morlet_plan_gauss_deriv": (ctypes.c_int, [_P(_vp), _i64, _dbl, _i32, _i64, _i32]),
    "morlet_plan_multiply": (ctypes.c_int, [_P(_vp), _i64, _dbl, _dbl, _i32, _i64]),
    "morlet_plan_gauss2d": (ctypes.c_int, [_P(_vp), _i64, _i64, _dbl, _dbl, _i32, _i64, _i64]),
    "morlet_tree_workspace_size": (ctypes.c_int, [_vp, _P(_sz)]),
    "morlet_plan_set_boundary": (ctypes.c_int, [_vp, ctypes.c_int]),
    "morlet_tree_forward": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp, _sz, _vp]),
    "gauss_smooth2d": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp, _sz, _vp]),
    "morlet_plan_gabor2d": (ctypes.c_int, [_P(_vp), _i64, _i64, _dbl, _dbl, _i32, _i64, _dbl, _i32, _i64]),
    "gabor2d": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp, _sz, _vp]),
    "gabor2d_backward": (ctypes.c_int, [_vp, _vp, _vp, _vp, _sz, _vp]),
    "gauss_smooth2d_grad": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp, _vp, _vp, _sz, _vp]),
    "gabor2d_grad": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp, _vp, _vp, _sz, _vp]),
    "gauss_smooth2d_backward": (ctypes.c_int, [_vp, _vp, _vp, _vp, _sz, _vp]),
    "morlet_image_axis_info": (ctypes.c_int, [_vp, _i32, _P(_i64), _P(_i64), _P(_dbl), _P(_dbl)]),
    "morlet_plan_set": (ctypes.c_int, [_vp, ctypes.c_int, _i64, ctypes.c_int]),
    "morlet_plan_refit": (ctypes.c_int, [_vp, _dbl, _dbl, _vp]),
    "morlet_plan_set_tile": (ctypes.c_int, [_vp, _i32]),
    "morlet_plan_set_schedule": (ctypes.c_int, [_vp, ctypes.c_int]),
    "morlet_plan_set_segments": (ctypes.c_int, [_vp, _i32]),
    "morlet_plan_autotune": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _i32, _P(_i32), _P(_i32), _vp]),
    "morlet_plan_info": (ctypes.c_int, [_vp, _P(_i64), _P(_i32), _P(_i64), _P(_dbl), _P(_dbl), _P(_dbl),
                                        _P(_dbl), _P(_dbl)]),
    "morlet_workspace_size": (ctypes.c_int, [_vp, _P(_sz)]),
    "morlet_workspace_init": (ctypes.c_int, [_vp, _sz, _vp]),
    "morlet_forward": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp, _sz, _vp]),
    "morlet_forward_noalloc": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp]),
    "gauss_smooth": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp, _sz, _vp]),
    "morlet_scalogram_plan": (ctypes.c_int, [_P(_vp), _i32, _P(_i64), _i32, _P(_dbl), _P(_dbl), _i32, _dbl]),
    "morlet_scalogram_scale_info": (ctypes.c_int, [_vp, _i32, _P(_i64), _P(_i32), _P(_i64), _P(_dbl), _P(_dbl),
                                                   _P(_dbl), _P(_dbl), _P(_dbl)]),
    "morlet_scalogram_forward": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp, _sz, _vp]),
    "morlet_backward_workspace_size": (ctypes.c_int, [_vp, _P(_sz)]),
    "morlet_backward": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp, _vp, _vp, _sz, _vp]),
    "gauss_smooth_backward": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp, _vp, _vp, _sz, _vp]),
    "morlet_scalogram_backward": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp, _vp, _vp, _sz, _vp]),
    "morlet_direct_forward": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _i64, _vp]),
    "morlet_choose_terms": (ctypes.c_int, [_dbl, _dbl, _dbl, _P(_i32), _P(_i64), _P(_dbl)]),
    "morlet_choose_terms_gauss": (ctypes.c_int, [_dbl, _dbl, _P(_i32), _P(_i64), _P(_dbl)]),
    "morlet_inject_failure": (ctypes.c_int, [ctypes.c_int, _i32]),
    "morlet_destroy": (None, [_vp]),
    "morlet_last_error": (ctypes.c_char_p, []),
}

_LIB = None


class MorletError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"morlet status {status}: {msg}")
        self.status = status


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built (there is no fallback path)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2110_11866_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def check(status: int) -> None:
    if status != MORLET_OK:
        raise MorletError(status, lib().morlet_last_error().decode())


# ----------------------------------------------------------------- same-name wrappers
def morlet_plan(N: int, sigma: float, xi: float, K: int, L: int) -> int:
    h = ctypes.c_void_p()
    check(lib().morlet_plan(ctypes.byref(h), N, sigma, xi, K, L))
    return h.value


def morlet_plan_gauss(N: int, sigma: float, K: int, L: int) -> int:
    h = ctypes.c_void_p()
    check(lib().morlet_plan_gauss(ctypes.byref(h), N, sigma, K, L))
    return h.value


def morlet_plan_gauss_deriv(N: int, sigma: float, K: int, L: int, order: int) -> int:
    h = ctypes.c_void_p()
    check(lib().morlet_plan_gauss_deriv(ctypes.byref(h), N, sigma, K, L, order))
    return h.value


def morlet_plan_multiply(N: int, sigma: float, xi: float, P_M: int, L: int) -> int:
    h = ctypes.c_void_p()
    check(lib().morlet_plan_multiply(ctypes.byref(h), N, sigma, xi, P_M, L))
    return h.value


def morlet_plan_gauss2d(H: int, W: int, sigma_y: float, sigma_x: float, K: int, L_y: int, L_x: int) -> int:
    h = ctypes.c_void_p()
    check(lib().morlet_plan_gauss2d(ctypes.byref(h), H, W, sigma_y, sigma_x, K, L_y, L_x))
    return h.value


def gauss_smooth2d(plan: int, x_ptr: int, dtype: int, y_ptr: int, ws_ptr: int, ws_bytes: int, stream: int) -> None:
    check(lib().gauss_smooth2d(plan, x_ptr, dtype, y_ptr, ws_ptr, ws_bytes, stream))


def morlet_plan_gabor2d(H: int, W: int, sigma_x: float, xi: float, K_x: int, L_x: int, sigma_y: float, K_y: int,
                        L_y: int) -> int:
    h = ctypes.c_void_p()
    check(lib().morlet_plan_gabor2d(ctypes.byref(h), H, W, sigma_x, xi, K_x, L_x, sigma_y, K_y, L_y))
    return h.value


def gabor2d(plan: int, x_ptr: int, dtype: int, y_ptr: int, ws_ptr: int, ws_bytes: int, stream: int) -> None:
    check(lib().gabor2d(plan, x_ptr, dtype, y_ptr, ws_ptr, ws_bytes, stream))


def gauss_smooth2d_grad(plan: int, x_ptr: int, dtype: int, gy_ptr: int, gx_ptr: int, gp_ptr: int, ws_ptr: int,
                        ws_bytes: int, stream: int) -> None:
    check(lib().gauss_smooth2d_grad(plan, x_ptr, dtype, gy_ptr, gx_ptr, gp_ptr, ws_ptr, ws_bytes, stream))


def gabor2d_grad(plan: int, x_ptr: int, dtype: int, gW_ptr: int, gx_ptr: int, gp_ptr: int, ws_ptr: int,
                 ws_bytes: int, stream: int) -> None:
    check(lib().gabor2d_grad(plan, x_ptr, dtype, gW_ptr, gx_ptr, gp_ptr, ws_ptr, ws_bytes, stream))


def gabor2d_backward(plan: int, gW_ptr: int, gx_ptr: int, ws_ptr: int, ws_bytes: int, stream: int) -> None:
    check(lib().gabor2d_backward(plan, gW_ptr, gx_ptr, ws_ptr, ws_bytes, stream))


def morlet_image_axis_info(plan: int, axis: int, K: int) -> dict:
    L, n0, rel = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
    cc = (ctypes.c_double * K)()
    check(lib().morlet_image_axis_info(plan, axis, ctypes.byref(L), ctypes.byref(n0), cc, ctypes.byref(rel)))
    return {"L": L.value, "n0": n0.value, "cos_coef": list(cc), "kernel_relrmse": rel.value}


def morlet_plan_set(plan: int, mode: int, n0: int, accum: int) -> None:
    check(lib().morlet_plan_set(plan, mode, n0, accum))


def morlet_plan_refit(plan: int, sigma: float, xi: float, stream: int) -> None:
    check(lib().morlet_plan_refit(plan, sigma, xi, stream))


def morlet_plan_set_tile(plan: int, R: int) -> None:
    check(lib().morlet_plan_set_tile(plan, R))


MORLET_SCHED_AUTO, MORLET_SCHED_TILES, MORLET_SCHED_ROWS, MORLET_SCHED_SEGMENTS = 0, 1, 2, 3


def morlet_plan_set_schedule(plan: int, schedule: int) -> None:
    check(lib().morlet_plan_set_schedule(plan, schedule))


def morlet_plan_set_segments(plan: int, tiles: int) -> None:
    check(lib().morlet_plan_set_segments(plan, tiles))


def morlet_plan_autotune(plan: int, x: int, dtype: int, out: int, reps: int, stream: int) -> tuple[int, int]:
    R, sched = ctypes.c_int32(), ctypes.c_int32()
    check(lib().morlet_plan_autotune(plan, x, dtype, out, reps, ctypes.byref(R), ctypes.byref(sched), stream))
    return R.value, sched.value


def morlet_plan_info(plan: int, K: int) -> dict:
    L, ps, n0 = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
    alpha, rel = ctypes.c_double(), ctypes.c_double()
    cc, sc, jac = (ctypes.c_double * K)(), (ctypes.c_double * K)(), (ctypes.c_double * (4 * K))()
    check(lib().morlet_plan_info(plan, ctypes.byref(L), ctypes.byref(ps), ctypes.byref(n0), ctypes.byref(alpha),
                                 cc, sc, jac, ctypes.byref(rel)))
    return {"L": L.value, "P_S": ps.value, "n0": n0.value, "alpha": alpha.value, "cos_coef": list(cc),
            "sin_coef": list(sc), "jac": list(jac), "kernel_relrmse": rel.value}


def morlet_workspace_size(plan: int) -> int:
    n = ctypes.c_size_t()
    check(lib().morlet_workspace_size(plan, ctypes.byref(n)))
    return n.value


def morlet_workspace_init(ws_ptr: int, nbytes: int, stream: int) -> None:
    check(lib().morlet_workspace_init(ws_ptr, nbytes, stream))


def morlet_forward(plan: int, x_ptr: int, dtype: int, W_ptr: int, ws_ptr: int, ws_bytes: int, stream: int) -> None:
    check(lib().morlet_forward(plan, x_ptr, dtype, W_ptr, ws_ptr, ws_bytes, stream))


def morlet_forward_noalloc(plan: int, x_ptr: int, dtype: int, W_ptr: int, stream: int) -> None:
    check(lib().morlet_forward_noalloc(plan, x_ptr, dtype, W_ptr, stream))


def gauss_smooth(plan: int, x_ptr: int, dtype: int, y_ptr: int, ws_ptr: int, ws_bytes: int, stream: int) -> None:
    check(lib().gauss_smooth(plan, x_ptr, dtype, y_ptr, ws_ptr, ws_bytes, stream))


def morlet_scalogram_plan(lengths, sigmas, xis, K: int, L_over_sigma: float = 0.0) -> int:
    B, S = len(lengths), len(sigmas)
    h = ctypes.c_void_p()
    ln = (ctypes.c_int64 * B)(*[int(v) for v in lengths])
    sg = (ctypes.c_double * S)(*[float(v) for v in sigmas])
    xs = (ctypes.c_double * S)(*[float(v) for v in xis])
    check(lib().morlet_scalogram_plan(ctypes.byref(h), B, ln, S, sg, xs, K, float(L_over_sigma)))
    return h.value


def morlet_scalogram_scale_info(plan: int, s: int, K: int) -> dict:
    L, ps, n0 = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
    alpha, rel = ctypes.c_double(), ctypes.c_double()
    cc, sc, jac = (ctypes.c_double * K)(), (ctypes.c_double * K)(), (ctypes.c_double * (4 * K))()
    check(lib().morlet_scalogram_scale_info(plan, s, ctypes.byref(L), ctypes.byref(ps), ctypes.byref(n0),
                                            ctypes.byref(alpha), cc, sc, jac, ctypes.byref(rel)))
    return {"L": L.value, "P_S": ps.value, "n0": n0.value, "alpha": alpha.value, "cos_coef": list(cc),
            "sin_coef": list(sc), "jac": list(jac), "kernel_relrmse": rel.value}


def morlet_scalogram_forward(plan: int, x_ptr: int, dtype: int, W_ptr: int, ws_ptr: int, ws_bytes: int,
                             stream: int) -> None:
    check(lib().morlet_scalogram_forward(plan, x_ptr, dtype, W_ptr, ws_ptr, ws_bytes, stream))


def morlet_backward_workspace_size(plan: int) -> int:
    n = ctypes.c_size_t()
    check(lib().morlet_backward_workspace_size(plan, ctypes.byref(n)))
    return n.value


def morlet_backward(plan, x_ptr, dtype, gW_ptr, gx_ptr, gparams_ptr, ws_ptr, ws_bytes, stream) -> None:
    check(lib().morlet_backward(plan, x_ptr, dtype, gW_ptr, gx_ptr, gparams_ptr, ws_ptr, ws_bytes, stream))


def gauss_smooth_backward(plan, x_ptr, dtype, gy_ptr, gx_ptr, gparams_ptr, ws_ptr, ws_bytes, stream) -> None:
    check(lib().gauss_smooth_backward(plan, x_ptr, dtype, gy_ptr, gx_ptr, gparams_ptr, ws_ptr, ws_bytes, stream))


def morlet_scalogram_backward(plan, x_ptr, dtype, gW_ptr, gx_ptr, gparams_ptr, ws_ptr, ws_bytes, stream) -> None:
    check(lib().morlet_scalogram_backward(plan, x_ptr, dtype, gW_ptr, gx_ptr, gparams_ptr, ws_ptr, ws_bytes,
                                          stream))


def morlet_direct_forward(plan, x_ptr, dtype, W_ptr, half_width, stream) -> None:
    check(lib().morlet_direct_forward(plan, x_ptr, dtype, W_ptr, half_width, stream))


def morlet_destroy(plan: int) -> None:
    lib().morlet_destroy(plan)


def morlet_last_error() -> str:
    return lib().morlet_last_error().decode()


def morlet_tree_workspace_size(plan: int) -> int:
    n = ctypes.c_size_t()
    check(lib().morlet_tree_workspace_size(plan, ctypes.byref(n)))
    return n.value


def morlet_tree_forward(plan: int, x_ptr: int, dtype: int, out_ptr: int, ws_ptr: int, ws_bytes: int,
                        stream: int) -> None:
    check(lib().morlet_tree_forward(plan, x_ptr, dtype, out_ptr, ws_ptr, ws_bytes, stream))


MORLET_BOUNDARY_ZERO, MORLET_BOUNDARY_EDGE = 0, 1


def morlet_plan_set_boundary(plan: int, boundary: int) -> None:
    check(lib().morlet_plan_set_boundary(plan, boundary))


def gauss_smooth2d_backward(plan: int, gy_ptr: int, gx_ptr: int, ws_ptr: int, ws_bytes: int, stream: int) -> None:
    check(lib().gauss_smooth2d_backward(plan, gy_ptr, gx_ptr, ws_ptr, ws_bytes, stream))


def morlet_choose_terms(sigma: float, xi: float, target: float, gauss: bool = False, strict: bool = True):
    """(K, L, kernel relRMSE) of the fewest terms reaching `target`; strict=False returns the
    most accurate K instead of raising when no K reaches it."""
    K, L, e = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_double()
    if gauss:
        st = lib().morlet_choose_terms_gauss(sigma, target, ctypes.byref(K), ctypes.byref(L), ctypes.byref(e))
    else:
        st = lib().morlet_choose_terms(sigma, xi, target, ctypes.byref(K), ctypes.byref(L), ctypes.byref(e))
    if st != MORLET_OK and (strict or st != MORLET_ERR_UNSUPPORTED):
        check(st)
    return K.value, L.value, e.value


def morlet_inject_failure(status: int, nth: int) -> None:
    check(lib().morlet_inject_failure(status, nth))
