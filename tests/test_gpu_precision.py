"""Precision stress: N = 2^22 random walk plus white noise stored as float16 / bfloat16,
sigma in {1024, 65536}, K = 6, window 4 sigma. Every scan mode against the FP64 oracle on
the dequantised stored values: the default, the float32 and the mixed scans within 1e-5
relative L2 (plain float32 SFT with a loose sanity bound), the compensated float32 scan and
the float64 scan within 1e-6. Each case prints its error ([result] lines)."""
import sys

import numpy as np
import pytest
import torch

import workloads
from oracle import morlet_oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def signal():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_11866_amd  # noqa: F401
    return workloads.precision_stress_signal()


_oracle_cache = {}


def _oracle(xq, key, sigma, K, L, mode, n0):
    k = (key, sigma, mode)
    if k not in _oracle_cache:
        p = O.plan_morlet(sigma, 6.0 / sigma, K, L, mode=mode, n0=n0 if mode == "asft" else None)
        _oracle_cache[k] = (O.forward(xq, p), p.P_S)
    return _oracle_cache[k]


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16])
@pytest.mark.parametrize("sigma", [1024.0, 65536.0])
# Plain float32 SFT (no attenuation) keeps the rounding of every tile aggregate in its state to
# the row's end; at 2^22 samples it is reported with a loose sanity bound, not held to 1e-5 (the
# default "auto" runs the mixed scan for SFT).
@pytest.mark.parametrize("mode,accum,tol", [("sft", "auto", 1e-5), ("asft", "auto", 1e-5),
                                            ("sft", "f32", 1e-3), ("asft", "f32", 1e-5),
                                            ("sft", "mixed", 1e-5), ("asft", "mixed", 1e-5),
                                            ("sft", "f64", 1e-6), ("asft", "f64", 1e-6),
                                            ("sft", "kahan", 1e-6), ("asft", "kahan", 1e-6)])
def test_precision_stress(signal, dtype, sigma, mode, accum, tol):
    import paper_2110_11866_amd as M
    print("[case] precision", dtype, sigma, mode, accum, flush=True)
    sys.stdout.flush()
    N, K, L = signal.shape[0], 6, int(4 * sigma)
    xt = torch.from_numpy(signal).to("cuda").to(dtype)
    plan = M.MorletPlan(N, sigma, 6.0 / sigma, K, L, mode=mode, accum=accum)
    got = plan.forward(xt).cpu().numpy()
    torch.cuda.synchronize()
    info = plan.info()
    want, ps = _oracle(xt.double().cpu().numpy(), str(dtype), sigma, K, L, mode, info["n0"])
    assert ps == info["P_S"]
    err = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    print(f"[result] {dtype} sigma={sigma} {mode}/{accum}: rel-L2 {err:.3e}", flush=True)
    assert err <= tol, err
