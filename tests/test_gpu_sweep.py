"""Seeded random sweep of the GPU path against the FP64 oracle: single-signal forwards over the
whole plan space (kind, mode, accumulation, input type, tile shape, boundary, size, sigma, K,
window) and random ragged scalograms. Each case is drawn from its own seed, so a failure names
a reproducible configuration."""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import morlet_oracle as O
from oracle_ps import checked_ps

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f64": 1e-6, "mixed": 1e-5}
DT = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def _announce(*args):
    print("[case]", *args, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def _draw(seed):
    rng = np.random.default_rng(seed)
    kind = ["morlet", "gauss", "gd1", "gd2"][int(rng.integers(0, 4))]
    mode = ["sft", "asft"][int(rng.integers(0, 2))]
    accum = ["f32", "f64"][int(rng.integers(0, 2))]
    dt = ["f32", "f16", "bf16"][int(rng.integers(0, 3))]
    tile = [4, 8, 16, 32][int(rng.integers(0, 4))]
    edge = bool(rng.integers(0, 4) == 0)
    N = int(math.exp(rng.uniform(0.0, math.log(2e5))))
    sigma = float(math.exp(rng.uniform(math.log(1.5), math.log(3000.0))))
    K = int(rng.integers(1, 13))
    L = 0 if rng.integers(0, 2) == 0 else max(K + 1, int(sigma * rng.uniform(2.0, 5.0)))
    return kind, mode, accum, dt, tile, edge, N, sigma, K, L


@pytest.mark.parametrize("seed", range(60))
def test_random_single_signal(seed):
    import paper_2110_11866_amd as M
    kind, mode, accum, dt, tile, edge, N, sigma, K, L = _draw(1000 + seed)
    _announce("sweep", seed, kind, mode, accum, dt, tile, "edge" if edge else "zero", N, round(sigma, 3), K, L)
    x = np.random.default_rng(seed).standard_normal(N).astype(np.float32)
    xt = torch.from_numpy(x).cuda().to(DT[dt])
    xi = 6.0 / sigma
    if kind == "morlet":
        plan = M.MorletPlan(N, sigma, xi, K, L, mode=mode, accum=accum)
    elif kind == "gauss":
        plan = M.GaussPlan(N, sigma, K, L, mode=mode, accum=accum)
    else:
        plan = M.GaussDerivPlan(N, sigma, K, L, order=1 if kind == "gd1" else 2, mode=mode, accum=accum)
    plan.set_tile(tile)
    if edge:
        plan.set_boundary("edge")
    got = plan.forward(xt).cpu().numpy()
    torch.cuda.synchronize()
    info = plan.info()
    n0 = info["n0"] if mode == "asft" else None
    if kind == "morlet":
        p = O.plan_morlet(sigma, xi, K, info["L"], mode=mode, n0=n0, P_S=checked_ps(sigma, xi, K, info))
    elif kind == "gauss":
        p = O.plan_gauss(sigma, K, info["L"], mode=mode, n0=n0)
    else:
        p = O.plan_gauss_deriv(sigma, K, info["L"], 1 if kind == "gd1" else 2, mode=mode, n0=n0)
    xd = xt.double().cpu().numpy()
    want = O.forward_edge(xd, p) if edge else O.forward(xd, p)
    # an extended constant through an odd or zero-mean kernel is exactly zero: judge such a
    # result against the input's scale instead
    scale = max(np.linalg.norm(want), 1e-6 * np.linalg.norm(xd) * np.abs(O.asft_kernel(p) if mode == "asft" else
                                                                         (O.kterm_morlet(p) if kind == "morlet" else
                                                                          O.kterm_gauss_deriv(p) if kind in ("gd1", "gd2")
                                                                          else O.kterm_gauss(p))).sum())
    err = float(np.linalg.norm(got - want) / scale)
    assert err <= TOL[accum], err


@pytest.mark.parametrize("seed", range(10))
def test_random_scalogram(seed):
    import paper_2110_11866_amd as M
    rng = np.random.default_rng(5000 + seed)
    B, S = int(rng.integers(1, 9)), int(rng.integers(1, 7))
    lengths = [int(math.exp(rng.uniform(0.0, math.log(60000)))) if rng.integers(0, 6) else 0 for _ in range(B)]
    sigmas = sorted(float(math.exp(rng.uniform(math.log(2.0), math.log(2000.0)))) for _ in range(S))
    xis = [float(rng.uniform(2.0, 8.0)) / s for s in sigmas]
    K = int(rng.integers(2, 9))
    mode = ["sft", "asft"][int(rng.integers(0, 2))]
    tile = [4, 8, 16, 32][int(rng.integers(0, 4))]
    schedule = ["auto", "tiles", "rows"][int(rng.integers(0, 3))]
    _announce("sweep-scalogram", seed, B, S, lengths, [round(s, 2) for s in sigmas], K, mode, tile, schedule)
    x = np.random.default_rng(seed).standard_normal(max(sum(lengths), 1)).astype(np.float32)[:sum(lengths)]
    plan = M.ScalogramPlan(lengths, sigmas, xis, K, 0.0, mode=mode)
    plan.set_tile(tile).set_schedule(schedule)
    if sum(lengths) == 0:
        return
    xt = torch.from_numpy(x).cuda()
    W = plan.forward(xt).cpu().numpy()
    torch.cuda.synchronize()
    offs = np.concatenate([[0], np.cumsum(lengths)])
    for b in range(B):
        for s in range(S):
            if lengths[b] == 0:
                continue
            info = plan.scale_info(s)
            p = O.plan_morlet(sigmas[s], xis[s], K, info["L"], mode=mode, n0=info["n0"] if mode == "asft" else None,
                              P_S=checked_ps(sigmas[s], xis[s], K, info))
            want = O.forward(x[offs[b]:offs[b + 1]].astype(np.float64), p)
            o = plan.out_offset(b, s)
            assert rel_l2(W[o:o + lengths[b]], want) <= 1e-5, (b, s, rel_l2(W[o:o + lengths[b]], want))


@pytest.mark.parametrize("seed", range(15))
def test_random_backward(seed):
    # dLoss/dx against the oracle adjoint and dLoss/dsigma, dLoss/dxi against the oracle's
    # parameter gradients (frozen plan), random cotangent
    import paper_2110_11866_amd as M
    rng = np.random.default_rng(9000 + seed)
    kind = ["morlet", "gauss"][int(rng.integers(0, 2))]
    mode = ["sft", "asft"][int(rng.integers(0, 2))]
    accum = ["f32", "f64"][int(rng.integers(0, 2))]
    tile = [4, 8, 16, 32][int(rng.integers(0, 4))]
    N = int(math.exp(rng.uniform(0.0, math.log(1e5))))
    sigma = float(math.exp(rng.uniform(math.log(2.0), math.log(1000.0))))
    K = int(rng.integers(2, 9))
    L = 0 if rng.integers(0, 2) == 0 else max(K + 1, int(sigma * rng.uniform(2.0, 5.0)))
    _announce("sweep-backward", seed, kind, mode, accum, tile, N, round(sigma, 3), K, L)
    x = rng.standard_normal(N).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    if kind == "morlet":
        plan = M.MorletPlan(N, sigma, 6.0 / sigma, K, L, mode=mode, accum=accum)
        g = (rng.standard_normal(N) + 1j * rng.standard_normal(N)).astype(np.complex64)
    else:
        plan = M.GaussPlan(N, sigma, K, L, mode=mode, accum=accum)
        g = rng.standard_normal(N).astype(np.float32)
    plan.set_tile(tile)
    gx, gp = plan.backward(xt, torch.from_numpy(g).cuda())
    torch.cuda.synchronize()
    info = plan.info()
    n0 = info["n0"] if mode == "asft" else None
    p = (O.plan_morlet(sigma, 6.0 / sigma, K, info["L"], mode=mode, n0=n0, P_S=checked_ps(sigma, 6.0 / sigma, K, info)) if kind == "morlet"
         else O.plan_gauss(sigma, K, info["L"], mode=mode, n0=n0))
    gn = g.astype(np.complex128 if kind == "morlet" else np.float64)
    assert rel_l2(gx.cpu().numpy(), O.adjoint(gn, p)) <= TOL[accum]
    want = O.param_grads(x.astype(np.float64), gn, p)
    got = gp.cpu().numpy()
    floor = 1e-9 * np.linalg.norm(x) * np.linalg.norm(g)
    idx = [0] if kind == "gauss" else [0, 1]
    assert np.all(np.abs(got[idx] - want[idx]) <= 1e-5 * np.abs(want[idx]) + floor), (got, want)
