"""Every compiled term count K = 1..12 (one kernel instantiation set per K) against the FP64
oracle: forward Morlet and Gaussian in SFT and ASFT, the adjoint and the parameter gradients,
on a signal that spans several tiles and ends in a ragged tail."""
import sys

import numpy as np
import pytest
import torch

from oracle import morlet_oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_11866_amd  # noqa: F401
    yield


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


@pytest.mark.parametrize("K", list(range(1, 13)))
def test_every_term_count(K):
    import paper_2110_11866_amd as M
    print("[case] K", K, flush=True)
    sys.stdout.flush()
    N, sigma = 20011, 12.0
    L = max(4 * int(sigma), K + 1)
    rng = np.random.default_rng(100 + K)
    x = rng.standard_normal(N).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    xd = x.astype(np.float64)
    for mode in ("sft", "asft"):
        mp = M.MorletPlan(N, sigma, 6.0 / sigma, K, L, mode=mode)
        info = mp.info()
        op = O.plan_morlet(sigma, 6.0 / sigma, K, L, mode=mode, n0=info["n0"] if mode == "asft" else None)
        assert op.P_S == info["P_S"]
        W = mp.forward(xt)
        assert rel(W.cpu().numpy(), O.forward(xd, op)) <= 1e-5, (mode, "morlet")
        g = torch.from_numpy((rng.standard_normal(N) + 1j * rng.standard_normal(N)).astype(np.complex64)).cuda()
        gx, gp = mp.backward(xt, g)
        gn = g.cpu().numpy().astype(np.complex128)
        assert rel(gx.cpu().numpy(), O.adjoint(gn, op)) <= 1e-5, (mode, "adjoint")
        want = O.param_grads(xd, gn, op)
        assert np.all(np.abs(gp.cpu().numpy() - want) <= 1e-5 * np.abs(want) + 1e-12), (mode, gp, want)

        gpn = M.GaussPlan(N, sigma, K, L, mode=mode)
        ginfo = gpn.info()
        og = O.plan_gauss(sigma, K, L, mode=mode, n0=ginfo["n0"] if mode == "asft" else None)
        assert rel(gpn.forward(xt).cpu().numpy(), O.forward(xd, og)) <= 1e-5, (mode, "gauss")
