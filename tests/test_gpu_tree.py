"""GPU parity of the paper's sliding-sum route (Sec. IV, Algorithm 1; comparison path) against
the FP64 oracle's SFT result."""
import sys

import numpy as np
import pytest
import torch

import workloads
from oracle import morlet_oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def _announce(*args):
    print("[case]", *args, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


@pytest.mark.parametrize("kind", ["morlet", "gauss"])
@pytest.mark.parametrize("N,sigma,K,L,dtype", [(1024, 16.0, 4, 64, torch.float32),
                                               (50000, 300.0, 6, 1200, torch.float32),
                                               (77777, 2000.0, 5, 8000, torch.bfloat16),
                                               (9000, 1.5, 12, 12, torch.float16),
                                               (1, 4.0, 2, 16, torch.float32),
                                               (3000, 40.0, 5, 255, torch.float32)])
def test_tree_parity(N, sigma, K, L, dtype, kind):
    import paper_2110_11866_amd as M
    _announce("tree", kind, N, sigma, K, L, dtype)
    x = np.random.default_rng(N + K).standard_normal(N).astype(np.float32)
    xt = torch.from_numpy(x).cuda().to(dtype)
    plan = M.MorletPlan(N, sigma, 6.0 / sigma, K, L) if kind == "morlet" else M.GaussPlan(N, sigma, K, L)
    got = plan.tree(xt).cpu().numpy()
    scan = plan.forward(xt).cpu().numpy()
    torch.cuda.synchronize()
    info = plan.info()
    p = (O.plan_morlet(sigma, 6.0 / sigma, K, info["L"]) if kind == "morlet" else O.plan_gauss(sigma, K, info["L"]))
    want = O.forward(xt.double().cpu().numpy(), p)
    print(f"[result] tree {rel_l2(got, want):.2e} scan {rel_l2(scan, want):.2e}", flush=True)
    assert rel_l2(got, want) <= 1e-5, rel_l2(got, want)


def test_tree_paper_scale():
    # N = 102400, sigma = 8192, K = 6, L = 32768: 17 doubling levels, 8 of them over global memory
    import paper_2110_11866_amd as M
    _announce("tree-paper-scale")
    N, sigma, K, L = 102400, 8192.0, 6, 32768
    x = workloads.paper_scale_signal(N)
    xt = torch.from_numpy(x).cuda()
    plan = M.MorletPlan(N, sigma, 6.0 / sigma, K, L)
    got = plan.tree(xt).cpu().numpy()
    torch.cuda.synchronize()
    p = O.plan_morlet(sigma, 6.0 / sigma, K, L)
    want = O.forward(x.astype(np.float64), p)
    print(f"[result] tree {rel_l2(got, want):.2e}", flush=True)
    assert rel_l2(got, want) <= 1e-5, rel_l2(got, want)
