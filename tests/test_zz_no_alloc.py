"""The forward entry point that allocates nothing (morlet_forward_noalloc): its workspace is the
library's fixed device array. Checked through the C ABI against morlet_forward and
morlet_scalogram_forward, which run the same kernels on a caller's workspace, so the outputs
must be equal bit for bit; two calls in a row, the second on a smaller input (the array keeps the
first call's contents); a launch that needs more than the array is refused before anything
runs."""
import ctypes
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_11866_amd  # noqa: F401
    yield


def _announce(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _noalloc(plan, x, W):
    from paper_2110_11866_amd import _abi
    _abi.morlet_forward_noalloc(plan.handle, x.data_ptr(), _abi.MORLET_F32, W.data_ptr(),
                                torch.cuda.current_stream().cuda_stream)


def test_noalloc_matches_forward_on_two_calls():
    import paper_2110_11866_amd as M
    rng = np.random.default_rng(71)
    # a multi-tile single signal (tiles schedule, tile states in the array), then a smaller one
    for N, sigma, K, L, mode in [(1 << 20, 64.0, 5, 0, "asft"), (5000, 16.0, 4, 64, "sft")]:
        _announce("noalloc single", N, sigma, K, L, mode)
        x = torch.from_numpy(rng.standard_normal(N).astype(np.float32)).cuda()
        plan = M.MorletPlan(N, sigma, 6.0 / sigma, K, L, mode=mode)
        want = plan.forward(x)
        got = torch.full_like(want, float("nan"))
        _noalloc(plan, x, got)
        torch.cuda.synchronize()
        assert torch.equal(got, want)


def test_noalloc_matches_scalogram_forward_on_two_calls():
    import paper_2110_11866_amd as M
    rng = np.random.default_rng(72)
    for lengths, mode in [([4096, 70000, 123, 30000, 9000], "asft"), ([3000, 0, 500], "asft")]:
        _announce("noalloc scalogram", lengths, mode)
        sigmas = [3.0, 20.0, 150.0, 900.0]
        plan = M.ScalogramPlan(lengths, sigmas, [6.0 / s for s in sigmas], 5, 0.0, mode=mode)
        x = torch.from_numpy(rng.standard_normal(sum(lengths)).astype(np.float32)).cuda()
        want = plan.forward(x)
        got = torch.full_like(want, float("nan"))
        _noalloc(plan, x, got)
        torch.cuda.synchronize()
        assert torch.equal(got, want)


def test_noalloc_refuses_beyond_its_array():
    # tiles schedule: K = 12 tile states take 640 B, and 2^26 samples at R = 16 need 16 385 tiles,
    # 10.5 MB > 8 MiB. The segments schedule (the automatic choice for this row) keeps one state
    # vector per segment, well inside the array, and matches morlet_forward bit for bit.
    import paper_2110_11866_amd as M
    from paper_2110_11866_amd import _abi
    _announce("noalloc limit")
    N = 1 << 26
    plan = M.MorletPlan(N, 8.0, 6.0 / 8.0, 12, 40).set_schedule("tiles")
    x = torch.randn(N, generator=torch.Generator(device="cuda").manual_seed(2), device="cuda")
    W = torch.zeros(N, dtype=torch.complex64, device="cuda")
    with pytest.raises(_abi.MorletError) as e:
        _noalloc(plan, x, W)
    assert e.value.status == _abi.MORLET_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(W)) == 0
    plan.set_schedule("segments")
    want = plan.forward(x)
    _noalloc(plan, x, W)
    torch.cuda.synchronize()
    assert torch.equal(W, want)
