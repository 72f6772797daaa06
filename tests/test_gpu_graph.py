"""Graph capture and the autotuner. A captured forward / backward is replayed several times,
with eager work and synchronizations between replays and the input changed in place, and
every replay is checked bitwise against the eager call on the same data (the scans are
deterministic). The autotuner must leave a plan whose results still match the oracle."""
import sys

import numpy as np
import pytest
import torch

from oracle import morlet_oracle as O
from oracle_ps import checked_ps

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


def _replays(fn, xt, fresh, n=4):
    """Capture fn() (which reads xt), then replay it n times on fresh inputs copied into xt,
    comparing each replay with the eager call on the same input."""
    torch.cuda.synchronize()
    fn()                                  # warm-up outside the capture (first-use queries)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        captured = fn()
    torch.cuda.synchronize()
    for k in range(n):
        xt.copy_(fresh(k))
        junk = torch.randn(4096, device=xt.device).sum()   # unrelated eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [c.clone() for c in captured]
        want = fn()
        torch.cuda.synchronize()
        for a, b in zip(got, want):
            assert torch.equal(a, b), k
        del junk


@pytest.mark.parametrize("mode", ["sft", "asft"])
def test_graph_forward_single(mode):
    import paper_2110_11866_amd as M
    _announce("graph-forward", mode)
    N = 50000
    rng = np.random.default_rng(21)
    xt = torch.from_numpy(rng.standard_normal(N).astype(np.float32)).cuda()
    plan = M.MorletPlan(N, 300.0, 6 / 300.0, 6, 1200, mode=mode)
    ws = plan.workspace(xt.device)
    out = torch.empty(N, dtype=torch.complex64, device=xt.device)
    fresh = lambda k: torch.from_numpy(np.random.default_rng(100 + k).standard_normal(N).astype(np.float32)).cuda()
    _replays(lambda: (plan.forward(xt, out=out, ws=ws),), xt, fresh)


@pytest.mark.parametrize("mode", ["sft", "asft"])
def test_graph_forward_segments(mode):
    # the segments schedule's three launches (segment sums, combination, scan with outputs)
    # captured together: 300 000 samples at R = 4, segments of 3 tiles
    import paper_2110_11866_amd as M
    _announce("graph-segments", mode)
    N = 300_000
    rng = np.random.default_rng(23)
    xt = torch.from_numpy(rng.standard_normal(N).astype(np.float32)).cuda()
    plan = M.MorletPlan(N, 64.0, 6 / 64.0, 5, 256, mode=mode)
    plan.set_tile(4).set_schedule("segments").set_segments(3)
    ws = plan.workspace(xt.device)
    out = torch.empty(N, dtype=torch.complex64, device=xt.device)
    fresh = lambda k: torch.from_numpy(np.random.default_rng(200 + k).standard_normal(N).astype(np.float32)).cuda()
    _replays(lambda: (plan.forward(xt, out=out, ws=ws),), xt, fresh)


@pytest.mark.parametrize("schedule", ["tiles", "rows"])
def test_graph_forward_scalogram(schedule):
    import paper_2110_11866_amd as M
    _announce("graph-scalogram", schedule)
    lengths = [0, 37, 4096, 5000, 20000, 123, 65536]
    sigmas = [3.0, 45.0, 1500.0]
    plan = M.ScalogramPlan(lengths, sigmas, [6 / s for s in sigmas], 5, 0.0, mode="asft").set_schedule(schedule)
    n = sum(lengths)
    xt = torch.zeros(n, dtype=torch.float32, device="cuda")
    ws = plan.workspace(xt.device)
    out = torch.empty(plan.S * n, dtype=torch.complex64, device=xt.device)
    fresh = lambda k: torch.from_numpy(np.random.default_rng(200 + k).standard_normal(n).astype(np.float32)).cuda()
    _replays(lambda: (plan.forward(xt, out=out, ws=ws),), xt, fresh)


def test_graph_backward():
    import paper_2110_11866_amd as M
    _announce("graph-backward")
    N = 30000
    plan = M.MorletPlan(N, 100.0, 0.06, 5, 400, mode="asft")
    xt = torch.zeros(N, dtype=torch.float32, device="cuda")
    g = torch.from_numpy((np.random.default_rng(7).standard_normal(N) + 0j).astype(np.complex64)).cuda()
    plan.workspace(xt.device, backward=True)
    fresh = lambda k: torch.from_numpy(np.random.default_rng(300 + k).standard_normal(N).astype(np.float32)).cuda()
    _replays(lambda: plan.backward(xt, g), xt, fresh)


def test_autotune_single_and_scalogram():
    import paper_2110_11866_amd as M
    _announce("autotune")
    N, sigma = 60000, 200.0
    rng = np.random.default_rng(31)
    x = rng.standard_normal(N).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    plan = M.MorletPlan(N, sigma, 6 / sigma, 5, 0, mode="asft")
    choice = plan.autotune(xt, reps=3)
    assert choice["R"] in (4, 8, 16, 32) and choice["schedule"] == "tiles"
    got = plan.forward(xt).cpu().numpy()
    info = plan.info()
    p = O.plan_morlet(sigma, 6 / sigma, 5, info["L"], mode="asft", n0=info["n0"], P_S=checked_ps(sigma, 6 / sigma, 5, info))
    want = O.forward(x.astype(np.float64), p)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) <= 1e-5

    lengths = [5000, 300, 20000]
    sigmas = [4.0, 30.0, 250.0]
    sp = M.ScalogramPlan(lengths, sigmas, [6 / s for s in sigmas], 5, 0.0, mode="asft")
    xs = rng.standard_normal(sum(lengths)).astype(np.float32)
    xst = torch.from_numpy(xs).cuda()
    choice = sp.autotune(xst, reps=2)
    assert choice["R"] in (4, 8, 16, 32) and choice["schedule"] in ("tiles", "rows")
    W = sp.forward(xst).cpu().numpy()
    offs = np.concatenate([[0], np.cumsum(lengths)])
    for b in range(len(lengths)):
        for s in range(len(sigmas)):
            info = sp.scale_info(s)
            p = O.plan_morlet(sigmas[s], 6 / sigmas[s], 5, info["L"], mode="asft", n0=info["n0"], P_S=checked_ps(sigmas[s], 6 / sigmas[s], 5, info))
            want = O.forward(xs[offs[b]:offs[b + 1]].astype(np.float64), p)
            o = sp.out_offset(b, s)
            got = W[o:o + lengths[b]]
            assert np.linalg.norm(got - want) / np.linalg.norm(want) <= 1e-5, (b, s)


def test_graph_newer_forward_paths():
    # the multiplication method (three kernels), the 2-D smoothing and the 2-D Gabor filter
    # (two scans, two transposes each) and the edge-extended forward (extension kernel, scan, device-to-device copy) replay
    # bitwise like their eager calls
    import paper_2110_11866_amd as M
    _announce("graph-newer")
    N = 40000
    xt = torch.from_numpy(np.random.default_rng(5).standard_normal(N).astype(np.float32)).cuda()
    fresh = lambda k: torch.from_numpy(np.random.default_rng(200 + k).standard_normal(N).astype(np.float32)).cuda()
    pm = M.MultiplyPlan(N, 50.0, 6 / 50.0, 3, mode="asft")
    wm, om = pm.workspace(xt.device), torch.empty(N, dtype=torch.complex64, device=xt.device)
    _replays(lambda: (pm.forward(xt, out=om, ws=wm),), xt, fresh)
    pe = M.GaussDerivPlan(N, 40.0, 5, 0, order=1, mode="asft").set_boundary("edge")
    we, oe = pe.workspace(xt.device), torch.empty(N, dtype=torch.float32, device=xt.device)
    _replays(lambda: (pe.forward(xt, out=oe, ws=we),), xt, fresh)
    H, W = 200, 200
    pi = M.Gauss2DPlan(H, W, 5.0, 7.0, 4, mode="asft")
    wi, oi = pi.workspace(xt.device), torch.empty(H, W, dtype=torch.float32, device=xt.device)
    _replays(lambda: (pi.forward(xt, out=oi, ws=wi),), xt, fresh)
    pg = M.Gabor2DPlan(H, W, 4.0, 1.5, 5, 6.0, 4, mode="asft")
    wg, og = pg.workspace(xt.device), torch.empty(H, W, dtype=torch.complex64, device=xt.device)
    _replays(lambda: (pg.forward(xt, out=og, ws=wg),), xt, fresh)


def test_graph_newer_backward_paths():
    # dLoss/dx of the multiplication method (transposed carriers around the three-row adjoint),
    # of the 2-D smoothing (two transposes, two adjoint scans) and of a differential (reversal,
    # forward scan, reversal) replay bitwise like their eager calls, the cotangent changed in place
    import paper_2110_11866_amd as M
    _announce("graph-newer-backward")
    N = 40000
    rnd = lambda seed, n: torch.from_numpy(np.random.default_rng(seed).standard_normal(n).astype(np.float32)).cuda()
    pm = M.MultiplyPlan(N, 50.0, 6 / 50.0, 3, mode="asft")
    gbuf = rnd(8, 2 * N)
    gW = gbuf.view(torch.complex64)
    _replays(lambda: (pm.backward(None, gW)[0],), gbuf, lambda k: rnd(400 + k, 2 * N))
    H, W = 200, 200
    pi = M.Gauss2DPlan(H, W, 5.0, 7.0, 4, mode="asft")
    gy = rnd(9, H * W)
    _replays(lambda: (pi.backward(gy.view(H, W)),), gy, lambda k: rnd(500 + k, H * W))
    xi_ = rnd(12, H * W)
    _replays(lambda: pi.grad(xi_.view(H, W), gy.view(H, W)), gy, lambda k: rnd(800 + k, H * W))
    pg = M.Gabor2DPlan(H, W, 4.0, 1.5, 5, 6.0, 4, mode="asft")
    gc = rnd(11, 2 * H * W)
    _replays(lambda: (pg.backward(gc.view(torch.complex64).view(H, W)),), gc, lambda k: rnd(700 + k, 2 * H * W))
    _replays(lambda: pg.grad(xi_.view(H, W), gc.view(torch.complex64).view(H, W)), gc,
             lambda k: rnd(900 + k, 2 * H * W))
    for mode in ("sft", "asft"):
        pd = M.GaussDerivPlan(N, 40.0, 5, 0, order=2, mode=mode)
        gd = rnd(10, N)
        _replays(lambda: (pd.backward(None, gd)[0],), gd, lambda k: rnd(600 + k, N))
