"""The segments schedule against the FP64 oracle: every row cut into segments of equal tile
counts, a launch for each segment's end state from a zero start, a combination of those into
each segment's incoming state (one block per row), and a launch with outputs. Cases cover
one-tile segments (several per thread of the combination), several tiles per segment with a
ragged last segment, segments longer than 64 tiles (the second level of the look-back weights),
the automatic length, Morlet, Gaussian and Gaussian differential plans in every accumulation,
launches of several rows (a small scalogram, the multiplication method's three rows), and
agreement with the tiles schedule. Bar: relative L2 1e-5 (float32 scan), 1e-6 (float64)."""
import sys

import numpy as np
import pytest
import torch

from oracle import morlet_oracle as O

pytestmark = pytest.mark.gpu

TOL = {"auto": 1e-5, "f32": 1e-5, "f64": 1e-6, "mixed": 1e-5, "kahan": 1e-6}


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_11866_amd  # noqa: F401  (loads libmorlet.so; raises if it is missing)
    yield


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def _announce(*args):
    print("[case]", *args, flush=True)
    sys.stdout.flush()


def _tiles(N, L, n0, R):
    return -(-(N + L - n0) // (256 * R))


# (N, sigma, K, L, R, tiles per segment): tile counts 196, 197, 293, 74
SHAPES = [(200_000, 64.0, 5, 256, 4, 1),        # 196 one-tile segments: 4 per lane of the combination
          (200_000, 300.0, 6, 1200, 4, 3),      # 66 segments, the last one of 2 tiles
          (300_000, 64.0, 4, 256, 4, 70),       # 5 segments of 70 tiles (> 64), the last of 13
          (300_000, 64.0, 4, 256, 16, 0)]       # automatic length


@pytest.mark.parametrize("accum", ["auto", "f32", "f64", "mixed"])
@pytest.mark.parametrize("mode", ["sft", "asft"])
@pytest.mark.parametrize("N,sigma,K,L,R,seg", SHAPES)
def test_morlet_segments_parity(N, sigma, K, L, R, seg, mode, accum):
    import paper_2110_11866_amd as M
    _announce("segments-morlet", N, sigma, K, L, R, seg, mode, accum)
    x = np.random.default_rng(N + K + seg).standard_normal(N).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    plan = M.MorletPlan(N, sigma, 6.0 / sigma, K, L, mode=mode, accum=accum)
    plan.set_tile(R).set_schedule("segments").set_segments(seg)
    got = plan.forward(xt)
    again = plan.forward(xt)
    torch.cuda.synchronize()
    assert torch.equal(got, again)
    info = plan.info()
    assert _tiles(N, info["L"], info["n0"], R) >= 74
    p = O.plan_morlet(sigma, 6.0 / sigma, K, info["L"], mode=mode, n0=info["n0"] if mode == "asft" else None)
    assert p.P_S == info["P_S"]
    want = O.forward(x.astype(np.float64), p)
    assert rel_l2(got.cpu().numpy(), want) <= TOL[accum], rel_l2(got.cpu().numpy(), want)


@pytest.mark.parametrize("mode", ["sft", "asft"])
def test_kahan_segments_parity(mode):
    # the compensated scan (R = 16): 74 tiles in segments of 5
    import paper_2110_11866_amd as M
    _announce("segments-kahan", mode)
    N, sigma, K, L = 300_000, 64.0, 4, 256
    x = np.random.default_rng(41).standard_normal(N).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    plan = M.MorletPlan(N, sigma, 6.0 / sigma, K, L, mode=mode, accum="kahan")
    plan.set_tile(16).set_schedule("segments").set_segments(5)
    got = plan.forward(xt).cpu().numpy()
    info = plan.info()
    p = O.plan_morlet(sigma, 6.0 / sigma, K, info["L"], mode=mode, n0=info["n0"] if mode == "asft" else None)
    want = O.forward(x.astype(np.float64), p)
    assert rel_l2(got, want) <= TOL["kahan"], rel_l2(got, want)


@pytest.mark.parametrize("seg", [1, 4, 0])
@pytest.mark.parametrize("kind", ["gauss", "gd1", "gd2"])
@pytest.mark.parametrize("mode", ["sft", "asft"])
def test_gaussian_segments_parity(kind, mode, seg):
    # Gaussian smoothing and its first and second differentials (real outputs), 147 tiles of 1024
    import paper_2110_11866_amd as M
    _announce("segments-gauss", kind, mode, seg)
    N, sigma, K = 150_000, 32.0, 5
    x = np.random.default_rng(7 + seg).standard_normal(N).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    if kind == "gauss":
        plan = M.GaussPlan(N, sigma, K, 128, mode=mode)
    else:
        plan = M.GaussDerivPlan(N, sigma, K, 128, order=1 if kind == "gd1" else 2, mode=mode)
    plan.set_tile(4).set_schedule("segments").set_segments(seg)
    got = plan.forward(xt).cpu().numpy()
    info = plan.info()
    n0 = info["n0"] if mode == "asft" else None
    if kind == "gauss":
        p = O.plan_gauss(sigma, K, info["L"], mode=mode, n0=n0)
    else:
        p = O.plan_gauss_deriv(sigma, K, info["L"], 1 if kind == "gd1" else 2, mode=mode, n0=n0)
    want = O.forward(x.astype(np.float64), p)
    assert rel_l2(got, want) <= 1e-5, rel_l2(got, want)


@pytest.mark.parametrize("mode", ["sft", "asft"])
def test_segments_against_tiles(mode):
    # the two schedules on one input differ only in the float64 rounding of the carried states
    import paper_2110_11866_amd as M
    _announce("segments-vs-tiles", mode)
    N, sigma, K, L = 2_000_000, 200.0, 5, 800
    x = np.random.default_rng(3).standard_normal(N).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    plan = M.MorletPlan(N, sigma, 6.0 / sigma, K, L, mode=mode)
    a = plan.set_schedule("tiles").forward(xt)
    b = plan.set_schedule("segments").forward(xt)
    torch.cuda.synchronize()
    an, bn = a.cpu().numpy(), b.cpu().numpy()
    assert rel_l2(bn, an) <= 1e-6, rel_l2(bn, an)


@pytest.mark.parametrize("seg", [3, 0])
def test_scalogram_few_rows_segments(seg):
    # a scalogram of two signals x two scales (four rows of different lengths and scales, within
    # the eight rows the schedule takes), every row cut on its own
    import paper_2110_11866_amd as M
    _announce("segments-scalogram", seg)
    lengths = [250_000, 131_071]
    sigmas = [30.0, 300.0]
    xis = [6.0 / s for s in sigmas]
    x = np.random.default_rng(11).standard_normal(sum(lengths)).astype(np.float32)
    plan = M.ScalogramPlan(lengths, sigmas, xis, 5, 0.0, mode="asft")
    plan.set_tile(4).set_schedule("segments").set_segments(seg)
    xt = torch.from_numpy(x).cuda()
    W = plan.forward(xt).cpu().numpy()
    ref = plan.set_schedule("tiles").forward(xt).cpu().numpy()
    assert rel_l2(W, ref) <= 1e-6, rel_l2(W, ref)
    offs = np.concatenate([[0], np.cumsum(lengths)])
    for s in range(len(sigmas)):
        info = plan.scale_info(s)
        p = O.plan_morlet(sigmas[s], xis[s], 5, info["L"], mode="asft", n0=info["n0"])
        assert p.P_S == info["P_S"]
        for b in range(len(lengths)):
            o = plan.out_offset(b, s)
            want = O.forward(x[offs[b]:offs[b + 1]].astype(np.float64), p)
            got = W[o:o + lengths[b]]
            assert rel_l2(got, want) <= 1e-5, (b, s, rel_l2(got, want))


@pytest.mark.parametrize("seg", [2, 0])
def test_multiply_segments(seg):
    # the multiplication method's three Gaussian rows under the segments schedule, against the
    # tiles schedule and the oracle
    import paper_2110_11866_amd as M
    _announce("segments-multiply", seg)
    N, sigma, PM = 400_000, 48.0, 2
    x = np.random.default_rng(13).standard_normal(N).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    plan = M.MultiplyPlan(N, sigma, 6.0 / sigma, PM)
    plan.set_tile(4).set_schedule("segments").set_segments(seg)
    got = plan.forward(xt).cpu().numpy()
    ref = plan.set_schedule("tiles").forward(xt).cpu().numpy()
    assert rel_l2(got, ref) <= 1e-6, rel_l2(got, ref)
    info = plan.info()
    p = O.plan_multiply(sigma, 6.0 / sigma, PM, info["L"])
    want = O.forward(x.astype(np.float64), p)
    assert rel_l2(got, want) <= 1e-5, rel_l2(got, want)


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16])
@pytest.mark.parametrize("mode", ["sft", "asft"])
def test_half_inputs_segments(dtype, mode):
    # 16-bit stored inputs through the segment sums' 16-bit loads and the scan with outputs;
    # the oracle sees the stored values (a random walk plus noise, 196 tiles in segments of 3)
    import paper_2110_11866_amd as M
    _announce("segments-half", dtype, mode)
    N, sigma, K, L = 200_000, 64.0, 5, 256
    x = (np.cumsum(np.random.default_rng(29).standard_normal(N)) / 30).astype(np.float32)
    xt = torch.from_numpy(x).cuda().to(dtype)
    plan = M.MorletPlan(N, sigma, 6.0 / sigma, K, L, mode=mode)
    plan.set_tile(4).set_schedule("segments").set_segments(3)
    got = plan.forward(xt).cpu().numpy()
    info = plan.info()
    p = O.plan_morlet(sigma, 6.0 / sigma, K, info["L"], mode=mode, n0=info["n0"] if mode == "asft" else None)
    want = O.forward(xt.double().cpu().numpy(), p)
    assert rel_l2(got, want) <= 1e-5, rel_l2(got, want)


@pytest.mark.parametrize("kind", ["morlet", "gauss"])
@pytest.mark.parametrize("mode", ["sft", "asft"])
def test_edge_extension_segments(kind, mode):
    # edge extension (the padded copy in the workspace) followed by the segments schedule
    import paper_2110_11866_amd as M
    _announce("segments-edge", kind, mode)
    N, sigma, K = 150_000, 40.0, 5
    x = (np.random.default_rng(31).standard_normal(N) + 2.0).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    if kind == "morlet":
        plan = M.MorletPlan(N, sigma, 6.0 / sigma, K, 160, mode=mode)
    else:
        plan = M.GaussPlan(N, sigma, K, 160, mode=mode)
    plan.set_boundary("edge")
    plan.set_tile(4).set_schedule("segments").set_segments(2)
    got = plan.forward(xt).cpu().numpy()
    info = plan.info()
    n0 = info["n0"] if mode == "asft" else None
    p = (O.plan_morlet(sigma, 6.0 / sigma, K, info["L"], mode=mode, n0=n0) if kind == "morlet"
         else O.plan_gauss(sigma, K, info["L"], mode=mode, n0=n0))
    want = O.forward_edge(x.astype(np.float64), p)
    assert rel_l2(got, want) <= 1e-5, rel_l2(got, want)
