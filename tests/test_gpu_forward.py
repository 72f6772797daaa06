"""Forward parity of the HIP path (through the C ABI) against the FP64 oracle on the same
seeded inputs. Floating-point bar: relative L2 error <= 1e-5 (float32 scan); the
float64 scan mode is held to 1e-6."""
import math
import sys

import numpy as np
import pytest
import torch

import workloads
from oracle import morlet_oracle as O
from oracle_ps import checked_ps

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


def run_gpu(x32, kind, sigma, K, L, mode="sft", n0=0, accum="auto", dtype=torch.float32, xi=None, repeats=1,
            tile=16):
    import paper_2110_11866_amd as M
    N = len(x32)
    xt = torch.from_numpy(np.ascontiguousarray(x32)).to("cuda").to(dtype)
    if kind == "morlet":
        plan = M.MorletPlan(N, sigma, xi if xi is not None else 6.0 / sigma, K, L, mode=mode, n0=n0, accum=accum)
    else:
        plan = M.GaussPlan(N, sigma, K, L, mode=mode, n0=n0, accum=accum)
    plan.set_tile(tile)
    outs = []
    for _ in range(repeats):
        outs.append(plan.forward(xt).cpu().numpy())
    torch.cuda.synchronize()
    info = plan.info()
    x_used = xt.double().cpu().numpy()        # the values the kernel actually read
    return outs, info, x_used


def oracle_of(x, kind, sigma, K, L, info, mode, xi=None):
    if kind == "morlet":
        xi = xi if xi is not None else 6.0 / sigma
        p = O.plan_morlet(sigma, xi, K, info["L"], mode=mode, n0=info["n0"] if mode == "asft" else None)
        assert p.P_S == info["P_S"]
    else:
        p = O.plan_gauss(sigma, K, info["L"], mode=mode, n0=info["n0"] if mode == "asft" else None)
    return O.forward(x, p), p


MODES = [("sft", "f32"), ("asft", "f32"), ("sft", "f64"), ("asft", "f64"), ("sft", "mixed"), ("asft", "mixed")]
# the compensated scan is built for R = 16 (the default tile) only
MODES16 = MODES + [("sft", "kahan"), ("asft", "kahan"), ("sft", "auto"), ("asft", "auto")]


@pytest.mark.parametrize("mode,accum", MODES16)
@pytest.mark.parametrize("kind", ["morlet", "gauss"])
def test_small_config_parity(kind, mode, accum):
    # N = 1024, sigma = 16, K = 4, L = 64 (one tile), i.i.d. N(0, 1)
    _announce("small", kind, mode, accum)
    x = workloads.small_signal().astype(np.float32)
    (got,), info, xu = run_gpu(x, kind, 16.0, 4, 64, mode=mode, accum=accum)
    want, _ = oracle_of(xu, kind, 16.0, 4, 64, info, mode)
    assert got.shape == want.shape
    assert rel_l2(got, want) <= TOL[accum], rel_l2(got, want)


@pytest.mark.parametrize("mode,accum", MODES16)
@pytest.mark.parametrize("N,sigma,K,L", [(50000, 300.0, 6, 1200), (4096 * 3, 40.0, 5, 160), (77777, 2000.0, 3, 8000),
                                         (9000, 1.5, 12, 12)])
def test_multi_tile_parity(N, sigma, K, L, mode, accum):
    _announce("multi", N, sigma, K, L, mode, accum)
    x = np.random.default_rng(N + K).standard_normal(N).astype(np.float32)
    (got,), info, xu = run_gpu(x, "morlet", sigma, K, L, mode=mode, accum=accum)
    want, _ = oracle_of(xu, "morlet", sigma, K, L, info, mode)
    assert rel_l2(got, want) <= TOL[accum], rel_l2(got, want)


@pytest.mark.parametrize("N", [1, 2, 7, 63, 64, 65, 129, 4095, 4096, 4097, 8191])
@pytest.mark.parametrize("mode", ["sft", "asft"])
def test_edge_lengths(N, mode):
    # signals shorter than the window, exactly one tile, one past a tile, ragged tails
    _announce("edge", N, mode)
    sigma, K, L = 16.0, 4, 64
    x = np.random.default_rng(N).standard_normal(N).astype(np.float32)
    for kind in ("morlet", "gauss"):
        (got,), info, xu = run_gpu(x, kind, sigma, K, L, mode=mode)
        want, _ = oracle_of(xu, kind, sigma, K, L, info, mode)
        assert got.shape == (N,)
        assert rel_l2(got, want) <= 1e-5, (kind, rel_l2(got, want))


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16])
@pytest.mark.parametrize("mode", ["sft", "asft"])
def test_half_inputs(dtype, mode):
    _announce("half", dtype, mode)
    N, sigma, K, L = 30000, 200.0, 6, 800
    x = (np.cumsum(np.random.default_rng(9).standard_normal(N)) / 30).astype(np.float32)
    (got,), info, xu = run_gpu(x, "morlet", sigma, K, L, mode=mode, dtype=dtype)
    want, _ = oracle_of(xu, "morlet", sigma, K, L, info, mode)   # oracle sees the stored half values
    assert rel_l2(got, want) <= 1e-5, rel_l2(got, want)


@pytest.mark.parametrize("mode,accum", MODES16)
def test_paper_scale_parity(mode, accum):
    # N = 102400, sigma = 8192, xi = 6/sigma, K = 6, L = 32768; three sinusoids plus noise
    _announce("paper-scale", mode, accum)
    x = workloads.paper_scale_signal()
    (got,), info, xu = run_gpu(x, "morlet", 8192.0, 6, 32768, mode=mode, accum=accum)
    want, p = oracle_of(xu, "morlet", 8192.0, 6, 32768, info, mode)
    assert info["P_S"] == 5
    assert rel_l2(got, want) <= TOL[accum], rel_l2(got, want)
    # the first and last L + n0 outputs (partial windows at the signal's ends) on their own
    e = info["L"] + info["n0"]
    assert rel_l2(got[:e], want[:e]) <= TOL[accum], rel_l2(got[:e], want[:e])
    assert rel_l2(got[-e:], want[-e:]) <= TOL[accum], rel_l2(got[-e:], want[-e:])


def test_long_row_lookback_and_repeat_determinism():
    # 2^20 samples: 256+ tiles in one row, look-back windows longer than 64 predecessors;
    # three calls on one workspace must give identical bits (workspace re-armed by the kernel)
    _announce("long-row")
    N, sigma, K, L = 1 << 20, 512.0, 5, 2048
    x = np.random.default_rng(21).standard_normal(N).astype(np.float32)
    outs, info, xu = run_gpu(x, "morlet", sigma, K, L, repeats=3)
    want, _ = oracle_of(xu, "morlet", sigma, K, L, info, "sft")
    assert rel_l2(outs[0], want) <= 1e-5, rel_l2(outs[0], want)
    assert np.array_equal(outs[0].view(np.uint32), outs[1].view(np.uint32))
    assert np.array_equal(outs[0].view(np.uint32), outs[2].view(np.uint32))


def test_impulse_response_on_gpu():
    _announce("impulse")
    N, sigma, K, L, c = 3000, 50.0, 6, 200, 1400
    x = np.zeros(N, np.float32)
    x[c] = 1.0
    (got,), info, xu = run_gpu(x, "morlet", sigma, K, L)
    p = O.plan_morlet(sigma, 6 / sigma, K, L)
    want = np.zeros(N, np.complex128)
    want[c - L:c + L + 1] = O.kterm_morlet(p)
    assert rel_l2(got, want) <= 1e-5


def test_kterm_bound_against_direct_convolution():
    # the K-term result is as far from the direct transform as the oracle says, no further
    _announce("direct-bound")
    N, sigma, K, L = 20000, 100.0, 6, 400
    x = np.random.default_rng(4).standard_normal(N).astype(np.float32)
    (got,), info, xu = run_gpu(x, "morlet", sigma, K, L)
    direct = O.forward_direct(xu, sigma, 6 / sigma, L)
    want, _ = oracle_of(xu, "morlet", sigma, K, L, info, "sft")
    assert np.linalg.norm(got - direct) <= np.linalg.norm(want - direct) + 1e-5 * np.linalg.norm(want)


@pytest.mark.parametrize("N,sigma,H,dtype", [(5000, 40.0, 120, torch.float32), (20000, 500.0, 1500, torch.float32),
                                             (3001, 300.0, 2000, torch.bfloat16), (777, 16.0, 0, torch.float16)])
def test_direct_convolution_baseline(N, sigma, H, dtype):
    # the truncated direct convolution the benchmark compares against, with the exact taps
    import paper_2110_11866_amd as M
    _announce("direct", N, sigma, H, dtype)
    rng = np.random.default_rng(N)
    xt = torch.from_numpy(rng.standard_normal(N).astype(np.float32)).to("cuda").to(dtype)
    plan = M.MorletPlan(N, sigma, 6.0 / sigma, 5, 4 * int(sigma))
    got = plan.direct(xt, H).cpu().numpy()
    torch.cuda.synchronize()
    want = O.forward_direct(xt.double().cpu().numpy(), sigma, 6.0 / sigma, H if H else plan.info()["L"])
    assert rel_l2(got, want) <= 1e-5, rel_l2(got, want)


@pytest.mark.parametrize("mode,accum", MODES)
@pytest.mark.parametrize("kind", ["morlet", "gauss"])
@pytest.mark.parametrize("N,sigma,K,L,dtype", [(50000, 300.0, 6, 1200, torch.float32),
                                               (77777, 2000.0, 3, 8000, torch.bfloat16),
                                               (9000, 1.5, 12, 12, torch.float16)])
def test_tile32_parity(N, sigma, K, L, dtype, kind, mode, accum):
    # 32 positions per thread (8192-position tiles, two store sub-runs per thread)
    _announce("tile32", N, sigma, K, L, dtype, kind, mode, accum)
    x = np.random.default_rng(N + K).standard_normal(N).astype(np.float32)
    (got,), info, xu = run_gpu(x, kind, sigma, K, L, mode=mode, accum=accum, dtype=dtype, tile=32)
    want, _ = oracle_of(xu, kind, sigma, K, L, info, mode)
    assert rel_l2(got, want) <= TOL[accum], rel_l2(got, want)


@pytest.mark.parametrize("tile", [4, 8])
@pytest.mark.parametrize("mode,accum", MODES)
@pytest.mark.parametrize("kind", ["morlet", "gauss"])
@pytest.mark.parametrize("N,sigma,K,L,dtype", [(50000, 300.0, 6, 1200, torch.float32),
                                               (77777, 2000.0, 3, 8000, torch.bfloat16),
                                               (9000, 1.5, 12, 12, torch.float16),
                                               (1, 4.0, 2, 16, torch.float32),
                                               (4099, 40.0, 5, 0, torch.float32)])
def test_small_tile_parity(N, sigma, K, L, dtype, kind, mode, accum, tile):
    # 4 or 8 positions per thread (1024- or 2048-position tiles, one store sub-run per thread)
    _announce("small-tile", tile, N, sigma, K, L, dtype, kind, mode, accum)
    x = np.random.default_rng(N + K + tile).standard_normal(N).astype(np.float32)
    (got,), info, xu = run_gpu(x, kind, sigma, K, L, mode=mode, accum=accum, dtype=dtype, tile=tile)
    want, _ = oracle_of(xu, kind, sigma, K, L, info, mode)
    assert rel_l2(got, want) <= TOL[accum], rel_l2(got, want)


@pytest.mark.parametrize("tile", [16, 4])
@pytest.mark.parametrize("mode", ["sft", "asft"])
def test_paper_scale_within_truncation_bound_of_direct(mode, tile):
    # N = 102400, sigma = 8192, K = 6, L = 32768: the K-term result against the exact Morlet
    # convolution on [-L, L] (oracle, FFT convolution) is held to the oracle's own K-term
    # truncation error plus the float32 bar, ||W_gpu - W_dir|| <= ||W_K - W_dir|| + 1e-5 ||W_K||;
    # the GPU direct convolution of the same window matches the oracle's within 1e-5
    import paper_2110_11866_amd as M
    _announce("paper-scale-vs-direct", mode, tile)
    N, sigma, K, L = 102400, 8192.0, 6, 32768
    x = workloads.paper_scale_signal(N)
    xt = torch.from_numpy(x).cuda()
    plan = M.MorletPlan(N, sigma, 6.0 / sigma, K, L, mode=mode)
    plan.set_tile(tile)
    got = plan.forward(xt).cpu().numpy().astype(np.complex128)
    gdir = plan.direct(xt, L).cpu().numpy().astype(np.complex128)
    torch.cuda.synchronize()
    info = plan.info()
    p = O.plan_morlet(sigma, 6.0 / sigma, K, L, mode=mode, n0=info["n0"] if mode == "asft" else None)
    xd = x.astype(np.float64)
    wk = O.forward(xd, p)
    wdir = O.forward_direct(xd, sigma, 6.0 / sigma, L)
    trunc = np.linalg.norm(wk - wdir)
    print(f"[result] {mode}: K-term vs direct {trunc / np.linalg.norm(wdir):.3e}", flush=True)
    assert rel_l2(got, wk) <= 1e-5, rel_l2(got, wk)
    assert np.linalg.norm(got - wdir) <= trunc + 1e-5 * np.linalg.norm(wk)
    assert rel_l2(gdir, wdir) <= 1e-5, rel_l2(gdir, wdir)


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("N,sigma,K,L,tile,dtype,accum", [
    (1024, 16.0, 4, 64, 16, torch.float32, "f32"),
    (50000, 300.0, 6, 1200, 16, torch.float32, "f32"),
    (77777, 2000.0, 5, 0, 32, torch.bfloat16, "f32"),
    (9000, 1.5, 12, 12, 16, torch.float16, "f32"),
    (50000, 300.0, 6, 1200, 16, torch.float32, "f64"),
    (30000, 100.0, 5, 0, 8, torch.float32, "f32"),
    (3000, 12.0, 3, 0, 4, torch.float32, "f32"),
])
def test_gaussian_differential_parity(N, sigma, K, L, tile, dtype, accum, order):
    # x_GD (sine components 1..K) and x_GDD (cosine components 0..K-1), SFT (Sec. II-A)
    import paper_2110_11866_amd as M
    _announce("gauss-deriv", order, N, sigma, K, L, tile, dtype, accum)
    x = np.random.default_rng(N + order).standard_normal(N).astype(np.float32)
    xt = torch.from_numpy(x).to("cuda").to(dtype)
    plan = M.GaussDerivPlan(N, sigma, K, L, order=order, accum=accum)
    plan.set_tile(tile)
    got = plan.forward(xt).cpu().numpy()
    torch.cuda.synchronize()
    info = plan.info()
    p = O.plan_gauss_deriv(sigma, K, info["L"], order)
    want = O.forward(xt.double().cpu().numpy(), p)
    assert rel_l2(got, want) <= TOL[accum], rel_l2(got, want)


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("N,sigma,K,L,n0,tile,dtype,accum", [
    (1024, 16.0, 4, 64, 2, 16, torch.float32, "f32"),
    (200, 66.0, 5, 256, 10, 16, torch.float32, "f32"),        # Table 1's setup, N < L
    (50000, 300.0, 6, 1200, 0, 16, torch.float32, "f32"),
    (77777, 2000.0, 5, 0, 0, 32, torch.bfloat16, "f32"),
    (9000, 3.0, 6, 12, 1, 16, torch.float16, "f32"),
    (4099, 40.0, 1, 120, 5, 16, torch.float32, "f32"),         # one term: cosine of order 0 only
    (50000, 300.0, 6, 1200, 0, 32, torch.float32, "f64"),
    (30000, 100.0, 5, 0, 0, 8, torch.float32, "f32"),
    (3000, 12.0, 3, 0, 2, 4, torch.float32, "f32"),
])
def test_gaussian_differential_asft_parity(N, sigma, K, L, n0, tile, dtype, accum, order):
    # x_GD and x_GDD by the attenuated transform (eq. gddAsft): orders 0..K-1, both components
    import paper_2110_11866_amd as M
    _announce("gauss-deriv-asft", order, N, sigma, K, L, n0, tile, dtype, accum)
    x = np.random.default_rng(N + 3 * order).standard_normal(N).astype(np.float32)
    xt = torch.from_numpy(x).to("cuda").to(dtype)
    plan = M.GaussDerivPlan(N, sigma, K, L, order=order, mode="asft", n0=n0, accum=accum)
    plan.set_tile(tile)
    got = plan.forward(xt).cpu().numpy()
    torch.cuda.synchronize()
    info = plan.info()
    assert info["P_S"] == 0 and info["n0"] >= 1
    p = O.plan_gauss_deriv(sigma, K, info["L"], order, mode="asft", n0=info["n0"])
    want = O.forward(xt.double().cpu().numpy(), p)
    assert rel_l2(got, want) <= TOL[accum], rel_l2(got, want)


@pytest.mark.parametrize("schedule", ["tiles", "segments"])
@pytest.mark.parametrize("mode", ["sft", "asft"])
def test_long_row_crosses_super_groups(mode, schedule):
    # one 17e6-sample row: 4153 tiles of 4096 positions, i.e. more than one super-group of
    # 64 x 64 tiles in the look-back (tiles), or 1385 segments of 3 tiles (segments, automatic
    # length); checked in full, and bitwise on a repeat
    import paper_2110_11866_amd as M
    _announce("long-row", mode, schedule)
    N, sigma, K, L = 17_000_000, 40.0, 4, 160
    x = np.random.default_rng(17).standard_normal(N).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    plan = M.MorletPlan(N, sigma, 6.0 / sigma, K, L, mode=mode).set_schedule(schedule)
    a = plan.forward(xt)
    b = plan.forward(xt)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    info = plan.info()
    p = O.plan_morlet(sigma, 6.0 / sigma, K, L, mode=mode, n0=info["n0"] if mode == "asft" else None)
    want = O.forward(x.astype(np.float64), p)
    assert rel_l2(a.cpu().numpy(), want) <= 1e-5, rel_l2(a.cpu().numpy(), want)


@pytest.mark.parametrize("schedule", ["tiles", "segments"])
@pytest.mark.parametrize("mode", ["sft", "asft"])
def test_max_single_row_sampled(mode, schedule):
    # one 2^30-sample row: 262144 tiles, 64 super-groups of the look-back (tiles), or 2048
    # segments of 128 tiles (segments, automatic length); outputs sampled at the ends, around
    # tile / group / super-group boundaries and at random, each checked against the oracle's
    # plain sum over its own window of the same (device-generated) input
    import paper_2110_11866_amd as M
    _announce("max-row", mode, schedule)
    N, sigma, K, L = 1 << 30, 64.0, 5, 0
    gen = torch.Generator(device="cuda").manual_seed(30)
    xt = torch.randn(N, generator=gen, device="cuda")
    plan = M.MorletPlan(N, sigma, 6.0 / sigma, K, L, mode=mode).set_schedule(schedule)
    W = plan.forward(xt)
    torch.cuda.synchronize()
    info = plan.info()
    L, n0 = info["L"], info["n0"]
    p = O.plan_morlet(sigma, 6.0 / sigma, K, L, mode=mode, n0=n0 if mode == "asft" else None, P_S=checked_ps(sigma, 6.0 / sigma, K, info))
    h, shift = (O.asft_kernel(p), n0) if mode == "asft" else (O.kterm_morlet(p), 0)
    T = 16 * 256
    ns = {0, 1, L, N - 1, N - 2, N - L - 1}
    # tile, group and super-group boundaries; segment boundaries (128 tiles) and the boundary
    # between two lanes' runs of 32 segments in the combination
    for j in (T, 64 * T, 4096 * T, 5 * 4096 * T, 63 * 4096 * T, 64 * 4096 * T - T, 128 * T, 32 * 128 * T,
              2047 * 128 * T):
        for d in (-1, 0, 1):
            ns.add(j + d - (L - n0))      # output at scan position j + d
    ns.update(int(v) for v in np.random.default_rng(31).integers(0, N, 40))
    ns = sorted(n for n in ns if 0 <= n < N)
    got = W[torch.tensor(ns, device="cuda")].cpu().numpy()
    want = np.zeros(len(ns), dtype=np.complex128)
    for i, n in enumerate(ns):
        a, b = max(0, n - shift - L), min(N, n - shift + L + 1)
        seg = xt[a:b].double().cpu().numpy()
        want[i] = O.conv_same_at(seg, h, L, np.array([n - a]), shift)[0]
    err = np.abs(got - want) / np.abs(want).max()
    print(f"[result] {mode}: {len(ns)} sampled outputs, max error {err.max():.2e} of the largest", flush=True)
    assert rel_l2(got, want) <= 1e-5, rel_l2(got, want)
    del W, xt
    torch.cuda.empty_cache()


@pytest.mark.parametrize("kind", ["morlet", "gauss", "gd1", "gd2"])
@pytest.mark.parametrize("mode", ["sft", "asft"])
@pytest.mark.parametrize("N,sigma,K,L,dtype,accum", [(3, 4.0, 3, 16, torch.float32, "f32"),
                                                     (37, 8.0, 4, 40, torch.float32, "f32"),
                                                     (5000, 30.0, 5, 0, torch.bfloat16, "f32"),
                                                     (50000, 300.0, 6, 1200, torch.float32, "f64")])
def test_edge_extension_parity(N, sigma, K, L, dtype, accum, mode, kind):
    # x extended by its edge values (Sec. II) instead of zeros (N >= 3: a 1-sample signal extends
    # to a constant, whose odd-kernel and zero-mean-kernel outputs are exactly zero)
    import paper_2110_11866_amd as M
    _announce("edge", kind, mode, N, sigma, K, L, dtype, accum)
    x = (np.random.default_rng(N + K).standard_normal(N) + 2.0).astype(np.float32)   # nonzero mean: edges matter
    xt = torch.from_numpy(x).cuda().to(dtype)
    if kind == "morlet":
        plan = M.MorletPlan(N, sigma, 6.0 / sigma, K, L, mode=mode, accum=accum)
    elif kind == "gauss":
        plan = M.GaussPlan(N, sigma, K, L, mode=mode, accum=accum)
    else:
        plan = M.GaussDerivPlan(N, sigma, K, L, order=1 if kind == "gd1" else 2, mode=mode, accum=accum)
    plan.set_boundary("edge")
    got = plan.forward(xt).cpu().numpy()
    torch.cuda.synchronize()
    info = plan.info()
    n0 = info["n0"] if mode == "asft" else None
    if kind == "morlet":
        p = O.plan_morlet(sigma, 6.0 / sigma, K, info["L"], mode=mode, n0=n0)
    elif kind == "gauss":
        p = O.plan_gauss(sigma, K, info["L"], mode=mode, n0=n0)
    else:
        p = O.plan_gauss_deriv(sigma, K, info["L"], 1 if kind == "gd1" else 2, mode=mode, n0=n0)
    want = O.forward_edge(xt.double().cpu().numpy(), p)
    assert rel_l2(got, want) <= TOL[accum], rel_l2(got, want)
