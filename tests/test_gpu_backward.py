"""Backward pass of the HIP path against the FP64 oracle: the adjoint (dLoss/dx), the
parameter gradients (dLoss/dsigma, dLoss/dxi with the plan frozen), the batched scalogram
backward and the autograd layer. Bars: relative L2 1e-5 for dLoss/dx (1e-6 in float64),
relative 1e-5 for the parameter gradients."""
import sys

import numpy as np
import pytest
import torch

import workloads
from oracle import morlet_oracle as O
from oracle_ps import checked_ps

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_11866_amd  # noqa: F401
    yield


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _announce(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _oracle_plan(kind, sigma, K, info, mode):
    if kind == "morlet":
        return O.plan_morlet(sigma, 6.0 / sigma, K, info["L"], mode=mode,
                             n0=info["n0"] if mode == "asft" else None, P_S=checked_ps(sigma, 6.0 / sigma, K, info))
    return O.plan_gauss(sigma, K, info["L"], mode=mode, n0=info["n0"] if mode == "asft" else None)


CASES = [(1024, 16.0, 4, 64, 16), (50000, 300.0, 6, 1200, 16), (9000, 40.0, 5, 0, 16), (70001, 300.0, 5, 1200, 32),
         (20000, 100.0, 5, 400, 8), (5000, 30.0, 4, 0, 4)]


@pytest.mark.parametrize("accum", ["f32", "f64"])
@pytest.mark.parametrize("mode", ["sft", "asft"])
@pytest.mark.parametrize("kind", ["morlet", "gauss"])
@pytest.mark.parametrize("N,sigma,K,L,tile", CASES)
def test_backward_matches_oracle(N, sigma, K, L, tile, kind, mode, accum):
    import paper_2110_11866_amd as M
    _announce("backward", N, sigma, K, L, tile, kind, mode, accum)
    rng = np.random.default_rng(N + K + len(mode))
    x = rng.standard_normal(N).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    if kind == "morlet":
        plan = M.MorletPlan(N, sigma, 6.0 / sigma, K, L, mode=mode, accum=accum)
        W = plan.forward(xt)
        w = torch.from_numpy(rng.uniform(size=N).astype(np.float32)).cuda()
        g = (2 * w * W).contiguous()             # cotangent of Loss = sum w |W|^2
    else:
        plan = M.GaussPlan(N, sigma, K, L, mode=mode, accum=accum)
        g = torch.from_numpy(rng.standard_normal(N).astype(np.float32)).cuda()
    plan.set_tile(tile)
    gx, gp = plan.backward(xt, g)
    torch.cuda.synchronize()
    info = plan.info()
    p = _oracle_plan(kind, sigma, K, info, mode)
    gn = g.cpu().numpy().astype(np.complex128 if kind == "morlet" else np.float64)
    want_gx = O.adjoint(gn, p)
    tol = 1e-6 if accum == "f64" else 1e-5
    assert rel(gx.cpu().numpy(), want_gx) <= tol, rel(gx.cpu().numpy(), want_gx)
    want_gp = O.param_grads(x.astype(np.float64), gn, p)
    got_gp = gp.cpu().numpy()
    if kind == "gauss":
        assert got_gp[1] == 0.0
        assert abs(got_gp[0] - want_gp[0]) <= 1e-5 * abs(want_gp[0]), (got_gp, want_gp)
    else:
        assert np.all(np.abs(got_gp - want_gp) <= 1e-5 * np.abs(want_gp)), (got_gp, want_gp)


def test_adjoint_identity_on_gpu():
    # Re <g, A x> = <x, A^T g> with both sides from the GPU kernels
    import paper_2110_11866_amd as M
    _announce("adjoint-identity")
    N = 70000
    rng = np.random.default_rng(3)
    x = torch.from_numpy(rng.standard_normal(N).astype(np.float32)).cuda()
    g = torch.from_numpy((rng.standard_normal(N) + 1j * rng.standard_normal(N)).astype(np.complex64)).cuda()
    for mode in ("sft", "asft"):
        plan = M.MorletPlan(N, 500.0, 6 / 500.0, 6, 2000, mode=mode)
        W = plan.forward(x).cpu().numpy().astype(np.complex128)
        gx, _ = plan.backward(None, g, want_params=False)
        lhs = np.sum((np.conj(g.cpu().numpy().astype(np.complex128)) * W).real)
        rhs = float(np.dot(x.cpu().numpy().astype(np.float64), gx.cpu().numpy().astype(np.float64)))
        assert abs(lhs - rhs) <= 2e-5 * (abs(lhs) + np.sqrt(N)), (mode, lhs, rhs)


def test_backward_repeat_bitwise():
    import paper_2110_11866_amd as M
    _announce("backward-repeat")
    N = 200000
    rng = np.random.default_rng(8)
    x = torch.from_numpy(rng.standard_normal(N).astype(np.float32)).cuda()
    g = torch.from_numpy((rng.standard_normal(N) + 1j * rng.standard_normal(N)).astype(np.complex64)).cuda()
    plan = M.MorletPlan(N, 100.0, 0.06, 5, 400, mode="asft")
    a = [plan.backward(x, g) for _ in range(3)]
    torch.cuda.synchronize()
    for gx, gp in a[1:]:
        assert torch.equal(gx, a[0][0]) and torch.equal(gp, a[0][1])


@pytest.mark.parametrize("schedule", ["tiles", "rows"])
@pytest.mark.parametrize("mode", ["sft", "asft"])
def test_scalogram_backward_small(mode, schedule):
    import paper_2110_11866_amd as M
    _announce("scalogram-backward", mode, schedule)
    lengths = [300, 5000, 1, 12000]
    sigmas = [4.0, 30.0, 200.0]
    xis = [6.0 / s for s in sigmas]
    rng = np.random.default_rng(5)
    x = rng.standard_normal(sum(lengths)).astype(np.float32)
    plan = M.ScalogramPlan(lengths, sigmas, xis, 5, 0.0, mode=mode).set_schedule(schedule)
    xt = torch.from_numpy(x).cuda()
    W = plan.forward(xt)
    g = torch.from_numpy((rng.standard_normal(W.numel()) + 1j * rng.standard_normal(W.numel()))
                         .astype(np.complex64)).cuda()
    gx, gp = plan.backward(xt, g)
    torch.cuda.synchronize()
    gn, gxn, gpn = g.cpu().numpy().astype(np.complex128), gx.cpu().numpy(), gp.cpu().numpy()
    offs = np.concatenate([[0], np.cumsum(lengths)])
    want_gx = np.zeros(sum(lengths))
    want_gp = np.zeros((len(sigmas), 2))
    for s in range(len(sigmas)):
        info = plan.scale_info(s)
        p = O.plan_morlet(sigmas[s], xis[s], 5, info["L"], mode=mode, n0=info["n0"] if mode == "asft" else None,
                          P_S=checked_ps(sigmas[s], xis[s], 5, info))
        for b in range(len(lengths)):
            n = lengths[b]
            o = plan.out_offset(b, s)
            gb = gn[o:o + n]
            want_gx[offs[b]:offs[b] + n] += O.adjoint(gb, p)
            if n:
                want_gp[s] += O.param_grads(x[offs[b]:offs[b] + n].astype(np.float64), gb, p)
    assert rel(gxn, want_gx) <= 1e-5, rel(gxn, want_gx)
    assert np.all(np.abs(gpn - want_gp) <= 1e-5 * np.abs(want_gp) + 1e-9), (gpn, want_gp)


@pytest.mark.parametrize("mode", ["sft", "asft"])
def test_autograd_layer_and_central_differences(mode):
    # Loss = sum w |W|^2: torch autograd through the layer against the oracle's gradients,
    # and the oracle's gradient against central differences at relative steps 1e-3 / 1e-4
    import paper_2110_11866_amd as M
    _announce("autograd", mode)
    N, sigma, xi, K = 4000, 25.0, 6 / 25.0, 5
    rng = np.random.default_rng(6)
    x = torch.from_numpy(rng.standard_normal(N).astype(np.float32)).cuda().requires_grad_(True)
    w = torch.from_numpy(rng.uniform(size=N).astype(np.float32)).cuda()
    layer = M.MorletTransform(N, sigma, xi, K, 0, mode=mode)
    W = layer(x)
    loss = (w * (W.real ** 2 + W.imag ** 2)).sum()
    loss.backward()
    torch.cuda.synchronize()
    p = layer.plan()
    info = p.info()
    op = O.plan_morlet(sigma, xi, K, info["L"], mode=mode, n0=info["n0"] if mode == "asft" else None,
                       P_S=checked_ps(sigma, xi, K, info))
    xd = x.detach().cpu().numpy().astype(np.float64)
    wd = w.cpu().numpy().astype(np.float64)
    Wo = O.forward(xd, op)
    go = 2 * wd * Wo
    want = O.param_grads(xd, go, op)
    # the backward at the cotangent autograd handed it (2 w W with the layer's own float32 W),
    # against the oracle's gradients at that same cotangent: float64 all the way to .grad
    assert layer.sigma.grad.dtype == torch.float64 and layer.xi.grad.dtype == torch.float64
    gl = 2 * wd * W.detach().cpu().numpy().astype(np.complex128)
    want_l = O.param_grads(xd, gl, op)
    assert abs(layer.sigma.grad.item() - want_l[0]) <= 1e-5 * abs(want_l[0]), (layer.sigma.grad.item(), want_l[0])
    assert abs(layer.xi.grad.item() - want_l[1]) <= 1e-5 * abs(want_l[1]), (layer.xi.grad.item(), want_l[1])
    assert rel(x.grad.cpu().numpy(), O.adjoint(gl, op)) <= 1e-5
    # and the whole chain (float32 forward included) against the oracle's own loss gradient
    assert abs(layer.sigma.grad.item() - want[0]) <= 1e-4 * abs(want[0]), (layer.sigma.grad.item(), want[0])
    assert abs(layer.xi.grad.item() - want[1]) <= 1e-4 * abs(want[1]), (layer.xi.grad.item(), want[1])

    def loss_o(s, xx):
        m, l = O.fit_morlet(s, xx, K, op.L, op.P_S)
        q = O.Plan("morlet", s, xx, K, op.L, op.P_S, mode, op.n0, m, l)
        return np.sum(wd * np.abs(O.forward(xd, q)) ** 2)

    for t, (base, grad) in enumerate(((sigma, want[0]), (xi, want[1]))):
        errs = []
        for h in (1e-3, 1e-4):
            a = (base * (1 + h), xi) if t == 0 else (sigma, base * (1 + h))
            b = (base * (1 - h), xi) if t == 0 else (sigma, base * (1 - h))
            fd = (loss_o(*a) - loss_o(*b)) / (2 * h * base)
            errs.append(abs(fd - grad) / abs(grad))
        assert errs[1] < 1e-4 and errs[1] < errs[0], errs


@pytest.mark.parametrize("mode", ["sft", "asft"])
def test_differentiation_workload_sampled(mode):
    # 64 signals x 32768 samples, 16 scales sigma = 8..2048, K = 5, Loss = sum w |W|^2 with
    # w ~ U[0,1] per (scale, n) shared over the batch; gradients for x (4 signals checked in
    # full) and for every (sigma_s, xi_s) (oracle summed over all 64 signals), from the tiles and
    # the rows schedule on the same cotangent
    import paper_2110_11866_amd as M
    _announce("differentiation-workload", mode)
    x, sigmas, xis, w = workloads.differentiation_batch()
    B, N = x.shape
    S = len(sigmas)
    plan = M.ScalogramPlan([N] * B, sigmas, xis, 5, 0.0, mode=mode)
    xt = torch.from_numpy(x.reshape(-1)).cuda()
    W = plan.forward(xt)
    wt = torch.from_numpy(np.tile(w.reshape(1, S, N), (B, 1, 1)).reshape(-1)).cuda()
    g = (2 * wt * W).contiguous()
    got = {}
    for schedule in ("tiles", "rows"):
        gx, gp = plan.set_schedule(schedule).backward(xt, g)
        torch.cuda.synchronize()
        got[schedule] = (gx.cpu().numpy().reshape(B, N), gp.cpu().numpy())
    gn = g.cpu().numpy().astype(np.complex128).reshape(B, S, N)
    plans = []
    for s in range(S):
        info = plan.scale_info(s)
        plans.append(O.plan_morlet(sigmas[s], xis[s], 5, info["L"], mode=mode,
                                   n0=info["n0"] if mode == "asft" else None,
                                   P_S=checked_ps(sigmas[s], xis[s], 5, info)))
    for b in (0, 17, 40, 63):
        want = sum(O.adjoint(gn[b, s], plans[s]) for s in range(S))
        for schedule, (gxn, _) in got.items():
            assert rel(gxn[b], want) <= 1e-5, (schedule, b, rel(gxn[b], want))
    want_gp = np.zeros((S, 2))
    for b in range(B):
        xb = x[b].astype(np.float64)
        for s in range(S):
            want_gp[s] += O.param_grads(xb, gn[b, s], plans[s])
    for schedule, (_, gpn) in got.items():
        assert np.all(np.abs(gpn - want_gp) <= 1e-5 * np.abs(want_gp)), (schedule, np.abs(gpn - want_gp) / np.abs(want_gp))


def _fold(gxe, N, P):
    # transpose of the edge extension x_ext[m] = x[clamp(m - P, 0, N - 1)]
    gx = gxe[P:P + N].copy()
    gx[0] += gxe[:P].sum()
    gx[N - 1] += gxe[P + N:].sum()
    return gx


@pytest.mark.parametrize("mode", ["sft", "asft"])
@pytest.mark.parametrize("kind", ["morlet", "gauss"])
@pytest.mark.parametrize("N,sigma,K,L", [(1, 6.0, 3, 20), (37, 8.0, 4, 40), (20000, 100.0, 5, 400)])
def test_backward_with_edge_extension(N, sigma, K, L, kind, mode):
    # the extension's transpose: adjoint of the padded row, folded onto the ends; parameter
    # gradients over the padded signal; and the adjoint identity with both sides on the GPU
    import paper_2110_11866_amd as M
    _announce("backward-edge", N, sigma, K, L, kind, mode)
    rng = np.random.default_rng(N + K)
    x = (rng.standard_normal(N) + 1.0).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    if kind == "morlet":
        plan = M.MorletPlan(N, sigma, 6.0 / sigma, K, L, mode=mode)
        g = (rng.standard_normal(N) + 1j * rng.standard_normal(N)).astype(np.complex64)
    else:
        plan = M.GaussPlan(N, sigma, K, L, mode=mode)
        g = rng.standard_normal(N).astype(np.float32)
    plan.set_boundary("edge")
    gt = torch.from_numpy(g).cuda()
    W = plan.forward(xt).cpu().numpy()
    gx, gp = plan.backward(xt, gt)
    torch.cuda.synchronize()
    info = plan.info()
    p = _oracle_plan(kind, sigma, K, info, mode)
    P = 2 * info["L"]
    gn = g.astype(np.complex128 if kind == "morlet" else np.float64)
    ge = np.concatenate([np.zeros(P, gn.dtype), gn, np.zeros(P, gn.dtype)])
    want_gx = _fold(O.adjoint(ge, p), N, P)
    assert rel(gx.cpu().numpy(), want_gx) <= 1e-5, rel(gx.cpu().numpy(), want_gx)
    xe = np.pad(x.astype(np.float64), (P, P), mode="edge")
    want_gp = O.param_grads(xe, ge, p)
    got_gp = gp.cpu().numpy()
    idx = [0] if kind == "gauss" else [0, 1]
    assert np.all(np.abs(got_gp[idx] - want_gp[idx]) <= 1e-5 * np.abs(want_gp[idx])), (got_gp, want_gp)
    lhs = float(np.sum((np.conj(gn) * W.astype(np.complex128)).real))
    rhs = float(np.dot(x.astype(np.float64), gx.cpu().numpy().astype(np.float64)))
    assert abs(lhs - rhs) <= 2e-5 * (abs(lhs) + np.sqrt(N)), (lhs, rhs)


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("N,sigma,K,L,mode,n0,tile,accum", [
    (3, 4.0, 4, 16, "sft", None, 16, "f32"),                 # N = 1 of order 1 is exactly 0
    (200, 66.0, 5, 256, "asft", 10, 16, "f32"),              # N < L
    (1024, 16.0, 4, 64, "sft", None, 16, "f32"),
    (50000, 300.0, 6, 1200, "asft", 0, 16, "f32"),
    (50000, 300.0, 6, 1200, "sft", None, 32, "f64"),
    (30001, 100.0, 5, 0, "asft", 0, 8, "f32"),
    (3000, 12.0, 3, 0, "sft", None, 4, "f32"),
])
def test_differential_backward(N, sigma, K, L, mode, n0, tile, accum, order):
    # dLoss/dx of x_GD / x_GDD: the oracle's adjoint of the differential taps, and the adjoint
    # identity <g, A x> = <A^T g, x> with both sides from the GPU
    import paper_2110_11866_amd as M
    _announce("deriv-backward", order, N, sigma, K, L, mode, n0, tile, accum)
    rng = np.random.default_rng(N + 7 * order)
    x = rng.standard_normal(N).astype(np.float32)
    g = rng.standard_normal(N).astype(np.float32)
    xt, gt = torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda()
    kw = dict(order=order, accum=accum, mode=mode)
    if mode == "asft":
        kw["n0"] = n0
    plan = M.GaussDerivPlan(N, sigma, K, L, **kw)
    plan.set_tile(tile)
    y = plan.forward(xt).cpu().numpy()
    gx, gp = plan.backward(None, gt)
    gx = gx.cpu().numpy()
    torch.cuda.synchronize()
    assert gp is None
    info = plan.info()
    p = O.plan_gauss_deriv(sigma, K, info["L"], order, mode=mode, n0=info["n0"] if mode == "asft" else None)
    want = O.adjoint(g.astype(np.float64), p)
    assert rel(gx, want) <= (1e-6 if accum == "f64" else 1e-5), rel(gx, want)
    lhs = float(np.dot(g.astype(np.float64), y.astype(np.float64)))
    rhs = float(np.dot(x.astype(np.float64), gx.astype(np.float64)))
    assert abs(lhs - rhs) <= 2e-5 * (np.linalg.norm(g) * np.linalg.norm(y) + 1e-30), (lhs, rhs)
    with pytest.raises(NotImplementedError):
        plan.backward(None, gt, want_params=True)


@pytest.mark.parametrize("mode", ["sft", "asft"])
@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("N,sigma,K,L", [(5, 6.0, 3, 20), (37, 8.0, 4, 40), (20000, 100.0, 5, 400)])
def test_differential_backward_with_edge_extension(N, sigma, K, L, order, mode):
    # E^T (R A_e R) C^T: the oracle's adjoint of the padded row folded onto the ends, and the
    # adjoint identity against the edge-extended forward on the GPU
    import paper_2110_11866_amd as M
    _announce("deriv-backward-edge", order, N, sigma, K, L, mode)
    rng = np.random.default_rng(N + 11 * order)
    x = (rng.standard_normal(N) + 1.0).astype(np.float32)
    g = rng.standard_normal(N).astype(np.float32)
    xt, gt = torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda()
    plan = M.GaussDerivPlan(N, sigma, K, L, order=order, mode=mode).set_boundary("edge")
    y = plan.forward(xt).cpu().numpy()
    gx, gp = plan.backward(None, gt)
    gx = gx.cpu().numpy()
    torch.cuda.synchronize()
    assert gp is None
    info = plan.info()
    p = O.plan_gauss_deriv(sigma, K, info["L"], order, mode=mode, n0=info["n0"] if mode == "asft" else None)
    P = 2 * info["L"]
    ge = np.concatenate([np.zeros(P), g.astype(np.float64), np.zeros(P)])
    want = _fold(O.adjoint(ge, p), N, P)
    assert rel(gx, want) <= 1e-5, rel(gx, want)
    lhs = float(np.dot(g.astype(np.float64), y.astype(np.float64)))
    rhs = float(np.dot(x.astype(np.float64), gx.astype(np.float64)))
    assert abs(lhs - rhs) <= 2e-5 * (np.linalg.norm(g) * np.linalg.norm(y) + np.sqrt(N)), (lhs, rhs)


@pytest.mark.parametrize("mode", ["sft", "asft"])
def test_layer_refits_into_its_table(mode):
    # an optimizer step moves sigma and xi; the layer refits its plan's coefficients into the
    # same device table (window, lowest order and shift frozen): the forward then equals, bit
    # for bit, a fresh plan built at the new parameters with the same window, order and shift,
    # and the oracle at those frozen settings
    import paper_2110_11866_amd as M
    _announce("layer-refit", mode)
    N, sigma, xi, K = 6000, 30.0, 6 / 30.0, 5
    rng = np.random.default_rng(8)
    x = torch.from_numpy(rng.standard_normal(N).astype(np.float32)).cuda()
    layer = M.MorletTransform(N, sigma, xi, K, 0, mode=mode)
    info0 = layer.plan().info()
    handle = layer.plan().handle
    with torch.no_grad():
        layer.sigma.mul_(1.03)
        layer.xi.mul_(0.98)
    W1 = layer(x)
    torch.cuda.synchronize()
    assert layer.plan().handle == handle
    s1, x1 = float(layer.sigma), float(layer.xi)
    info1 = layer.plan().info()
    assert (info1["L"], info1["P_S"], info1["n0"]) == (info0["L"], info0["P_S"], info0["n0"])
    fresh = M.MorletPlan(N, s1, x1, K, info0["L"])
    if mode == "asft":
        fresh.set("asft", info0["n0"])
    assert fresh.info()["P_S"] == info0["P_S"]
    W2 = fresh.forward(x)
    torch.cuda.synchronize()
    assert torch.equal(W1.view(torch.float32), W2.view(torch.float32))
    op = O.plan_morlet(s1, x1, K, info0["L"], mode=mode, n0=info0["n0"] if mode == "asft" else None,
                       P_S=info0["P_S"])
    assert rel(W1.detach().cpu().numpy(), O.forward(x.double().cpu().numpy(), op)) <= 1e-5
