"""GPU parity of the separable 2-D Gabor filter (Morlet rows, then Gaussian columns of the real
and imaginary parts) against the FP64 oracle."""
import sys

import numpy as np
import pytest
import torch

from oracle import morlet_oracle as O
from oracle_ps import checked_ps

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f64": 1e-6, "mixed": 1e-5}


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def _announce(*args):
    print("[case]", *args, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def _oracle_plans(plan, W, mode):
    import paper_2110_11866_amd as M
    ix, iy = plan.axis_info(0), plan.axis_info(1)
    # the row pass's order offset P_S, from a 1-D plan of the same row parameters
    P_S = checked_ps(plan.sigma_x, plan.xi, plan.K_x, M.MorletPlan(W, plan.sigma_x, plan.xi, plan.K_x, ix["L"]).info())
    px = O.plan_morlet(plan.sigma_x, plan.xi, plan.K_x, ix["L"], mode=mode,
                       n0=ix["n0"] if mode == "asft" else None, P_S=P_S)
    py = O.plan_gauss(plan.sigma_y, plan.K_y, iy["L"], mode=mode, n0=iy["n0"] if mode == "asft" else None)
    assert np.allclose(ix["cos_coef"], px.cos_coef, rtol=1e-9, atol=1e-12)
    return px, py


@pytest.mark.parametrize("H,W,sx,xi0,Kx,sy,Ky,mode,accum,dtype,tile", [
    (1, 1, 2.0, 6.0, 3, 2.0, 3, "sft", "f32", torch.float32, 16),
    (5, 300, 10.0, 6.0, 5, 3.0, 4, "sft", "f32", torch.float32, 16),
    (257, 513, 5.0, 6.0, 5, 8.0, 4, "asft", "f32", torch.float32, 16),
    (300, 200, 6.0, 4.0, 4, 4.0, 4, "sft", "f32", torch.float16, 8),
    (200, 333, 6.0, 6.0, 5, 6.0, 4, "asft", "f32", torch.bfloat16, 4),
    (640, 480, 16.0, 6.0, 6, 16.0, 6, "asft", "f64", torch.float32, 32),
    (64, 4096, 2.0, 6.0, 4, 100.0, 4, "sft", "f32", torch.float32, 16),
    (1000, 70, 3.0, 5.0, 5, 2.5, 3, "asft", "f32", torch.float32, 16),
])
def test_gabor_parity(H, W, sx, xi0, Kx, sy, Ky, mode, accum, dtype, tile):
    import paper_2110_11866_amd as M
    _announce("gabor", H, W, sx, xi0, Kx, sy, Ky, mode, accum, dtype, tile)
    img = np.random.default_rng(H * 5 + W).standard_normal((H, W)).astype(np.float32)
    xt = torch.from_numpy(img).cuda().to(dtype)
    plan = M.Gabor2DPlan(H, W, sx, xi0 / sx, Kx, sy, Ky, mode=mode, accum=accum)
    plan.set_tile(tile)
    got = plan.forward(xt).cpu().numpy()
    torch.cuda.synchronize()
    px, py = _oracle_plans(plan, W, mode)
    want = O.gabor_2d(xt.double().cpu().numpy(), px, py)
    assert got.shape == (H, W) and got.dtype == np.complex64
    assert rel_l2(got, want) <= TOL[accum], rel_l2(got, want)


def test_gabor_empty_and_repeat():
    # empty images launch nothing; a repeated call (schedules, tiles changed in between) is
    # bitwise identical to the first for the same settings
    import paper_2110_11866_amd as M
    _announce("gabor-empty-repeat")
    for H, W in ((0, 10), (10, 0)):
        out = M.Gabor2DPlan(H, W, 4.0, 1.5, 4, 3.0, 4).forward(torch.zeros(H, W, device="cuda"))
        assert out.shape == (H, W)
    H, W = 300, 700
    xt = torch.from_numpy(np.random.default_rng(1).standard_normal((H, W)).astype(np.float32)).cuda()
    plan = M.Gabor2DPlan(H, W, 8.0, 0.75, 5, 5.0, 4, mode="asft")
    a = plan.forward(xt).clone()
    plan.set_schedule("tiles")
    b = plan.forward(xt).clone()
    plan.set_schedule("auto").set_tile(8)
    plan.set_tile(16)
    c = plan.forward(xt).clone()
    torch.cuda.synchronize()
    assert torch.equal(a, c)
    assert rel_l2(b.cpu().numpy(), a.cpu().numpy()) <= 1e-6


@pytest.mark.parametrize("H,W,sx,xi0,Kx,sy,Ky,mode,tile", [
    (1, 1, 2.0, 6.0, 3, 2.0, 3, "sft", 16),
    (37, 300, 10.0, 6.0, 5, 3.0, 4, "asft", 16),
    (257, 129, 5.0, 6.0, 5, 8.0, 4, "sft", 8),
    (300, 200, 6.0, 4.0, 4, 4.0, 4, "asft", 32),
])
def test_gabor_backward(H, W, sx, xi0, Kx, sy, Ky, mode, tile):
    # dLoss/dx against the oracle's adjoint, and the adjoint identity with both sides on the GPU
    import paper_2110_11866_amd as M
    _announce("gabor-backward", H, W, sx, xi0, Kx, sy, Ky, mode, tile)
    rng = np.random.default_rng(H + 3 * W)
    img = rng.standard_normal((H, W)).astype(np.float32)
    g = (rng.standard_normal((H, W)) + 1j * rng.standard_normal((H, W))).astype(np.complex64)
    xt, gt = torch.from_numpy(img).cuda(), torch.from_numpy(g).cuda()
    plan = M.Gabor2DPlan(H, W, sx, xi0 / sx, Kx, sy, Ky, mode=mode)
    plan.set_tile(tile)
    y = plan.forward(xt).cpu().numpy()
    gx = plan.backward(gt).cpu().numpy()
    torch.cuda.synchronize()
    px, py = _oracle_plans(plan, W, mode)
    want = O.gabor_2d_adjoint(g.astype(np.complex128), px, py)
    assert gx.shape == (H, W)
    assert rel_l2(gx, want) <= 1e-5, rel_l2(gx, want)
    lhs = float(np.sum((np.conj(g.astype(np.complex128)) * y.astype(np.complex128)).real))
    rhs = float(np.sum(img.astype(np.float64) * gx.astype(np.float64)))
    assert abs(lhs - rhs) <= 2e-5 * (np.linalg.norm(g) * np.linalg.norm(y) + 1.0), (lhs, rhs)


@pytest.mark.parametrize("H,W,sx,xi0,Kx,sy,Ky,mode", [
    (1, 1, 2.0, 6.0, 3, 2.0, 3, "sft"),
    (37, 300, 10.0, 6.0, 5, 3.0, 4, "asft"),
    (257, 129, 5.0, 6.0, 5, 8.0, 4, "sft"),
    (300, 200, 6.0, 4.0, 4, 4.0, 4, "asft"),
])
def test_gabor_parameter_gradients(H, W, sx, xi0, Kx, sy, Ky, mode):
    # dsigma_y: the column lines of both parts of the row transform against the cotangent's;
    # dsigma_x, dxi: the rows of x against the rows' complex cotangent; each a sum over lines of
    # the oracle's frozen-plan gradient. gx as the plain backward, bitwise
    import paper_2110_11866_amd as M
    _announce("gabor-grad", H, W, sx, xi0, Kx, sy, Ky, mode)
    rng = np.random.default_rng(7 * H + W)
    img = rng.standard_normal((H, W)).astype(np.float32)
    g = (rng.standard_normal((H, W)) + 1j * rng.standard_normal((H, W))).astype(np.complex64)
    xt, gt = torch.from_numpy(img).cuda(), torch.from_numpy(g).cuda()
    plan = M.Gabor2DPlan(H, W, sx, xi0 / sx, Kx, sy, Ky, mode=mode)
    gx, gp = plan.grad(xt, gt)
    gx0 = plan.backward(gt)
    gx, gp, gx0 = gx.cpu().numpy(), gp.cpu().numpy(), gx0.cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(gx, gx0)
    px, py = _oracle_plans(plan, W, mode)
    x64, g64 = img.astype(np.float64), g.astype(np.complex128)
    y1 = np.stack([O.forward(x64[r], px) for r in range(H)])
    want_y = sum(O.param_grads(y1[:, c].real, g64[:, c].real, py)[0] + O.param_grads(y1[:, c].imag, g64[:, c].imag, py)[0]
                 for c in range(W))
    g1 = np.stack([O.adjoint(g64[:, c].real, py) + 1j * O.adjoint(g64[:, c].imag, py) for c in range(W)], axis=1)
    want_x = sum(O.param_grads(x64[r], g1[r], px) for r in range(H))
    want = np.array([want_y, want_x[0], want_x[1]])
    assert np.all(np.abs(gp - want) <= 1e-5 * np.abs(want) + 1e-9), (gp, want)


@pytest.mark.parametrize("mode", ["sft", "asft"])
def test_gabor_4096_benchmark_workload(mode):
    # the benchmark's 4096 x 4096 Gabor filter (Morlet rows sigma = 8, xi = 6/8, K = 5; Gaussian
    # columns sigma = 8, K = 4; error-optimal windows): every pixel against the oracle (its lines
    # spread over the host's cores), plus the first and last rows and columns on their own
    import paper_2110_11866_amd as M
    from oracle_pool import mapper, pool
    _announce("gabor-4096", mode)
    H = W = 4096
    x = torch.randn(H, W, generator=torch.Generator().manual_seed(19)).cuda()
    plan = M.Gabor2DPlan(H, W, 8.0, 6.0 / 8.0, 5, 8.0, 4, mode=mode)
    got = plan.forward(x).cpu().numpy()
    torch.cuda.synchronize()
    px, py = _oracle_plans(plan, W, mode)
    with pool() as ex:
        want = O.gabor_2d(x.double().cpu().numpy(), px, py, map_lines=mapper(ex))
    assert rel_l2(got, want) <= 1e-5, rel_l2(got, want)
    ix, iy = plan.axis_info(0), plan.axis_info(1)
    ey, ex_ = iy["L"] + iy["n0"], ix["L"] + ix["n0"]
    for sl in (np.s_[:ey, :], np.s_[-ey:, :], np.s_[:, :ex_], np.s_[:, -ex_:]):
        assert rel_l2(got[sl], want[sl]) <= 1e-5, (sl, rel_l2(got[sl], want[sl]))
