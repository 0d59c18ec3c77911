"""GPU parity of the weight families of tab:SpecialCases (the L and q of
eq:weights_unnormalized; JS: L = 0, p = 2; Ai-JS and Ai-Z with the
descaler of eq:aimu) against the oracle, through the C ABI: interface
fluxes at the flux bar (FP64: 1e-12 of the component scale; FP32
reconstruction: 3e-5, as for the default weights), a short 2D solve at the
state bar, the even orders, and argument checks."""
import numpy as np
import pytest

import oracle as orc
from paper_2603_26272_amd import workloads as W
from paper_2603_26272_amd.problem import Problem

from tests.test_gpu_parity import assert_close, gpu_fluxes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FAMILIES = {
    "JS": dict(weight_L=0.0, p=2.0),
    "Ai-JS": dict(weight_L=0.0, p=2.0, affine_invariant=1, mu0=1e-40),
    "Ai-Z p=2": dict(p=2.0, affine_invariant=1, mu0=1e-40),
    "L=0.5 q=1.5": dict(weight_L=0.5, weight_q=1.5),
    "L=0 q=2": dict(weight_L=0.0, weight_q=2.0),
}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2603_26272_amd import za
    za.lib()
    return torch.device("cuda:0")


@pytest.mark.parametrize("name", list(FAMILIES))
def test_fluxes_2d(dev, name):
    P, q0 = W.quadrants_2d(13, 96, 80)
    P = P.with_(**FAMILIES[name])
    fx, fy = gpu_fluxes(P, q0, dev)
    rx, ry, st = orc.fluxes(P, q0)
    assert st == 0
    assert_close(fx, rx, 1e-12, f"{name} x")
    assert_close(fy, ry, 1e-12, f"{name} y")


@pytest.mark.parametrize("name", list(FAMILIES))
def test_fluxes_1d(dev, name):
    for N in (7, 65, 300):
        P, q0 = W.riemann_1d(N % 5, max(N, 8))
        q0 = np.ascontiguousarray(q0[:, :, :N])
        P = P.with_(nx=N, **FAMILIES[name])
        fx, _ = gpu_fluxes(P, q0, dev)
        ref, _, st = orc.fluxes(P, q0)
        assert st == 0
        assert_close(fx, ref, 1e-12, f"{name} N={N}")


@pytest.mark.parametrize("r", [2, 4, 5])
def test_fluxes_even_orders_js(dev, r):
    P, q0 = W.quadrants_2d(r, 70, 66)
    # a 1e-3 density ripple rules out exactly tied indicators (r = 2)
    x = np.arange(70)[None, :] + 0.37 * np.arange(66)[:, None]
    q0 = q0.copy()
    q0[0] *= 1 + 1e-3 * np.sin(x)
    P = P.with_(order=r, weight_L=0.0, p=2.0)
    fx, fy = gpu_fluxes(P, q0, dev)
    rx, ry, st = orc.fluxes(P, q0)
    assert st == 0
    assert_close(fx, rx, 1e-12, f"r={r} x")
    assert_close(fy, ry, 1e-12, f"r={r} y")


def test_fp32_js(dev):
    P, q0 = W.quadrants_2d(3, 96, 90)
    P = P.fp32().with_(weight_L=0.0, p=2.0)
    fx, fy = gpu_fluxes(P, q0, dev)
    rx, ry, st = orc.fluxes(P, q0)
    assert_close(fx, rx, 3e-5, "fp32 JS fx")
    assert_close(fy, ry, 3e-5, "fp32 JS fy")


def test_solve_2d_js(dev):
    from paper_2603_26272_amd.za import Context
    P, q0 = W.quadrants_2d(2, 128, 112)
    P = P.with_(weight_L=0.0, p=2.0)
    q = torch.from_numpy(q0).to(dev)
    with Context(P) as ctx:
        info = ctx.solve(q, 0.0, 10)
    orc.set_threads(16)
    ref, steps, t, st = orc.solve(P, q0, 0.0, 10)
    assert st == 0 and steps == 10 and info["steps"] == 10
    assert_close(q.cpu().numpy(), ref, 1e-10, "JS 2D solve")


def test_arguments(dev):
    from paper_2603_26272_amd import za
    for kw in (dict(weight_q=0.5), dict(weight_L=-1.0), dict(weight_L=float("nan")), dict(weight_L=1.0, weight_q=0.0)):
        with pytest.raises(za.ZaError) as ei:
            za.Context(Problem(dim=1, nx=32, **kw))
        assert ei.value.status == za.ZA_ERR_ARG, kw
    with za.Context(Problem(dim=1, nx=32, weight_L=0.0, weight_q=0.0)):   # both 0: the paper's 1, 1
        pass
    P, q0 = W.riemann_1d(0, 64)
    with za.Server(1 << 26, 2) as sv:
        with pytest.raises(za.ZaError) as ei:
            sv.submit(P.with_(weight_L=0.0, p=2.0), q0, 5)
        assert ei.value.status == za.ZA_ERR_UNSUPPORTED
