"""GPU parity at the largest sizes these tests exercise: the 2D Euler
quadrants at 4096^2 (four times the benchmark grid; sampled fluxes and one
full RK3 step in the stage kernels' launch configuration) and a 1D Euler
line of 2^20 + 3 cells (every flux), against the oracle."""
import numpy as np
import pytest

import oracle as orc
from paper_2603_26272_amd import workloads as W

from tests.test_gpu_parity import Ctx, assert_close, gpu_fluxes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2603_26272_amd import za
    za.lib()
    return torch.device("cuda:0")


def test_fluxes_4096_sampled(dev):
    P, q0 = W.quadrants_2d(1, 4096)
    fx, fy = gpu_fluxes(P, q0, dev)
    rng = np.random.default_rng(1)
    lines = sorted(set([0, 1, 2047, 2048, 4094, 4095] + list(rng.integers(0, 4096, 10))))
    rx, st = orc.fluxes_lines(P, q0, 0, lines)
    assert st == 0
    for j, l in enumerate(lines):
        assert_close(fx[:, l, :], rx[j], 1e-12, f"row {l}")
    ry, st = orc.fluxes_lines(P, q0, 1, lines)
    for j, l in enumerate(lines):
        assert_close(fy[:, :, l], ry[j], 1e-12, f"col {l}")


def test_one_step_4096(dev):
    """One RK3 step at 4096^2 through the looped x-sweep and the banded
    y-sweep (their launch shapes at this size differ from 2048^2), every cell
    against the oracle."""
    P, q0 = W.quadrants_2d(1, 4096)
    q = torch.from_numpy(q0).to(dev)
    with Ctx(P) as ctx:
        info = ctx.solve(q, 0.0, 1)
    orc.set_threads(16)
    ref, steps, t, st = orc.solve(P, q0, 0.0, 1)
    assert st == 0 and steps == 1 and info["steps"] == 1
    assert_close(q.cpu().numpy(), ref, 1e-10, "4096^2, one step")


def test_fluxes_1d_two_to_the_twenty(dev):
    N = (1 << 20) + 3
    P, q0 = W.riemann_1d(2, N)
    fx, _ = gpu_fluxes(P, q0, dev)
    ref, _, st = orc.fluxes(P, q0)
    assert st == 0
    assert_close(fx, ref, 1e-12, f"1D N={N}")
