"""Long GPU runs against the oracle.

* The 2D Euler workload (seeded four-quadrant Riemann data, transmissive,
  CFL 0.5) at its full length of 200 RK3 steps on a 512 x 512 grid, every
  cell against the oracle's 200 steps.
* The 2D Riemann configuration 3 at 400 x 400 to T = 0.8 with CFL 0.45, the
  setting of the CPU timing table of Section 4.4: the GPU must take exactly
  the oracle's number of steps (stored by tests/golden/gen_config3_steps.py,
  which runs the oracle only; the CPU suite ties that number to the paper's
  3497).
"""
import json
import os

import numpy as np
import pytest

import oracle as orc
from paper_2603_26272_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2603_26272_amd import za
    za.lib()
    return torch.device("cuda:0")


def Ctx(P):
    from paper_2603_26272_amd.za import Context
    return Context(P)


def rel_err(got, ref):
    scale = np.abs(ref) + np.abs(ref).max(axis=(1, 2), keepdims=True)
    return float((np.abs(got - ref) / scale).max())


def test_c2_full_length_512(dev):
    """200 steps of the 2048^2 workload's generator at 512^2: every cell
    within 1e-10 of the oracle (relative to the value plus the component's
    largest magnitude)."""
    P, q0 = W.quadrants_2d(0, 512)
    q = torch.from_numpy(q0).to(dev)
    with Ctx(P) as ctx:
        info = ctx.solve(q, 0.0, 200)
    orc.set_threads(16)
    ref, steps, t, st = orc.solve(P, q0, 0.0, 200)
    assert st == 0 and steps == 200 and info["steps"] == 200
    assert abs(info["t"] - t) <= 1e-13 * t
    drift = rel_err(q.cpu().numpy(), ref)
    print(f"c2 512^2 200 steps: max relative difference to the oracle {drift:.3e}, t = {t!r}", flush=True)
    assert drift <= 1e-10, drift


def test_config3_400_step_count_equals_oracle(dev):
    with open(os.path.join(HERE, "golden", "config3_400_oracle.json")) as fh:
        gold = json.load(fh)
    P, q0, T = W.riemann_config3(400)
    q = torch.from_numpy(q0).to(dev)
    with Ctx(P) as ctx:
        info = ctx.solve(q, T)
    print(f"config 3, 400^2, T = {T}: GPU {info['steps']} steps, oracle {gold['steps']}, paper {gold['paper_steps']}",
          flush=True)
    assert info["t"] == T
    assert info["steps"] == gold["steps"]
    rho = q[0].cpu().numpy()
    assert rho.min() > 0.0
    assert abs(rho.min() - gold["rho_min"]) <= 1e-3 * gold["rho_min"]
    assert abs(rho.max() - gold["rho_max"]) <= 1e-3 * gold["rho_max"]
