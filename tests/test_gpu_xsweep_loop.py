"""GPU: the looped x-sweep of the stages (row segments of 64 nc - 1 cells
walked in chunks of 64 interfaces, records carried in an LDS ring; in 2D the
partial stage, in 1D the whole stage and the wave-speed maxima of the new
state, one row per wavefront) against the one-shot sweep and the oracle,
through the C ABI.  ZA_XL_CHUNKS forces the chunk count (0: one-shot sweep).
Both sweeps evaluate every interface flux and cell update with the same
arithmetic and take exact maxima, so their states (and CFL time steps) agree
bitwise; segment boundaries, the flux carry between chunks, ragged row ends
and both boundary conditions are covered by the shapes below."""
import numpy as np
import pytest

import oracle as orc
from paper_2603_26272_amd import workloads as W
from paper_2603_26272_amd.problem import ADVECTION, PERIODIC, TRANSMISSIVE, Problem

from tests.test_gpu_parity import assert_close

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


def _steps(P, q0, n, dev, monkeypatch, chunks):
    from paper_2603_26272_amd.za import Context
    if chunks is None:
        monkeypatch.delenv("ZA_XL_CHUNKS", raising=False)
    else:
        monkeypatch.setenv("ZA_XL_CHUNKS", str(chunks))
    q = torch.from_numpy(np.ascontiguousarray(q0)).to(dev)
    with Context(P) as ctx:
        info = ctx.solve(q, 0.0, n)
    monkeypatch.delenv("ZA_XL_CHUNKS", raising=False)
    assert info["steps"] == n
    return q.cpu().numpy(), info["t"]


@pytest.mark.parametrize("nx,ny", [(1, 3), (5, 4), (63, 5), (64, 5), (65, 3), (127, 4), (128, 4), (300, 6),
                                   (703, 3), (1500, 2)])
def test_looped_equals_one_shot(dev, monkeypatch, nx, ny):
    for bcx in (TRANSMISSIVE, PERIODIC):
        P, q0 = W.quadrants_2d(nx + 7 * ny, nx, ny)
        P = P.with_(bc_x=bcx, bc_y=PERIODIC)
        ref = _steps(P, q0, 3, dev, monkeypatch, 0)
        for nc in (1, 2, 3, 5, 11):
            got = _steps(P, q0, 3, dev, monkeypatch, nc)
            assert np.array_equal(got[0], ref[0]) and got[1] == ref[1], (nx, ny, bcx, nc)


def test_looped_advection_equals_one_shot(dev, monkeypatch):
    nx, ny = 700, 5
    x = W.centres(nx, 0.0, 1.0)
    y = W.centres(ny, 0.0, 1.0)
    q0 = (np.sin(2 * np.pi * x)[None, :] + 0.3 * np.cos(2 * np.pi * y)[:, None] + (x > 0.6)[None, :]).reshape(1, ny, nx)
    P = Problem(dim=2, system=ADVECTION, nx=nx, ny=ny, bc_x=PERIODIC, bc_y=PERIODIC, adv_speed=(1.0, 0.5))
    ref = _steps(P, q0, 4, dev, monkeypatch, 0)[0]
    for nc in (1, 3, 11):
        assert np.array_equal(_steps(P, q0, 4, dev, monkeypatch, nc)[0], ref), nc


def test_looped_against_oracle(dev, monkeypatch):
    P, q0 = W.quadrants_2d(5, 400, 24)
    got = _steps(P, q0, 5, dev, monkeypatch, 3)[0]
    orc.set_threads(16)
    ref, steps, t, st = orc.solve(P, q0, 0.0, 5)
    assert st == 0 and steps == 5
    assert_close(got, ref, 1e-10, "looped x-sweep, 5 steps")


def test_default_choice_at_full_size(dev, monkeypatch):
    """The chunk count the library picks for the 2048^2 workload gives the
    one-shot sweep's states bitwise."""
    P, q0 = W.quadrants_2d(0, 2048)
    a = _steps(P, q0, 2, dev, monkeypatch, None)[0]
    b = _steps(P, q0, 2, dev, monkeypatch, 0)[0]
    assert np.array_equal(a, b)


# ---- 1D stages: the sweep also leaves the wave speeds of the new state ----

@pytest.mark.parametrize("nx", [1, 2, 5, 63, 64, 65, 127, 128, 191, 300, 4096, 70001])
def test_looped_1d_euler_equals_one_shot(dev, monkeypatch, nx):
    """Riemann data, 6 CFL steps: the step sizes come from the maxima the
    looped sweep leaves per wavefront, so equal times check those too."""
    for bcx in (TRANSMISSIVE, PERIODIC):
        P, q0 = W.riemann_1d(nx % 97, nx)
        P = P.with_(bc_x=bcx)
        ref = _steps(P, q0, 6, dev, monkeypatch, 0)
        for nc in (1, 2, 3, 5, 11):
            got = _steps(P, q0, 6, dev, monkeypatch, nc)
            assert np.array_equal(got[0], ref[0]) and got[1] == ref[1], (nx, bcx, nc)


@pytest.mark.parametrize("name", ["advection", "burgers", "buckley"])
def test_looped_1d_scalar_equals_one_shot(dev, monkeypatch, name):
    P, q0 = {"advection": W.multiwave(700), "burgers": W.burgers_sine(700), "buckley": W.buckley_step(700)}[name]
    ref = _steps(P, q0, 8, dev, monkeypatch, 0)
    for nc in (1, 2, 3, 11):
        got = _steps(P, q0, 8, dev, monkeypatch, nc)
        assert np.array_equal(got[0], ref[0]) and got[1] == ref[1], (name, nc)


def test_looped_1d_against_oracle(dev, monkeypatch):
    P, q0 = W.riemann_1d(11, 1000)
    got = _steps(P, q0, 40, dev, monkeypatch, 3)[0]
    ref, steps, t, st = orc.solve(P, q0, 0.0, 40)
    assert st == 0 and steps == 40
    assert_close(got, ref, 1e-10, "looped 1D x-sweep, 40 steps")


def test_default_choice_1d_large(dev, monkeypatch):
    """The chunk count the library picks for a long 1D line (2^20 + 3 cells)
    gives the one-shot sweep's states and step sizes bitwise."""
    P, q0 = W.riemann_1d(2, (1 << 20) + 3)
    a = _steps(P, q0, 2, dev, monkeypatch, None)
    b = _steps(P, q0, 2, dev, monkeypatch, 0)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]
