"""GPU parity at the largest sizes these tests exercise: the 2D Euler
quadrants at 4096^2 (four times the benchmark grid; sampled fluxes and one
full RK3 step in the stage kernels' launch configuration) and a 1D Euler
line of 2^20 + 3 cells (every flux), against the oracle; and a 33000^2 grid
(half the library's 2^31-cell limit, past 32-bit offsets) that tiles a
periodic 3000^2 one and a 1D line of 1.09998e9 cells that tiles a periodic
line of 999983, bitwise against the small grids' results."""
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


def _tiles_equal(big, small, k, nt):
    """big [m][k nt (+1)][k nt (+1)] against small [m][nt (+1)][nt (+1)]
    repeated k x k times, bit for bit (the extra interface row or column of a
    flux array compared with the small grid's own)."""
    ey, ex = big.shape[1] - k * nt, big.shape[2] - k * nt
    for i in range(k):
        for j in range(k):
            if not torch.equal(big[:, i * nt:(i + 1) * nt, j * nt:(j + 1) * nt], small[:, :nt, :nt]):
                return f"tile ({i}, {j})"
        if ex and not torch.equal(big[:, i * nt:(i + 1) * nt, k * nt], small[:, :nt, nt]):
            return f"last column of tile row {i}"
    for j in range(k):
        if ey and not torch.equal(big[:, k * nt, j * nt:(j + 1) * nt], small[:, nt, :nt]):
            return f"last row of tile column {j}"
    return None


@pytest.mark.parametrize("fp32", [False, True])
def test_tiled_grid_past_32_bit_offsets_bitwise(dev, fp32):
    """33000^2 = 1.089e9 cells: the state's byte offsets pass 2^32 in its
    first component and its element offsets pass 2^31 in the second, so a
    32-bit index product anywhere in the sweeps or the stage updates would
    read or write the wrong cells.  The state tiles a periodic 3000^2 grid
    11 x 11 times (smooth and discontinuous parts, every component varying
    along both directions), with the same mesh width: every interface of the large grid then
    sees the stencil values of its image in the small grid, and the global
    wave speeds are maxima over the same values, so the interface fluxes,
    the CFL step and the stepped state must equal the small grid's, tiled,
    bit for bit.  The small grid's step is checked against the oracle (FP32
    reconstruction, whose stage sweeps are the one-shot kernels: against
    its FP32 reading, to the 1e-4 of the component scale that the flux bar
    of 3e-5 allows a step; the two readings differ by up to 8.2e-6 at this
    data's sharpest points)."""
    nt, k = 3000, 11
    n = nt * k
    free, _ = torch.cuda.mem_get_info()
    need = 6 * 4 * n * n * 8 + (4 << 30)   # state, three context states, two flux arrays
    if free < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory, {free / 2**30:.0f} GiB free")
    from paper_2603_26272_amd.problem import EULER, PERIODIC, Problem
    x = W.centres(nt, 0.0, 1.0)[None, :]
    y = W.centres(nt, 0.0, 1.0)[:, None]
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * (2 * x + y)) + 0.5 * ((x > 0.55) & (y > 0.4))
    u = 0.4 * np.sin(2 * np.pi * (y + 0.1)) + 0.1 * np.cos(2 * np.pi * x)
    v = 0.3 * np.cos(6 * np.pi * x) + 0.2 * np.sin(4 * np.pi * y)
    p = 1.0 + 0.2 * np.cos(2 * np.pi * (x - 2 * y)) + 0.4 * (x + y > 1.0)
    q_t = np.ascontiguousarray(W.conservative(rho, u, v, p, dim=2))
    Pt = Problem(dim=2, system=EULER, nx=nt, ny=nt, bc_x=PERIODIC, bc_y=PERIODIC, cfl=0.5)
    if fp32:
        Pt = Pt.fp32()
    Pb = Pt.with_(nx=n, ny=n, xhi=float(k), yhi=float(k))
    assert Pb.dx == Pt.dx and Pb.dy == Pt.dy

    qs = torch.from_numpy(q_t).to(dev)
    with Ctx(Pt) as ctx:
        fxs, fys = ctx.rhs_fluxes(qs)
        dts = ctx.step(qs, 0.0, sync=True)
    torch.cuda.synchronize()
    orc.set_threads(16)
    assert dts == orc.cfl_dt(Pt, q_t)
    ref, steps, t, st = orc.solve(Pt, q_t, 0.0, 1)
    assert st == 0 and steps == 1 and t == dts
    assert_close(qs.cpu().numpy(), ref, 1e-4 if fp32 else 1e-10, "3000^2 periodic, one step")

    qb = torch.from_numpy(q_t).to(dev).repeat(1, k, k)
    try:
        with Ctx(Pb) as ctx:
            fxb, fyb = ctx.rhs_fluxes(qb)
            torch.cuda.synchronize()
            assert _tiles_equal(fxb, fxs, k, nt) is None, "x fluxes: " + str(_tiles_equal(fxb, fxs, k, nt))
            assert _tiles_equal(fyb, fys, k, nt) is None, "y fluxes: " + str(_tiles_equal(fyb, fys, k, nt))
            del fxb, fyb
            dtb = ctx.step(qb, 0.0, sync=True)
        torch.cuda.synchronize()
        assert dtb == dts
        bad = _tiles_equal(qb, qs, k, nt)
        assert bad is None, "stepped state: " + bad
    finally:
        del qb
        torch.cuda.empty_cache()


def test_tiled_line_past_32_bit_offsets_bitwise(dev):
    """A 1D Euler line of 1.09998e9 cells tiling a periodic line of 999983
    cells 1100 times (the same mesh width): byte offsets pass 2^32 within the
    first component and element offsets pass 2^31 in the second, through the
    1D paths (the looped stage sweep with its maxima rows per wavefront, the
    one-shot flux sweep).  Fluxes, the CFL step and the stepped state equal
    the short line's, tiled, bit for bit; the short line's step is checked
    against the oracle."""
    nt, k = 999983, 1100
    n = nt * k
    free, _ = torch.cuda.mem_get_info()
    need = 4 * 3 * n * 8 + (4 << 30)   # state, two context states, the fluxes
    if free < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory, {free / 2**30:.0f} GiB free")
    from paper_2603_26272_amd.problem import EULER, PERIODIC, Problem
    x = W.centres(nt, 0.0, 1.0)
    rho = 1.0 + 0.3 * np.sin(6 * np.pi * x) + 0.5 * (x > 0.4)
    u = 0.4 * np.sin(2 * np.pi * x) + 0.1 * np.cos(10 * np.pi * x)
    p = 1.0 + 0.2 * np.cos(10 * np.pi * x) + 0.4 * (x > 0.7)
    q_t = np.ascontiguousarray(W.conservative(rho, u, 0.0, p, dim=1).reshape(3, 1, nt))
    Pt = Problem(dim=1, system=EULER, nx=nt, bc_x=PERIODIC, cfl=0.5)
    Pb = Pt.with_(nx=n, xhi=float(k))
    assert Pb.dx == Pt.dx

    qs = torch.from_numpy(q_t).to(dev)
    with Ctx(Pt) as ctx:
        fs, _ = ctx.rhs_fluxes(qs)
        dts = ctx.step(qs, 0.0, sync=True)
    torch.cuda.synchronize()
    assert dts == orc.cfl_dt(Pt, q_t)
    ref, steps, t, st = orc.solve(Pt, q_t, 0.0, 1)
    assert st == 0 and steps == 1 and t == dts
    assert_close(qs.cpu().numpy(), ref, 1e-10, "periodic line of 999983 cells, one step")

    qb = torch.from_numpy(q_t).to(dev).repeat(1, 1, k)
    try:
        with Ctx(Pb) as ctx:
            fb, _ = ctx.rhs_fluxes(qb)
            torch.cuda.synchronize()
            assert bool((fb[:, 0, :n].view(3, k, nt) == fs[:, 0, :nt].view(3, 1, nt)).all()), "fluxes"
            assert torch.equal(fb[:, 0, n], fs[:, 0, nt]), "last interface"
            del fb
            dtb = ctx.step(qb, 0.0, sync=True)
        torch.cuda.synchronize()
        assert dtb == dts
        assert bool((qb.view(3, k, nt) == qs.view(3, 1, nt)).all()), "stepped state"
    finally:
        del qb
        torch.cuda.empty_cache()
