"""Translation invariance of the oracle under periodic tiling (CPU).

With periodic boundaries, a grid that repeats a tile k times in each
direction (same mesh width) presents every interface with the stencil
values of its image in the tile, and the global Lax-Friedrichs speeds of
eq:LF are maxima over the same values; the CFL step follows from those
maxima.  So the oracle's fluxes, its CFL step and one SSP-RK3 step on the
tiled grid must equal the tile's, repeated, bit for bit.  A periodic ghost
taken from the wrong end, or a global speed taken over part of the grid,
breaks this.  The GPU test of the same property runs it past 32-bit offsets.
"""
import numpy as np
import pytest

import oracle as orc
from paper_2603_26272_amd import workloads as W
from paper_2603_26272_amd.problem import EULER, PERIODIC, Problem


def tile_2d(nt_x, nt_y):
    x = W.centres(nt_x, 0.0, 1.0)[None, :]
    y = W.centres(nt_y, 0.0, 1.0)[:, None]
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * (2 * x + y)) + 0.5 * ((x > 0.55) & (y > 0.4))
    u = 0.4 * np.sin(2 * np.pi * (y + 0.1)) + 0.1 * np.cos(2 * np.pi * x)
    v = 0.3 * np.cos(6 * np.pi * x) + 0.2 * np.sin(4 * np.pi * y)
    p = 1.0 + 0.2 * np.cos(2 * np.pi * (x - 2 * y)) + 0.4 * (x + y > 1.0)
    return np.ascontiguousarray(W.conservative(rho, u, v, p, dim=2))


@pytest.mark.parametrize("fp32", [False, True])
def test_tiled_2d_equals_tile(fp32):
    ntx, nty, kx, ky = 40, 36, 3, 2
    qt = tile_2d(ntx, nty)
    Pt = Problem(dim=2, system=EULER, nx=ntx, ny=nty, bc_x=PERIODIC, bc_y=PERIODIC, cfl=0.5)
    if fp32:
        Pt = Pt.fp32()
    Pb = Pt.with_(nx=kx * ntx, ny=ky * nty, xhi=float(kx), yhi=float(ky))
    assert Pb.dx == Pt.dx and Pb.dy == Pt.dy
    qb = np.tile(qt, (1, ky, kx))
    fxt, fyt, st = orc.fluxes(Pt, qt)
    assert st == 0
    fxb, fyb, st = orc.fluxes(Pb, qb)
    assert st == 0
    # interface I of the tiled grid is interface I mod nt of the tile, the
    # last one (I = k nt) the tile's last (nt), which periodicity makes its first
    assert np.array_equal(fxb[:, :, :-1], np.tile(fxt[:, :, :-1], (1, ky, kx)))
    assert np.array_equal(fxb[:, :, -1], np.tile(fxt[:, :, -1], (1, ky)))
    assert np.array_equal(fyb[:, :-1, :], np.tile(fyt[:, :-1, :], (1, ky, kx)))
    assert np.array_equal(fyb[:, -1, :], np.tile(fyt[:, -1, :], (1, kx)))
    assert orc.cfl_dt(Pb, qb) == orc.cfl_dt(Pt, qt)
    q1t, dtt, st = orc.step(Pt, qt)
    assert st == 0
    q1b, dtb, st = orc.step(Pb, qb)
    assert st == 0 and dtb == dtt
    assert np.array_equal(q1b, np.tile(q1t, (1, ky, kx)))


def test_tiled_1d_equals_tile():
    nt, k = 301, 5
    x = W.centres(nt, 0.0, 1.0)
    rho = 1.0 + 0.3 * np.sin(6 * np.pi * x) + 0.5 * (x > 0.4)
    u = 0.4 * np.sin(2 * np.pi * x) + 0.1 * np.cos(10 * np.pi * x)
    p = 1.0 + 0.2 * np.cos(10 * np.pi * x) + 0.4 * (x > 0.7)
    qt = np.ascontiguousarray(W.conservative(rho, u, 0.0, p, dim=1).reshape(3, 1, nt))
    Pt = Problem(dim=1, system=EULER, nx=nt, bc_x=PERIODIC, cfl=0.5)
    Pb = Pt.with_(nx=k * nt, xhi=float(k))
    assert Pb.dx == Pt.dx
    qb = np.tile(qt, (1, 1, k))
    fxt, _, st = orc.fluxes(Pt, qt)
    fxb, _, st2 = orc.fluxes(Pb, qb)
    assert st == 0 and st2 == 0
    assert np.array_equal(fxb[:, :, :-1], np.tile(fxt[:, :, :-1], (1, 1, k)))
    assert np.array_equal(fxb[:, :, -1], fxt[:, :, -1])
    q1t, dtt, st = orc.step(Pt, qt)
    q1b, dtb, st2 = orc.step(Pb, qb)
    assert st == 0 and st2 == 0 and dtb == dtt
    assert np.array_equal(q1b, np.tile(q1t, (1, 1, k)))


def test_tiling_detects_a_shifted_tile():
    """Negative control: the same check fails when one tile of the large grid
    is shifted by one cell, so equality is not vacuous."""
    ntx, nty, kx, ky = 40, 36, 2, 2
    qt = tile_2d(ntx, nty)
    Pt = Problem(dim=2, system=EULER, nx=ntx, ny=nty, bc_x=PERIODIC, bc_y=PERIODIC, cfl=0.5)
    Pb = Pt.with_(nx=kx * ntx, ny=ky * nty, xhi=float(kx), yhi=float(ky))
    qb = np.tile(qt, (1, ky, kx))
    qb[:, nty:, ntx:] = np.roll(qt, 1, axis=2)
    fxt, _, _ = orc.fluxes(Pt, qt)
    fxb, _, _ = orc.fluxes(Pb, qb)
    assert not np.array_equal(fxb[:, :, :-1], np.tile(fxt[:, :, :-1], (1, ky, kx)))
