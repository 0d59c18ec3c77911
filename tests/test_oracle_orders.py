"""Pins of the oracle's even-order (2r, r = 2..5) central-upwind schemes.

The coefficient tables are derived in exact arithmetic from the definitions
(oracle/coeffs.py) and must reproduce the tables the paper prints (Section 3
for r = 3, Appendix A for r = 2, 4, 5; tests/golden/order_tables.json), the
closed form of the ideal weights, and the polynomial exactness that defines
them.  The C oracle's generic reconstruction is pinned against the separately
written sixth-order routine, against the linear central flux, and by the
convergence order of its right-hand side on smooth data.
"""
import json
import os
from fractions import Fraction as Fr
from math import comb

import numpy as np
import pytest

import oracle
from oracle import coeffs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "order_tables.json")


def _printed(r):
    g = json.load(open(GOLDEN))[str(r)]
    out = {"c2r": [Fr(n, g["c2r"]["den"]) for n in g["c2r"]["num"]],
           "d": [Fr(n, g["d"]["den"]) for n in g["d"]["num"]],
           "ctau": [Fr(n) for n in g["ctau"]]}
    ck = {int(k): [Fr(n, g["ck"]["den"]) for n in v] for k, v in g["ck"]["num"].items()}
    for k, src in g["ck"]["rev"].items():
        ck[int(k)] = list(reversed(ck[int(src)]))
    out["ck"] = [ck[k] for k in range(r + 1)]
    den = g["B"]["den"]
    B = {}
    for k, v in g["B"]["num"].items():
        B[k] = [[Fr(n, den) for n in row] for row in v]
    for k, src in g["B"]["rev"].items():
        M = B[src]
        B[k] = [list(reversed(row)) for row in reversed(M)]
    out["B"] = [B[str(k)] for k in range(r)]
    out["Bd"] = B["d"]
    return out


@pytest.mark.parametrize("r", [2, 3, 4, 5])
def test_derived_tables_equal_printed(r):
    t = coeffs.tables(r)
    p = _printed(r)
    assert t["c2r"] == p["c2r"]
    assert t["ck"] == p["ck"]
    assert t["d"] == p["d"]
    assert t["ctau"] == p["ctau"]
    assert t["B"] == p["B"]
    assert t["Bd"] == p["Bd"]


@pytest.mark.parametrize("r", [2, 3, 4, 5, 6])
def test_ideal_weights_closed_form(r):
    t = coeffs.tables(r)
    assert t["d"] == [Fr(comb(r, k) ** 2, comb(2 * r, r)) for k in range(r + 1)]


def _cell_avg_power(o, m):
    a, b = Fr(2 * o - 1, 2), Fr(2 * o + 1, 2)
    return (b ** (m + 1) - a ** (m + 1)) / (m + 1)


@pytest.mark.parametrize("r", [2, 3, 4, 5])
def test_polynomial_exactness(r):
    """c_2r reproduces h(x_{i+1/2}) from the cell averages of h = x^m for
    m <= 2r-1 and not for m = 2r (order exactly 2r); each c_k for m <= r-1."""
    t = coeffs.tables(r)
    big = list(range(-r + 1, r + 1))
    for m in range(2 * r + 1):
        f = [_cell_avg_power(o, m) for o in big]
        val = sum(c * x for c, x in zip(t["c2r"], f))
        if m <= 2 * r - 1:
            assert val == Fr(1, 2) ** m
        else:
            assert val != Fr(1, 2) ** m
    for k in range(r + 1):
        offs = coeffs.substencil_offsets(r, k)
        for m in range(r):
            f = [_cell_avg_power(o, m) for o in offs]
            assert sum(c * x for c, x in zip(t["ck"][k], f)) == Fr(1, 2) ** m


@pytest.mark.parametrize("r", [2, 3, 4, 5])
def test_indicator_matrices(r):
    """Symmetric, constants in the null space, positive semidefinite, and a
    linear ramp (slope 1 per cell) has indicator exactly 1 on every
    substencil (only the first-derivative term survives)."""
    t = coeffs.tables(r)
    for B in t["B"] + [t["Bd"]]:
        n = len(B)
        assert all(B[i][j] == B[j][i] for i in range(n) for j in range(n))
        assert all(sum(row) == 0 for row in B)
        ev = np.linalg.eigvalsh(np.array([[float(x) for x in row] for row in B]))
        assert ev.min() > -1e-9 * ev.max()
        ramp = [Fr(j) for j in range(n)]
        assert sum(ramp[i] * B[i][j] * ramp[j] for i in range(n) for j in range(n)) == 1


def test_generic_sixth_order_matches_za6_routine():
    """Two independent writings of the r = 3 reconstruction (the generic
    tables with the integral form of eq:SI, and the closed-form sixth-order
    routine) agree to rounding."""
    rng = np.random.default_rng(7)
    for t in range(3000):
        scale = rng.choice([1e-3, 1.0, 1e3])
        v = rng.standard_normal(6) * scale
        if t % 3 == 0:
            v[3:] += 5 * scale * rng.standard_normal()
        a, b = oracle.recon(v), oracle.recon_r(3, v)
        assert abs(a - b) <= 5e-13 * (abs(a) + np.abs(v).max())


@pytest.mark.parametrize("r", [2, 4, 5])
def test_linear_weights_give_central_flux(r):
    c2r = [float(c) for c in coeffs.tables(r)["c2r"]]
    rng = np.random.default_rng(r)
    for _ in range(200):
        v = rng.standard_normal(2 * r)
        ref = sum(c * x for c, x in zip(c2r, v))
        assert abs(oracle.recon_r(r, v, linear=1) - ref) <= 1e-14 * (1 + np.abs(v).sum())


@pytest.mark.parametrize("r", [2, 4, 5])
def test_quad_and_fp64_agree(r):
    rng = np.random.default_rng(10 + r)
    for _ in range(200):
        v = rng.standard_normal(2 * r)
        a, b = oracle.recon_r(r, v), oracle.recon_r(r, v, prec=2)
        assert abs(a - b) <= 1e-13 * (1 + np.abs(v).max())


@pytest.mark.parametrize("r", [2, 4, 5])
def test_jump_excludes_crossing_substencils(r):
    """A step between f_i and f_{i+1}: only S_0 (cells i-r+1..i) lies on one
    side, every other substencil crosses the jump, so omega_0 -> 1 and the
    flux is the left state."""
    v = np.array([1.0] * r + [0.0] * r)
    out, det = oracle.recon_r(r, v, detail=True)
    assert det["omega"][0] > 1 - 1e-12
    assert abs(out - 1.0) < 1e-12


@pytest.mark.parametrize("r", [2, 4, 5])
def test_smooth_weights_approach_ideal(r):
    d = np.array([float(x) for x in coeffs.tables(r)["d"]])
    devs = []
    for h in (0.4, 0.2, 0.1, 0.05):
        x = (np.arange(2 * r) - r + 0.5) * h + 0.3
        _, det = oracle.recon_r(r, np.exp(x), detail=True)
        devs.append(np.abs(det["omega"] - d).max())
    for a, b in zip(devs, devs[1:]):
        assert b < a or b < 1e-14, devs
    assert devs[-1] < 1e-6


def _rhs_error(r, N, smooth):
    if smooth == "exp":   # no critical point
        P = {"dim": 1, "system": 0, "nx": N, "xlo": 0.0, "xhi": 1.0, "bc_x": 1, "order": r,
             "adv_speed": (1.0, 0.0)}
        x = (np.arange(N) + 0.5) / N
        q = np.exp(3 * x)[None, None, :].copy()
        L = np.asarray(oracle.rhs(P, q)[0]).reshape(-1)
        inner = slice(r + 2, N - r - 2)
        return np.abs(L + 3 * np.exp(3 * x))[inner].max()
    P = {"dim": 1, "system": 0, "nx": N, "xlo": -1.0, "xhi": 1.0, "bc_x": 0, "order": r,
         "adv_speed": (1.0, 0.0)}
    x = -1 + (np.arange(N) + 0.5) * 2 / N
    q = np.sin(np.pi * x + 0.3)[None, None, :].copy()
    L = np.asarray(oracle.rhs(P, q)[0]).reshape(-1)
    return np.abs(L + np.pi * np.cos(np.pi * x + 0.3)).max()


@pytest.mark.parametrize("r,smooth,sizes", [(2, "exp", (32, 64, 128)), (3, "sin", (16, 32, 64)),
                                            (4, "sin", (16, 32, 64)), (5, "sin", (12, 24, 48))])
def test_rhs_convergence_order(r, smooth, sizes):
    """The spatial operator converges at order 2r on smooth data (scalar
    advection, -u_x).  r = 2 uses data without critical points: next to an
    extremum two neighbouring values can nearly coincide, the two-point
    indicator then nearly vanishes and the fourth-order scheme falls back on
    one candidate there."""
    e = [_rhs_error(r, n, smooth) for n in sizes]
    rates = [np.log2(e[i] / e[i + 1]) for i in range(len(e) - 1)]
    assert min(rates) > 2 * r - 0.5, (e, rates)


@pytest.mark.parametrize("r", [2, 4, 5])
@pytest.mark.parametrize("name", ["sod", "lax"])
def test_shock_tubes_converge_all_orders(r, name):
    """Characteristic-wise Euler solver of order 2r against the exact Riemann
    solution (shock tubes of the paper's 1D Riemann table)."""
    from paper_2603_26272_amd import workloads as W
    from tests.riemann_exact import sample as riemann_sample
    errs = []
    for N in (100, 200, 400):
        P, q0, T = W.shock_tube(name, N)
        q, steps, t, st = oracle.solve(P.with_(order=r), q0, T)
        assert st == 0 and abs(t - T) < 1e-12
        (rl, ul, pl), (rr, ur, pr), _ = W.SHOCK_TUBES[name]
        ex = riemann_sample((rl, ul, pl), (rr, ur, pr), W.centres(N, -5.0, 5.0), T)
        errs.append(np.abs(q[0, 0] - ex[0]).mean() * 10.0)
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[1] < {"sod": 0.03, "lax": 0.1}[name], errs


@pytest.mark.parametrize("r,sizes", [(4, (16, 32, 64)), (5, (16, 32))])
def test_euler_operator_order(r, sizes):
    """Entropy wave rho = 1 + 0.2 sin(2 pi x), u = p = 1: the density RHS
    converges to -u rho_x at order 2r."""
    from paper_2603_26272_amd import workloads as W
    es = []
    for N in sizes:
        P, q = W.entropy_wave_1d(N)
        L = oracle.rhs(P.with_(order=r), q)[0]
        x = W.centres(N, 0.0, 1.0)
        es.append(np.abs(L[0, 0] + 0.4 * np.pi * np.cos(2 * np.pi * x)).max())
    rates = [np.log2(es[i] / es[i + 1]) for i in range(len(es) - 1)]
    assert min(rates) > 2 * r - 0.5, (es, rates)


@pytest.mark.parametrize("r", [2, 4, 5])
def test_2d_transpose_symmetry_all_orders(r):
    """Swapping x and y (and the momenta) commutes with the 2D RHS."""
    from paper_2603_26272_amd import workloads as W
    P, q = W.quadrants_2d(3, 20, 14)
    rng = np.random.default_rng(r)
    q = q.copy()
    q[0] *= 1 + 0.01 * rng.random(q[0].shape)          # break plateaus (tau = 0 ties)
    L = oracle.rhs(P.with_(order=r), q)[0]
    qt = np.ascontiguousarray(np.stack([q[0].T, q[2].T, q[1].T, q[3].T]))
    Lt = oracle.rhs(P.with_(order=r, nx=14, ny=20), qt)[0]
    back = np.stack([Lt[0].T, Lt[2].T, Lt[1].T, Lt[3].T])
    assert np.abs(L - back).max() <= 1e-12 * (1 + np.abs(L).max())
