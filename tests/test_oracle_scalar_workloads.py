"""Pins of the scalar-law workloads of Section 4.1 (multi-wave advection,
Burgers, Buckley-Leverett) and of the oracle's Lax-Friedrichs speed for the
non-convex Buckley-Leverett flux."""
import math

import numpy as np
import pytest

from paper_2603_26272_amd import workloads as W


def _brute_max_speed(lo, hi):
    u = np.linspace(lo, hi, 400001)
    D = u * u + 0.25 * (1 - u) ** 2
    fp = np.abs((2 * u * D - u * u * (2 * u - 0.5 * (1 - u))) / (D * D))   # quotient rule of f = u^2/D
    i = int(fp.argmax())
    a, b = u[max(i - 1, 0)], u[min(i + 1, len(u) - 1)]
    v = np.linspace(a, b, 200001)
    D = v * v + 0.25 * (1 - v) ** 2
    return float(np.abs((2 * v * D - v * v * (2 * v - 0.5 * (1 - v))) / (D * D)).max())


@pytest.mark.parametrize("lo,hi", [(0.0, 1.0), (0.5, 1.0), (0.1, 0.2), (-0.3, 0.1), (-0.6, 1.6),
                                   (0.3, 0.3), (1.2, 1.45)])
def test_buckley_lf_speed_is_max_over_data_range(orc, lo, hi):
    """The oracle's LF speed for Buckley-Leverett is max |f'| over [min u,
    max u] (brute force over a fine sampling of the range, f' by the quotient
    rule)."""
    q = np.array([lo, hi, 0.5 * (lo + hi)]).reshape(1, 1, 3)
    P = {"dim": 1, "system": 3, "nx": 3, "bc_x": 1}
    a, s, st = orc.wave_speeds(P, q)
    ref = _brute_max_speed(lo, hi)
    assert st == 0
    assert abs(a[0, 0] - ref) <= 1e-9 * ref and abs(s[0] - ref) <= 1e-9 * ref


def test_multiwave_initial_data_closed_forms():
    d = 0.005
    x = np.array([-0.7, -0.3, 0.1, 0.5, 0.0, 0.2, 0.9, -0.9])
    q = W.multiwave_exact(x)
    assert q[0] == pytest.approx((4.0 + 2.0 * 2.0 ** (-1.0 / 36.0)) / 6.0, rel=1e-15)  # Gaussian peak
    assert q[1] == 1.0                                                            # square wave
    assert q[2] == pytest.approx(1.0, abs=1e-15)                                  # triangle apex
    assert q[3] == pytest.approx((4.0 + 2.0 * math.sqrt(1.0 - 100.0 * d * d)) / 6.0, rel=1e-15)  # ellipse
    assert q[4] == 0.0 and q[5] == pytest.approx(0.0, abs=1e-15)                  # triangle feet
    assert q[6] == 0.0 and q[7] == 0.0


@pytest.mark.parametrize("t", [0.0, 0.1, 0.15, 0.2])
def test_burgers_exact_solves_characteristics(t):
    x = np.linspace(0.0, 1.0, 301)[:-1]
    u = W.burgers_sine_exact(x, t)
    assert np.abs(u - (0.5 + np.sin(2 * np.pi * (x - u * t)))).max() < 1e-13


def test_burgers_exact_shock_position():
    """After breaking (t = 1/(2 pi)) the solution jumps at x_s = 1/2 + t/2
    from above the mean to below it."""
    t = 0.2
    xs = 0.5 + 0.5 * t
    u = W.burgers_sine_exact(np.array([xs - 1e-9, xs + 1e-9]), t)
    assert u[0] > 0.5 + 0.3 and u[1] < 0.5 - 0.3


def test_oracle_burgers_converges_before_breaking(orc):
    errs = []
    for N in (80, 160, 320):
        P, q0 = W.burgers_sine(N)
        q, steps, t, st = orc.solve(P, q0, 0.1)
        errs.append(np.abs(q[0, 0] - W.burgers_sine_exact(W.centres(N, 0.0, 1.0), 0.1)).max())
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-6, errs


def test_oracle_multiwave_eno(orc):
    """Ten periods of the multi-wave data (N = 400, T = 20): nearly free of
    over- and undershoots, and close to the exact (initial) profile."""
    P, q0 = W.multiwave(400)
    q, steps, t, st = orc.solve(P, q0, W.MULTIWAVE_T)
    assert st == 0 and t == W.MULTIWAVE_T
    assert q.max() < 1.0 + 1e-4 and q.min() > -1e-4
    e = np.abs(q[0, 0] - W.multiwave_exact(W.centres(400, -1.0, 1.0)))
    assert e.mean() * 2.0 < 0.05


def test_oracle_buckley_bounded_conservative_convergent(orc):
    P, q0 = W.buckley_step(200)
    q, steps, t, st = orc.solve(P, q0, W.BUCKLEY_T)
    assert st == 0 and t == W.BUCKLEY_T
    assert q.max() < 1.0 + 1e-6 and q.min() > -1e-6
    dx = 2.0 / 200
    assert abs(q.sum() * dx - q0.sum() * dx) < 1e-13           # transmissive, zero flux at the ends
    Pf, qf = W.buckley_step(1600)
    rf, _, _, _ = orc.solve(Pf, qf, W.BUCKLEY_T)
    ref = rf[0, 0].reshape(200, 8).mean(axis=1)
    assert np.abs(q[0, 0] - ref).mean() * 2.0 < 0.02
