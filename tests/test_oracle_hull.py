"""The flux validity check used where rounding alone sets the weights
(tests/test_gpu_ties.py), on the oracle alone: the oracle's fluxes satisfy it
at every interface, and values just outside the bounds, or a reconstruction
with a weight outside [0, 1], fail it."""
import numpy as np

import oracle as orc
from paper_2603_26272_amd import workloads as W

from tests.char_hull import hull, hull_violation


def test_oracle_fluxes_valid_everywhere():
    """The validity check itself, on the oracle alone: every interface of
    tied and untied data, 1D r = 2 and 2D r = 3 both directions."""
    P, q0 = W.riemann_1d(1, 120)
    P = P.with_(order=2)
    rx, _, _ = orc.fluxes(P, q0)
    alpha = orc.wave_speeds(P, q0)[0][0]
    for k in range(0, 121, 3):
        assert hull_violation(*hull(P, q0, 0, 0, k, alpha, 2), rx[:, 0, k]).max() <= 1.0
    P, q0 = W.quadrants_2d(3, 24, 20)
    rx, ry, _ = orc.fluxes(P, q0)
    a = orc.wave_speeds(P, q0)[0]
    for line in (0, 7, 19):
        for k in range(0, 25, 4):
            assert hull_violation(*hull(P, q0, 0, line, k, a[0], 3), rx[:, line, k]).max() <= 1.0
    for line in (0, 11, 23):
        for k in range(0, 21, 4):
            assert hull_violation(*hull(P, q0, 1, line, k, a[1], 3), ry[:, k, line]).max() <= 1.0


def test_check_rejects_invalid_reconstructions():
    """Plant the mistakes on the oracle's side: a flux just outside the
    bounds of one field, and one whose field value combines the candidates
    with weights (-0.5, 1.5) instead of a convex combination."""
    P, q0 = W.riemann_1d(2, 120)
    P = P.with_(order=2)
    rx, _, _ = orc.fluxes(P, q0)
    alpha = orc.wave_speeds(P, q0)[0][0]
    bad = eligible = 0
    for k in range(10, 111, 10):
        Lm, lo, hi = hull(P, q0, 0, 0, k, alpha, 2)
        g = Lm @ rx[:, 0, k]
        out = g.copy()
        out[1] = hi[1] + 1e-9 * (abs(hi[1]) + 1)
        assert hull_violation(Lm, lo, hi, np.linalg.solve(Lm, out)).max() > 1.0
        # extrapolating past the extreme candidates leaves the bounds
        if hi[1] - lo[1] > 1e-6 * (abs(hi[1]) + abs(lo[1])):
            eligible += 1
            ext = g.copy()
            ext[1] = -0.5 * lo[1] + 1.5 * hi[1]
            bad += hull_violation(Lm, lo, hi, np.linalg.solve(Lm, ext)).max() > 1.0
    assert eligible >= 3 and bad == eligible
