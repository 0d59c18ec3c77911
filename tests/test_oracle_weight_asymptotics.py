"""Weights next to a discontinuity (Section 2.2), as properties of the
oracle's nonlinear weights (d = (1, 9, 9, 1)/20, eps = 1e-40, so eps = 0
for these data):

  * a substencil D that contains a jump against a smooth substencil S:
    (d_S / d_D)(omega_D / omega_S) = O(dx^(2p)) when f'(x_i) != 0;
  * the downwind weight against the discontinuous substencil D with the
    largest indicator: (d_3 / d_D)(omega_D / omega_3) lies in (c^p, 1] with
    c = beta_3 / beta_D, and equals (1 + Theta)/(1 + c^(-p) Theta),
    Theta = (tau / beta_D)^p.
"""
import numpy as np
import pytest

D = np.array([1.0, 9.0, 9.0, 1.0]) / 20


def _stencil(h):
    """f = sin(x) + [x > 1.5 h] at x_j = j h, j = -2..3: S_0 and S_1 are
    smooth, S_2 = {0, 1, 2} and the downwind S_3 = {1, 2, 3} hold the jump."""
    x = h * np.arange(-2, 4)
    return np.sin(x) + (x > 1.5 * h)


@pytest.mark.parametrize("p", [1.0, 1.5, 2.0])
def test_discontinuous_over_smooth_is_order_dx_2p(orc, p):
    hs = [0.1 / 2 ** k for k in range(5)]
    ratios = []
    for h in hs:
        _, d = orc.recon(_stencil(h), p=p, detail=True)
        om = d["omega"]
        ratios.append((D[0] / D[2]) * (om[2] / om[0]))
    rates = np.log2(np.array(ratios[:-1]) / np.array(ratios[1:]))
    assert np.all(np.abs(rates - 2 * p) < 0.15), (p, rates)


@pytest.mark.parametrize("p", [1.0, 1.5, 2.0])
def test_downwind_against_discontinuous_in_c_p_to_1(orc, p):
    rng = np.random.default_rng(int(10 * p))
    seen = 0
    for _ in range(300):
        v = rng.standard_normal(6) * 0.1
        v[rng.integers(1, 6):] += rng.choice([-1.0, 1.0]) * rng.uniform(0.5, 3.0)   # one jump
        _, d = orc.recon(v, p=p, detail=True)
        beta = d["beta"]           # beta_0, beta_1, beta_2, beta_d, beta_3
        b = [beta[0], beta[1], beta[2]]
        k = int(np.argmax(b))      # the upwind substencil with the largest indicator
        bD, b3, tau = b[k], beta[4], d["tau"]
        if tau < 1e-6 * bD:
            continue
        c = b3 / bD
        if c > 1:
            continue               # beta_d dominates: the estimate is stated for beta_3 <= beta_D
        om = d["omega"]
        ratio = (D[3] / D[k]) * (om[k] / om[3])
        theta = (tau / bD) ** p
        assert abs(ratio - (1 + theta) / (1 + theta / c ** p)) <= 1e-10 * ratio
        assert c ** p * (1 - 1e-12) < ratio <= 1 + 1e-12
        seen += 1
    assert seen > 100
