"""The weight families of tab:SpecialCases through the parameters L and q of
eq:weights_unnormalized, alpha_k = d_k (L + Gamma_k)^q, checked in the
oracle against what the mathematics fixes:

  * L = 0, p = 2 is the Jiang-Shu form d_k / (beta_k + eps)^2 (the factor
    tau^2 cancels in omega), compared with exact rational candidates and
    indicators from the definitions (tests/test_oracle_bruteforce.py);
  * where tau = 0 (data of degree <= 4) every family with L > 0 has
    omega = d and reproduces the six-point central flux exactly, and L = 0
    gives the same Jiang-Shu weights (the limit tau -> 0+);
  * L = q = 1 is the default scheme, bit for bit;
  * with the descaler mu[f] of eq:aimu (Ai-JS, Ai-Z) the reconstruction
    scales with the data (affine invariance at amplitudes 1e-20 .. 1e20).
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from tests.test_oracle_bruteforce import brute, ideal_weights

EPS = 1e-40


def _js_flux(v, p=2):
    b = brute(v)
    d = ideal_weights()
    al = [d[k] / (b["beta"][k if k < 3 else 4] + Fr(EPS)) ** p for k in range(4)]
    s = sum(al)
    return float(sum(a / s * q for a, q in zip(al, b["q"]))), [float(a / s) for a in al]


def _cases(n=40, seed=11):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        v = rng.standard_normal(6)
        if i % 3 == 1:
            v[3:] += 5.0                       # a jump inside the stencil
        if i % 3 == 2:
            v = np.cumsum(np.abs(v))           # monotone data
        out.append([float(Fr(x).limit_denominator(1 << 20)) for x in v])
    return out


def test_L0_p2_is_jiang_shu(orc):
    for v in _cases():
        ref, om_ref = _js_flux(v)
        got, d = orc.recon_lq(np.array(v), 0.0, 1.0, p=2.0, detail=True)
        assert abs(got - ref) <= 1e-13 * (1 + abs(ref)), (v, got, ref)
        assert np.allclose(d["omega"], om_ref, rtol=1e-12, atol=1e-15)
        # the same weights as p = 1 with q = 2 (only the product pq enters)
        assert abs(orc.recon_lq(np.array(v), 0.0, 2.0, p=1.0) - got) <= 1e-14 * (1 + abs(got))


def test_tau_zero_gives_ideal_weights_or_js(orc):
    x = np.arange(-2, 4, dtype=float)
    for coeffs in ([1, 0.5, -0.25, 0.125, 0.0625], [2, -1, 0, 0.375, 0], [0, 0, 1, 0, 0]):
        v = sum(c * x ** k for k, c in enumerate(coeffs))
        b = brute([Fr(t) for t in v])
        assert b["tau"] == 0
        central = float(b["central"])
        for L, q, p in ((1.0, 1.0, 1.0), (0.5, 2.0, 1.0), (3.0, 1.5, 2.0)):
            got = orc.recon_lq(v, L, q, p=p)
            assert abs(got - central) <= 1e-13 * (1 + abs(central)), (coeffs, L, q)
        js, _ = _js_flux([Fr(t) for t in v])
        assert abs(orc.recon_lq(v, 0.0, 1.0, p=2.0) - js) <= 1e-13 * (1 + abs(js))


def test_default_parameters_are_the_paper_scheme(orc):
    for v in _cases(20, seed=3):
        v = np.array(v)
        assert orc.recon_lq(v, 1.0, 1.0) == orc.recon(v)
        assert orc.recon_lq(v, 1.0, 1.0, p=1.5, ai=1) == orc.recon(v, p=1.5, ai=1)


@pytest.mark.parametrize("L,p", [(0.0, 2.0), (1.0, 2.0), (1.0, 1.0)])
def test_ai_families_scale_with_the_data(orc, L, p):
    for v in _cases(15, seed=7):
        v = np.array(v)
        base = orc.recon_lq(v, L, 1.0, p=p, ai=1, mu0=1e-300)
        for lam in (1e-20, 1e-5, 1e5, 1e20):
            got = orc.recon_lq(lam * v, L, 1.0, p=p, ai=1, mu0=1e-300)
            assert abs(got - lam * base) <= 1e-12 * lam * (1 + abs(base)), (L, p, lam)


def test_order_2r_families(orc):
    """r = 2..5 share the weight code: L = 0, p = 2 there also gives
    omega proportional to d_k / (beta_k + eps)^2 with the oracle's own
    indicators, and tau = 0 data (degree <= 2r - 2) the central flux."""
    rng = np.random.default_rng(5)
    for r in (2, 4, 5):
        for _ in range(10):
            v = rng.standard_normal(2 * r)
            ref, d = orc.recon_r(r, v, detail=True)
            betas = list(d["beta"]) + [d["beta_r"]]
            w = [dk / (b + EPS) ** 2 for dk, b in zip(_ideal(orc, r), betas)]
            js = sum(wi * qi for wi, qi in zip(w, d["q"])) / sum(w)
            got = orc.recon_r_lq(r, v, 0.0, 1.0, p=2.0)
            assert abs(got - js) <= 1e-12 * (1 + abs(js)), r
        x = np.arange(-r + 1, r + 1, dtype=float)
        v = 0.3 + 0.2 * x + 0.05 * x ** 2
        central = orc.recon_r(r, v, linear=1)
        assert abs(orc.recon_r_lq(r, v, 0.5, 2.0) - central) <= 1e-13 * (1 + abs(central))


def _ideal(orc, r):
    from oracle import coeffs
    return [float(x) for x in coeffs.tables(r)["d"]]


def test_q_raises_the_weight_ratios_to_the_power_q(orc):
    """(omega_i / d_i) / (omega_j / d_j) = ((L + Gamma_i) / (L + Gamma_j))^q, so
    going from q = 1 to q = 2 squares every such ratio (catches q applied to
    Gamma alone, or not at all)."""
    d = [float(x) for x in ideal_weights()]
    for v in _cases(20, seed=9):
        v = np.array(v)
        for L in (0.5, 1.0, 2.0):
            _, a = orc.recon_lq(v, L, 1.0, detail=True)
            _, b = orc.recon_lq(v, L, 2.0, detail=True)
            ra = np.array(a["omega"]) / d
            rb = np.array(b["omega"]) / d
            for i in range(1, 4):
                assert np.isclose(rb[i] / rb[0], (ra[i] / ra[0]) ** 2, rtol=1e-10), (L, i)
