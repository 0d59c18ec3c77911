"""The algebra behind the kernels' difference-form WENO-ZA6 (za6_diff and
split_diff in csrc/za_device.hpp), checked on the CPU against the oracle's
reconstruction (Section 3, r = 3: eq:subflux_S6_coeffs, eq:SI_S6,
eq:SI_downwind, eq:GSI, eq:weights_unnormalized, and the splitting of
eq:LF).  The constants of the indicators' sums of two squares are read from
the kernel header itself, so a mistyped digit there fails here.

What the GPU parity tests check element by element is the kernels'
arithmetic; this file pins the reading those kernels implement: that
  * each indicator 6 beta_k is x^2 + y^2 of the header's one-FMA forms,
  * 6 tau = 1.5 t5^2 with t5 the fifth difference,
  * the anchored candidates 3 (q_k - s_A) have the stated coefficients for
    both anchors,
  * the split flux g_2 + (X^+ + X^-)/6 equals the two halves of eq:LF
    reconstructed by the oracle.
"""
import os
import re

import numpy as np
import pytest

import oracle as orc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_2603_26272_amd", "csrc", "za_device.hpp")
S39 = np.sqrt(39.0)


def header_constants():
    src = open(HEADER).read()
    body = src[src.index("__device__ __forceinline__ T za6_diff("):]
    body = body[:body.index("\n}\n")]
    vals = dict((k, float(v)) for k, v in re.findall(r"\b(k[AC][013])\s*=\s*T\(([-0-9.eE+]+)\)", body))
    assert sorted(vals) == ["kA0", "kA1", "kA3", "kC0", "kC1", "kC3"], vals
    return vals


def test_constants_are_the_closed_forms():
    """Each constant is its closed form correctly rounded to FP64 (evaluated
    in 40-digit decimal arithmetic)."""
    from decimal import Decimal, getcontext
    getcontext().prec = 40
    s = Decimal(39).sqrt()
    want = {"kA0": (11 + s) / 8, "kC0": (11 - s) / 8, "kA1": (5 + s) / 8, "kC1": (5 - s) / 8,
            "kA3": (58 - s) / 40, "kC3": (29 + 2 * s) / 40}
    k = header_constants()
    for name, v in want.items():
        assert k[name] == float(v), name


def test_constants_match_the_quadratic_forms():
    """(kA w - u)^2 + (kC w - u)^2 = (kA^2 + kC^2) w^2 - 2 (kA + kC) u w + 2 u^2
    must be 6 beta_k = (3/8)((13/3) e^2 + g^2) in the two differences of the
    stencil: 5 w^2 - 5.5 u w + 2 u^2 (k = 0), 2 w^2 - 2.5 u w + 2 u^2 (k = 1);
    k = 2 mirrors k = 0; the downwind form (kA3 u - w)^2 + (kC3 u - w/2)^2,
    kept at a quarter, must be 2.75 u^2 - 3.625 u w + 1.25 w^2."""
    k = header_constants()
    assert k["kA0"] + k["kC0"] == pytest.approx(2.75, rel=1e-15)
    assert k["kA0"] ** 2 + k["kC0"] ** 2 == pytest.approx(5.0, rel=1e-15)
    assert k["kA1"] + k["kC1"] == pytest.approx(1.25, rel=1e-15)
    assert k["kA1"] ** 2 + k["kC1"] ** 2 == pytest.approx(2.0, rel=1e-15)
    assert k["kA3"] + 0.5 * k["kC3"] == pytest.approx(1.8125, rel=1e-15)
    assert k["kA3"] ** 2 + k["kC3"] ** 2 == pytest.approx(2.75, rel=1e-15)


def diff_form(d, anchor, eps, k):
    """3 (R - s_A) from the differences d of s = 2 f, as the kernels form it."""
    d0, d1, d2, d3, d4 = d
    x = [k["kA0"] * d1 - d0, k["kA1"] * d2 - d1, k["kA0"] * d2 - d3, k["kA3"] * d3 - d4]
    y = [k["kC0"] * d1 - d0, k["kC1"] * d2 - d1, k["kC0"] * d2 - d3, k["kC3"] * d3 - 0.5 * d4]
    b = [x[i] ** 2 + y[i] ** 2 + 6 * eps for i in range(3)]
    bq = x[3] ** 2 + y[3] ** 2 + 1.5 * eps          # the downwind indicator / 4
    b.append(0.25 * (b[0] + b[1] + b[2]) + bq)
    t5 = d0 - 4 * d1 + 6 * d2 - 4 * d3 + d4
    tau = 1.5 * t5 * t5
    if anchor == 2:
        t = [2.5 * d1 - d0, 0.5 * d1 + d2, 2 * d2 - 0.5 * d3, 3 * d2 - 2.5 * d3 + d4]
    else:
        t = [2.5 * d1 - d0 - 3 * d2, 0.5 * d1 - 2 * d2, -d2 - 0.5 * d3, d4 - 2.5 * d3]
    a = np.array([1.0, 9.0, 9.0, 1.0]) * (1 + tau / np.array(b))
    return float(a @ np.array(t) / a.sum()), b, tau, t


def stencils(seed, n):
    rng = np.random.default_rng(seed)
    for i in range(n):
        f = rng.standard_normal(6) * rng.choice([1e-3, 1.0, 1e3])
        if i % 3 == 0:
            f[3:] += rng.choice([-1, 1]) * 10 * abs(f).max()     # a jump inside the stencil
        if i % 5 == 0:
            f[:] = f[0] + 1e-9 * rng.standard_normal(6)           # nearly flat
        yield f


def test_indicators_tau_and_candidates_against_the_oracle():
    k = header_constants()
    for f in stencils(1, 400):
        _, det = orc.recon(f, eps=1e-40, detail=True)
        d = np.diff(2 * f)
        _, b, tau, t = diff_form(d, 2, 0.0, k)
        beta = det["beta"]                       # beta_0, beta_1, beta_2, beta_d, average
        # both sides round differences of values up to |2f| in size: quadratic
        # quantities carry errors of order ulp(|2f|) |d|
        tol = 1e-13 * (6 * beta.max() + np.abs(2 * f).max() * np.abs(d).max())
        for i in range(3):
            assert abs(b[i] - 6 * beta[i]) <= tol
        assert abs(b[3] - 6 * beta[4]) <= tol
        assert abs(tau - 6 * det["tau"]) <= 100 * tol
        s2, s3 = 2 * f[2], 2 * f[3]
        q = det["q"]
        for i in range(4):
            assert abs(t[i] / 3 - (2 * q[i] - s2)) <= 1e-13 * np.abs(2 * f).max()
        _, _, _, t3 = diff_form(d, 3, 0.0, k)
        for i in range(4):
            assert abs(t3[i] / 3 - (2 * q[i] - s3)) <= 1e-13 * np.abs(2 * f).max()


@pytest.mark.parametrize("eps", [1e-40, 1e-6])
def test_split_flux_equals_the_two_reconstructed_halves(eps):
    """g_2 + (X^+ + X^-)/6 with the negative half's differences reversed and
    negated (anchor s^-_2) equals f^+ reconstructed left-biased plus f^-
    reconstructed from the mirrored stencil (eq:LF), both by the oracle."""
    k = header_constants()
    rng = np.random.default_rng(7)
    worst = 0.0
    for f in stencils(3, 300):
        w = rng.standard_normal(6) * np.abs(f).max()
        a = abs(rng.standard_normal()) + 0.1
        fp, fm = 0.5 * (f + a * w), 0.5 * (f - a * w)
        ref = orc.recon(fp, eps=eps) + orc.recon(fm[::-1].copy(), eps=eps)
        dg, dw = np.diff(f), np.diff(w)
        dp = a * dw + dg
        dm = (a * dw - dg)[::-1]
        xp, *_ = diff_form(dp, 2, eps, k)
        xm, *_ = diff_form(dm, 3, eps, k)
        got = f[2] + (xp + xm) / 6
        sc = np.abs(fp).max() + np.abs(fm).max()
        worst = max(worst, abs(got - ref) / sc)
    assert worst < 1e-13, worst
