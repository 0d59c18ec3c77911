"""Exact rational brute force of one WENO-ZA6 reconstruction, built from the
paper's definitions rather than its printed coefficients:

  * candidate polynomials from the cell-average conditions
    (eq:poly_h_coeffs) on each three-point substencil, evaluated at x_{i+1/2};
  * the six-point central flux from the same conditions on S^6;
  * ideal weights d solving <c_6, f> = <d, q> for every f
    (eq:numerical_flux_FD_linear_comb);
  * smoothness indicators as the integral of eq:SI over I_i;
  * tau as the square of the fifth derivative of the six-point polynomial.

The derived constants must equal the printed ones (Section 3), and the
oracle's per-interface values must match the brute force to 1e-14.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest


def _solve(A, b):
    """Exact Gaussian elimination over the rationals (square, nonsingular)."""
    n = len(A)
    M = [list(A[i]) + [b[i]] for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [M[i][n] / M[i][i] for i in range(n)]


def _fit(offsets, f):
    """Polynomial a_0 + a_1 xi + .. whose cell averages over
    [l - 1/2, l + 1/2] equal f at the given offsets l (dx = 1, x_i = 0)."""
    deg = len(offsets)
    A = [[(Fr(2 * l + 1, 2) ** (n + 1) - Fr(2 * l - 1, 2) ** (n + 1)) / (n + 1) for n in range(deg)]
         for l in offsets]
    return _solve(A, list(f))


def _val(a, x):
    return sum(c * x ** n for n, c in enumerate(a))


def _der(a):
    return [n * a[n] for n in range(1, len(a))]


def _int_sq(a, lo, hi):
    """Exact integral of (sum a_n x^n)^2 over [lo, hi]."""
    sq = {}
    for i, ai in enumerate(a):
        for j, aj in enumerate(a):
            sq[i + j] = sq.get(i + j, 0) + ai * aj
    return sum(c * (hi ** (k + 1) - lo ** (k + 1)) / (k + 1) for k, c in sq.items())


SUB = [[-2, -1, 0], [-1, 0, 1], [0, 1, 2], [1, 2, 3]]   # S_0..S_3 offsets
FULL = [-2, -1, 0, 1, 2, 3]                            # S^6


def brute(v, p=1, eps=Fr(0), linear=False):
    """Everything about one reconstruction from v = (f_{i-2}, .., f_{i+3})."""
    v = [Fr(x) for x in v]
    half = Fr(1, 2)
    q, beta = [], []
    for k, offs in enumerate(SUB):
        a = _fit(offs, v[k:k + 3])
        q.append(_val(a, half))
        b = Fr(0)
        d = a
        for _ in range(2):      # l = 1, 2 (r - 1 = 2)
            d = _der(d)
            b += _int_sq(d, -half, half)
        beta.append(b)
    a6 = _fit(FULL, v)
    central = _val(a6, half)
    tau = (120 * a6[5]) ** 2
    b3 = (beta[0] + beta[1] + beta[2] + beta[3]) / 4
    bk = [beta[0], beta[1], beta[2], b3]
    dk = ideal_weights()
    if linear:
        om = dk
    else:
        al = [dk[k] * (1 + (tau / (bk[k] + eps)) ** p) for k in range(4)]
        s = sum(al)
        om = [x / s for x in al]
    return {"q": q, "beta": beta + [b3], "tau": tau, "omega": om,
            "flux": sum(o * x for o, x in zip(om, q)), "central": central}


def _lin_coeffs(fun, n):
    """Coefficient vector of a linear functional of n inputs."""
    out = []
    for j in range(n):
        e = [Fr(0)] * n
        e[j] = Fr(1)
        out.append(fun(e))
    return out


_D = None


def ideal_weights():
    global _D
    if _D is None:
        # q_k(f) and the central flux as linear functionals of the 6 inputs
        qc = [_lin_coeffs(lambda e, k=k: _val(_fit(SUB[k], e[k:k + 3]), Fr(1, 2)), 6) for k in range(4)]
        c6 = _lin_coeffs(lambda e: _val(_fit(FULL, e), Fr(1, 2)), 6)
        # 6 equations sum_k d_k qc[k][j] = c6[j]; solve with 4, verify all
        rows = [0, 1, 4, 5]
        d = _solve([[qc[k][j] for k in range(4)] for j in rows], [c6[j] for j in rows])
        for j in range(6):
            assert sum(d[k] * qc[k][j] for k in range(4)) == c6[j]
        _D = d
    return _D


def test_derived_constants_equal_printed():
    """Section 3: c_6, c_k, d, B_k, c_tau as printed."""
    c6 = _lin_coeffs(lambda e: _val(_fit(FULL, e), Fr(1, 2)), 6)
    assert c6 == [Fr(x, 60) for x in (1, -8, 37, 37, -8, 1)]
    printed_ck = [(2, -7, 11), (-1, 5, 2), (2, 5, -1), (11, -7, 2)]
    for k in range(4):
        ck = _lin_coeffs(lambda e, k=k: _val(_fit(SUB[k], e), Fr(1, 2)), 3)
        assert ck == [Fr(x, 6) for x in printed_ck[k]]
    assert ideal_weights() == [Fr(1, 20), Fr(9, 20), Fr(9, 20), Fr(1, 20)]
    # d_k = C(r,k)^2 / C(2r,r) for r = 3
    from math import comb
    assert ideal_weights() == [Fr(comb(3, k) ** 2, comb(6, 3)) for k in range(4)]
    ctau = _lin_coeffs(lambda e: 120 * _fit(FULL, e)[5], 6)
    assert ctau == [-1, 5, -10, 10, -5, 1]


PRINTED_B = {
    0: [[8, -19, 11], [-19, 50, -31], [11, -31, 20]],
    1: [[8, -13, 5], [-13, 26, -13], [5, -13, 8]],
    3: [[44, -73, 29], [-73, 122, -49], [29, -49, 20]],  # B_d
}


def test_printed_smoothness_matrices():
    """beta_k = <f_k, B_k f_k> with the printed matrices (eq:SI_S6), B_2 =
    rev(B_0), equals the integral definition eq:SI for arbitrary data."""
    rng = np.random.default_rng(7)
    B = dict(PRINTED_B)
    B[2] = [row[::-1] for row in PRINTED_B[0][::-1]]
    for _ in range(20):
        v = [Fr(int(x), 7) for x in rng.integers(-50, 50, size=6)]
        b = brute(v)["beta"]
        for k in range(4):
            fk = v[k:k + 3]
            quad = sum(Fr(B[k][i][j], 6) * fk[i] * fk[j] for i in range(3) for j in range(3))
            assert quad == b[k]


def _cases():
    rng = np.random.default_rng(2603)
    cases = [rng.normal(size=6) for _ in range(40)]
    cases += [np.where(np.arange(6) < j, 1.0, 0.0) + 0.01 * rng.normal(size=6) for j in range(1, 6)]
    cases += [np.sin(0.3 * np.arange(6) + 0.2), np.arange(6.0) ** 2, np.full(6, 0.7)]
    cases += [np.array([1.0, 1.0, 1.0, 0.1, 0.1, 0.1]), np.array([0.0, 0, 0, 0, 1.0, 1.0])]
    return cases


@pytest.mark.parametrize("ai", [0])
def test_oracle_matches_bruteforce(orc, ai):
    eps = 1e-40
    for v in _cases():
        r, det = orc.recon(v, p=1.0, eps=eps, ai=ai, detail=True)
        b = brute(v, p=1, eps=Fr(eps))
        scale = max(abs(x) for x in v) + 1e-300
        for k in range(4):
            assert abs(det["q"][k] - float(b["q"][k])) <= 1e-14 * scale
        bscale = float(max(b["beta"])) + 1e-300
        for k in range(5):
            assert abs(det["beta"][k] - float(b["beta"][k])) <= 1e-13 * bscale
        assert abs(det["tau"] - float(b["tau"])) <= 1e-12 * (float(b["tau"]) + 1e-14 * scale ** 2)
        assert abs(r - float(b["flux"])) <= 1e-14 * scale, (v, r, float(b["flux"]))


def test_oracle_linear_mode_is_central_flux(orc):
    for v in _cases():
        r = orc.recon(v, linear=1)
        b = brute(v, linear=True)
        assert b["flux"] == b["central"]              # <d, q> = <c_6, f> exactly
        assert abs(r - float(b["central"])) <= 1e-15 * (max(abs(x) for x in v) + 1e-300)


def test_oracle_p32_matches_bruteforce(orc):
    """p = 3/2 (tab:ncp1): compare with the brute force in high precision."""
    import mpmath as mp
    mp.mp.dps = 40
    for v in _cases()[:20]:
        b = brute(v, p=1, eps=Fr(1e-40))
        dk = ideal_weights()
        bk = [b["beta"][0], b["beta"][1], b["beta"][2], b["beta"][4]]
        al = [mp.mpf(dk[k].numerator) / dk[k].denominator *
              (1 + (mp.mpf(b["tau"].numerator) / b["tau"].denominator /
                    (mp.mpf(bk[k].numerator) / bk[k].denominator + mp.mpf(1e-40))) ** mp.mpf(1.5))
              for k in range(4)]
        fl = sum(a * (mp.mpf(x.numerator) / x.denominator) for a, x in zip(al, b["q"])) / sum(al)
        r = orc.recon(v, p=1.5, eps=1e-40)
        assert abs(r - float(fl)) <= 1e-14 * (max(abs(x) for x in v) + 1e-300)


def test_quad_recon_matches_bruteforce(orc):
    """The quad build agrees with exact arithmetic far below FP64 rounding."""
    v = [Fr(1, 3), Fr(2, 7), Fr(-5, 11), Fr(3, 13), Fr(1, 17), Fr(-2, 19)]
    b = brute(v, p=1, eps=Fr(0))
    import mpmath as mp
    mp.mp.dps = 40
    strs = [mp.nstr(mp.mpf(x.numerator) / x.denominator, 38) for x in v]
    got = mp.mpf(orc.recon_quad(strs, eps=0.0))
    exact = mp.mpf(b["flux"].numerator) / b["flux"].denominator
    assert abs(got - exact) <= mp.mpf(10) ** -31 * abs(exact)


def test_mirror_rule_reverses_stencil(orc):
    """f^-_{i+1/2} is the positive reconstruction applied to the mirrored
    stencil (f^-_{i+3}, .., f^-_{i-2}): a linear ramp reconstructs to the
    interface value from both sides."""
    v = np.arange(6.0) * 0.25 + 1.0          # f(x) = 1 + x/4 on nodes i-2..i+3
    exact = 1.0 + 0.25 * 2.5                 # h at x_{i+1/2} (linear: h = f)
    assert abs(orc.recon(v) - exact) < 1e-14
    assert abs(orc.recon(v[::-1]) - exact) < 1e-14
