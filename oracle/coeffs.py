"""Exact coefficients of the even-order central-upwind WENO schemes.

Test infrastructure (oracle side).  Everything is derived from the
definitions, in exact rational arithmetic, for any r >= 2 (order 2r):

* Point values f_j are read as cell averages of a function h over the cells
  [x_j - dx/2, x_j + dx/2]; the numerical flux at x_{i+1/2} is the value there
  of the polynomial with those averages (Section 2, eq:numerical_flux_FD_plus
  and eq:numerical_subflux).  With dx = 1 and x_i = 0 cell o spans
  [o - 1/2, o + 1/2].
* Big stencil S^{2r}: cells i-r+1 .. i+r -> c_{2r}.  Substencils S_k, k = 0..r:
  cells i-r+1+k .. i+k (r cells); S_0 .. S_{r-1} are upwind, S_r is the
  downwind one -> c_k.
* Ideal weights d: sum_k d_k c_k (placed in the big stencil) = c_{2r}
  (eq:numerical_flux_FD_linear_comb).
* Smoothness indicator of a substencil polynomial p (eq:SI with dx = 1):
  beta = sum_{l=1}^{r-1} int_{-1/2}^{1/2} (d^l p / dx^l)^2 dx, over I_i for
  every substencil, the downwind one included (beta_d); the downwind weight
  uses the mean of beta_0..beta_{r-1} and beta_d (eq:SI_downwind).
* Global indicator tau = <c_tau, f>^2 with c_tau the (2r-1)-th difference
  (eq:GSI).

`tables(r)` returns these as Fractions; `derivative_maps(r)` gives, per
substencil, the linear maps f -> coefficients of p^(l), which the C oracle
uses to evaluate beta as the defining integral (a sum of products of
derivative coefficients, free of the cancellation the expanded quadratic
form suffers for large, smooth f).
"""
from fractions import Fraction as Fr
from math import comb, factorial


def _avg_moment(o, m):
    """Average of xi^m over the cell [o - 1/2, o + 1/2]."""
    a, b = Fr(2 * o - 1, 2), Fr(2 * o + 1, 2)
    return (b ** (m + 1) - a ** (m + 1)) / (m + 1)


def _inverse(M):
    """Exact inverse of a square matrix of Fractions (Gauss-Jordan)."""
    n = len(M)
    A = [list(row) + [Fr(int(i == j)) for j in range(n)] for i, row in enumerate(M)]
    for col in range(n):
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        p = A[col][col]
        A[col] = [x / p for x in A[col]]
        for r in range(n):
            if r != col and A[r][col] != 0:
                f = A[r][col]
                A[r] = [x - f * y for x, y in zip(A[r], A[col])]
    return [row[n:] for row in A]


def poly_map(offsets):
    """P[m][j]: coefficient of xi^m of the polynomial whose averages over the
    cells `offsets` are f_j, as a linear map of f."""
    n = len(offsets)
    M = [[_avg_moment(o, m) for m in range(n)] for o in offsets]   # M a = f
    return _inverse(M)


def eval_at(P, x):
    n = len(P)
    return [sum(P[m][j] * x ** m for m in range(n)) for j in range(n)]


def deriv_map(P, l):
    """D[m][j]: coefficient of xi^m of p^(l) as a linear map of f."""
    n = len(P)
    return [[P[m + l][j] * Fr(factorial(m + l), factorial(m)) for j in range(n)] for m in range(n - l)]


def interval_moment(s):
    """int_{-1/2}^{1/2} xi^s dxi."""
    return Fr(0) if s % 2 else Fr(2, s + 1) * Fr(1, 2) ** (s + 1)


def indicator_matrix(P):
    """B with beta = f^T B f = sum_l int_{-1/2}^{1/2} (p^(l))^2."""
    n = len(P)
    B = [[Fr(0)] * n for _ in range(n)]
    for l in range(1, n):
        D = deriv_map(P, l)
        for a in range(len(D)):
            for b in range(len(D)):
                w = interval_moment(a + b)
                if w == 0:
                    continue
                for i in range(n):
                    if D[a][i] == 0:
                        continue
                    for j in range(n):
                        B[i][j] += w * D[a][i] * D[b][j]
    return B


def substencil_offsets(r, k):
    return list(range(-r + 1 + k, k + 1))


def _solve_ideal_weights(r, ck, c2r):
    """d with sum_k d_k ck (shifted by k into the big stencil) = c2r; the
    system has 2r equations for r+1 unknowns and must be consistent."""
    rows = []
    for j in range(2 * r):
        rows.append([ck[k][j - k] if 0 <= j - k < r else Fr(0) for k in range(r + 1)])
    # normal equations (exact), then check every equation
    n = r + 1
    AtA = [[sum(rows[j][a] * rows[j][b] for j in range(2 * r)) for b in range(n)] for a in range(n)]
    Atb = [sum(rows[j][a] * c2r[j] for j in range(2 * r)) for a in range(n)]
    inv = _inverse(AtA)
    d = [sum(inv[a][b] * Atb[b] for b in range(n)) for a in range(n)]
    for j in range(2 * r):
        if sum(rows[j][k] * d[k] for k in range(n)) != c2r[j]:
            raise ArithmeticError("ideal weights do not reproduce c_2r")
    return d


def tables(r):
    """Exact tables of the order-2r scheme: dict with c2r, ck, d, B (upwind
    k = 0..r-1), Bd (downwind polynomial over I_i), ctau."""
    if r < 2:
        raise ValueError("r >= 2")
    big = list(range(-r + 1, r + 1))
    c2r = eval_at(poly_map(big), Fr(1, 2))
    ck, B = [], []
    for k in range(r + 1):
        P = poly_map(substencil_offsets(r, k))
        ck.append(eval_at(P, Fr(1, 2)))
        B.append(indicator_matrix(P))
    d = _solve_ideal_weights(r, ck, c2r)
    ctau = [Fr((-1) ** (2 * r - 1 - j) * comb(2 * r - 1, j)) for j in range(2 * r)]
    return {"r": r, "c2r": c2r, "ck": ck, "d": d, "B": B[:r], "Bd": B[r], "ctau": ctau}


def derivative_maps(r):
    """Per substencil k = 0..r (k = r: downwind), the maps D_l (l = 1..r-1)."""
    out = []
    for k in range(r + 1):
        P = poly_map(substencil_offsets(r, k))
        out.append([deriv_map(P, l) for l in range(1, r)])
    return out


def flat_rationals(r):
    """The C oracle's table layout for order 2r, as (numerator, denominator)
    pairs: ck[(r+1) r], d[r+1], ctau[2r], then for k = 0..r and l = 1..r-1
    the derivative map D_{k,l} [(r-l) r], then the moments I_s, s = 0..2r-4."""
    t = tables(r)
    D = derivative_maps(r)
    vals = []
    for k in range(r + 1):
        vals += t["ck"][k]
    vals += t["d"]
    vals += t["ctau"]
    for k in range(r + 1):
        for l in range(1, r):
            for row in D[k][l - 1]:
                vals += row
    vals += [interval_moment(s) for s in range(2 * r - 3)]
    return [(v.numerator, v.denominator) for v in vals]
