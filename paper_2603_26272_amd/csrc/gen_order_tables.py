"""Write za_order_tables.hpp: device constants of the order-2r schemes.

Source: the coefficient tables printed in the paper (Section 3 for r = 3,
Appendix A for r = 2, 4, 5), entered below exactly as printed (common
denominators, 'rev' = the reversal operator).  From them this script forms,
in exact rational arithmetic, the factored smoothness indicators the kernels
evaluate:

  beta_k = <f_k, B_k f_k> = g^T C_k g,  g_j = f_{j+1} - f_j  (B_k 1 = 0),
  C_k = L^T B_k L with L the cumulative-sum map,  C_k = U^T diag(lam) U
  (U unit upper triangular), so beta_k = sum_l lam_l (sum_b U_lb g_b)^2:
  a sum of squares of differences, without the cancellation of the expanded
  quadratic form on large, smooth data.

Usage: python gen_order_tables.py   (rewrites za_order_tables.hpp next to it)
"""
import os
from fractions import Fraction as Fr

HERE = os.path.dirname(os.path.abspath(__file__))

# As printed: ck numerators (den), d (den), B numerators (den), c_tau.
PRINTED = {
    2: {"ck_den": 2, "ck": {0: [-1, 3], 1: [1, 1]}, "ck_rev": {2: 0},
        "d_den": 6, "d": [1, 4, 1],
        "B_den": 1, "B": {0: [[1, -1], [-1, 1]], "d": [[1, -1], [-1, 1]]}, "B_rev": {1: 0},
        "ctau": [-1, 3, -3, 1]},
    3: {"ck_den": 6, "ck": {0: [2, -7, 11], 1: [-1, 5, 2], 2: [2, 5, -1], 3: [11, -7, 2]}, "ck_rev": {},
        "d_den": 20, "d": [1, 9, 9, 1],
        "B_den": 6, "B": {0: [[8, -19, 11], [-19, 50, -31], [11, -31, 20]],
                          1: [[8, -13, 5], [-13, 26, -13], [5, -13, 8]],
                          "d": [[44, -73, 29], [-73, 122, -49], [29, -49, 20]]}, "B_rev": {2: 0},
        "ctau": [-1, 5, -10, 10, -5, 1]},
    4: {"ck_den": 12, "ck": {0: [-3, 13, -23, 25], 1: [1, -5, 13, 3], 2: [-1, 7, 7, -1]},
        "ck_rev": {4: 0, 3: 1},
        "d_den": 70, "d": [1, 16, 36, 16, 1],
        "B_den": 240, "B": {
            0: [[547, -1941, 2321, -927], [-1941, 7043, -8623, 3521], [2321, -8623, 11003, -4701],
                [-927, 3521, -4701, 2107]],
            1: [[267, -821, 801, -247], [-821, 2843, -2983, 961], [801, -2983, 3443, -1261],
                [-247, 961, -1261, 547]],
            "d": [[7107, -16901, 13521, -3727], [-16901, 40643, -32863, 9121],
                  [13521, -32863, 26843, -7501], [-3727, 9121, -7501, 2107]]},
        "B_rev": {3: 0, 2: 1},
        "ctau": [-1, 7, -21, 35, -35, 21, -7, 1]},
    5: {"ck_den": 60, "ck": {0: [12, -63, 137, -163, 137], 1: [-3, 17, -43, 77, 12], 2: [2, -13, 47, 27, -3]},
        "ck_rev": {5: 0, 4: 1, 3: 2},
        "d_den": 252, "d": [1, 25, 100, 100, 25, 1],
        "B_den": 10080, "B": {
            0: [[45316, -208501, 364863, -288007, 86329], [-208501, 965926, -1704396, 1358458, -411487],
                [364863, -1704396, 3042786, -2462076, 758823], [-288007, 1358458, -2462076, 2041126, -649501],
                [86329, -411487, 758823, -649501, 215836]],
            1: [[13816, -60871, 99213, -70237, 18079], [-60871, 277126, -464976, 337018, -88297],
                [99213, -464976, 812586, -611976, 165153], [-70237, 337018, -611976, 485446, -140251],
                [18079, -88297, 165153, -140251, 45316]],
            2: [[13816, -51001, 67923, -38947, 8209], [-51001, 209926, -299076, 179098, -38947],
                [67923, -299076, 462306, -299076, 67923], [-38947, 179098, -299076, 209926, -51001],
                [8209, -38947, 67923, -51001, 13816]],
            "d": [[942016, -2964751, 3597813, -2004757, 429679], [-2964751, 9449926, -11584896, 6499258, -1399537],
                  [3597813, -11584896, 14319786, -8079576, 1746873], [-2004757, 6499258, -8079576, 4577926, -992851],
                  [429679, -1399537, 1746873, -992851, 215836]]},
        "B_rev": {4: 0, 3: 1},
        "ctau": [-1, 9, -36, 84, -126, 126, -84, 36, -9, 1]},
}


def tables(r):
    t = PRINTED[r]
    ck = {k: [Fr(n, t["ck_den"]) for n in v] for k, v in t["ck"].items()}
    for k, src in t["ck_rev"].items():
        ck[k] = list(reversed(ck[src]))
    B = {k: [[Fr(n, t["B_den"]) for n in row] for row in v] for k, v in t["B"].items()}
    for k, src in t["B_rev"].items():
        B[k] = [list(reversed(row)) for row in reversed(B[src])]
    Bs = [B[k] for k in range(r)] + [B["d"]]     # index r: downwind polynomial
    return ([ck[k] for k in range(r + 1)], [Fr(n, t["d_den"]) for n in t["d"]],
            [Fr(n) for n in t["ctau"]], Bs)


def factor(B):
    """lam, U with g^T C g = sum_l lam_l (sum_b U[l][b] g_b)^2, C = L^T B L."""
    n = len(B)
    m = n - 1
    # f_j - f_0 = sum_{b < j} g_b: L[j][b] = 1 for b < j (j = 1..n-1)
    C = [[Fr(0)] * m for _ in range(m)]
    for a in range(m):
        for b in range(m):
            C[a][b] = sum(B[i][j] for i in range(a + 1, n) for j in range(b + 1, n))
    lam, U = [], [[Fr(0)] * m for _ in range(m)]
    A = [row[:] for row in C]
    for l in range(m):
        p = A[l][l]
        if p < 0:
            raise ArithmeticError("indicator matrix not positive semidefinite")
        lam.append(p)
        U[l][l] = Fr(1)
        for b in range(l + 1, m):
            U[l][b] = A[l][b] / p if p != 0 else Fr(0)
        for a in range(l + 1, m):
            for b in range(l + 1, m):
                A[a][b] -= (A[a][l] * A[l][b] / p) if p != 0 else 0
    return lam, U


def lit(x):
    x = Fr(x)
    if x.denominator == 1:
        return f"{x.numerator}.0"
    return f"({x.numerator}.0 / {x.denominator}.0)"


def emit(r):
    ck, d, ctau, Bs = tables(r)
    m = r - 1
    fac = [factor(B) for B in Bs]
    out = [f"template <> struct OrderTables<{r}> {{"]
    rows = ", ".join("{" + ", ".join(lit(x) for x in row) + "}" for row in ck)
    out.append(f"  __host__ __device__ static constexpr double ck(int k, int j) {{\n"
               f"    constexpr double t[{r + 1}][{r}] = {{{rows}}};\n    return t[k][j];\n  }}")
    out.append(f"  __host__ __device__ static constexpr double d(int k) {{\n"
               f"    constexpr double t[{r + 1}] = {{{', '.join(lit(x) for x in d)}}};\n    return t[k];\n  }}")
    out.append(f"  __host__ __device__ static constexpr double ctau(int j) {{\n"
               f"    constexpr double t[{2 * r}] = {{{', '.join(lit(x) for x in ctau)}}};\n    return t[j];\n  }}")
    lam_rows = ", ".join("{" + ", ".join(lit(x) for x in lam) + "}" for lam, _ in fac)
    out.append(f"  __host__ __device__ static constexpr double lam(int k, int l) {{\n"
               f"    constexpr double t[{r + 1}][{m}] = {{{lam_rows}}};\n    return t[k][l];\n  }}")
    u_blocks = ", ".join("{" + ", ".join("{" + ", ".join(lit(x) for x in row) + "}" for row in U) + "}"
                         for _, U in fac)
    out.append(f"  __host__ __device__ static constexpr double U(int k, int l, int b) {{\n"
               f"    constexpr double t[{r + 1}][{m}][{m}] = {{{u_blocks}}};\n    return t[k][l][b];\n  }}")
    out.append("};")
    return "\n".join(out)


def main():
    hdr = ["// Generated by gen_order_tables.py from the coefficient tables printed",
           "// in the paper (Section 3: r = 3; Appendix A: r = 2, 4, 5).  Do not edit.",
           "//",
           "// OrderTables<r>: candidate coefficients ck(k, j) on S_k (k = 0..r, k = r",
           "// downwind), ideal weights d(k), c_tau(j) of eq:GSI, and the factored",
           "// indicators: beta_k = sum_l lam(k, l) (sum_{b >= l} U(k, l, b) g_{k+b})^2",
           "// with g_j = f_{j+1} - f_j; k = r gives beta_d (downwind polynomial on I_i).",
           "#pragma once",
           "#include <hip/hip_runtime.h>",
           "",
           "namespace za {",
           "template <int R> struct OrderTables;"]
    body = [emit(r) for r in (2, 3, 4, 5)]
    text = "\n".join(hdr) + "\n" + "\n\n".join(body) + "\n}  // namespace za\n"
    with open(os.path.join(HERE, "za_order_tables.hpp"), "w") as fh:
        fh.write(text)


if __name__ == "__main__":
    main()
