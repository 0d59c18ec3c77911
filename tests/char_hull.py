"""Validity of a WENO flux where the weights are ill conditioned: the
characteristic projection of an interface and the bounds that any convex
combination of the candidate values gives (eq:weights_general; Section 4.2
for the projection).  Test helpers, built on the oracle."""
import numpy as np

import oracle as orc
from paper_2603_26272_amd.problem import PERIODIC


def phys_flux(Q, gamma, d):
    """Euler flux of one cell (conserved variables, m = 3 or 4) in direction d."""
    if len(Q) == 3:
        rho, mx, E = Q
        u = mx / rho
        p = (gamma - 1) * (E - 0.5 * mx * u)
        return np.array([mx, mx * u + p, (E + p) * u])
    rho, mx, my, E = Q
    u, v = mx / rho, my / rho
    p = (gamma - 1) * (E - 0.5 * (mx * u + my * v))
    if d == 0:
        return np.array([mx, mx * u + p, my * u, (E + p) * u])
    return np.array([my, mx * v, my * v + p, (E + p) * v])


def line_cells(P, q, d, line):
    """Cells of one line (row `line` for d = 0, column for d = 1) as [n][m]
    and the ghost rule of that direction."""
    if d == 0:
        cells, bc = q[:, line, :].T, P.bc_x
    else:
        cells, bc = q[:, :, line].T, P.bc_y
    return cells, bc


def hull(P, q, d, line, k, alpha, r):
    """Characteristic projection L of interface k of a line (between cells
    k - 1 and k) and, per field, the bounds of f^+ + f^- over the candidate
    values of the two split stencils (cells k - r .. k + r - 1)."""
    cells, bc = line_cells(P, q, d, line)
    n, m = cells.shape
    idx = (lambda j: j % n) if bc == PERIODIC else (lambda j: min(max(j, 0), n - 1))
    u, v, H, c = orc.roe_state(m, P.gamma, cells[idx(k - 1)], cells[idx(k)])
    _, Lm = orc.euler_eigen(m, d, P.gamma, u, v, H, c)
    st = [cells[idx(j)] for j in range(k - r, k + r)]
    Wc = np.array([Lm @ Q for Q in st])
    Gc = np.array([Lm @ phys_flux(Q, P.gamma, d) for Q in st])
    lo, hi = np.zeros(m), np.zeros(m)
    for s in range(m):
        vp = 0.5 * (Gc[:, s] + alpha[s] * Wc[:, s])
        vm = (0.5 * (Gc[:, s] - alpha[s] * Wc[:, s]))[::-1].copy()
        _, dp = orc.recon_r(r, vp, eps=P.eps, detail=True)
        _, dm = orc.recon_r(r, vm, eps=P.eps, detail=True)
        lo[s] = dp["q"].min() + dm["q"].min()
        hi[s] = dp["q"].max() + dm["q"].max()
    return Lm, lo, hi


def hull_violation(Lm, lo, hi, F):
    """How far L F lies outside [lo, hi], per field, in units of the
    rounding scale of the projection and of the bounds."""
    g = Lm @ F
    tol = 1e-12 * (np.abs(Lm) @ np.abs(F) + np.abs(lo) + np.abs(hi)) + 1e-300
    return np.maximum(lo - g, g - hi) / tol
