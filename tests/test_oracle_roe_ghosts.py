"""Pins of two oracle steps that the paper leaves to the reader: the average
state whose eigenvectors the characteristic-wise splitting projects with
(Section 4.2 names the splitting, not the average; the Roe average is the
reading), and the transmissive ghost cells of the Euler workloads.

* The Roe state Q~ is defined by A(Q~)(Q_R - Q_L) = F(Q_R) - F(Q_L), with
  A = R diag(lambda) L.  The test rebuilds A from the oracle's own Roe state
  and eigenvectors and checks the jump condition on random admissible pairs,
  in 1D and in both directions of a 2D sweep.  The arithmetic mean and the
  Roe weights swapped are computed here as negative controls: both must fail
  the same check, so the check can tell the Roe average from them.
* Transmissive ghosts are zero-gradient copies, Q_{-k} = Q_0 and
  Q_{n-1+k} = Q_{n-1}.  The test pads the data by hand (numpy's edge mode)
  and evaluates every interface of a line from the pinned single-interface
  pieces: one split reconstruction (orc.recon), the Roe state and the
  eigenvectors.  The oracle's full sweep must agree on data that vary right
  up to the boundary.
"""
import numpy as np
import pytest

from paper_2603_26272_amd import workloads as W
from paper_2603_26272_amd.problem import (BURGERS, EULER, PERIODIC, TRANSMISSIVE, Problem)

GAMMA = 1.4


def _flux(Q, direction, gamma=GAMMA):
    """Physical flux of the Euler equations from its definition (m = 3 or 4)."""
    m = len(Q)
    rho = Q[0]
    u = Q[1] / rho
    if m == 3:
        p = (gamma - 1) * (Q[2] - 0.5 * rho * u * u)
        return np.array([Q[1], Q[1] * u + p, (Q[2] + p) * u])
    v = Q[2] / rho
    p = (gamma - 1) * (Q[3] - 0.5 * rho * (u * u + v * v))
    un = u if direction == 0 else v
    return np.array([rho * un, Q[1] * un + (p if direction == 0 else 0.0),
                     Q[2] * un + (p if direction == 1 else 0.0), (Q[3] + p) * un])


def _cons(rho, u, v, p, m, gamma=GAMMA):
    if m == 3:
        return np.array([rho, rho * u, p / (gamma - 1) + 0.5 * rho * u * u])
    return np.array([rho, rho * u, rho * v, p / (gamma - 1) + 0.5 * rho * (u * u + v * v)])


def _primitive_H(Q, gamma=GAMMA):
    m = len(Q)
    rho = Q[0]
    u = Q[1] / rho
    v = Q[2] / rho if m == 4 else 0.0
    p = (gamma - 1) * (Q[-1] - 0.5 * rho * (u * u + v * v))
    return u, v, (Q[-1] + p) / rho


def _jump_residual(orc, m, direction, state, QL, QR, gamma=GAMMA):
    """|R diag(lambda) L (Q_R - Q_L) - (F_R - F_L)|_inf / |F|_inf at the
    average state (u, v, H); c from the state's own enthalpy."""
    u, v, H = state
    q2 = 0.5 * (u * u + v * v) if m == 4 else 0.5 * u * u
    c = np.sqrt((gamma - 1) * (H - q2))
    Rm, Lm = orc.euler_eigen(m, direction, gamma, u, v, H, c)
    un = u if direction == 0 else v
    lam = np.array([un - c, un, un + c] if m == 3 else [un - c, un, un, un + c])
    dF = Rm @ (lam * (Lm @ (QR - QL)))
    FL, FR = _flux(QL, direction, gamma), _flux(QR, direction, gamma)
    scale = max(np.abs(FL).max(), np.abs(FR).max())
    return np.abs(dF - (FR - FL)).max() / scale


def _random_pairs(seed, m, n=200):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        s = [(rng.uniform(0.1, 2.0), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.1, 2.0))
             for _ in range(2)]
        out.append((_cons(*s[0], m), _cons(*s[1], m)))
    return out


@pytest.mark.parametrize("m,direction", [(3, 0), (4, 0), (4, 1)])
def test_roe_state_satisfies_the_jump_condition(orc, m, direction):
    worst = 0.0
    for QL, QR in _random_pairs(7 + m + direction, m):
        u, v, H, c = orc.roe_state(m, GAMMA, QL, QR)
        # the returned sound speed is the one the state's enthalpy implies
        q2 = 0.5 * (u * u + v * v)
        assert abs(c * c - (GAMMA - 1) * (H - q2)) <= 1e-14 * c * c
        if m == 3:
            assert v == 0.0
        worst = max(worst, _jump_residual(orc, m, direction, (u, v, H), QL, QR))
    assert worst <= 1e-13, worst


@pytest.mark.parametrize("m,direction", [(3, 0), (4, 0), (4, 1)])
def test_other_averages_fail_the_jump_condition(orc, m, direction):
    """Negative controls: the arithmetic mean of (u, v, H) and the Roe
    weights swapped violate the jump condition by orders of magnitude more
    than the tolerance the Roe state meets."""
    mean_res, swap_res = [], []
    for QL, QR in _random_pairs(70 + m + direction, m, n=50):
        uL, vL, HL = _primitive_H(QL)
        uR, vR, HR = _primitive_H(QR)
        mean_res.append(_jump_residual(orc, m, direction, (0.5 * (uL + uR), 0.5 * (vL + vR), 0.5 * (HL + HR)),
                                       QL, QR))
        sl, sr = np.sqrt(QL[0]), np.sqrt(QR[0])
        wl, wr = sr / (sl + sr), sl / (sl + sr)
        swap_res.append(_jump_residual(orc, m, direction, (wl * uL + wr * uR, wl * vL + wr * vR, wl * HL + wr * HR),
                                       QL, QR))
    assert np.median(mean_res) > 1e-4 and np.median(swap_res) > 1e-4, (np.median(mean_res), np.median(swap_res))


def test_roe_state_of_equal_cells_is_the_cell(orc):
    Q = _cons(0.7, 0.3, -0.2, 1.1, 4)
    u, v, H, c = orc.roe_state(4, GAMMA, Q, Q)
    uu, vv, HH = _primitive_H(Q)
    assert abs(u - uu) <= 1e-16 and abs(v - vv) <= 1e-16 and abs(H - HH) <= 1e-15 * HH
    p = 0.4 * (Q[3] - 0.5 * Q[0] * (uu * uu + vv * vv))
    assert abs(c - np.sqrt(GAMMA * p / Q[0])) <= 1e-14


# ---------------------------------------------------------------------------
# transmissive ghosts
# ---------------------------------------------------------------------------
def _scalar_line_fluxes(orc, u, alpha, f):
    """Every interface flux of a padded scalar line (3 ghosts per side) from
    one split reconstruction per half: F = R(f+) + R(f- mirrored)."""
    n = len(u) - 6
    fp = 0.5 * (f + alpha * u)
    fm = 0.5 * (f - alpha * u)
    out = np.zeros(n + 1)
    for k in range(n + 1):        # interface between cells k-1 and k
        j = k + 3                 # padded index of cell k
        out[k] = orc.recon(fp[j - 3:j + 3]) + orc.recon(fm[j - 3:j + 3][::-1])
    return out


def _euler_line_fluxes(orc, Q, alpha, direction, gamma=GAMMA):
    """Every interface flux of a padded Euler line Q[m][n+6] by the
    characteristic-wise splitting: Roe state of the two cells, project the
    six-point stencil of Q and F, split with the per-field speeds, one
    reconstruction per half and field, project back."""
    m, npad = Q.shape
    n = npad - 6
    F = np.stack([_flux(Q[:, j], direction, gamma) for j in range(npad)], axis=1)
    out = np.zeros((m, n + 1))
    for k in range(n + 1):
        j = k + 3
        u, v, H, c = orc.roe_state(m, gamma, Q[:, j - 1], Q[:, j])
        Rm, Lm = orc.euler_eigen(m, direction, gamma, u, v, H, c)
        Wc = Lm @ Q[:, j - 3:j + 3]
        Gc = Lm @ F[:, j - 3:j + 3]
        gh = np.zeros(m)
        for s in range(m):
            fp = 0.5 * (Gc[s] + alpha[s] * Wc[s])
            fm = 0.5 * (Gc[s] - alpha[s] * Wc[s])
            gh[s] = orc.recon(fp) + orc.recon(fm[::-1])
        out[:, k] = Rm @ gh
    return out


def test_transmissive_ghosts_scalar(orc):
    """Burgers data with a jump next to each end and a slope at the ends."""
    n = 40
    x = W.centres(n, 0.0, 1.0)
    rng = np.random.default_rng(3)
    u = 0.5 + 0.6 * x + 0.1 * rng.standard_normal(n)
    u[1] += 0.8
    u[-2] -= 0.7
    P = Problem(dim=1, system=BURGERS, nx=n, ny=1, bc_x=TRANSMISSIVE)
    fx, _, st = orc.fluxes(P, u.reshape(1, 1, n))
    assert st == 0
    up = np.pad(u, 3, mode="edge")
    alpha = np.abs(u).max()                    # max |f'(u)| over the cells
    ref = _scalar_line_fluxes(orc, up, alpha, 0.5 * up * up)
    assert np.array_equal(fx[0, 0], ref)
    # the ghost rule matters: periodic or mirrored ghosts change the end fluxes
    for wrong in (np.pad(u, 3, mode="wrap"), np.pad(u, 3, mode="symmetric")):
        bad = _scalar_line_fluxes(orc, wrong, alpha, 0.5 * wrong * wrong)
        assert np.abs(bad - ref)[[0, 1, 2, -3, -2, -1]].max() > 1e-3


def test_transmissive_ghosts_euler_1d(orc):
    n = 32
    rng = np.random.default_rng(11)
    rho = rng.uniform(0.3, 1.2, n)
    u = rng.uniform(-0.5, 0.5, n)
    p = rng.uniform(0.3, 1.2, n)
    q = np.stack([rho, rho * u, p / 0.4 + 0.5 * rho * u * u]).reshape(3, 1, n)
    P = Problem(dim=1, system=EULER, nx=n, ny=1, bc_x=TRANSMISSIVE)
    fx, _, st = orc.fluxes(P, q)
    assert st == 0
    a, _, _ = orc.wave_speeds(P, q)
    alpha = a[0][:3]     # 1D: (|u - c|, |u|, |u + c|) maxima
    ref = _euler_line_fluxes(orc, np.pad(q[:, 0, :], ((0, 0), (3, 3)), mode="edge"), alpha, 0)
    scale = np.abs(ref).max(axis=1, keepdims=True)
    assert np.all(np.abs(fx[:, 0, :] - ref) <= 1e-13 * (np.abs(ref) + scale))


@pytest.mark.parametrize("bc", [TRANSMISSIVE, PERIODIC])
def test_ghosts_euler_2d_both_directions(orc, bc):
    """Rows (x-sweep) and columns (y-sweep) of random 2D data against the
    hand-padded composition; periodic ghosts as a second rule."""
    nx, ny = 14, 11
    rng = np.random.default_rng(5)
    rho = rng.uniform(0.3, 1.2, (ny, nx))
    u = rng.uniform(-0.5, 0.5, (ny, nx))
    v = rng.uniform(-0.5, 0.5, (ny, nx))
    p = rng.uniform(0.3, 1.2, (ny, nx))
    q = np.stack([rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v)])
    P = Problem(dim=2, system=EULER, nx=nx, ny=ny, bc_x=bc, bc_y=bc)
    fx, fy, st = orc.fluxes(P, q)
    assert st == 0
    a, _, _ = orc.wave_speeds(P, q)
    mode = "edge" if bc == TRANSMISSIVE else "wrap"
    for y in (0, 5, ny - 1):
        ref = _euler_line_fluxes(orc, np.pad(q[:, y, :], ((0, 0), (3, 3)), mode=mode), a[0], 0)
        scale = np.abs(ref).max(axis=1, keepdims=True)
        assert np.all(np.abs(fx[:, y, :] - ref) <= 1e-13 * (np.abs(ref) + scale)), y
    for x in (0, 6, nx - 1):
        ref = _euler_line_fluxes(orc, np.pad(q[:, :, x], ((0, 0), (3, 3)), mode=mode), a[1], 1)
        scale = np.abs(ref).max(axis=1, keepdims=True)
        assert np.all(np.abs(fy[:, :, x] - ref) <= 1e-13 * (np.abs(ref) + scale)), x
