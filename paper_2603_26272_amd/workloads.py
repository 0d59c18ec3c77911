"""Seeded synthetic inputs (initial data) for the WENO-ZA6 workloads.

This module only draws and lays out initial conditions; it holds none of the
scheme's arithmetic.  Every generator is deterministic for a given seed
(numpy PCG64 via ``default_rng``) and returns ``(Problem, q0)`` with q0 a
float64 array in SoA layout [m][ny][nx] of point values at cell centres.

Workloads (the paper has no datasets: all of its tests use analytic initial
data, and these generators stand in for them):
  * ``advection_sine``   - u_t + u_x = 0 on periodic [-1, 1], u0 = sin(pi x),
                           dt = 0.5 dx^2 (time error below the sixth-order
                           spatial error).
  * ``riemann_1d``       - 1D Euler, 1-3 random Riemann discontinuities plus a
                           smooth density perturbation on one side.
  * ``quadrants_2d``     - 2D Euler four-quadrant Riemann data with a random
                           corner (the shape of the paper's 2D Riemann tests).
  * ``smooth_wave_2d``   - 2D Euler density wave sin(2 pi (x + y)), periodic.
  * ``entropy_wave_1d``  - 1D Euler density wave, periodic.
  * ``shock_tube``       - Sod / Lax / 123 tubes of the paper's 1D table.
  * ``riemann_config3``  - the paper's 2D Riemann configuration 3.
  * ``multiwave``        - u_t + u_x = 0 with the Gaussian / square / triangle /
                           semi-ellipse initial data of Section 4.1 (N = 400,
                           T = 20 on periodic [-1, 1]).
  * ``burgers_sine``     - Burgers u0 = 1/2 + sin(2 pi x) (tab:scalar_fluxes).
  * ``buckley_step``     - Buckley-Leverett step data (tab:scalar_fluxes).
  * ``vacuum_tube``, ``leblanc``, ``vacuum_quadrants_2d`` - near-vacuum
                           Euler data for the positivity-preserving limiter.
  * ``serving_stream``   - a Poisson stream of mixed 1D / 2D solve requests.
"""
import math
from dataclasses import dataclass
from typing import List, Optional, Tuple

import numpy as np

from .problem import (ADVECTION, BUCKLEY, BURGERS, DT_CFL, DT_CFL_H2, EULER, FP32_RECON, FP64,
                      PERIODIC, TRANSMISSIVE, Problem)

GAMMA = 1.4


def conservative(rho, u, v, p, gamma=GAMMA, dim=2):
    """Primitive -> conservative point values (equation of state of the
    Euler equations: E = p/(gamma-1) + rho |u|^2 / 2)."""
    rho = np.asarray(rho, dtype=np.float64)
    u = np.broadcast_to(np.asarray(u, dtype=np.float64), rho.shape)
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), rho.shape)
    if dim == 1:
        E = p / (gamma - 1.0) + 0.5 * rho * u * u
        return np.stack([rho, rho * u, E])
    v = np.broadcast_to(np.asarray(v, dtype=np.float64), rho.shape)
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.stack([rho, rho * u, rho * v, E])


def centres(n, lo, hi):
    h = (hi - lo) / n
    return lo + (np.arange(n) + 0.5) * h


def _sound(rho, p, gamma=GAMMA):
    return math.sqrt(gamma * p / rho)


def _near_vacuum(rl, ul, pl, rr, ur, pr, gamma=GAMMA) -> bool:
    """Reject pairs whose normal-velocity jump reaches half the vacuum
    threshold 2 (c_L + c_R) / (gamma - 1)."""
    return (ur - ul) >= 0.5 * 2.0 * (_sound(rl, pl) + _sound(rr, pr)) / (gamma - 1.0)


# --------------------------------------------------------------------------
def advection_sine(N: int = 200) -> Tuple[Problem, np.ndarray]:
    P = Problem(dim=1, system=ADVECTION, nx=N, ny=1, xlo=-1.0, xhi=1.0, bc_x=PERIODIC,
                adv_speed=(1.0, 0.0), cfl=0.5, dt_rule=DT_CFL_H2)
    x = centres(N, -1.0, 1.0)
    return P, np.sin(np.pi * x).reshape(1, 1, N)


def riemann_1d(seed: int, N: int = 4096, stats: Optional[dict] = None) -> Tuple[Problem, np.ndarray]:
    rng = np.random.default_rng(seed)
    K = int(rng.integers(1, 4))
    while True:
        pos = np.sort(rng.uniform(0.1, 0.9, size=K))
        if K == 1 or np.min(np.diff(pos)) >= 0.05:
            break
    rejections = 0
    while True:
        rho = rng.uniform(0.1, 1.0, size=K + 1)
        u = rng.uniform(-1.0, 1.0, size=K + 1)
        p = rng.uniform(0.1, 1.0, size=K + 1)
        if not any(_near_vacuum(rho[i], u[i], p[i], rho[i + 1], u[i + 1], p[i + 1]) for i in range(K)):
            break
        rejections += 1
    k = int(rng.integers(1, 9))
    left_side = bool(rng.integers(0, 2))
    x = centres(N, 0.0, 1.0)
    seg = np.searchsorted(pos, x)          # state index of each cell
    r = rho[seg]
    pert = 1.0 + 0.2 * np.sin(2.0 * np.pi * k * x)
    mask = (x < pos[0]) if left_side else (x > pos[-1])
    r = np.where(mask, r * pert, r)
    q = conservative(r, u[seg], 0.0, p[seg], dim=1)
    if stats is not None:
        stats.update(K=K, positions=pos.tolist(), k=k, left=left_side, rejections=rejections)
    P = Problem(dim=1, system=EULER, nx=N, ny=1, xlo=0.0, xhi=1.0, bc_x=TRANSMISSIVE, cfl=0.5)
    return P, q.reshape(3, 1, N)


def quadrants_2d(seed: int, n: int = 2048, ny: Optional[int] = None,
                 stats: Optional[dict] = None) -> Tuple[Problem, np.ndarray]:
    ny = n if ny is None else ny
    rng = np.random.default_rng(seed)
    cx, cy = 0.5 + rng.uniform(-0.1, 0.1, size=2)
    rejections = 0
    while True:
        rho = rng.uniform(0.1, 1.5, size=4)
        p = rng.uniform(0.1, 1.5, size=4)
        u = rng.uniform(-0.8, 0.8, size=4)
        v = rng.uniform(-0.8, 0.8, size=4)
        # quadrants: 0 NE, 1 NW, 2 SW, 3 SE
        pairs_x = [(1, 0), (2, 3)]     # (left, right)
        pairs_y = [(2, 1), (3, 0)]     # (bottom, top)
        bad = any(_near_vacuum(rho[a], u[a], p[a], rho[b], u[b], p[b]) for a, b in pairs_x)
        bad = bad or any(_near_vacuum(rho[a], v[a], p[a], rho[b], v[b], p[b]) for a, b in pairs_y)
        if not bad:
            break
        rejections += 1
    x = centres(n, 0.0, 1.0)[None, :]
    y = centres(ny, 0.0, 1.0)[:, None]
    east = x > cx
    north = y > cy
    quad = np.where(north, np.where(east, 0, 1), np.where(east, 3, 2))
    q = conservative(rho[quad], u[quad], v[quad], p[quad], dim=2)
    if stats is not None:
        stats.update(corner=(float(cx), float(cy)), rejections=rejections)
    P = Problem(dim=2, system=EULER, nx=n, ny=ny, bc_x=TRANSMISSIVE, bc_y=TRANSMISSIVE, cfl=0.5)
    return P, np.ascontiguousarray(q)


def smooth_wave_2d(n: int) -> Tuple[Problem, np.ndarray]:
    x = centres(n, 0.0, 1.0)[None, :]
    y = centres(n, 0.0, 1.0)[:, None]
    rho = 1.0 + 0.2 * np.sin(2.0 * np.pi * (x + y))
    q = conservative(rho, 1.0, 1.0, 1.0, dim=2)
    P = Problem(dim=2, system=EULER, nx=n, ny=n, bc_x=PERIODIC, bc_y=PERIODIC, cfl=0.5,
                dt_rule=DT_CFL_H2)
    return P, np.ascontiguousarray(q)


def smooth_wave_2d_exact(n: int, t: float) -> np.ndarray:
    x = centres(n, 0.0, 1.0)[None, :]
    y = centres(n, 0.0, 1.0)[:, None]
    return 1.0 + 0.2 * np.sin(2.0 * np.pi * ((x - t) + (y - t)))


def entropy_wave_1d(N: int) -> Tuple[Problem, np.ndarray]:
    x = centres(N, 0.0, 1.0)
    rho = 1.0 + 0.2 * np.sin(2.0 * np.pi * x)
    q = conservative(rho, 1.0, 0.0, 1.0, dim=1)
    P = Problem(dim=1, system=EULER, nx=N, ny=1, bc_x=PERIODIC, cfl=0.5, dt_rule=DT_CFL_H2)
    return P, q.reshape(3, 1, N)


# Shock tubes of the paper's 1D Riemann table, on [-5, 5] with the jump at x = 0.
SHOCK_TUBES = {
    "sod": ((0.125, 0.0, 0.1), (1.0, 0.0, 1.0), 2.0),
    "lax": ((0.445, 0.698, 3.528), (0.5, 0.0, 0.571), 1.3),
    "123": ((1.0, -2.0, 0.4), (1.0, 2.0, 0.4), 1.0),
}


def shock_tube(name: str, N: int = 200):
    (rl, ul, pl), (rr, ur, pr), T = SHOCK_TUBES[name]
    x = centres(N, -5.0, 5.0)
    left = x < 0.0
    q = conservative(np.where(left, rl, rr), np.where(left, ul, ur), 0.0,
                     np.where(left, pl, pr), dim=1)
    P = Problem(dim=1, system=EULER, nx=N, ny=1, xlo=-5.0, xhi=5.0, bc_x=TRANSMISSIVE, cfl=0.45)
    return P, q.reshape(3, 1, N), T


def riemann_config3(n: int = 400):
    """2D Riemann configuration 3 on [0,1]^2, quadrants split at 0.8."""
    x = centres(n, 0.0, 1.0)[None, :]
    y = centres(n, 0.0, 1.0)[:, None]
    east = x > 0.8
    north = y > 0.8
    states = {  # rho, u, v, p
        (1, 1): (1.5, 0.0, 0.0, 1.5),
        (0, 1): (0.5323, 1.206, 0.0, 0.3),
        (0, 0): (0.138, 1.206, 1.206, 0.029),
        (1, 0): (0.5323, 0.0, 1.206, 0.3),
    }
    prim = np.zeros((4, n, n))
    for (e, nn), s in states.items():
        msk = (east == bool(e)) & (north == bool(nn))
        for c in range(4):
            prim[c][msk] = s[c]
    q = conservative(prim[0], prim[1], prim[2], prim[3], dim=2)
    P = Problem(dim=2, system=EULER, nx=n, ny=n, bc_x=TRANSMISSIVE, bc_y=TRANSMISSIVE, cfl=0.45)
    return P, np.ascontiguousarray(q), 0.8


# --------------------------------------------------------------------------
@dataclass
class Request:
    rid: int
    arrival: float          # seconds after stream start
    problem: Problem
    q0: np.ndarray
    steps: int
    kind: str               # "riemann" or "smooth"


def serving_stream(lam: float, n_requests: int = 512, seed: Optional[int] = None,
                   max_1d: int = 65536, max_2d: int = 1024) -> List[Request]:
    """Poisson arrivals at rate lam (req/s).  Half the requests are 1D Euler
    with N log-uniform in [512, max_1d], half 2D with n log-uniform in
    [128, max_2d]; Riemann or smooth-perturbation data by coin flip; 50-500
    RK3 steps; FP64 or FP32 reconstruction by coin flip."""
    rng = np.random.default_rng(int(lam) if seed is None else seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / lam)
        two_d = bool(rng.integers(0, 2))
        smooth = bool(rng.integers(0, 2))
        steps = int(rng.integers(50, 501))
        fp32 = bool(rng.integers(0, 2))
        sub = int(rng.integers(0, 2**31 - 1))
        if two_d:
            n = int(round(math.exp(rng.uniform(math.log(128), math.log(max_2d)))))
            if smooth:
                P, q = smooth_wave_2d(n)
                P = P.with_(dt_rule=DT_CFL, bc_x=PERIODIC, bc_y=PERIODIC)
            else:
                P, q = quadrants_2d(sub, n)
        else:
            N = int(round(math.exp(rng.uniform(math.log(512), math.log(max_1d)))))
            if smooth:
                P, q = entropy_wave_1d(N)
                P = P.with_(dt_rule=DT_CFL)
            else:
                P, q = riemann_1d(sub, N)
        if fp32:
            P = P.fp32()
        out.append(Request(i, t, P, q, steps, "smooth" if smooth else "riemann"))
    return out


# --------------------------------------------------------------------------
# Scalar laws of Section 4.1.  Domains and boundaries the paper leaves open
# are readings: Burgers on periodic [0, 1] (one period of the sine),
# Buckley-Leverett on [-1, 1] with transmissive boundaries (the waves stay
# inside up to T = 0.3).
MULTIWAVE_T = 20.0


def multiwave_exact(x: np.ndarray) -> np.ndarray:
    """The multi-wave initial data (= the exact solution at T = 20, ten
    periods later): Gaussian, square, triangle, semi-ellipse."""
    delta, z, alpha, y = 0.005, -0.7, 10.0, 0.5
    beta = math.log(2.0) / (36.0 * delta * delta)

    def G(zz):
        return np.exp(-beta * (x - zz) ** 2)

    def F(yy):
        return np.sqrt(np.maximum(1.0 - alpha * alpha * (x - yy) ** 2, 0.0))

    q = np.zeros_like(x)
    m = (x >= -0.8) & (x <= -0.6)
    q[m] = ((G(z - delta) + 4.0 * G(z) + G(z + delta)) / 6.0)[m]
    q[(x >= -0.4) & (x <= -0.2)] = 1.0
    m = (x >= 0.0) & (x <= 0.2)
    q[m] = (1.0 - np.abs(10.0 * (x - 0.1)))[m]
    m = (x >= 0.4) & (x <= 0.6)
    q[m] = ((F(y - delta) + 4.0 * F(y) + F(y + delta)) / 6.0)[m]
    return q


def multiwave(N: int = 400) -> Tuple[Problem, np.ndarray]:
    P = Problem(dim=1, system=ADVECTION, nx=N, ny=1, xlo=-1.0, xhi=1.0, bc_x=PERIODIC,
                adv_speed=(1.0, 0.0), cfl=0.45)
    return P, multiwave_exact(centres(N, -1.0, 1.0)).reshape(1, 1, N)


BURGERS_T = 0.2


def burgers_sine(N: int = 80) -> Tuple[Problem, np.ndarray]:
    P = Problem(dim=1, system=BURGERS, nx=N, ny=1, xlo=0.0, xhi=1.0, bc_x=PERIODIC, cfl=0.45)
    x = centres(N, 0.0, 1.0)
    return P, (0.5 + np.sin(2.0 * math.pi * x)).reshape(1, 1, N)


def burgers_sine_exact(x: np.ndarray, t: float) -> np.ndarray:
    """Entropy solution of u_t + (u^2/2)_x = 0, u0 = 1/2 + sin(2 pi x) on
    periodic [0, 1], by characteristics.  With v = u - 1/2 and x' = x - t/2
    the data are odd about x' = 0, so the shock that forms at t = 1/(2 pi)
    stays at x' = 1/2; for x' in [-1/2, 1/2) the value comes from the foot xi
    in (-1/2, 1/2) with xi + t sin(2 pi xi) = x', taken on the branch where
    that map is increasing (|xi| < xi_c, cos(2 pi xi_c) = -1/(2 pi t))."""
    if t * 2.0 * math.pi < 1.0:
        lim = 0.5
    else:
        lim = math.acos(-1.0 / (2.0 * math.pi * t)) / (2.0 * math.pi)
    out = np.empty_like(x, dtype=float)
    for i, xv in enumerate(np.asarray(x, dtype=float)):
        xp = ((xv - 0.5 * t) + 0.5) % 1.0 - 0.5
        a, b = -lim, lim
        for _ in range(200):
            m = 0.5 * (a + b)
            if m <= a or m >= b:
                break
            if m + t * math.sin(2.0 * math.pi * m) < xp:
                a = m
            else:
                b = m
        out[i] = 0.5 + math.sin(2.0 * math.pi * a)
    return out


BUCKLEY_T = 0.3


def buckley_step(N: int = 200) -> Tuple[Problem, np.ndarray]:
    P = Problem(dim=1, system=BUCKLEY, nx=N, ny=1, xlo=-1.0, xhi=1.0, bc_x=TRANSMISSIVE, cfl=0.45)
    x = centres(N, -1.0, 1.0)
    return P, np.where((x >= -0.5) & (x <= 0.0), 1.0, 0.0).reshape(1, 1, N)


# --------------------------------------------------------------------------
# Near-vacuum Euler data (positivity-preserving limiter).
def _tube(left, right, N, lo, hi, x0, gamma, periodic=False):
    x = centres(N, lo, hi)
    L = x < x0
    if periodic:
        # the right state also fills the first quarter: two opposite jumps
        L = L & (x >= lo + 0.5 * (x0 - lo))
    q = conservative(np.where(L, left[0], right[0]), np.where(L, left[1], right[1]), 0.0,
                     np.where(L, left[2], right[2]), gamma=gamma, dim=1)
    P = Problem(dim=1, system=EULER, nx=N, ny=1, xlo=lo, xhi=hi, bc_x=PERIODIC if periodic else TRANSMISSIVE,
                cfl=0.45, gamma=gamma)
    return P, q.reshape(3, 1, N)


def vacuum_tube(N: int = 200, speed: float = 8.0, periodic: bool = False):
    """Double rarefaction rho = 1, p = 0.4, u = -speed | +speed at x = 0 on
    [-5, 5] (T = 0.6): for speed > 3.74 the exact solution contains vacuum.
    periodic: the domain wraps and a second, colliding jump sits at x = -2.5."""
    return _tube((1.0, -speed, 0.4), (1.0, speed, 0.4), N, -5.0, 5.0, 0.0, 1.4, periodic), 0.6


def leblanc(N: int = 400):
    """Leblanc's shock tube: gamma = 5/3, (rho, u, p) = (1, 0, 2/3 10^-1) |
    (10^-3, 0, 2/3 10^-10) at x = 3 on [0, 9], T = 6."""
    g = 5.0 / 3.0
    return _tube((1.0, 0.0, (g - 1.0) * 1e-1), (1e-3, 0.0, (g - 1.0) * 1e-10), N, 0.0, 9.0, 3.0, g), 6.0


def vacuum_quadrants_2d(n: int = 64, speed: float = 6.0):
    """Four quadrants rho = 1, p = 0.4 moving apart from the centre of
    [0, 1]^2 (velocities (+-speed, +-speed)), transmissive; near vacuum
    forms at the centre."""
    x = centres(n, 0.0, 1.0)[None, :]
    y = centres(n, 0.0, 1.0)[:, None]
    u = np.where(x > 0.5, speed, -speed) * np.ones_like(y)
    v = np.where(y > 0.5, speed, -speed) * np.ones_like(x)
    q = conservative(np.ones((n, n)), u, v, np.full((n, n), 0.4), dim=2)
    P = Problem(dim=2, system=EULER, nx=n, ny=n, bc_x=TRANSMISSIVE, bc_y=TRANSMISSIVE, cfl=0.45)
    return P, np.ascontiguousarray(q)
