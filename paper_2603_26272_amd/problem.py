"""Problem description shared by the Python binding and the workload generators.

Field meanings follow the paper's problem statement (Section 2): a hyperbolic
conservation law on a uniform mesh of nx (x ny) cells over [xlo, xhi]
(x [ylo, yhi]), point values at cell centres, boundary conditions, and the
WENO-ZA6 weight parameters of eq:weight_nonlinear / eq:aimu.
"""
from dataclasses import dataclass, field, replace
from typing import Tuple

# system
ADVECTION, EULER, BURGERS, BUCKLEY = 0, 1, 2, 3
# boundary conditions
PERIODIC, TRANSMISSIVE = 0, 1
# precision of the interface reconstruction (state and RK3 are always FP64)
FP64, FP32_RECON = 0, 1
# time-step rule
DT_CFL, DT_CFL_H2 = 0, 1
# Lax-Friedrichs speed for systems
LF_PER_FIELD, LF_SCALAR = 0, 1


@dataclass
class Problem:
    dim: int = 1
    system: int = EULER
    nx: int = 64
    ny: int = 1
    xlo: float = 0.0
    xhi: float = 1.0
    ylo: float = 0.0
    yhi: float = 1.0
    bc_x: int = TRANSMISSIVE
    bc_y: int = TRANSMISSIVE
    gamma: float = 1.4
    adv_speed: Tuple[float, float] = (1.0, 0.0)
    cfl: float = 0.5
    dt_rule: int = DT_CFL
    precision: int = FP64
    p: float = 1.0
    eps: float = 1e-40
    affine_invariant: int = 0
    mu0: float = 1e-40
    lf: int = LF_PER_FIELD
    linear_weights: int = 0
    order: int = 3          # r of the order-2r central-upwind scheme (3: WENO-ZA6)
    pp_limiter: int = 0     # 1: positivity-preserving flux limiter in time steps (Euler, FP64)
    alt_tau: int = 0        # 1: the alternative global indicator tau' (eq:GSI_alt; r = 3)
    weight_L: float = 1.0   # L and q of eq:weights_unnormalized (JS family: L = 0, p = 2)
    weight_q: float = 1.0

    @property
    def m(self) -> int:
        if self.system == EULER:
            return 3 if self.dim == 1 else 4
        return 1

    @property
    def shape(self):
        """SoA state shape [m][ny][nx]."""
        return (self.m, self.ny, self.nx)

    @property
    def dx(self) -> float:
        return (self.xhi - self.xlo) / self.nx

    @property
    def dy(self) -> float:
        return (self.yhi - self.ylo) / self.ny if self.dim == 2 else 1.0

    def interfaces_per_rhs(self) -> int:
        """Interface reconstructions (full flux vectors) in one RHS evaluation."""
        if self.dim == 1:
            return self.nx + 1
        return (self.nx + 1) * self.ny + self.nx * (self.ny + 1)

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)

    def fp32(self) -> "Problem":
        """FP32-reconstruction variant with epsilon rescaled to FP32 range."""
        return replace(self, precision=FP32_RECON, eps=1e-20, mu0=1e-8)
