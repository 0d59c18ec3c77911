"""Approximate dispersion relation (ADR) of the schemes, on the GPU.

The ADR analysis of Section 3.2 (after Pirozzoli): for a nonlinear scheme the
modified wavenumber is measured by applying the semi-discrete operator of
u_t + u_x = 0 (periodic, dx = 1, global Lax-Friedrichs splitting with
alpha = 1, so only the upwind flux f+ = u is reconstructed) to one sampled
Fourier mode u_j = A cos(phi j), phi = 2 pi k / N, and projecting the result
on that mode:

    Phi(phi) = i * sum_j L_j e^{-i phi j} / sum_j u_j e^{-i phi j}.

The exact derivative gives Phi = phi; Re Phi measures dispersion, Im Phi
dissipation (negative: damping; positive: anti-dissipation).  Every
right-hand side is computed by libza's kernels (za_rhs); only the projection
onto the mode happens here.
"""
from typing import Dict, Tuple

import numpy as np

from .problem import ADVECTION, PERIODIC, Problem


def adr_problem(N: int = 256, order: int = 3, linear: int = 0, alt_tau: int = 0) -> Problem:
    return Problem(dim=1, system=ADVECTION, nx=N, ny=1, xlo=0.0, xhi=float(N), bc_x=PERIODIC,
                   adv_speed=(1.0, 0.0), order=order, linear_weights=linear, alt_tau=alt_tau)


def modes(N: int) -> np.ndarray:
    """The resolvable frequencies phi_k = 2 pi k / N, k = 1 .. N/2."""
    return 2.0 * np.pi * np.arange(1, N // 2 + 1) / N


def project(phi: float, u: np.ndarray, L: np.ndarray) -> complex:
    j = np.arange(u.size)
    e = np.exp(-1j * phi * j)
    return complex(1j * np.sum(L * e) / np.sum(u * e))


def adr_gpu(N: int = 256, order: int = 3, linear: int = 0, alt_tau: int = 0, amplitude: float = 1.0,
            device=None) -> Tuple[np.ndarray, np.ndarray]:
    """(phi, Phi(phi)) of the scheme selected by (order, linear, alt_tau)."""
    import torch

    from .za import Context
    dev = device if device is not None else torch.device("cuda:0")
    P = adr_problem(N, order, linear, alt_tau)
    phis = modes(N)
    out = np.empty(phis.size, dtype=complex)
    j = np.arange(N)
    with Context(P) as ctx:
        for i, phi in enumerate(phis):
            u = amplitude * np.cos(phi * j)
            q = torch.from_numpy(u.reshape(1, 1, N).copy()).to(dev)
            L = ctx.rhs(q).cpu().numpy().reshape(-1)
            out[i] = project(phi, u, L)
    return phis, out


SCHEMES: Dict[str, dict] = {
    "CT6": dict(order=3, linear=1),        # the linear sixth-order central scheme (omega = d)
    "ZA6": dict(order=3),                  # WENO-ZA6 with tau (eq:GSI)
    "ZA6-tau'": dict(order=3, alt_tau=1),  # WENO-ZA6 with tau' (eq:GSI_alt)
    "ZA4": dict(order=2),
    "ZA8": dict(order=4),
    "ZA10": dict(order=5),
}
