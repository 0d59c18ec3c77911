"""Algorithmic FLOPs of the WENO-ZA6 sweeps, counted by running the oracle
with its counting scalar (add/sub, mul, div, sqrt = 1 FLOP each; operations a
compiler folds away are not counted).

A sweep over L lines of n cells costs L * ((n + 6) * a + (n + 1) * b) in the
oracle's interface part (a: physical flux per cell including ghosts,
b: per interface).  Counting two sizes separates a and b.  Per-cell FP64
closed forms are added for the flux difference (sub + div per component),
the 2D accumulation L_x + L_y (1 per component) and the SSP-RK3 stage
a Qn + b (Q + dt L) (5 per component).

Run:  python -m oracle.count_flops   (prints JSON)
"""
import json
import sys

import numpy as np

from . import count_ops


def _prob(dim, system, nx, ny, fp32=0, order=3):
    return {"dim": dim, "system": system, "nx": nx, "ny": ny, "bc_x": 0, "bc_y": 0,
            "precision": fp32, "eps": 1e-20 if fp32 else 1e-40, "mu0": 1e-8 if fp32 else 1e-40,
            "adv_speed": (1.0, 0.5), "order": order}


def _state(dim, system, nx, ny, seed=0):
    rng = np.random.default_rng(seed)
    if system != 1:
        return rng.uniform(0.2, 0.8, size=(1, ny, nx))
    rho = rng.uniform(0.5, 1.5, size=(ny, nx))
    u = rng.uniform(-0.5, 0.5, size=(ny, nx))
    v = rng.uniform(-0.5, 0.5, size=(ny, nx))
    p = rng.uniform(0.5, 1.5, size=(ny, nx))
    if dim == 1:
        return np.stack([rho, rho * u, p / 0.4 + 0.5 * rho * u * u])
    return np.stack([rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v)])


def per_cell_and_interface(dim, system, direction, fp32=0, order=3):
    """(a, b): FLOPs per cell (with its 2r ghosts) and per interface of one
    sweep of the order-2r scheme."""
    out = []
    for n in (64, 128):
        if dim == 1:
            nx, ny = n, 1
        elif direction == 0:
            nx, ny = n, 4
        else:
            nx, ny = 4, n
        q = np.ascontiguousarray(_state(dim, system, nx, ny))
        nir, c = count_ops(_prob(dim, system, nx, ny, fp32, order), q, 1 << direction)
        flops = c["add"] + c["mul"] + c["div"] + c["sqrt"]
        lines = ny if direction == 0 else nx
        out.append((n, flops / lines))
    (n1, f1), (n2, f2) = out
    # f = (n + 2r) a + (n + 1) b, two equations
    g = 2 * order
    A = np.array([[n1 + g, n1 + 1], [n2 + g, n2 + 1]], dtype=float)
    a, b = np.linalg.solve(A, np.array([f1, f2]))
    return float(a), float(b)


def table():
    res = {}
    for name, dim, system, m in (("advection_1d", 1, 0, 1), ("euler_1d", 1, 1, 3), ("euler_2d", 2, 1, 4)):
        for fp32 in (0, 1):
            dirs = (0,) if dim == 1 else (0, 1)
            for d in dirs:
                a, b = per_cell_and_interface(dim, system, d, fp32)
                key = f"{name}{'_fp32' if fp32 else ''}_{'xy'[d]}"
                diff = 2 * m
                if dim == 1:
                    extra = diff + 5 * m          # difference + stage
                elif d == 0:
                    extra = diff                  # L_x
                else:
                    extra = diff + m + 5 * m      # difference + accumulate + stage
                res[key] = {"cell_flux": round(a, 3), "interface": round(b, 3), "cell_update": extra}
    # 2D Euler with the other orders (FP64)
    for r in (2, 4, 5):
        for d in (0, 1):
            a, b = per_cell_and_interface(2, 1, d, 0, r)
            extra = 8 if d == 0 else 8 + 4 + 20
            res[f"euler_2d_r{r}_{'xy'[d]}"] = {"cell_flux": round(a, 3), "interface": round(b, 3),
                                              "cell_update": extra}
    return res


if __name__ == "__main__":
    json.dump(table(), sys.stdout, indent=1)
    print()
