"""The oracle's FP32-reconstruction reading (the same templated code in
float, eps = 1e-20) pinned to its FP64 result within FP32 rounding: single
reconstructions on random stencils, and whole-grid 1D / 2D Euler fluxes on
the workloads (observed 2e-7 of the component scale; bound 2e-6, well
below what a wrong constant or a dropped term in the FP32 path would give).  Constant
states are exact in both (tests/test_oracle_schemes.py)."""
import numpy as np

from paper_2603_26272_amd import workloads as W

EPS32 = np.finfo(np.float32).eps


def test_single_reconstructions_within_fp32_rounding(orc):
    rng = np.random.default_rng(32)
    worst = 0.0
    for i in range(500):
        v = rng.standard_normal(6)
        if i % 2:
            v[rng.integers(1, 6):] += rng.uniform(1, 5)
        v = v.astype(np.float32).astype(np.float64)      # representable in FP32
        r64 = orc.recon(v)
        r32 = orc.recon_f32(v, eps=1e-20)
        err = abs(r32 - r64) / (EPS32 * np.abs(v).max())
        worst = max(worst, err)
    assert worst < 8, worst


def _close(a, b, rel):
    ax = tuple(range(1, a.ndim))
    scale = np.abs(b).max(axis=ax, keepdims=True)
    return np.all(np.abs(a - b) <= rel * (np.abs(b) + scale))


def test_euler_fluxes_fp32_reading(orc):
    P, q0 = W.riemann_1d(4, 1000)
    f64, _, st = orc.fluxes(P, q0)
    f32, _, st32 = orc.fluxes(P.fp32(), q0)
    assert st == 0 and st32 == 0
    assert _close(f32, f64, 2e-6)
    P, q0 = W.quadrants_2d(3, 96, 90)
    fx64, fy64, _ = orc.fluxes(P, q0)
    fx32, fy32, _ = orc.fluxes(P.fp32(), q0)
    assert _close(fx32, fx64, 2e-6) and _close(fy32, fy64, 2e-6)
