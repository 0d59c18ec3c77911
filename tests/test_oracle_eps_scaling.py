"""How much the sensitivity epsilon of eq:weight_nonlinear moves a
reconstruction when the data are rescaled.

The GPU kernels carry Euler's two acoustic characteristic fields scaled by
2c.  Reconstructing s f with epsilon eps equals s times reconstructing f with
epsilon eps / s^2 (the indicators and tau scale by s^2).  The general kernels
rescale epsilon exactly; the FP64 Z-weight kernels run only for eps <= 1e-40
and apply it unscaled.  This pins, with the oracle's own reconstruction, that
at eps = 1e-40 replacing eps by eps / s^2 (s = 2c for sound speeds from 0.05
to 50) moves the reconstruction by less than 5e-13 of the stencil's largest
value, on random, nearly flat, partly flat and tiny-magnitude stencils, and
that at eps = 1e-30 it does not (hence the threshold)."""
import numpy as np


def _stencils(rng, n):
    out = []
    for t in range(n):
        kind = t % 4
        if kind == 0:
            v = rng.normal(size=6)
        elif kind == 1:
            v = 1 + 10.0 ** rng.uniform(-15, -3) * rng.normal(size=6)
        elif kind == 2:
            v = np.ones(6) * rng.normal()
            k = int(rng.integers(1, 5))
            v[k:] += 10.0 ** rng.uniform(-15, 0) * rng.normal(size=6 - k)
        else:
            v = 10.0 ** rng.uniform(-8, 8) * (1 + 10.0 ** rng.uniform(-15, -1) * rng.normal(size=6))
        out.append(v)
    return out


def _worst_shift(orc, eps, stencils):
    worst = 0.0
    for v in stencils:
        base = orc.recon(v, eps=eps)
        for c in (0.05, 0.3, 1.0, 5.0, 50.0):
            s2 = (2 * c) ** 2
            worst = max(worst, abs(orc.recon(v, eps=eps / s2) - base) / np.abs(v).max())
    return worst


def test_unscaled_epsilon_is_within_parity_at_the_papers_epsilon(orc):
    st = _stencils(np.random.default_rng(0), 2000)
    assert _worst_shift(orc, 1e-40, st) <= 5e-13
    assert _worst_shift(orc, 1e-30, st) > 1e-12
