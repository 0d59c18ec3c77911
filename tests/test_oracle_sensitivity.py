"""Conditioning of the shock workloads (CPU): a one-ulp change of the input
grows to well above 1e-10 relative within a few hundred RK3 steps of the 1D
Euler Riemann data.  This bounds how long any two FP64 implementations (the
oracle and the GPU path) can agree to the 1e-10 final-state bar."""
import numpy as np

from paper_2603_26272_amd import workloads as W


def test_one_ulp_input_change_grows_past_final_state_bar(orc):
    P, q0 = W.riemann_1d(0, 4096)
    rng = np.random.default_rng(1)
    q1 = q0 * (1 + 2.2e-16 * rng.choice([-1, 0, 1], size=q0.shape))
    a, *_ = orc.solve(P, q0, 0.0, 500)
    b, *_ = orc.solve(P, q1, 0.0, 500)
    scale = np.abs(a) + np.abs(a).max(axis=(1, 2), keepdims=True)
    d = (np.abs(a - b) / scale).max()
    assert 1e-10 < d < 1e-6, d
