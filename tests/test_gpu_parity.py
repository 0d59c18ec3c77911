"""GPU parity: libza (HIP, through the C ABI) against the oracle.

Bars (from the design): FP64 interface fluxes within
1e-12 * (|F_oracle| + max |F_oracle| of that component), final states within
1e-10 * (|Q_oracle| + max |Q_oracle| of that component); integer-like
outcomes (step counts, status codes) exact.
"""
import math

import numpy as np
import pytest

import oracle as orc
from paper_2603_26272_amd import workloads as W
from paper_2603_26272_amd.problem import (ADVECTION, BUCKLEY, BURGERS, EULER, PERIODIC,
                                          TRANSMISSIVE, Problem)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2603_26272_amd import za
    za.lib()
    return torch.device("cuda:0")


def Ctx(P):
    from paper_2603_26272_amd.za import Context
    return Context(P)


def comp_tol(ref, rel):
    """rel * (|ref| + max over the component), broadcast over [m][...]."""
    ax = tuple(range(1, ref.ndim))
    return rel * (np.abs(ref) + np.abs(ref).max(axis=ax, keepdims=True))


def assert_close(got, ref, rel, what=""):
    tol = comp_tol(ref, rel)
    err = np.abs(got - ref)
    bad = err > tol
    if bad.any():
        i = np.unravel_index(np.argmax(err / np.maximum(tol, 1e-300)), err.shape)
        raise AssertionError(f"{what}: {bad.sum()} entries off; worst at {i}: got {got[i]!r} ref {ref[i]!r} "
                             f"tol {tol[i]:.3e} (max rel-to-tol {float((err / np.maximum(tol, 1e-300)).max()):.3g})")


def gpu_fluxes(P, q0, dev):
    q = torch.from_numpy(np.ascontiguousarray(q0)).to(dev)
    with Ctx(P) as ctx:
        fx, fy = ctx.rhs_fluxes(q)
        torch.cuda.synchronize()
        return fx.cpu().numpy(), None if fy is None else fy.cpu().numpy()


# ---------------------------------------------------------------------------
# interface fluxes
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("N", [1, 2, 3, 7, 25, 63, 64, 65, 200])
@pytest.mark.parametrize("system", [ADVECTION, BURGERS, BUCKLEY])
def test_fluxes_1d_scalar(dev, N, system):
    rng = np.random.default_rng(N + 17 * system)
    x = W.centres(N, -1.0, 1.0)
    q0 = (np.sin(np.pi * x) + (x > 0.3) * 0.7 + 0.05 * rng.normal(size=N)).reshape(1, 1, N)
    if system == BUCKLEY:
        q0 = np.clip(np.abs(q0), 0, 1)
    for bc in (PERIODIC, TRANSMISSIVE):
        P = Problem(dim=1, system=system, nx=N, xlo=-1.0, xhi=1.0, bc_x=bc, adv_speed=(1.3, 0.0))
        fx, _ = gpu_fluxes(P, q0, dev)
        ref, _, st = orc.fluxes(P, q0)
        assert st == 0
        assert_close(fx, ref, 1e-12, f"scalar {system} N={N} bc={bc}")


@pytest.mark.parametrize("N", [1, 3, 6, 63, 64, 65, 127, 300])
def test_fluxes_1d_euler_ragged(dev, N):
    for bc in (PERIODIC, TRANSMISSIVE):
        P, q0 = W.riemann_1d(N, max(N, 8))
        q0 = np.ascontiguousarray(q0[:, :, :N])
        P = P.with_(nx=N, bc_x=bc)
        fx, _ = gpu_fluxes(P, q0, dev)
        ref, _, st = orc.fluxes(P, q0)
        assert st == 0
        assert_close(fx, ref, 1e-12, f"euler1d N={N} bc={bc}")


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_fluxes_1d_euler_full_size(dev, seed):
    """The 1D Euler workload at its full size (N = 4096), every interface."""
    P, q0 = W.riemann_1d(seed, 4096)
    fx, _ = gpu_fluxes(P, q0, dev)
    ref, _, st = orc.fluxes(P, q0)
    assert st == 0
    assert_close(fx, ref, 1e-12, f"euler1d seed={seed}")


@pytest.mark.parametrize("shape", [(1, 1), (2, 3), (5, 7), (63, 65), (96, 80), (130, 67)])
def test_fluxes_2d_euler(dev, shape):
    nx, ny = shape
    for bcx, bcy in ((TRANSMISSIVE, TRANSMISSIVE), (PERIODIC, TRANSMISSIVE), (PERIODIC, PERIODIC)):
        P, q0 = W.quadrants_2d(nx * 7 + ny, nx, ny)
        P = P.with_(bc_x=bcx, bc_y=bcy)
        # On tiny periodic grids a quadrant plateau can fill a stencil
        # symmetrically (S N N N N S): then <c_tau, f> = 0 exactly, every
        # Gamma_k is 0 in exact arithmetic, and rounding noise alone picks the
        # weights, so no two implementations agree.  A 1% density ripple
        # removes the exact symmetry.
        rng = np.random.default_rng(nx * ny)
        q0 = q0.copy()
        q0[0] *= 1.0 + 1e-2 * rng.random(q0[0].shape)
        fx, fy = gpu_fluxes(P, q0, dev)
        rx, ry, st = orc.fluxes(P, q0)
        assert st == 0
        assert_close(fx, rx, 1e-12, f"2d fx {shape}")
        assert_close(fy, ry, 1e-12, f"2d fy {shape}")


def test_fluxes_2d_full_size_sampled(dev):
    """The 2D Euler workload at its full size (2048^2): every GPU flux is
    computed in the benchmark's launch configuration; 24 rows and 24 columns
    (including both boundaries) are recomputed by the oracle."""
    P, q0 = W.quadrants_2d(0, 2048)
    fx, fy = gpu_fluxes(P, q0, dev)
    rng = np.random.default_rng(0)
    lines = sorted(set([0, 1, 2, 3, 1023, 1024, 2044, 2045, 2046, 2047] + list(rng.integers(0, 2048, 14))))
    rx, st = orc.fluxes_lines(P, q0, 0, lines)
    assert st == 0
    for j, l in enumerate(lines):
        assert_close(fx[:, l, :], rx[j], 1e-12, f"row {l}")
    ry, st = orc.fluxes_lines(P, q0, 1, lines)
    for j, l in enumerate(lines):
        assert_close(fy[:, :, l], ry[j], 1e-12, f"col {l}")


def test_fluxes_2d_full_size_sampled_fp32(dev):
    """FP32 reconstruction at the full 2048^2 size of the benchmark's FP32
    leg: 16 rows and 16 columns (both boundaries included) against the
    oracle's FP32 reading, to the 3e-5 of the small FP32 case."""
    P, q0 = W.quadrants_2d(0, 2048)
    P = P.fp32()
    fx, fy = gpu_fluxes(P, q0, dev)
    rng = np.random.default_rng(1)
    lines = sorted(set([0, 1, 2, 1023, 1024, 2045, 2046, 2047] + list(rng.integers(0, 2048, 8))))
    rx, st = orc.fluxes_lines(P, q0, 0, lines)
    assert st == 0
    for j, l in enumerate(lines):
        assert_close(fx[:, l, :], rx[j], 3e-5, f"fp32 row {l}")
    ry, st = orc.fluxes_lines(P, q0, 1, lines)
    assert st == 0
    for j, l in enumerate(lines):
        assert_close(fy[:, :, l], ry[j], 3e-5, f"fp32 col {l}")


def test_fluxes_2d_advection(dev):
    N = 40
    x = W.centres(N, 0, 1)[None, :]
    y = W.centres(N + 3, 0, 1)[:, None]
    q0 = (np.sin(2 * np.pi * (x + 2 * y)) + (x > 0.5) * (y < 0.4)).reshape(1, N + 3, N)
    P = Problem(dim=2, system=ADVECTION, nx=N, ny=N + 3, bc_x=PERIODIC, bc_y=PERIODIC, adv_speed=(1.0, -0.5))
    fx, fy = gpu_fluxes(P, np.ascontiguousarray(q0), dev)
    rx, ry, st = orc.fluxes(P, np.ascontiguousarray(q0))
    assert_close(fx, rx, 1e-12, "adv2d fx")
    assert_close(fy, ry, 1e-12, "adv2d fy")


@pytest.mark.parametrize("variant", ["ai", "p15", "linear", "lf_scalar"])
def test_fluxes_weight_variants(dev, variant):
    P, q0 = W.quadrants_2d(9, 70, 66)
    kw = {"ai": dict(affine_invariant=1, mu0=1e-40), "p15": dict(p=1.5), "linear": dict(linear_weights=1),
          "lf_scalar": dict(lf=1)}[variant]
    P = P.with_(**kw)
    fx, fy = gpu_fluxes(P, q0, dev)
    rx, ry, st = orc.fluxes(P, q0)
    assert_close(fx, rx, 1e-12, variant)
    assert_close(fy, ry, 1e-12, variant)


@pytest.mark.parametrize("variant", ["z_eps1e-6", "z_eps1e-30", "js_eps1e-6", "ai_mu0_1e-3", "fp32_eps1e-6"])
@pytest.mark.parametrize("dim", [1, 2])
def test_fluxes_euler_nondefault_eps(dev, variant, dim):
    """Euler fluxes with an epsilon (and mu_0) large enough to matter
    (eq:weight_nonlinear, eq:aimu): a small smooth ripple on Riemann data
    makes the indicators comparable to epsilon.  The kernels carry the two
    acoustic characteristic fields scaled by 2c, so they must scale epsilon
    by 4c^2 (and mu_0 by 2c) to reconstruct what the oracle reconstructs;
    FP64 problems with eps above 1e-40 run the general kernels, which do."""
    kw = {"z_eps1e-6": dict(eps=1e-6), "z_eps1e-30": dict(eps=1e-30),
          "js_eps1e-6": dict(eps=1e-6, weight_L=0.0, weight_q=1.0, p=2.0),
          "ai_mu0_1e-3": dict(affine_invariant=1, mu0=1e-3, eps=1e-6), "fp32_eps1e-6": dict(eps=1e-6)}[variant]
    if dim == 1:
        P, q0 = W.riemann_1d(4, 300)
        x = W.centres(300, 0.0, 1.0)
        q0 = q0.copy()
        q0[0] *= 1.0 + 1e-2 * np.sin(6 * np.pi * x)
    else:
        P, q0 = W.quadrants_2d(9, 70, 66)
        x = W.centres(70, 0.0, 1.0)[None, :]
        y = W.centres(66, 0.0, 1.0)[:, None]
        q0 = q0.copy()
        q0[0] *= 1.0 + 1e-2 * np.sin(2 * np.pi * (3 * x + 2 * y))
    P = P.with_(**kw)
    rel = 1e-12
    if variant.startswith("fp32"):
        P = P.fp32().with_(eps=1e-6)
        rel = 3e-5
    fx, fy = gpu_fluxes(P, q0, dev)
    rx, ry, st = orc.fluxes(P, q0)
    assert st == 0
    assert_close(fx, rx, rel, f"{variant} fx")
    if dim == 2:
        assert_close(fy, ry, rel, f"{variant} fy")


# ---------------------------------------------------------------------------
# right-hand side, steps, solves
# ---------------------------------------------------------------------------
def test_rhs_2d(dev):
    P, q0 = W.quadrants_2d(4, 96, 80)
    q = torch.from_numpy(q0).to(dev)
    with Ctx(P) as ctx:
        L = ctx.rhs(q).cpu().numpy()
    ref, st = orc.rhs(P, q0)
    assert st == 0
    assert_close(L, ref, 1e-11, "rhs 2d")


def test_rhs_1d(dev):
    P, q0 = W.riemann_1d(5, 4096)
    q = torch.from_numpy(q0).to(dev)
    with Ctx(P) as ctx:
        L = ctx.rhs(q).cpu().numpy()
    ref, st = orc.rhs(P, q0)
    assert_close(L, ref, 1e-11, "rhs 1d")


@pytest.mark.parametrize("fp32", [0, 1])
def test_constant_state_bitwise(dev, fp32):
    for P in (Problem(dim=1, nx=100), Problem(dim=2, nx=70, ny=33, bc_x=PERIODIC)):
        P = P.fp32() if fp32 else P
        prim = (0.8, 0.3, -0.6, 1.7)
        if P.dim == 1:
            q0 = W.conservative(np.full(P.nx, prim[0]), prim[1], 0, prim[3], dim=1).reshape(3, 1, P.nx)
        else:
            q0 = W.conservative(np.full((P.ny, P.nx), prim[0]), prim[1], prim[2], prim[3], dim=2)
        q = torch.from_numpy(np.ascontiguousarray(q0)).to(dev)
        with Ctx(P) as ctx:
            L = ctx.rhs(q).cpu().numpy()
            assert np.all(L == 0.0)
            q1 = q.clone()
            ctx.solve(q1, 0.0, 5)
            # the RK3 convex combinations of equal states round to within 1 ulp
            assert torch.allclose(q1, q, rtol=4e-16, atol=0)


def test_step_cfl_dt_and_state(dev):
    P, q0 = W.quadrants_2d(6, 64, 72)
    q = torch.from_numpy(q0).to(dev)
    with Ctx(P) as ctx:
        dt = ctx.step(q, 0.0, sync=True)
    ref, dt_ref, st = orc.step(P, q0, 0.0)
    # the wave speeds are maxima of correctly rounded per-cell values and the
    # CFL rule one more correctly rounded expression: bit for bit
    assert dt == dt_ref, (dt, dt_ref)
    assert_close(q.cpu().numpy(), ref, 1e-10, "step")


@pytest.mark.parametrize("case", ["1d", "2d", "2d_full", "config3"])
def test_cfl_dt_bitwise(dev, case):
    """The CFL step of eq:LF's wave speeds equals the oracle's bit for bit:
    1D and 2D Riemann data, the 2048^2 workload, and the 2D Riemann
    configuration 3 at 400^2 (CFL 0.45), on the first and a later step."""
    if case == "1d":
        P, q0 = W.riemann_1d(3, 4096)
    elif case == "2d":
        P, q0 = W.quadrants_2d(12, 130, 67)
    elif case == "2d_full":
        P, q0 = W.quadrants_2d(0, 2048)
    else:
        P, q0, _ = W.riemann_config3(400)
    q = torch.from_numpy(q0).to(dev)
    with Ctx(P) as ctx:
        dt1 = ctx.step(q, 0.0, sync=True)
        q1 = q.cpu().numpy()
        dt2 = ctx.step(q, 0.0, sync=True)
    assert dt1 == orc.cfl_dt(P, q0)
    assert dt2 == orc.cfl_dt(P, q1)


def test_cfl_dt_bitwise_random_states(dev):
    """Random states per cell (zero and nonzero momenta, densities and
    pressures over eight decades) on 24 small grids: each CFL step is set by
    a different cell, and every one must equal the oracle's bit for bit."""
    rng = np.random.default_rng(77)
    for trial in range(24):
        dim = 1 if trial % 3 == 0 else 2
        nx, ny = (int(rng.integers(5, 300)), 1) if dim == 1 else (int(rng.integers(3, 70)), int(rng.integers(3, 70)))
        shape = (ny, nx)
        rho = 10.0 ** rng.uniform(-4, 4, shape)
        p = 10.0 ** rng.uniform(-4, 4, shape)
        u = rng.normal(size=shape) * 10.0 ** rng.uniform(-3, 3, shape) * (rng.random(shape) < 0.8)
        v = rng.normal(size=shape) * (rng.random(shape) < 0.5)
        if dim == 1:
            q0 = W.conservative(rho[0], u[0], 0.0, p[0], dim=1).reshape(3, 1, nx)
            P = Problem(dim=1, nx=nx, bc_x=TRANSMISSIVE)
        else:
            q0 = W.conservative(rho, u, v, p, dim=2)
            P = Problem(dim=2, nx=nx, ny=ny, bc_x=TRANSMISSIVE, bc_y=PERIODIC)
        q = torch.from_numpy(np.ascontiguousarray(q0)).to(dev)
        with Ctx(P) as ctx:
            # the step may turn non-physical in a later stage; its dt comes
            # from the (physical) initial state all the same
            import ctypes
            from paper_2603_26272_amd import za
            used = ctypes.c_double(0.0)
            st = za.lib().za_step(ctx._h, ctypes.c_void_p(q.data_ptr()), 0.0, ctypes.byref(used))
            assert st in (za.ZA_OK, za.ZA_ERR_NONFINITE), st
            dt = used.value
        assert dt == orc.cfl_dt(P, q0), (trial, dt, orc.cfl_dt(P, q0))


def test_solve_advection_c0(dev):
    """The smooth-advection workload (N = 200, T = 2, dt = 0.5 dx^2): GPU vs
    oracle final state, and the sixth-order error of the closed form."""
    P, q0 = W.advection_sine(200)
    q = torch.from_numpy(q0).to(dev)
    with Ctx(P) as ctx:
        info = ctx.solve(q, 2.0)
    ref, steps, t, st = orc.solve(P, q0, 2.0)
    assert info["steps"] == steps == 40000 and info["t"] == 2.0
    got = q.cpu().numpy()
    assert_close(got, ref, 1e-10, "c0")
    x = W.centres(200, -1.0, 1.0)
    e = np.abs(got[0, 0] - np.sin(np.pi * (x - 2.0))).max()
    assert abs(e - 4.31e-11) <= 0.02 * 4.31e-11


@pytest.mark.parametrize("seed", [0, 1])
def test_solve_euler_1d(dev, seed):
    P, q0 = W.riemann_1d(seed, 4096)
    q = torch.from_numpy(q0).to(dev)
    with Ctx(P) as ctx:
        info = ctx.solve(q, 0.0, 100)
    ref, steps, t, st = orc.solve(P, q0, 0.0, 100)
    assert st == 0 and info["steps"] == steps == 100
    assert abs(info["t"] - t) <= 1e-13 * t
    assert_close(q.cpu().numpy(), ref, 1e-10, f"c1 seed {seed}")


def test_solve_euler_2d(dev):
    P, q0 = W.quadrants_2d(2, 160, 144)
    q = torch.from_numpy(q0).to(dev)
    with Ctx(P) as ctx:
        info = ctx.solve(q, 0.0, 20)
    orc.set_threads(16)
    ref, steps, t, st = orc.solve(P, q0, 0.0, 20)
    assert info["steps"] == 20
    assert_close(q.cpu().numpy(), ref, 1e-10, "2d solve")


@pytest.mark.parametrize("eps", [1e-60, 1e-100, 1e-300])
def test_solve_tiny_eps_on_flat_states(dev, eps):
    """eq:weight_nonlinear with an epsilon far below the paper's 1e-40 on
    Riemann data, whose constant regions give all-zero indicators: the
    weights are then the linear ones, and the GPU steps match the oracle's.
    (The fast kernels form products of four (16 eps) terms and run only down
    to eps = 1e-70; smaller eps takes the general kernels.)"""
    P, q0 = W.quadrants_2d(3, 96, 80)
    P = P.with_(eps=eps)
    q = torch.from_numpy(q0).to(dev)
    with Ctx(P) as ctx:
        info = ctx.solve(q, 0.0, 5)
    ref, steps, t, st = orc.solve(P, q0, 0.0, 5)
    assert st == 0 and info["steps"] == steps == 5
    assert_close(q.cpu().numpy(), ref, 1e-10, f"eps {eps:g}")


def test_solve_to_time_clips_last_step(dev):
    P, q0, T = W.shock_tube("sod", 200)
    q = torch.from_numpy(q0).to(dev)
    with Ctx(P) as ctx:
        info = ctx.solve(q, T)
    ref, steps, t, st = orc.solve(P, q0, T)
    assert info["t"] == T and info["steps"] == steps
    assert_close(q.cpu().numpy(), ref, 1e-10, "sod")


def test_fp32_recon_parity(dev):
    """FP32 reconstruction against the oracle's FP32 reading.  Both round
    every operation to FP32 but in different orders and with different
    reciprocals, so agreement is bounded by FP32 rounding amplified by the
    weights: 3e-5 relative to the component scale."""
    P, q0 = W.quadrants_2d(3, 96, 90)
    P = P.fp32()
    fx, fy = gpu_fluxes(P, q0, dev)
    rx, ry, st = orc.fluxes(P, q0)
    assert_close(fx, rx, 3e-5, "fp32 fx")
    assert_close(fy, ry, 3e-5, "fp32 fy")


def test_two_steps_full_size_fp32_against_oracle(dev):
    """Two RK3 steps of the 2048^2 workload with FP32 reconstruction (the
    benchmark's FP32 leg), every cell against the oracle's FP32 reading and
    against its FP64 run.  The flux bar of 3e-5 bounds a stage's update by
    about 6e-5 of the component scale per direction; the two readings
    observed 1.0e-7 apart (2.8e-8 from FP64), and both bars here are 1e-6.
    The second step's dt follows the FP32-rounded states, so the times agree
    to 1e-7 relative rather than bit for bit."""
    P64, q0 = W.quadrants_2d(0, 2048)
    P = P64.fp32()
    q = torch.from_numpy(q0).to(dev)
    with Ctx(P) as ctx:
        info = ctx.solve(q, 0.0, 2)
    got = q.cpu().numpy()
    orc.set_threads(16)
    ref, steps, t, st = orc.solve(P, q0, 0.0, 2)
    assert st == 0 and steps == 2 and info["steps"] == 2
    assert abs(info["t"] - t) <= 1e-7 * t
    assert_close(got, ref, 1e-6, "fp32 2048^2, two steps")
    ref64, steps, t64, st = orc.solve(P64, q0, 0.0, 2)
    assert st == 0 and steps == 2
    assert_close(got, ref64, 1e-6, "fp32 2048^2 against the FP64 oracle")


def test_determinism_bitwise(dev):
    P, q0 = W.quadrants_2d(8, 128, 128)
    outs = []
    for _ in range(2):
        q = torch.from_numpy(q0).to(dev)
        with Ctx(P) as ctx:
            ctx.solve(q, 0.0, 10)
        outs.append(q.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_conserved_sums_periodic(dev):
    P, q0 = W.quadrants_2d(5, 128, 96)
    P = P.with_(bc_x=PERIODIC, bc_y=PERIODIC)
    q = torch.from_numpy(q0).to(dev)
    with Ctx(P) as ctx:
        s0 = np.array(ctx.conserved_sums(q))
        ctx.solve(q, 0.0, 25)
        s1 = np.array(ctx.conserved_sums(q))
    scale = np.abs(q0).reshape(4, -1).sum(axis=1)
    assert np.all(np.abs(s1 - s0) <= 1e-12 * scale)


def test_nonfinite_reported(dev):
    from paper_2603_26272_amd.za import ZA_ERR_NONFINITE
    P, q0 = W.riemann_1d(0, 512)
    q0 = q0.copy()
    q0[0, 0, 100] = np.nan
    q = torch.from_numpy(q0).to(dev)
    with Ctx(P) as ctx:
        res = ctx.solve(q, 0.0, 10, check=False)
    assert res["status"] == ZA_ERR_NONFINITE and res["nonfinite_step"] == 0 and res["steps"] == 0


def test_invalid_arguments(dev):
    from paper_2603_26272_amd.za import ZA_ERR_ARG, ZaError
    for bad in (Problem(dim=3), Problem(nx=0), Problem(dim=1, ny=4), Problem(cfl=-1.0), Problem(p=0.5),
                Problem(precision=1, eps=1e-40), Problem(dim=2, nx=1 << 16, ny=(1 << 15) + 1)):
        with pytest.raises(ZaError) as ei:
            Ctx(bad)
        assert ei.value.status == ZA_ERR_ARG
    P = Problem(dim=1, nx=32)
    with Ctx(P) as ctx:
        with pytest.raises(ValueError):
            ctx.rhs(torch.zeros((3, 1, 31), dtype=torch.float64, device=dev))
        with pytest.raises(TypeError):
            ctx.rhs(torch.zeros((3, 1, 32), dtype=torch.float32, device=dev))


def test_full_length_1d_drift_bounded_by_self_sensitivity(dev):
    """The 1D Euler workload at full length (N = 4096, 2000 steps).  Shock
    data amplify rounding: the oracle against itself with its input perturbed
    by one ulp drifts to ~5e-8 relative after 2000 steps.  The GPU result must
    stay within 10x of that self-sensitivity (and every flux of the first step
    within 1e-12, checked elsewhere)."""
    P, q0 = W.riemann_1d(0, 4096)
    q = torch.from_numpy(q0).to(dev)
    with Ctx(P) as ctx:
        info = ctx.solve(q, 0.0, 2000)
    assert info["steps"] == 2000
    ref, *_ = orc.solve(P, q0, 0.0, 2000)
    rng = np.random.default_rng(1)
    q1 = q0 * (1 + 2.2e-16 * rng.choice([-1, 0, 1], size=q0.shape))
    ref1, *_ = orc.solve(P, q1, 0.0, 2000)
    scale = np.abs(ref) + np.abs(ref).max(axis=(1, 2), keepdims=True)
    self_sens = (np.abs(ref1 - ref) / scale).max()
    gpu_drift = (np.abs(q.cpu().numpy() - ref) / scale).max()
    print(f"1D Euler N = 4096, 2000 steps: GPU vs oracle {gpu_drift:.3e}, oracle vs its one-ulp "
          f"perturbation {self_sens:.3e}", flush=True)
    assert self_sens > 1e-10            # the problem itself is this sensitive
    assert gpu_drift <= 10 * self_sens, (gpu_drift, self_sens)


def test_two_steps_full_size_against_oracle(dev):
    """Two RK3 steps of the 2D Euler workload at 2048^2 in the benchmark's
    launch configuration (looped x-sweep, banded y-sweep, wave-speed maxima
    fused into the stage epilogue, step end merged into the next reduction),
    every cell against the oracle's two steps."""
    P, q0 = W.quadrants_2d(0, 2048)
    q = torch.from_numpy(q0).to(dev)
    with Ctx(P) as ctx:
        info = ctx.solve(q, 0.0, 2)
    orc.set_threads(16)
    ref, steps, t, st = orc.solve(P, q0, 0.0, 2)
    assert st == 0 and steps == 2 and info["steps"] == 2
    assert abs(info["t"] - t) <= 1e-14 * t
    assert_close(q.cpu().numpy(), ref, 1e-10, "2048^2, two steps")
