"""WENO-ZA6 oracle: TEST INFRASTRUCTURE ONLY.

ctypes front end of ``liboracle_za.so`` (built from ``za_oracle.cpp`` by
``oracle/build.py``), a plain, slow FP64 / FP32 / quad CPU implementation
written from the paper (arXiv 2603.26272).  Only the test-suite, the smoke
check and the benchmark's CPU-baseline leg may import this package; the
product path never does, and this package imports nothing from it.

Problem descriptions are duck-typed: any object (or dict) with the fields
dim, system, nx, ny, xlo, xhi, ylo, yhi, bc_x, bc_y, gamma, adv_speed, cfl,
dt_rule, precision (1 = FP32 reconstruction), p, eps, affine_invariant, mu0,
lf, linear_weights.  State arrays are float64 numpy arrays in SoA layout
[m][ny][nx] of point values at the cell centres.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle_za.so")
_lib = None

SYS_ADVECTION, SYS_EULER, SYS_BURGERS, SYS_BUCKLEY = 0, 1, 2, 3


class _Problem(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("system", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
        ("xlo", C.c_double), ("xhi", C.c_double), ("ylo", C.c_double), ("yhi", C.c_double),
        ("bc_x", C.c_int32), ("bc_y", C.c_int32),
        ("gamma", C.c_double),
        ("adv_speed", C.c_double * 2),
        ("cfl", C.c_double),
        ("dt_rule", C.c_int32),
        ("recon_fp32", C.c_int32),
        ("p", C.c_double), ("eps", C.c_double),
        ("ai", C.c_int32),
        ("mu0", C.c_double),
        ("lf", C.c_int32),
        ("linear_weights", C.c_int32),
        ("order", C.c_int32),
        ("pp_limiter", C.c_int32),
        ("alt_tau", C.c_int32),
        ("weight_L", C.c_double),
        ("weight_q", C.c_double),
    ]


_DP = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        L.orc_recon.restype = C.c_double
        L.orc_recon.argtypes = [_DP, C.c_double, C.c_double, C.c_int, C.c_double, C.c_int, _DP]
        L.orc_recon_alt.restype = C.c_double
        L.orc_recon_alt.argtypes = [_DP, C.c_double, C.c_double, C.c_int, C.c_double, _DP]
        L.orc_recon_f32.restype = C.c_double
        L.orc_recon_f32.argtypes = [_DP, C.c_double, C.c_double, C.c_int, C.c_double, C.c_int]
        L.orc_recon_q.restype = C.c_double
        L.orc_recon_q.argtypes = [C.POINTER(C.c_char_p), C.c_double, C.c_double, C.c_int,
                                  C.c_double, C.c_char_p, C.c_int]
        L.orc_critical_point_test.restype = C.c_double
        L.orc_critical_point_test.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_double,
                                              C.c_int, C.c_double, C.c_int]
        PP = C.POINTER(_Problem)
        L.orc_ncomp.restype = C.c_int
        L.orc_ncomp.argtypes = [PP]
        L.orc_wave_speeds.restype = C.c_int
        L.orc_wave_speeds.argtypes = [PP, _DP, _DP, _DP]
        L.orc_fluxes.restype = C.c_int
        L.orc_fluxes.argtypes = [PP, _DP, _DP, _DP]
        L.orc_fluxes_lines.restype = C.c_int
        L.orc_fluxes_lines.argtypes = [PP, _DP, C.c_int, C.POINTER(C.c_int), C.c_int, _DP]
        L.orc_rhs.restype = C.c_int
        L.orc_rhs.argtypes = [PP, _DP, _DP]
        L.orc_cfl_dt.restype = C.c_double
        L.orc_cfl_dt.argtypes = [PP, _DP]
        L.orc_step.restype = C.c_int
        L.orc_step.argtypes = [PP, _DP, C.c_double, _DP]
        L.orc_solve.restype = C.c_int
        L.orc_solve.argtypes = [PP, _DP, C.c_double, C.c_int64, C.POINTER(C.c_int64), _DP]
        L.orc_count_ops.restype = C.c_int64
        L.orc_count_ops.argtypes = [PP, _DP, C.c_int, C.POINTER(C.c_int64)]
        L.orc_euler_eigen.restype = None
        L.orc_euler_eigen.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                      C.c_double, C.c_double, _DP, _DP]
        L.orc_roe_state.restype = None
        L.orc_roe_state.argtypes = [C.c_int, C.c_double, _DP, _DP, _DP]
        L.orc_set_order_tables.restype = C.c_int
        L.orc_set_order_tables.argtypes = [C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.c_int]
        L.orc_recon_lq.restype = C.c_double
        L.orc_recon_lq.argtypes = [_DP, C.c_double, C.c_double, C.c_int, C.c_double, C.c_double, C.c_double,
                                   _DP]
        L.orc_recon_r_lq.restype = C.c_double
        L.orc_recon_r_lq.argtypes = [C.c_int, _DP, C.c_double, C.c_double, C.c_int, C.c_double, C.c_double,
                                     C.c_double, _DP]
        L.orc_recon_r.restype = C.c_double
        L.orc_recon_r.argtypes = [C.c_int, _DP, C.c_double, C.c_double, C.c_int, C.c_double, C.c_int,
                                  C.c_int, _DP]
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.restype = C.c_int
        L.orc_get_threads.argtypes = []
        _lib = L
    return _lib


def _get(pb, name, default=None):
    if isinstance(pb, dict):
        return pb.get(name, default)
    return getattr(pb, name, default)


def _problem(pb) -> _Problem:
    P = _Problem()
    P.dim = int(_get(pb, "dim", 1))
    P.system = int(_get(pb, "system", SYS_EULER))
    P.nx = int(_get(pb, "nx"))
    P.ny = int(_get(pb, "ny", 1))
    P.xlo = float(_get(pb, "xlo", 0.0)); P.xhi = float(_get(pb, "xhi", 1.0))
    P.ylo = float(_get(pb, "ylo", 0.0)); P.yhi = float(_get(pb, "yhi", 1.0))
    P.bc_x = int(_get(pb, "bc_x", 1)); P.bc_y = int(_get(pb, "bc_y", 1))
    P.gamma = float(_get(pb, "gamma", 1.4))
    a = _get(pb, "adv_speed", (1.0, 0.0))
    P.adv_speed[0] = float(a[0]); P.adv_speed[1] = float(a[1])
    P.cfl = float(_get(pb, "cfl", 0.5))
    P.dt_rule = int(_get(pb, "dt_rule", 0))
    P.recon_fp32 = int(_get(pb, "precision", 0))
    P.p = float(_get(pb, "p", 1.0))
    P.eps = float(_get(pb, "eps", 1e-40))
    P.ai = int(_get(pb, "affine_invariant", 0))
    P.mu0 = float(_get(pb, "mu0", 1e-40))
    P.lf = int(_get(pb, "lf", 0))
    P.linear_weights = int(_get(pb, "linear_weights", 0))
    P.order = int(_get(pb, "order", 3))
    P.pp_limiter = int(_get(pb, "pp_limiter", 0))
    P.alt_tau = int(_get(pb, "alt_tau", 0))
    P.weight_L = float(_get(pb, "weight_L", 1.0))
    P.weight_q = float(_get(pb, "weight_q", 1.0))
    _ensure_order(P.order)
    return P


_orders_set = set()


def _ensure_order(r: int) -> None:
    """Hand the exact tables of the order-2r scheme to the C oracle once."""
    if r in _orders_set or not (2 <= r <= 6):
        return
    from . import coeffs
    pairs = coeffs.flat_rationals(r)
    n = len(pairs)
    num = (C.c_int64 * n)(*[a for a, _ in pairs])
    den = (C.c_int64 * n)(*[b for _, b in pairs])
    if lib().orc_set_order_tables(int(r), num, den, n) != 0:
        raise RuntimeError(f"oracle rejected the order-{2 * r} tables")
    _orders_set.add(r)


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_DP)


def ncomp(pb) -> int:
    return lib().orc_ncomp(C.byref(_problem(pb)))


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return lib().orc_get_threads()


def recon(v6, p=1.0, eps=1e-40, ai=0, mu0=1e-40, linear=0, detail=False):
    """O1: one positive split reconstruction from (f_{i-2}, .., f_{i+3})."""
    v = np.ascontiguousarray(v6, dtype=np.float64)
    assert v.shape == (6,)
    if detail:
        d = np.zeros(15)
        r = lib().orc_recon(_ptr(v), p, eps, ai, mu0, linear, _ptr(d))
        return r, {"q": d[0:4].copy(), "beta": d[4:9].copy(), "tau": d[9], "mu": d[10],
                   "omega": d[11:15].copy()}
    return lib().orc_recon(_ptr(v), p, eps, ai, mu0, linear, None)


def recon_r(r, v, p=1.0, eps=1e-40, ai=0, mu0=1e-40, linear=0, prec=0, detail=False):
    """O1 for the order-2r scheme from v = (f_{i-r+1}, .., f_{i+r}); prec 0 FP64,
    1 FP32, 2 quad (rounded to FP64)."""
    _ensure_order(int(r))
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert v.shape == (2 * r,)
    if detail:
        d = np.zeros(3 * r + 6)
        out = lib().orc_recon_r(int(r), _ptr(v), p, eps, ai, mu0, linear, prec, _ptr(d))
        return out, {"q": d[0:r + 1].copy(), "beta": d[r + 1:2 * r + 1].copy(), "beta_d": d[2 * r + 1],
                     "beta_r": d[2 * r + 2], "tau": d[2 * r + 3], "mu": d[2 * r + 4],
                     "omega": d[2 * r + 5:3 * r + 6].copy()}
    return lib().orc_recon_r(int(r), _ptr(v), p, eps, ai, mu0, linear, prec, None)


def recon_lq(v6, L, q, p=1.0, eps=1e-40, ai=0, mu0=1e-40, detail=False):
    """O1 with the weight parameters L and q of eq:weights_unnormalized."""
    v = np.ascontiguousarray(v6, dtype=np.float64)
    assert v.shape == (6,)
    if detail:
        d = np.zeros(15)
        r = lib().orc_recon_lq(_ptr(v), p, eps, ai, mu0, L, q, _ptr(d))
        return r, {"q": d[0:4].copy(), "beta": d[4:9].copy(), "tau": d[9], "mu": d[10],
                   "omega": d[11:15].copy()}
    return lib().orc_recon_lq(_ptr(v), p, eps, ai, mu0, L, q, None)


def recon_r_lq(r, v, L, q, p=1.0, eps=1e-40, ai=0, mu0=1e-40):
    """O1 of the order-2r scheme (FP64) with the weight parameters L and q."""
    _ensure_order(int(r))
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert v.shape == (2 * r,)
    return lib().orc_recon_r_lq(int(r), _ptr(v), p, eps, ai, mu0, L, q, None)


def recon_alt(v6, p=1.0, eps=1e-40, ai=0, mu0=1e-40, detail=False):
    """O1 with the alternative global indicator tau' (eq:GSI_alt)."""
    v = np.ascontiguousarray(v6, dtype=np.float64)
    assert v.shape == (6,)
    if detail:
        d = np.zeros(15)
        r = lib().orc_recon_alt(_ptr(v), p, eps, ai, mu0, _ptr(d))
        return r, {"q": d[0:4].copy(), "beta": d[4:9].copy(), "tau": d[9], "mu": d[10],
                   "omega": d[11:15].copy()}
    return lib().orc_recon_alt(_ptr(v), p, eps, ai, mu0, None)


def recon_f32(v6, p=1.0, eps=1e-20, ai=0, mu0=1e-8, linear=0):
    v = np.ascontiguousarray(v6, dtype=np.float64)
    return lib().orc_recon_f32(_ptr(v), p, eps, ai, mu0, linear)


def recon_quad(v6_strings, p=1.0, eps=1e-40, ai=0, mu0=1e-100):
    """O1 in quad precision; inputs and result as decimal strings."""
    arr = (C.c_char_p * 6)(*[s.encode() for s in v6_strings])
    buf = C.create_string_buffer(64)
    lib().orc_recon_q(arr, p, eps, ai, mu0, buf, 64)
    return buf.value.decode()


def critical_point_test(ncp, inv_dx, p=1.0, eps_mode=0, eps=1e-40, ai=0, mu0=1e-100, quad=True):
    """Section 3.1 operator test: L-infinity error of (h_{j+1/2}-h_{j-1/2})/dx
    against f'(x_j) for f = x^(ncp+1) exp(0.75 x) on [-1, 1]."""
    return lib().orc_critical_point_test(int(ncp), int(inv_dx), float(p), int(eps_mode),
                                         float(eps), int(ai), float(mu0), 1 if quad else 0)


def _state(pb, q):
    q = np.ascontiguousarray(q, dtype=np.float64)
    return q


def wave_speeds(pb, q):
    P = _problem(pb)
    q = _state(pb, q)
    a = np.zeros(8); s = np.zeros(2)
    st = lib().orc_wave_speeds(C.byref(P), _ptr(q), _ptr(a), _ptr(s))
    return a.reshape(2, 4), s, st


def fluxes(pb, q):
    """Interface fluxes: fx [m][ny][nx+1], fy [m][ny+1][nx] (2D) or None."""
    P = _problem(pb)
    q = _state(pb, q)
    m = lib().orc_ncomp(C.byref(P))
    fx = np.zeros((m, P.ny, P.nx + 1))
    fy = np.zeros((m, P.ny + 1, P.nx)) if P.dim == 2 else None
    st = lib().orc_fluxes(C.byref(P), _ptr(q), _ptr(fx), _ptr(fy) if fy is not None else None)
    return fx, fy, st


def fluxes_lines(pb, q, direction, lines):
    """Fluxes of selected rows (direction 0, [l][m][nx+1]) or columns
    (direction 1, [l][m][ny+1]) with the global LF speeds of q."""
    P = _problem(pb)
    q = _state(pb, q)
    m = lib().orc_ncomp(C.byref(P))
    n = P.nx if direction == 0 else P.ny
    ln = np.ascontiguousarray(lines, dtype=np.int32)
    out = np.zeros((len(ln), m, n + 1))
    st = lib().orc_fluxes_lines(C.byref(P), _ptr(q), int(direction),
                                ln.ctypes.data_as(C.POINTER(C.c_int)), len(ln), _ptr(out))
    return out, st


def rhs(pb, q):
    P = _problem(pb)
    q = _state(pb, q)
    out = np.zeros_like(q)
    st = lib().orc_rhs(C.byref(P), _ptr(q), _ptr(out))
    return out, st


def cfl_dt(pb, q):
    P = _problem(pb)
    q = _state(pb, q)
    return lib().orc_cfl_dt(C.byref(P), _ptr(q))


def step(pb, q, dt=0.0):
    """One SSP-RK3 step on a copy of q; dt <= 0 takes the CFL step."""
    P = _problem(pb)
    q = np.array(q, dtype=np.float64, copy=True, order="C")
    used = C.c_double(0)
    st = lib().orc_step(C.byref(P), _ptr(q), float(dt), C.byref(used))
    return q, used.value, st


def solve(pb, q, t_final, max_steps=0):
    """Integrate a copy of q; returns (q, steps, t, status)."""
    P = _problem(pb)
    q = np.array(q, dtype=np.float64, copy=True, order="C")
    steps = C.c_int64(0); t = C.c_double(0)
    st = lib().orc_solve(C.byref(P), _ptr(q), float(t_final), int(max_steps), C.byref(steps), C.byref(t))
    return q, steps.value, t.value, st


def count_ops(pb, q, dir_mask=3):
    """Algorithmic op counts of the interface fluxes of one RHS (interface
    work + physical flux per cell incl. ghosts).  Returns (n_interfaces, dict)."""
    P = _problem(pb)
    q = _state(pb, q)
    cnt = (C.c_int64 * 5)()
    nir = lib().orc_count_ops(C.byref(P), _ptr(q), int(dir_mask), cnt)
    return nir, {"add": cnt[0], "mul": cnt[1], "div": cnt[2], "sqrt": cnt[3], "other": cnt[4]}


def roe_state(m, gamma, QL, QR):
    """(u~, v~, H~, c~): the Roe-averaged state of cells QL, QR (conserved
    variables, m = 3 or 4) that the interface fluxes project with."""
    ql = np.ascontiguousarray(QL, dtype=np.float64)
    qr = np.ascontiguousarray(QR, dtype=np.float64)
    out = np.zeros(4)
    lib().orc_roe_state(int(m), float(gamma), _ptr(ql), _ptr(qr), _ptr(out))
    return tuple(float(x) for x in out)


def euler_eigen(m, direction, gamma, u, v, H, c):
    """(R, L) eigenvector matrices of the characteristic projection."""
    Rm = np.zeros(m * m); Lm = np.zeros(m * m)
    lib().orc_euler_eigen(int(m), int(direction), float(gamma), float(u), float(v), float(H),
                          float(c), _ptr(Rm), _ptr(Lm))
    return Rm.reshape(m, m), Lm.reshape(m, m)
