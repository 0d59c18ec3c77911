"""Python binding of libza (ctypes; argument marshalling only).

Every computation runs in libza's HIP kernels.  PyTorch supplies device
memory and streams: state tensors are float64 CUDA tensors of shape
(m, ny, nx), contiguous, on the context's device.  The functions mirror the
C ABI in include/za.h (za_rhs, za_rhs_fluxes, za_step, za_solve, ...).

There is no fallback: if libza.so is missing or the HIP runtime cannot be
reached, loading raises.
"""
import ctypes as C
import os
from typing import Optional, Tuple

from .problem import Problem

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libza.so")

ZA_OK, ZA_ERR_ARG, ZA_ERR_NOMEM, ZA_ERR_DEVICE, ZA_ERR_NONFINITE, ZA_ERR_UNSUPPORTED, ZA_ERR_BUSY = range(7)

EXPORTED = [
    "za_ctx_create", "za_ctx_destroy", "za_ctx_set_stream", "za_state_count", "za_workspace_bytes",
    "za_rhs", "za_rhs_fluxes", "za_rhs_noalloc", "za_step", "za_solve", "za_conserved_sums", "za_status_str",
    "za_ctx_last_error", "za_ctx_set_timing", "za_ctx_kernel_times",
    "za_server_create", "za_server_submit", "za_server_poll", "za_server_drain", "za_server_destroy",
]


class ZaProblem(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("system", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
        ("xlo", C.c_double), ("xhi", C.c_double), ("ylo", C.c_double), ("yhi", C.c_double),
        ("bc_x", C.c_int32), ("bc_y", C.c_int32),
        ("gamma", C.c_double),
        ("adv_speed", C.c_double * 2),
        ("cfl", C.c_double),
        ("dt_rule", C.c_int32),
        ("precision", C.c_int32),
        ("p", C.c_double),
        ("eps", C.c_double),
        ("affine_invariant", C.c_int32),
        ("mu0", C.c_double),
        ("lf", C.c_int32),
        ("linear_weights", C.c_int32),
        ("order", C.c_int32),
        ("pp_limiter", C.c_int32),
        ("alt_tau", C.c_int32),
        ("weight_L", C.c_double),
        ("weight_q", C.c_double),
    ]

    @classmethod
    def from_problem(cls, P: Problem) -> "ZaProblem":
        z = cls()
        for name, _ in cls._fields_:
            if name == "adv_speed":
                z.adv_speed[0] = float(P.adv_speed[0])
                z.adv_speed[1] = float(P.adv_speed[1])
            else:
                setattr(z, name, getattr(P, name))
        return z


class ZaSolveInfo(C.Structure):
    _fields_ = [("steps", C.c_int64), ("t", C.c_double), ("dt_min", C.c_double),
                ("dt_max", C.c_double), ("nonfinite_step", C.c_int64)]


class ZaReqStats(C.Structure):
    _fields_ = [("arrival_ns", C.c_int64), ("admit_ns", C.c_int64), ("finish_ns", C.c_int64),
                ("steps", C.c_int64), ("interfaces", C.c_int64), ("status", C.c_int32)]


class ZaError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        super().__init__(f"libza status {status}: {msg}")
        self.status = status


_lib = None


def lib() -> C.CDLL:
    """Load libza.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    vp, dp = C.c_void_p, C.POINTER(C.c_double)
    PP = C.POINTER(ZaProblem)
    L.za_ctx_create.argtypes = [PP, vp, C.POINTER(vp)]
    L.za_ctx_destroy.argtypes = [vp]
    L.za_ctx_set_stream.argtypes = [vp, vp]
    L.za_state_count.argtypes = [PP]
    L.za_state_count.restype = C.c_size_t
    L.za_workspace_bytes.argtypes = [PP]
    L.za_workspace_bytes.restype = C.c_size_t
    L.za_rhs.argtypes = [vp, vp, vp]
    L.za_rhs_fluxes.argtypes = [vp, vp, vp, vp]
    L.za_rhs_noalloc.argtypes = [PP, vp, vp, vp]
    L.za_step.argtypes = [vp, vp, C.c_double, dp]
    L.za_solve.argtypes = [vp, vp, C.c_double, C.c_int64, C.POINTER(ZaSolveInfo)]
    L.za_conserved_sums.argtypes = [vp, vp, dp]
    L.za_status_str.argtypes = [C.c_int]
    L.za_status_str.restype = C.c_char_p
    L.za_ctx_last_error.argtypes = [vp]
    L.za_ctx_last_error.restype = C.c_char_p
    L.za_ctx_set_timing.argtypes = [vp, C.c_int32]
    L.za_ctx_kernel_times.argtypes = [vp, dp, C.POINTER(C.c_int64)]
    L.za_server_create.argtypes = [C.c_size_t, C.c_int32, C.c_int32, C.POINTER(vp)]
    L.za_server_submit.argtypes = [vp, PP, dp, C.c_int64, C.POINTER(C.c_int64)]
    L.za_server_poll.argtypes = [vp, C.c_int64, C.POINTER(C.c_int32), dp, C.POINTER(ZaReqStats)]
    L.za_server_drain.argtypes = [vp]
    L.za_server_destroy.argtypes = [vp]
    for name in EXPORTED:
        getattr(L, name)          # raises if a declared entry point is missing
    _lib = L
    return L


def status_str(st: int) -> str:
    return lib().za_status_str(int(st)).decode()


def state_count(P: Problem) -> int:
    z = ZaProblem.from_problem(P)
    return int(lib().za_state_count(C.byref(z)))


def workspace_bytes(P: Problem) -> int:
    z = ZaProblem.from_problem(P)
    return int(lib().za_workspace_bytes(C.byref(z)))


def _check_state(P: Problem, t, name="q"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float64")
    return t


def rhs_noalloc(P: Problem, q, out=None, stream=None):
    """za_rhs_noalloc: L(q) without a context and without any device
    allocation by the library (the output tensor, if not given, is
    allocated here by PyTorch).  Asynchronous on `stream` (default: the
    current stream)."""
    import torch
    _check_state(P, q, "q")
    out = torch.empty_like(q) if out is None else out
    _check_state(P, out, "rhs")
    if tuple(q.shape) != tuple(P.shape) or tuple(out.shape) != tuple(P.shape):
        raise ValueError(f"q and rhs must have shape {tuple(P.shape)}")
    s = (stream or torch.cuda.current_stream()).cuda_stream
    z = ZaProblem.from_problem(P)
    st = lib().za_rhs_noalloc(C.byref(z), C.c_void_p(q.data_ptr()), C.c_void_p(out.data_ptr()), C.c_void_p(s))
    if st != ZA_OK:
        raise ZaError(st, status_str(st))
    return out


class Context:
    """A libza context for one problem shape on the current device/stream."""

    def __init__(self, P: Problem, stream=None):
        import torch
        self.P = P
        self._torch = torch
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        self._z = ZaProblem.from_problem(P)
        h = C.c_void_p()
        st = lib().za_ctx_create(C.byref(self._z), C.c_void_p(self._stream.cuda_stream), C.byref(h))
        if st != ZA_OK:
            raise ZaError(st, status_str(st))
        self._h = h

    # -- helpers ------------------------------------------------------------
    def _err(self, st):
        if st != ZA_OK:
            msg = lib().za_ctx_last_error(self._h).decode()
            raise ZaError(st, f"{status_str(st)} {msg}")

    def _expect(self, t, shape, name):
        _check_state(self.P, t, name)
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        return C.c_void_p(t.data_ptr())

    @property
    def shape(self):
        return self.P.shape

    # -- C ABI -------------------------------------------------------------------
    def rhs(self, q, out=None):
        out = self._torch.empty_like(q) if out is None else out
        self._err(lib().za_rhs(self._h, self._expect(q, self.shape, "q"), self._expect(out, self.shape, "rhs")))
        return out

    def rhs_fluxes(self, q) -> Tuple[object, Optional[object]]:
        P = self.P
        fx = self._torch.empty((P.m, P.ny, P.nx + 1), dtype=self._torch.float64, device=q.device)
        fy = None
        if P.dim == 2:
            fy = self._torch.empty((P.m, P.ny + 1, P.nx), dtype=self._torch.float64, device=q.device)
        self._err(lib().za_rhs_fluxes(self._h, self._expect(q, self.shape, "q"), C.c_void_p(fx.data_ptr()),
                                      C.c_void_p(fy.data_ptr()) if fy is not None else None))
        return fx, fy

    def step(self, q, dt: float = 0.0, sync: bool = False) -> Optional[float]:
        used = C.c_double(0.0)
        st = lib().za_step(self._h, self._expect(q, self.shape, "q"), float(dt), C.byref(used) if sync else None)
        self._err(st)
        return used.value if sync else None

    def solve(self, q, t_final: float = 0.0, max_steps: int = 0, check: bool = True) -> dict:
        info = ZaSolveInfo()
        st = lib().za_solve(self._h, self._expect(q, self.shape, "q"), float(t_final), int(max_steps),
                            C.byref(info))
        res = {"status": st, "steps": info.steps, "t": info.t, "dt_min": info.dt_min,
               "dt_max": info.dt_max, "nonfinite_step": info.nonfinite_step}
        if check and st != ZA_OK:
            self._err(st)
        return res

    def conserved_sums(self, q):
        out = (C.c_double * self.P.m)()
        self._err(lib().za_conserved_sums(self._h, self._expect(q, self.shape, "q"), out))
        return [out[i] for i in range(self.P.m)]

    def set_timing(self, on: bool = True):
        self._err(lib().za_ctx_set_timing(self._h, 1 if on else 0))

    def kernel_times(self):
        """Average per-launch device ms of (x-sweep, y-sweep, wave-speed) and counts."""
        avg = (C.c_double * 3)()
        cnt = (C.c_int64 * 3)()
        self._err(lib().za_ctx_kernel_times(self._h, avg, cnt))
        return [avg[i] for i in range(3)], [cnt[i] for i in range(3)]

    def set_stream(self, stream):
        self._stream = stream
        self._err(lib().za_ctx_set_stream(self._h, C.c_void_p(stream.cuda_stream)))

    def close(self):
        if getattr(self, "_h", None):
            lib().za_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Server:
    """Continuous-batching solve server (za_server_*): requests are admitted
    by HBM footprint and advanced together by batched RK3 steps."""

    def __init__(self, hbm_budget_bytes: int = 4 << 30, max_slots: int = 64, device: int = 0):
        h = C.c_void_p()
        st = lib().za_server_create(C.c_size_t(int(hbm_budget_bytes)), int(max_slots), int(device), C.byref(h))
        if st != ZA_OK:
            raise ZaError(st, status_str(st))
        self._h = h

    def submit(self, P: Problem, q0, n_steps: int) -> int:
        import numpy as np
        q = np.ascontiguousarray(q0, dtype=np.float64)
        if q.shape != tuple(P.shape):
            raise ValueError(f"q0 has shape {q.shape}, expected {tuple(P.shape)}")
        z = ZaProblem.from_problem(P)
        rid = C.c_int64(0)
        st = lib().za_server_submit(self._h, C.byref(z), q.ctypes.data_as(C.POINTER(C.c_double)), int(n_steps),
                                    C.byref(rid))
        if st != ZA_OK:
            raise ZaError(st, status_str(st))
        return rid.value

    def poll(self, rid: int, P: Optional[Problem] = None):
        """(done, status, q or None, stats).  With P given and the request
        finished, the result is returned and the request released."""
        import numpy as np
        done = C.c_int32(0)
        stats = ZaReqStats()
        out = np.empty(P.shape, dtype=np.float64) if P is not None else None
        st = lib().za_server_poll(self._h, int(rid), C.byref(done),
                                  out.ctypes.data_as(C.POINTER(C.c_double)) if out is not None else None,
                                  C.byref(stats))
        if st == ZA_ERR_ARG:
            raise ZaError(st, "unknown request")
        s = {"arrival_ns": stats.arrival_ns, "admit_ns": stats.admit_ns, "finish_ns": stats.finish_ns,
             "steps": stats.steps, "interfaces": stats.interfaces, "status": stats.status}
        if not done.value:
            return False, ZA_OK, None, s
        return True, stats.status, out, s

    def drain(self):
        st = lib().za_server_drain(self._h)
        if st != ZA_OK:
            raise ZaError(st, status_str(st))

    def close(self):
        if getattr(self, "_h", None):
            lib().za_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
