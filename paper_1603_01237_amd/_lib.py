"""ctypes binding of libism (argument marshalling only; every step runs in the HIP library).

The library must be built (``python -m paper_1603_01237_amd.build``); importing this
module raises if ``libism.so`` is missing -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as ct
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libism.so")

ISM_OK, ISM_E_ARG, ISM_E_NOMEM, ISM_E_DEVICE, ISM_E_STATE, ISM_E_NUMERIC, ISM_E_UNSUPPORTED, ISM_E_BUDGET = range(8)
FP64, FP32_MIXED = 0, 1
STATE, GATE, DENSITY = 0, 1, 2
KINDS = {"state": STATE, "gate": GATE, "density": DENSITY}
STEP_EXP, STEP_CN = 0, 1
STEP_MAPS = {"exp": STEP_EXP, "cn": STEP_CN}
PRECISIONS = {"fp64": FP64, "fp32": FP32_MIXED, "fp32_mixed": FP32_MIXED}

EXPORTED = [
    "ism_default_options", "ism_problem_create", "ism_problem_create_gpe", "ism_problem_destroy",
    "ism_set_controls", "ism_get_controls", "ism_forward", "ism_adjoint", "ism_gradient",
    "ism_iterate", "ism_iterate_inner", "ism_iterate_static", "ism_iterate_newton", "ism_fidelity", "ism_problem_info", "ism_taylor_params", "ism_status_string", "ism_problem_footprint",
    "ism_set_timing", "ism_kernel_times",
    "ism_server_clock", "ism_server_create", "ism_server_submit", "ism_server_progress",
    "ism_server_poll", "ism_server_take", "ism_server_stats_get", "ism_server_destroy",
]
ISM_STATIC_HIST_MAX = 131072       # doubles in the fixed J-history array of ism_iterate_static
REQ_FINITE, REQ_GPE = 0, 1
REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = range(4)


class IsmError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {status_string(code)} (status {code})")
        self.code = code


class Options(ct.Structure):
    _fields_ = [("precision", ct.c_int), ("kind", ct.c_int), ("batch", ct.c_int),
                ("h0_batched", ct.c_int), ("alpha", ct.POINTER(ct.c_double)),
                ("alpha_len", ct.c_int), ("device", ct.c_int), ("stream", ct.c_void_p),
                ("io_device", ct.c_int), ("alloc_async", ct.c_int), ("step_map", ct.c_int),
                ("launch_per_pass", ct.c_int), ("gpe_frozen", ct.c_int)]


class Info(ct.Structure):
    _fields_ = [("path", ct.c_int), ("d", ct.c_int), ("n_ctrl", ct.c_int), ("K", ct.c_int),
                ("N", ct.c_int), ("batch", ct.c_int), ("precision", ct.c_int), ("kind", ct.c_int),
                ("ell_width", ct.c_int), ("device_bytes", ct.c_size_t), ("taylor_m", ct.c_int),
                ("taylor_S", ct.c_int)]


class KernelTime(ct.Structure):
    _fields_ = [("name", ct.c_char_p), ("launches", ct.c_int), ("total_ms", ct.c_double)]


class Request(ct.Structure):
    _fields_ = [("model", ct.c_int), ("kind", ct.c_int), ("precision", ct.c_int),
                ("d", ct.c_int), ("n_ctrl", ct.c_int), ("H0", ct.c_void_p), ("Hc", ct.c_void_p),
                ("n_grid", ct.c_int), ("L", ct.c_double), ("g", ct.c_double), ("V2", ct.c_double),
                ("V0", ct.c_void_p), ("V1", ct.c_void_p), ("psi0", ct.c_void_p),
                ("target", ct.c_void_p), ("T", ct.c_double), ("K", ct.c_int), ("N", ct.c_int),
                ("u0", ct.c_void_p), ("max_iter", ct.c_int), ("rho", ct.c_double),
                ("fid_stop", ct.c_double)]


class Result(ct.Structure):
    _fields_ = [("state", ct.c_int), ("status", ct.c_int), ("iters", ct.c_int),
                ("J", ct.c_double), ("F", ct.c_double), ("t_arrival", ct.c_double),
                ("t_admit", ct.c_double), ("t_done", ct.c_double), ("device_bytes", ct.c_size_t)]


class ServerStats(ct.Structure):
    _fields_ = [("submitted", ct.c_uint64), ("completed", ct.c_uint64), ("failed", ct.c_uint64),
                ("queued", ct.c_int), ("running", ct.c_int), ("bytes_in_use", ct.c_size_t),
                ("bytes_peak", ct.c_size_t), ("busy_s", ct.c_double), ("groups", ct.c_uint64),
                ("merged", ct.c_uint64)]


_lib = None


def lib():
    """Load libism.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not built; run python -m paper_1603_01237_amd.build")
    # PyTorch ships its own HIP runtime under the same soname (libamdhip64.so.7).  Loading
    # torch first makes libism bind to that runtime, so one process never holds two HIP
    # runtimes (device memory and streams from torch then work with libism handles).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ct.CDLL(LIB_PATH)
    dp = ct.POINTER(ct.c_double)
    vp = ct.c_void_p
    L.ism_default_options.argtypes = [ct.POINTER(Options)]
    L.ism_default_options.restype = None
    L.ism_problem_create.argtypes = [ct.POINTER(vp), ct.c_int, ct.c_int, vp, vp, vp, vp,
                                     ct.c_double, ct.c_int, ct.c_int, ct.POINTER(Options)]
    L.ism_problem_create_gpe.argtypes = [ct.POINTER(vp), ct.c_int, ct.c_double, ct.c_double, vp,
                                         vp, ct.c_double, vp, vp, ct.c_double, ct.c_int, ct.c_int,
                                         ct.POINTER(Options)]
    L.ism_problem_destroy.argtypes = [vp]
    L.ism_problem_destroy.restype = None
    for name in ("ism_set_controls", "ism_get_controls", "ism_forward", "ism_adjoint",
                 "ism_gradient"):
        getattr(L, name).argtypes = [vp, vp]
    L.ism_iterate.argtypes = [vp, ct.c_int, ct.c_double, ct.c_double, vp, ct.POINTER(ct.c_int)]
    L.ism_iterate_static.argtypes = [vp, ct.c_int, ct.c_double, ct.c_double, vp,
                                     ct.POINTER(ct.c_int)]
    L.ism_iterate_inner.argtypes = [vp, ct.c_int, ct.c_int, ct.c_double, ct.c_double, ct.c_double,
                                    vp, vp, ct.POINTER(ct.c_int)]
    L.ism_iterate_newton.argtypes = [vp, ct.c_int, ct.c_int, ct.c_double, ct.c_double, vp,
                                     ct.POINTER(ct.c_int)]
    L.ism_fidelity.argtypes = [vp, vp, vp]
    L.ism_problem_info.argtypes = [vp, ct.POINTER(Info)]
    L.ism_taylor_params.argtypes = [vp, ct.POINTER(ct.c_int), ct.POINTER(ct.c_int)]
    L.ism_taylor_params.restype = ct.c_int
    L.ism_status_string.argtypes = [ct.c_int]
    L.ism_status_string.restype = ct.c_char_p
    L.ism_set_timing.argtypes = [vp, ct.c_int]
    L.ism_set_timing.restype = ct.c_int
    L.ism_kernel_times.argtypes = [vp, ct.POINTER(KernelTime), ct.c_int, ct.POINTER(ct.c_int)]
    L.ism_kernel_times.restype = ct.c_int
    L.ism_problem_footprint.argtypes = [ct.c_int] * 7 + [ct.c_int]
    L.ism_problem_footprint.restype = ct.c_size_t
    L.ism_server_clock.argtypes = []
    L.ism_server_clock.restype = ct.c_double
    L.ism_server_create.argtypes = [ct.POINTER(vp), ct.c_int, ct.c_size_t, ct.c_int, ct.c_int]
    L.ism_server_submit.argtypes = [vp, ct.POINTER(Request), ct.c_double,
                                    ct.POINTER(ct.c_uint64)]
    L.ism_server_progress.argtypes = [vp, ct.POINTER(ct.c_int), ct.POINTER(ct.c_int)]
    L.ism_server_poll.argtypes = [vp, ct.c_uint64, ct.POINTER(Result)]
    L.ism_server_take.argtypes = [vp, ct.c_uint64, ct.POINTER(Result), vp]
    L.ism_server_stats_get.argtypes = [vp, ct.POINTER(ServerStats)]
    L.ism_server_destroy.argtypes = [vp]
    L.ism_server_destroy.restype = None
    for name in ("ism_server_create", "ism_server_submit", "ism_server_progress",
                 "ism_server_poll", "ism_server_take", "ism_server_stats_get"):
        getattr(L, name).restype = ct.c_int
    for name in ("ism_problem_create", "ism_problem_create_gpe", "ism_set_controls",
                 "ism_get_controls", "ism_forward", "ism_adjoint", "ism_gradient", "ism_iterate",
                 "ism_iterate_inner", "ism_iterate_static", "ism_iterate_newton", "ism_fidelity",
                 "ism_problem_info"):
        getattr(L, name).restype = ct.c_int
    _lib = L
    return L


def status_string(code: int) -> str:
    return lib().ism_status_string(code).decode()


def _check(code: int, what: str):
    if code != ISM_OK:
        raise IsmError(code, what)


def _cptr(a: np.ndarray):
    return a.ctypes.data_as(ct.c_void_p)


def _as_c128(x, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
    if shape is not None and a.shape != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _handle_stream(stream, io_device, device):
    """(torch stream, raw stream pointer) for a new handle.  A handle exchanging device
    tensors gets a stream torch knows, so that callers (the autograd wrapper) can order it
    against torch's current stream: the caller's stream pointer wrapped as an external
    stream, or a new torch stream of default priority.  Host-I/O handles keep the caller's
    pointer, or NULL for a library-owned stream."""
    if not io_device:
        return None, stream
    import torch
    if stream is None:
        ts = torch.cuda.Stream(device=device)
    else:
        ts = torch.cuda.ExternalStream(int(stream), device=device)
    return ts, ts.cuda_stream


def footprint(d, n_ctrl, K, N, batch=1, kind=STATE, precision=FP64, gpe_grid=0) -> int:
    return int(lib().ism_problem_footprint(d, n_ctrl, K, N, batch, kind, precision, gpe_grid))


class Problem:
    """One libism handle.  Host I/O uses NumPy arrays; with ``io_device=True`` the
    controls, gradients and states are exchanged as device tensors (torch.cuda),
    passed by pointer."""

    def __init__(self, handle, shape_state, d, C, K, N, B, io_device, gpe_n=0, T=1.0):
        self._h = handle
        self.state_shape = shape_state
        self.d, self.C, self.K, self.N, self.B = d, C, K, N, B
        self.T = float(T)
        self.io_device = io_device
        self.gpe_n = gpe_n
        self.version = 0          # incremented whenever the controls are set
        self.torch_stream = None  # the handle's stream as a torch stream (io_device handles)

    # ------------------------------------------------------------------ creation
    @classmethod
    def create(cls, H0, Hc, psi0, target, T, K, N, precision="fp64", kind="state", batch=1,
               h0_batched=False, alpha=None, device=0, stream=None, io_device=False,
               step_map="exp", launch_per_pass=False):
        L = lib()
        Hc = _as_c128(Hc)
        C, d = Hc.shape[0], Hc.shape[-1]
        H0 = _as_c128(H0)
        if h0_batched and H0.shape != (batch, d, d):
            raise ValueError("batched H0 must have shape (batch, d, d)")
        kind_i = KINDS[kind] if isinstance(kind, str) else int(kind)
        sshape = (d, d) if kind_i in (GATE, DENSITY) else (d,)
        psi0 = _as_c128(psi0, sshape)
        target = _as_c128(target, sshape)
        o = Options()
        L.ism_default_options(ct.byref(o))
        o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        o.kind = kind_i
        o.batch = int(batch)
        o.h0_batched = 1 if h0_batched else 0
        al = None
        if alpha is not None:
            al = np.ascontiguousarray(np.atleast_1d(np.asarray(alpha, dtype=np.float64)))
            o.alpha = al.ctypes.data_as(ct.POINTER(ct.c_double))
            o.alpha_len = al.shape[0]
        o.device = int(device)
        tstream, stream = _handle_stream(stream, io_device, device)
        o.stream = stream
        o.io_device = 1 if io_device else 0
        o.step_map = STEP_MAPS[step_map] if isinstance(step_map, str) else int(step_map)
        o.launch_per_pass = 1 if launch_per_pass else 0
        h = ct.c_void_p()
        _check(L.ism_problem_create(ct.byref(h), d, C, _cptr(H0), _cptr(Hc), _cptr(psi0),
                                    _cptr(target), float(T), int(K), int(N), ct.byref(o)),
               "ism_problem_create")
        obj = cls(h, sshape, d, C, int(K), int(N), int(batch), io_device, T=T)
        obj.torch_stream = tstream
        return obj

    @classmethod
    def create_gpe(cls, n, L_box, g, V0, V1, V2, psi0, target, T, K, N, precision="fp64",
                   batch=1, device=0, stream=None, io_device=False, gpe_frozen=False):
        L = lib()
        V0 = np.ascontiguousarray(np.asarray(V0, dtype=np.float64))
        V1 = np.ascontiguousarray(np.asarray(V1, dtype=np.float64))
        psi0 = _as_c128(psi0, (n,))
        target = _as_c128(target, (n,))
        o = Options()
        L.ism_default_options(ct.byref(o))
        o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        o.batch = int(batch)
        o.device = int(device)
        tstream, stream = _handle_stream(stream, io_device, device)
        o.stream = stream
        o.io_device = 1 if io_device else 0
        o.gpe_frozen = 1 if gpe_frozen else 0
        h = ct.c_void_p()
        _check(L.ism_problem_create_gpe(ct.byref(h), int(n), float(L_box), float(g), _cptr(V0),
                                        _cptr(V1), float(V2), _cptr(psi0), _cptr(target),
                                        float(T), int(K), int(N), ct.byref(o)),
               "ism_problem_create_gpe")
        obj = cls(h, (n,), n, 1, int(K), int(N), int(batch), io_device, gpe_n=n, T=T)
        obj.torch_stream = tstream
        return obj

    # ------------------------------------------------------------------ lifetime
    def close(self):
        if self._h:
            lib().ism_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    # ------------------------------------------------------------------ helpers
    def _out(self, shape, dtype):
        if self.io_device:
            import torch
            tdt = torch.float64 if dtype == np.float64 else torch.complex128
            return torch.empty(shape, dtype=tdt, device="cuda")
        return np.empty(shape, dtype=dtype)

    @staticmethod
    def _ptr(a):
        if hasattr(a, "data_ptr"):
            return ct.c_void_p(a.data_ptr())
        return _cptr(a)

    # ------------------------------------------------------------------ API
    def set_controls(self, u):
        self.version += 1
        if self.io_device:
            if tuple(u.shape) != (self.B, self.K, self.C) or not u.is_contiguous():
                raise ValueError("controls must be a contiguous (B, K, C) float64 device tensor")
            _check(lib().ism_set_controls(self._h, self._ptr(u)), "ism_set_controls")
            return
        a = np.ascontiguousarray(np.asarray(u, dtype=np.float64)).reshape(self.B, self.K, self.C)
        _check(lib().ism_set_controls(self._h, _cptr(a)), "ism_set_controls")

    def get_controls(self):
        out = self._out((self.B, self.K, self.C), np.float64)
        _check(lib().ism_get_controls(self._h, self._ptr(out)), "ism_get_controls")
        return out

    def forward(self, want_state=True):
        out = self._out((self.B,) + self.state_shape, np.complex128) if want_state else None
        _check(lib().ism_forward(self._h, self._ptr(out) if out is not None else None), "ism_forward")
        return out

    def adjoint(self, want_state=True):
        out = self._out((self.B,) + self.state_shape, np.complex128) if want_state else None
        _check(lib().ism_adjoint(self._h, self._ptr(out) if out is not None else None), "ism_adjoint")
        return out

    def gradient(self):
        out = self._out((self.B, self.K, self.C), np.float64)
        _check(lib().ism_gradient(self._h, self._ptr(out)), "ism_gradient")
        return out

    def iterate(self, n_iter, rho, fid_stop=2.0, record=True):
        Jh = self._out((max(n_iter, 1), self.B), np.float64) if record else None
        done = ct.c_int(0)
        _check(lib().ism_iterate(self._h, int(n_iter), float(rho), float(fid_stop),
                                 self._ptr(Jh) if Jh is not None else None, ct.byref(done)),
               "ism_iterate")
        if Jh is not None:
            Jh = Jh[:n_iter]
        return Jh, done.value

    def iterate_static(self, n_iter, rho, fid_stop=2.0, record=True):
        """ism_iterate_static: as iterate, with the J history in the library's fixed device
        array (no allocation).  Rows past the ones the call wrote are NaN."""
        Jh = self._out((max(n_iter, 1), self.B), np.float64) if record else None
        if Jh is not None:
            Jh[...] = np.nan
        done = ct.c_int(0)
        _check(lib().ism_iterate_static(self._h, int(n_iter), float(rho), float(fid_stop),
                                        self._ptr(Jh) if Jh is not None else None,
                                        ct.byref(done)),
               "ism_iterate_static")
        if Jh is not None:
            Jh = Jh[:n_iter]
        return Jh, done.value

    def iterate_inner(self, n_iter, n_inner, rho, fid_stop=2.0, err_stop=0.0, record=True):
        """ism_iterate_inner: returns (J history [n_iter, B], Err history [iters_done, B],
        iters_done)."""
        Jh = self._out((max(n_iter, 1), self.B), np.float64) if record else None
        Eh = self._out((max(n_iter, 1), self.B), np.float64) if record else None
        done = ct.c_int(0)
        _check(lib().ism_iterate_inner(self._h, int(n_iter), int(n_inner), float(rho),
                                       float(fid_stop), float(err_stop),
                                       self._ptr(Jh) if Jh is not None else None,
                                       self._ptr(Eh) if Eh is not None else None, ct.byref(done)),
               "ism_iterate_inner")
        if Jh is not None:
            Jh = Jh[:n_iter]
            Eh = Eh[:done.value]
        return Jh, Eh, done.value

    def iterate_newton(self, n_iter, gmres_m, fd_eps=1e-5, fid_stop=2.0, record=True):
        """ism_iterate_newton: returns (J history [rows, B], iters_done), rows =
        min(n_iter, iters_done + 1), the rows the call wrote."""
        Jh = self._out((max(n_iter, 1), self.B), np.float64) if record else None
        done = ct.c_int(0)
        _check(lib().ism_iterate_newton(self._h, int(n_iter), int(gmres_m), float(fd_eps),
                                        float(fid_stop),
                                        self._ptr(Jh) if Jh is not None else None,
                                        ct.byref(done)),
               "ism_iterate_newton")
        if Jh is not None:
            Jh = Jh[:min(n_iter, done.value + 1)]
        return Jh, done.value

    def fidelity(self):
        J = self._out((self.B,), np.float64)
        F = self._out((self.B,), np.float64)
        _check(lib().ism_fidelity(self._h, self._ptr(J), self._ptr(F)), "ism_fidelity")
        return J, F

    def set_timing(self, enable=True):
        _check(lib().ism_set_timing(self._h, 1 if enable else 0), "ism_set_timing")

    def kernel_times(self) -> dict:
        """{kernel name: (launches, total ms)} since the last call (synchronises)."""
        arr = (KernelTime * 32)()
        n = ct.c_int(0)
        _check(lib().ism_kernel_times(self._h, arr, 32, ct.byref(n)), "ism_kernel_times")
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(n.value)}

    def taylor_params(self):
        """Per-instance series terms m[b] and sub-steps S[b] of the sparse path."""
        m = (ct.c_int * self.B)()
        S = (ct.c_int * self.B)()
        _check(lib().ism_taylor_params(self._h, m, S), "ism_taylor_params")
        return list(m), list(S)

    def info(self) -> dict:
        i = Info()
        _check(lib().ism_problem_info(self._h, ct.byref(i)), "ism_problem_info")
        return {f: getattr(i, f) for f, _ in Info._fields_}


def from_problem(prob, precision="fp64", N=None, batch=None, device=0, stream=None,
                 io_device=False, set_u=True, step_map="exp", launch_per_pass=False,
                 gpe_frozen=False):
    """Create a handle from a ``problems.FiniteProblem`` (or ``problems.GpeProblem``)."""
    if hasattr(prob, "V0"):
        B = prob.batch if batch is None else batch
        p = Problem.create_gpe(prob.n, prob.L, prob.g, prob.V0, prob.V1, prob.V2, prob.psi0,
                               prob.target, prob.T, prob.K, prob.N if N is None else N,
                               precision=precision, batch=B, device=device, stream=stream,
                               io_device=io_device, gpe_frozen=gpe_frozen)
        if set_u:
            p.set_controls(prob.u0[:B])
        return p
    B = prob.batch if batch is None else batch
    H0 = prob.H0[:B] if prob.H0.ndim == 3 else prob.H0
    al = prob.alpha if np.any(prob.alpha != 0) else None
    p = Problem.create(H0, prob.Hc, prob.psi0, prob.target, prob.T, prob.K,
                       prob.N if N is None else N, precision=precision, kind=prob.kind, batch=B,
                       h0_batched=prob.H0.ndim == 3, alpha=al, device=device, stream=stream,
                       io_device=io_device, step_map=step_map,
                       launch_per_pass=launch_per_pass)
    if set_u:
        p.set_controls(prob.u0[:B])
    return p


def _result_dict(r: Result) -> dict:
    return {f: getattr(r, f) for f, _ in Result._fields_}


class Server:
    """libism serving loop (admission by device-memory budget, one handle and stream per
    admitted request, chunked iterations, non-blocking completion polling)."""

    def __init__(self, hbm_budget: int, iters_per_round: int = 10, max_running: int = 64,
                 device: int = 0):
        L = lib()
        h = ct.c_void_p()
        _check(L.ism_server_create(ct.byref(h), int(device), int(hbm_budget),
                                   int(iters_per_round), int(max_running)), "ism_server_create")
        self._h = h
        self._meta = {}

    @staticmethod
    def clock() -> float:
        return float(lib().ism_server_clock())

    def submit(self, prob, max_iter: int, rho: float, fid_stop: float = 2.0,
               precision="fp32", t_arrival: float = -1.0) -> int:
        """Queue the solve of ``prob`` (a problems.FiniteProblem with batch 1, or a
        problems.GpeProblem) from its u0; returns the ticket."""
        r = Request()
        keep = []

        def ptr(a, dt):
            a = np.ascontiguousarray(np.asarray(a, dtype=dt))
            keep.append(a)
            return a.ctypes.data

        r.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        if hasattr(prob, "V0"):
            r.model = REQ_GPE
            r.n_grid, r.L, r.g, r.V2 = prob.n, prob.L, prob.g, prob.V2
            r.V0, r.V1 = ptr(prob.V0, np.float64), ptr(prob.V1, np.float64)
            C = 1
        else:
            if prob.H0.ndim == 3 and prob.H0.shape[0] != 1:
                raise ValueError("a served request holds one instance")
            r.model = REQ_FINITE
            r.kind = KINDS[prob.kind]
            r.d, r.n_ctrl = prob.Hc.shape[-1], prob.Hc.shape[0]
            r.H0 = ptr(prob.H0.reshape(r.d, r.d), np.complex128)
            r.Hc = ptr(prob.Hc, np.complex128)
            C = r.n_ctrl
        r.psi0, r.target = ptr(prob.psi0, np.complex128), ptr(prob.target, np.complex128)
        r.T, r.K, r.N = float(prob.T), int(prob.K), int(prob.N)
        u0 = np.asarray(prob.u0, dtype=np.float64).reshape(-1, prob.K, C)[0]
        r.u0 = ptr(u0, np.float64)
        r.max_iter, r.rho, r.fid_stop = int(max_iter), float(rho), float(fid_stop)
        t = ct.c_uint64(0)
        _check(lib().ism_server_submit(self._h, ct.byref(r), float(t_arrival), ct.byref(t)),
               "ism_server_submit")
        self._meta[t.value] = (prob.K, C)
        return t.value

    def progress(self):
        q, r = ct.c_int(0), ct.c_int(0)
        _check(lib().ism_server_progress(self._h, ct.byref(q), ct.byref(r)), "ism_server_progress")
        return q.value, r.value

    def poll(self, ticket: int) -> dict:
        r = Result()
        _check(lib().ism_server_poll(self._h, ticket, ct.byref(r)), "ism_server_poll")
        return _result_dict(r)

    def take(self, ticket: int):
        """(result dict, final controls (K, C) or None if the request failed)."""
        K, C = self._meta[ticket]
        u = np.empty((K, C), dtype=np.float64)
        r = Result()
        _check(lib().ism_server_take(self._h, ticket, ct.byref(r), _cptr(u)), "ism_server_take")
        del self._meta[ticket]
        return _result_dict(r), (u if r.state == REQ_DONE else None)

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().ism_server_stats_get(self._h, ct.byref(st)), "ism_server_stats_get")
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self._h:
            lib().ism_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
