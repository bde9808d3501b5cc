"""ctypes binding of libsawave.so (the C ABI in include/sawave.h).

Argument marshalling only: numpy arrays travel as host pointers (SA_MEM_HOST), CUDA tensors of
PyTorch-ROCm as device pointers (SA_MEM_DEVICE) on the tensor's current stream. Every step of
the solve runs in the library's HIP kernels; this module computes nothing. If the library is
missing the import of this module raises, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import sys
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsawave.so")

SA_OK, SA_NOCONV = 0, 1
SA_EBUSY = -7
SA_PERIODIC, SA_WALLS = 0, 1
SA_PC = {"none": 0, "line": 1, "mg": 2, "ilu0": 3}
SA_GUESS = {"cold": 0, "previous": 1, "ewma": 2, "range": 3}
SA_PRECISION = {"fp64": 0, "fp32_ir": 1}
SA_DECAY = {"solves": 0, "time": 1}
SA_MEM_HOST, SA_MEM_DEVICE = 0, 1
SA_SYNC, SA_ASYNC = 0, 1


class SaGrid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("nz", C.c_int32), ("bc", C.c_int32), ("length", C.c_double)]


class SaOptions(C.Structure):
    _fields_ = [
        ("restart", C.c_int32), ("max_restarts", C.c_int32), ("rtol", C.c_double),
        ("precond", C.c_int32), ("nu1", C.c_int32), ("nu2", C.c_int32), ("omega", C.c_double),
        ("max_levels", C.c_int32), ("guess", C.c_int32), ("k", C.c_int32), ("r", C.c_double),
        ("seed", C.c_uint64), ("n_init", C.c_int32), ("tau_drop", C.c_double),
        ("precision", C.c_int32), ("rtol_inner", C.c_double), ("max_refine", C.c_int32),
        ("cluster", C.c_int32), ("profile", C.c_int32), ("coarse_max", C.c_int32), ("window", C.c_int32),
        ("decay", C.c_int32), ("decay_dtau", C.c_double), ("orthonormalize", C.c_int32),
    ]


class SaSolveInfo(C.Structure):
    _fields_ = [
        ("iters", C.c_int32), ("restarts", C.c_int32), ("refinements", C.c_int32), ("status", C.c_int32),
        ("rank", C.c_int32), ("checks", C.c_int32), ("relres0", C.c_double), ("relres", C.c_double),
    ]


class SaGrid3(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("bc_x", C.c_int32), ("bc_y", C.c_int32),
                ("length_x", C.c_double), ("length_y", C.c_double)]


class SaServerOptions(C.Structure):
    _fields_ = [("hbm_budget", C.c_int64), ("max_inflight", C.c_int32), ("max_batch", C.c_int32),
                ("unknowns_per_workgroup", C.c_int32), ("queue_admission", C.c_int32)]


class SaCompletion(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("sim", C.c_int32), ("reserved", C.c_int32), ("info", SaSolveInfo),
                ("t_submit_ms", C.c_double), ("t_launch_ms", C.c_double), ("t_done_ms", C.c_double)]


@dataclass
class SolveInfo:
    iters: int
    restarts: int
    refinements: int
    status: int
    rank: int
    checks: int
    relres0: float
    relres: float

    @classmethod
    def of(cls, s: SaSolveInfo) -> "SolveInfo":
        return cls(s.iters, s.restarts, s.refinements, s.status, s.rank, s.checks, s.relres0, s.relres)


class SawaveError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sawave error {code}: {msg}")
        self.code = code


def _torch_first():
    """Let PyTorch bring up its HIP runtime before this library does.

    The PyTorch-ROCm wheel ships its own HIP and HSA runtimes beside the system ROCm ones this
    library links; both can serve one process (device pointers are shared), but PyTorch finds no
    device when it initialises after the system runtime has. Nothing happens without torch or
    without a GPU."""
    try:
        import torch
    except Exception:
        return
    try:
        if torch.cuda.is_available():
            torch.cuda.init()
    except Exception:
        pass


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2511_18071_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    D = C.POINTER(C.c_double)
    sig = {
        "sa_default_options": (None, [C.POINTER(SaOptions)]),
        "sa_create": (C.c_int, [C.POINTER(SaGrid), D, C.POINTER(SaOptions), P, C.POINTER(P)]),
        "sa_destroy": (None, [P]),
        "sa_size": (C.c_int64, [P]),
        "sa_ncol": (C.c_int32, [P]),
        "sa_set_surface": (C.c_int, [P, P, P, C.c_int32]),
        "sa_push_rhs": (C.c_int, [P, P, C.c_int32]),
        "sa_set_time": (C.c_int, [P, C.c_double]),
        "sa_solve": (C.c_int, [P, C.POINTER(SaSolveInfo), C.c_int32]),
        "sa_read_log": (C.c_int, [P, C.POINTER(SaSolveInfo), C.c_int32, C.POINTER(C.c_int32)]),
        "sa_get_solution": (C.c_int, [P, P, C.c_int32]),
        "sa_get_solution_async": (C.c_int, [P, P]),
        "sa_debug_abort": (C.c_int, [P]),
        "sa_save_state": (C.c_int, [P, P, C.POINTER(C.c_size_t)]),
        "sa_load_state": (C.c_int, [P, P, C.c_size_t]),
        "sa_apply_operator": (C.c_int, [P, P, P, C.c_int32]),
        "sa_apply_precond": (C.c_int, [P, P, P, C.c_int32]),
        "sa_apply_operator_static": (C.c_int, [C.POINTER(SaGrid), D, D, D, P, P, P]),
        "sa_apply_operator_f32": (C.c_int, [P, P, P, C.c_int32]),
        "sa_apply_precond_f32": (C.c_int, [P, P, P, C.c_int32]),
        "sa_sketch_draws": (C.c_int, [C.c_uint64, C.c_int64, C.c_int32, D]),
        "sa_get_sketch": (C.c_int, [P, P, C.c_int32]),
        "sa_sketch_count": (C.c_int64, [P]),
        "sa_last_error": (C.c_char_p, []),
        "sa_build_info": (C.c_char_p, []),
        "sa_get_phase_times": (C.c_int, [P, D, C.c_int32]),
        "sa_problem_footprint": (C.c_int, [C.POINTER(SaGrid), D, C.POINTER(SaOptions), C.POINTER(C.c_int64)]),
        "sa_loop_create": (C.c_int, [P, C.c_double, C.POINTER(P)]),
        "sa_loop_set_state": (C.c_int, [P, P, P, P, C.c_int32]),
        "sa_loop_step": (C.c_int, [P, C.POINTER(SaSolveInfo)]),
        "sa_loop_get_state": (C.c_int, [P, P, P, P, C.c_int32]),
        "sa_loop_destroy": (None, [P]),
        "sa_op3d_create": (C.c_int, [C.POINTER(SaGrid3), D, P, C.POINTER(P)]),
        "sa_op3d_set_surface": (C.c_int, [P, P, P, C.c_int32]),
        "sa_op3d_apply": (C.c_int, [P, P, P, C.c_int32]),
        "sa_op3d_sync": (C.c_int, [P]),
        "sa_op3d_size": (C.c_int64, [P]),
        "sa_op3d_workgroups": (C.c_int, [P]),
        "sa_op3d_destroy": (None, [P]),
        "sa_server_default_options": (None, [C.POINTER(SaServerOptions)]),
        "sa_server_create": (C.c_int, [C.POINTER(SaServerOptions), P, C.POINTER(P)]),
        "sa_server_destroy": (None, [P]),
        "sa_server_open": (C.c_int, [P, C.POINTER(SaGrid), D, C.POINTER(SaOptions), C.POINTER(C.c_int32)]),
        "sa_server_close": (C.c_int, [P, C.c_int32]),
        "sa_server_submit": (C.c_int, [P, C.c_int32, P, P, P, C.c_int32, P, C.POINTER(C.c_uint64)]),
        "sa_server_admitted": (C.c_int32, [P, C.c_int32]),
        "sa_server_clock_ms": (C.c_double, [P]),
        "sa_server_stats": (C.c_int, [P, D, C.c_int32]),
        "sa_server_poll": (C.c_int, [P, C.POINTER(SaCompletion), C.c_int32, C.POINTER(C.c_int32), C.c_int32]),
        "sa_server_outstanding": (C.c_int64, [P]),
        "sa_server_bytes_used": (C.c_int64, [P]),
        "sa_server_problem": (P, [P, C.c_int32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_torch_first()
lib = _load()


def _check(code: int, allow=(SA_OK, SA_NOCONV)) -> int:
    if code not in allow:
        raise SawaveError(code, lib.sa_last_error().decode())
    return code


def default_options() -> SaOptions:
    o = SaOptions()
    lib.sa_default_options(C.byref(o))
    return o


def sketch_draws(seed: int, index: int, k: int) -> np.ndarray:
    out = np.zeros(k)
    _check(lib.sa_sketch_draws(seed, index, k, out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def _is_torch_cuda(a) -> bool:
    return hasattr(a, "is_cuda") and bool(a.is_cuda)


def _ptr(a, n_expected: int | None = None, dtype=np.float64):
    """(pointer, mem kind, keep-alive) of a numpy array or CUDA tensor of the given dtype."""
    if _is_torch_cuda(a):
        import torch
        tdt = torch.float64 if dtype == np.float64 else torch.float32
        if a.dtype != tdt or not a.is_contiguous():
            raise ValueError(f"device arrays must be contiguous {tdt} tensors")
        if n_expected is not None and a.numel() != n_expected:
            raise ValueError(f"expected {n_expected} values, got {a.numel()}")
        return C.c_void_p(a.data_ptr()), SA_MEM_DEVICE, a
    arr = np.ascontiguousarray(a, dtype=dtype)
    if n_expected is not None and arr.size != n_expected:
        raise ValueError(f"expected {n_expected} values, got {arr.size}")
    return C.c_void_p(arr.ctypes.data), SA_MEM_HOST, arr


def _stream_handle(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return C.c_void_p(torch.cuda.current_stream().cuda_stream)
        except Exception:
            pass
        return C.c_void_p(0)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def make_options(**opts) -> SaOptions:
    """sa_options from keyword arguments (names of include/sawave.h; enum values by name)."""
    o = default_options()
    for key, val in opts.items():
        names = {"precond": SA_PC, "guess": SA_GUESS, "precision": SA_PRECISION, "decay": SA_DECAY}.get(key)
        if names is not None and isinstance(val, str):
            val = names[val]
        if not hasattr(o, key):
            raise KeyError(key)
        setattr(o, key, val)
    return o


def workload_args(w, **overrides):
    """(grid, depth, options) of a synthetic workload."""
    kw = dict(restart=w.restart, rtol=w.rtol, precond=w.precond, nu2=w.nu2, tau_drop=w.tau_drop, k=w.k, r=w.r,
              seed=w.seed, coarse_max=w.coarse_max)
    kw.update(overrides)
    grid = SaGrid(w.nx, w.nz, SA_PERIODIC if w.bc == "periodic" else SA_WALLS, float(w.length))
    return grid, np.ascontiguousarray(w.depth(), dtype=np.float64), make_options(**kw)


def apply_operator_static(w, eta_prev, eta_cur, x, y, stream=None):
    """y = A(eta_prev, eta_cur) x of workload w's grid through the allocation-free entry point
    (x, y: device tensors; eta: host arrays)."""
    grid, h, _ = workload_args(w)
    e1 = np.ascontiguousarray(eta_prev, dtype=np.float64)
    e2 = np.ascontiguousarray(eta_cur, dtype=np.float64)
    px, mx, _ = _ptr(x, w.n)
    py, my, _ = _ptr(y, w.n)
    if mx != SA_MEM_DEVICE or my != SA_MEM_DEVICE:
        raise ValueError("x and y must be device tensors")
    D = C.POINTER(C.c_double)
    _check(lib.sa_apply_operator_static(C.byref(grid), h.ctypes.data_as(D), e1.ctypes.data_as(D),
                                        e2.ctypes.data_as(D), px, py, _stream_handle(stream)))
    return y


def footprint(w, **overrides) -> int:
    """Device bytes a problem of workload w would allocate."""
    grid, h, o = workload_args(w, **overrides)
    out = C.c_int64(0)
    _check(lib.sa_problem_footprint(C.byref(grid), h.ctypes.data_as(C.POINTER(C.c_double)), C.byref(o), C.byref(out)))
    return int(out.value)


class Problem:
    """One simulation's sequence of systems on the GPU (see include/sawave.h)."""

    def __init__(self, nx: int, nz: int, bc: str, length: float, h, stream=None, **opts):
        self.grid = SaGrid(nx, nz, SA_PERIODIC if bc == "periodic" else SA_WALLS, float(length))
        o = make_options(**opts)
        self.options = o
        hh = np.ascontiguousarray(h, dtype=np.float64)
        self._stream = _stream_handle(stream)
        handle = C.c_void_p()
        _check(lib.sa_create(C.byref(self.grid), hh.ctypes.data_as(C.POINTER(C.c_double)), C.byref(o),
                             self._stream, C.byref(handle)))
        self._h = handle
        self.n = int(lib.sa_size(handle))
        self.ncol = int(lib.sa_ncol(handle))
        self.nphys = nx - 1 if bc == "periodic" else nx
        self._keep = []

    @classmethod
    def from_workload(cls, w, stream=None, **overrides):
        kw = dict(restart=w.restart, rtol=w.rtol, precond=w.precond, nu2=w.nu2, tau_drop=w.tau_drop, k=w.k, r=w.r,
              seed=w.seed, coarse_max=w.coarse_max)
        kw.update(overrides)
        return cls(w.nx, w.nz, w.bc, w.length, w.depth(), stream=stream, **kw)

    def close(self):
        if getattr(self, "_h", None):
            lib.sa_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # no HIP calls while the interpreter shuts down: the runtime (or a profiler wrapped
        # around it) may already be gone; the process exit releases the device memory (the
        # check is bound at definition: module globals may be cleared by then)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---- inputs ---------------------------------------------------------------------------
    def set_surface(self, eta_prev, eta_cur):
        pa, ma, ka = _ptr(eta_prev, self.nphys)
        pb, mb, kb = _ptr(eta_cur, self.nphys)
        if ma != mb:
            raise ValueError("both surfaces must live in the same memory")
        _check(lib.sa_set_surface(self._h, pa, pb, ma))
        self._keep_surface = (ka, kb)

    def push_rhs(self, b):
        pb, mb, kb = _ptr(b, self.n)
        _check(lib.sa_push_rhs(self._h, pb, mb))
        self._keep_rhs = kb

    def set_time(self, tau: float):
        _check(lib.sa_set_time(self._h, float(tau)))

    # ---- solve ------------------------------------------------------------------------------
    def solve(self, sync: bool = True):
        info = SaSolveInfo()
        code = lib.sa_solve(self._h, C.byref(info), SA_SYNC if sync else SA_ASYNC)
        _check(code)
        return SolveInfo.of(info) if sync else None

    def read_log(self, max_entries: int = 4096) -> list:
        buf = (SaSolveInfo * max_entries)()
        cnt = C.c_int32(0)
        _check(lib.sa_read_log(self._h, buf, max_entries, C.byref(cnt)))
        return [SolveInfo.of(buf[i]) for i in range(cnt.value)]

    def solution(self, out=None):
        if out is None:
            out = np.zeros(self.n)
        p, m, _ = _ptr(out, self.n)
        _check(lib.sa_get_solution(self._h, p, m))
        return out

    def save_state(self) -> bytes:
        """The solver state carried between solves (sketch, last solution, counters)."""
        ln = C.c_size_t(0)
        _check(lib.sa_save_state(self._h, None, C.byref(ln)))
        buf = C.create_string_buffer(ln.value)
        _check(lib.sa_save_state(self._h, buf, C.byref(ln)))
        return buf.raw[: ln.value]

    def load_state(self, state: bytes):
        buf = C.create_string_buffer(state, len(state))
        _check(lib.sa_load_state(self._h, buf, len(state)))

    def solution_async(self, out):
        """Enqueue a copy of the last solution into the device tensor `out` (no wait)."""
        p, m, _ = _ptr(out, self.n)
        if m != SA_MEM_DEVICE:
            raise ValueError("solution_async writes device memory only")
        _check(lib.sa_get_solution_async(self._h, p))
        return out

    def apply_operator(self, x, out=None):
        if out is None:
            out = np.zeros(self.n) if not _is_torch_cuda(x) else x.new_zeros(self.n)
        px, mx, kx = _ptr(x, self.n)
        py, my, _ = _ptr(out, self.n)
        if mx != my:
            raise ValueError("x and y must live in the same memory")
        _check(lib.sa_apply_operator(self._h, px, py, mx))
        return out

    def apply_precond(self, x, out=None):
        if out is None:
            out = np.zeros(self.n) if not _is_torch_cuda(x) else x.new_zeros(self.n)
        px, mx, kx = _ptr(x, self.n)
        py, my, _ = _ptr(out, self.n)
        if mx != my:
            raise ValueError("x and y must live in the same memory")
        _check(lib.sa_apply_precond(self._h, px, py, mx))
        return out

    def apply_operator_f32(self, x, out=None):
        return self._apply32(lib.sa_apply_operator_f32, x, out)

    def apply_precond_f32(self, x, out=None):
        return self._apply32(lib.sa_apply_precond_f32, x, out)

    def _apply32(self, fn, x, out):
        if out is None:
            out = np.zeros(self.n, dtype=np.float32) if not _is_torch_cuda(x) else x.new_zeros(self.n)
        px, mx, kx = _ptr(x, self.n, np.float32)
        py, my, _ = _ptr(out, self.n, np.float32)
        if mx != my:
            raise ValueError("x and y must live in the same memory")
        if not isinstance(out, np.ndarray) or out.dtype == np.float32:
            _check(fn(self._h, px, py, mx))
        return out

    def sketch(self) -> np.ndarray:
        k = self.options.k
        out = np.zeros(k * self.n)
        _check(lib.sa_get_sketch(self._h, C.c_void_p(out.ctypes.data), SA_MEM_HOST))
        return out.reshape(k, self.n).T.copy()

    PHASES = ("geometry", "guess", "small_solve", "operator", "precond", "orthogonalisation", "other", "total")

    def phase_times(self, detail: bool = False):
        out = np.zeros(57)
        _check(lib.sa_get_phase_times(self._h, out.ctypes.data_as(C.POINTER(C.c_double)), 57))
        totals = dict(zip(self.PHASES, out[:8].tolist()))
        if not detail:
            return totals
        return totals, out[8:]

    @property
    def sketch_count(self) -> int:
        return int(lib.sa_sketch_count(self._h))


@dataclass
class Completion:
    ticket: int
    sim: int
    info: SolveInfo
    t_submit_ms: float
    t_launch_ms: float
    t_done_ms: float


class Server:
    """Continuous-batching server of independent simulations (sa_server_* in include/sawave.h)."""

    def __init__(self, stream=None, **opts):
        o = SaServerOptions()
        lib.sa_server_default_options(C.byref(o))
        for key, val in opts.items():
            if not hasattr(o, key):
                raise KeyError(key)
            setattr(o, key, val)
        self.options = o
        self._stream = _stream_handle(stream)
        h = C.c_void_p()
        _check(lib.sa_server_create(C.byref(o), self._stream, C.byref(h)))
        self._h = h
        self._keep = {}
        self._sims = {}

    def close(self):
        if getattr(self, "_h", None):
            lib.sa_server_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # no HIP calls while the interpreter shuts down: the runtime (or a profiler wrapped
        # around it) may already be gone; the process exit releases the device memory (the
        # check is bound at definition: module globals may be cleared by then)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def open(self, w, **overrides) -> int | None:
        """Admit workload w; None when its arena does not fit the HBM budget now (without
        queue_admission), else its simulation id (check admitted() with queue_admission)."""
        grid, h, o = workload_args(w, **overrides)
        sid = C.c_int32(-1)
        code = lib.sa_server_open(self._h, C.byref(grid), h.ctypes.data_as(C.POINTER(C.c_double)), C.byref(o),
                                  C.byref(sid))
        if code == SA_EBUSY:
            return None
        _check(code)
        self._sims[sid.value] = (w.n, w.nx - 1 if w.bc == "periodic" else w.nx)
        return sid.value

    def admitted(self, sim: int) -> int:
        return int(lib.sa_server_admitted(self._h, sim))

    def close_sim(self, sim: int):
        _check(lib.sa_server_close(self._h, sim))
        self._sims.pop(sim, None)

    def submit(self, sim: int, eta_prev, eta_cur, b, x_out=None) -> int:
        """Queue the next system of `sim`; x_out (same memory kind as the inputs) receives the
        solution when the completion is harvested."""
        n, nphys = self._sims[sim]
        pa, ma, ka = _ptr(eta_prev, nphys)
        pb, mb, kb = _ptr(eta_cur, nphys)
        pr, mr, kr = _ptr(b, n)
        px, kx = C.c_void_p(0), None
        if x_out is not None:
            px, mx, kx = _ptr(x_out, n)
            if mx != ma or (mx == SA_MEM_HOST and kx is not x_out):
                raise ValueError("x_out must be a contiguous float64 array in the inputs' memory")
        if not (ma == mb == mr):
            raise ValueError("all inputs must live in the same memory")
        t = C.c_uint64(0)
        _check(lib.sa_server_submit(self._h, sim, pa, pb, pr, ma, px, C.byref(t)))
        if ma == SA_MEM_DEVICE or kx is not None:
            self._keep[t.value] = (ka, kb, kr, kx)  # inputs and output stay alive until completion
        return t.value

    def poll(self, wait: bool = False, timeout_s: float | None = None, max_entries: int = 1024) -> list:
        """Completions harvested so far; with wait, block until one is available (at most
        timeout_s seconds when given)."""
        buf = (SaCompletion * max_entries)()
        cnt = C.c_int32(0)
        wait_us = 0 if not wait else (-1 if timeout_s is None else max(1, int(timeout_s * 1e6)))
        _check(lib.sa_server_poll(self._h, buf, max_entries, C.byref(cnt), wait_us))
        out = []
        for i in range(cnt.value):
            c = buf[i]
            self._keep.pop(c.ticket, None)
            out.append(Completion(c.ticket, c.sim, SolveInfo.of(c.info), c.t_submit_ms, c.t_launch_ms, c.t_done_ms))
        return out

    def clock_ms(self) -> float:
        return float(lib.sa_server_clock_ms(self._h))

    def stats(self) -> dict:
        out = np.zeros(7)
        _check(lib.sa_server_stats(self._h, out.ctypes.data_as(C.POINTER(C.c_double)), 7))
        return dict(ticks=int(out[0]), solves=int(out[1]), launch_host_ms=float(out[2]), tick_ms=float(out[3]),
                    capacity=int(out[4]), tick_budget=int(out[5]), device_failed=int(out[6]))

    @property
    def outstanding(self) -> int:
        return int(lib.sa_server_outstanding(self._h))

    @property
    def bytes_used(self) -> int:
        return int(lib.sa_server_bytes_used(self._h))

    def apply_operator(self, sim: int, eta_prev, eta_cur, x, out):
        """out = A(eta_prev, eta_cur) x with simulation `sim`'s operator (before it has work)."""
        n, nphys = self._sims[sim]
        p = lib.sa_server_problem(self._h, sim)
        if not p:
            raise SawaveError(-1, f"no simulation {sim}")
        pa, ma, _ = _ptr(eta_prev, nphys)
        pb, mb, _ = _ptr(eta_cur, nphys)
        px, mx, _ = _ptr(x, n)
        py, my, _ = _ptr(out, n)
        if not (ma == mb == mx == my):
            raise ValueError("all arrays must live in the same memory")
        _check(lib.sa_set_surface(p, pa, pb, ma))
        _check(lib.sa_apply_operator(p, px, py, mx))
        return out

    def debug_abort(self, sim: int):
        """Raise the device abort flag of an idle simulation (failure-handling tests)."""
        p = lib.sa_server_problem(self._h, sim)
        if not p:
            raise SawaveError(-1, f"simulation {sim} has no idle problem")
        _check(lib.sa_debug_abort(p))

    def solution(self, sim: int, out=None):
        n, _ = self._sims[sim]
        p = lib.sa_server_problem(self._h, sim)
        if not p:
            raise SawaveError(-1, f"no simulation {sim}")
        if out is None:
            out = np.zeros(n)
        ptr, m, _ = _ptr(out, n)
        _check(lib.sa_get_solution(p, ptr, m))
        return out


class Operator3D:
    """The mixed-stage operator on a (chi, gamma, sigma) grid (see include/sawave.h, sa_op3d_*).

    h, eta: plane arrays of the physical points (ny or ny - 1 rows of nx or nx - 1 values, chi
    fastest); vectors: (nz + 1) x nrow x ncol values, chi fastest. numpy arrays are staged and
    waited for; CUDA tensors are read and written on the operator's stream without waiting."""

    def __init__(self, nx: int, ny: int, nz: int, bc_x: str, bc_y: str, length_x: float, length_y: float, h,
                 stream=None):
        code = lambda bc: SA_PERIODIC if bc == "periodic" else SA_WALLS
        self.grid = SaGrid3(nx, ny, nz, code(bc_x), code(bc_y), float(length_x), float(length_y))
        self.nxp = nx - 1 if bc_x == "periodic" else nx
        self.nyp = ny - 1 if bc_y == "periodic" else ny
        hh = np.ascontiguousarray(h, dtype=np.float64)
        if hh.size != self.nxp * self.nyp:
            raise ValueError(f"h must hold {self.nyp} x {self.nxp} values")
        self._stream = _stream_handle(stream)
        handle = C.c_void_p()
        _check(lib.sa_op3d_create(C.byref(self.grid), hh.ctypes.data_as(C.POINTER(C.c_double)), self._stream,
                                  C.byref(handle)))
        self._h = handle
        self.n = int(lib.sa_op3d_size(handle))
        self.workgroups = int(lib.sa_op3d_workgroups(handle))
        self._keep = []

    def close(self):
        if getattr(self, "_h", None):
            lib.sa_op3d_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_surface(self, eta_prev, eta_cur):
        npl = self.nxp * self.nyp
        pa, ma, ka = _ptr(eta_prev, npl)
        pb, mb, kb = _ptr(eta_cur, npl)
        if ma != mb:
            raise ValueError("both surfaces must live in the same memory")
        self._keep = [ka, kb]
        _check(lib.sa_op3d_set_surface(self._h, pa, pb, ma))

    def apply(self, x, y=None):
        """y = A x; returns y (a new numpy array for numpy input)."""
        px, mx, kx = _ptr(x, self.n)
        if y is None:
            if mx == SA_MEM_DEVICE:
                raise ValueError("give y for device input")
            y = np.empty(self.n)
        py, my, ky = _ptr(y, self.n)
        if mx != my:
            raise ValueError("x and y must live in the same memory")
        _check(lib.sa_op3d_apply(self._h, px, py, mx))
        return y

    def sync(self):
        _check(lib.sa_op3d_sync(self._h))


class ClosedLoop:
    """LSERK45 stepping of a periodic problem's velocity field and surface (sa_loop_*): each
    step makes five mixed-stage pressure systems and solves them with the problem's solver."""

    def __init__(self, problem: "Problem", dtau: float):
        handle = C.c_void_p()
        _check(lib.sa_loop_create(problem._h, float(dtau), C.byref(handle)))
        self._h = handle
        self.problem = problem
        self.n, self.ncol = problem.n, problem.ncol

    def close(self):
        if getattr(self, "_h", None):
            lib.sa_loop_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_state(self, eta, u, w):
        pe, me, ke = _ptr(eta, self.ncol)
        pu, mu, ku = _ptr(u, self.n)
        pw, mw, kw = _ptr(w, self.n)
        if not (me == mu == mw):
            raise ValueError("eta, u and w must live in the same memory")
        _check(lib.sa_loop_set_state(self._h, pe, pu, pw, me))

    def step(self):
        infos = (SaSolveInfo * 5)()
        _check(lib.sa_loop_step(self._h, infos), allow=(SA_OK,))
        return [SolveInfo.of(i) for i in infos]

    def state(self):
        eta, u, w = np.empty(self.ncol), np.empty(self.n), np.empty(self.n)
        _check(lib.sa_loop_get_state(self._h, eta.ctypes.data_as(C.c_void_p), u.ctypes.data_as(C.c_void_p),
                                     w.ctypes.data_as(C.c_void_p), SA_MEM_HOST))
        return eta, u, w
