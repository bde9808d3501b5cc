"""ctypes binding of libsawave.so (the C ABI in include/sawave.h).

Argument marshalling only: numpy arrays travel as host pointers (SA_MEM_HOST), CUDA tensors of
PyTorch-ROCm as device pointers (SA_MEM_DEVICE) on the tensor's current stream. Every step of
the solve runs in the library's HIP kernels; this module computes nothing. If the library is
missing the import of this module raises, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsawave.so")

SA_OK, SA_NOCONV = 0, 1
SA_PERIODIC, SA_WALLS = 0, 1
SA_PC = {"none": 0, "line": 1, "mg": 2}
SA_GUESS = {"cold": 0, "previous": 1, "ewma": 2}
SA_PRECISION = {"fp64": 0, "fp32_ir": 1}
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
        ("cluster", C.c_int32), ("profile", C.c_int32), ("coarse_max", C.c_int32),
    ]


class SaSolveInfo(C.Structure):
    _fields_ = [
        ("iters", C.c_int32), ("restarts", C.c_int32), ("refinements", C.c_int32), ("status", C.c_int32),
        ("rank", C.c_int32), ("checks", C.c_int32), ("relres0", C.c_double), ("relres", C.c_double),
    ]


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
        "sa_solve": (C.c_int, [P, C.POINTER(SaSolveInfo), C.c_int32]),
        "sa_read_log": (C.c_int, [P, C.POINTER(SaSolveInfo), C.c_int32, C.POINTER(C.c_int32)]),
        "sa_get_solution": (C.c_int, [P, P, C.c_int32]),
        "sa_apply_operator": (C.c_int, [P, P, P, C.c_int32]),
        "sa_apply_precond": (C.c_int, [P, P, P, C.c_int32]),
        "sa_apply_operator_f32": (C.c_int, [P, P, P, C.c_int32]),
        "sa_apply_precond_f32": (C.c_int, [P, P, P, C.c_int32]),
        "sa_sketch_draws": (C.c_int, [C.c_uint64, C.c_int64, C.c_int32, D]),
        "sa_get_sketch": (C.c_int, [P, P, C.c_int32]),
        "sa_sketch_count": (C.c_int64, [P]),
        "sa_last_error": (C.c_char_p, []),
        "sa_build_info": (C.c_char_p, []),
        "sa_get_phase_times": (C.c_int, [P, D, C.c_int32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


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


class Problem:
    """One simulation's sequence of systems on the GPU (see include/sawave.h)."""

    def __init__(self, nx: int, nz: int, bc: str, length: float, h, stream=None, **opts):
        self.grid = SaGrid(nx, nz, SA_PERIODIC if bc == "periodic" else SA_WALLS, float(length))
        o = default_options()
        for key, val in opts.items():
            names = {"precond": SA_PC, "guess": SA_GUESS, "precision": SA_PRECISION}.get(key)
            if names is not None and isinstance(val, str):
                val = names[val]
            if not hasattr(o, key):
                raise KeyError(key)
            setattr(o, key, val)
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
        kw = dict(restart=w.restart, rtol=w.rtol, precond=w.precond, k=w.k, r=w.r, seed=w.seed)
        kw.update(overrides)
        return cls(w.nx, w.nz, w.bc, w.length, w.depth(), stream=stream, **kw)

    def close(self):
        if getattr(self, "_h", None):
            lib.sa_destroy(self._h)
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
