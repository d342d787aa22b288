"""ctypes binding of libcbgmres.so (the gfx950 HIP library).

Argument marshalling only: every step of the solve runs in the library's
kernels. torch provides device memory and the current stream. There is no
fallback: if the library is missing this module raises on first use.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcbgmres.so")

FORMATS = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3, "e4m3": 4, "int32": 5, "int16": 6}
FORMAT_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2, "e4m3": 1, "int32": 4, "int16": 2}
PRECONDS = {"none": 0, "jacobi": 1, "sparse": 2}
OK, NOT_CONVERGED = 0, 1
E_ARG, E_WORKSPACE, E_HIP, E_NONFINITE, E_UNSUPPORTED = -1, -2, -3, -4, -5
FLAG_PROFILE = 1
MAX_RESTART = 512

EXPORTS = ["cbg_strerror", "cbg_basis_ld", "cbg_workspace_bytes", "cbg_kernel_workspace_bytes",
           "cbgmres_solve", "cbg_encode", "cbg_decode", "cbg_spmv", "cbg_multidot",
           "cbg_update"]


class CbgCsr(C.Structure):
    _fields_ = [("n", C.c_int32), ("reserved", C.c_int32), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p)]


class CbgOpts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("format", C.c_int32), ("tol", C.c_double),
                ("maxiter", C.c_int64), ("eta", C.c_double), ("precond", C.c_int32),
                ("fallback", C.c_int32), ("p_val", C.c_void_p), ("flags", C.c_int32),
                ("reserved", C.c_int32)]


class CbgResult(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("restarts", C.c_int64), ("reorths", C.c_int64),
                ("status", C.c_int32), ("breakdowns", C.c_int32), ("fell_back", C.c_int32),
                ("reserved", C.c_int32), ("true_rel_res", C.c_double),
                ("recurrence_rel_res", C.c_double), ("seconds", C.c_double),
                ("model_bytes", C.c_double), ("prof_orth_ms", C.c_double),
                ("prof_orth_bytes", C.c_double), ("prof_orth_launches", C.c_int64),
                ("prof_dot_ms", C.c_double), ("prof_dot_bytes", C.c_double),
                ("prof_dot_launches", C.c_int64)]


class CbgError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {strerror(status)} ({status})")
        self.status = status


_lib = None


def lib():
    """Load libcbgmres.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2009_12101_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        L.cbg_strerror.argtypes = [C.c_int]
        L.cbg_strerror.restype = C.c_char_p
        L.cbg_basis_ld.argtypes = [i32]
        L.cbg_basis_ld.restype = i64
        L.cbg_workspace_bytes.argtypes = [i32, i32, i32, i32]
        L.cbg_workspace_bytes.restype = sz
        L.cbg_kernel_workspace_bytes.argtypes = [i32, i32]
        L.cbg_kernel_workspace_bytes.restype = sz
        L.cbgmres_solve.argtypes = [C.POINTER(CbgCsr), vp, vp, C.POINTER(CbgOpts), vp, sz, vp,
                                    C.POINTER(CbgResult), vp, i64]
        L.cbg_encode.argtypes = [i32, vp, i32, vp, vp, vp, sz, vp]
        L.cbg_decode.argtypes = [i32, vp, vp, i32, vp, vp]
        L.cbg_spmv.argtypes = [C.POINTER(CbgCsr), vp, vp, vp, vp, sz, vp]
        L.cbg_multidot.argtypes = [i32, vp, i64, vp, i32, i32, vp, vp, vp, sz, vp]
        L.cbg_update.argtypes = [i32, vp, i64, vp, i32, i32, vp, vp, vp, vp, sz, vp]
        for f in ("cbgmres_solve", "cbg_encode", "cbg_decode", "cbg_spmv", "cbg_multidot",
                  "cbg_update"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def strerror(status: int) -> str:
    return lib().cbg_strerror(int(status)).decode()


def basis_ld(n: int) -> int:
    return int(lib().cbg_basis_ld(int(n)))


def workspace_bytes(n: int, restart: int, fmt: str, precond: str = "none") -> int:
    return int(lib().cbg_workspace_bytes(int(n), int(restart), FORMATS[fmt], PRECONDS[precond]))


def kernel_workspace_bytes(n: int, j: int) -> int:
    return int(lib().cbg_kernel_workspace_bytes(int(n), int(j)))


# ---------------------------------------------------------------- torch glue

def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(rc: int, where: str):
    if rc < 0:
        raise CbgError(rc, where)
    return rc


@dataclasses.dataclass
class DeviceCSR:
    """A CSR matrix resident in device memory (int32 indices, fp64 values)."""
    n: int
    nnz: int
    row_ptr: "object"
    col_idx: "object"
    val: "object"

    @classmethod
    def from_host(cls, A, device="cuda"):
        torch = _torch()
        rp = torch.from_numpy(np.ascontiguousarray(A.row_ptr, dtype=np.int32)).to(device)
        ci = torch.from_numpy(np.ascontiguousarray(A.col_idx, dtype=np.int32)).to(device)
        va = torch.from_numpy(np.ascontiguousarray(A.val, dtype=np.float64)).to(device)
        return cls(int(A.n), int(A.nnz), rp, ci, va)

    def cstruct(self) -> CbgCsr:
        return CbgCsr(self.n, 0, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(),
                      self.val.data_ptr())


@dataclasses.dataclass
class SolveResult:
    x: "object"
    status: int
    iterations: int
    restarts: int
    reorths: int
    breakdowns: int
    fell_back: int
    true_rel_res: float
    recurrence_rel_res: float
    seconds: float
    model_bytes: float
    hist: np.ndarray
    prof_orth_ms: float = 0.0
    prof_orth_bytes: float = 0.0
    prof_orth_launches: int = 0
    prof_dot_ms: float = 0.0
    prof_dot_bytes: float = 0.0
    prof_dot_launches: int = 0


def solve(A: DeviceCSR, b, x0=None, restart=100, fmt="fp64", tol=1e-10, maxiter=10000,
          eta=0.0, precond="none", p_val=None, fallback=False, profile=False, workspace=None,
          hist=True) -> SolveResult:
    """cbgmres_solve on device tensors; returns the solution and counters.
    Raises CbgError on a negative status."""
    torch = _torch()
    x = torch.zeros(A.n, dtype=torch.float64, device=b.device) if x0 is None else x0.clone()
    need = workspace_bytes(A.n, restart, fmt, precond)
    if need == 0 and A.n > 0:
        raise CbgError(E_ARG, "cbg_workspace_bytes")
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=b.device)
    opts = CbgOpts(restart, FORMATS[fmt], tol, maxiter, eta, PRECONDS[precond],
                   int(bool(fallback)), None if p_val is None else p_val.data_ptr(),
                   FLAG_PROFILE if profile else 0, 0)
    res = CbgResult()
    hl = int(maxiter) if hist else 0
    h = np.zeros(max(hl, 1))
    csr = A.cstruct()
    rc = lib().cbgmres_solve(C.byref(csr), _ptr(b), _ptr(x), C.byref(opts), _ptr(workspace),
                             workspace.numel(), _stream(), C.byref(res),
                             h.ctypes.data_as(C.c_void_p) if hl else None, hl)
    _check(rc, "cbgmres_solve")
    return SolveResult(x=x, status=rc, iterations=res.iterations, restarts=res.restarts,
                       reorths=res.reorths, breakdowns=res.breakdowns, fell_back=res.fell_back,
                       true_rel_res=res.true_rel_res, recurrence_rel_res=res.recurrence_rel_res,
                       seconds=res.seconds, model_bytes=res.model_bytes,
                       hist=h[:min(res.iterations, hl)].copy(),
                       prof_orth_ms=res.prof_orth_ms, prof_orth_bytes=res.prof_orth_bytes,
                       prof_orth_launches=res.prof_orth_launches, prof_dot_ms=res.prof_dot_ms,
                       prof_dot_bytes=res.prof_dot_bytes,
                       prof_dot_launches=res.prof_dot_launches)


def _kws(n, j, device):
    torch = _torch()
    return torch.empty(max(kernel_workspace_bytes(n, j), 256), dtype=torch.uint8, device=device)


def encode(fmt: str, v, out=None, scale=None, ws=None):
    """The accessor's store: returns (q, scale) on the device."""
    torch = _torch()
    n = v.numel()
    dt = {"fp64": torch.float64, "fp32": torch.float32, "fp16": torch.int16, "bf16": torch.int16,
          "e4m3": torch.uint8, "int32": torch.int32, "int16": torch.int16}[fmt]
    q = torch.empty(n, dtype=dt, device=v.device) if out is None else out
    sc = torch.empty(1, dtype=torch.float64, device=v.device) if scale is None else scale
    ws = _kws(n, 0, v.device) if ws is None else ws
    _check(lib().cbg_encode(FORMATS[fmt], _ptr(v), n, _ptr(q), _ptr(sc), _ptr(ws), ws.numel(),
                            _stream()), "cbg_encode")
    return q, sc


def decode(fmt: str, q, scale, n=None):
    torch = _torch()
    n = q.numel() if n is None else n
    v = torch.empty(n, dtype=torch.float64, device=q.device)
    _check(lib().cbg_decode(FORMATS[fmt], _ptr(q), _ptr(scale), n, _ptr(v), _stream()),
           "cbg_decode")
    return v


def spmv(A: DeviceCSR, x, y=None, want_norm=False):
    torch = _torch()
    y = torch.empty(A.n, dtype=torch.float64, device=x.device) if y is None else y
    nrm = torch.empty(1, dtype=torch.float64, device=x.device) if want_norm else None
    ws = _kws(A.n, 0, x.device) if want_norm else None
    csr = A.cstruct()
    _check(lib().cbg_spmv(C.byref(csr), _ptr(x), _ptr(y), _ptr(nrm), _ptr(ws),
                          0 if ws is None else ws.numel(), _stream()), "cbg_spmv")
    return (y, nrm) if want_norm else y


def multidot(fmt: str, V, ld: int, scales, n: int, j: int, w, h=None, ws=None):
    torch = _torch()
    h = torch.empty(max(j, 1), dtype=torch.float64, device=w.device) if h is None else h
    ws = _kws(n, j, w.device) if ws is None else ws
    _check(lib().cbg_multidot(FORMATS[fmt], _ptr(V), ld, _ptr(scales), n, j, _ptr(w), _ptr(h),
                              _ptr(ws), ws.numel(), _stream()), "cbg_multidot")
    return h[:j]


def update(fmt: str, V, ld: int, scales, n: int, j: int, h, w, norms=None, ws=None):
    torch = _torch()
    norms = torch.empty(2, dtype=torch.float64, device=w.device) if norms is None else norms
    ws = _kws(n, 0, w.device) if ws is None else ws
    _check(lib().cbg_update(FORMATS[fmt], _ptr(V), ld, _ptr(scales), n, j, _ptr(h), _ptr(w),
                            _ptr(norms), _ptr(ws), ws.numel(), _stream()), "cbg_update")
    return norms
