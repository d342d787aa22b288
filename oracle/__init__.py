"""CB-GMRES CPU oracle -- TEST INFRASTRUCTURE ONLY.

ctypes binding of ``liboracle.so`` (plain C, FP64, OpenMP), a slow reference
implementation of compressed-basis GMRES written from the paper (Fig. 1 of
Section 3; the compressed basis of Sections 4 and 5.2). Only the test suite,
the smoke check and the benchmark's CPU-baseline leg may import this package;
the product path never does. It shares no code with the HIP library.

All arrays are numpy arrays on the host.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# CBG_ORACLE_LIB names another build of oracle.c to load in place of the
# in-tree one (the mutation test loads copies with planted mistakes this way).
LIB_PATH = os.environ.get("CBG_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
SRC = os.path.join(_HERE, "oracle.c")

FORMATS = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3, "e4m3": 4, "int32": 5, "int16": 6,
           "fp16s": 7}
FORMAT_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2, "e4m3": 1, "int32": 4, "int16": 2,
                "fp16s": 2}
STORAGE_DTYPE = {"fp64": np.float64, "fp32": np.float32, "fp16": np.uint16, "bf16": np.uint16,
                 "e4m3": np.uint8, "int32": np.int32, "int16": np.int16, "fp16s": np.uint16}
# Arnoldi-step variants for ablations (bits of the options' `variant`)
# ("explicit_redot" names the default, the re-dot Fig. 1 writes)
VARIANTS = {"spmv_vhat": 1, "always_reorth": 2, "mgs": 4, "gram": 8, "explicit_redot": 0,
            "onepass": 16}
PRECONDS = {"none": 0, "jacobi": 1, "sparse": 2, "block_jacobi": 3, "stencil": 4}
OK, NOT_CONVERGED, E_ARG, E_NONFINITE = 0, 1, -1, -4


def build(verbose: bool = False) -> str:
    """Compile liboracle.so from oracle.c (gcc, C11, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fopenmp", "-fPIC", "-shared",
           "-ffp-contract=off", "-fno-fast-math", SRC, "-o", LIB_PATH + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class _Opts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("format", C.c_int32), ("tol", C.c_double),
                ("maxiter", C.c_int64), ("eta", C.c_double), ("precond", C.c_int32),
                ("p_val", C.c_void_p), ("fallback", C.c_int32), ("pc_block", C.c_int32),
                ("pc_prec", C.c_int32), ("variant", C.c_int32), ("pad", C.c_int32),
                ("p_stencil", C.c_void_p), ("grid", C.c_int32 * 3), ("st_ld", C.c_int32)]


class _Result(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("restarts", C.c_int64), ("reorths", C.c_int64),
                ("status", C.c_int32), ("breakdowns", C.c_int32), ("fell_back", C.c_int32),
                ("pad", C.c_int32), ("true_rel_res", C.c_double),
                ("recurrence_rel_res", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.orc_format_bytes.argtypes = [C.c_int]
        L.orc_encode.argtypes = [C.c_int, i64, vp, vp, C.POINTER(dbl)]
        L.orc_decode.argtypes = [C.c_int, i64, vp, dbl, vp]
        L.orc_spmv.argtypes = [i32, vp, vp, vp, vp, vp]
        L.orc_spmv.restype = None
        L.orc_dot.argtypes = [i64, vp, vp]
        L.orc_dot.restype = dbl
        L.orc_gmres.argtypes = [i32, vp, vp, vp, vp, vp, C.POINTER(_Opts), C.POINTER(_Result),
                                vp, vp, vp, vp, vp, C.POINTER(i32)]
        L.orc_block_jacobi.argtypes = [i32, vp, vp, vp, i32, i32, vp, vp]
        L.orc_block_jacobi.restype = C.c_int
        L.orc_stencil_apply.argtypes = [i32, vp, vp, vp, C.POINTER(i32), vp, i64, vp, vp]
        L.orc_stencil_apply.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = None
        L.orc_get_threads.argtypes = []
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(k: int) -> None:
    lib().orc_set_threads(int(k))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def encode(fmt: str, v):
    """Compress v (float64) to the storage format; returns (q, scale)."""
    v = _f64(v)
    q = np.empty(v.shape[0], dtype=STORAGE_DTYPE[fmt])
    sc = C.c_double(0.0)
    rc = lib().orc_encode(FORMATS[fmt], v.shape[0], _p(v), _p(q), C.byref(sc))
    if rc != 0:
        raise ValueError(f"orc_encode: {rc}")
    return q, sc.value


def decode(fmt: str, q, scale: float = 1.0) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=STORAGE_DTYPE[fmt])
    out = np.empty(q.shape[0], dtype=np.float64)
    rc = lib().orc_decode(FORMATS[fmt], q.shape[0], _p(q), float(scale), _p(out))
    if rc != 0:
        raise ValueError(f"orc_decode: {rc}")
    return out


def spmv(A, x) -> np.ndarray:
    x = _f64(x)
    y = np.empty(A.n, dtype=np.float64)
    lib().orc_spmv(A.n, _p(A.row_ptr), _p(A.col_idx), _p(A.val), _p(x), _p(y))
    return y


def dot(x, y) -> float:
    x, y = _f64(x), _f64(y)
    return float(lib().orc_dot(x.shape[0], _p(x), _p(y)))


def block_jacobi(A, bs=4, prec_min=16):
    """The block-Jacobi preconditioner's stored inverse blocks: (vals, prec)
    with vals (n_blocks, bs, bs) float64 (the stored values) and prec
    (n_blocks,) int8 in {16, 32, 64}.  Raises ValueError for a singular block."""
    nblk = (A.n + bs - 1) // bs
    vals = np.zeros(nblk * bs * bs)
    prec = np.zeros(nblk, dtype=np.int8)
    rc = lib().orc_block_jacobi(A.n, _p(A.row_ptr), _p(A.col_idx), _p(A.val), bs, prec_min,
                                _p(vals), _p(prec))
    if rc != 0:
        raise ValueError(f"orc_block_jacobi: {rc}")
    return vals.reshape(nblk, bs, bs), prec


def stencil_apply(A, grid, codes, v):
    """z = M^-1 v for the stencil preconditioner (orc_opts, ORC_PC_STENCIL):
    codes (27, ld) uint16 float16 codes, slot-major."""
    codes = np.ascontiguousarray(codes, dtype=np.uint16)
    v = _f64(v)
    z = np.empty(A.n, dtype=np.float64)
    g = (C.c_int32 * 3)(*[int(t) for t in grid])
    rc = lib().orc_stencil_apply(A.n, _p(A.row_ptr), _p(A.col_idx), _p(A.val), g, _p(codes),
                                 codes.shape[1], _p(v), _p(z))
    if rc != 0:
        raise ValueError(f"orc_stencil_apply: {rc}")
    return z


def gmres(A, b, x0=None, restart=100, fmt="fp64", tol=1e-10, maxiter=10000, eta=0.0,
          precond="none", p_val=None, fallback=False, debug=False, pc_block=0, pc_prec=0,
          variant=(), p_stencil=None, grid=(0, 0, 0)):
    """Run the oracle solver. Returns a dict with x, status, counts, the
    recurrence-residual history and the explicit residual per cycle; with
    ``debug`` also the first cycle's decoded basis V (k x n) and its
    Hessenberg matrix H ((m+1) x m, before Givens).  ``variant``: names from
    VARIANTS (ablations of the Arnoldi step; empty is Fig. 1 as written)."""
    n = A.n
    b = _f64(b)
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    pv = None
    if precond == "sparse":
        pv = np.ascontiguousarray(p_val, dtype=np.float32)
    st = None
    if precond == "stencil":
        st = np.ascontiguousarray(p_stencil, dtype=np.uint16)
    vbits = 0
    for name in ((variant,) if isinstance(variant, str) else variant):
        vbits |= VARIANTS[name]
    opts = _Opts(restart, FORMATS[fmt], tol, maxiter, eta, PRECONDS[precond],
                 None if pv is None else pv.ctypes.data, int(bool(fallback)), pc_block, pc_prec,
                 vbits, 0, None if st is None else st.ctypes.data,
                 (C.c_int32 * 3)(*[int(t) for t in grid]), 0 if st is None else st.shape[1])
    res = _Result()
    hist = np.full(max(maxiter, 1), np.nan)
    cyc = np.full(max(maxiter, 1) + 2, np.nan)
    clen = np.zeros(max(maxiter, 1) + 1, dtype=np.int32)
    V = H = None
    steps = (C.c_int32 * 2)(0, 0)
    if debug:
        V = np.zeros((restart + 1, n))
        H = np.zeros((restart, restart + 1))   # column-major (m+1) x m
    rc = lib().orc_gmres(n, _p(A.row_ptr), _p(A.col_idx), _p(A.val), _p(b), _p(x),
                         C.byref(opts), C.byref(res), _p(hist), _p(cyc), _p(clen), _p(V), _p(H),
                         steps)
    out = dict(x=x, status=rc, iterations=res.iterations, restarts=res.restarts,
               reorths=res.reorths, breakdowns=res.breakdowns, fell_back=res.fell_back,
               true_rel_res=res.true_rel_res, recurrence_rel_res=res.recurrence_rel_res,
               hist=hist[:res.iterations].copy(),
               cycle_res=cyc[:res.restarts + 1].copy(),
               cycle_len=clen[:res.restarts].copy())
    if debug:
        k, nv = steps[0], steps[1]
        out["V"] = V[:nv]
        out["H"] = H.T[:k + 1, :k]
        out["steps"] = k
    return out
