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

FORMATS = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3, "e4m3": 4, "int32": 5, "int16": 6,
           "fp16s": 7}
FORMAT_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2, "e4m3": 1, "int32": 4, "int16": 2,
                "fp16s": 2}
PRECONDS = {"none": 0, "jacobi": 1, "sparse": 2, "block_jacobi": 3, "stencil": 4}
OK, NOT_CONVERGED = 0, 1
E_ARG, E_WORKSPACE, E_HIP, E_NONFINITE, E_UNSUPPORTED = -1, -2, -3, -4, -5
FLAG_PROFILE = 1
FLAG_NO_FUSE = 2
FLAG_PROFILE_DOT = 4
FLAG_SPMV_VHAT = 8
FLAG_ALWAYS_REORTH = 16
FLAG_MGS = 32
FLAG_NORMALISE_PASS = 64
FLAG_NORMALISE_GATHER = 128
FLAG_EXPLICIT_REDOT = 256
FLAG_TWO_PASS = 512
FLAG_PROFILE_SPMV = 1024
FLAG_PROFILE_SAMPLED = 2048
PROFILE_STRIDE = 8
# where steps 13-14 run: solve(..., normalise=...)
NORMALISE = {"auto": 0, "pass": FLAG_NORMALISE_PASS, "gather": FLAG_NORMALISE_GATHER}
# Arnoldi-step variants by name, the names the oracle uses: "gram" is the
# Gram-form re-dot with separate passes, ("gram", "onepass") steps 5-10 in
# one update (the library's default), "explicit_redot" the form Fig. 1
# writes; an empty variant is the library's default.
VARIANTS = ("spmv_vhat", "always_reorth", "mgs", "gram", "onepass", "explicit_redot")


def variant_flags(names) -> int:
    names = set((names,) if isinstance(names, str) else names)
    unknown = names - set(VARIANTS)
    if unknown:
        raise KeyError(f"unknown variant(s) {sorted(unknown)}")
    if "onepass" in names and "gram" not in names:
        raise KeyError("onepass needs gram")
    f = 0
    f |= FLAG_SPMV_VHAT if "spmv_vhat" in names else 0
    f |= FLAG_ALWAYS_REORTH if "always_reorth" in names else 0
    f |= FLAG_MGS if "mgs" in names else 0
    f |= FLAG_EXPLICIT_REDOT if "explicit_redot" in names else 0
    f |= FLAG_TWO_PASS if "gram" in names and "onepass" not in names else 0
    return f

EXPORTS = ["cbg_strerror", "cbg_last_hip_error", "cbg_basis_ld", "cbg_workspace_bytes", "cbg_kernel_workspace_bytes",
           "cbg_workspace_basis", "cbgmres_solve", "cbg_encode", "cbg_decode", "cbg_spmv",
           "cbg_multidot", "cbg_multidot_noalloc", "cbg_update", "cbg_update_redot",
           "cbg_sell_ptr", "cbg_sell_fill", "cbg_sell_diag",
           "cbg_block_jacobi_setup",
           "cbg_block_jacobi_apply", "cbg_spai_workspace_bytes", "cbg_spai_features", "cbg_mlp_forward",
           "cbg_spai_assemble", "cbg_learned_build", "cbg_learned_build_stencil",
           "cbg_stencil_apply", "cbg_csr_transpose_values", "cbg_spai_pack", "cbg_spai_grad_p", "cbg_spai_grad_o", "cbg_mlp_backward",
           "cbg_spai_loss_grad", "cbg_spai_round_weights", "cbg_adam_step"]

SPAI_NFEAT, SPAI_NHID, SPAI_NOUT = 64, 64, 32
SPAI_NPARAM, SPAI_NWEIGHT, SPAI_MAX_K = 10400, 10240, 32


class CbgCsr(C.Structure):
    _fields_ = [("n", C.c_int32), ("reserved", C.c_int32), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p),
                ("sell_ptr", C.c_void_p), ("sell_col", C.c_void_p), ("sell_val", C.c_void_p),
                ("sell_entries", C.c_int64), ("sell_dix", C.c_void_p), ("sell_diag", C.c_void_p),
                ("sell_ndiag", C.c_int32), ("reserved2", C.c_int32)]


class CbgOpts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("format", C.c_int32), ("tol", C.c_double),
                ("maxiter", C.c_int64), ("eta", C.c_double), ("precond", C.c_int32),
                ("fallback", C.c_int32), ("p_val", C.c_void_p), ("flags", C.c_int32),
                ("reserved", C.c_int32), ("pc_block", C.c_int32), ("pc_prec", C.c_int32),
                ("p_stencil", C.c_void_p), ("grid", C.c_int32 * 3), ("reserved2", C.c_int32)]


class CbgResult(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("restarts", C.c_int64), ("reorths", C.c_int64),
                ("status", C.c_int32), ("breakdowns", C.c_int32), ("fell_back", C.c_int32),
                ("reserved", C.c_int32), ("true_rel_res", C.c_double),
                ("recurrence_rel_res", C.c_double), ("seconds", C.c_double),
                ("model_bytes", C.c_double), ("prof_orth_ms", C.c_double),
                ("prof_orth_bytes", C.c_double), ("prof_orth_launches", C.c_int64),
                ("prof_dot_ms", C.c_double), ("prof_dot_bytes", C.c_double),
                ("prof_dot_launches", C.c_int64), ("prof_fused_ms", C.c_double),
                ("prof_fused_bytes", C.c_double), ("prof_fused_launches", C.c_int64),
                ("explicit_steps", C.c_int64), ("prof_spmv_ms", C.c_double),
                ("prof_spmv_bytes", C.c_double), ("prof_spmv_launches", C.c_int64)]


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
        # torch first: the library then binds to the HIP runtime torch has
        # loaded, so device pointers and streams from torch are valid in it
        # (loaded the other way round, a second runtime reports no device)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        L.cbg_strerror.argtypes = [C.c_int]
        L.cbg_strerror.restype = C.c_char_p
        L.cbg_last_hip_error.argtypes = [C.POINTER(C.c_int), C.POINTER(C.c_char_p)]
        L.cbg_last_hip_error.restype = C.c_int
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
        L.cbg_sell_ptr.argtypes = [C.POINTER(CbgCsr), vp, C.POINTER(i64), vp]
        L.cbg_sell_fill.argtypes = [C.POINTER(CbgCsr), vp, vp, vp, vp]
        L.cbg_sell_diag.argtypes = [C.POINTER(CbgCsr), vp, vp, C.POINTER(i32), vp, sz, vp]
        L.cbg_multidot.argtypes = [i32, vp, i64, vp, i32, i32, vp, vp, vp, sz, vp]
        L.cbg_multidot_noalloc.argtypes = [i32, vp, i64, vp, i32, i32, vp, vp, vp]
        L.cbg_update.argtypes = [i32, vp, i64, vp, i32, i32, vp, vp, vp, vp, sz, vp]
        L.cbg_update_redot.argtypes = [i32, vp, i64, vp, i32, i32, vp, vp, vp, vp, vp, sz, vp]
        L.cbg_block_jacobi_setup.argtypes = [C.POINTER(CbgCsr), i32, i32, vp, vp, vp, vp, vp, sz,
                                             vp]
        L.cbg_block_jacobi_apply.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp]
        L.cbg_workspace_basis.argtypes = [i32, i32, i32, i32, C.POINTER(sz), C.POINTER(sz)]
        pcsr, f64 = C.POINTER(CbgCsr), C.c_double
        L.cbg_spai_workspace_bytes.argtypes = [i32, i64, i32]
        L.cbg_spai_workspace_bytes.restype = sz
        L.cbg_spai_features.argtypes = [pcsr, vp, vp, vp, sz, vp]
        L.cbg_mlp_forward.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp]
        L.cbg_spai_assemble.argtypes = [pcsr, vp, vp, vp, vp]
        L.cbg_learned_build.argtypes = [pcsr, vp, vp, vp, vp, vp, sz, vp]
        L.cbg_learned_build_stencil.argtypes = [pcsr, vp, vp, vp, vp, vp, sz, vp]
        L.cbg_stencil_apply.argtypes = [pcsr, vp, vp, vp, vp, vp, sz, vp]
        L.cbg_csr_transpose_values.argtypes = [pcsr, vp, vp, sz, vp]
        L.cbg_spai_pack.argtypes = [vp, i64, i32, i32, i32, i32, vp, vp]
        L.cbg_spai_grad_p.argtypes = [pcsr, vp, vp, i32, vp, f64, vp, i32, vp, vp, sz, vp]
        L.cbg_spai_grad_o.argtypes = [pcsr, vp, vp, vp, vp]
        L.cbg_mlp_backward.argtypes = [i32, vp, vp, vp, vp, vp, vp, i32, vp, sz, vp]
        L.cbg_spai_loss_grad.argtypes = [pcsr, vp, vp, vp, vp, vp, i32, vp, f64, vp, vp, i32,
                                         vp, sz, vp]
        L.cbg_spai_round_weights.argtypes = [vp, vp, vp]
        L.cbg_adam_step.argtypes = [vp, vp, vp, vp, vp, i64, f64, f64, f64, f64, vp]
        for f in ("cbgmres_solve", "cbg_encode", "cbg_decode", "cbg_spmv", "cbg_multidot",
                  "cbg_multidot_noalloc", "cbg_sell_ptr", "cbg_sell_fill", "cbg_sell_diag",
                  "cbg_update", "cbg_update_redot", "cbg_block_jacobi_setup",
                  "cbg_block_jacobi_apply", "cbg_workspace_basis", "cbg_spai_features", "cbg_mlp_forward",
                  "cbg_spai_assemble", "cbg_learned_build", "cbg_learned_build_stencil",
                  "cbg_stencil_apply", "cbg_csr_transpose_values",
                  "cbg_spai_pack", "cbg_spai_grad_p", "cbg_spai_grad_o", "cbg_mlp_backward",
                  "cbg_spai_loss_grad", "cbg_spai_round_weights", "cbg_adam_step"):
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


def workspace_basis(n: int, restart: int, fmt: str, precond: str = "none"):
    """(basis_offset, scales_offset) in bytes inside a solve workspace."""
    bo, so = C.c_size_t(), C.c_size_t()
    _check(lib().cbg_workspace_basis(int(n), int(restart), FORMATS[fmt], PRECONDS[precond],
                                     C.byref(bo), C.byref(so)), "cbg_workspace_basis")
    return int(bo.value), int(so.value)


def spai_workspace_bytes(n: int, nnz: int, K: int = 0) -> int:
    return int(lib().cbg_spai_workspace_bytes(int(n), int(nnz), int(K)))


# ---------------------------------------------------------------- torch glue

def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, name: str, dtype, numel: int, device=None, exact: bool = False, gpu: bool = True):
    """Raise ValueError unless t is a contiguous tensor of `dtype` holding at
    least `numel` elements (exactly `numel` with exact=True) on a GPU
    (`device`, if given).  The C ABI takes bare pointers and cannot check
    lengths, so a short or mistyped tensor would let the kernels read or
    write past its allocation."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if (t.numel() != numel) if exact else (t.numel() < numel):
        raise ValueError(f"{name}: {t.numel()} elements, expected "
                         f"{'' if exact else 'at least '}{numel}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor is not contiguous")
    if not gpu:
        return t
    if t.device.type != "cuda":
        raise ValueError(f"{name}: tensor on {t.device}, expected a GPU tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name}: tensor on {t.device}, expected {device}")
    return t


def _dev_of(A):
    return A.val.device


def last_hip_error():
    """(hipError_t, library source line, error name) of the last failing HIP
    call on this thread (0 if none)."""
    line = C.c_int(0)
    name = C.c_char_p()
    code = lib().cbg_last_hip_error(C.byref(line), C.byref(name))
    return code, line.value, (name.value or b"").decode()


def _check(rc: int, where: str):
    if rc < 0:
        if rc == E_HIP:
            code, line, name = last_hip_error()
            where = f"{where} [{name} ({code}) at line {line}]"
        raise CbgError(rc, where)
    return rc


SELL_SLICE = 64
# the sliced-ELL copy is kept when its padding is at most this fraction of nnz
SELL_MAX_PADDING = 0.25
SELL_MAX_DIAG = 256


@dataclasses.dataclass
class DeviceCSR:
    """A CSR matrix resident in device memory (int32 indices, fp64 values),
    with an optional sliced-ELL copy (SELL-64, cbg_sell_ptr / cbg_sell_fill)
    that the SpMV with A reads when present."""
    n: int
    nnz: int
    row_ptr: "object"
    col_idx: "object"
    val: "object"
    sell_ptr: "object" = None
    sell_col: "object" = None
    sell_val: "object" = None
    sell_dix: "object" = None
    sell_diag: "object" = None
    sell_ndiag: int = 0

    @classmethod
    def from_host(cls, A, device="cuda", sell="auto", diag=True):
        """Copy a host CSR matrix to the GPU.  sell: "auto" builds the
        sliced-ELL copy unless its padding exceeds SELL_MAX_PADDING of nnz;
        True builds it regardless; False keeps the CSR kernels.  diag: store
        the copy's columns as diagonal indices when A has at most
        SELL_MAX_DIAG distinct offsets col - row."""
        torch = _torch()
        rp = torch.from_numpy(np.ascontiguousarray(A.row_ptr, dtype=np.int32)).to(device)
        ci = torch.from_numpy(np.ascontiguousarray(A.col_idx, dtype=np.int32)).to(device)
        va = torch.from_numpy(np.ascontiguousarray(A.val, dtype=np.float64)).to(device)
        D = cls(int(A.n), int(A.nnz), rp, ci, va)
        if sell and D.n > 0 and (sell is True or D.val.device.type == "cuda"):
            D.build_sell(max_padding=None if sell is True else SELL_MAX_PADDING, diag=diag)
        return D

    def build_sell(self, max_padding=None, diag=True, keep_col=False):
        """Build the sliced-ELL copy on the GPU (kept only if its padding is
        at most max_padding of nnz, when given), with diagonal-index columns
        when diag and A has few enough distinct offsets (then the int32
        columns are dropped unless keep_col).  Returns self."""
        torch = _torch()
        self.drop_sell()
        dev = self.val.device
        nslice = (self.n + SELL_SLICE - 1) // SELL_SLICE
        sp = torch.empty(nslice + 1, dtype=torch.int64, device=dev)
        ent = C.c_int64(0)
        csr = self.cstruct()
        _check(lib().cbg_sell_ptr(C.byref(csr), _ptr(sp), C.byref(ent), _stream()),
               "cbg_sell_ptr")
        entries = int(ent.value)
        if max_padding is not None and entries > (1.0 + max_padding) * max(self.nnz, 1):
            return self
        sc = torch.empty(max(entries, 1), dtype=torch.int32, device=dev)
        sv = torch.empty(max(entries, 1), dtype=torch.float64, device=dev)
        _check(lib().cbg_sell_fill(C.byref(csr), _ptr(sp), _ptr(sc), _ptr(sv), _stream()),
               "cbg_sell_fill")
        self.sell_ptr, self.sell_col, self.sell_val = sp, sc[:entries], sv[:entries]
        if diag:
            dg = torch.empty(SELL_MAX_DIAG, dtype=torch.int32, device=dev)
            dx = torch.empty(max(entries, 1), dtype=torch.uint8, device=dev)
            nd = C.c_int32(0)
            csr = self.cstruct()
            ws = _kws(self.n, 0, dev)
            rc = lib().cbg_sell_diag(C.byref(csr), _ptr(dg), _ptr(dx), C.byref(nd), _ptr(ws),
                                     ws.numel(), _stream())
            if rc == E_UNSUPPORTED:
                return self                     # too many distinct offsets: int32 columns
            _check(rc, "cbg_sell_diag")
            self.sell_dix, self.sell_diag, self.sell_ndiag = dx[:entries], dg, int(nd.value)
            if not keep_col:
                self.sell_col = None
        return self

    def drop_sell(self):
        """Forget the sliced-ELL copy (the CSR kernels run).  Returns self."""
        self.sell_ptr = self.sell_col = self.sell_val = None
        self.sell_dix = self.sell_diag = None
        self.sell_ndiag = 0
        return self

    @property
    def sell_entries(self) -> int:
        return 0 if self.sell_val is None else int(self.sell_val.numel())

    def check(self):
        """Raise ValueError unless the arrays match n and nnz (int32 indices,
        fp64 values, contiguous, one GPU), and the sliced-ELL arrays, if any,
        match each other."""
        torch = _torch()
        if self.n < 0 or self.nnz < 0:
            raise ValueError(f"CSR: n = {self.n}, nnz = {self.nnz}")
        dev = self.val.device
        arrays = [(self.row_ptr, "A.row_ptr", torch.int32, self.n + 1),
                  (self.col_idx, "A.col_idx", torch.int32, self.nnz),
                  (self.val, "A.val", torch.float64, self.nnz)]
        dix = (self.sell_dix, self.sell_diag)
        if any(t is not None for t in dix) and (any(t is None for t in dix) or
                                                not 1 <= self.sell_ndiag <= SELL_MAX_DIAG):
            raise ValueError("A.sell_dix / sell_diag / sell_ndiag: given together, "
                             f"1 <= ndiag <= {SELL_MAX_DIAG}")
        cols = self.sell_col if self.sell_col is not None else self.sell_dix
        sell = (self.sell_ptr, cols, self.sell_val)
        if any(t is not None for t in sell):
            if any(t is None for t in sell):
                raise ValueError("A.sell_*: the sliced-ELL arrays are all given or none")
            ent = self.sell_entries
            if ent < self.nnz or ent % SELL_SLICE:
                raise ValueError(f"A.sell_val: {ent} entries for nnz = {self.nnz}")
            arrays += [(self.sell_ptr, "A.sell_ptr", torch.int64,
                        (self.n + SELL_SLICE - 1) // SELL_SLICE + 1),
                       (self.sell_val, "A.sell_val", torch.float64, ent)]
            if self.sell_col is not None:
                arrays.append((self.sell_col, "A.sell_col", torch.int32, ent))
            if self.sell_dix is not None:
                arrays += [(self.sell_dix, "A.sell_dix", torch.uint8, ent),
                           (self.sell_diag, "A.sell_diag", torch.int32, SELL_MAX_DIAG)]
        for gpu in (False, True):           # shapes first, then the device
            for t, nm, dt, cnt in arrays:
                _need(t, nm, dt, cnt, dev, exact=True, gpu=gpu)
        return self

    def cstruct(self) -> CbgCsr:
        self.check()
        ptr = lambda t: None if t is None else t.data_ptr()
        if self.sell_val is None:
            return CbgCsr(self.n, 0, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(),
                          self.val.data_ptr(), None, None, None, 0, None, None, 0, 0)
        return CbgCsr(self.n, 0, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(),
                      self.val.data_ptr(), ptr(self.sell_ptr), ptr(self.sell_col),
                      ptr(self.sell_val), self.sell_entries, ptr(self.sell_dix),
                      ptr(self.sell_diag), self.sell_ndiag if self.sell_dix is not None else 0, 0)


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
    prof_fused_ms: float = 0.0
    prof_fused_bytes: float = 0.0
    prof_fused_launches: int = 0
    explicit_steps: int = 0
    prof_spmv_ms: float = 0.0
    prof_spmv_bytes: float = 0.0
    prof_spmv_launches: int = 0


def solve(A: DeviceCSR, b, x0=None, restart=100, fmt="fp64", tol=1e-10, maxiter=10000,
          eta=0.0, precond="none", p_val=None, fallback=False, profile=False, workspace=None,
          hist=True, fuse=True, pc_block=0, pc_prec=0, variant=(),
          normalise="auto", p_stencil=None, grid=None) -> SolveResult:
    """cbgmres_solve on device tensors; returns the solution and counters.
    precond "stencil" takes p_stencil (27 * basis_ld(n) int16 float16 codes,
    from learned_build_stencil) and grid (nx, ny, nz).
    profile: False, True (event-time every basis-streaming launch), "dot"
    (only the multi-dot launches), "spmv" (only the steps' SpMV with A) or
    "all" (both kinds); a suffix "/sampled" (e.g. "spmv/sampled") times only
    every PROFILE_STRIDE-th Arnoldi step's launches.  variant: names from VARIANTS (ablations
    of the Arnoldi step).  normalise: "auto", "pass" or "gather" (where
    v_j = w / t is formed; the same bits either way).  Raises CbgError on a
    negative status."""
    torch = _torch()
    A.check()
    dev = _dev_of(A)
    _need(b, "b", torch.float64, A.n, dev, exact=True)
    if x0 is not None:
        _need(x0, "x0", torch.float64, A.n, dev, exact=True)
    if precond == "sparse" or p_val is not None:
        if p_val is None:
            raise ValueError("p_val: the sparse preconditioner needs its values")
        _need(p_val, "p_val", torch.float32, A.nnz, dev, exact=True)
    g3 = (0, 0, 0)
    if precond == "stencil" or p_stencil is not None:
        if p_stencil is None or grid is None:
            raise ValueError("the stencil preconditioner needs p_stencil and grid")
        _need(p_stencil, "p_stencil", torch.int16, 27 * basis_ld(A.n), dev, exact=True)
        g3 = tuple(_grid3(grid, A.n))
    x = torch.zeros(A.n, dtype=torch.float64, device=b.device) if x0 is None else x0.clone()
    need = workspace_bytes(A.n, restart, fmt, precond)
    if need == 0 and A.n > 0:
        raise CbgError(E_ARG, "cbg_workspace_bytes")
    if workspace is not None:
        _need(workspace, "workspace", torch.uint8, 0, dev)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=b.device)
    kind, _, sampled = str(profile).partition("/")
    flags = {"False": 0, "True": FLAG_PROFILE, "dot": FLAG_PROFILE_DOT,
             "spmv": FLAG_PROFILE_SPMV, "all": FLAG_PROFILE | FLAG_PROFILE_SPMV}[kind] \
        | (0 if fuse else FLAG_NO_FUSE) | NORMALISE[normalise]
    if sampled:
        if sampled != "sampled" or kind == "False":
            raise ValueError(f"profile: {profile!r}")
        flags |= FLAG_PROFILE_SAMPLED
    flags |= variant_flags(variant)
    opts = CbgOpts(restart, FORMATS[fmt], tol, maxiter, eta, PRECONDS[precond],
                   int(bool(fallback)), None if p_val is None else p_val.data_ptr(),
                   flags, 0, pc_block, pc_prec,
                   None if p_stencil is None else p_stencil.data_ptr(),
                   (C.c_int32 * 3)(*g3), 0)
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
                       prof_dot_launches=res.prof_dot_launches,
                       prof_fused_ms=res.prof_fused_ms, prof_fused_bytes=res.prof_fused_bytes,
                       prof_fused_launches=res.prof_fused_launches,
                       explicit_steps=res.explicit_steps, prof_spmv_ms=res.prof_spmv_ms,
                       prof_spmv_bytes=res.prof_spmv_bytes,
                       prof_spmv_launches=res.prof_spmv_launches)


def _kws(n, j, device):
    torch = _torch()
    return torch.empty(max(kernel_workspace_bytes(n, j), 256), dtype=torch.uint8, device=device)


def encode(fmt: str, v, out=None, scale=None, ws=None):
    """The accessor's store: returns (q, scale) on the device."""
    torch = _torch()
    n = v.numel()
    _need(v, "v", torch.float64, n)
    dt = {"fp64": torch.float64, "fp32": torch.float32, "fp16": torch.int16, "bf16": torch.int16,
          "e4m3": torch.uint8, "int32": torch.int32, "int16": torch.int16,
          "fp16s": torch.int16}[fmt]
    q = torch.empty(n, dtype=dt, device=v.device) if out is None else out
    sc = torch.empty(1, dtype=torch.float64, device=v.device) if scale is None else scale
    ws = _kws(n, 0, v.device) if ws is None else ws
    _need(q, "q", dt, n, v.device)
    _need(sc, "scale", torch.float64, 1, v.device)
    _need(ws, "ws", torch.uint8, kernel_workspace_bytes(n, 0), v.device)
    _check(lib().cbg_encode(FORMATS[fmt], _ptr(v), n, _ptr(q), _ptr(sc), _ptr(ws), ws.numel(),
                            _stream()), "cbg_encode")
    return q, sc


def decode(fmt: str, q, scale, n=None):
    torch = _torch()
    n = q.numel() if n is None else n
    if q.dtype not in (torch.float64, torch.float32, torch.int16, torch.uint8, torch.int32) or \
            q.element_size() != FORMAT_BYTES[fmt]:
        raise ValueError(f"q: dtype {q.dtype} does not hold {fmt} codes")
    _need(q, "q", q.dtype, n)
    _need(scale, "scale", torch.float64, 1, q.device)
    v = torch.empty(n, dtype=torch.float64, device=q.device)
    _check(lib().cbg_decode(FORMATS[fmt], _ptr(q), _ptr(scale), n, _ptr(v), _stream()),
           "cbg_decode")
    return v


def spmv(A: DeviceCSR, x, y=None, want_norm=False):
    torch = _torch()
    A.check()
    _need(x, "x", torch.float64, A.n, _dev_of(A))
    y = torch.empty(A.n, dtype=torch.float64, device=x.device) if y is None else y
    _need(y, "y", torch.float64, A.n, _dev_of(A))
    nrm = torch.empty(1, dtype=torch.float64, device=x.device) if want_norm else None
    ws = _kws(A.n, 0, x.device) if want_norm else None
    csr = A.cstruct()
    _check(lib().cbg_spmv(C.byref(csr), _ptr(x), _ptr(y), _ptr(nrm), _ptr(ws),
                          0 if ws is None else ws.numel(), _stream()), "cbg_spmv")
    return (y, nrm) if want_norm else y


def _check_basis(fmt, V, ld, scales, n, j, device):
    """The stored basis: j vectors of ld entries (ld >= n) in `fmt`, one fp64
    scale each."""
    torch = _torch()
    if ld < n:
        raise ValueError(f"ld = {ld} < n = {n}")
    if j > 0:
        if not isinstance(V, torch.Tensor) or V.device != device or not V.is_contiguous():
            raise ValueError("V: expected a contiguous tensor on the GPU of w")
        if V.numel() * V.element_size() < j * ld * FORMAT_BYTES[fmt]:
            raise ValueError(f"V: {V.numel() * V.element_size()} bytes, expected at least "
                             f"{j * ld * FORMAT_BYTES[fmt]} ({j} vectors of {ld} {fmt} entries)")
        _need(scales, "scales", torch.float64, j, device)


def multidot(fmt: str, V, ld: int, scales, n: int, j: int, w, h=None, ws=None):
    torch = _torch()
    _need(w, "w", torch.float64, n)
    _check_basis(fmt, V, ld, scales, n, j, w.device)
    h = torch.empty(max(j, 1), dtype=torch.float64, device=w.device) if h is None else h
    ws = _kws(n, j, w.device) if ws is None else ws
    _need(h, "h", torch.float64, j, w.device)
    _need(ws, "ws", torch.uint8, kernel_workspace_bytes(n, j), w.device)
    _check(lib().cbg_multidot(FORMATS[fmt], _ptr(V), ld, _ptr(scales), n, j, _ptr(w), _ptr(h),
                              _ptr(ws), ws.numel(), _stream()), "cbg_multidot")
    return h[:j]


NOALLOC_MAX_J = 128


def multidot_noalloc(fmt: str, V, ld: int, scales, n: int, j: int, w, h):
    """cbg_multidot_noalloc: h[:j] = V^T w with the library's own per-GPU
    scratch array (no workspace argument; h is the caller's)."""
    torch = _torch()
    _need(w, "w", torch.float64, n)
    _check_basis(fmt, V, ld, scales, n, j, w.device)
    _need(h, "h", torch.float64, j, w.device)
    _check(lib().cbg_multidot_noalloc(FORMATS[fmt], _ptr(V), ld, _ptr(scales), n, j, _ptr(w),
                                      _ptr(h), _stream()), "cbg_multidot_noalloc")
    return h[:j]


def update(fmt: str, V, ld: int, scales, n: int, j: int, h, w, norms=None, ws=None):
    torch = _torch()
    _need(w, "w", torch.float64, n)
    _check_basis(fmt, V, ld, scales, n, j, w.device)
    _need(h, "h", torch.float64, j, w.device)
    norms = torch.empty(2, dtype=torch.float64, device=w.device) if norms is None else norms
    ws = _kws(n, 0, w.device) if ws is None else ws
    _need(norms, "norms", torch.float64, 2, w.device)
    _need(ws, "ws", torch.uint8, kernel_workspace_bytes(n, 0), w.device)
    _check(lib().cbg_update(FORMATS[fmt], _ptr(V), ld, _ptr(scales), n, j, _ptr(h), _ptr(w),
                            _ptr(norms), _ptr(ws), ws.numel(), _stream()), "cbg_update")
    return norms


def update_redot(fmt: str, V, ld: int, scales, n: int, j: int, h, w, ws=None):
    """w -= V h, then (u = V^T w, norms = [||w||_2, ||w||_inf]) in one pass."""
    torch = _torch()
    _need(w, "w", torch.float64, n)
    _check_basis(fmt, V, ld, scales, n, j, w.device)
    _need(h, "h", torch.float64, j, w.device)
    u = torch.empty(max(j, 1), dtype=torch.float64, device=w.device)
    norms = torch.empty(2, dtype=torch.float64, device=w.device)
    ws = _kws(n, j, w.device) if ws is None else ws
    _need(ws, "ws", torch.uint8, kernel_workspace_bytes(n, j), w.device)
    _check(lib().cbg_update_redot(FORMATS[fmt], _ptr(V), ld, _ptr(scales), n, j, _ptr(h),
                                  _ptr(w), _ptr(u), _ptr(norms), _ptr(ws), ws.numel(),
                                  _stream()), "cbg_update_redot")
    return u[:j], norms


def block_jacobi_setup(A: DeviceCSR, bs=4, prec_min=16):
    """(tags int8[nblk], x64, x32, x16) device tensors of the block-Jacobi
    preconditioner's stored inverse blocks."""
    torch = _torch()
    dev = A.val.device
    nblk = (A.n + bs - 1) // bs
    tags = torch.empty(max(nblk, 1), dtype=torch.int8, device=dev)
    x64 = torch.zeros(max(nblk * bs * bs, 1), dtype=torch.float64, device=dev)
    x32 = torch.zeros_like(x64, dtype=torch.float32)
    x16 = torch.zeros_like(x64, dtype=torch.int16)
    ws = _kws(A.n, 0, dev)
    csr = A.cstruct()
    _check(lib().cbg_block_jacobi_setup(C.byref(csr), bs, prec_min, _ptr(tags), _ptr(x64),
                                        _ptr(x32), _ptr(x16), _ptr(ws), ws.numel(), _stream()),
           "cbg_block_jacobi_setup")
    return tags, x64, x32, x16


def block_jacobi_apply(n, bs, blocks, v, z=None):
    torch = _torch()
    tags, x64, x32, x16 = blocks
    nblk = (n + bs - 1) // bs
    _need(v, "v", torch.float64, n)
    _need(tags, "tags", torch.int8, nblk, v.device)
    for t, nm, dt in ((x64, "x64", torch.float64), (x32, "x32", torch.float32),
                      (x16, "x16", torch.int16)):
        _need(t, nm, dt, nblk * bs * bs, v.device)
    z = torch.empty(n, dtype=torch.float64, device=v.device) if z is None else z
    _need(z, "z", torch.float64, n, v.device)
    _check(lib().cbg_block_jacobi_apply(n, bs, _ptr(tags), _ptr(x64), _ptr(x32), _ptr(x16),
                                        _ptr(v), _ptr(z), _stream()), "cbg_block_jacobi_apply")
    return z


# ------------------------------------------------ learned preconditioner

def _grid3(grid, n=None):
    g = [int(v) for v in grid]
    if len(g) != 3 or min(g) < 1 or (n is not None and g[0] * g[1] * g[2] != n):
        raise ValueError(f"grid {tuple(grid)} does not number the {n} rows")
    return (C.c_int32 * 3)(*g)


def _sws(n, nnz, K, device):
    torch = _torch()
    return torch.empty(max(spai_workspace_bytes(n, nnz, K), 256), dtype=torch.uint8,
                       device=device)


def spai_features(A: DeviceCSR, grid, feat=None, ws=None):
    """(n, 64) int16 tensor of bf16 feature bit patterns."""
    torch = _torch()
    dev = A.val.device
    feat = torch.empty((A.n, SPAI_NFEAT), dtype=torch.int16, device=dev) if feat is None else feat
    ws = _sws(A.n, A.nnz, 0, dev) if ws is None else ws
    _need(feat, "feat", torch.int16, A.n * SPAI_NFEAT, dev)
    _need(ws, "ws", torch.uint8, spai_workspace_bytes(A.n, A.nnz, 0), dev)
    csr = A.cstruct()
    _check(lib().cbg_spai_features(C.byref(csr), _grid3(grid, A.n), _ptr(feat), _ptr(ws), ws.numel(),
                                   _stream()), "cbg_spai_features")
    return feat


def mlp_forward(feat, weights, params, keep_activations=False):
    """Returns O (n, 32) fp32, and (H1, H2) bf16 bit patterns if asked."""
    torch = _torch()
    n, dev = feat.shape[0], feat.device
    _need(feat, "feat", torch.int16, n * SPAI_NFEAT)
    _need(weights, "weights", torch.int16, SPAI_NWEIGHT, dev)
    _need(params, "params", torch.float32, SPAI_NPARAM, dev)
    O = torch.empty((n, SPAI_NOUT), dtype=torch.float32, device=dev)
    h1 = h2 = None
    if keep_activations:
        h1 = torch.empty((n, SPAI_NHID), dtype=torch.int16, device=dev)
        h2 = torch.empty((n, SPAI_NHID), dtype=torch.int16, device=dev)
    _check(lib().cbg_mlp_forward(n, _ptr(feat), _ptr(weights), _ptr(params), _ptr(O), _ptr(h1),
                                 _ptr(h2), _stream()), "cbg_mlp_forward")
    return (O, h1, h2) if keep_activations else O


def spai_assemble(A: DeviceCSR, grid, O, p_val=None):
    torch = _torch()
    p_val = torch.empty(A.nnz, dtype=torch.float32, device=O.device) if p_val is None else p_val
    _need(O, "O", torch.float32, A.n * SPAI_NOUT, _dev_of(A))
    _need(p_val, "p_val", torch.float32, A.nnz, _dev_of(A))
    csr = A.cstruct()
    _check(lib().cbg_spai_assemble(C.byref(csr), _grid3(grid, A.n), _ptr(O), _ptr(p_val), _stream()),
           "cbg_spai_assemble")
    return p_val


def learned_build(A: DeviceCSR, grid, weights, params, p_val=None, ws=None):
    """P values (nnz fp32) on A's pattern: features, forward pass, assembly."""
    torch = _torch()
    dev = A.val.device
    p_val = torch.empty(A.nnz, dtype=torch.float32, device=dev) if p_val is None else p_val
    ws = _sws(A.n, A.nnz, 0, dev) if ws is None else ws
    _need(weights, "weights", torch.int16, SPAI_NWEIGHT, dev)
    _need(params, "params", torch.float32, SPAI_NPARAM, dev)
    _need(p_val, "p_val", torch.float32, A.nnz, dev)
    _need(ws, "ws", torch.uint8, spai_workspace_bytes(A.n, A.nnz, 0), dev)
    csr = A.cstruct()
    _check(lib().cbg_learned_build(C.byref(csr), _grid3(grid, A.n), _ptr(weights), _ptr(params),
                                   _ptr(p_val), _ptr(ws), ws.numel(), _stream()),
           "cbg_learned_build")
    return p_val


def learned_build_stencil(A: DeviceCSR, grid, weights, params, p_stencil=None, ws=None):
    """The stored form for precond "stencil": (27 * basis_ld(n),) int16
    float16 codes, slot-major (features, forward pass, packing)."""
    torch = _torch()
    dev = A.val.device
    n_codes = 27 * basis_ld(A.n)
    p_stencil = torch.empty(n_codes, dtype=torch.int16, device=dev) if p_stencil is None \
        else p_stencil
    ws = _sws(A.n, A.nnz, 0, dev) if ws is None else ws
    _need(weights, "weights", torch.int16, SPAI_NWEIGHT, dev)
    _need(params, "params", torch.float32, SPAI_NPARAM, dev)
    _need(p_stencil, "p_stencil", torch.int16, n_codes, dev)
    _need(ws, "ws", torch.uint8, spai_workspace_bytes(A.n, A.nnz, 0), dev)
    csr = A.cstruct()
    _check(lib().cbg_learned_build_stencil(C.byref(csr), _grid3(grid, A.n), _ptr(weights),
                                           _ptr(params), _ptr(p_stencil), _ptr(ws), ws.numel(),
                                           _stream()), "cbg_learned_build_stencil")
    return p_stencil


def stencil_apply(A: DeviceCSR, grid, p_stencil, v, z=None, ws=None):
    """z = M^-1 v for the stencil preconditioner's stored form."""
    torch = _torch()
    dev = A.val.device
    _need(p_stencil, "p_stencil", torch.int16, 27 * basis_ld(A.n), dev)
    _need(v, "v", torch.float64, A.n, dev)
    z = torch.empty(A.n, dtype=torch.float64, device=dev) if z is None else z
    _need(z, "z", torch.float64, A.n, dev)
    ws = _sws(A.n, A.nnz, 0, dev) if ws is None else ws
    _need(ws, "ws", torch.uint8, spai_workspace_bytes(A.n, A.nnz, 0), dev)
    csr = A.cstruct()
    _check(lib().cbg_stencil_apply(C.byref(csr), _grid3(grid, A.n), _ptr(p_stencil), _ptr(v),
                                   _ptr(z), _ptr(ws), ws.numel(), _stream()),
           "cbg_stencil_apply")
    return z


def csr_transpose_values(A: DeviceCSR, ws=None):
    torch = _torch()
    dev = A.val.device
    t = torch.empty(A.nnz, dtype=torch.float64, device=dev)
    ws = _sws(A.n, A.nnz, 0, dev) if ws is None else ws
    _need(ws, "ws", torch.uint8, spai_workspace_bytes(A.n, A.nnz, 0), dev)
    csr = A.cstruct()
    _check(lib().cbg_csr_transpose_values(C.byref(csr), _ptr(t), _ptr(ws), ws.numel(),
                                          _stream()), "cbg_csr_transpose_values")
    return t


def spai_pack(V, ld: int, n: int, K: int, first: int = 0, stride: int = 1, out=None):
    """(n, K) int16 tensor of fp16 bit patterns from K FP64 vectors in V."""
    torch = _torch()
    if K < 1 or K > SPAI_MAX_K or first < 0 or stride < 1 or ld < n:
        raise ValueError(f"spai_pack: K = {K}, first = {first}, stride = {stride}, ld = {ld}")
    _need(V, "V", torch.float64, (first + (K - 1) * stride) * ld + n)
    out = torch.empty((n, K), dtype=torch.int16, device=V.device) if out is None else out
    _need(out, "out", torch.int16, n * K, V.device)
    _check(lib().cbg_spai_pack(_ptr(V), int(ld), int(n), int(K), int(first), int(stride),
                               _ptr(out), _stream()), "cbg_spai_pack")
    return out


def spai_grad_p(A: DeviceCSR, t_val, p_val, V, scale, ws=None):
    """(loss tensor[1], dP tensor[nnz]) for V (n, K) fp16 bit patterns."""
    torch = _torch()
    dev = A.val.device
    K = V.shape[1]
    _need(t_val, "t_val", torch.float64, A.nnz, dev)
    _need(p_val, "p_val", torch.float32, A.nnz, dev)
    _need(V, "V", torch.int16, A.n * K, dev)
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    dP = torch.empty(A.nnz, dtype=torch.float64, device=dev)
    ws = _sws(A.n, A.nnz, K, dev) if ws is None else ws
    _need(ws, "ws", torch.uint8, spai_workspace_bytes(A.n, A.nnz, K), dev)
    csr = A.cstruct()
    _check(lib().cbg_spai_grad_p(C.byref(csr), _ptr(t_val), _ptr(p_val), K, _ptr(V),
                                 float(scale), _ptr(loss), 0, _ptr(dP), _ptr(ws), ws.numel(),
                                 _stream()), "cbg_spai_grad_p")
    return loss, dP


def spai_grad_o(A: DeviceCSR, grid, dP):
    torch = _torch()
    _need(dP, "dP", torch.float64, A.nnz, _dev_of(A))
    dO = torch.empty((A.n, SPAI_NOUT), dtype=torch.int16, device=dP.device)
    csr = A.cstruct()
    _check(lib().cbg_spai_grad_o(C.byref(csr), _grid3(grid, A.n), _ptr(dP), _ptr(dO), _stream()),
           "cbg_spai_grad_o")
    return dO


def mlp_backward(feat, h1, h2, dO, weights, grad=None, accumulate=False, ws=None):
    torch = _torch()
    n, dev = feat.shape[0], feat.device
    grad = torch.empty(SPAI_NPARAM, dtype=torch.float64, device=dev) if grad is None else grad
    ws = _sws(n, 0, 0, dev) if ws is None else ws
    _need(feat, "feat", torch.int16, n * SPAI_NFEAT, dev)
    _need(h1, "h1", torch.int16, n * SPAI_NHID, dev)
    _need(h2, "h2", torch.int16, n * SPAI_NHID, dev)
    _need(dO, "dO", torch.int16, n * SPAI_NOUT, dev)
    _need(weights, "weights", torch.int16, SPAI_NWEIGHT, dev)
    _need(grad, "grad", torch.float64, SPAI_NPARAM, dev)
    _need(ws, "ws", torch.uint8, spai_workspace_bytes(n, 0, 0), dev)
    _check(lib().cbg_mlp_backward(n, _ptr(feat), _ptr(h1), _ptr(h2), _ptr(dO), _ptr(weights),
                                  _ptr(grad), int(bool(accumulate)), _ptr(ws), ws.numel(),
                                  _stream()), "cbg_mlp_backward")
    return grad


def spai_loss_grad(A: DeviceCSR, t_val, grid, feat, weights, params, V, scale, loss, grad,
                   accumulate=False, ws=None):
    """loss[1], grad[NPARAM] (+)= one matrix's loss and parameter gradient."""
    torch = _torch()
    dev = A.val.device
    K = V.shape[1]
    ws = _sws(A.n, A.nnz, K, dev) if ws is None else ws
    _need(t_val, "t_val", torch.float64, A.nnz, dev)
    _need(feat, "feat", torch.int16, A.n * SPAI_NFEAT, dev)
    _need(weights, "weights", torch.int16, SPAI_NWEIGHT, dev)
    _need(params, "params", torch.float32, SPAI_NPARAM, dev)
    _need(V, "V", torch.int16, A.n * K, dev)
    _need(loss, "loss", torch.float64, 1, dev)
    _need(grad, "grad", torch.float64, SPAI_NPARAM, dev)
    _need(ws, "ws", torch.uint8, spai_workspace_bytes(A.n, A.nnz, K), dev)
    csr = A.cstruct()
    _check(lib().cbg_spai_loss_grad(C.byref(csr), _ptr(t_val), _grid3(grid, A.n), _ptr(feat),
                                    _ptr(weights), _ptr(params), K, _ptr(V), float(scale),
                                    _ptr(loss), _ptr(grad), int(bool(accumulate)), _ptr(ws),
                                    ws.numel(), _stream()), "cbg_spai_loss_grad")


def spai_round_weights(params, weights):
    torch = _torch()
    _need(params, "params", torch.float32, SPAI_NPARAM)
    _need(weights, "weights", torch.int16, SPAI_NWEIGHT, params.device)
    _check(lib().cbg_spai_round_weights(_ptr(params), _ptr(weights), _stream()),
           "cbg_spai_round_weights")
    return weights


def adam_step(params, m1, m2, weights, grad, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    torch = _torch()
    _need(params, "params", torch.float32, SPAI_NPARAM)
    for tt, nm in ((m1, "m1"), (m2, "m2")):
        _need(tt, nm, torch.float32, SPAI_NPARAM, params.device)
    _need(weights, "weights", torch.int16, SPAI_NWEIGHT, params.device)
    _need(grad, "grad", torch.float64, SPAI_NPARAM, params.device)
    _check(lib().cbg_adam_step(_ptr(params), _ptr(m1), _ptr(m2), _ptr(weights), _ptr(grad),
                               int(t), float(lr), float(beta1), float(beta2), float(eps),
                               _stream()), "cbg_adam_step")
