"""The C-ABI library loads, exports every symbol its header declares, and
rejects invalid arguments on the host before any HIP call (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cbgmres.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(cbg\w*|cbgmres\w*)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    from paper_2009_12101_amd import _binding
    return _binding.lib()


def test_header_functions_are_exported(L):
    names = declared_functions()
    assert "cbgmres_solve" in names and len(names) >= 10
    for nm in names:
        assert hasattr(L, nm), nm
    from paper_2009_12101_amd import _binding
    assert sorted(_binding.EXPORTS) == names


def test_strerror_and_sizes(L):
    from paper_2009_12101_amd import _binding as B
    for code in (0, 1, -1, -2, -3, -4, -5, 42):
        assert isinstance(B.strerror(code), str) and B.strerror(code)
    assert B.basis_ld(1) == 256 and B.basis_ld(256) == 256 and B.basis_ld(257) == 512
    assert B.workspace_bytes(1000, 0, "fp16") == 0           # restart < 1
    assert B.workspace_bytes(1000, 513, "fp16") == 0         # restart > max
    small = B.workspace_bytes(1000, 10, "fp16")
    big = B.workspace_bytes(1000, 10, "fp64")
    assert 0 < small < big
    # the basis dominates: (m+1) * ld * bytes
    d = B.workspace_bytes(10 ** 6, 100, "fp64") - B.workspace_bytes(10 ** 6, 100, "fp16")
    assert d == 101 * B.basis_ld(10 ** 6) * 6
    assert B.kernel_workspace_bytes(100, 10) > 0
    assert B.kernel_workspace_bytes(100, 10 ** 6) == 0
    # no HIP call has failed on this thread: code 0, no line
    assert B.last_hip_error() == (0, 0, "hipSuccess")


def test_solve_rejects_bad_arguments_on_host(L):
    from paper_2009_12101_amd import _binding as B
    res = B.CbgResult()
    csr = B.CbgCsr(4, 0, 4, 16, 32, 48)          # fake but 16-aligned device pointers
    good = dict(restart=10, format=2, tol=1e-10, maxiter=100, eta=0.0, precond=0, fallback=0,
                p_val=None, flags=0, reserved=0)

    def call(A=csr, b=64, x=128, ws=None, wsb=0, **over):
        o = dict(good)
        o.update(over)
        opts = B.CbgOpts(**o)
        return L.cbgmres_solve(C.byref(A) if A is not None else None, C.c_void_p(b),
                               C.c_void_p(x), C.byref(opts), C.c_void_p(ws), wsb, None,
                               C.byref(res), None, 0)

    assert call(restart=0) == B.E_ARG and res.status == B.E_ARG
    assert call(restart=513) == B.E_ARG
    assert call(format=9) == B.E_ARG
    assert call(tol=-1.0) == B.E_ARG
    assert call(tol=float("nan")) == B.E_ARG
    assert call(maxiter=-5) == B.E_ARG
    assert call(precond=7) == B.E_ARG
    assert call(precond=2) == B.E_ARG              # sparse P without values
    assert call(b=0) == B.E_ARG                   # null b
    assert call(x=8) == B.E_ARG                   # misaligned x
    assert call(A=None) == B.E_ARG
    assert call(ws=None) == B.E_WORKSPACE          # missing workspace
    assert call(ws=4096 + 8, wsb=1 << 40) == B.E_WORKSPACE   # misaligned workspace
    assert call(ws=4096, wsb=10) == B.E_WORKSPACE            # too small
    # formats 0..7 (7: scaled float16), flag bits 1..2048, block-Jacobi sizes
    assert call(format=8) == B.E_ARG
    assert call(format=7) == B.E_WORKSPACE                    # valid: reaches the workspace check
    assert call(flags=4096) == B.E_ARG
    assert call(flags=B.FLAG_PROFILE_SPMV | B.FLAG_PROFILE_SAMPLED) == B.E_WORKSPACE
    assert call(flags=B.FLAG_TWO_PASS | B.FLAG_EXPLICIT_REDOT) == B.E_ARG
    assert call(flags=B.FLAG_TWO_PASS | B.FLAG_MGS) == B.E_ARG
    assert call(flags=B.FLAG_TWO_PASS) == B.E_WORKSPACE
    assert call(flags=B.FLAG_EXPLICIT_REDOT | B.FLAG_MGS) == B.E_WORKSPACE
    assert call(flags=B.FLAG_NORMALISE_PASS | B.FLAG_NORMALISE_GATHER) == B.E_ARG
    assert call(flags=B.FLAG_NORMALISE_PASS) == B.E_WORKSPACE
    assert call(flags=B.FLAG_NORMALISE_GATHER) == B.E_WORKSPACE
    assert call(flags=B.FLAG_SPMV_VHAT | B.FLAG_ALWAYS_REORTH | B.FLAG_MGS) == B.E_WORKSPACE
    assert call(precond=3, pc_block=9) == B.E_ARG
    assert call(precond=3, pc_prec=20) == B.E_ARG
    assert call(precond=3, pc_block=8, pc_prec=32) == B.E_WORKSPACE
    # MGS with event timing: refused before any HIP call (host arithmetic only
    # runs between the workspace check and this test)
    assert call(flags=B.FLAG_MGS | B.FLAG_PROFILE, ws=1 << 20, wsb=1 << 40) == B.E_UNSUPPORTED
    empty = B.CbgCsr(0, 0, 0, None, None, None)
    assert call(A=empty, b=0, x=0) == B.OK                   # n = 0: nothing to do
    assert L.cbgmres_solve(C.byref(csr), None, None, None, None, 0, None, C.byref(res),
                           None, 0) == B.E_ARG


def test_kernel_calls_reject_bad_arguments_on_host(L):
    from paper_2009_12101_amd import _binding as B
    vp = C.c_void_p
    assert L.cbg_encode(9, vp(16), 10, vp(32), vp(48), vp(256), 1 << 20, None) == B.E_ARG
    assert L.cbg_encode(2, vp(16), -1, vp(32), vp(48), vp(256), 1 << 20, None) == B.E_ARG
    assert L.cbg_encode(2, vp(16), 10, vp(32), vp(48), None, 0, None) == B.E_WORKSPACE
    assert L.cbg_decode(2, vp(16), None, 10, vp(32), None) == B.E_ARG
    # ld must be >= n and a multiple of 16
    assert L.cbg_multidot(2, vp(16), 10, vp(32), 20, 3, vp(48), vp(64), vp(256), 1 << 20,
                          None) == B.E_ARG
    assert L.cbg_multidot(2, vp(16), 24, vp(32), 20, 3, vp(48), vp(64), vp(256), 1 << 20,
                          None) == B.E_ARG
    assert L.cbg_update(2, vp(16), 32, vp(32), 20, 600, vp(48), vp(64), vp(80), vp(256),
                        1 << 20, None) == B.E_ARG
    bad = B.CbgCsr(-1, 0, 0, None, None, None)
    assert L.cbg_spmv(C.byref(bad), vp(16), vp(32), None, None, 0, None) == B.E_ARG


def test_sell_arguments_rejected_on_host(L):
    """The sliced-ELL fields of cbg_csr are all set or all NULL, with an
    entry count that is a multiple of 64 and at least nnz; the set-up calls
    check their pointers.  All before any HIP call."""
    from paper_2009_12101_amd import _binding as B
    vp = C.c_void_p
    ent = C.c_int64(-1)
    A = B.CbgCsr(100, 0, 500, 16, 32, 48)
    assert L.cbg_sell_ptr(C.byref(A), None, C.byref(ent), None) == B.E_ARG
    assert L.cbg_sell_ptr(C.byref(A), vp(64), None, None) == B.E_ARG
    assert L.cbg_sell_ptr(C.byref(A), vp(68), C.byref(ent), None) == B.E_ARG   # misaligned
    assert L.cbg_sell_ptr(None, vp(64), C.byref(ent), None) == B.E_ARG
    assert L.cbg_sell_fill(C.byref(A), None, vp(64), vp(128), None) == B.E_ARG
    assert L.cbg_sell_fill(C.byref(A), vp(64), None, vp(128), None) == B.E_ARG
    assert L.cbg_sell_fill(C.byref(A), vp(64), vp(64), None, None) == B.E_ARG
    # partial or implausible sliced-ELL fields: refused by the SpMV and the solve
    res = B.CbgResult()
    opts = B.CbgOpts(restart=10, format=2, tol=1e-10, maxiter=100)
    for fields in ((64, None, None, 512), (64, 80, 96, 100), (64, 80, 96, 448)):
        Ab = B.CbgCsr(100, 0, 500, 16, 32, 48, *fields)
        assert L.cbg_spmv(C.byref(Ab), vp(16), vp(32), None, None, 0, None) == B.E_ARG
        assert L.cbgmres_solve(C.byref(Ab), vp(64), vp(128), C.byref(opts), None, 0, None,
                               C.byref(res), None, 0) == B.E_ARG
    # complete fields pass the check (and reach the workspace test)
    Ag = B.CbgCsr(100, 0, 500, 16, 32, 48, 64, 80, 96, 512)
    assert L.cbgmres_solve(C.byref(Ag), vp(64), vp(128), C.byref(opts), None, 0, None,
                           C.byref(res), None, 0) == B.E_WORKSPACE
    # diagonal-index columns: indices and table together, 1 <= ndiag <= 256;
    # then the int32 columns may be absent
    for dix in ((112, None, 27), (None, 128, 27), (112, 128, 0), (112, 128, 257)):
        Ad = B.CbgCsr(100, 0, 500, 16, 32, 48, 64, 80, 96, 512, *dix)
        assert L.cbgmres_solve(C.byref(Ad), vp(64), vp(128), C.byref(opts), None, 0, None,
                               C.byref(res), None, 0) == B.E_ARG
    Ad = B.CbgCsr(100, 0, 500, 16, 32, 48, 64, None, 96, 512, 112, 128, 27)
    assert L.cbgmres_solve(C.byref(Ad), vp(64), vp(128), C.byref(opts), None, 0, None,
                           C.byref(res), None, 0) == B.E_WORKSPACE
    Ad = B.CbgCsr(100, 0, 500, 16, 32, 48, 64, None, 96, 512)     # no columns at all
    assert L.cbg_spmv(C.byref(Ad), vp(16), vp(32), None, None, 0, None) == B.E_ARG
    # cbg_sell_diag: pointers, then the workspace
    nd = C.c_int32(-1)
    assert L.cbg_sell_diag(C.byref(Ag), None, vp(64), C.byref(nd), vp(256), 1 << 20,
                           None) == B.E_ARG
    assert L.cbg_sell_diag(C.byref(Ag), vp(64), None, C.byref(nd), vp(256), 1 << 20,
                           None) == B.E_ARG
    assert L.cbg_sell_diag(C.byref(Ag), vp(64), vp(64), None, vp(256), 1 << 20, None) == B.E_ARG
    assert L.cbg_sell_diag(C.byref(Ag), vp(64), vp(64), C.byref(nd), None, 0, None) == \
        B.E_WORKSPACE


def test_variant_names_map_to_flags():
    """Variant names mean what the oracle's names mean; an empty variant is
    the library default (the Gram-form re-dot with steps 5-10 in one
    update), so "gram" alone asks for the two-pass form."""
    from paper_2009_12101_amd import _binding as B
    assert B.variant_flags(()) == 0
    assert B.variant_flags(("gram", "onepass")) == 0
    assert B.variant_flags("gram") == B.FLAG_TWO_PASS
    assert B.variant_flags("explicit_redot") == B.FLAG_EXPLICIT_REDOT
    assert B.variant_flags(("mgs", "always_reorth")) == B.FLAG_MGS | B.FLAG_ALWAYS_REORTH
    assert B.variant_flags(("gram", "spmv_vhat")) == B.FLAG_TWO_PASS | B.FLAG_SPMV_VHAT
    for bad in ("onepass", "cgs3", ("gram", "nope")):
        with pytest.raises(KeyError):
            B.variant_flags(bad)


def test_binding_checks_tensors_before_the_call():
    """The C ABI takes bare pointers, so the binding checks dtype, length,
    contiguity and device of every tensor it passes; a mismatch is a
    ValueError raised before the library is called."""
    import numpy as np
    torch = pytest.importorskip("torch")
    from paper_2009_12101_amd import _binding as B
    from paper_2009_12101_amd import problems as P
    f64 = torch.zeros(8, dtype=torch.float64)
    with pytest.raises(ValueError, match="dtype"):
        B._need(f64.float(), "b", torch.float64, 8)
    with pytest.raises(ValueError, match="at least 9"):
        B._need(f64, "b", torch.float64, 9)
    with pytest.raises(ValueError, match="expected 7"):
        B._need(f64, "b", torch.float64, 7, exact=True)
    with pytest.raises(ValueError, match="contiguous"):
        B._need(torch.zeros(16, dtype=torch.float64)[::2], "b", torch.float64, 8)
    with pytest.raises(ValueError, match="GPU"):
        B._need(f64, "b", torch.float64, 8)
    with pytest.raises(ValueError, match="torch tensor"):
        B._need(np.zeros(8), "b", torch.float64, 8)
    # a CSR whose arrays do not match n and nnz
    A = P.poisson2d(4)
    D = B.DeviceCSR.from_host(A, "cpu")
    bad = B.DeviceCSR(D.n, D.nnz, D.row_ptr, D.col_idx, D.val.float())
    with pytest.raises(ValueError, match="A.val: dtype"):
        bad.check()
    short = B.DeviceCSR(D.n, D.nnz, D.row_ptr[:-1].clone(), D.col_idx, D.val)
    with pytest.raises(ValueError, match="A.row_ptr"):
        short.check()
    # every wrapper checks before it calls: CPU tensors never reach the ABI
    b = torch.from_numpy(P.rhs_uniform(A.n, 0))
    with pytest.raises(ValueError):
        B.solve(D, b, restart=5)
    with pytest.raises(ValueError):
        B.spmv(D, b)
    with pytest.raises(ValueError):
        B.multidot("fp16", torch.zeros(256, dtype=torch.int16), 256, torch.ones(1), A.n, 1, b)
    with pytest.raises(ValueError, match="grid"):
        B._grid3((4, 4, 2), A.n)
