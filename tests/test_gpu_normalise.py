"""Steps 13-14 of Fig. 1 (v_j = w / t, stored through the accessor) in a pass
of their own against the same steps inside the next SpMV's gather.

Both divide the same FP64 w by the same t with IEEE division, store through
the same codec and feed the same SpMV kernel the same operand, so the two
paths give the same bits: equal counts, equal residual histories and
bitwise-equal solutions, for every format and for the identity, Jacobi and
sparse preconditioners, on a 27-point matrix (mean row length above 12, where
the solver picks the pass by itself) and a 7-point one (where it picks the
gather, except with Jacobi).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2009_12101_amd import problems as P

TOL = 1e-10


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def cbg():
    import paper_2009_12101_amd as cbg
    cbg.lib()
    return cbg


SYSTEMS = {"lognormal27_11": lambda: P.lognormal27(11, 4), "convdiff7_13": lambda: P.convdiff7(13)}


def sparse_p(A, seed):
    """float32 values on A's pattern: 1 / a_ii on the diagonal and small
    off-diagonal terms, a nonsingular right preconditioner."""
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    diag = A.col_idx == rows
    pv = (0.02 * rng.standard_normal(A.nnz) / np.abs(A.val).max()).astype(np.float32)
    pv[diag] = (1.0 / A.val[diag]).astype(np.float32)
    return pv


def bits(t):
    return t.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("system", list(SYSTEMS))
@pytest.mark.parametrize("precond", ["none", "jacobi", "sparse"])
@pytest.mark.parametrize("fmt", ["fp64", "fp32", "fp16", "bf16", "int16", "e4m3", "fp16s"])
def test_pass_and_gather_give_the_same_bits(cbg, dev, system, precond, fmt):
    print(f"normalise {system} {precond} {fmt}", flush=True)
    A = SYSTEMS[system]()
    b = torch.from_numpy(P.rhs_uniform(A.n, 5)).to(dev)
    Ad = cbg.DeviceCSR.from_host(A, dev)
    kw = dict(restart=25, fmt=fmt, tol=TOL, maxiter=4000, precond=precond)
    if precond == "sparse":
        kw["p_val"] = torch.from_numpy(sparse_p(A, 3)).to(dev)
    rp = cbg.solve(Ad, b, normalise="pass", **kw)
    rg = cbg.solve(Ad, b, normalise="gather", **kw)
    ra = cbg.solve(Ad, b, **kw)
    assert rp.status == 0
    for r in (rg, ra):
        assert r.status == rp.status and r.iterations == rp.iterations
        assert r.reorths == rp.reorths and r.restarts == rp.restarts
        assert np.array_equal(r.hist.view(np.uint64), rp.hist.view(np.uint64))
        assert np.array_equal(bits(r.x), bits(rp.x))
    # the byte model counts the pass's extra write and read of v; the
    # solver's own choice is the pass for long rows and for Jacobi
    auto_pass = A.nnz > 12 * A.n or precond == "jacobi"
    assert (ra.model_bytes == rp.model_bytes) == auto_pass
    assert (ra.model_bytes == rg.model_bytes) == (not auto_pass)
    assert rp.model_bytes > rg.model_bytes


def test_spmv_vhat_ignores_the_pass_flag(cbg, dev):
    """The stored-vector ablation keeps its gather path: forcing the pass
    changes nothing."""
    A = P.lognormal27(9, 2)
    b = torch.from_numpy(P.rhs_uniform(A.n, 2)).to(dev)
    Ad = cbg.DeviceCSR.from_host(A, dev)
    kw = dict(restart=20, fmt="fp16", tol=TOL, maxiter=3000, variant="spmv_vhat")
    r0 = cbg.solve(Ad, b, normalise="gather", **kw)
    r1 = cbg.solve(Ad, b, normalise="pass", **kw)
    assert r0.iterations == r1.iterations and r0.model_bytes == r1.model_bytes
    assert np.array_equal(bits(r0.x), bits(r1.x))
