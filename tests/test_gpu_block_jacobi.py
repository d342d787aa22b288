"""GPU block-Jacobi preconditioner against the CPU oracle, through the C ABI.

The set-up is exact arithmetic in a fixed order on both sides (Gauss-Jordan
with partial pivoting, no fused operations, the same norm and rule), so the
precision tags and the stored codes are compared bit for bit, ragged last
blocks and row swaps included.  The apply sums a block row with FMAs on the
GPU and separately rounded products in the oracle: within the FP64 bound.
Solves follow the fp64-basis parity rule (counts within one step,
iteration-matched x within 1e-8) and, with an fp16 basis, reach the
tolerance with the first steps equal to rounding.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2009_12101_amd import problems as P
from tests._helpers import FIG1
from tests._helpers import csr_from_dense

U = 2.0 ** -53


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


def crafted():
    rng = np.random.default_rng(3)
    blocks = [np.array([[0.0, 2.0, 1.0], [3.0, 1.0, 0.0], [1.0, 0.0, 4.0]]),   # row swap
              np.diag([1.0, 1.0, 1e-3]), np.diag([1.0, 1.0, 1e-10]),
              rng.standard_normal((3, 3)) + 5 * np.eye(3), np.eye(3) * 1e-5,
              np.array([[2.0]])]                                             # ragged tail
    n = sum(b.shape[0] for b in blocks)
    M = np.zeros((n, n))
    o = 0
    for b in blocks:
        k = b.shape[0]
        M[o:o + k, o:o + k] = b
        o += k
    M += np.diag(np.ones(n - 1), 1) * 0.01                # couplings across blocks
    return csr_from_dense(M)


SYSTEMS = {
    "convdiff7_10": lambda: P.convdiff7(10),
    "lognormal27_9": lambda: P.lognormal27(9, 4),
    "poisson2d_24": lambda: P.poisson2d(24),
    "crafted": crafted,
}


def decoded(blocks, bs):
    tags, x64, x32, x16 = (t.cpu().numpy() for t in blocks)
    nblk = len(tags)
    v64 = x64[:nblk * bs * bs].reshape(nblk, bs, bs)
    v32 = x32[:nblk * bs * bs].astype(np.float64).reshape(nblk, bs, bs)
    v16 = x16[:nblk * bs * bs].view(np.float16).astype(np.float64).reshape(nblk, bs, bs)
    out = np.where(tags[:, None, None] == 16, v16, np.where(tags[:, None, None] == 32, v32, v64))
    return tags, out


@pytest.mark.parametrize("name", list(SYSTEMS))
@pytest.mark.parametrize("bs,prec", [(1, 16), (3, 16), (4, 16), (4, 32), (4, 64), (8, 16)])
def test_setup_bit_exact(cbg, orc, dev, name, bs, prec):
    A = SYSTEMS[name]()
    Ad = cbg.DeviceCSR.from_host(A, dev)
    try:
        ref_vals, ref_tags = orc.block_jacobi(A, bs, prec)
    except ValueError:                  # a singular block (crafted, bs = 1): both refuse
        with pytest.raises(cbg.CbgError):
            cbg.block_jacobi_setup(Ad, bs, prec)
        return
    blocks = cbg.block_jacobi_setup(Ad, bs, prec)
    torch.cuda.synchronize()
    tags, vals = decoded(blocks, bs)
    assert np.array_equal(tags, ref_tags)
    assert np.array_equal(vals, ref_vals)


def test_singular_block_is_an_argument_error(cbg, dev):
    M = np.eye(6)
    M[2:4, 2:4] = 1.0
    Ad = cbg.DeviceCSR.from_host(csr_from_dense(M), dev)
    with pytest.raises(cbg.CbgError) as e:
        cbg.block_jacobi_setup(Ad, 2, 16)
    assert e.value.status == -1
    with pytest.raises(cbg.CbgError):
        cbg.solve(Ad, torch.ones(6, dtype=torch.float64, device=dev), restart=4,
                  precond="block_jacobi", pc_block=2)


@pytest.mark.parametrize("bs", [1, 4, 7])
def test_apply_within_fp64_bound(cbg, orc, dev, bs):
    A = P.lognormal27(10, 2)
    Ad = cbg.DeviceCSR.from_host(A, dev)
    blocks = cbg.block_jacobi_setup(Ad, bs, 16)
    v = np.random.default_rng(bs).standard_normal(A.n)
    z = cbg.block_jacobi_apply(A.n, bs, blocks, torch.from_numpy(v).to(dev)).cpu().numpy()
    vals, _ = orc.block_jacobi(A, bs, 16)
    zr = np.zeros(A.n)
    bound = np.zeros(A.n)
    for b in range(vals.shape[0]):
        i0 = b * bs
        sz = min(bs, A.n - i0)
        X = vals[b, :sz, :sz]
        zr[i0:i0 + sz] = X @ v[i0:i0 + sz]
        bound[i0:i0 + sz] = 2 * bs * U * (np.abs(X) @ np.abs(v[i0:i0 + sz]))
    assert np.all(np.abs(z - zr) <= bound + 1e-300)


@pytest.mark.parametrize("name", ["convdiff7_10", "lognormal27_9"])
@pytest.mark.parametrize("bs", [2, 4])
def test_fp64_solve_parity(cbg, orc, dev, name, bs):
    A = SYSTEMS[name]()
    b = P.rhs_uniform(A.n, 5)
    ref = orc.gmres(A, b, restart=30, fmt="fp64", tol=1e-10, maxiter=3000, variant=FIG1,
                    precond="block_jacobi", pc_block=bs)
    Ad = cbg.DeviceCSR.from_host(A, dev)
    bd = torch.from_numpy(b).to(dev)
    r = cbg.solve(Ad, bd, restart=30, fmt="fp64", tol=1e-10, maxiter=3000,
                  precond="block_jacobi", pc_block=bs)
    assert r.status == 0 and ref["status"] == 0
    assert abs(r.iterations - ref["iterations"]) <= 1
    assert np.linalg.norm(b - orc.spmv(A, r.x.cpu().numpy())) <= 1e-10 * np.linalg.norm(b)
    rm = cbg.solve(Ad, bd, restart=30, fmt="fp64", tol=1e-10, maxiter=ref["iterations"],
                   precond="block_jacobi", pc_block=bs)
    assert np.linalg.norm(rm.x.cpu().numpy() - ref["x"]) <= 1e-8 * np.linalg.norm(ref["x"])
    k = min(30, ref["iterations"])          # the first cycle
    assert np.allclose(r.hist[:k], ref["hist"][:k], rtol=1e-9, atol=0)


def test_fp16_solve_reaches_tolerance(cbg, orc, dev):
    A = P.convdiff7(16)
    b = P.rhs_uniform(A.n, 6)
    ref = orc.gmres(A, b, restart=30, fmt="fp16", tol=1e-10, maxiter=3000, variant=FIG1,
                    precond="block_jacobi", pc_block=4)
    Ad = cbg.DeviceCSR.from_host(A, dev)
    r = cbg.solve(Ad, torch.from_numpy(b).to(dev), restart=30, fmt="fp16", tol=1e-10,
                  maxiter=3000, precond="block_jacobi", pc_block=4)
    assert r.status == 0
    assert np.linalg.norm(b - orc.spmv(A, r.x.cpu().numpy())) <= 1e-10 * np.linalg.norm(b)
    assert np.allclose(r.hist[:3], ref["hist"][:3], rtol=1e-12, atol=0)
    assert abs(r.iterations - ref["iterations"]) <= 0.15 * ref["iterations"] + 3
