"""The sliced-ELL copy of A (SELL-64) and the SpMV on it, through the C ABI.

* Layout: cbg_sell_ptr / cbg_sell_fill produce exactly the arrays the
  layout in include/cbgmres.h defines (built here in numpy from that
  definition), on stencil matrices, on n not a multiple of 64 (ragged last
  slice), on irregular rows (empty rows, one long row, a diagonal-only
  matrix) and on n = 1; cbg_sell_diag gives the sorted distinct offsets
  col - row (0 included) and each entry's index, or refuses a matrix with
  more than 256 of them.
* SpMV: y = A x on the copy (int32 columns, and diagonal indices where the
  matrix allows them) equals the oracle's row-sequential CSR sum bit
  for bit (products and sums rounded separately, in CSR order; padding adds
  0 * x_row), on the same matrices and on the 27-point 160^3 system the
  benchmark solves (n = 4,096,000, the launch configuration of the solve).
* Solve: the default solver path reads the copy; with and without it, the
  fp64-basis solve matches the oracle's iteration count.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


def sell_reference(A):
    """(sell_ptr, sell_col, sell_val) from the layout's definition."""
    n = A.n
    rp = A.row_ptr.astype(np.int64)
    ns = (n + 63) // 64
    ptr = np.zeros(ns + 1, np.int64)
    cols, vals = [], []
    for s in range(ns):
        rows = range(64 * s, 64 * s + 64)
        lens = [rp[r + 1] - rp[r] if r < n else 0 for r in rows]
        w = max(lens)
        ptr[s + 1] = ptr[s] + 64 * w
        c = np.empty((w, 64), np.int32)
        v = np.zeros((w, 64), np.float64)
        for lane, r in enumerate(rows):
            L = lens[lane]
            c[:, lane] = min(r, n - 1)
            if L:
                c[:L, lane] = A.col_idx[rp[r]:rp[r] + L]
                v[:L, lane] = A.val[rp[r]:rp[r] + L]
        cols.append(c.reshape(-1))
        vals.append(v.reshape(-1))
    return ptr, np.concatenate(cols), np.concatenate(vals)


def irregular(n, seed, long_row=None, empty_every=7):
    """Random sparse rows of 0..12 entries (every empty_every-th row empty),
    a nonzero diagonal elsewhere, and optionally one row of 300 entries."""
    from paper_2009_12101_amd.problems import CSR
    rng = np.random.default_rng(seed)
    rp, ci, va = [0], [], []
    for i in range(n):
        if empty_every and i % empty_every == 3:
            cnt = 0
        elif i == long_row:
            cnt = min(300, n)
        else:
            cnt = int(rng.integers(1, 13))
        cols = set(rng.choice(n, size=min(cnt, n), replace=False).tolist()) if cnt else set()
        if cnt:
            cols.add(i)
        cols = sorted(cols)
        ci += cols
        va += [4.0 + rng.random() if c == i else rng.standard_normal() for c in cols]
        rp.append(len(ci))
    return CSR(n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(va, np.float64))


def cases():
    from paper_2009_12101_amd import problems as P
    out = [("poisson2d_20", P.poisson2d(20)),            # n = 400: ragged last slice
           ("convdiff7_10", P.convdiff7(10)),            # n = 1000
           ("lognormal27_12", P.lognormal27(12, 0)),     # n = 1728 = 27 slices
           ("irregular_1000", irregular(1000, 1, long_row=517)),
           ("irregular_65", irregular(65, 2)),
           ("irregular_63", irregular(63, 3, empty_every=0)),
           ("diag_130", P.CSR(130, np.arange(131, dtype=np.int32),
                              np.arange(130, dtype=np.int32), np.linspace(1, 2, 130))),
           ("one", P.CSR(1, np.array([0, 1], np.int32), np.array([0], np.int32),
                         np.array([3.0])))]
    return out


CASES = cases()


@pytest.mark.parametrize("name,A", CASES, ids=[c[0] for c in CASES])
def test_sell_layout(cbg, dev, name, A):
    print(f"sell layout {name} n={A.n} nnz={A.nnz}", flush=True)
    D = cbg.DeviceCSR.from_host(A, dev, sell=True, diag=False)
    ptr, col, val = sell_reference(A)
    assert np.array_equal(D.sell_ptr.cpu().numpy(), ptr)
    assert D.sell_entries == ptr[-1]
    assert np.array_equal(D.sell_col.cpu().numpy(), col)
    assert np.array_equal(D.sell_val.cpu().numpy().view(np.uint64), val.view(np.uint64))
    assert D.sell_dix is None


def diag_reference(A, ptr, col):
    """Per entry the offset col - row (0 for rows >= n), and the sorted
    distinct offsets with 0 included."""
    ns = len(ptr) - 1
    off = np.empty(len(col), np.int64)
    for s in range(ns):
        w = (ptr[s + 1] - ptr[s]) // 64
        rows = 64 * s + np.arange(64)
        blk = col[ptr[s]:ptr[s + 1]].reshape(w, 64).astype(np.int64) - rows
        blk[:, rows >= A.n] = 0
        off[ptr[s]:ptr[s + 1]] = blk.reshape(-1)
    return off, np.unique(np.concatenate([off, [0]]))


@pytest.mark.parametrize("name,A", CASES, ids=[c[0] for c in CASES])
def test_sell_diag_layout(cbg, dev, name, A):
    print(f"sell diag layout {name} n={A.n}", flush=True)
    D = cbg.DeviceCSR.from_host(A, dev, sell=True, diag=True)
    ptr, col, _ = sell_reference(A)
    off, uniq = diag_reference(A, ptr, col)
    if len(uniq) > 256:
        assert D.sell_dix is None and D.sell_col is not None      # refused: int32 columns
        return
    assert D.sell_ndiag == len(uniq)
    assert np.array_equal(D.sell_diag.cpu().numpy()[:len(uniq)], uniq)
    dix = D.sell_dix.cpu().numpy()
    assert np.array_equal(uniq[dix], off)
    assert D.sell_col is None                                     # dropped with the indices


def test_sell_diag_refuses_many_offsets(cbg, dev):
    """300 distinct offsets: cbg_sell_diag reports the count (at least 257)
    and refuses; the copy keeps int32 columns and stays bit-exact."""
    from paper_2009_12101_amd.problems import CSR
    n = 600
    rp, ci, va = [0], [], []
    for i in range(n):
        cols = sorted({i, (i + 1 + (i % 300)) % n})
        ci += cols
        va += [3.0 if c == i else -1.0 for c in cols]
        rp.append(len(ci))
    A = CSR(n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(va))
    D = cbg.DeviceCSR.from_host(A, dev, sell=True, diag=True)
    assert D.sell_dix is None and D.sell_col is not None


@pytest.mark.parametrize("diag", [False, True], ids=["col", "dix"])
@pytest.mark.parametrize("name,A", CASES, ids=[c[0] for c in CASES])
def test_sell_spmv_bit_exact(cbg, orc, dev, name, A, diag):
    print(f"sell spmv {name} n={A.n} diag={diag}", flush=True)
    D = cbg.DeviceCSR.from_host(A, dev, sell=True, diag=diag)
    assert (D.sell_dix is not None) == (diag and name != "irregular_1000")
    for seed in (0, 1):
        x = np.random.default_rng(seed).standard_normal(A.n) * 10.0 ** np.random.default_rng(
            seed + 9).uniform(-3, 3, A.n)
        y, nrm = cbg.spmv(D, torch.from_numpy(x).to(dev), want_norm=True)
        yo = orc.spmv(A, x)
        assert np.array_equal(y.cpu().numpy().view(np.uint64), yo.view(np.uint64))
        assert abs(nrm.item() - np.linalg.norm(yo)) <= 1e-13 * np.linalg.norm(yo)


def test_sell_auto_keeps_csr_when_padding_is_large(cbg, dev):
    """One full row among rows of two entries: the copy would hold 8320
    entries for 382 nonzeros, so "auto" keeps the CSR kernels."""
    from paper_2009_12101_amd.problems import CSR
    n = 128
    rp, ci, va = [0], [], []
    for i in range(n):
        cols = list(range(n)) if i == 5 else sorted({i, (i + 1) % n})
        ci += cols
        va += [2.0 if c == i else -0.5 for c in cols]
        rp.append(len(ci))
    A = CSR(n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(va))
    assert A.nnz == 382
    assert cbg.DeviceCSR.from_host(A, dev).sell_val is None
    D = cbg.DeviceCSR.from_host(A, dev, sell=True)
    assert D.sell_entries == 64 * n + 64 * 2


def test_sell_spmv_fullsize_160(cbg, orc, dev):
    """The 27-point 160^3 system (n = 4,096,000): every entry of y = A x bit
    for bit against the oracle."""
    from paper_2009_12101_amd import problems as P
    A = P.lognormal27(160, 0)
    print(f"sell spmv 160^3 n={A.n} nnz={A.nnz}", flush=True)
    D = cbg.DeviceCSR.from_host(A, dev)
    assert D.sell_dix is not None and D.sell_ndiag == 27
    assert D.sell_entries < 1.01 * A.nnz
    x = P.rhs_uniform(A.n, 5)
    y = cbg.spmv(D, torch.from_numpy(x).to(dev)).cpu().numpy()
    yo = orc.spmv(A, x)
    assert np.array_equal(y.view(np.uint64), yo.view(np.uint64))
    del D
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name", ["convdiff7_20", "lognormal27_12"])
def test_solve_with_and_without_sell(cbg, orc, dev, name):
    from paper_2009_12101_amd import problems as P
    A, b, _ = P.workload(name)
    o = orc.gmres(A, b, restart=30, fmt="fp64", tol=1e-10, maxiter=3000)
    bd = torch.from_numpy(b).to(dev)
    its = []
    for sell, diag in ((True, True), (True, False), (False, False)):
        D = cbg.DeviceCSR.from_host(A, dev, sell=sell, diag=diag)
        r = cbg.solve(D, bd, restart=30, fmt="fp64", tol=1e-10, maxiter=3000)
        assert r.status == 0
        x = r.x.cpu().numpy()
        assert np.linalg.norm(b - orc.spmv(A, x)) <= 1e-10 * np.linalg.norm(b)
        its.append(r.iterations)
    assert all(abs(i - o["iterations"]) <= 1 for i in its), (its, o["iterations"])
