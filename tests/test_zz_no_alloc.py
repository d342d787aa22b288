"""cbg_multidot_noalloc (the multi-dot for callers that cannot allocate)
against cbg_multidot, through the C ABI.

Both run the same kernels; the no-allocation entry keeps its block
partials in the library's per-GPU scratch array instead of a workspace, so
its results must equal cbg_multidot's bit for bit, and both lie within the
FP64 dot-product bound of the oracle's dots.  Two calls in a row, the second
smaller (the array keeps the first call's contents), a call at the largest
j, the j beyond it (refused before any HIP call) and n = 0.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

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


def _case(cbg, orc, dev, fmt, n, j, seed):
    from tests.test_gpu_kernels import _basis
    ld = cbg.basis_ld(n)
    raw, dec, scales = _basis(orc, fmt, n, j, ld, seed=seed)
    w = np.random.default_rng(seed + 1).standard_normal(n)
    Vd = torch.from_numpy(raw.view(np.uint8).reshape(-1)).to(dev)
    sd = torch.from_numpy(scales).to(dev)
    wd = torch.from_numpy(w).to(dev)
    return ld, dec, w, Vd, sd, wd


@pytest.mark.parametrize("fmt", ["fp16", "fp64", "int16", "e4m3"])
def test_noalloc_equals_multidot_twice(cbg, orc, dev, fmt):
    for n, j, seed in [(300001, 100, 1), (5001, 17, 2)]:
        print(f"noalloc {fmt} n={n} j={j}", flush=True)
        ld, dec, w, Vd, sd, wd = _case(cbg, orc, dev, fmt, n, j, seed)
        h0 = torch.full((j,), np.nan, dtype=torch.float64, device=dev)
        got = cbg.multidot_noalloc(fmt, Vd, ld, sd, n, j, wd, h0).cpu().numpy()
        want = cbg.multidot(fmt, Vd, ld, sd, n, j, wd).cpu().numpy()
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
        ho = np.array([orc.dot(dec[k], w) for k in range(j)])
        bound = 4 * n * U * (np.abs(dec) @ np.abs(w)) + 1e-300
        assert np.all(np.abs(got - ho) <= bound)


def test_noalloc_limits(cbg, orc, dev):
    jmax = cbg.NOALLOC_MAX_J
    n = 70001
    ld, dec, w, Vd, sd, wd = _case(cbg, orc, dev, "fp16", n, jmax + 1, 5)
    h = torch.empty(jmax + 1, dtype=torch.float64, device=dev)
    got = cbg.multidot_noalloc("fp16", Vd, ld, sd, n, jmax, wd, h).cpu().numpy()
    want = cbg.multidot("fp16", Vd, ld, sd, n, jmax, wd).cpu().numpy()
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
    with pytest.raises(cbg.CbgError) as e:
        cbg.multidot_noalloc("fp16", Vd, ld, sd, n, jmax + 1, wd, h)
    assert e.value.status == -5
    # n = 0: h = 0, written by a fill kernel
    h = torch.full((4,), 7.0, dtype=torch.float64, device=dev)
    e0 = torch.empty(0, dtype=torch.float64, device=dev)
    cbg.multidot_noalloc("fp16", Vd, 16, sd, 0, 4, e0, h)
    assert np.all(h.cpu().numpy() == 0.0)
