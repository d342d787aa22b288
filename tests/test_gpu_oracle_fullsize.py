"""Full-size solves against the FP64 CPU oracle's own full solve: the error
of every compressed-basis solution against the oracle's fp64 solution.

Both solutions meet ||b - A x|| <= tol ||b||, so they can differ by at most
2 tol ||b|| / sigma_min(A), with a lower bound on sigma_min that needs no
eigen solve:
* 27-point lognormal system: a weighted graph Laplacian plus non-negative
  ghost terms plus 1e-2 I, symmetric, so sigma_min = lambda_min >= 1e-2;
* convection-diffusion: for unit x, ||A x|| >= x^T A x = x^T S x with S the
  symmetric part, so sigma_min(A) >= lambda_min(S); S is separable, each
  axis contributing c tridiag(-1, 2, -1) with c = 1 + beta h / 2, so
  lambda_min(S) = 6 c (1 - cos(pi h)) (1.85e-3 at 128^3).

The oracle solves one restart cycle per call and prints a line per cycle
(its full solves take about a minute of host time on a 16-core host).
"""
import math

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


def lam_min_convdiff(N):
    """lambda_min of the symmetric part of the 7-point upwind
    convection-diffusion matrix (entries scaled by h^2, beta = 10 per axis):
    diagonal 6 + 3 beta h = 6 c, axis neighbours -(1 + beta h / 2) = -c,
    so 3 c (2 - 2 cos(pi h))."""
    h = 1.0 / (N + 1)
    c = 1.0 + 10.0 * h / 2.0
    return 6.0 * c * (1.0 - math.cos(math.pi * h))


def oracle_solve(orc, A, b):
    """The oracle's fp64 solve one restart cycle per call, each starting
    from the previous iterate: restarted GMRES carries only x from a cycle
    to the next, so this is the same iteration as one call, with a line
    printed per cycle."""
    x = np.zeros(A.n)
    it = 0
    while True:
        o = orc.gmres(A, b, x0=x, restart=100, fmt="fp64", tol=TOL, maxiter=100)
        it += o["iterations"]
        x = o["x"]
        print(f"{A.name} oracle fp64: {it} steps, true residual {o['true_rel_res']:.3e}",
              flush=True)
        if o["status"] == 0:
            return dict(x=x, iterations=it)
        assert o["status"] == 1 and it < 20000


def run(cbg, orc, dev, A, b, fmts, lam):
    xo = oracle_solve(orc, A, b)
    nb = np.linalg.norm(b)
    bound = 2.0 * TOL * nb / lam
    Ad = cbg.DeviceCSR.from_host(A, dev)
    bd = torch.from_numpy(b).to(dev)
    out = {}
    for fmt in fmts:
        r = cbg.solve(Ad, bd, restart=100, fmt=fmt, tol=TOL, maxiter=20000)
        x = r.x.cpu().numpy()
        res = np.linalg.norm(b - orc.spmv(A, x)) / nb
        err = np.linalg.norm(x - xo["x"])
        print(f"{A.name} {fmt}: gpu it={r.iterations} res={res:.3e} | oracle fp64 "
              f"it={xo['iterations']} | ||x - x_oracle|| / ||x_oracle|| = "
              f"{err / np.linalg.norm(xo['x']):.3e} (bound {bound / np.linalg.norm(xo['x']):.3e})",
              flush=True)
        assert r.status == 0 and res <= TOL
        assert err <= bound
        out[fmt] = err
    return out


def test_lognormal27_128_against_fp64_oracle(cbg, orc, dev):
    A = P.lognormal27(128, 0)
    b = P.rhs_uniform(A.n, 0)
    run(cbg, orc, dev, A, b, ["fp64", "fp16", "bf16", "e4m3"], lam=1e-2)


def test_convdiff7_128_against_fp64_oracle(cbg, orc, dev):
    A = P.convdiff7(128)
    b = P.rhs_uniform(A.n, 0)
    run(cbg, orc, dev, A, b, ["fp64", "fp16", "int16"], lam=lam_min_convdiff(128))
