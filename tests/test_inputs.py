"""Pins of the seeded input generators (paper_2009_12101_amd/problems.py).

The generators feed both the oracle and the GPU path, so they are checked
against things other than themselves: SplitMix64's published output sequence,
the distributions the draws must follow, the matrices' construction as
Kronecker sums of 1D operators, and the properties each system is stated to
have (symmetry, a Gershgorin bound on the spectrum, zero interior row sums).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.stats as st

from paper_2009_12101_amd import problems as P


def _dense(A):
    return sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n, A.n)).toarray()


def test_splitmix64_output_function_matches_the_published_sequence():
    # SplitMix64 (Steele, Lea and Flood 2014; Vigna's reference code) from
    # state 0: the k-th output is the mix of k * 0x9E3779B97F4A7C15
    with np.errstate(over="ignore"):
        states = np.arange(1, 4, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)
    out = [int(v) for v in P._mix(states)]
    assert out == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_counter_based_draws_are_addressable_and_distinct():
    a = P.splitmix64(3, 1, 1000)
    assert np.array_equal(a[500:], P.splitmix64(3, 1, 500, start=500))
    assert len(np.unique(a)) == 1000
    assert not np.array_equal(a, P.splitmix64(3, 2, 1000))   # another stream
    assert not np.array_equal(a, P.splitmix64(4, 1, 1000))   # another seed


def test_uniform_and_normal_draws_follow_their_distributions():
    u = P.uniform01(0, 5, 200_000)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert st.kstest(u, "uniform").pvalue > 1e-3
    z = P.normal(0, 5, 200_000)
    assert st.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 5e-3 and abs(z.var() - 1.0) < 1e-2
    b = P.rhs_uniform(100_000, 7)
    assert b.min() >= -1.0 and b.max() < 1.0
    assert st.kstest(b, "uniform", args=(-1.0, 2.0)).pvalue > 1e-3


def _lap1d(N):
    return sp.diags([-np.ones(N - 1), 2.0 * np.ones(N), -np.ones(N - 1)], [-1, 0, 1])


def test_poisson2d_is_the_kronecker_sum_of_1d_laplacians():
    N = 7
    I = sp.identity(N)
    K = (sp.kron(I, _lap1d(N)) + sp.kron(_lap1d(N), I)).toarray()
    assert np.array_equal(_dense(P.poisson2d(N)), K)


@pytest.mark.parametrize("cell_peclet", [False, True])
def test_convdiff7_is_the_kronecker_sum_of_1d_upwind_operators(cell_peclet):
    N, beta = 5, 10.0
    bh = beta if cell_peclet else beta / (N + 1)
    # 1D: -u'' + beta u' scaled by h^2, first-order upwind (beta > 0): the
    # neighbour at x - h carries -1 - beta h, the one at x + h carries -1
    T = sp.diags([-(1.0 + bh) * np.ones(N - 1), (2.0 + bh) * np.ones(N), -np.ones(N - 1)],
                 [-1, 0, 1])
    I = sp.identity(N)
    K = (sp.kron(sp.kron(I, I), T) + sp.kron(sp.kron(I, T), I) + sp.kron(sp.kron(T, I), I))
    A = _dense(P.convdiff7(N, beta, cell_peclet=cell_peclet))
    assert np.allclose(A, K.toarray(), rtol=1e-15, atol=0.0)
    # interior rows sum to zero (a constant is in the operator's kernel there)
    i = 2 + 2 * N + 2 * N * N
    assert abs(A[i].sum()) < 1e-14
    assert not np.array_equal(A, A.T)


def test_lognormal27_is_symmetric_and_its_spectrum_sits_above_the_shift():
    N, shift = 4, 1e-2
    A = P.lognormal27(N, 3, shift=shift)
    D = _dense(A)
    assert np.array_equal(D, D.T)
    assert np.all(np.diff(A.row_ptr) <= 27) and A.nnz == (3 * N - 2) ** 3
    off = np.abs(D).sum(axis=1) - np.abs(np.diag(D))
    assert np.all(np.diag(D) - off >= shift * (1 - 1e-12))         # Gershgorin
    lam = np.linalg.eigvalsh(D)
    assert lam.min() >= shift * (1 - 1e-9)
    # an interior row: the 26 weights sqrt(kappa_i kappa_j) plus the shift
    kap = P.lognormal_kappa(N, 3)
    i = 1 + N + N * N
    nbr = [i + dx + dy * N + dz * N * N for dz in (-1, 0, 1) for dy in (-1, 0, 1)
           for dx in (-1, 0, 1) if (dx, dy, dz) != (0, 0, 0)]
    w = np.sqrt(kap[i] * kap[nbr])
    assert np.allclose(-D[i, nbr], w, rtol=1e-15)
    assert D[i, i] == pytest.approx(w.sum() + shift, rel=1e-14)


def test_right_hand_sides():
    assert np.array_equal(P.rhs_sin(4), np.sin([1.0, 2.0, 3.0, 4.0]))
    A = P.poisson2d(5)
    assert np.allclose(P.rhs_row_sums(A), _dense(A).sum(axis=1), rtol=0, atol=1e-15)
