"""Pins of the oracle's block-Jacobi preconditioner (an extension; the
definition is this project's own).

The stored inverses are checked against numpy's LU-based inverse, their
precision choice against the stated rule on blocks of known condition, the
stored fp16/fp32 values against numpy's single-rounding casts of the FP64
inverse; with one-row blocks at fp64 storage the solve is the Jacobi solve
bit for bit, and a block-diagonal matrix is solved in one step.
"""
import numpy as np
import pytest

from paper_2009_12101_amd import problems as P
from tests._helpers import csr_from_dense


def blockdiag(blocks):
    n = sum(b.shape[0] for b in blocks)
    M = np.zeros((n, n))
    o = 0
    for b in blocks:
        k = b.shape[0]
        M[o:o + k, o:o + k] = b
        o += k
    return M


def test_one_row_blocks_at_fp64_are_jacobi(orc):
    A = P.convdiff7(9)
    b = P.rhs_uniform(A.n, 4)
    r1 = orc.gmres(A, b, restart=20, fmt="fp64", tol=1e-10, maxiter=2000, precond="jacobi")
    r2 = orc.gmres(A, b, restart=20, fmt="fp64", tol=1e-10, maxiter=2000,
                   precond="block_jacobi", pc_block=1, pc_prec=64)
    assert r1["iterations"] == r2["iterations"]
    assert np.array_equal(r1["x"], r2["x"])


@pytest.mark.parametrize("bs", [2, 4, 5])
def test_inverse_matches_numpy_and_block_diagonal_solves_in_one_step(orc, bs):
    rng = np.random.default_rng(bs)
    sizes = [bs] * 6 + [3 if bs > 3 else 1]          # ragged last block
    blocks = [rng.standard_normal((k, k)) + 3 * k * np.eye(k) for k in sizes]
    A = csr_from_dense(blockdiag(blocks))
    vals, prec = orc.block_jacobi(A, bs=bs, prec_min=64)
    assert np.all(prec == 64)
    for i, B in enumerate(blocks):
        k = B.shape[0]
        inv = np.linalg.inv(B)
        kappa = np.linalg.norm(B, 1) * np.linalg.norm(inv, 1)
        assert np.allclose(vals[i, :k, :k], inv, rtol=0, atol=8 * kappa * 2.0 ** -52 *
                           np.abs(inv).max())
        assert np.all(vals[i, k:, :] == 0) and np.all(vals[i, :, k:] == 0)
    b = rng.standard_normal(A.n)
    r = orc.gmres(A, b, restart=10, fmt="fp64", tol=1e-12, maxiter=50,
                  precond="block_jacobi", pc_block=bs, pc_prec=64)
    assert r["iterations"] == 1 and r["status"] == 0
    assert np.linalg.norm(r["x"] - np.linalg.solve(blockdiag(blocks), b)) <= \
        1e-12 * np.linalg.norm(r["x"])


def test_precision_rule_on_blocks_of_known_condition(orc):
    # kappa_1 of diag(1, ..., 1, 1/c) is c exactly
    well = np.eye(4) * 2.0                                      # kappa 1 -> fp16
    mid = np.diag([1.0, 1.0, 1.0, 1e-3])                         # kappa 1e3 -> fp32
    bad = np.diag([1.0, 1.0, 1.0, 1e-10])                        # kappa 1e10 -> fp64
    big = np.eye(4) * 1e-5                                      # inverse 1e5 > 65504 -> fp32
    tiny = np.eye(4) * 1e5                                      # inverse 1e-5 < 2^-14 -> fp32
    edge_lo = np.diag([1.0, 1.0, 1.0, 1.0 / 20.48])             # kappa 20.48: 0.01 exactly -> fp16
    edge_hi = np.diag([1.0, 1.0, 1.0, 1.0 / 20.5])              # kappa 20.5 > 20.48 -> fp32
    blocks = [well, mid, bad, big, tiny, edge_lo, edge_hi]
    A = csr_from_dense(blockdiag(blocks))
    _, prec = orc.block_jacobi(A, bs=4, prec_min=16)
    assert list(prec) == [16, 32, 64, 32, 32, 16, 32]
    _, prec = orc.block_jacobi(A, bs=4, prec_min=32)
    assert list(prec) == [32, 32, 64, 32, 32, 32, 32]
    _, prec = orc.block_jacobi(A, bs=4, prec_min=64)
    assert np.all(prec == 64)


def test_precision_rule_takes_the_one_norm_condition_number(orc):
    # U = I + 2 (e_1 e_2^T + e_1 e_3^T + e_1 e_4^T) and its inverse I - 2(...)
    # have column sums at most 3 and row sums up to 7: kappa_1 = 9 (fp16) while
    # kappa_inf = 49 (fp32); U^T swaps the two
    U = np.eye(4)
    U[0, 1:] = 2.0
    A = csr_from_dense(blockdiag([U, U.T.copy()]))
    _, prec = orc.block_jacobi(A, bs=4, prec_min=16)
    assert list(prec) == [16, 32]


def test_stored_values_are_single_roundings(orc):
    A = P.lognormal27(6, 2)
    v64, p64 = orc.block_jacobi(A, bs=4, prec_min=64)
    v, p = orc.block_jacobi(A, bs=4, prec_min=16)
    assert set(np.unique(p)) <= {16, 32, 64}
    for i in range(len(p)):
        if p[i] == 16:
            expect = v64[i].astype(np.float16).astype(np.float64)
        elif p[i] == 32:
            expect = v64[i].astype(np.float32).astype(np.float64)
        else:
            expect = v64[i]
        assert np.array_equal(v[i], expect)


def test_pivoting_and_singular_blocks(orc):
    needs_swap = np.array([[0.0, 2.0], [3.0, 1.0]])           # zero leading pivot
    A = csr_from_dense(blockdiag([needs_swap, np.eye(2)]))
    vals, prec = orc.block_jacobi(A, bs=2, prec_min=64)
    assert np.allclose(vals[0] @ needs_swap, np.eye(2), atol=1e-15)
    S = csr_from_dense(blockdiag([np.ones((2, 2)), np.eye(2)]))  # singular block
    with pytest.raises(ValueError):
        orc.block_jacobi(S, bs=2)
    r = orc.gmres(S, np.ones(4), restart=4, fmt="fp64", tol=1e-10, maxiter=10,
                  precond="block_jacobi", pc_block=2)
    assert r["status"] == -1
