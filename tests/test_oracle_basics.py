"""Pins of the oracle's basic operations against independent references.

* SpMV y = A x: equal to scipy's CSR product bit for bit on integer data
  (every product and partial sum exact), and within the FP64 bound of
  scipy's on random data, ragged rows and empty rows included.
* dot: exact on integer vectors; within n u sum|x_i y_i| of the exactly
  rounded sum (math.fsum) on random data; the fixed block order (blocks of
  1024 consecutive entries, then the block sums in order) reproduced by a
  plain loop written from that definition.
"""
import math

import numpy as np
import pytest

from tests._helpers import csr_from_dense

U = 2.0 ** -53


def random_csr(n, density, seed, integer=False):
    rng = np.random.default_rng(seed)
    M = np.where(rng.random((n, n)) < density, 1.0, 0.0)
    M[rng.integers(0, n, 3)] = 0.0                    # a few empty rows
    vals = rng.integers(-9, 10, (n, n)) if integer else rng.standard_normal((n, n))
    return csr_from_dense(M * vals)


@pytest.mark.parametrize("seed", range(3))
def test_spmv_integer_data_is_exact(orc, seed):
    A = random_csr(300, 0.05, seed, integer=True)
    x = np.random.default_rng(seed + 10).integers(-1000, 1000, A.n).astype(np.float64)
    y = orc.spmv(A, x)
    assert np.array_equal(y, A.to_scipy() @ x)


@pytest.mark.parametrize("seed", range(3))
def test_spmv_random_data_within_fp64_bound(orc, seed):
    A = random_csr(400, 0.03, seed)
    x = np.random.default_rng(seed + 20).standard_normal(A.n)
    y = orc.spmv(A, x)
    S = A.to_scipy()
    ref = S @ x
    rowlen = np.diff(A.row_ptr)
    bound = 2 * np.maximum(rowlen, 1) * U * (abs(S) @ np.abs(x))
    assert np.all(np.abs(y - ref) <= bound)


def test_dot_exact_on_integers(orc):
    rng = np.random.default_rng(1)
    x = rng.integers(-2 ** 20, 2 ** 20, 5001).astype(np.float64)
    y = rng.integers(-2 ** 20, 2 ** 20, 5001).astype(np.float64)
    assert orc.dot(x, y) == float(np.dot(x.astype(np.int64), y.astype(np.int64)))


@pytest.mark.parametrize("n", [1, 1023, 1024, 1025, 7777])
def test_dot_block_order_and_bound(orc, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) * 10.0 ** rng.uniform(-3, 3, n)
    y = rng.standard_normal(n)
    d = orc.dot(x, y)
    exact = math.fsum(float(a) * float(b) for a, b in zip(x, y))
    assert abs(d - exact) <= n * U * float(np.sum(np.abs(x * y))) + 1e-300
    # the stated order: each block of 1024 in index order, then the blocks
    blocks = []
    for b0 in range(0, n, 1024):
        s = 0.0
        for i in range(b0, min(b0 + 1024, n)):
            s += float(x[i]) * float(y[i])
        blocks.append(s)
    t = 0.0
    for s in blocks:
        t += s
    assert d == t
