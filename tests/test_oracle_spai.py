"""Pins of the learned-preconditioner oracle (oracle/spai.py).

The network, features and loss are this project's own definitions; the pins
check them against closed forms and finite differences, not against
themselves: an untrained network is exactly fp32 Jacobi, the identity
network returns ReLU(features), known stencil coefficients give known
features, P = 0 and P = A^-1 give known losses, central differences match
every gradient with rounding switched off, and one Adam step from rest
moves each weight by lr * sign(g).
"""
import numpy as np
import pytest

from paper_2009_12101_amd import problems as P


@pytest.fixture(scope="module")
def S():
    from oracle import spai
    return spai


def unit_vectors(n, K, seed):
    V = np.random.default_rng(seed).standard_normal((K, n))
    return V / np.linalg.norm(V, axis=1, keepdims=True)


def test_untrained_network_is_fp32_jacobi(S):
    A = P.lognormal27(5, 2)
    F = S.features(A, A.grid)
    prm = S.init_params(7)
    _, _, O = S.forward(F, prm["W1"], prm["b1"], prm["W2"], prm["b2"], prm["W3"], prm["b3"])
    assert np.all(O == 0.0)
    pv = S.p_values(A, A.grid, O)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    diag = A.col_idx == rows
    expect = np.where(diag, (1.0 / A.val).astype(np.float32).astype(np.float64), 0.0)
    assert np.array_equal(pv, expect)


def test_features_of_constant_coefficient_stencil(S):
    A = P.lognormal27(4, 0, sigma=0.0)        # kappa = 1: -1 off the diagonal, 26.01 on it
    F = S.features(A, A.grid)
    b = lambda x: float(np.float64(np.float32(x)))
    f_off = S.bf16(np.array([b(-1.0 / 26.01)]))[0]
    # an interior row (1,1,1): all 27 slots present
    i = 1 + 4 + 16
    assert np.all(F[i, :27][np.arange(27) != 13] == f_off)
    assert F[i, 13] == 1.0
    assert F[i, 27] == S.bf16(np.array([b((26.01 - 26.0) / 26.01)]))[0]
    assert np.all(F[i, 28:32] == 0.0)
    # neighbour diagonals: every in-grid neighbour of (1,1,1) on a 4^3 grid
    # has 26 weights of 1 plus the shift, so each ratio is exactly 1
    assert np.all(F[i, 32:59] == 1.0)
    assert np.all(F[i, 59:] == 0.0)
    # the corner row 0: 7 off-diagonal neighbours, all others absent
    present = [13, 14, 16, 17, 22, 23, 25, 26]
    for p in range(27):
        assert F[0, p] == (1.0 if p == 13 else f_off if p in present else 0.0)
        assert F[0, 32 + p] == (1.0 if p in present else 0.0)
    assert F[0, 27] == S.bf16(np.array([b((26.01 - 7.0) / 26.01)]))[0]


@pytest.mark.parametrize("axis", ["x", "z"])
def test_features_of_a_chain_with_varying_diagonal(S, axis):
    # three unknowns in a line along x (slots 12, 14) or z (slots 4, 22),
    # diagonal 2, 4, 8 and -1 between neighbours; every feature is a ratio of
    # small powers of two, exact in bfloat16
    from _helpers import csr_from_dense
    M = np.diag([2.0, 4.0, 8.0]) - np.eye(3, k=1) - np.eye(3, k=-1)
    A = csr_from_dense(M)
    grid = (3, 1, 1) if axis == "x" else (1, 1, 3)
    lo, hi = (12, 14) if axis == "x" else (4, 22)
    F = S.features(A, grid)
    expect = np.zeros((3, 64))
    expect[:, 13] = expect[:, 32 + 13] = 1.0
    expect[0, hi], expect[0, 32 + hi], expect[0, 27] = -0.5, 2.0, 0.5
    expect[1, lo], expect[1, hi], expect[1, 27] = -0.25, -0.25, 0.5
    expect[1, 32 + lo], expect[1, 32 + hi] = 0.5, 2.0
    expect[2, lo], expect[2, 32 + lo], expect[2, 27] = -0.125, 0.5, 0.875
    assert np.array_equal(F, expect)


def test_identity_network_returns_relu_of_features(S):
    A = P.lognormal27(4, 3)
    F = S.features(A, A.grid)
    W1 = np.eye(64)
    W2 = np.eye(64)
    W3 = np.zeros((64, 32)); W3[:32, :32] = np.eye(32)
    _, _, O = S.forward(F, W1, np.zeros(64), W2, np.zeros(64), W3, np.zeros(32))
    assert np.array_equal(O, np.maximum(F[:, :32], 0.0))
    W3 = np.zeros((64, 32)); W3[32:, :] = np.eye(32)
    _, _, O = S.forward(F, W1, np.zeros(64), W2, np.zeros(64), W3, np.zeros(32))
    assert np.array_equal(O, np.maximum(F[:, 32:], 0.0))


def test_loss_closed_forms(S):
    A = P.lognormal27(4, 1)
    V = unit_vectors(A.n, 3, 0) * np.array([[1.0], [2.0], [0.5]])
    L, dP = S.loss_and_grad_p(A, np.zeros(A.nnz), V)
    assert L == pytest.approx(np.mean(np.sum(V * V, axis=1)), rel=1e-14)
    # A = 4 I on a grid (only the diagonal slot stored) and P = 1/4: A P = I
    n = 27
    from _helpers import csr_from_dense
    D = csr_from_dense(4.0 * np.eye(n))
    L, dP = S.loss_and_grad_p(D, np.full(n, 0.25), unit_vectors(n, 2, 1))
    assert L == 0.0 and np.all(dP == 0.0)


def _loss_of_params(S, A, F, V, prm):
    _, _, O = S.forward(F, prm["W1"], prm["b1"], prm["W2"], prm["b2"], prm["W3"], prm["b3"],
                        rounding=False)
    pv = S.p_values(A, A.grid, O, rounding=False)
    return S.loss_and_grad_p(A, pv, V)[0]


def test_gradients_match_central_differences(S):
    A = P.lognormal27(4, 5)
    F = S.features(A, A.grid)
    V = unit_vectors(A.n, 2, 3)
    rng = np.random.default_rng(11)
    prm = dict(W1=rng.standard_normal((64, 64)) * 0.3, b1=rng.standard_normal(64) * 0.1,
               W2=rng.standard_normal((64, 64)) * 0.2, b2=rng.standard_normal(64) * 0.1,
               W3=rng.standard_normal((64, 32)) * 0.05, b3=rng.standard_normal(32) * 0.01)
    H1, H2, O = S.forward(F, prm["W1"], prm["b1"], prm["W2"], prm["b2"], prm["W3"], prm["b3"],
                          rounding=False)
    pv = S.p_values(A, A.grid, O, rounding=False)
    L, dP = S.loss_and_grad_p(A, pv, V)
    # dL/dP
    for e in rng.choice(A.nnz, 12, replace=False):
        h = 1e-6
        pp, pm = pv.copy(), pv.copy()
        pp[e] += h
        pm[e] -= h
        fd = (S.loss_and_grad_p(A, pp, V)[0] - S.loss_and_grad_p(A, pm, V)[0]) / (2 * h)
        assert abs(fd - dP[e]) <= 1e-6 * max(abs(fd), 1e-3)
    # dL/dparams through the network
    g = S.backward(F, H1, H2, prm["W2"], prm["W3"], S.grad_o(A, A.grid, dP), rounding=False)
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in prm[name].shape)
            h = 1e-6
            pp = {k: v.copy() for k, v in prm.items()}
            pm = {k: v.copy() for k, v in prm.items()}
            pp[name][idx] += h
            pm[name][idx] -= h
            fd = (_loss_of_params(S, A, F, V, pp) - _loss_of_params(S, A, F, V, pm)) / (2 * h)
            assert abs(fd - g[name][idx]) <= 1e-6 * max(abs(fd), 1e-4), (name, idx)


def test_adam_first_step_is_lr_sign(S):
    rng = np.random.default_rng(0)
    prm = dict(W1=np.zeros((64, 64)), b1=np.zeros(64), W2=np.zeros((64, 64)), b2=np.zeros(64),
               W3=np.zeros((64, 32)), b3=np.zeros(32))
    g = {k: rng.standard_normal(v.shape) for k, v in prm.items()}
    view = S.adam_step(prm, g, {}, 1, lr=1e-3)
    for k in prm:
        expect = -1e-3 * g[k].astype(np.float32) / (np.abs(g[k].astype(np.float32)) + 1e-8)
        assert np.allclose(prm[k], expect, rtol=1e-6, atol=0)
        # the network reads bfloat16 weights (torch's round-to-nearest-even
        # cast of the fp32 masters) and fp32 biases
        if k.startswith("W"):
            import torch
            bf = torch.from_numpy(prm[k].astype(np.float32)).to(torch.bfloat16).double().numpy()
            assert np.array_equal(view[k], bf)
        else:
            assert np.array_equal(view[k], prm[k])


# ---------------------------------------------------------------- stored form

def _stencil_csr(A, grid, codes):
    """The stored form assembled independently as a scipy CSR matrix:
    M = diag(1/a_ii) (I + O16) with O16 the decoded codes at the grid
    neighbour of each slot (numpy's float16 decode)."""
    import scipy.sparse as sp
    nx, ny, nz = grid
    n = A.n
    rows, cols, vals = [], [], []
    dinv = 1.0 / np.array([A.val[A.row_ptr[i]:A.row_ptr[i + 1]][
        A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]] == i][-1] for i in range(n)])
    o = codes.view(np.float16).astype(np.float64)
    for i in range(n):
        x, y, z = i % nx, (i // nx) % ny, i // (nx * ny)
        for p in range(27):
            dz, dy, dx = p // 9 - 1, (p // 3) % 3 - 1, p % 3 - 1
            if 0 <= x + dx < nx and 0 <= y + dy < ny and 0 <= z + dz < nz:
                c = (1.0 if p == 13 else 0.0) + o[p, i]
                if c != 0.0:
                    rows.append(i)
                    cols.append(i + dz * nx * ny + dy * nx + dx)
                    vals.append(dinv[i] * c)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n)), dinv


def test_stencil_codes_are_fp16_of_the_present_slots(S):
    """Codes: fp16(O) on the slots row i stores, 0 on the others (a 7-point
    matrix leaves 20 of the 27 grid slots of an interior row empty), at
    stride ld; checked entry by entry against the CSR pattern."""
    A = P.convdiff7(4)
    O = np.random.default_rng(1).standard_normal((A.n, 32)).astype(np.float32)
    ld = A.n + 5
    codes = S.stencil_codes(A, A.grid, O, ld)
    assert codes.shape == (27, ld) and np.all(codes[:, A.n:] == 0)
    nx, ny, _ = A.grid
    for i in range(A.n):
        present = {}
        for q in range(A.row_ptr[i], A.row_ptr[i + 1]):
            d = int(A.col_idx[q]) - i
            dz = 1 if d >= nx * ny - nx - 1 else (-1 if d <= -(nx * ny - nx - 1) else 0)
            rem = d - dz * nx * ny
            dy = 1 if rem >= nx - 1 else (-1 if rem <= -(nx - 1) else 0)
            dx = rem - dy * nx
            present[9 * (dz + 1) + 3 * (dy + 1) + dx + 1] = True
        for p in range(27):
            want = np.float16(O[i, p]).view(np.uint16) if p in present else 0
            assert codes[p, i] == want, (i, p)
    assert sum(1 for p in range(27) if codes[p, 21 + 16] != 0) <= 7


def test_stencil_apply_against_assembled_matrix(S):
    import oracle as orc
    A = P.lognormal27(5, 4)
    O = (0.3 * np.random.default_rng(2).standard_normal((A.n, 32))).astype(np.float32)
    codes = S.stencil_codes(A, A.grid, O)
    M, dinv = _stencil_csr(A, A.grid, codes)
    v = np.random.default_rng(3).standard_normal(A.n)
    z = orc.stencil_apply(A, A.grid, codes, v)
    bound = 30 * 2.0 ** -53 * (abs(M) @ np.abs(v))
    assert np.all(np.abs(z - M @ v) <= bound)
    # a hand-computed row: the interior row (1,1,1) of a 3^3 grid sees all 27
    A3 = P.lognormal27(3, 5)
    O3 = np.zeros((A3.n, 32), np.float32)
    O3[13, 12], O3[13, 14], O3[13, 13], O3[13, 4] = 0.5, -0.25, 0.125, 2.0
    c3 = S.stencil_codes(A3, A3.grid, O3)
    v3 = np.arange(1.0, 28.0)
    d13 = A3.val[A3.row_ptr[13]:A3.row_ptr[14]][A3.col_idx[A3.row_ptr[13]:A3.row_ptr[14]] == 13]
    want = (1.0 / d13[0]) * (0.5 * v3[12] + 1.125 * v3[13] - 0.25 * v3[14] + 2.0 * v3[4])
    assert orc.stencil_apply(A3, A3.grid, c3, v3)[13] == want


def test_stencil_zero_codes_are_jacobi_bit_for_bit(S):
    import oracle as orc
    A = P.lognormal27(6, 1)
    codes = np.zeros((27, A.n), np.uint16)
    v = np.random.default_rng(0).standard_normal(A.n)
    assert np.array_equal(orc.stencil_apply(A, A.grid, codes, v), (1.0 / S.diagonal(A)) * v)
    b = P.rhs_uniform(A.n, 1)
    for fmt in ("fp64", "fp16"):
        rj = orc.gmres(A, b, restart=20, fmt=fmt, tol=1e-10, maxiter=500, precond="jacobi")
        rs = orc.gmres(A, b, restart=20, fmt=fmt, tol=1e-10, maxiter=500, precond="stencil",
                       p_stencil=codes, grid=A.grid)
        assert rj["iterations"] == rs["iterations"]
        assert np.array_equal(rj["x"], rs["x"])


def test_stencil_solve_equals_change_of_variables(S):
    """Right preconditioning with the stored form: GMRES on A M^-1 y = b,
    x = M^-1 y, against a plain run on the explicitly assembled A M."""
    import oracle as orc
    from tests._helpers import csr_from_scipy
    A = P.lognormal27(5, 3)
    b = P.rhs_uniform(A.n, 3)
    O = (0.02 * np.random.default_rng(4).standard_normal((A.n, 32))).astype(np.float32)
    codes = S.stencil_codes(A, A.grid, O)
    M, _ = _stencil_csr(A, A.grid, codes)
    AM = csr_from_scipy(A.to_scipy() @ M)
    rs = orc.gmres(A, b, restart=20, fmt="fp64", tol=1e-10, maxiter=2000, precond="stencil",
                   p_stencil=codes, grid=A.grid)
    rp = orc.gmres(AM, b, restart=20, fmt="fp64", tol=1e-10, maxiter=2000)
    assert rs["status"] == 0 and rp["status"] == 0
    assert abs(rs["iterations"] - rp["iterations"]) <= 1
    x = M @ rp["x"]
    assert np.linalg.norm(rs["x"] - x) <= 1e-7 * np.linalg.norm(x)


def test_stencil_fallback_and_argument_checks(S):
    import oracle as orc
    A = P.lognormal27(4, 2)
    b = P.rhs_uniform(A.n, 2)
    # codes of -1 on the diagonal slot make M^-1 = 0 on every row: non-finite
    # values in the first cycle, so the solver drops M and finishes with M = I
    codes = np.zeros((27, A.n), np.uint16)
    codes[13, :] = np.float16(-1.0).view(np.uint16)
    r = orc.gmres(A, b, restart=20, fmt="fp64", tol=1e-10, maxiter=3000, precond="stencil",
                  p_stencil=codes, grid=A.grid, fallback=True)
    assert r["status"] == 0 and r["fell_back"] == 1 and r["true_rel_res"] <= 1e-10
    r = orc.gmres(A, b, restart=20, fmt="fp64", tol=1e-10, maxiter=3000, precond="stencil",
                  p_stencil=codes, grid=(4, 4, 3))
    assert r["status"] == -1                      # the grid does not number the rows
    with pytest.raises(ValueError):
        orc.stencil_apply(A, (4, 4, 3), codes, b)
