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
    S.adam_step(prm, g, {}, 1, lr=1e-3)
    for k in prm:
        expect = -1e-3 * g[k].astype(np.float32) / (np.abs(g[k].astype(np.float32)) + 1e-8)
        assert np.allclose(prm[k], expect, rtol=1e-6, atol=0)
