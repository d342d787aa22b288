"""Learned sparse-approximate-inverse preconditioner -- CPU oracle.

TEST INFRASTRUCTURE ONLY: used by the test suite and the smoke check to
check the gfx950 kernels; the product path never imports it.

This preconditioner is an extension of the paper, not part of it. The paper
runs its solver with a scalar Jacobi right preconditioner (Section 6) and
discusses block-Jacobi ones. Here a small per-row network proposes the
values of a right preconditioner P on A's sparsity pattern. Every definition
below is this project's own; FP64 arithmetic is used except at the stated
rounding points.

* Slots. On an nx*ny*nz grid with x-fastest numbering, slot p = 0..26 is the
  offset (dz, dy, dx) = (p//9 - 1, (p//3)%3 - 1, p%3 - 1); slot 13 is the
  diagonal. The entry (i, c) of A has the slot of the grid offset from row i
  to column c.
* Features of row i (64 values): f_p = fl32(a_{i,c(p)} / a_ii) for slots
  present in row i (0 otherwise); f_27 = fl32((a_ii - sum_{c != i} |a_ic|)
  / a_ii), the sum taken in CSR order; f_28..31 = 0; f_{32+p} =
  fl32(a_{c(p),c(p)} / a_ii), the neighbour's diagonal relative to the
  row's, for slots present in row i (0 otherwise); f_59..63 = 0. Each is
  then rounded to bf16 (round to nearest even). The neighbour diagonals
  carry what row i alone cannot: an entry of a good approximate inverse
  near (i, c) depends on the size of a_cc as well as on row i.
* Network, 64 -> 64 -> 64 -> 32: H1 = bf16(ReLU(F W1 + b1)),
  H2 = bf16(ReLU(H1 W2 + b2)), O = H2 W3 + b3. Weights are bf16 and biases
  fp32. The oracle accumulates in FP64 and rounds at the bf16 points.
* P values: P_{i,c} = fl32((delta_{p,13} + O_{i,p}) / a_ii) on A's
  pattern (p = slot of (i, c)). With W3 = 0 and b3 = 0 this is
  P = fl32(D^-1): scalar Jacobi.
* Loss over unit Arnoldi vectors v_k, k in a batch B:
  L = (1/|B|) sum_k ||A P v_k - v_k||_2^2.
* Gradient: G_k = (2/|B|) A^T (A P v_k - v_k); dP_{i,c} = sum_k G_k[i] v_k[c];
  dO_{i,p} = dP_{i,c(p)} / a_ii; then the network's backward pass, with dO,
  dH2 and dH1 rounded to bf16 before each product (as the GPU feeds them to
  bf16 matrix units).
* Adam (Kingma and Ba, 2015) on fp32 master weights; the bf16 weights are
  the round-to-nearest-even of the masters.
* Stored form for the solve: the corrections O_{i,p} of the slots present
  in row i, rounded once to float16 (round to nearest even from the fp32
  network output; 0 for absent slots), slot-major (27 rows of ld codes).
  The solve applies z_i = fl(1/a_ii) * sum_p ([p = 13] + o_{p,i}) v at the
  slot's grid neighbour (ORC_PC_STENCIL of the oracle's options): the same
  operator as D^-1 (I + O) up to the float16 rounding of O, with zero
  codes giving Jacobi bit for bit.
"""
from __future__ import annotations

import numpy as np

from . import decode, encode

NFEAT, NHID, NOUT, NSLOT, CENTER = 64, 64, 32, 27, 13
NBR = 32                     # first neighbour-diagonal feature


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    q, _ = encode("bf16", x.reshape(-1))
    return decode("bf16", q).reshape(x.shape)


def fl32(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def entry_slots(A, grid) -> np.ndarray:
    """Slot (0..26) of every stored entry of A; -1 if not a 27-point offset."""
    nx, ny, nz = grid
    rows = np.repeat(np.arange(A.n, dtype=np.int64), np.diff(A.row_ptr))
    cols = A.col_idx.astype(np.int64)
    xr, yr, zr = rows % nx, (rows // nx) % ny, rows // (nx * ny)
    xc, yc, zc = cols % nx, (cols // nx) % ny, cols // (nx * ny)
    dx, dy, dz = xc - xr, yc - yr, zc - zr
    ok = (np.abs(dx) <= 1) & (np.abs(dy) <= 1) & (np.abs(dz) <= 1)
    return np.where(ok, (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1), -1).astype(np.int64)


def diagonal(A) -> np.ndarray:
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    d = np.zeros(A.n)
    m = A.col_idx == rows
    d[rows[m]] = A.val[m]
    return d


def features(A, grid) -> np.ndarray:
    """(n, 64) features, bf16-representable float64 values."""
    n = A.n
    slots = entry_slots(A, grid)
    d = diagonal(A)
    rows = np.repeat(np.arange(n), np.diff(A.row_ptr))
    F = np.zeros((n, NFEAT))
    good = slots >= 0
    F[rows[good], slots[good]] = fl32(A.val[good] / d[rows[good]])
    F[rows[good], NBR + slots[good]] = fl32(d[A.col_idx[good]] / d[rows[good]])
    # off-diagonal absolute sum of each row, accumulated in CSR order
    off = np.where(A.col_idx == rows, 0.0, np.abs(A.val))
    lens = np.diff(A.row_ptr)
    s = np.zeros(n)
    for t in range(int(lens.max()) if n else 0):
        has = lens > t
        s[has] = s[has] + off[A.row_ptr[:-1][has] + t]
    F[:, 27] = fl32((d - s) / d)
    return bf16(F)


def forward(F, W1, b1, W2, b2, W3, b3, rounding=True):
    """Returns (H1, H2, O). Weights are taken as given (bf16 values)."""
    r = bf16 if rounding else (lambda z: z)
    H1 = r(np.maximum(F @ W1 + b1, 0.0))
    H2 = r(np.maximum(H1 @ W2 + b2, 0.0))
    O = H2 @ W3 + b3
    return H1, H2, O


def p_values(A, grid, O, rounding=True) -> np.ndarray:
    """Values of P on A's pattern (float64 holding fp32 values)."""
    slots = entry_slots(A, grid)
    d = diagonal(A)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    o = np.where(slots >= 0, O[rows, np.maximum(slots, 0)], 0.0)
    delta = (slots == CENTER).astype(np.float64)
    val = (delta + np.where(slots >= 0, o, 0.0)) / d[rows]
    val = np.where(slots >= 0, val, 0.0)
    return fl32(val) if rounding else val


def stencil_codes(A, grid, O, ld=None) -> np.ndarray:
    """(27, ld) uint16 float16 codes of the stored form: slot p of row i holds
    fp16(O_{i,p}) if row i stores that slot, else 0.  O (n, >= 27) holds
    fp32 values; numpy's float32 -> float16 cast rounds once to nearest
    even."""
    ld = A.n if ld is None else ld
    slots = entry_slots(A, grid)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    good = slots >= 0
    codes = np.zeros((NSLOT, ld), dtype=np.uint16)
    o16 = np.asarray(O, dtype=np.float32)[rows[good], slots[good]].astype(np.float16)
    codes[slots[good], rows[good]] = o16.view(np.uint16)
    return codes


def _csr_matvec(A, vals, X):
    import scipy.sparse as sp
    M = sp.csr_matrix((vals, A.col_idx, A.row_ptr), shape=(A.n, A.n))
    return M @ X


def loss_and_grad_p(A, pvals, V):
    """V: (K, n) vectors.  Returns (L, dP) with dP on A's pattern."""
    K = V.shape[0]
    Y = _csr_matvec(A, pvals, V.T)              # P v_k      (n, K)
    R = _csr_matvec(A, A.val, Y) - V.T          # A P v_k - v_k
    L = float(np.sum(R * R)) / K
    import scipy.sparse as sp
    At = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n, A.n)).T.tocsr()
    G = (2.0 / K) * (At @ R)                    # (n, K)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    dP = np.einsum("ek,ek->e", G[rows], V.T[A.col_idx])
    return L, dP


def grad_o(A, grid, dP) -> np.ndarray:
    """dL/dO (n, 32) from dL/dP through P = (delta + O) / a_ii."""
    slots = entry_slots(A, grid)
    d = diagonal(A)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    dO = np.zeros((A.n, NOUT))
    good = slots >= 0
    dO[rows[good], slots[good]] = dP[good] / d[rows[good]]
    return dO


def backward(F, H1, H2, W2, W3, dO, rounding=True):
    """Gradients of the weights and biases given dL/dO."""
    r = bf16 if rounding else (lambda z: z)
    dO = r(dO)
    dW3 = H2.T @ dO
    db3 = dO.sum(axis=0)
    dH2 = r((dO @ W3.T) * (H2 > 0))
    dW2 = H1.T @ dH2
    db2 = dH2.sum(axis=0)
    dH1 = r((dH2 @ W2.T) * (H1 > 0))
    dW1 = F.T @ dH1
    db1 = dH1.sum(axis=0)
    return dict(W1=dW1, b1=db1, W2=dW2, b2=db2, W3=dW3, b3=db3)


def init_params(seed: int):
    """He-normal W1, W2 (seeded, counter-based); W3 = 0, biases 0."""
    from paper_2009_12101_amd.problems import STREAM_WEIGHTS, normal
    z = normal(seed, STREAM_WEIGHTS, NFEAT * NHID + NHID * NHID)
    W1 = (z[:NFEAT * NHID] * np.sqrt(2.0 / NFEAT)).reshape(NFEAT, NHID)
    W2 = (z[NFEAT * NHID:] * np.sqrt(2.0 / NHID)).reshape(NHID, NHID)
    return dict(W1=fl32(W1), b1=np.zeros(NHID), W2=fl32(W2), b2=np.zeros(NHID),
                W3=np.zeros((NHID, NOUT)), b3=np.zeros(NOUT))


def adam_step(params, grads, state, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (bias-corrected), fp32 masters; returns the bf16 view
    of the weights (biases stay fp32)."""
    for k in params:
        g = grads[k]
        m = state.setdefault("m_" + k, np.zeros_like(g))
        v = state.setdefault("v_" + k, np.zeros_like(g))
        m[...] = fl32(beta1 * m + (1 - beta1) * g)
        v[...] = fl32(beta2 * v + (1 - beta2) * g * g)
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        params[k] = fl32(params[k] - lr * mh / (np.sqrt(vh) + eps))
    return {k: (bf16(v) if k.startswith("W") else v) for k, v in params.items()}
