"""Seeded synthetic sparse systems A x = b.

This module builds the inputs only: matrices in CSR form and right-hand sides.
It holds none of the solver's arithmetic and imports nothing from the HIP
library or from the CPU oracle, so both sides consume the same bytes.

The paper evaluates on large SuiteSparse matrices with 4-82 nonzeros per row
(Section 6, Table 1). Those are not available here; the stencil systems below
stand in for the two shape groups that table spans:

* ``convdiff7``  -- 7 nonzeros per row (the 5-7 nnz/row group),
* ``lognormal27`` -- 27 nonzeros per row (the 21-35 nnz/row group),
* ``poisson2d``  -- a tiny 5-point system for correctness runs.

All grids use lexicographic numbering with x fastest and Dirichlet boundaries
(out-of-grid neighbours are dropped), so every CSR row has its column indices
sorted ascending. Indices are int32, values float64.

Random numbers come from counter-based SplitMix64 (Steele, Lea and Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014): element ``i``
of stream ``s`` under seed ``seed`` is the SplitMix64 output at counter
``i + 1`` of the state ``mix(mix(seed) + s)``.
"""
from __future__ import annotations

import dataclasses

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# stream identifiers, one per kind of random draw
STREAM_RHS = 1
STREAM_COEF = 2
STREAM_WEIGHTS = 3


def _mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (wrapping uint64 arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, stream: int, count: int, start: int = 0) -> np.ndarray:
    """``count`` raw 64-bit draws of (seed, stream) at counters start+1 ..."""
    with np.errstate(over="ignore"):
        base = _mix(_mix(np.uint64(seed) + _GAMMA) + np.uint64(stream))
        ctr = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
        return _mix(base + ctr * _GAMMA)


def uniform01(seed: int, stream: int, count: int, start: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits of each draw."""
    u = splitmix64(seed, stream, count, start) >> np.uint64(11)
    return u.astype(np.float64) * (2.0 ** -53)


def normal(seed: int, stream: int, count: int) -> np.ndarray:
    """Standard normals by Box-Muller on counters (2i, 2i+1)."""
    u = uniform01(seed, stream, 2 * count).reshape(count, 2)
    r = np.sqrt(-2.0 * np.log1p(-u[:, 0]))          # 1-u in (0, 1]
    return r * np.cos(2.0 * np.pi * u[:, 1])


@dataclasses.dataclass
class CSR:
    """A square sparse matrix in CSR form (0-based, sorted columns)."""
    n: int
    row_ptr: np.ndarray   # int32, n+1
    col_idx: np.ndarray   # int32, nnz
    val: np.ndarray       # float64, nnz
    grid: tuple | None = None   # (nx, ny, nz) for structured-grid matrices
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.n, self.n))


def _stencil_csr(dims, offsets, values, name):
    """Assemble CSR from per-offset value arrays on an nx*ny*nz grid.

    ``offsets`` is a list of (dz, dy, dx) in lexicographic order, which is
    also ascending column order for x-fastest numbering. ``values[p]`` is an
    (n,) float64 array with the entry of row i at offset p; entries whose
    neighbour is outside the grid are dropped.
    """
    nx, ny, nz = dims
    n = nx * ny * nz
    idx = np.arange(n, dtype=np.int64)
    x = idx % nx
    y = (idx // nx) % ny
    z = idx // (nx * ny)
    ncol = len(offsets)
    mask = np.empty((n, ncol), dtype=bool)
    cols = np.empty((n, ncol), dtype=np.int64)
    for p, (dz, dy, dx) in enumerate(offsets):
        mask[:, p] = ((x + dx >= 0) & (x + dx < nx) & (y + dy >= 0) & (y + dy < ny)
                      & (z + dz >= 0) & (z + dz < nz))
        cols[:, p] = idx + dx + dy * nx + dz * nx * ny
    vals = np.stack(values, axis=1)
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col_idx = cols[mask].astype(np.int32)
    val = np.ascontiguousarray(vals[mask], dtype=np.float64)
    assert row_ptr[-1] < 2 ** 31
    return CSR(n, row_ptr.astype(np.int32), col_idx, val, grid=dims, name=name)


def poisson2d(nx: int) -> CSR:
    """2D 5-point Poisson on an nx*nx grid: 4 on the diagonal, -1 off it."""
    n = nx * nx
    offs = [(0, -1, 0), (0, 0, -1), (0, 0, 0), (0, 0, 1), (0, 1, 0)]
    one = np.ones(n)
    vals = [-one, -one, 4.0 * one, -one, -one]
    return _stencil_csr((nx, nx, 1), offs, vals, f"poisson2d_{nx}")


def convdiff7(N: int, beta: float = 10.0, cell_peclet: bool = False) -> CSR:
    """3D 7-point upwind convection-diffusion on an N^3 grid of the unit cube.

    -Laplace(u) + beta . grad(u) with beta = (beta, beta, beta), mesh width
    h = 1/(N+1), first-order upwind convection, all entries scaled by h^2:
    diagonal 6 + 3*beta*h, upwind neighbours -1 - beta*h, downwind -1.
    Nonsymmetric. ``cell_peclet=True`` takes ``beta`` as the cell Peclet
    number beta*h instead (so diagonal 6 + 3*beta).
    """
    n = N ** 3
    bh = beta if cell_peclet else beta / (N + 1)
    one = np.ones(n)
    offs = [(-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 0), (0, 0, 1), (0, 1, 0), (1, 0, 0)]
    up = -(1.0 + bh) * one
    down = -1.0 * one
    diag = (6.0 + 3.0 * bh) * one
    vals = [up, up, up, diag, down, down, down]
    return _stencil_csr((N, N, N), offs, vals, f"convdiff7_{N}")


def lognormal_kappa(N: int, seed: int, sigma: float = 1.0) -> np.ndarray:
    """Node coefficients kappa_i = exp(sigma * z_i), z_i ~ N(0, 1) i.i.d."""
    return np.exp(sigma * normal(seed, STREAM_COEF, N ** 3))


def lognormal27(N: int, seed: int = 0, sigma: float = 1.0, shift: float = 1e-2) -> CSR:
    """3D 27-point variable-coefficient diffusion on an N^3 grid.

    Edge weight w_ij = sqrt(kappa_i * kappa_j) for each of the 26 neighbours,
    a_ij = -w_ij, a_ii = sum of the 26 weights (an out-of-grid neighbour uses
    kappa_i, i.e. weight kappa_i) + ``shift``. Symmetric positive definite.
    """
    n = N ** 3
    kap = lognormal_kappa(N, seed, sigma)
    idx = np.arange(n, dtype=np.int64)
    x = idx % N
    y = (idx // N) % N
    z = idx // (N * N)
    offs = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    vals = []
    diag = np.zeros(n)
    for (dz, dy, dx) in offs:
        if (dz, dy, dx) == (0, 0, 0):
            vals.append(None)
            continue
        inside = ((x + dx >= 0) & (x + dx < N) & (y + dy >= 0) & (y + dy < N)
                  & (z + dz >= 0) & (z + dz < N))
        j = np.where(inside, idx + dx + dy * N + dz * N * N, idx)
        w = np.sqrt(kap * kap[j])
        diag += w
        vals.append(-w)
    vals[13] = diag + shift
    return _stencil_csr((N, N, N), offs, vals, f"lognormal27_{N}_s{seed}")


def rhs_uniform(n: int, seed: int = 0) -> np.ndarray:
    """b_i ~ U[-1, 1) from (seed, STREAM_RHS)."""
    return 2.0 * uniform01(seed, STREAM_RHS, n) - 1.0


def rhs_sin(n: int) -> np.ndarray:
    """b_i = sin(i), i = 1..n (the right-hand side of the paper's Section 6)."""
    return np.sin(np.arange(1, n + 1, dtype=np.float64))


def rhs_row_sums(A: CSR) -> np.ndarray:
    """b = A * ones, i.e. the row sums (exact solution x* = 1)."""
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    return np.bincount(rows, weights=A.val, minlength=A.n)


# Named workloads. Each entry builds (A, b); sizes follow the stencil
# families above.
def workload(name: str):
    """Return (A, b, defaults) for a named synthetic workload."""
    if name == "poisson2d_64":
        A = poisson2d(64)
        return A, rhs_row_sums(A), dict(restart=100, tol=1e-10, format="fp32")
    if name.startswith("convdiff7_"):
        N = int(name.split("_")[1])
        A = convdiff7(N)
        return A, rhs_uniform(A.n, 0), dict(restart=100, tol=1e-10, format="fp16")
    if name.startswith("lognormal27_"):
        parts = name.split("_")
        N = int(parts[1])
        seed = int(parts[2][1:]) if len(parts) > 2 else 0
        A = lognormal27(N, seed)
        return A, rhs_uniform(A.n, seed), dict(restart=100, tol=1e-10, format="bf16")
    raise KeyError(name)
