"""Pins of the oracle's ablation variants of the Arnoldi step and of the
scaled float16 storage format (extensions; the unablated step is Fig. 1).

* fp16s: the stored codes are numpy's single-rounding float16 cast of
  v * 2^-k with the stated choice of k; the scaling commutes with rounding
  where neither side is subnormal, so fp16s equals fp16 there; every finite
  float16 code survives a round trip; small entries keep relative accuracy.
* SpMV on the stored vector: then A dec(v^_j) - sum_k h_kj dec(v^_k) is
  h_{j+1,j} times the unit vector v_{j+1} before storage, so its norm is
  h_{j+1,j} to FP64 rounding; with the FP64 v of Fig. 1 it misses by the
  storage error.  In fp64 storage the variant changes nothing.
* always re-orthogonalise (CGS2): every step re-orthogonalises and the FP64
  basis stays orthogonal to working precision even after convergence
  ("twice is enough", Giraud, Langou and Rozloznik 2005), while one-pass CGS
  loses orthogonality completely.
* MGS: with SpMV on the stored vector, each Hessenberg column is the
  sequential projection of A dec(v^_j) against the decoded stored vectors in
  order, which on an fp16 basis differs from the CGS column far above
  rounding; in fp64 storage, exact arithmetic makes MGS and CGS equal.
* Gram re-dot: with SpMV on the stored vector and a second pass on every
  step, each Hessenberg column is h + (h - V^T V h), h = V^T A dec(v^_j),
  recomputed here with numpy from the decoded basis; the explicit re-dot
  V^T (w - V h) gives the same column to rounding.  h - G h cancels, so on an
  FP64 basis the Gram form keeps orthogonality to u64 omega / t rather than
  u64 (1e-13 against 1e-14 on a near-identity matrix).
"""
import numpy as np
import pytest

from paper_2009_12101_amd import problems as P
from tests._helpers import csr_from_dense

TINY_ETA = 1e-300          # step 7's test never fires: one pass per step


def fp16s_ref(v):
    vinf = np.max(np.abs(v)) if v.size else 0.0
    k = 0
    if vinf > 0:
        k = int(np.floor(np.log2(vinf))) - 15
        if np.ldexp(vinf, -k) > 65504.0:
            k += 1
    return np.ldexp(v, -k).astype(np.float16), np.ldexp(1.0, k)


@pytest.mark.parametrize("seed", range(6))
def test_fp16s_codes_are_single_roundings_of_the_scaled_vector(orc, seed):
    rng = np.random.default_rng(seed)
    mag = 10.0 ** rng.uniform(-30, 30)
    v = rng.standard_normal(3001) * mag
    v[::7] *= 1e-9                                  # entries far below the largest
    q, s = orc.encode("fp16s", v)
    ref, sref = fp16s_ref(v)
    assert s == sref
    assert 32752.0 < np.max(np.abs(v)) / s <= 65504.0
    assert np.array_equal(q, ref.view(np.uint16))
    assert np.array_equal(orc.decode("fp16s", q, s), ref.astype(np.float64) * s)


def test_fp16s_scale_edges(orc):
    q, s = orc.encode("fp16s", np.array([65504.0, -1.0]))
    assert s == 1.0                                 # max exactly 65504: k = 0
    q, s = orc.encode("fp16s", np.array([65505.0]))
    assert s == 2.0                                 # just above: k = 1, (32752, 65504]
    q, s = orc.encode("fp16s", np.zeros(5))
    assert s == 1.0 and np.all(q == 0)


@pytest.mark.parametrize("k", [-40, -3, 0, 17])
def test_fp16s_round_trip_of_every_finite_code(orc, k):
    codes = np.arange(65536, dtype=np.uint16)
    vals = codes.view(np.float16).astype(np.float64)
    keep = np.isfinite(vals)
    v = vals[keep] * 2.0 ** k                       # largest is 65504 * 2^k: scale 2^k
    q, s = orc.encode("fp16s", v)
    assert s == 2.0 ** k
    # -0 and +0 both decode to zero; every other code comes back unchanged
    assert np.array_equal(q[v != 0], codes[keep][v != 0])
    assert np.array_equal(orc.decode("fp16s", q, s), v)


def test_fp16s_equals_fp16_away_from_subnormals_and_beats_it_below(orc):
    rng = np.random.default_rng(9)
    v = rng.uniform(0.25, 1.0, 4000) * np.where(rng.random(4000) < 0.5, -1, 1)
    a = orc.decode("fp16", *orc.encode("fp16", v))
    b = orc.decode("fp16s", *orc.encode("fp16s", v))
    assert np.array_equal(a, b)                    # 2^k scaling commutes with RNE
    w = v * 1e-7                                    # below fp16's normal range
    ea = np.abs(orc.decode("fp16", *orc.encode("fp16", w)) - w) / np.abs(w)
    eb = np.abs(orc.decode("fp16s", *orc.encode("fp16s", w)) - w) / np.abs(w)
    assert eb.max() <= 2.0 ** -11
    assert ea.max() > 0.1


def column_dev(orc, A, V, H, k):
    """|(||A V_j - V_{:j+1} H_{:j+1,j}|| - H_{j+1,j})| / H_{j+1,j} per column."""
    out = []
    for j in range(k - 1):
        r = orc.spmv(A, V[j]) - V[:j + 1].T @ H[:j + 1, j]
        out.append(abs(np.linalg.norm(r) - H[j + 1, j]) / H[j + 1, j])
    return np.array(out)


@pytest.mark.parametrize("fmt", ["fp16", "fp16s", "bf16", "int16", "e4m3"])
def test_spmv_on_stored_vector_column_norms(orc, fmt):
    A = P.convdiff7(10)
    b = P.rhs_uniform(A.n, 1)
    on = orc.gmres(A, b, restart=20, fmt=fmt, tol=0.0, maxiter=20, debug=True,
                   variant="spmv_vhat")
    off = orc.gmres(A, b, restart=20, fmt=fmt, tol=0.0, maxiter=20, debug=True)
    assert column_dev(orc, A, on["V"], on["H"], on["steps"]).max() <= 1e-13
    assert column_dev(orc, A, off["V"], off["H"], off["steps"]).max() >= 1e-7


def test_spmv_on_stored_vector_is_identity_in_fp64(orc):
    A = P.lognormal27(6, 3)
    b = P.rhs_uniform(A.n, 2)
    r0 = orc.gmres(A, b, restart=15, fmt="fp64", tol=1e-10, maxiter=500)
    r1 = orc.gmres(A, b, restart=15, fmt="fp64", tol=1e-10, maxiter=500, variant="spmv_vhat")
    assert r0["iterations"] == r1["iterations"]
    assert np.array_equal(r0["x"], r1["x"])


def test_always_reorth_counts_and_keeps_orthogonality(orc):
    n = 120
    rng = np.random.default_rng(0)
    A = csr_from_dense(np.eye(n) + 0.05 * rng.standard_normal((n, n)) / np.sqrt(n))
    b = rng.standard_normal(n)
    r2 = orc.gmres(A, b, restart=40, fmt="fp64", tol=0.0, maxiter=40, debug=True,
                   variant="always_reorth")
    r1 = orc.gmres(A, b, restart=40, fmt="fp64", tol=0.0, maxiter=40, debug=True, eta=TINY_ETA)
    assert r2["reorths"] == r2["iterations"] == 40 and r1["reorths"] == 0
    k = r2["V"].shape[0]
    assert np.linalg.norm(np.eye(k) - r2["V"] @ r2["V"].T) <= 1e-14
    assert np.linalg.norm(np.eye(k) - r1["V"] @ r1["V"].T) >= 1.0


def test_always_reorth_changes_only_the_pass_count_where_the_test_rarely_fires(orc):
    # an orthogonal matrix: step 7's test rarely fires, and the second passes
    # the flag adds make corrections at rounding level
    n = 64
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = csr_from_dense(Q)
    b = rng.standard_normal(n)
    r0 = orc.gmres(A, b, restart=n, fmt="fp64", tol=1e-12, maxiter=n)
    r2 = orc.gmres(A, b, restart=n, fmt="fp64", tol=1e-12, maxiter=n, variant="always_reorth")
    assert r0["reorths"] < r0["iterations"] // 4 and r2["reorths"] == r2["iterations"]
    assert np.allclose(r2["hist"][:10], r0["hist"][:10], rtol=1e-10, atol=0)


def mgs_columns(orc, A, V, k):
    cols = []
    for j in range(k - 1):
        w = orc.spmv(A, V[j])
        h = np.zeros(j + 2)
        for i in range(j + 1):
            h[i] = V[i] @ w
            w = w - h[i] * V[i]
        h[j + 1] = np.linalg.norm(w)
        cols.append(h)
    return cols


@pytest.mark.parametrize("fmt", ["fp16", "int16"])
def test_mgs_columns_are_sequential_projections(orc, fmt):
    A = P.convdiff7(9)
    b = P.rhs_uniform(A.n, 3)
    kw = dict(restart=16, fmt=fmt, tol=0.0, maxiter=16, debug=True, eta=TINY_ETA)
    rm = orc.gmres(A, b, variant=("mgs", "spmv_vhat"), **kw)
    rc = orc.gmres(A, b, variant="spmv_vhat", **kw)
    cols = mgs_columns(orc, A, rm["V"], rm["steps"])
    worst_m = worst_c = 0.0
    for j, h in enumerate(cols):
        worst_m = max(worst_m, np.max(np.abs(rm["H"][:j + 2, j] - h)) / np.linalg.norm(h))
    # the CGS run's own basis, projected sequentially, differs from its H
    for j, h in enumerate(mgs_columns(orc, A, rc["V"], rc["steps"])):
        worst_c = max(worst_c, np.max(np.abs(rc["H"][:j + 2, j] - h)) / np.linalg.norm(h))
    assert worst_m <= 1e-12
    assert worst_c >= 1e-7


def test_mgs_equals_cgs_in_fp64_and_full_gmres_solves(orc):
    A = P.poisson2d(12)
    b = P.rhs_uniform(A.n, 5)
    kw = dict(restart=30, fmt="fp64", tol=0.0, maxiter=30, debug=True)
    rm = orc.gmres(A, b, variant="mgs", **kw)
    rc = orc.gmres(A, b, **kw)
    k = rm["steps"]
    assert np.allclose(rm["H"][:, :k], rc["H"][:, :k], rtol=0, atol=1e-11)
    # m = n: full GMRES reaches the solution
    n = 24
    rng = np.random.default_rng(2)
    M = np.eye(n) * 4 + rng.standard_normal((n, n)) * 0.3
    B = csr_from_dense(M)
    bb = rng.standard_normal(n)
    r = orc.gmres(B, bb, restart=n, fmt="fp64", tol=1e-13, maxiter=n, variant="mgs",
                  eta=TINY_ETA)
    assert r["status"] == 0
    assert np.linalg.norm(r["x"] - np.linalg.solve(M, bb)) <= 1e-11 * np.linalg.norm(r["x"])


def test_unknown_variant_bits_are_rejected(orc):
    import ctypes as C
    import oracle as O
    A = P.poisson2d(4)
    b = np.ones(A.n)
    x = np.zeros(A.n)
    opts = O._Opts(10, 0, 1e-10, 10, 0.0, 0, None, 0, 0, 0, 32, 0)
    res = O._Result()
    rc = O.lib().orc_gmres(A.n, O._p(A.row_ptr), O._p(A.col_idx), O._p(A.val), O._p(b),
                           O._p(x), C.byref(opts), C.byref(res), None, None, None, None,
                           None, None)
    assert rc == O.E_ARG


def gram_columns(orc, A, V, k):
    """h + u with u = h - G h: the Gram-form second pass, from the decoded
    stored vectors V (rows) alone."""
    cols = []
    for j in range(k - 1):
        Vj = V[:j + 1]
        w = orc.spmv(A, V[j])
        h = Vj @ w
        G = Vj @ Vj.T
        u = h - G @ h
        w2 = w - Vj.T @ h - Vj.T @ u
        cols.append(np.concatenate([h + u, [np.linalg.norm(w2)]]))
    return cols


@pytest.mark.parametrize("fmt", ["fp16", "int16", "e4m3"])
def test_gram_columns_are_h_plus_h_minus_gh(orc, fmt):
    A = P.convdiff7(9)
    b = P.rhs_uniform(A.n, 3)
    kw = dict(restart=16, fmt=fmt, tol=0.0, maxiter=16, debug=True)
    rg = orc.gmres(A, b, variant=("gram", "spmv_vhat", "always_reorth"), **kw)
    re = orc.gmres(A, b, variant=("spmv_vhat", "always_reorth"), **kw)
    assert rg["reorths"] == rg["iterations"] == 16
    worst = 0.0
    for j, h in enumerate(gram_columns(orc, A, rg["V"], rg["steps"])):
        worst = max(worst, np.max(np.abs(rg["H"][:j + 2, j] - h)) / np.linalg.norm(h))
    assert worst <= 1e-12
    # the explicit re-dot reaches the same columns to rounding, by other bits
    k = rg["steps"]
    assert np.allclose(rg["H"][:, :k - 1], re["H"][:, :k - 1], rtol=0,
                       atol=1e-12 * np.abs(re["H"]).max())
    assert not np.array_equal(rg["H"], re["H"])


def test_gram_keeps_the_fp64_basis_orthogonal_to_a_cancellation_bound(orc):
    """h - G h cancels: its FP64 error is about u64 ||h||, against a result
    of size t = h_{j+1,j}, so the second pass leaves a component of relative
    size u64 omega / t along the basis (the explicit re-dot measures it
    instead).  On this near-identity matrix omega / t is about 20: the Gram
    form keeps the basis orthogonal to 1e-13, the explicit re-dot to 1e-14."""
    n = 120
    rng = np.random.default_rng(0)
    A = csr_from_dense(np.eye(n) + 0.05 * rng.standard_normal((n, n)) / np.sqrt(n))
    b = rng.standard_normal(n)
    kw = dict(restart=40, fmt="fp64", tol=0.0, maxiter=40, debug=True)
    rg = orc.gmres(A, b, variant=("gram", "always_reorth"), **kw)
    re = orc.gmres(A, b, variant="always_reorth", **kw)
    assert rg["reorths"] == 40
    k = rg["V"].shape[0]
    lg = np.linalg.norm(np.eye(k) - rg["V"] @ rg["V"].T)
    le = np.linalg.norm(np.eye(k) - re["V"] @ re["V"].T)
    assert lg <= 1e-13 and le <= 1e-14


@pytest.mark.parametrize("fmt", ["fp64", "fp16", "bf16"])
def test_gram_solves_like_the_explicit_re_dot(orc, fmt):
    A = P.lognormal27(8, 1)
    b = P.rhs_uniform(A.n, 1)
    kw = dict(restart=25, fmt=fmt, tol=1e-10, maxiter=5000)
    rg = orc.gmres(A, b, variant="gram", **kw)
    re = orc.gmres(A, b, **kw)
    assert rg["status"] == re["status"] == 0
    assert abs(rg["iterations"] - re["iterations"]) <= 0.02 * re["iterations"] + 1
    assert np.allclose(rg["hist"][:10], re["hist"][:10], rtol=1e-10, atol=0)


def test_gram_with_mgs_is_rejected(orc):
    A = P.poisson2d(4)
    r = orc.gmres(A, np.ones(A.n), restart=5, variant=("gram", "mgs"))
    assert r["status"] == -1


# One-pass CGS2: u = h - G h and t1^2 = omega^2 - h^T h - h^T u known before
# any update, so the step-7 decision comes first and one update applies
# h + u (or h).  Pins: the columns against numpy, the decisions and counts
# against the two-pass Gram form, the textbook breakdowns against Fig. 1.

@pytest.mark.parametrize("fmt", ["fp16", "int16", "e4m3"])
def test_onepass_columns_are_h_plus_u_with_one_update(orc, fmt):
    A = P.convdiff7(9)
    b = P.rhs_uniform(A.n, 3)
    kw = dict(restart=16, fmt=fmt, tol=0.0, maxiter=16, debug=True)
    r = orc.gmres(A, b, variant=("gram", "onepass", "spmv_vhat", "always_reorth"), **kw)
    assert r["reorths"] == r["iterations"] == 16
    worst = 0.0
    for j, h in enumerate(gram_columns(orc, A, r["V"], r["steps"])):
        worst = max(worst, np.max(np.abs(r["H"][:j + 2, j] - h)) / np.linalg.norm(h))
    assert worst <= 1e-12


@pytest.mark.parametrize("fmt", ["fp64", "fp16", "bf16", "int16"])
@pytest.mark.parametrize("system", ["convdiff7", "lognormal27"])
def test_onepass_decides_like_the_two_pass_gram_form(orc, fmt, system):
    A = P.convdiff7(10) if system == "convdiff7" else P.lognormal27(8, 1)
    b = P.rhs_uniform(A.n, 2)
    kw = dict(restart=25, fmt=fmt, tol=1e-10, maxiter=5000)
    r1 = orc.gmres(A, b, variant=("gram", "onepass"), **kw)
    r2 = orc.gmres(A, b, variant="gram", **kw)
    assert r1["status"] == r2["status"] == 0
    # counts to within the spread that 1e-15 perturbations of b give either
    # form (int16 on convdiff7(10): 66 to 71 steps over twelve of them)
    assert abs(r1["iterations"] - r2["iterations"]) <= 0.08 * r2["iterations"] + 1
    assert abs(r1["reorths"] - r2["reorths"]) <= 0.08 * r2["reorths"] + 1
    assert np.allclose(r1["hist"][:10], r2["hist"][:10], rtol=1e-10, atol=0)


@pytest.mark.parametrize("fmt", ["fp64", "fp16"])
def test_onepass_textbook_breakdowns(orc, fmt):
    """A = I breaks down after one step; a diagonal with five distinct
    eigenvalues after five (fp64): the same counts and breakdowns as Fig. 1."""
    cases = [(np.eye(50), np.random.default_rng(0).standard_normal(50)),
             (np.diag(np.tile([1.0, 2, 3, 4, 5], 10)), np.ones(50))]
    for M, b in cases:
        A = csr_from_dense(M)
        kw = dict(restart=20, fmt=fmt, tol=1e-12, maxiter=40)
        r1 = orc.gmres(A, b, variant=("gram", "onepass"), **kw)
        r0 = orc.gmres(A, b, **kw)
        assert r1["status"] == r0["status"] == 0
        assert (r1["iterations"], r1["breakdowns"]) == (r0["iterations"], r0["breakdowns"])
        assert r1["breakdowns"] >= 1


def test_onepass_sees_the_exhausted_krylov_space(orc):
    """A = Q diag(d) Q^T with k distinct eigenvalues (random orthogonal Q):
    the Krylov space has dimension k, so w of step k lies in span(V_k) and
    h_{k+1,k} = 0 in exact arithmetic; after rounding, the one-pass form's
    floored t1 must still report the breakdown at step k, with x the
    solution.  (Fig. 1's two-pass form, read as in step 12, goes on with a
    rounding-level vector here; its stop test ends it at step k instead.)"""
    for seed in range(24):
        rng = np.random.default_rng(seed)
        n, k = 24, 3 + seed % 4
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        d = np.repeat(np.arange(1.0, k + 1), -(-n // k))[:n]
        M = Q @ np.diag(d) @ Q.T
        b = rng.standard_normal(n)
        A = csr_from_dense(M)
        r = orc.gmres(A, b, restart=20, fmt="fp64", tol=1e-30, maxiter=k,
                      variant=("gram", "onepass"))
        assert (r["iterations"], r["breakdowns"]) == (k, 1), seed
        xs = np.linalg.solve(M, b)
        assert np.linalg.norm(r["x"] - xs) <= 1e-10 * np.linalg.norm(xs), seed
        r0 = orc.gmres(A, b, restart=20, fmt="fp64", tol=1e-12, maxiter=40)
        assert r0["status"] == 0 and r0["iterations"] == k, seed


def test_onepass_needs_the_gram_form(orc):
    A = P.poisson2d(4)
    assert orc.gmres(A, np.ones(A.n), restart=5, variant="onepass")["status"] == -1
