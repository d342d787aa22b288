"""Mutation check of the oracle's pins.

Each case below plants one plausible mistake in a copy of oracle/oracle.c (a
dropped term, a wrong sign, a wrong index or a transposed operand, in the
codecs, the SpMV and dot, the Arnoldi step of Fig. 1, the Givens update and
back substitution of step 17, and the preconditioners), builds the copy with
gcc, and runs the oracle's own pin tests against it in a child process (the
oracle package loads the copy named by CBG_ORACLE_LIB).  The pins compare the
oracle with what the paper and the mathematics fix (closed forms, brute
force, numpy/scipy/torch routines, invariants), so every planted mistake must
make at least one of them fail; the unmodified source must pass them all.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")
PIN_TESTS = ["test_oracle_basics.py", "test_oracle_codec.py", "test_oracle_solver.py",
             "test_oracle_ablations.py", "test_oracle_block_jacobi.py", "test_oracle_spai.py"]

# (name, the pin file expected to catch it, what the mistake is, text in
# oracle.c, text it is replaced with).  The expected file runs first and the
# others after it, so a mutant that file misses is still looked for.
MUTANTS = [
    # storage formats (Sections 4 and 5.2)
    ("round_truncates", "codec", "rounding to p bits truncates instead of ties-to-even",
     "double q = rint(ldexp(x, p - 1 - e));", "double q = trunc(ldexp(x, p - 1 - e));"),
    ("no_subnormal_quantum", "codec", "the subnormal range keeps p significant bits",
     "    if (e < emin)\n        e = emin;", "    if (e < emin - 64)\n        e = emin;"),
    ("bf16_emin", "codec", "bfloat16's smallest normal exponent off by one",
     "BF16 = {8, 8, -126,", "BF16 = {8, 8, -125,"),
    ("e4m3_scale_binade", "codec", "e4m3's scale leaves the largest entry one binade low",
     "k = ilogb(vinf) - 8;", "k = ilogb(vinf) - 7;"),
    ("e4m3_decode_unscaled", "codec", "e4m3 decode drops the vector's scale",
     "out[i] = tab_e4m3[((const uint8_t *)q)[i0 + i]] * s;",
     "out[i] = tab_e4m3[((const uint8_t *)q)[i0 + i]];"),
    ("fixed_point_truncates", "codec", "fixed-point codes truncate instead of rounding",
     "rint(v[i] / sigma)", "trunc(v[i] / sigma)"),
    ("fixed_point_scale", "codec", "fixed-point scale divides by max_int + 1",
     "double sigma = vinf / M;", "double sigma = vinf / (M + 1.0);"),
    ("fp16s_scale_binade", "ablations", "scaled float16 leaves the largest entry one binade low",
     "k = ilogb(vinf) - 15;", "k = ilogb(vinf) - 14;"),
    # SpMV and dot
    ("spmv_row_operand", "basics", "SpMV multiplies by x at the row instead of the column",
     "s += val[p] * x[ci[p]];", "s += val[p] * x[i];"),
    ("spmv_drops_last", "basics", "SpMV drops each row's last entry",
     "for (int32_t p = rp[i]; p < rp[i + 1]; ++p)\n            s += val[p] * x[ci[p]];",
     "for (int32_t p = rp[i]; p < rp[i + 1] - 1; ++p)\n            s += val[p] * x[ci[p]];"),
    ("dot_ragged_tail", "basics", "dot drops the last entry of a ragged tail",
     "int64_t i1 = (b + 1) * BLK < n ? (b + 1) * BLK : n;",
     "int64_t i1 = (b + 1) * BLK < n ? (b + 1) * BLK : n - 1;"),
    ("dot_operand", "basics", "dot squares x instead of pairing x with y",
     "s += x[i] * y[i];", "s += x[i] * x[i];"),
    # Fig. 1 steps 5-14
    ("multidot_offset", "solver", "multi-dot pairs a block of V with the wrong block of w",
     "s += buf[i - i0] * w[i];", "s += buf[i - i0] * w[i - i0];"),
    ("combine_reversed", "solver", "V c applies the coefficients in reverse",
     "acc[i - i0] += c[k] * buf[i - i0];", "acc[i - i0] += c[j - 1 - k] * buf[i - i0];"),
    ("cgs_adds", "solver", "step 5 adds V h instead of subtracting it",
     "                multidot(fmt, j, Q, sc, n, w, h, part);\n"
     "                basis_combine(fmt, j, Q, sc, n, h, s);\n"
     "#pragma omp parallel for schedule(static)\n"
     "                for (int32_t i = 0; i < n; ++i)\n"
     "                    w[i] = w[i] - s[i];",
     "                multidot(fmt, j, Q, sc, n, w, h, part);\n"
     "                basis_combine(fmt, j, Q, sc, n, h, s);\n"
     "#pragma omp parallel for schedule(static)\n"
     "                for (int32_t i = 0; i < n; ++i)\n"
     "                    w[i] = w[i] + s[i];"),
    ("reorth_not_accumulated", "ablations", "step 10 does not add the second pass to h",
     "                for (int32_t k = 0; k < j; ++k)\n"
     "                    h[k] = h[k] + u[k];\n"
     "                double t2",
     "                for (int32_t k = 0; k < j; ++k)\n"
     "                    h[k] = h[k] + 0.0 * u[k];\n"
     "                double t2"),
    ("gram_sign", "ablations", "the Gram form takes h + G h for the second pass",
     "                            u[k] = h[k] - gh;", "                            u[k] = h[k] + gh;"),
    ("gram_row_unmirrored", "ablations", "the Gram row is stored in one triangle only",
     "                for (int32_t k = 0; k < j; ++k)\n"
     "                    G[(size_t)jc * (m + 1) + k] = G[(size_t)k * (m + 1) + jc] = grow[k];\n"
     "            }\n            /* Step 6 */",
     "                for (int32_t k = 0; k < j; ++k)\n"
     "                    G[(size_t)jc * (m + 1) + k] = grow[k];\n"
     "            }\n            /* Step 6 */"),
    ("onepass_pythagoras_sign", "ablations", "the one-pass norm adds h^T u instead of subtracting it",
     "const double t1sq = omega * omega - hh - hu;", "const double t1sq = omega * omega - hh + hu;"),
    ("subdiag_is_omega", "solver", "h_{j+1,j} takes ||w|| before orthogonalisation",
     "    HH(j, jc) = t;", "    HH(j, jc) = omega;"),
    ("v1_unnormalised", "solver", "the first basis vector is r, not r / beta",
     "            v[i] = r[i] / rho;", "            v[i] = r[i];"),
    ("vnext_unnormalised", "solver", "steps 13-14 store w without dividing by h_{j+1,j}",
     "                v[i] = w[i] / t;", "                v[i] = w[i];"),
    # step 17: Givens rotations and back substitution
    ("givens_apply_sign", "solver", "applying a previous rotation loses the sign of s",
     "HH(i + 1, jc) = -sn[i] * a0 + cs[i] * a1;", "HH(i + 1, jc) = sn[i] * a0 + cs[i] * a1;"),
    ("givens_skips_last", "solver", "the newest previous rotation is not applied",
     "for (int32_t i = 0; i < jc; ++i) {\n                double a0",
     "for (int32_t i = 0; i + 1 < jc; ++i) {\n                double a0"),
    ("givens_g_sign", "solver", "the rotated right-hand side loses the sign of s",
     "g[j] = -sn[jc] * g[jc];", "g[j] = sn[jc] * g[jc];"),
    ("givens_swapped", "solver", "cos and sin of the new rotation swapped",
     "cs[jc] = a / rr;\n                    sn[jc] = bb / rr;",
     "cs[jc] = bb / rr;\n                    sn[jc] = a / rr;"),
    ("backsolve_transposed", "solver", "back substitution reads R transposed",
     "acc -= HH(i, k) * y[k];", "acc -= HH(k, i) * y[k];"),
    ("update_without_precond", "solver", "step 17 adds V y without M^{-1}",
     "            x[i] = x[i] + z[i];\n        cycle += 1;",
     "            x[i] = x[i] + s[i];\n        cycle += 1;"),
    ("residual_sign", "solver", "step 1 forms b + A x",
     "            r[i] = b[i] - r[i];\n        double rho", "            r[i] = b[i] + r[i];\n        double rho"),
    ("stop_test_absolute", "solver", "the stop test drops the ||b|| reference",
     "if (rho <= tau * nb) {", "if (rho <= tau) {"),
    # preconditioners
    ("jacobi_multiplies_by_aii", "solver", "Jacobi multiplies by a_ii",
     "z[i] = M->dinv[i] * v[i];", "z[i] = v[i] / M->dinv[i];"),
    ("stencil_without_dinv", "spai", "the stored form leaves out diag(1/a_ii)",
     "z[i] = M->dinv[i] * s;", "z[i] = s;"),
    ("fallback_keeps_nonfinite_x", "solver", "the non-finite fallback keeps the broken iterate",
     "memcpy(x, xprev, (size_t)n * sizeof(double));\n                M.kind = ORC_PC_NONE;",
     "M.kind = ORC_PC_NONE;"),
    ("stencil_slot_order", "spai", "the stencil's slots run x-major instead of z-major",
     "const int p = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1);",
     "const int p = 9 * (dx + 1) + 3 * (dy + 1) + (dz + 1);"),
    ("stencil_centre", "spai", "the stencil's identity sits on the wrong slot",
     "(p == 13 ? 1.0 : 0.0)", "(p == 12 ? 1.0 : 0.0)"),
    ("gj_transposed_factor", "block_jacobi", "Gauss-Jordan takes the eliminator from the pivot row",
     "const double f = D[i * bs + c];", "const double f = D[c * bs + i];"),
    ("bj_fp16_unit", "block_jacobi", "block-Jacobi's fp16 rule uses fp32's unit roundoff",
     "kappa * ldexp(1.0, -11) <= 0.01", "kappa * ldexp(1.0, -24) <= 0.01"),
    ("norm1_by_rows", "block_jacobi", "kappa_1 sums rows instead of columns",
     "s = s + fabs(M[i * bs + k]);", "s = s + fabs(M[k * bs + i]);"),
    ("stagnation_late", "solver", "the stagnation fallback waits for a third flat cycle",
     "if (stagnant >= 2) {", "if (stagnant >= 3) {"),
    ("eta_half", "solver", "the re-orthogonalisation threshold is 1/2, not 1/sqrt(2)",
     "#define ETA_DEFAULT 0.70710678118654752440", "#define ETA_DEFAULT 0.5"),
    ("breakdown_only_exact", "solver", "step 12 ends a cycle only on an exact zero",
     "brk = (t2 == 0.0) || (t2 < eta * t);", "brk = (t2 == 0.0);"),
    ("spmv_vhat_first_column", "ablations", "the stored-vector SpMV reads the first column",
     "orc_decode(fmt, n, Q[jc], sc[jc], v);", "orc_decode(fmt, n, Q[0], sc[0], v);"),
    ("onepass_criterion_inverted", "ablations", "the one-pass step re-orthogonalises when t1 is large",
     "const int ro = always_reorth || t1 < eta * omega;",
     "const int ro = always_reorth || t1 > eta * omega;"),
    ("onepass_no_floor", "ablations", "the one-pass norm has no rounding floor",
     "const double floor2 = 4.0 * (j + 1) * 0x1p-53 * omega * omega;",
     "const double floor2 = 0.0;"),
    ("sparse_pc_row_operand", "solver", "the sparse P multiplies by v at the row",
     "s += (double)val[p] * x[ci[p]];", "s += (double)val[p] * x[i];"),
    ("bj_apply_operand", "block_jacobi", "block-Jacobi pairs the block row with the block's first v",
     "s = s + row[l] * v[i0 + l];", "s = s + row[l] * v[i0];"),
    ("gj_smallest_pivot", "block_jacobi", "Gauss-Jordan pivots on the smallest entry",
     "if (fabs(D[i * bs + c]) > best) {", "if (fabs(D[i * bs + c]) < best) {"),
    ("e4m3_scale_edge", "codec", "e4m3's scale steps up when the top entry is exactly 448",
     "if (ldexp(vinf, -k) > 448.0)", "if (ldexp(vinf, -k) >= 448.0)"),
    ("fp16s_scale_edge", "ablations", "scaled float16 steps up when the top entry is exactly 65504",
     "if (ldexp(vinf, -k) > 65504.0)", "if (ldexp(vinf, -k) >= 65504.0)"),
    ("mgs_adds", "ablations", "the MGS pass adds h_k v_k",
     "w[i] = w[i] - hk * buf[i];", "w[i] = w[i] + hk * buf[i];"),
    ("history_lags", "solver", "the residual history records the previous step's estimate",
     "hist[it - 1] = last_rec;", "hist[it - 1] = fabs(g[jc]) / nb;"),
    ("cycle_length_short", "solver", "a cycle's length is reported one short",
     "cycle_len[cycle] = meff;", "cycle_len[cycle] = meff - 1;"),
    ("cycle_residual_unscaled", "solver", "the restart residual is reported without 1/||b||",
     "cycle_res[cycle] = rho / nb;", "cycle_res[cycle] = rho;"),
    ("true_residual_unscaled", "solver", "the true residual is reported without 1/||b||",
     "res->true_rel_res = sqrt(orc_dot(n, r, r)) / nb;",
     "res->true_rel_res = sqrt(orc_dot(n, r, r));"),
    ("bj_block_row", "block_jacobi", "block-Jacobi applies row i of the block with the wrong stride",
     "(size_t)(i - i0) * bs;", "(size_t)(i - i0);"),
]

# The learned preconditioner's oracle (oracle/spai.py, an extension of the
# paper: features, network, loss and gradients, Adam), checked the same way
# against tests/test_oracle_spai.py: (name, what the mistake is, text in
# spai.py, text it is replaced with).
SPAI_SRC = os.path.join(ROOT, "oracle", "spai.py")
SPAI_MUTANTS = [
    ("slot_axes_swapped", "slots run x-major instead of z-major",
     "(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)", "(dx + 1) * 9 + (dy + 1) * 3 + (dz + 1)"),
    ("row_y_unwrapped", "a row's y coordinate is not taken modulo ny",
     "xr, yr, zr = rows % nx, (rows // nx) % ny,", "xr, yr, zr = rows % nx, (rows // nx),"),
    ("coef_by_column_diagonal", "a coefficient feature divides by the column's a_jj",
     "fl32(A.val[good] / d[rows[good]])", "fl32(A.val[good] / d[A.col_idx[good]])"),
    ("neighbour_ratio_inverted", "the neighbour-diagonal feature is inverted",
     "fl32(d[A.col_idx[good]] / d[rows[good]])", "fl32(d[rows[good]] / d[A.col_idx[good]])"),
    ("dominance_sign", "the dominance feature adds the off-diagonal sum",
     "F[:, 27] = fl32((d - s) / d)", "F[:, 27] = fl32((d + s) / d)"),
    ("no_first_relu", "the first hidden layer has no ReLU",
     "H1 = r(np.maximum(F @ W1 + b1, 0.0))", "H1 = r(F @ W1 + b1)"),
    ("drops_b2", "the second layer drops its bias",
     "H2 = r(np.maximum(H1 @ W2 + b2, 0.0))", "H2 = r(np.maximum(H1 @ W2, 0.0))"),
    ("p_minus_o", "P takes delta - O",
     "val = (delta + np.where(slots >= 0, o, 0.0)) / d[rows]",
     "val = (delta - np.where(slots >= 0, o, 0.0)) / d[rows]"),
    ("p_times_aii", "P multiplies by a_ii",
     "val = (delta + np.where(slots >= 0, o, 0.0)) / d[rows]",
     "val = (delta + np.where(slots >= 0, o, 0.0)) * d[rows]"),
    ("codes_by_column", "a stored code goes to the column's row",
     "codes[slots[good], rows[good]] = o16", "codes[slots[good], A.col_idx[good]] = o16"),
    ("loss_scale", "the loss divides by K n instead of K",
     "L = float(np.sum(R * R)) / K", "L = float(np.sum(R * R)) / (K * A.n)"),
    ("grad_factor", "dL/dP loses the factor 2",
     "G = (2.0 / K) * (At @ R)", "G = (1.0 / K) * (At @ R)"),
    ("grad_p_transposed", "dP pairs G's column with v's row",
     'np.einsum("ek,ek->e", G[rows], V.T[A.col_idx])',
     'np.einsum("ek,ek->e", G[A.col_idx], V.T[rows])'),
    ("grad_o_times_aii", "dL/dO multiplies by a_ii",
     "dO[rows[good], slots[good]] = dP[good] / d[rows[good]]",
     "dO[rows[good], slots[good]] = dP[good] * d[rows[good]]"),
    ("dw2_wrong_layer", "dW2 takes H2 in place of H1",
     "dW2 = H1.T @ dH2", "dW2 = H2.T @ dH2"),
    ("relu_mask_wrong_layer", "dH2 is masked by H1's ReLU",
     "dH2 = r((dO @ W3.T) * (H2 > 0))", "dH2 = r((dO @ W3.T) * (H1 > 0))"),
    ("w2_not_transposed", "dH1 multiplies by W2 instead of its transpose",
     "dH1 = r((dH2 @ W2.T) * (H1 > 0))", "dH1 = r((dH2 @ W2) * (H1 > 0))"),
    ("adam_second_moment_linear", "Adam's second moment accumulates g, not g^2",
     "v[...] = fl32(beta2 * v + (1 - beta2) * g * g)", "v[...] = fl32(beta2 * v + (1 - beta2) * g)"),
    ("weights_not_bf16", "the weights the network sees are not rounded to bfloat16",
     '(bf16(v) if k.startswith("W") else v)', "v"),
    ("dominance_signed", "the dominance feature sums signed off-diagonals",
     "off = np.where(A.col_idx == rows, 0.0, np.abs(A.val))",
     "off = np.where(A.col_idx == rows, 0.0, A.val)"),
    ("drops_b3", "the output layer drops its bias",
     "O = H2 @ W3 + b3", "O = H2 @ W3"),
    ("adam_no_bias_correction", "Adam drops the first moment's bias correction",
     "mh = m / (1 - beta1 ** t)", "mh = m"),
    ("adam_no_sqrt", "Adam divides by v instead of sqrt(v)",
     "lr * mh / (np.sqrt(vh) + eps)", "lr * mh / (vh + eps)"),
]

_SPAI_CHILD = """
import importlib.util, sys
sys.path.insert(0, sys.argv[1])
import oracle
spec = importlib.util.spec_from_file_location("oracle.spai", sys.argv[2])
mod = importlib.util.module_from_spec(spec)
sys.modules["oracle.spai"] = mod
spec.loader.exec_module(mod)
oracle.spai = mod
import pytest
sys.exit(pytest.main(["-x", "-q", "-p", "no:cacheprovider", sys.argv[3]]))
"""


def _build(src_text, out):
    c = out + ".c"
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc", "-O1", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                    "-fno-fast-math", "-I", os.path.join(ROOT, "oracle"), c, "-o", out, "-lm"],
                   check=True, capture_output=True, text=True)


def _run_pins(lib, first=None, timeout=240):
    # passive OpenMP waits: several children share the host's cores
    env = dict(os.environ, CBG_ORACLE_LIB=lib, OMP_NUM_THREADS="2", OMP_WAIT_POLICY="PASSIVE")
    files = PIN_TESTS if first is None else \
        [f"test_oracle_{first}.py"] + [t for t in PIN_TESTS if t != f"test_oracle_{first}.py"]
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
           *[os.path.join(ROOT, "tests", t) for t in files]]
    try:
        r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True,
                           timeout=timeout)
    except subprocess.TimeoutExpired:
        return None, "timed out"
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("FAILED") or "error" in ln]
    return r.returncode, (lines[0] if lines else r.stdout.strip().splitlines()[-1:])


def test_mutant_table_applies_once():
    src = open(SRC).read()
    names = [m[0] for m in MUTANTS]
    assert len(set(names)) == len(names)
    for name, first, _, old, new in MUTANTS:
        assert src.count(old) == 1, name
        assert old != new, name
        assert f"test_oracle_{first}.py" in PIN_TESTS, name


@pytest.mark.slow
def test_every_planted_mistake_fails_a_pin(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    src = open(SRC).read()
    jobs = [("unmodified", None, src)] + [(n, f, src.replace(old, new))
                                          for n, f, _, old, new in MUTANTS]

    def one(job):
        name, first, text = job
        lib = str(tmp_path / f"lib_{name}.so")
        _build(text, lib)
        return name, _run_pins(lib, first)

    with ThreadPoolExecutor(max_workers=4) as ex:
        results = dict(ex.map(one, jobs))
    rc, msg = results.pop("unmodified")
    assert rc == 0, f"the unmodified oracle fails its pins: {msg}"
    survivors = {n: msg for n, (rc, msg) in results.items() if rc == 0}
    assert not survivors, f"planted mistakes no pin catches: {survivors}"


def _run_spai_pins(path, timeout=240):
    env = dict(os.environ, OMP_NUM_THREADS="2", OMP_WAIT_POLICY="PASSIVE")
    cmd = [sys.executable, "-c", _SPAI_CHILD, ROOT, path,
           os.path.join(ROOT, "tests", "test_oracle_spai.py")]
    try:
        r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True,
                           timeout=timeout)
    except subprocess.TimeoutExpired:
        return None, "timed out"
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("FAILED") or "rror" in ln]
    return r.returncode, (lines[0] if lines else r.stdout.strip().splitlines()[-1:])


def test_spai_mutant_table_applies_once():
    src = open(SPAI_SRC).read()
    names = [m[0] for m in SPAI_MUTANTS]
    assert len(set(names)) == len(names)
    for name, _, old, new in SPAI_MUTANTS:
        assert src.count(old) == 1, name
        assert old != new, name


@pytest.mark.slow
def test_every_planted_mistake_in_the_network_oracle_fails_a_pin(tmp_path):
    src = open(SPAI_SRC).read()
    jobs = [("unmodified", src)] + [(n, src.replace(old, new)) for n, _, old, new in SPAI_MUTANTS]

    def one(job):
        name, text = job
        path = str(tmp_path / f"spai_{name}.py")
        with open(path, "w") as f:
            f.write(text)
        return name, _run_spai_pins(path)

    with ThreadPoolExecutor(max_workers=4) as ex:
        results = dict(ex.map(one, jobs))
    rc, msg = results.pop("unmodified")
    assert rc == 0, f"the unmodified network oracle fails its pins: {msg}"
    survivors = {n: msg for n, (rc, msg) in results.items() if rc == 0}
    assert not survivors, f"planted mistakes no pin catches: {survivors}"
