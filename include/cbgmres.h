/*
 * cbgmres.h -- C ABI of the MI355X (gfx950) compressed-basis GMRES library.
 *
 * Solves A x = b (A sparse n x n in CSR form, b and x dense; the problem of
 * the paper's Eq. (1)) with the restarted GMRES of Fig. 1 (Section 3), whose
 * Krylov basis V is stored in a reduced format and widened to FP64 in
 * registers on every read (Section 4, "CB-GMRES"; Section 5.2, "Memory
 * accessor").  All arithmetic is FP64.
 *
 * Conventions for every entry point:
 *  - Pointers marked [dev] are device pointers (HIP global memory) owned by
 *    the caller; [host] pointers are host memory owned by the caller.  The
 *    library never calls hipMalloc/hipFree: scratch space comes from a
 *    caller-provided device workspace sized by the matching *_bytes query.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Kernel-level calls are asynchronous on that stream; cbgmres_solve
 *    returns after the solve has finished.
 *  - Vectors handed to kernel-level calls must be 16-byte aligned; basis
 *    leading dimensions must be multiples of 16 elements.
 *  - Return value: 0 on success, >0 "finished without meeting the
 *    tolerance", <0 an error (cbg_strerror).  Argument errors are detected
 *    on the host before any HIP call, and then no output is written.
 *  - Calls sharing a workspace must not overlap; distinct workspaces may be
 *    used concurrently on distinct streams.
 */
#ifndef CBGMRES_H
#define CBGMRES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Storage format of the Krylov basis (Section 5.2 lists float64, float32,
 * float16, int32 and int16; bf16, fp8 e4m3 and the scaled float16 are
 * extensions stored the same way).  Bytes per entry: 8, 4, 2, 2, 1, 4, 2, 2.
 *   CBG_FP32/FP16/BF16: one round-to-nearest-even conversion from FP64.
 *   CBG_E4M3 (OCP E4M3FN): per-vector power-of-two scale 2^k chosen so that
 *     max|v| * 2^-k lies in (224, 448]; entries RNE(v_i * 2^-k).
 *   CBG_FP16S: float16 with a per-vector power-of-two scale 2^k chosen so
 *     that max|v| * 2^-k lies in (32752, 65504]; entries RNE(v_i * 2^-k), so
 *     entries far below the largest keep float16's relative precision.
 *   CBG_INT32/INT16: fixed point with per-vector scale
 *     sigma = max|v| / max_int (the scale of Section 5.2 for a unit vector);
 *     entries rint(v_i / sigma) clamped to [-max_int, max_int]. */
typedef enum {
    CBG_FP64 = 0, CBG_FP32 = 1, CBG_FP16 = 2, CBG_BF16 = 3,
    CBG_E4M3 = 4, CBG_INT32 = 5, CBG_INT16 = 6, CBG_FP16S = 7
} cbg_format;

/* Right preconditioner M^{-1} of Fig. 1 steps 3 and 17. */
typedef enum {
    CBG_PC_NONE = 0,     /* M = I */
    CBG_PC_JACOBI = 1,   /* M^{-1} = diag(1 / a_ii), the paper's default (Section 6) */
    CBG_PC_SPARSE = 2,   /* M^{-1} = P, single-precision values on A's pattern */
    CBG_PC_BLOCK_JACOBI = 3, /* M^{-1} = blockdiag(D_b^{-1}), adaptive-precision storage
                               (cbg_block_jacobi_setup; Section 6 discusses block-Jacobi) */
    CBG_PC_STENCIL = 4   /* M^{-1} = D^{-1} (I + O) on a grid's 27-point stencil, O in
                            float16 (the learned preconditioner's stored form, see
                            cbg_learned_build_stencil) */
} cbg_precond_kind;

enum {
    CBG_OK = 0,
    CBG_NOT_CONVERGED = 1,   /* maxiter reached before ||b - A x|| <= tol ||b|| */
    CBG_E_ARG = -1,          /* invalid argument (nothing was launched) */
    CBG_E_WORKSPACE = -2,    /* workspace missing, misaligned or too small */
    CBG_E_HIP = -3,          /* a HIP runtime call failed */
    CBG_E_NONFINITE = -4,    /* NaN/Inf met (b, x0, A, or during the solve) */
    CBG_E_UNSUPPORTED = -5   /* valid request the library does not support */
};

/* CSR matrix, 0-based, column indices sorted within each row.
 * row_ptr [dev] n+1 int32; col_idx [dev] nnz int32; val [dev] nnz double.
 *
 * Optional sliced-ELL copy of the same matrix (SELL-64; built by
 * cbg_sell_ptr + cbg_sell_fill), used by the SpMV with A (Fig. 1 steps 1, 3
 * and 18) when sell_ptr, sell_col and sell_val are all non-NULL; NULL
 * selects the CSR kernels.  Rows are grouped in slices of CBG_SELL_SLICE = 64
 * consecutive rows; slice s stores width_s entries per row, width_s the
 * longest row of the slice, column-major: entry k of row 64 s + r (k-th
 * nonzero in CSR order) sits at sell_ptr[s] + 64 k + r.  Entries beyond a
 * row's length, and the rows >= n of the last slice, hold value 0 and
 * column min(row, n - 1).  sell_ptr [dev] (n + 63) / 64 + 1 int64 (offsets,
 * sell_ptr[0] = 0); sell_col [dev] int32 and sell_val [dev] double, each
 * sell_entries = sell_ptr[last] long.  Each row's products are summed in
 * CSR order with separately rounded products and sums, so y = A x equals
 * the row-sequential CSR sum bit for bit (for finite x; a padding entry
 * multiplies x at the row's own index by 0).  The CSR arrays stay required:
 * the preconditioner set-ups and the sparse-P products read them.
 *
 * Diagonal-index columns (cbg_sell_diag): when A has at most
 * CBG_SELL_MAX_DIAG distinct offsets col - row (banded and stencil
 * matrices), sell_dix [dev] (sell_entries uint8) holds per entry the index
 * of its offset in sell_diag [dev] (sell_ndiag int32, sorted ascending,
 * 0 included), so a column is row + sell_diag[sell_dix[e]] (padding
 * entries: offset 0) and the SpMV reads 9 instead of 12 bytes per entry.
 * With sell_dix, sell_diag and sell_ndiag set, sell_col may be NULL. */
typedef struct {
    int32_t n;
    int32_t reserved;
    int64_t nnz;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const double *val;
    const int64_t *sell_ptr;
    const int32_t *sell_col;
    const double *sell_val;
    int64_t sell_entries;
    const uint8_t *sell_dix;
    const int32_t *sell_diag;
    int32_t sell_ndiag;
    int32_t reserved2;
} cbg_csr;

#define CBG_SELL_MAX_DIAG 256

#define CBG_SELL_SLICE 64

/* Solver options.  restart: m of Fig. 1 (1 .. CBG_MAX_RESTART).  tol: tau of
 * the stop test ||b - A x||_2 <= tau ||b||_2 (Section 3).  maxiter: limit on
 * Arnoldi steps over all cycles.  eta: re-orthogonalisation threshold of
 * Fig. 1 step 7; <= 0 selects 1/sqrt(2).  p_val [dev]: CBG_PC_SPARSE values
 * (nnz floats on A's pattern).  fallback: with CBG_PC_SPARSE or CBG_PC_STENCIL, drop M and
 * continue with M = I when the explicit residual fails to fall below 0.99x
 * its previous value in two consecutive cycles or a non-finite value
 * appears.  flags: CBG_FLAG_* bits.  A singular diagonal block with
 * CBG_PC_BLOCK_JACOBI (or a zero diagonal with CBG_PC_JACOBI) returns
 * CBG_E_ARG. */
typedef struct {
    int32_t restart;
    int32_t format;
    double tol;
    int64_t maxiter;
    double eta;
    int32_t precond;
    int32_t fallback;
    const float *p_val;
    int32_t flags;
    int32_t reserved;
    int32_t pc_block;    /* CBG_PC_BLOCK_JACOBI: block size 1..8 (0 selects 4) */
    int32_t pc_prec;     /* CBG_PC_BLOCK_JACOBI: lowest storage precision of the
                            inverted blocks, 16, 32 or 64 bits (0 selects 16) */
    const uint16_t *p_stencil; /* CBG_PC_STENCIL [dev]: 27 x cbg_basis_ld(n) float16
                            codes, slot-major (see cbg_learned_build_stencil) */
    int32_t grid[3];     /* CBG_PC_STENCIL: nx, ny, nz with nx ny nz = n */
    int32_t reserved2;
} cbg_opts;

#define CBG_MAX_RESTART 512
/* time the orthogonalisation kernels with HIP events (cbg_result.prof_*) */
#define CBG_FLAG_PROFILE 1
/* with CBG_FLAG_EXPLICIT_REDOT: run the update of step 5 and the re-dot of
 * step 8 as two basis passes (otherwise they share one pass while j fits
 * the fused kernel's register tile; the arithmetic is the same, the
 * summation order of u differs); no effect on the default form */
#define CBG_FLAG_NO_FUSE 2
/* time only the multi-dot launches with HIP events (cbg_result.prof_dot_*;
 * one event pair per step instead of one per basis-streaming launch) */
#define CBG_FLAG_PROFILE_DOT 4
/* Ablations of the Arnoldi step (numerical studies; off by default).
 * SPMV_VHAT: step 3 multiplies by the stored vector read back, dec(v^_j),
 * instead of the FP64 v_j that step 13 formed (the solver's default, which
 * takes the accessor to serve steps 5, 8, 13-14 and 17 only).
 * ALWAYS_REORTH: re-orthogonalise on every step (CGS2) instead of only when
 * step 7's test h_{j+1,j} < eta * omega fires; the breakdown test is
 * unchanged. */
#define CBG_FLAG_SPMV_VHAT 8
#define CBG_FLAG_ALWAYS_REORTH 16
/* MGS: modified Gram-Schmidt for steps 5 and 8 -- for k = 1..j in order,
 * h_k = dec(v^_k)^T w, then w -= h_k dec(v^_k); one kernel launch and one
 * fold per stored vector and pass (slow by design: the ablation measures
 * what the sequential projections buy).  Not combinable with the PROFILE
 * flags (CBG_E_UNSUPPORTED). */
#define CBG_FLAG_MGS 32
/* Where steps 13-14 of the previous step run (same bits either way):
 * NORMALISE_PASS: a pass of their own (v_j = w / t written once, stored
 * through the accessor, and with Jacobi multiplied by D^-1 there), then
 * step 3's SpMV reads the result;
 * NORMALISE_GATHER: inside step 3's SpMV, which divides each gathered
 * entry by t (one division per nonzero instead of per row) and with Jacobi
 * reads D^-1 per nonzero.
 * Neither bit: the pass when the mean row length exceeds 12 nonzeros or the
 * preconditioner is Jacobi, the gather otherwise.  Both bits: argument
 * error.  SPMV_VHAT and the block-Jacobi preconditioner always take their
 * own paths. */
#define CBG_FLAG_NORMALISE_PASS 64
#define CBG_FLAG_NORMALISE_GATHER 128
/* Steps 5-10 (CGS with the conditional second pass).  By default:
 * the step-5 multi-dot h = V^T w also forms the newest row of G = V^T V,
 * the Gram matrix of the decoded stored vectors; then u = h - G h (step 8's
 * re-dot, since V^T (w - V h) = h - G h) and t1^2 = ||w - V h||^2 =
 * omega^2 - h^T h - h^T u (step 6, by Pythagoras) are known before any
 * update, so step 7 decides first and one update w -= V (h + u) (or V h)
 * does steps 5 and 9.  A re-orthogonalised step reads the basis twice (the
 * multi-dot and the update) instead of four times.  Both identities are
 * exact; in FP64 they cancel, leaving components of relative size about
 * 2^-53 omega / t1 along the basis where the explicit passes leave 2^-53.
 * So a step whose t1^2 falls below 10^-4 omega^2 (t1 < omega / 100: a
 * near-breakdown, as on clustered spectra) takes Fig. 1's explicit form
 * instead: w1 = w - V h, t1 = ||w1||, u = V^T w1 (in the same basis pass),
 * then w1 -= V u and its norm; cbg_result.explicit_steps counts them.  The
 * loss of orthogonality of an FP64 basis then stays near 10^2 2^-53, and
 * step 12 always compares the final norm with a t1 that was summed, not
 * cancelled.
 * EXPLICIT_REDOT: the form Fig. 1 writes: update, norm, and a second
 * multi-dot of the updated w (fused with the update while j fits the fused
 * kernel's register tile; NO_FUSE splits it), then the second update.
 * TWO_PASS: the Gram-form re-dot with the update of step 5, the norm of
 * step 6 and the second update as separate passes.  With EXPLICIT_REDOT or
 * MGS: argument error.  MGS takes its own path. */
#define CBG_FLAG_EXPLICIT_REDOT 256
#define CBG_FLAG_TWO_PASS 512
/* time the Arnoldi steps' SpMV with A (w = A M^-1 v, Fig. 1 step 3) with HIP
 * events at each launch's own start and end (cbg_result.prof_spmv_*) */
#define CBG_FLAG_PROFILE_SPMV 1024
/* with the PROFILE flags: time the launches of every 8th Arnoldi step only
 * (steps counted over the whole solve, across cycles, the ones that found
 * their cycle finished included).  An event pair delays the launch it
 * brackets by a few microseconds; sampling cuts that cost eightfold, and
 * the prof_* sums then cover the sampled launches. */
#define CBG_FLAG_PROFILE_SAMPLED 2048
#define CBG_PROFILE_STRIDE 8
#define CBG_FLAG_ALL 4095   /* any other bit is an argument error */

typedef struct {
    int64_t iterations;        /* Arnoldi steps (SpMVs with A inside cycles) */
    int64_t restarts;          /* cycles run */
    int64_t reorths;           /* steps that re-orthogonalised (Fig. 1 step 7) */
    int32_t status;            /* same value as returned */
    int32_t breakdowns;        /* cycles ended by the breakdown test (step 12) */
    int32_t fell_back;         /* 1 if CBG_PC_SPARSE was dropped */
    int32_t reserved;
    double true_rel_res;       /* ||b - A x||_2 / ||b||_2 of the returned x */
    double recurrence_rel_res; /* last |g_{j+1}| / ||b||_2 of the least squares */
    double seconds;            /* host wall time of the call */
    double model_bytes;        /* algorithmic HBM bytes of the solve */
    /* with CBG_FLAG_PROFILE: summed event-timed duration, algorithmic bytes
     * and launch count of the basis-streaming kernels of the Arnoldi steps
     * (multi-dot h = V^T w; update w -= V h fused with the re-dot, or the
     * update and the re-dot as two passes; the re-orthogonalising update).
     * Every launch is counted, also the ones that found their step skipped
     * (no re-orthogonalisation, or the cycle already finished); those add
     * time but no bytes.  The events are recorded at each kernel's own start
     * and end (hipExtLaunchKernelGGL). */
    double prof_orth_ms;
    double prof_orth_bytes;
    int64_t prof_orth_launches;
    double prof_dot_ms;        /* the multi-dot kernel alone (every multi-dot launch) */
    double prof_dot_bytes;
    int64_t prof_dot_launches;
    double prof_fused_ms;      /* the fused update + re-dot kernel alone (explicit form) */
    double prof_fused_bytes;
    int64_t prof_fused_launches;
    int64_t explicit_steps;    /* default form: steps that took Fig. 1's explicit form
                                  because t1 < omega / 100 (see CBG_FLAG_TWO_PASS) */
    double prof_spmv_ms;       /* with CBG_FLAG_PROFILE_SPMV: the steps' SpMV with A */
    double prof_spmv_bytes;
    int64_t prof_spmv_launches;
} cbg_result;

/* Device workspace bytes cbgmres_solve needs for this problem shape
 * (0 for invalid arguments).  The workspace must be 256-byte aligned.
 * For CBG_PC_BLOCK_JACOBI it is sized for any block size up to 8. */
size_t cbg_workspace_bytes(int32_t n, int32_t restart, int32_t format, int32_t precond);

/* Restarted CB-GMRES (Fig. 1 of the paper).
 * A [host struct, dev arrays]; b [dev] n doubles; x [dev] n doubles, x0 on
 * entry, the solution on exit.  workspace [dev] ws_bytes >=
 * cbg_workspace_bytes(...).  res [host] always filled (also on error).
 * hist [host, optional] receives the recurrence residual |g_{j+1}|/||b|| of
 * every Arnoldi step, up to hist_len entries.
 * The residual is recomputed explicitly at every restart (Section 3) and
 * whenever the recurrence residual signals convergence (Section 6.2: the
 * solve continues from the explicit residual if it misses tol).
 * If ||b|| = 0 the solution is x = 0.  The host synchronises with the
 * stream once per restart cycle. */
int cbgmres_solve(const cbg_csr *A, const double *b, double *x, const cbg_opts *opt,
                  void *workspace, size_t ws_bytes, void *stream, cbg_result *res,
                  double *hist, int64_t hist_len);

/* Where a cbgmres_solve workspace of this shape keeps the Krylov basis:
 * after a solve, basis vector k (0-based) of the last cycle is stored at
 * byte workspace + basis_offset + k * cbg_basis_ld(n) * bytes(format) in
 * the chosen format (FP64 values for CBG_FP64), with its scale (double) at
 * workspace + scales_offset + 8k, for k below that cycle's step count (the
 * vector formed after a cycle's last step is not stored).  A solve that
 * stops on maxiter leaves the basis of its last cycle in place.  Returns
 * CBG_OK or CBG_E_ARG. */
int cbg_workspace_basis(int32_t n, int32_t restart, int32_t format, int32_t precond,
                        size_t *basis_offset, size_t *scales_offset);

/* Static description of a status code. */
const char *cbg_strerror(int status);

/* After a call returned CBG_E_HIP: the hipError_t of the HIP runtime call
 * that failed (0 if none has failed on this host thread), the source line
 * of the library where it was made (line, optional) and the runtime's name
 * for the error (name, optional; a static string). */
int cbg_last_hip_error(int *line, const char **name);

/* Padded leading dimension (elements) the solver uses for basis vectors of
 * length n: a multiple of 256.  Kernel-level calls accept any ld >= n that
 * is a multiple of 16. */
int64_t cbg_basis_ld(int32_t n);

/* Device workspace bytes the kernel-level reductions below need for
 * vectors of length n and up to j basis vectors. */
size_t cbg_kernel_workspace_bytes(int32_t n, int32_t j);

/* ---------------- kernel-level entry points (asynchronous) -------------- */

/* The accessor's store (Fig. 1 steps 13-14): q = enc_F(v), scale = the
 * per-vector scale (1 for unscaled formats).  v [dev] n doubles; q [dev]
 * n entries of the format; scale [dev] 1 double; ws [dev]. */
int cbg_encode(int32_t format, const double *v, int32_t n, void *q, double *scale,
               void *ws, size_t ws_bytes, void *stream);

/* The accessor's load (steps 5, 8, 17): v = dec_F(q) * scale, exactly. */
int cbg_decode(int32_t format, const void *q, const double *scale, int32_t n, double *v,
               void *stream);

/* Sliced-ELL copy of A (see cbg_csr), first half: sell_ptr [dev]
 * (n + 63) / 64 + 1 int64 receives the slice offsets and *entries [host] the
 * total number of entries (sell_ptr's last value; the call synchronises the
 * stream).  Reads A's CSR arrays only.  The caller sizes sell_col and
 * sell_val from *entries (entries / nnz - 1 is the padding; the caller may
 * keep the CSR kernels when it is large). */
int cbg_sell_ptr(const cbg_csr *A, int64_t *sell_ptr, int64_t *entries, void *stream);

/* Second half: fills sell_col [dev] and sell_val [dev] (entries long, from
 * cbg_sell_ptr) from A's CSR arrays and sell_ptr. */
int cbg_sell_fill(const cbg_csr *A, const int64_t *sell_ptr, int32_t *sell_col,
                  double *sell_val, void *stream);

/* Diagonal-index columns of the sliced-ELL copy (see cbg_csr): from A's
 * sell_ptr and sell_col, finds the distinct offsets col - row of the rows
 * < n (padding counts as offset 0).  With at most CBG_SELL_MAX_DIAG of them,
 * writes them sorted to sell_diag [dev] (CBG_SELL_MAX_DIAG int32), the
 * per-entry indices to sell_dix [dev] (sell_entries uint8) and their count
 * to *ndiag [host], and returns CBG_OK; with more, writes only *ndiag (the
 * count, or more than CBG_SELL_MAX_DIAG when the search stopped early) and
 * returns CBG_E_UNSUPPORTED.  ws: cbg_kernel_workspace_bytes(n, 0) bytes.
 * Synchronises the stream. */
int cbg_sell_diag(const cbg_csr *A, int32_t *sell_diag, uint8_t *sell_dix, int32_t *ndiag,
                  void *ws, size_t ws_bytes, void *stream);

/* y = A x (step 3); if norm2 [dev, nullable] is given, *norm2 = ||y||_2
 * (step 4).  x [dev] n doubles, y [dev] n doubles.  With A's sliced-ELL
 * copy present, y equals the row-sequential CSR sum bit for bit. */
int cbg_spmv(const cbg_csr *A, const double *x, double *y, double *norm2, void *ws,
             size_t ws_bytes, void *stream);

/* Multi-dot of step 5 through the accessor: h_k = sum_i dec(V_k)_i w_i for
 * k < j.  V [dev] j vectors of ld entries (vector k at byte offset
 * k*ld*bytes(format)); scales [dev] j doubles; w [dev] n doubles;
 * h [dev] j doubles. */
int cbg_multidot(int32_t format, const void *V, int64_t ld, const double *scales,
                 int32_t n, int32_t j, const double *w, double *h, void *ws,
                 size_t ws_bytes, void *stream);

/* cbg_multidot for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and results, with the block partials in a fixed array of this
 * library on each GPU (CBG_NOALLOC_MAX_J + 4 rows of 4096 doubles, about
 * 4.3 MB per GPU, held until the process ends, located once per device)
 * instead of a workspace argument.  Allocates nothing and records no memset.
 * j > CBG_NOALLOC_MAX_J returns CBG_E_UNSUPPORTED before any HIP call.  All
 * calls on one GPU share its array: calls that overlap in time on one GPU
 * (different streams, or host threads without ordering) race and must not
 * be issued. */
#define CBG_NOALLOC_MAX_J 128
int cbg_multidot_noalloc(int32_t format, const void *V, int64_t ld, const double *scales,
                         int32_t n, int32_t j, const double *w, double *h, void *stream);

/* Update of step 5: w -= sum_k h_k dec(V_k), then norms[0] = ||w||_2 and
 * norms[1] = ||w||_inf (Section 5.2: both norms in one pass).
 * norms [dev, nullable] 2 doubles. */
int cbg_update(int32_t format, const void *V, int64_t ld, const double *scales, int32_t n,
               int32_t j, const double *h, double *w, double *norms, void *ws,
               size_t ws_bytes, void *stream);


/* Steps 5-8 in one basis pass: w -= sum_k h_k dec(V_k), then
 * u_k = sum_i dec(V_k)_i w_i (the re-dot of step 8) for k < j, norms[0] =
 * ||w||_2 and norms[1] = ||w||_inf of the updated w.  While j fits the
 * kernel's register tile (j <= 104 for fp64, fp32, fp16, int32; 80 for
 * int16; 48 for bf16; e4m3 never) each lane keeps the bytes it loaded of
 * every stored vector and the basis is read once; beyond it, the same
 * arithmetic runs as an update and a multi-dot.  u [dev] j
 * doubles; norms [dev] 2 doubles; other arguments as cbg_update. */
int cbg_update_redot(int32_t format, const void *V, int64_t ld, const double *scales, int32_t n,
                     int32_t j, const double *h, double *w, double *u, double *norms, void *ws,
                     size_t ws_bytes, void *stream);

/* ---------------- block-Jacobi preconditioner ------------------------- */
/* An extension: the paper's Section 6 discusses block-Jacobi
 * preconditioners, and its references store the inverted blocks at a
 * precision chosen per block; the rule here is this project's own.  Block b
 * covers rows and columns [b*bs, min((b+1)*bs, n)); D_b is A restricted to
 * it, inverted by Gauss-Jordan elimination with partial pivoting in FP64
 * (first row with the largest |entry| as pivot; no fused operations).  With
 * kappa_b = ||D_b||_1 ||D_b^-1||_1, the inverse is stored in the lowest of
 * fp16 (u = 2^-11) and fp32 (u = 2^-24), not below prec_min bits, with
 * kappa_b u <= 1/100 and the block's largest entry in the format's normal
 * range, else in fp64 (round to nearest even).
 * tags [dev] ceil(n/bs) int8: 16, 32 or 64 per block; x64/x32/x16 [dev]
 * ceil(n/bs)*bs*bs entries each: block b's inverse at b*bs*bs, row-major,
 * row stride bs, zeros beyond the block, in the array of its precision.
 * Synchronises; CBG_E_ARG for a singular block (or bad arguments). */
int cbg_block_jacobi_setup(const cbg_csr *A, int32_t bs, int32_t prec_min, int8_t *tags,
                           double *x64, float *x32, uint16_t *x16, void *ws, size_t ws_bytes,
                           void *stream);

/* z = M^-1 v (n doubles each [dev]) with the blocks of cbg_block_jacobi_setup. */
int cbg_block_jacobi_apply(int32_t n, int32_t bs, const int8_t *tags, const double *x64,
                           const float *x32, const uint16_t *x16, const double *v, double *z,
                           void *stream);

/* ---------------- learned sparse approximate inverse ------------------- */
/* An extension of the paper (which uses scalar Jacobi, Section 6): a per-row
 * network proposes the values of a right preconditioner P on A's pattern, for
 * matrices on an nx*ny*nz grid (x fastest, row = x + nx*(y + ny*z), n =
 * nx*ny*nz) whose pattern lies within the 27-point stencil.
 *
 * Slots: entry (i, c) has slot p = (dz+1)*9 + (dy+1)*3 + (dx+1), the grid
 * offset from row i to column c; slot 13 is the diagonal; entries outside the
 * 27-point stencil have no slot.
 * Features (n x 64 bf16, row-major): f_p = bf16(fl32(a_ic / a_ii)) and
 * f_{32+p} = bf16(fl32(a_cc / a_ii)) (the neighbour's diagonal) for the row's
 * slots p (column c), f_27 = bf16(fl32((a_ii - sum_{c != i} |a_ic|) / a_ii))
 * with the sum in CSR order, all else 0.
 * Network: H1 = bf16(ReLU(F W1 + b1)), H2 = bf16(ReLU(H1 W2 + b2)),
 * O = H2 W3 + b3 (32 outputs, slots 0..26 used); bf16 weights, fp32 biases,
 * fp32 accumulation on the matrix cores.
 * P: P_ic = fl32((delta_{p,13} + O_ip) / a_ii) on A's pattern (0 where the
 * entry has no slot); W3 = 0 and b3 = 0 give P = D^-1 (Jacobi).
 * Loss over K unit vectors v_k: L = scale * sum_k ||A P v_k - v_k||_2^2.
 *
 * Parameters: `params` [dev] CBG_SPAI_NPARAM fp32 masters in the order W1
 * (64x64, row-major: [in][out]), b1 (64), W2 (64x64), b2 (64), W3 (64x32),
 * b3 (32); `weights` [dev] CBG_SPAI_NWEIGHT bf16 (uint16 bit patterns) of W1,
 * W2, W3 in the same layout.  Vectors for the loss: `V` [dev] n x K fp16 bit
 * patterns, row-major (entry (i, k) at i*K + k), K <= CBG_SPAI_MAX_K.
 * All [dev] arrays 16-byte aligned; workspaces 256-byte aligned and sized by
 * cbg_spai_workspace_bytes(n, nnz, K) (K = 0 where no vectors are used). */
#define CBG_SPAI_NFEAT 64
#define CBG_SPAI_NHID 64
#define CBG_SPAI_NOUT 32
#define CBG_SPAI_NPARAM 10400
#define CBG_SPAI_NWEIGHT 10240
#define CBG_SPAI_MAX_K 32

size_t cbg_spai_workspace_bytes(int32_t n, int64_t nnz, int32_t K);

/* Features of every row (see above).  grid [host] {nx, ny, nz}; feat [dev]
 * n x 64 bf16.  Synchronises with the stream; returns CBG_E_NONFINITE if a
 * row has a zero (or missing) diagonal or a non-finite feature.  This call,
 * cbg_learned_build, cbg_learned_build_stencil and cbg_stencil_apply read
 * A's sliced-ELL copy when A carries one with diagonal indices (sell_ptr,
 * sell_val, sell_dix, sell_diag), else the CSR arrays; the results are the
 * same bit for bit. */
int cbg_spai_features(const cbg_csr *A, const int32_t grid[3], uint16_t *feat, void *ws,
                      size_t ws_bytes, void *stream);

/* Network forward pass on n feature rows.  out [dev] n x 32 fp32; h1, h2
 * [dev, nullable together] n x 64 bf16 activations kept for the backward
 * pass. */
int cbg_mlp_forward(int32_t n, const uint16_t *feat, const uint16_t *weights, const float *params,
                    float *out, uint16_t *h1, uint16_t *h2, void *stream);

/* P values on A's pattern from the network output.  out [dev] n x 32 fp32;
 * p_val [dev] nnz fp32 (the CBG_PC_SPARSE values of cbg_opts). */
int cbg_spai_assemble(const cbg_csr *A, const int32_t grid[3], const float *out, float *p_val,
                      void *stream);

/* Inference: features, forward pass and assembly of P in one call (once
 * per matrix, before cbgmres_solve with CBG_PC_SPARSE).  Synchronises;
 * CBG_E_NONFINITE as cbg_spai_features. */
int cbg_learned_build(const cbg_csr *A, const int32_t grid[3], const uint16_t *weights,
                      const float *params, float *p_val, void *ws, size_t ws_bytes, void *stream);

/* Stored form of the learned preconditioner for CBG_PC_STENCIL: the network's
 * corrections O_ip of the slots row i stores, each rounded once to float16
 * (round to nearest even from fp32; 0 for slots the row does not store),
 * slot-major: the code of slot p of row i at p_stencil[p * ld + i], ld =
 * cbg_basis_ld(n), rows [n, ld) 0.  The solve applies
 *   z_i = fl(1 / a_ii) * sum_p ([p = 13] + o_ip) v_(grid neighbour p of i)
 * over the slots whose grid point exists: the operator P above up to the
 * float16 rounding of O (instead of P's fp32 rounding), read as 54 bytes per
 * row with no column indices.  All codes 0 (W3 = 0, b3 = 0) is Jacobi.
 * p_stencil [dev] 27 * ld uint16.  Synchronises; CBG_E_NONFINITE as
 * cbg_spai_features. */
int cbg_learned_build_stencil(const cbg_csr *A, const int32_t grid[3], const uint16_t *weights,
                              const float *params, uint16_t *p_stencil, void *ws,
                              size_t ws_bytes, void *stream);

/* z = M^-1 v for CBG_PC_STENCIL (v, z [dev] n doubles; p_stencil as above;
 * ws of cbg_spai_workspace_bytes(n, nnz, 0)).  Synchronises; CBG_E_ARG if a
 * diagonal entry is zero or missing. */
int cbg_stencil_apply(const cbg_csr *A, const int32_t grid[3], const uint16_t *p_stencil,
                      const double *v, double *z, void *ws, size_t ws_bytes, void *stream);

/* Values of A^T on A's pattern: t_val[p] = a_ci for entry p = (i, c).  A
 * must be structurally symmetric; synchronises and returns
 * CBG_E_UNSUPPORTED if some (c, i) is missing. */
int cbg_csr_transpose_values(const cbg_csr *A, double *t_val, void *ws, size_t ws_bytes,
                             void *stream);

/* Training vectors: out (n x K fp16, row-major, one round-to-nearest-even)
 * from the FP64 vectors V + (first + k*stride)*ld, k < K (e.g. a cycle's
 * basis in a cbgmres_solve workspace, see cbg_workspace_basis_offset). */
int cbg_spai_pack(const double *V, int64_t ld, int32_t n, int32_t K, int32_t first,
                  int32_t stride, uint16_t *out, void *stream);

/* Loss and its gradient with respect to P's values: R = A P V - V,
 * *loss (+)= scale * ||R||_F^2, G = 2 scale A^T R, dP_e = sum_k G[i][k]
 * V[c][k] for entry e = (i, c).  t_val [dev] from cbg_csr_transpose_values;
 * p_val [dev] nnz fp32; loss [dev] 1 double; dP [dev] nnz doubles.
 * accumulate = 0 overwrites *loss, 1 adds to it. */
int cbg_spai_grad_p(const cbg_csr *A, const double *t_val, const float *p_val, int32_t K,
                    const uint16_t *V, double scale, double *loss, int32_t accumulate,
                    double *dP, void *ws, size_t ws_bytes, void *stream);

/* dL/dO (n x 32 bf16, one rounding from FP64): dO_ip = dP_e / a_ii for the
 * entry e of slot p in row i, 0 elsewhere. */
int cbg_spai_grad_o(const cbg_csr *A, const int32_t grid[3], const double *dP, uint16_t *dO,
                    void *stream);

/* Network backward pass: grad [dev] CBG_SPAI_NPARAM doubles (+)= dL/dparams
 * (params order) for the activations h1, h2 of cbg_mlp_forward and dL/dO
 * (bf16); dH2 and dH1 are rounded to bf16 before their products. */
int cbg_mlp_backward(int32_t n, const uint16_t *feat, const uint16_t *h1, const uint16_t *h2,
                     const uint16_t *dO, const uint16_t *weights, double *grad,
                     int32_t accumulate, void *ws, size_t ws_bytes, void *stream);

/* One training evaluation on one matrix: forward, assembly, grad_p, grad_o
 * and backward; *loss and grad (+)= the loss and its parameter gradient. */
int cbg_spai_loss_grad(const cbg_csr *A, const double *t_val, const int32_t grid[3],
                       const uint16_t *feat, const uint16_t *weights, const float *params,
                       int32_t K, const uint16_t *V, double scale, double *loss, double *grad,
                       int32_t accumulate, void *ws, size_t ws_bytes, void *stream);

/* weights [dev] = the bf16 rounding (nearest even) of the W1, W2, W3 parts
 * of params [dev]: sets the bf16 copy after the masters are initialised or
 * loaded. */
int cbg_spai_round_weights(const float *params, uint16_t *weights, void *stream);

/* Adam step t >= 1 (Kingma and Ba, 2015, with bias correction) on the fp32
 * masters; m1, m2 [dev] NPARAM fp32 moments (zero before step 1); moments and
 * parameters are formed in FP64 and stored as fp32; weights is refreshed
 * with their bf16 rounding. */
int cbg_adam_step(float *params, float *m1, float *m2, uint16_t *weights, const double *grad,
                  int64_t t, double lr, double beta1, double beta2, double eps, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* CBGMRES_H */
