/*
 * CB-GMRES CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 implementation of compressed-basis GMRES as described in
 * Aliaga, Anzt, Gruetzmacher, Quintana-Orti, Tomas, "Compressed Basis GMRES on
 * High Performance GPUs" (arXiv 2009.12101): the restarted GMRES of Fig. 1
 * (Section 3) whose Krylov basis is stored in a reduced format and widened to
 * FP64 on every read (Section 4, "CB-GMRES"; Section 5.2, "Memory accessor").
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library. It shares no source, header, table or helper with
 * the HIP library; the two meet only through the seeded input generators.
 *
 * All pointers are host pointers owned by the caller. Functions never
 * allocate memory the caller must free.
 */
#ifndef CBG_ORACLE_H
#define CBG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Storage formats of the basis (Section 5.2 lists float64, float32, float16,
 * int32, int16; bf16, e4m3 and the scaled float16 are extensions defined the
 * same way). */
enum {
    ORC_FP64 = 0, ORC_FP32 = 1, ORC_FP16 = 2, ORC_BF16 = 3,
    ORC_E4M3 = 4, ORC_INT32 = 5, ORC_INT16 = 6, ORC_FP16S = 7
};

/* Variants of the Arnoldi step for numerical ablations (bits of
 * orc_opts.variant; 0 is Fig. 1 as written):
 *   ORC_V_SPMV_VHAT     step 3 multiplies by the decoded stored vector
 *                       dec(v^_j) instead of the FP64 v_j;
 *   ORC_V_ALWAYS_REORTH step 7's test is replaced by "always" (CGS2); the
 *                       breakdown test of step 12 is unchanged;
 *   ORC_V_MGS           modified Gram-Schmidt: steps 5 and 8 project out
 *                       one stored vector at a time, h_k = dec(v^_k)^T w
 *                       followed by w -= h_k dec(v^_k), k = 1..j in order;
 *   ORC_V_GRAM          step 8's re-dot u = V^T w' (w' = w - V h after
 *                       step 5) formed from the Gram matrix G = V^T V of the
 *                       decoded stored vectors: u = h - G h, equal in exact
 *                       arithmetic.  Row j of G (dec(v^_k)^T dec(v^_j),
 *                       k <= j) is formed once, at step j.  Not combinable
 *                       with ORC_V_MGS;
 *   ORC_V_ONEPASS       with ORC_V_GRAM: steps 5-10 as one update.  u = h - G h
 *                       and t1^2 = ||w - V h||^2 = omega^2 - h^T h - h^T u
 *                       (Pythagoras, exact) are known before any update, so
 *                       step 7 decides first and w -= V (h + u) (or V h)
 *                       runs once; t1^2 is floored at 4 (j+1) u64 omega^2,
 *                       below which it is rounding alone.
 *                       Step 12's test compares the final norm with t1. */
enum { ORC_V_SPMV_VHAT = 1, ORC_V_ALWAYS_REORTH = 2, ORC_V_MGS = 4, ORC_V_GRAM = 8,
       ORC_V_ONEPASS = 16 };

/* Right preconditioners M^-1 (Fig. 1 step 3; step 17):
 *   ORC_PC_JACOBI       z_i = d_i v_i, d_i = fl(1 / a_ii) (Section 6 uses it);
 *   ORC_PC_SPARSE       z = P v, P with float values on A's pattern;
 *   ORC_PC_BLOCK_JACOBI see orc_block_jacobi;
 *   ORC_PC_STENCIL      the learned preconditioner in its stored form (this
 *                       project's definition): on an nx x ny x nz grid
 *                       (x fastest), row i's 27 stencil slots p = 9(dz+1) +
 *                       3(dy+1) + (dx+1) carry float16 codes o_{p,i}
 *                       (slot-major: code of slot p of row i at p ld + i,
 *                       ld = the row stride given), and
 *                         z_i = d_i * sum_p c_{p,i} v_{i + dz nx ny + dy nx + dx}
 *                       over the slots whose grid point exists, in slot
 *                       order, with c_{p,i} = [p = 13] + dec16(o_{p,i})
 *                       (exact in FP64) and d_i = fl(1 / a_ii).  All codes
 *                       0 gives Jacobi bit for bit. */
enum { ORC_PC_NONE = 0, ORC_PC_JACOBI = 1, ORC_PC_SPARSE = 2, ORC_PC_BLOCK_JACOBI = 3,
       ORC_PC_STENCIL = 4 };

enum { ORC_OK = 0, ORC_NOT_CONVERGED = 1, ORC_E_ARG = -1, ORC_E_NONFINITE = -4 };

/* bytes per stored entry, or 0 for an unknown format */
int orc_format_bytes(int fmt);

/* Encode n entries of v into q (orc_format_bytes(fmt)*n bytes) and the
 * per-vector scale.  Scale meaning: fp64/fp32/fp16/bf16: 1; e4m3: 2^k with
 * max|v| 2^-k in (224, 448]; fp16s: 2^k with max|v| 2^-k in (32752, 65504];
 * int: sigma = max|v| / max_int.  Returns 0, or ORC_E_ARG. */
int orc_encode(int fmt, int64_t n, const double *v, void *q, double *scale);
/* Widen n stored entries to FP64. */
int orc_decode(int fmt, int64_t n, const void *q, double scale, double *out);

/* y = A x for a CSR matrix (row_ptr n+1, 0-based). */
void orc_spmv(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
              const double *val, const double *x, double *y);
/* sum_i x_i y_i in fixed 1024-entry blocks (see the source). */
double orc_dot(int64_t n, const double *x, const double *y);

typedef struct {
    int32_t restart;          /* m of Fig. 1 */
    int32_t format;           /* ORC_FP64 ... ORC_INT16 */
    double  tol;              /* tau: stop when ||b - A x||_2 <= tau ||b||_2 */
    int64_t maxiter;          /* limit on Arnoldi steps over all cycles */
    double  eta;              /* re-orthogonalisation threshold; <= 0 -> 1/sqrt(2) */
    int32_t precond;          /* ORC_PC_* */
    const float *p_val;       /* ORC_PC_SPARSE: values of P on A's pattern */
    int32_t fallback;         /* ORC_PC_SPARSE: switch to M = I on stagnation */
    int32_t pc_block;         /* ORC_PC_BLOCK_JACOBI: block size 1..8 (0: 4) */
    int32_t pc_prec;          /* ORC_PC_BLOCK_JACOBI: lowest storage precision 16, 32
                                 or 64 bits (0: 16) */
    int32_t variant;          /* ORC_V_* bits (0: Fig. 1 as written) */
    int32_t pad;
    const uint16_t *p_stencil; /* ORC_PC_STENCIL: 27 x st_ld float16 codes, slot-major */
    int32_t grid[3];          /* ORC_PC_STENCIL: nx, ny, nz with nx ny nz = n */
    int32_t st_ld;            /* ORC_PC_STENCIL: slot stride (>= n) */
} orc_opts;

typedef struct {
    int64_t iterations;       /* Arnoldi steps taken */
    int64_t restarts;         /* cycles started */
    int64_t reorths;          /* steps that re-orthogonalised */
    int32_t status;           /* ORC_OK / ORC_NOT_CONVERGED / error */
    int32_t breakdowns;       /* cycles ended by the breakdown test */
    int32_t fell_back;        /* 1 if the sparse preconditioner was dropped */
    int32_t pad;
    double  true_rel_res;     /* ||b - A x||_2 / ||b||_2 at exit */
    double  recurrence_rel_res; /* last |g_{j+1}| / ||b||_2 */
} orc_result;

/* Block-Jacobi preconditioner with adaptive-precision storage (this
 * project's definition; the paper's Section 6 discusses block-Jacobi and
 * its references store the inverted blocks at a precision chosen per block).
 * Blocks are the consecutive index ranges [b*bs, min((b+1)*bs, n)); D_b is A
 * restricted to block b.  Each D_b is inverted by Gauss-Jordan elimination
 * with partial pivoting in FP64 (the first row with the largest |entry| is
 * the pivot).  kappa_b = ||D_b||_1 ||D_b^-1||_1.  The inverse is stored in
 * the lowest precision, not below prec_min bits, whose unit roundoff u
 * (2^-11 for fp16, 2^-24 for fp32) gives kappa_b * u <= 1/100 and whose
 * normal range holds the block's largest entry (smaller entries may round
 * to subnormals, with absolute error below u times the largest); otherwise
 * in fp64; entries are rounded to nearest even.  vals [n_blocks*bs*bs]: the stored values (as
 * doubles), block b at b*bs*bs, row-major with row stride bs, zero beyond
 * the block's size; prec [n_blocks]: 16, 32 or 64.  Returns 0, or ORC_E_ARG
 * for invalid arguments or a singular block. */
int orc_block_jacobi(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                     const double *val, int32_t bs, int32_t prec_min, double *vals,
                     int8_t *prec);

/* Restarted CB-GMRES (Fig. 1).  x is x0 on entry and the result on exit.
 * hist (optional, maxiter entries): recurrence residual |g_{j+1}|/||b|| per
 * Arnoldi step.  cycle_res (optional, maxiter+1 entries): explicit residual
 * ||b - A x||/||b|| at the start of every cycle and at exit.  cycle_len
 * (optional, maxiter entries): Arnoldi steps taken in each cycle.
 * dbg_V (optional, n*(restart+1)): decoded basis vectors of the FIRST cycle,
 * vector-major; dbg_H (optional, (restart+1)*restart, column-major): the
 * Hessenberg matrix of the first cycle before any Givens rotation;
 * dbg_steps[0..1] receive that cycle's step count and the number of basis
 * vectors stored.  When dbg_V is given, the vector v_{j+1} after the
 * cycle's last step j is also formed (if h_{j+1,j} > 0) so the Arnoldi
 * relation can be checked; the solution is unaffected. */
int orc_gmres(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
              const double *val, const double *b, double *x,
              const orc_opts *opt, orc_result *res,
              double *hist, double *cycle_res, int32_t *cycle_len,
              double *dbg_V, double *dbg_H, int32_t *dbg_steps);

void orc_set_threads(int nthreads);
int  orc_get_threads(void);

/* z = M^-1 v for ORC_PC_STENCIL alone (the definition above); returns
 * ORC_E_ARG if a diagonal entry is missing or zero or the grid does not
 * number the n rows. */
int orc_stencil_apply(int32_t n, const int32_t *rp, const int32_t *ci, const double *val,
                      const int32_t grid[3], const uint16_t *codes, int64_t st_ld,
                      const double *v, double *z);

#ifdef __cplusplus
}
#endif
#endif
