// Host-side launch interface between the C ABI / solver loop and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cbg {

struct DevState;

// Block-partial scratch carved from a workspace (value-major, see RedArgs).
struct RedWs {
    double *orth;     // multi-dot / update partials: (max j + 2) rows of `stride`
    double *spmv;     // SpMV / norm partials: 2 rows of `sstride`
    int stride;       // >= the grid of every producer of `orth`
    int sstride;      // >= the grid of every producer of `spmv`
};

struct SpmvArgs {
    int n;
    int64_t ldy;          // rows written (>= n; [n, ldy) written as 0)
    const int32_t *rp, *ci;
    const double *val;
    const float *fval;
    const double *x, *dinv, *b;
    double *y;
    RedWs ws;
    int mode;             // SP_* of the kernels (8 | base: Arnoldi-step variant)
    int role;             // SR_*: 0 none, 1 step (partials, skipped when done), 2 free
    int sg;               // launch shape (SPMV_*, from spmv_shape_of)
    const DevState *st;
    void *Q;              // step variants: basis slot receiving enc(x / t)
    const double *qscale; // step variants: that slot's scale
    int fmt;              // step variants: storage format
    hipEvent_t ev0, ev1;  // optional: recorded at the kernel's own start and end
    // optional sliced-ELL copy of A (used when sp is set and the mode allows)
    const int64_t *sp;
    const int32_t *sc;
    const double *sv;
    const uint8_t *sd;    // diagonal-index columns (with sdiag, ndiag), or null
    const int32_t *sdiag;
    int ndiag;
    int64_t nslice;
    int sell_nt;          // stream values and columns past the caches (long rows)
};

struct OrthArgs {
    int fmt;
    const void *V;
    int64_t ld;
    const double *scales;
    int n, j;
    const double *w;      // multi-dot input
    int gated;            // multi-dot: skipped once the cycle is done
    int with_norms;       // multi-dot: also partials of ||w||^2 and max|w_i|
    int gram;             // multi-dot: also the newest Gram row, dec(V_k)^T dec(V_{j-1})
    double *u;            // one-pass update: receives u (Gram form, or a hard step's explicit re-dot)
    DevState *stw;        // one-pass update: the step-7 decision and t1
    const double *G;      // one-pass update: the Gram matrix of the stored basis
    const void *sa;       // one-pass update: the step arrays (H, cs, sn) of the column block
    const double *coef;   // update coefficients
    double *wio;          // update: the vector updated in place (or written)
    const double *dinv;
    int role;             // update U_*
    RedWs ws;
    const DevState *st;
    hipEvent_t ev0, ev1;  // optional: recorded at the kernel's own start and end
};

// reduce roles (k_reduce)
enum { RR_NB = 0, RR_SCALE = 1, RR_NORM2 = 2, RR_RESID = 3, RR_H = 4, RR_U = 5, RR_T2 = 6,
       RR_VALUES = 7, RR_NORMS = 8, RR_MGS_H = 9, RR_MGS_U = 10, RR_MGS_T = 11,
       RR_HG = 12,   // RR_H plus the newest Gram row from the multi-dot's rows j+2+k
       RR_UG = 13,   // step 6-7 from the update's norm partials, u = h - G h
       RR_C2 = 14 }; // close of the one-pass update (rows 0 and 1; a hard step's rows j+2, j+3)

// SpMV launch shapes: rows per block and LDS product-buffer entries
enum { SPMV_R256_C2K = 0, SPMV_R64_C2K = 1, SPMV_R64_C4K = 2, SPMV_R32_C4K = 3,
       SPMV_RP64_C2K = 4 };   // row-parallel gather (k_spmv_rp)
int spmv_shape_of(int n, int64_t nnz);     // from the mean row length
int spmv_rows(int shape);
int spmv_grid(int shape, int64_t ldy);
int orth_grid(int fmt, int64_t n);
int launch_spmv(const SpmvArgs &a, hipStream_t s);
bool sell_takes(int mode);                 // modes the sliced-ELL kernel runs
void launch_sell_ptr(int n, const int32_t *rp, int64_t nslice, int64_t *sp, hipStream_t s);
// 0: done; 1: more distinct offsets than the diagonal-index form holds
// (*count_host tells how many); -1: HIP error.  Reads the count back.
int launch_sell_diag(int n, int64_t nslice, const int64_t *sp, const int32_t *sc, int32_t *diag,
                     uint8_t *sd, void *ws, hipStream_t s, int32_t *count_host);
void launch_sell_fill(int n, const int32_t *rp, const int32_t *ci, const double *val,
                      int64_t nslice, const int64_t *sp, int32_t *sc, double *sv, hipStream_t s);
void launch_multidot(const OrthArgs &a, hipStream_t s);
void launch_update(const OrthArgs &a, hipStream_t s);
// Fused update + re-dot with norms (w -= V coef; partials of V^T w, ||w||^2,
// max|w| as the multi-dot with norms).  Returns the grid size (the number of
// partials per value), or 0 if j is beyond the fused kernel's register tile
// (then nothing is launched).
int launch_update_redot(const OrthArgs &a, hipStream_t s);
// Block-Jacobi: invert the bs x bs diagonal blocks (1 <= bs <= 8) and store
// each in fp16/fp32/fp64 by the precision rule (-1: bs out of range).
int launch_bj_setup(int n, const int32_t *rp, const int32_t *ci, const double *val, int bs,
                    int prec_min, int8_t *tags, double *x64, float *x32, uint16_t *x16,
                    unsigned *bad, hipStream_t s);
// With st: v = w / t stored as basis vector (Q, qscale) for rows < ldq and
// z = M^-1 v (z = M^-1 dec(enc(v)) with quant); without: z (+)= M^-1 w.
void launch_bj_apply(int n, int64_t ldq, int bs, const int8_t *tags, const double *x64,
                     const float *x32, const uint16_t *x16, const double *w, double *z,
                     int accumulate, const DevState *st, void *Q, const double *qscale, int fmt,
                     int quant, hipStream_t s);
int fused_jmax(int fmt);   // largest j launch_update_redot takes
// Records a failing HIP call (error code, library source line) for
// cbg_last_hip_error.
void note_hip_error(hipError_t e, int line);
// One launch of a modified Gram-Schmidt pass over the stored vectors (the
// MGS ablation of steps 5 and 8): w -= coef[k-1] dec(V_{k-1}) for k > 0,
// then partials of dec(V_k)^T w (k < j) or of ||w||^2, max|w| (k = j).
// pass 1 is skipped once the cycle is done, pass 2 also unless the step
// re-orthogonalises.  Returns the grid (the number of partials).
int launch_mgs(int fmt, const void *V, int64_t ld, const double *scales, int n, int k, int j,
               double *w, const double *coef, const RedWs &ws, const DevState *st, int pass,
               hipStream_t s);
// Whether launch_update_redot takes step j for basis vectors of leading
// dimension ld (the one predicate the solver and the launcher share).
bool fused_takes(int fmt, int64_t ld, int j);
void launch_reduce(const RedWs &ws, int role, int nb_orth, int nb_spmv, int j, DevState *st,
                   const void *sa, double *out, int fmt, hipStream_t s);
void launch_normalize(int fmt, const double *w, int n, int64_t nst, double *v_out, void *Q,
                      const double *scale_slot, const double *tptr, double tval,
                      const DevState *st, int check_done, hipStream_t s);
// steps 13-14 as a pass: v = w / t stored through the accessor, z = v, or
// dinv .* v when dinv is given; skipped once the cycle is done
void launch_step_normalize(int fmt, const double *w, int n, int64_t ld, const double *dinv,
                           double *z, void *Q, const double *scale_slot, const DevState *st,
                           hipStream_t s);
void launch_decode(int fmt, const void *Q, int n, const double *scale, double *v, hipStream_t s);
// The stencil preconditioner's stored form (CBG_PC_STENCIL) on ld rows (a
// multiple of 16; w, dinv and z hold ld entries, z in ACC mode n):
// mode 0 (step): z = M^-1 (w / t) and v_j = w / t stored (skipped once the
// cycle is done); 1: z = M^-1 w; 2: z += M^-1 w.
void launch_stencil(int fmt, int mode, const double *w, int n, int64_t ld, const int32_t grid[3],
                    const uint16_t *codes, const double *dinv, double *z, void *Q,
                    const double *scale_slot, const DevState *st, hipStream_t s);
int launch_norm(const double *x, int64_t n, const RedWs &ws, hipStream_t s);
void launch_init_state(DevState *st, int n, int m, int fmt, double tol, double eta,
                       int64_t maxiter, int reorth_all, hipStream_t s);
// dinv = 1 / a_ii for rows < n, 0 for rows in [n, ld): from the sliced-ELL
// copy with diagonal indices when `a` carries one (set_matrix), else from CSR
void launch_jacobi_setup(const SpmvArgs &a, int64_t ld, double *dinv, unsigned *bad,
                         hipStream_t s);
void launch_clear_flags(DevState *st, unsigned *bad, hipStream_t s);
void launch_fill_zero(double *p, int count, hipStream_t s);
void launch_backsolve(const DevState *st, const void *sa, hipStream_t s);
size_t step_arrays_size();
void make_step_arrays(void *out, double *H, double *h, double *u, double *cs, double *sn,
                      double *g, double *y, double *hist, double *scales, int32_t *flags);
// the Gram matrix ((m+1) x (m+1) doubles) for the RR_HG / RR_UG folds
void set_step_gram(void *sa, double *G);

}  // namespace cbg
