// gfx950 kernels of the CB-GMRES hot path and their host launchers.
//
// One Arnoldi step of Fig. 1 (Section 3) runs as
//   spmv       w = A M^-1 v; block partials of ||w||^2           (steps 3-4)
//   multidot   block partials of h = V_j^T w                     (step 5)
//   reduce     h, omega = ||A M^-1 v||
//   update     w -= V_j h                                        (step 5)
//   multidot   block partials of u = V_j^T w, ||w||^2, max|w_i|  (steps 6, 8)
//   reduce     u, h_{j+1,j} = ||w||; re-orthogonalise iff
//              h_{j+1,j} < eta * omega (step 7), else finish the step
//   update     w -= V_j u, partials of ||w||^2, max|w_i|         (steps 8-10)
//   reduce     h += u, h_{j+1,j}; breakdown test; Givens         (steps 11-12, 16-17)
//   normalize  v = w / h_{j+1,j}; V_{j+1} = enc(v)               (steps 13-14)
// The re-dot u = V_j^T w is computed with the norm of w in the same pass;
// it is used only when step 7 asks for it.  Producers write block partials
// with plain stores and a one-block reduce kernel folds them in fixed order,
// so sums are bitwise reproducible and no block fences against another.
// The host only enqueues kernels; it synchronises once per restart cycle.
#include <hip/hip_ext.h>

#include "cbg_device.hpp"
#include "cbg_launch.hpp"

#ifndef CBG_MD_ATTR
#define CBG_MD_ATTR
#endif

namespace cbg {

// ---------------------------------------------------------------------------
// Vector chunk helpers.
// ---------------------------------------------------------------------------

template <int VW>
__device__ __forceinline__ void load_w(const double *__restrict__ w, int64_t n, int64_t i0,
                                       double *o)
{
    if (i0 + VW <= n) {
#pragma unroll
        for (int e = 0; e < VW; e += 2) {
            f64x2 p = *(const f64x2 *)(w + i0 + e);
            o[e] = p.x;
            o[e + 1] = p.y;
        }
    } else {
#pragma unroll
        for (int e = 0; e < VW; ++e)
            o[e] = (i0 + e < n) ? w[i0 + e] : 0.0;
    }
}

template <int VW>
__device__ __forceinline__ void store_w(double *__restrict__ w, int64_t n, int64_t i0,
                                        const double *o)
{
    if (i0 + VW <= n) {
#pragma unroll
        for (int e = 0; e < VW; e += 2) {
            f64x2 p = {o[e], o[e + 1]};
            *(f64x2 *)(w + i0 + e) = p;
        }
    } else {
#pragma unroll
        for (int e = 0; e < VW; ++e)
            if (i0 + e < n)
                w[i0 + e] = o[e];
    }
}

// Decode the chunk of stored vector Vk starting at entry i0 (entries >= n
// read as 0).  A chunk that starts below n lies inside the vector's leading
// dimension (a multiple of 16 >= n), so its 16-byte load is in bounds.
template <int F>
__device__ __forceinline__ void load_dec(const uint8_t *__restrict__ Vk, int64_t i0, int64_t n,
                                         double s, double *d)
{
    using T = Fmt<F>;
    constexpr int VW = T::VW;
    if (i0 < n) {
        u32x4 q = __builtin_nontemporal_load((const u32x4 *)(Vk + i0 * fmt_bytes(F)));
        T::dec(q, s, d);
        if (i0 + VW > n) {
#pragma unroll
            for (int e = 0; e < VW; ++e)
                if (i0 + e >= n)
                    d[e] = 0.0;
        }
    } else {
#pragma unroll
        for (int e = 0; e < VW; ++e)
            d[e] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// Scalar work of a step, done by the last block of a reduction.
// ---------------------------------------------------------------------------

struct StepArrays {
    double *H;         // (m+1) x m, column-major, rotated in place
    double *h, *u;     // m+1
    double *cs, *sn;   // m
    double *g;         // m+2
    double *y;         // m
    double *hist;      // m: recurrence residual of each step of the cycle
    double *scales;    // m+1: per-vector scales of the stored basis
    int32_t *flags;    // m: bit0 re-orthogonalised, bit1 breakdown
    double *G;         // (m+1) x (m+1), row-major: Gram matrix of the stored basis
};

// Step 16's first part: the j-1 stored rotations applied to the new column
// c (c_k, k < j, in LDS).  Rotation i maps the carried entry x to
// -s_i x + c_i c_{i+1} and writes H_i = c_i x + s_i c_{i+1}.  The carries are
// the prefix compositions of these affine maps, formed by a block-wide
// Hillis-Steele scan (log2 j rounds) instead of a serial chain of j-1
// rotations.  Writes rows 0 .. j-2 of the column to Hc and returns the
// carry (row j-1 before the new rotation) to every thread.  pa, pb: LDS
// scratch of 2 x MAX_RESTART doubles each.  Block-uniform call.
__device__ double rotate_column(const double *c, int j, const double *__restrict__ cs,
                                const double *__restrict__ sn, double *__restrict__ Hc,
                                double (*pa)[MAX_RESTART], double (*pb)[MAX_RESTART])
{
    const int tid = threadIdx.x, nth = blockDim.x;
    const int jc = j - 1;
    for (int i = tid; i < jc; i += nth) {
        pa[0][i] = -sn[i];
        pb[0][i] = cs[i] * c[i + 1];
    }
    __syncthreads();
    int cur = 0;
    for (int d = 1; d < jc; d <<= 1) {
        // inclusive scan: map i composed after map i - d
        for (int i = tid; i < jc; i += nth) {
            double A = pa[cur][i], B = pb[cur][i];
            if (i >= d) {
                B = fma(A, pb[cur][i - d], B);
                A = A * pa[cur][i - d];
            }
            pa[cur ^ 1][i] = A;
            pb[cur ^ 1][i] = B;
        }
        __syncthreads();
        cur ^= 1;
    }
    for (int i = tid; i < jc; i += nth) {
        const double x = i == 0 ? c[0] : fma(pa[cur][i - 1], c[0], pb[cur][i - 1]);
        Hc[i] = fma(cs[i], x, sn[i] * c[i + 1]);
    }
    const double carry = jc == 0 ? c[0] : fma(pa[cur][jc - 1], c[0], pb[cur][jc - 1]);
    __syncthreads();
    return carry;
}

// Fig. 1 steps 9-12 and step 16, run by every thread of a one-block kernel.
// Reading of step 12 (the literal test would end every re-orthogonalised
// cycle): breakdown iff h_{j+1,j} = 0, or the second pass again lost more
// than a factor eta.  The new column (h, plus u after a
// re-orthogonalisation) meets the j-1 stored rotations (rotate_column), or,
// with `rotated`, that was done already by the one-pass update's column
// block (rows 0 .. j-2 in H, the carry in the state); thread 0 then forms
// the new rotation and updates g.
__device__ void finish_step(DevState *st, const StepArrays &a, int j, bool reorth, double t2,
                            double wmax2, bool rotated = false)
{
    __shared__ double lh[MAX_RESTART];
    __shared__ double pa[2][MAX_RESTART], pb[2][MAX_RESTART];
    const int tid = threadIdx.x;
    const int jc = j - 1;
    const int m = st->m;
    double *Hc = a.H + (size_t)jc * (m + 1);
    double carry;
    if (rotated) {
        carry = st->carry;
    } else {
        for (int k = tid; k < j; k += blockDim.x)
            lh[k] = reorth ? a.h[k] + a.u[k] : a.h[k];
        __syncthreads();
        carry = rotate_column(lh, j, a.cs, a.sn, Hc, pa, pb);
    }
    if (tid != 0)
        return;
    double t = st->t;
    bool brk;
    if (reorth) {
        brk = (t2 == 0.0) || (t2 < st->eta * t);
        t = t2;
        st->wmax = wmax2;
        st->reorths += 1;
    } else {
        brk = (t == 0.0);
    }
    st->t = t;
    const double rr = sqrt(carry * carry + t * t);
    double c = 1.0, sn = 0.0;
    if (rr > 0.0) {
        c = carry / rr;
        sn = t / rr;
    }
    a.cs[jc] = c;
    a.sn[jc] = sn;
    Hc[jc] = rr;
    Hc[j] = 0.0;
    const double gj = a.g[jc];
    const double gnew = -sn * gj;
    a.g[j] = gnew;
    a.g[jc] = c * gj;
    st->it += 1;
    const double rec = fabs(gnew) / st->nb;
    a.hist[jc] = rec;
    st->last_rec = rec;
    const bool finite = isfinite(st->omega) && isfinite(t) && isfinite(gnew);
    const bool conv = fabs(gnew) <= st->tau_nb;
    if (brk)
        st->breakdowns += 1;
    a.flags[jc] = (reorth ? 1 : 0) | (brk ? 2 : 0) | (st->hard ? 4 : 0);
    st->jeff = j;
    if (!finite)
        st->nonfinite = 1;
    if (brk || conv || st->it >= st->maxiter || !finite || j == m) {
        st->done = 1;
        st->conv = conv ? 1 : 0;
    } else {
        a.scales[j] = make_param(st->fmt, st->wmax / t).scale;
    }
}

// ---------------------------------------------------------------------------
// Utility kernels.
// ---------------------------------------------------------------------------

__global__ void k_init_state(DevState *st, int n, int m, int fmt, double tol, double eta,
                             int64_t maxiter, int reorth_all)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        DevState s{};
        s.n = n;
        s.m = m;
        s.fmt = fmt;
        s.eta = eta;
        s.maxiter = maxiter;
        s.reorth_all = reorth_all;
        s.tau_nb = tol;       // scaled by ||b|| once it is known
        *st = s;
    }
}

// dinv_i = 1 / a_ii (Jacobi), a_ii the row's last diagonal entry in CSR
// order; rows in [n, ld) get 0.  bad != 0 if a diagonal entry is missing,
// zero or not finite.  A half-wave per row reads its indices as one
// contiguous run.
__global__ __launch_bounds__(BLK) void k_jacobi_setup(int n, int64_t ld,
                                                      const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ ci,
                                                      const double *__restrict__ val,
                                                      double *__restrict__ dinv, unsigned *bad)
{
    constexpr int RPB = BLK / 32;                   // rows per block
    const int g = threadIdx.x >> 5, lane = threadIdx.x & 31;
    for (int64_t base = (int64_t)blockIdx.x * RPB; base < ld; base += (int64_t)gridDim.x * RPB) {
        const int64_t i = base + g;
        const bool live = i < n;
        const int beg = live ? rp[i] : 0, end = live ? rp[i + 1] : 0;
        const int ch = (end - beg + 31) / 32;
        const int chunks = max(ch, __shfl_xor(ch, 32));          // uniform over the wave
        const double d = hw_row_diag(i, beg, end, chunks, ci, val);
        if (lane != 0 || i >= ld)
            continue;
        if (!live) {
            dinv[i] = 0.0;
            continue;
        }
        if (d == 0.0 || !isfinite(d))
            atomicOr(bad, 1u);
        dinv[i] = 1.0 / d;
    }
}

constexpr int SELL_MAX_DIAG = 256;  // distinct offsets col - row of the diagonal-index form

// The same from A's sliced-ELL copy with one-byte diagonal indices: a lane
// per row (a wave per 64-row slice) walks the row's CSR-length prefix of the
// copy's index bytes and reads the value of the last entry at offset 0 only.
// Rows in [n, ld) get 0.
__global__ __launch_bounds__(BLK) void k_jacobi_setup_sell(
    int n, int64_t ld, const int32_t *__restrict__ rp, const int64_t *__restrict__ sp,
    const uint8_t *__restrict__ sd, const double *__restrict__ sv,
    const int32_t *__restrict__ sdiag, int ndiag, double *__restrict__ dinv, unsigned *bad)
{
    constexpr int B = 9;
    __shared__ int32_t ldg[SELL_MAX_DIAG];
    for (int t = threadIdx.x; t < ndiag; t += BLK)
        ldg[t] = sdiag[t];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < ld;
         i += (int64_t)gridDim.x * BLK) {
        if (i >= n) {
            dinv[i] = 0.0;
            continue;
        }
        const int64_t sl = i / 64, beg = sp[sl];
        const int width = (int)((sp[sl + 1] - beg) / 64);
        const int len = rp[i + 1] - rp[i];
        int64_t hit = -1;
        for (int k0 = 0; k0 < len; k0 += B) {
            uint32_t dx[B];
#pragma unroll
            for (int u = 0; u < B; ++u)
                dx[u] = sd[beg + (int64_t)min(k0 + u, width - 1) * 64 + (i & 63)];
#pragma unroll
            for (int u = 0; u < B; ++u)
                if (k0 + u < len && ldg[dx[u]] == 0)
                    hit = beg + (int64_t)(k0 + u) * 64 + (i & 63);
        }
        const double d = hit >= 0 ? sv[hit] : 0.0;
        if (d == 0.0 || !isfinite(d))
            atomicOr(bad, 1u);
        dinv[i] = 1.0 / d;
    }
}

// Block partials of ||x||_2^2 and ||x||_inf of a length-n vector (two
// values, in the SpMV partial region).
__global__ __launch_bounds__(BLK) void k_norm(const double *__restrict__ x, int64_t n, RedArgs ra)
{
    double s = 0.0, m = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)BLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLK) {
        double v = x[i];
        s += v * v;
        m = fmax(m, fabs(v));
    }
    block_sum_max(s, m);
    if (threadIdx.x == 0) {
        ra.part[blockIdx.x] = s;
        ra.part[(size_t)ra.stride + blockIdx.x] = m;
    }
}

// ---------------------------------------------------------------------------
// CSR SpMV, CSR-stream style (after Greathouse and Daga, SC'14): a block owns
// RPB consecutive rows.  Phase 1 walks the block's nonzeros with unit stride
// across the threads (coalesced val/col loads, x gathered through the
// caches) and stages the products a_p * x_col(p) in LDS; phase 2 sums each
// row from LDS with 256/RPB threads per row.  A block whose rows hold more
// than CAP nonzeros sums them straight from memory instead.  Rows in
// [n, ldy) are written as 0 (padding of the solver's work vectors).
// ---------------------------------------------------------------------------

enum {
    SP_PLAIN = 0,      // y = A x
    SP_JACOBI = 1,     // y = A (dinv .* x)
    SP_RESID = 2,      // y = b - A x
    SP_FLOATVAL = 3,   // y = P x, P with float values on A's pattern
    SP_ACCUM = 4,      // y += P x (P float values), y of length n
    // Arnoldi-step variants: the input is the previous step's orthogonalised
    // w and t = h_{j+1,j}; the kernel gathers v = w / t (IEEE division, the
    // same bits as Fig. 1 step 13 produces) and stores v's compressed form
    // for its own rows (step 14) while it computes A M^-1 v (step 3)
    SP_STEP_PLAIN = 8 | SP_PLAIN,
    SP_STEP_JACOBI = 8 | SP_JACOBI,
    SP_STEP_FLOATVAL = 8 | SP_FLOATVAL,
    // ablation: the step variants multiply by dec(enc(v)), the stored vector
    // read back, instead of the FP64 v
    SP_QUANT = 16,
    SP_STEP_PLAIN_Q = SP_QUANT | SP_STEP_PLAIN,
    SP_STEP_JACOBI_Q = SP_QUANT | SP_STEP_JACOBI,
    SP_STEP_FLOATVAL_Q = SP_QUANT | SP_STEP_FLOATVAL
};
// roles: SR_NONE no partials (skipped once the cycle is done); SR_STEP
// partials of ||y||^2 and max|y_i| (skipped once done); SR_FREE partials,
// never skipped (explicit residual, kernel-level calls).
enum { SR_NONE = 0, SR_STEP = 1, SR_FREE = 2 };

constexpr bool sp_step(int mode) { return (mode & 8) != 0; }
constexpr bool sp_quant(int mode) { return (mode & SP_QUANT) != 0; }

// Store entry i of a vector through the accessor (one entry; the vector's
// scale parameters in p).
__device__ __forceinline__ void store_entry(int fmt, uint8_t *__restrict__ Q, int64_t i, double v,
                                            EncParam p)
{
    switch (fmt) {
    case F_FP64: ((double *)Q)[i] = v; break;
    case F_FP32: ((float *)Q)[i] = (float)v; break;
    case F_FP16: ((uint16_t *)Q)[i] = (uint16_t)Fmt<F_FP16>::code(v, p); break;
    case F_BF16: ((uint16_t *)Q)[i] = (uint16_t)Fmt<F_BF16>::code(v, p); break;
    case F_E4M3: Q[i] = (uint8_t)Fmt<F_E4M3>::code(v, p); break;
    case F_INT32: ((uint32_t *)Q)[i] = Fmt<F_INT32>::code(v, p); break;
    case F_FP16S: ((uint16_t *)Q)[i] = (uint16_t)Fmt<F_FP16S>::code(v, p); break;
    default: ((uint16_t *)Q)[i] = (uint16_t)Fmt<F_INT16>::code(v, p); break;
    }
}

// dec(enc(v)): the value entry v reads back as once stored with the vector's
// scale parameters p (the SpMV-on-the-stored-vector ablation).
__device__ __forceinline__ double quantize(int fmt, double v, EncParam p)
{
    switch (fmt) {
    case F_FP64: return v;
    case F_FP32: return (double)(float)v;
    case F_FP16: return Fmt<F_FP16>::one(Fmt<F_FP16>::code(v, p), p.scale);
    case F_BF16: return Fmt<F_BF16>::one(Fmt<F_BF16>::code(v, p), p.scale);
    case F_E4M3: return dec_e4m3(Fmt<F_E4M3>::code(v, p)) * p.scale;
    case F_INT32: return p.scale * (double)(int32_t)Fmt<F_INT32>::code(v, p);
    case F_FP16S: return Fmt<F_FP16S>::one(Fmt<F_FP16S>::code(v, p), p.scale);
    default: return Fmt<F_INT16>::one(Fmt<F_INT16>::code(v, p), p.scale);
    }
}

template <int MODE>
__device__ __forceinline__ double spmv_term(int p, const int32_t *__restrict__ ci,
                                            const double *__restrict__ val,
                                            const float *__restrict__ fval,
                                            const double *__restrict__ x,
                                            const double *__restrict__ dinv, double tdiv,
                                            int fmt, EncParam ep)
{
    constexpr int BASE = MODE & 7;
    const int c = ci[p];
    double a;
    if constexpr (BASE == SP_FLOATVAL || BASE == SP_ACCUM)
        a = (double)fval[p];
    else
        a = val[p];
    double xv = x[c];
    if constexpr (sp_step(MODE))
        xv = xv / tdiv;
    if constexpr (sp_quant(MODE))
        xv = quantize(fmt, xv, ep);
    if constexpr (BASE == SP_JACOBI)
        xv = dinv[c] * xv;
    return a * xv;
}

template <int RPB, int CAP, int MODE>
__global__ __launch_bounds__(BLK) void k_spmv(int n, int64_t ldy, const int32_t *__restrict__ rp,
                                              const int32_t *__restrict__ ci,
                                              const double *__restrict__ val,
                                              const float *__restrict__ fval,
                                              const double *__restrict__ x,
                                              const double *__restrict__ dinv,
                                              const double *__restrict__ b,
                                              double *__restrict__ y, RedArgs ra, int role,
                                              const DevState *st, uint8_t *__restrict__ Q,
                                              const double *__restrict__ qscale, int fmt)
{
    if (st && role != SR_FREE && st->done)
        return;
    double tdiv = 1.0;
    EncParam ep{1.0, 0};
    if constexpr (sp_step(MODE)) {
        tdiv = st->t;
        ep = param_from_scale(fmt, *qscale);
    }
    constexpr int TPR = BLK / RPB;          // threads per row in the sum phase
    // products per thread per batch: eight on the short-row shape (one batch
    // covers the block's 256 rows of a 7-point matrix: 36.1 against 38.1 us
    // at 128^3), four on the long-row shapes (27-point rows: 165 against 167)
    constexpr int UNR = RPB >= 256 ? 8 : 4;
    __shared__ double prod[CAP];
    __shared__ int lrp[RPB + 1];
    const int tid = threadIdx.x;
    double ssq = 0.0, mx = 0.0;
    const int64_t nblk = (ldy + RPB - 1) / RPB;
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const int64_t r0 = blk * RPB;
        const int nr = r0 < n ? (int)min((int64_t)RPB, (int64_t)n - r0) : 0;   // rows with entries
        __syncthreads();                    // LDS reuse across iterations
        for (int t = tid; t <= nr && nr > 0; t += BLK)
            lrp[t] = rp[r0 + t];
        __syncthreads();
        const int p0 = nr > 0 ? lrp[0] : 0;
        const int cnt = nr > 0 ? lrp[nr] - p0 : 0;
        const bool staged = cnt <= CAP;
        if (staged && cnt > 0) {
            for (int q = tid; q < cnt; q += BLK * UNR) {
                double v[UNR];
#pragma unroll
                for (int u = 0; u < UNR; ++u) {
                    const int qq = min(q + u * BLK, cnt - 1);      // clamped: loads stay in bounds
                    v[u] = spmv_term<MODE>(p0 + qq, ci, val, fval, x, dinv, tdiv, fmt, ep);
                }
#pragma unroll
                for (int u = 0; u < UNR; ++u)
                    if (q + u * BLK < cnt)
                        prod[q + u * BLK] = v[u];
            }
        }
        __syncthreads();
        const int lr = tid / TPR, part = tid % TPR;
        const int64_t row = r0 + lr;
        double s = 0.0;
        if (lr < nr) {
            const int a0 = lrp[lr] - p0, a1 = lrp[lr + 1] - p0;
            if (staged) {
                for (int q = a0 + part; q < a1; q += TPR)
                    s += prod[q];
            } else {
                for (int q = a0 + part; q < a1; q += TPR)
                    s += spmv_term<MODE>(p0 + q, ci, val, fval, x, dinv, tdiv, fmt, ep);
            }
        }
#pragma unroll
        for (int d = TPR / 2; d >= 1; d >>= 1)
            s += __shfl_xor(s, d);
        if constexpr (sp_step(MODE)) {
            // steps 13-14 for this block's rows: v = w / t, stored through
            // the accessor (rows in [n, ldy) hold w = 0 and store 0)
            if (part == 0 && row < ldy)
                store_entry(fmt, Q, row, x[row] / tdiv, ep);
        }
        if (part == 0 && row < ldy) {
            double yv;
            if constexpr ((MODE & 7) == SP_RESID)
                yv = row < n ? b[row] - s : 0.0;
            else if constexpr ((MODE & 7) == SP_ACCUM)
                yv = y[row] + s;
            else
                yv = row < n ? s : 0.0;
            y[row] = yv;
            ssq += yv * yv;
            mx = fmax(mx, fabs(yv));
        }
    }
    if (role == SR_NONE)
        return;
    block_sum_max(ssq, mx);
    if (threadIdx.x == 0) {
        ra.part[blockIdx.x] = ssq;
        ra.part[(size_t)ra.stride + blockIdx.x] = mx;
    }
}

// ---------------------------------------------------------------------------
// CSR SpMV with a row-parallel gather, for long rows: a block owns RPB
// consecutive rows.  Phase 1 loads the block's values and column indices
// with unit stride across the threads (coalesced) into LDS.  Phase 2 gives
// wave p the entries p, p + NPART, ... of every row, lane r for row r: one
// gather instruction reads x at the same stencil offset for RPB consecutive
// rows, i.e. contiguous addresses on a structured matrix, where gathering in
// entry order (CSR-stream) touches about three times as many cache lines per
// instruction on 27-point rows and is bound by them.  The NPART partial sums
// of a row are added in wave order.  A block whose rows hold more than CAP
// entries reads them from memory in phase 2.  Same modes, padding rows and
// partials as k_spmv.
// ---------------------------------------------------------------------------

template <int MODE>
__device__ __forceinline__ double spmv_x(int c, const double *__restrict__ x,
                                         const double *__restrict__ dinv, double tdiv, int fmt,
                                         EncParam ep)
{
    double xv = x[c];
    if constexpr (sp_step(MODE))
        xv = xv / tdiv;
    if constexpr (sp_quant(MODE))
        xv = quantize(fmt, xv, ep);
    if constexpr ((MODE & 7) == SP_JACOBI)
        xv = dinv[c] * xv;
    return xv;
}

template <int RPB, int CAP, int MODE>
__global__ __launch_bounds__(BLK) void k_spmv_rp(int n, int64_t ldy,
                                                 const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ ci,
                                                 const double *__restrict__ val,
                                                 const float *__restrict__ fval,
                                                 const double *__restrict__ x,
                                                 const double *__restrict__ dinv,
                                                 const double *__restrict__ b,
                                                 double *__restrict__ y, RedArgs ra, int role,
                                                 const DevState *st, uint8_t *__restrict__ Q,
                                                 const double *__restrict__ qscale, int fmt)
{
    constexpr int NPART = BLK / RPB;
    constexpr int UNR = 4;
    constexpr bool FLT = (MODE & 7) == SP_FLOATVAL || (MODE & 7) == SP_ACCUM;
    if (st && role != SR_FREE && st->done)
        return;
    double tdiv = 1.0;
    EncParam ep{1.0, 0};
    if constexpr (sp_step(MODE)) {
        tdiv = st->t;
        ep = param_from_scale(fmt, *qscale);
    }
    __shared__ double lv[CAP];
    __shared__ int lc[CAP];
    __shared__ int lrp[RPB + 1];
    __shared__ double ls[NPART][RPB];
    const int tid = threadIdx.x;
    const int r = tid % RPB, part = tid / RPB;
    double ssq = 0.0, mx = 0.0;
    const int64_t nblk = (ldy + RPB - 1) / RPB;
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const int64_t r0 = blk * RPB;
        const int nr = r0 < n ? (int)min((int64_t)RPB, (int64_t)n - r0) : 0;   // rows with entries
        __syncthreads();                    // LDS reuse across iterations
        for (int t = tid; t <= nr && nr > 0; t += BLK)
            lrp[t] = rp[r0 + t];
        __syncthreads();
        const int p0 = nr > 0 ? lrp[0] : 0;
        const int cnt = nr > 0 ? lrp[nr] - p0 : 0;
        const bool staged = cnt <= CAP;
        if (staged && cnt > 0) {
            for (int q = tid; q < cnt; q += BLK * UNR) {
                double v[UNR];
                int c[UNR];
#pragma unroll
                for (int u = 0; u < UNR; ++u) {
                    const int qq = min(q + u * BLK, cnt - 1);   // clamped: loads stay in bounds
                    v[u] = FLT ? (double)fval[p0 + qq] : val[p0 + qq];
                    c[u] = ci[p0 + qq];
                }
#pragma unroll
                for (int u = 0; u < UNR; ++u)
                    if (q + u * BLK < cnt) {
                        lv[q + u * BLK] = v[u];
                        lc[q + u * BLK] = c[u];
                    }
            }
        }
        __syncthreads();
        double s = 0.0;
        if (r < nr) {
            const int a0 = lrp[r] - p0, a1 = lrp[r + 1] - p0;
            if (staged) {
                int k = a0 + part;
                for (; k + 3 * NPART < a1; k += 4 * NPART) {
                    const double x0 = spmv_x<MODE>(lc[k], x, dinv, tdiv, fmt, ep);
                    const double x1 = spmv_x<MODE>(lc[k + NPART], x, dinv, tdiv, fmt, ep);
                    const double x2 = spmv_x<MODE>(lc[k + 2 * NPART], x, dinv, tdiv, fmt, ep);
                    const double x3 = spmv_x<MODE>(lc[k + 3 * NPART], x, dinv, tdiv, fmt, ep);
                    s += lv[k] * x0;
                    s += lv[k + NPART] * x1;
                    s += lv[k + 2 * NPART] * x2;
                    s += lv[k + 3 * NPART] * x3;
                }
                for (; k < a1; k += NPART)
                    s += lv[k] * spmv_x<MODE>(lc[k], x, dinv, tdiv, fmt, ep);
            } else {
                for (int k = a0 + part; k < a1; k += NPART)
                    s += spmv_term<MODE>(p0 + k, ci, val, fval, x, dinv, tdiv, fmt, ep);
            }
        }
        ls[part][r] = s;
        __syncthreads();
        if (tid < RPB) {
            const int64_t row = r0 + tid;
            double t = ls[0][tid];
#pragma unroll
            for (int q = 1; q < NPART; ++q)
                t += ls[q][tid];
            if (row < ldy) {
                if constexpr (sp_step(MODE)) {
                    // steps 13-14 for this block's rows: v = w / t, stored
                    // through the accessor (rows in [n, ldy) hold w = 0)
                    store_entry(fmt, Q, row, x[row] / tdiv, ep);
                }
                double yv;
                if constexpr ((MODE & 7) == SP_RESID)
                    yv = row < n ? b[row] - t : 0.0;
                else if constexpr ((MODE & 7) == SP_ACCUM)
                    yv = y[row] + t;
                else
                    yv = row < n ? t : 0.0;
                y[row] = yv;
                ssq += yv * yv;
                mx = fmax(mx, fabs(yv));
            }
        }
    }
    if (role == SR_NONE)
        return;
    block_sum_max(ssq, mx);
    if (threadIdx.x == 0) {
        ra.part[blockIdx.x] = ssq;
        ra.part[(size_t)ra.stride + blockIdx.x] = mx;
    }
}

// ---------------------------------------------------------------------------
// SpMV on the sliced-ELL copy of A (SELL-64; layout in include/cbgmres.h):
// one wave per slice of 64 rows, lane = row, so the value and column loads
// of one entry index are 512 and 256 contiguous bytes and, on a stencil
// matrix, the gather of x at one stencil offset reads 64 consecutive
// entries.  No LDS and no barrier inside the slice loop.  Each row is summed
// in CSR order with separately rounded products and sums (floating-point
// contraction off), the order of the row-sequential CSR sum, so y = A x is
// that sum bit for bit; a padding entry adds 0 * x_row.  NT: stream the
// values and columns past the caches (non-temporal loads), which keeps x
// resident in L2 on long rows.  Modes as k_spmv's, without the sparse-P
// ones (those read float values on the CSR pattern).
// ---------------------------------------------------------------------------

template <int MODE>
__device__ __forceinline__ double sell_x(int c, const double *__restrict__ x,
                                         const double *__restrict__ dinv, double tdiv, int fmt,
                                         EncParam ep)
{
#pragma clang fp contract(off)
    double xv = x[c];
    if constexpr (sp_step(MODE))
        xv = xv / tdiv;
    if constexpr (sp_quant(MODE))
        xv = quantize(fmt, xv, ep);
    if constexpr ((MODE & 7) == SP_JACOBI)
        xv = dinv[c] * xv;
    return xv;
}

template <bool NT, typename T>
__device__ __forceinline__ T sell_ld(const T *p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

constexpr int SELL_UNR = 9;      // entries per row in flight (a third of a 27-point row)

template <int MODE, bool NT, bool DIX>
__global__ __launch_bounds__(BLK) void k_spmv_sell(
    int n, int64_t ldy, int64_t nslice, const int64_t *__restrict__ sp,
    const int32_t *__restrict__ sc, const uint8_t *__restrict__ sd,
    const int32_t *__restrict__ sdiag, int ndiag, const double *__restrict__ sv,
    const double *__restrict__ x, const double *__restrict__ dinv, const double *__restrict__ b,
    double *__restrict__ y, RedArgs ra, int role, const DevState *st, uint8_t *__restrict__ Q,
    const double *__restrict__ qscale, int fmt)
{
#pragma clang fp contract(off)
    if (st && role != SR_FREE && st->done)
        return;
    // DIX: columns as row + offset, the offset's index one byte per entry
    __shared__ int32_t ldg[DIX ? SELL_MAX_DIAG : 1];
    if constexpr (DIX) {
        for (int k = threadIdx.x; k < ndiag; k += BLK)
            ldg[k] = sdiag[k];
        __syncthreads();
    }
    double tdiv = 1.0;
    EncParam ep{1.0, 0};
    if constexpr (sp_step(MODE)) {
        tdiv = st->t;
        ep = param_from_scale(fmt, *qscale);
    }
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nsy = (ldy + 63) / 64;        // slices of rows to write (>= nslice)
    double ssq = 0.0, mx = 0.0;
    for (int64_t s = (int64_t)blockIdx.x * NWAVE + wv; s < nsy;
         s += (int64_t)gridDim.x * NWAVE) {
        const int64_t row = s * 64 + lane;
        double acc = 0.0;
        if (s < nslice) {
            const int64_t o = sp[s];
            const int w = (int)((sp[s + 1] - o) >> 6);
            const int32_t *c = sc + o + lane;
            const uint8_t *cd = sd + o + lane;
            const double *v = sv + o + lane;
            const int32_t rowc = (int32_t)min(row, (int64_t)n - 1);   // rows >= n: padding only
            // batches of SELL_UNR entries, every load of a batch in flight
            // before the first product; a short last batch re-reads entry
            // w - 1 for its missing slots and adds nothing for them
            for (int k = 0; k < w; k += SELL_UNR) {
                int32_t cc[SELL_UNR];
                double vv[SELL_UNR];
#pragma unroll
                for (int u = 0; u < SELL_UNR; ++u) {
                    const int64_t e = (int64_t)min(k + u, w - 1) * 64;
                    if constexpr (DIX)
                        cc[u] = sell_ld<NT>(cd + e);
                    else
                        cc[u] = sell_ld<NT>(c + e);
                    vv[u] = sell_ld<NT>(v + e);
                }
                if constexpr (DIX) {
#pragma unroll
                    for (int u = 0; u < SELL_UNR; ++u)
                        cc[u] = rowc + ldg[cc[u]];
                }
#pragma unroll
                for (int u = 0; u < SELL_UNR; ++u) {
                    const double t = vv[u] * sell_x<MODE>(cc[u], x, dinv, tdiv, fmt, ep);
                    if (k + u < w)
                        acc = acc + t;
                }
            }
        }
        if (row < ldy) {
            if constexpr (sp_step(MODE))
                store_entry(fmt, Q, row, x[row] / tdiv, ep);   // steps 13-14 for this row
            double yv;
            if constexpr ((MODE & 7) == SP_RESID)
                yv = row < n ? b[row] - acc : 0.0;
            else
                yv = row < n ? acc : 0.0;
            y[row] = yv;
            ssq += yv * yv;
            mx = fmax(mx, fabs(yv));
        }
    }
    if (role == SR_NONE)
        return;
    block_sum_max(ssq, mx);
    if (threadIdx.x == 0) {
        ra.part[blockIdx.x] = ssq;
        ra.part[(size_t)ra.stride + blockIdx.x] = mx;
    }
}

// Set-up of the sliced-ELL copy.  sp[s + 1] = 64 * (longest row of slice
// s), sp[0] = 0; one wave per slice.
__global__ __launch_bounds__(BLK) void k_sell_width(int n, const int32_t *__restrict__ rp,
                                                    int64_t nslice, int64_t *__restrict__ sp)
{
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    for (int64_t s = (int64_t)blockIdx.x * NWAVE + wv; s < nslice;
         s += (int64_t)gridDim.x * NWAVE) {
        const int64_t row = s * 64 + lane;
        int len = row < n ? rp[row + 1] - rp[row] : 0;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1)
            len = max(len, __shfl_xor(len, d));
        if (lane == 0)
            sp[s + 1] = 64 * (int64_t)len;
        if (s == 0 && lane == 0)
            sp[0] = 0;
    }
}

// In-place inclusive scan of sp[1 .. nslice], one block of 1024 threads,
// 1024 entries per round with the running total carried between rounds.
constexpr int SCAN_BLK = 1024;
__global__ __launch_bounds__(SCAN_BLK) void k_sell_scan(int64_t nslice, int64_t *__restrict__ sp)
{
    __shared__ int64_t buf[2][SCAN_BLK];
    __shared__ int64_t carry;
    const int tid = threadIdx.x;
    if (tid == 0)
        carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nslice; base += SCAN_BLK) {
        const int64_t i = base + tid;
        int cur = 0;
        buf[cur][tid] = i < nslice ? sp[1 + i] : 0;
        __syncthreads();
        for (int d = 1; d < SCAN_BLK; d <<= 1) {     // Hillis-Steele, double-buffered
            const int64_t v = buf[cur][tid] + (tid >= d ? buf[cur][tid - d] : 0);
            buf[cur ^ 1][tid] = v;
            cur ^= 1;
            __syncthreads();
        }
        const int64_t total = buf[cur][SCAN_BLK - 1];
        if (i < nslice)
            sp[1 + i] = carry + buf[cur][tid];
        __syncthreads();                 // every thread has read carry
        if (tid == 0)
            carry += total;
        __syncthreads();
    }
}

// Fills the entries: one wave per slice, lane = row, entry k at
// sp[s] + 64 k + lane.
__global__ __launch_bounds__(BLK) void k_sell_fill(int n, const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci,
                                                   const double *__restrict__ val, int64_t nslice,
                                                   const int64_t *__restrict__ sp,
                                                   int32_t *__restrict__ sc,
                                                   double *__restrict__ sv)
{
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    for (int64_t s = (int64_t)blockIdx.x * NWAVE + wv; s < nslice;
         s += (int64_t)gridDim.x * NWAVE) {
        const int64_t row = s * 64 + lane;
        const int p0 = row < n ? rp[row] : 0;
        const int len = row < n ? rp[row + 1] - p0 : 0;
        const int pad = (int)min(row, (int64_t)n - 1);
        const int64_t o = sp[s];
        const int w = (int)((sp[s + 1] - o) >> 6);
        for (int k = 0; k < w; ++k) {
            const int64_t e = o + (int64_t)k * 64 + lane;
            sc[e] = k < len ? ci[p0 + k] : pad;
            sv[e] = k < len ? val[p0 + k] : 0.0;
        }
    }
}

// Diagonal-index form of the sliced-ELL columns.  The distinct offsets
// col - row go into an open-addressing hash set (DIAG_HASH int32 slots,
// empty = INT32_MIN, which no offset can equal), then one block collects
// and sorts them, and a last pass writes each entry's index.  Set-up only:
// the hash insertion uses atomics, the result does not depend on their
// order (the offsets are sorted).
constexpr int DIAG_HASH = 4096;
constexpr int32_t DIAG_EMPTY = INT32_MIN;

__device__ __forceinline__ int32_t entry_offset(const int32_t *__restrict__ sc, int64_t e,
                                                int64_t row, int n)
{
    return row < n ? (int32_t)(sc[e] - row) : 0;        // rows >= n: padding, offset 0
}

// inserts v; returns false when the table is full
__device__ bool diag_insert(int32_t *hash, int32_t v)
{
    uint32_t h = ((uint32_t)v * 2654435761u) & (DIAG_HASH - 1);   // Knuth's multiplicative hash
    for (int probe = 0; probe < DIAG_HASH; ++probe) {
        const int32_t cur = __hip_atomic_load(&hash[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == v)
            return true;
        if (cur == DIAG_EMPTY) {
            const int32_t old = atomicCAS(&hash[h], DIAG_EMPTY, v);
            if (old == DIAG_EMPTY || old == v)
                return true;
        }
        h = (h + 1) & (DIAG_HASH - 1);
    }
    return false;
}

__global__ __launch_bounds__(BLK) void k_diag_insert(int n, int64_t nslice,
                                                     const int64_t *__restrict__ sp,
                                                     const int32_t *__restrict__ sc,
                                                     int32_t *hash, unsigned *full)
{
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    if (blockIdx.x == 0 && threadIdx.x == 0 && !diag_insert(hash, 0))
        atomicOr(full, 1u);
    for (int64_t s = (int64_t)blockIdx.x * NWAVE + wv; s < nslice;
         s += (int64_t)gridDim.x * NWAVE) {
        const int64_t row = s * 64 + lane;
        const int64_t o = sp[s];
        const int w = (int)((sp[s + 1] - o) >> 6);
        for (int k = 0; k < w; ++k) {
            const int32_t off = entry_offset(sc, o + (int64_t)k * 64 + lane, row, n);
            // one insertion per wave when all lanes share the offset
            const int32_t first = __shfl(off, 0);
            const bool same = __all(off == first);
            if ((!same || lane == 0) && !diag_insert(hash, off))
                atomicOr(full, 1u);
            if (*(volatile unsigned *)full)
                return;
        }
    }
}

// One block: the distinct offsets, sorted, into diag[0 .. count) when
// count <= SELL_MAX_DIAG; count (or more than SELL_MAX_DIAG when the table
// overflowed) into *count_out.
__global__ __launch_bounds__(BLK) void k_diag_collect(const int32_t *__restrict__ hash,
                                                      const unsigned *full, int32_t *diag,
                                                      int32_t *count_out)
{
    __shared__ int32_t list[SELL_MAX_DIAG];
    __shared__ int cnt;
    if (threadIdx.x == 0)
        cnt = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < DIAG_HASH; i += BLK) {
        const int32_t v = hash[i];
        if (v != DIAG_EMPTY) {
            const int at = atomicAdd(&cnt, 1);
            if (at < SELL_MAX_DIAG)
                list[at] = v;
        }
    }
    __syncthreads();
    const int c = cnt;
    if (*full || c > SELL_MAX_DIAG) {
        if (threadIdx.x == 0)
            *count_out = max(c, SELL_MAX_DIAG + 1);
        return;
    }
    // rank sort of distinct values
    for (int t = threadIdx.x; t < c; t += BLK) {
        const int32_t v = list[t];
        int rank = 0;
        for (int u = 0; u < c; ++u)
            rank += list[u] < v ? 1 : 0;
        diag[rank] = v;
    }
    if (threadIdx.x == 0)
        *count_out = c;
}

// Each entry's offset index, by binary search in the sorted table.
__global__ __launch_bounds__(BLK) void k_diag_index(int n, int64_t nslice,
                                                    const int64_t *__restrict__ sp,
                                                    const int32_t *__restrict__ sc,
                                                    const int32_t *__restrict__ diag, int ndiag,
                                                    uint8_t *__restrict__ sd)
{
    __shared__ int32_t ld[SELL_MAX_DIAG];
    for (int k = threadIdx.x; k < ndiag; k += BLK)
        ld[k] = diag[k];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    for (int64_t s = (int64_t)blockIdx.x * NWAVE + wv; s < nslice;
         s += (int64_t)gridDim.x * NWAVE) {
        const int64_t row = s * 64 + lane;
        const int64_t o = sp[s];
        const int w = (int)((sp[s + 1] - o) >> 6);
        for (int k = 0; k < w; ++k) {
            const int64_t e = o + (int64_t)k * 64 + lane;
            const int32_t off = entry_offset(sc, e, row, n);
            int lo = 0, hi = ndiag - 1;                 // off is in the table
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (ld[mid] < off)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            sd[e] = (uint8_t)lo;
        }
    }
}

__global__ void k_fill_i32(int32_t *p, int count, int32_t v)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// Multi-dot through the accessor: h_k = sum_i dec(V_k)_i w_i, k < j.
// Each block keeps a tile of w in registers and streams the stored vectors
// KC at a time.  In full tiles every load of a batch is issued before any
// is used (no bounds test between them); only the ragged last tile takes
// the guarded path.  Per-lane partials are reduced across the wave by a
// transposing butterfly, across waves in LDS, across tiles in LDS, and
// across blocks by the fixed-order grid reduction.
// ---------------------------------------------------------------------------


template <int F>
__device__ __forceinline__ u32x4 ld_chunk(const uint8_t *__restrict__ V, int64_t ldb, int k,
                                          int64_t i0)
{
    return __builtin_nontemporal_load(
        (const u32x4 *)(V + (int64_t)k * ldb + i0 * fmt_bytes(F)));
}

// GRAM: the same pass also forms g_k = dec(V_k)^T dec(V_{j-1}), k < j, the
// newest row of the Gram matrix of the stored vectors (partials in rows
// j + 2 + k), from a register tile of the newest vector.
template <int F, bool GRAM>
__global__ __launch_bounds__(BLK) CBG_MD_ATTR void k_multidot(const uint8_t *__restrict__ V, int64_t ld,
                                                  const double *__restrict__ scales, int n, int j,
                                                  const double *__restrict__ w, RedArgs ra,
                                                  const DevState *st, int gated, int with_norms)
{
    if (gated && st->done)
        return;
    using T = Fmt<F>;
    constexpr int VW = T::VW, CH = T::CH, KC = T::KC;
    constexpr int NV = GRAM ? 2 : 1;                  // values per stored vector
    constexpr int WROW = MAX_RESTART + 1;
    constexpr int TILE = BLK * VW * CH;
    const int64_t ldb = ld * fmt_bytes(F);
    // per-wave running sums over the block's tiles: no barrier until the end
    __shared__ double wacc[NWAVE][NV * WROW];
    for (int k = threadIdx.x; k < NWAVE * NV * WROW; k += BLK)
        (&wacc[0][0])[k] = 0.0;
    __syncthreads();
    const int64_t ntiles = ((int64_t)n + TILE - 1) / TILE;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double ssq = 0.0, mx = 0.0;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const bool full = (tile + 1) * TILE <= n;
        double wr[CH * VW];
        double gr[GRAM ? CH * VW : 1];
        int64_t i0[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            i0[c] = tile * TILE + ((int64_t)c * BLK + threadIdx.x) * VW;
            load_w<VW>(w, n, i0[c], wr + c * VW);
        }
        if constexpr (GRAM) {
            const double sg = T::SCALED ? scales[j - 1] : 1.0;
#pragma unroll
            for (int c = 0; c < CH; ++c)
                load_dec<F>(V + (int64_t)(j - 1) * ldb, i0[c], n, sg, gr + c * VW);
        }
        if (with_norms) {
#pragma unroll
            for (int e = 0; e < CH * VW; ++e) {
                ssq += wr[e] * wr[e];
                mx = fmax(mx, fabs(wr[e]));
            }
        }
        for (int kc = 0; kc < j; kc += KC) {
            double acc[NV * KC];
            if (full) {
                u32x4 raw[KC][CH];
#pragma unroll
                for (int kk = 0; kk < KC; ++kk)
#pragma unroll
                    for (int c = 0; c < CH; ++c)
                        raw[kk][c] = ld_chunk<F>(V, ldb, min(kc + kk, j - 1), i0[c]);
                // keep the batch's loads together, ahead of its arithmetic: under
                // the Gram tile's register pressure the scheduler would otherwise
                // interleave them with the FMAs, one load in flight per wave
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int kk = 0; kk < KC; ++kk) {
                    const double s = T::SCALED ? scales[min(kc + kk, j - 1)] : 1.0;
                    double a = 0.0, g = 0.0;
#pragma unroll
                    for (int c = 0; c < CH; ++c) {
                        double d[VW];
                        T::dec(raw[kk][c], s, d);
#pragma unroll
                        for (int e = 0; e < VW; ++e) {
                            a = fma(d[e], wr[c * VW + e], a);
                            if constexpr (GRAM)
                                g = fma(d[e], gr[c * VW + e], g);
                        }
                    }
                    acc[kk] = a;
                    if constexpr (GRAM)
                        acc[KC + kk] = g;
                }
            } else {
#pragma unroll
                for (int kk = 0; kk < KC; ++kk) {
                    const int k = min(kc + kk, j - 1);
                    const double s = T::SCALED ? scales[k] : 1.0;
                    const uint8_t *Vk = V + (int64_t)k * ldb;
                    double a = 0.0, g = 0.0;
#pragma unroll
                    for (int c = 0; c < CH; ++c) {
                        double d[VW];
                        load_dec<F>(Vk, i0[c], n, s, d);
#pragma unroll
                        for (int e = 0; e < VW; ++e) {
                            a = fma(d[e], wr[c * VW + e], a);
                            if constexpr (GRAM)
                                g = fma(d[e], gr[c * VW + e], g);
                        }
                    }
                    acc[kk] = a;
                    if constexpr (GRAM)
                        acc[KC + kk] = g;
                }
            }
            wave_transpose_sum<NV * KC>(acc);
            if (lane < NV * KC) {
                const int idx = bitrev<NV * KC>(lane);
                const int k = kc + (idx < KC ? idx : idx - KC);
                if (k < j)
                    wacc[wave][(idx < KC ? 0 : WROW) + k] += acc[0];
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < NV * j; k += BLK) {
        const int src = k < j ? k : WROW + (k - j);
        double t = wacc[0][src];
#pragma unroll
        for (int q = 1; q < NWAVE; ++q)
            t += wacc[q][src];
        const int row = k < j ? k : j + 2 + (k - j);       // g_k in row j + 2 + k
        ra.part[(size_t)row * ra.stride + blockIdx.x] = t;
    }
    if (with_norms) {
        block_sum_max(ssq, mx);
        if (threadIdx.x == 0) {
            ra.part[(size_t)j * ra.stride + blockIdx.x] = ssq;
            ra.part[(size_t)(j + 1) * ra.stride + blockIdx.x] = mx;
        }
    }
}

// ---------------------------------------------------------------------------
// Basis combination through the accessor: s = sum_k c_k dec(V_k), k < j.
//   U_PLAIN / U_STEP1 / U_STEP2 / U_STEP1N: w -= s, with ||w||_2 and
//   ||w||_inf (partials in rows 0 and 1, except U_STEP1);
//   U_CGS2: steps 5-10 in one update (coef = h; see below).
//   U_SOLUTION: x += dinv .* s (Jacobi) or x += s;  U_COMBINE: out = s.
// Full tiles stream the vectors UNR at a time with the next batch's loads
// in flight while the current batch is decoded and accumulated.
// ---------------------------------------------------------------------------

// Fixed-order folds of block partials (used by the reduce kernel and by
// the second pass of a hard step).
constexpr int RBLK = 256;
constexpr int RWAVES = RBLK / 64;

// One wave folds block partials src[0 .. nb) (16 independent loads in flight
// per lane, fixed order); every lane returns the total.  nb = 0 gives 0.
__device__ __forceinline__ double wave_fold(const double *__restrict__ src, int nb, bool is_max)
{
    constexpr int U = 16;
    const int lane = threadIdx.x & 63;
    double acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
        acc[u] = 0.0;
    for (int b0 = lane; b0 < nb; b0 += 64 * U) {
        double x[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            x[u] = src[min(b0 + 64 * u, nb - 1)];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double xv = (b0 + 64 * u < nb) ? x[u] : 0.0;
            acc[u] = is_max ? fmax(acc[u], xv) : acc[u] + xv;
        }
    }
    double a = acc[0];
#pragma unroll
    for (int u = 1; u < U; ++u)
        a = is_max ? fmax(a, acc[u]) : a + acc[u];
    return is_max ? wave_max(a) : wave_sum(a);
}

// The whole block folds src[0 .. nb): wave w takes the contiguous quarter
// starting at w * ceil(nb / 4), and the four wave totals are combined in
// wave order (so the result depends on nb only, not on timing).  Every
// thread returns the total; block-uniform call.
__device__ double block_fold(const double *__restrict__ src, int nb, bool is_max)
{
    __shared__ double part[RWAVES];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = (nb + RWAVES - 1) / RWAVES;
    const int lo = min(wave * q, nb), hi = min(lo + q, nb);
    const double a = wave_fold(src + lo, hi - lo, is_max);
    if (lane == 0)
        part[wave] = a;
    __syncthreads();
    double t = part[0];
#pragma unroll
    for (int w = 1; w < RWAVES; ++w)
        t = is_max ? fmax(t, part[w]) : t + part[w];
    __syncthreads();
    return t;
}

enum { U_PLAIN = 0, U_STEP1 = 1, U_STEP2 = 2, U_SOLUTION = 3, U_COMBINE = 4, U_STEP1N = 5,
       U_CGS2 = 6, U_HARD = 7 };

// A step of the one-pass update is "hard" when t1^2 = omega^2 - h^T h -
// h^T u falls below HARD_RATIO omega^2 (t1 < omega / 100).  There the
// cancellation in t1^2 and the Gram-form re-dot (which cannot see the
// rounding of the first update, an error of about u64 omega / t1 in the
// orthogonality of the new vector) are no longer negligible, so the step
// takes Fig. 1's explicit form instead: w1 = w - V h, t1 = ||w1||,
// u = V^T w1, w2 = w1 - V u, t2 = ||w2||.  On the stencil systems here
// t / omega stays above 0.3, so the explicit form is a safeguard for
// near-breakdowns (clustered spectra), not the common path.
constexpr double HARD_RATIO = 1e-4;
// Tile blocks of the second-pass kernel (U_HARD).  It is launched on every
// step and returns at once unless the step is hard, so a small grid keeps
// that launch cheap; a hard step's second pass streams the basis with it.
constexpr int HARD_BLOCKS = 256;

// The one-pass update's G h for one wave: out[k] = sum over l in [l0, l1) of
// G[l][k] h_l, for k = lane + 64 q < j (q < NK), each sum in increasing l
// as one FMA chain.  The NK columns of a row are loaded together and UL
// rows at a time (column indices clamped into [0, j); the extra sums are
// not stored), so a wave keeps NK * UL loads of G in flight instead of
// walking its columns one after another.
template <int NK>
__device__ __forceinline__ void gram_times_h(const double *__restrict__ G, size_t ldg,
                                             const double *lh, int j, int l0, int l1, int lane,
                                             double *out)
{
    constexpr int UL = NK == 1 ? 8 : NK == 2 ? 4 : NK == 3 ? 3 : 2;
    int kc[NK];
    double acc[NK];
#pragma unroll
    for (int q = 0; q < NK; ++q) {
        kc[q] = min(lane + 64 * q, j - 1);
        acc[q] = 0.0;
    }
    int l = l0;
    for (; l + UL <= l1; l += UL) {
        double g[UL][NK];
#pragma unroll
        for (int u = 0; u < UL; ++u)
#pragma unroll
            for (int q = 0; q < NK; ++q)
                g[u][q] = G[(size_t)(l + u) * ldg + kc[q]];
#pragma unroll
        for (int u = 0; u < UL; ++u) {
            const double hl = lh[l + u];
#pragma unroll
            for (int q = 0; q < NK; ++q)
                acc[q] = fma(g[u][q], hl, acc[q]);
        }
    }
    for (; l < l1; ++l) {
        const double hl = lh[l];
#pragma unroll
        for (int q = 0; q < NK; ++q)
            acc[q] = fma(G[(size_t)l * ldg + kc[q]], hl, acc[q]);
    }
#pragma unroll
    for (int q = 0; q < NK; ++q)
        if (lane + 64 * q < j)
            out[lane + 64 * q] = acc[q];
}

template <int F, int ROLE>
__global__ __launch_bounds__(BLK) void k_update(const uint8_t *__restrict__ V, int64_t ld,
                                                const double *__restrict__ scales, int n, int j_arg,
                                                const double *__restrict__ coef,
                                                double *__restrict__ w,
                                                const double *__restrict__ dinv, RedArgs ra,
                                                const DevState *st,
                                                double *__restrict__ uio, DevState *stw,
                                                const double *__restrict__ G, StepArrays sa,
                                                int nb_first)
{
    int j = j_arg;
    if constexpr (ROLE == U_STEP1 || ROLE == U_STEP2 || ROLE == U_STEP1N || ROLE == U_CGS2 ||
                  ROLE == U_HARD) {
        if (st->done)
            return;
        if (ROLE == U_STEP2 && !st->reorth)
            return;
        if (ROLE == U_HARD && !st->hard)
            return;
    }
    if constexpr (ROLE == U_SOLUTION || ROLE == U_COMBINE)
        j = st->jeff;
    using T = Fmt<F>;
    constexpr int VW = T::VW, CH = T::CH, UNR = T::UNR;
    constexpr int TILE = BLK * VW * CH;
    const int64_t ldb = ld * fmt_bytes(F);
    const int64_t ntiles = ((int64_t)n + TILE - 1) / TILE;
    double ssq = 0.0, mx = 0.0;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // U_CGS2: Gram-form re-dot u = h - G h, then steps 5-10 in one update;
    // U_HARD: the explicit second pass of a hard step.  lp holds partial sums
    // of G h in the prologue and, on a hard step, the per-wave re-dot sums.
    // Both run one block more than the grid of tiles: that column block,
    // once the step's final coefficients are known, applies the stored
    // Givens rotations to the new Hessenberg column (rotate_column; rows
    // 0 .. j-2 into H, the carry into the state) while the other blocks
    // stream the basis, which leaves the closing fold only the new rotation.
    constexpr bool ONEPASS = ROLE == U_CGS2 || ROLE == U_HARD;
    __shared__ double lc[ONEPASS ? MAX_RESTART : 1];
    __shared__ double lh[ONEPASS ? MAX_RESTART : 1];
    __shared__ double lp[ONEPASS ? NWAVE * MAX_RESTART : 1];
    __shared__ double lr[2][NWAVE];
    const int ntb = ONEPASS ? (int)gridDim.x - 1 : (int)gridDim.x;    // blocks with tiles
    const bool colblk = ONEPASS && (int)blockIdx.x == ntb;
    auto rotate = [&](const double *c) {
        double *Hc = sa.H + (size_t)(j - 1) * ((size_t)st->m + 1);
        double(*pa)[MAX_RESTART] = (double(*)[MAX_RESTART])lp;
        double(*pb)[MAX_RESTART] = (double(*)[MAX_RESTART])(lp + 2 * MAX_RESTART);
        const double carry = rotate_column(c, j, sa.cs, sa.sn, Hc, pa, pb);
        if (tid == 0)
            stw->carry = carry;
    };
    bool hard = false;
    if constexpr (ROLE == U_CGS2) {
        // Every block forms the same u = h - G h (G symmetric: wave wv sums
        // G[l][k] h_l over its quarter of l for k = lane, lane + 64, ...,
        // reading rows of G, contiguous in k), then the same t1^2 =
        // ||w - V h||^2 = omega^2 - h^T h - h^T u, decides step 7, and updates
        // with h + u (re-orthogonalising) or h.  Block 0 publishes u, the
        // decision and t1 for the closing fold.  A hard step updates with h
        // only and adds the explicit re-dot of the result.
        for (int k = tid; k < j; k += BLK)
            lh[k] = coef[k];
        __syncthreads();
        const size_t ldg = (size_t)st->m + 1;
        const int q = (j + NWAVE - 1) / NWAVE;
        const int l0 = min(wv * q, j), l1 = min(l0 + q, j);
        switch ((j + 63) / 64) {
        case 1: gram_times_h<1>(G, ldg, lh, j, l0, l1, lane, lp + wv * MAX_RESTART); break;
        case 2: gram_times_h<2>(G, ldg, lh, j, l0, l1, lane, lp + wv * MAX_RESTART); break;
        case 3: gram_times_h<3>(G, ldg, lh, j, l0, l1, lane, lp + wv * MAX_RESTART); break;
        case 4: gram_times_h<4>(G, ldg, lh, j, l0, l1, lane, lp + wv * MAX_RESTART); break;
        default:
            for (int k0 = 0; k0 < j; k0 += 256)
                gram_times_h<4>(G + k0, ldg, lh, j - k0, l0, l1, lane, lp + wv * MAX_RESTART + k0);
            break;
        }
        __syncthreads();
        double phh = 0.0, phu = 0.0;
        for (int k = tid; k < j; k += BLK) {
            double gh = lp[k];
#pragma unroll
            for (int w2 = 1; w2 < NWAVE; ++w2)
                gh += lp[w2 * MAX_RESTART + k];
            const double hk = lh[k], uk = hk - gh;
            lc[k] = uk;
            phh += hk * hk;
            phu += hk * uk;
        }
        phh = wave_sum(phh);
        phu = wave_sum(phu);
        if (lane == 0) {
            lr[0][wv] = phh;
            lr[1][wv] = phu;
        }
        __syncthreads();
        double hh = lr[0][0], hu = lr[1][0];
#pragma unroll
        for (int w2 = 1; w2 < NWAVE; ++w2) {
            hh += lr[0][w2];
            hu += lr[1][w2];
        }
        const double omega = st->omega;
        const double t1sq = omega * omega - hh - hu;
        hard = !(t1sq >= HARD_RATIO * omega * omega);       // also when not finite
        const double t1 = hard ? 0.0 : sqrt(t1sq);
        const bool ro = !hard && (st->reorth_all || t1 < st->eta * omega);
        for (int k = tid; k < j; k += BLK) {
            const double uk = lc[k];
            if (blockIdx.x == 0)
                uio[k] = uk;
            lc[k] = ro ? lh[k] + uk : lh[k];
        }
        if (blockIdx.x == 0 && tid == 0) {
            stw->hard = hard ? 1 : 0;
            if (!hard) {
                stw->reorth = ro ? 1 : 0;
                stw->t = t1;
            }
        }
        if (colblk) {
            // a hard step's column waits for its second pass (U_HARD)
            if (!hard) {
                __syncthreads();                // lc complete
                rotate(lc);
            }
            return;
        }
        if (hard) {
            // per-wave re-dot sums, accumulated over the block's tiles
            for (int k = tid; k < NWAVE * j; k += BLK)
                lp[k] = 0.0;
        }
        __syncthreads();
        coef = lc;
    }
    if constexpr (ROLE == U_HARD) {
        // The hard step's explicit second pass.  Every block folds, from the
        // first pass's partials (rows 0..j-1: u = V^T w1; rows j, j+1:
        // ||w1||^2, max|w1|), u and t1, decides step 7 against t1, and
        // updates w1 -= V u.  Block 0 publishes u, t1, max|w1| and the
        // decision; the norms go to rows j+2, j+3 for the closing fold.
        const int nb = nb_first;             // the first pass's tile blocks
        for (int k = wv; k < j; k += NWAVE) {
            const double a = wave_fold(ra.part + (size_t)k * ra.stride, nb, false);
            if (lane == 0)
                lc[k] = a;
        }
        if (wv < 2) {
            const double a = wave_fold(ra.part + (size_t)(j + wv) * ra.stride, nb, wv == 1);
            if (lane == 0)
                lr[0][wv] = a;
        }
        __syncthreads();
        const double t1 = sqrt(lr[0][0]);
        const bool ro = st->reorth_all || t1 < st->eta * st->omega;
        if (blockIdx.x == 0) {
            for (int k = tid; k < j; k += BLK)
                uio[k] = lc[k];
            if (tid == 0) {
                stw->t = t1;
                stw->wmax = lr[0][1];
                stw->reorth = ro ? 1 : 0;
            }
        }
        if (colblk) {
            // the column: h + u when the second pass re-orthogonalises, else h
            for (int k = tid; k < j; k += BLK)
                lh[k] = ro ? coef[k] + lc[k] : coef[k];
            __syncthreads();
            rotate(lh);
            return;
        }
        if (!ro)
            return;
        coef = lc;
    }
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += ntb) {
        const bool full = (tile + 1) * TILE <= n;
        double s[CH * VW];
        int64_t i0[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            i0[c] = tile * TILE + ((int64_t)c * BLK + threadIdx.x) * VW;
#pragma unroll
            for (int e = 0; e < VW; ++e)
                s[c * VW + e] = 0.0;
        }
        if (full && j > 0) {
            u32x4 cur[UNR][CH];
#pragma unroll
            for (int u = 0; u < UNR; ++u)
#pragma unroll
                for (int c = 0; c < CH; ++c)
                    cur[u][c] = ld_chunk<F>(V, ldb, min(u, j - 1), i0[c]);
            for (int kg = 0; kg < j; kg += UNR) {
                u32x4 nxt[UNR][CH];
#pragma unroll
                for (int u = 0; u < UNR; ++u)
#pragma unroll
                    for (int c = 0; c < CH; ++c)
                        nxt[u][c] = ld_chunk<F>(V, ldb, min(kg + UNR + u, j - 1), i0[c]);
#pragma unroll
                for (int u = 0; u < UNR; ++u) {
                    const int k = min(kg + u, j - 1);
                    const double ck = (kg + u < j) ? coef[k] : 0.0;
                    const double sk = T::SCALED ? scales[k] : 1.0;
#pragma unroll
                    for (int c = 0; c < CH; ++c) {
                        double d[VW];
                        T::dec(cur[u][c], sk, d);
#pragma unroll
                        for (int e = 0; e < VW; ++e)
                            s[c * VW + e] = fma(ck, d[e], s[c * VW + e]);
                    }
                }
#pragma unroll
                for (int u = 0; u < UNR; ++u)
#pragma unroll
                    for (int c = 0; c < CH; ++c)
                        cur[u][c] = nxt[u][c];
            }
        } else {
            for (int k = 0; k < j; ++k) {
                const double ck = coef[k];
                const double sk = T::SCALED ? scales[k] : 1.0;
                const uint8_t *Vk = V + (int64_t)k * ldb;
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    double d[VW];
                    load_dec<F>(Vk, i0[c], n, sk, d);
#pragma unroll
                    for (int e = 0; e < VW; ++e)
                        s[c * VW + e] = fma(ck, d[e], s[c * VW + e]);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            double o[VW];
            if constexpr (ROLE == U_COMBINE) {
#pragma unroll
                for (int e = 0; e < VW; ++e)
                    o[e] = s[c * VW + e];
            } else if constexpr (ROLE == U_SOLUTION) {
                load_w<VW>(w, n, i0[c], o);
                if (dinv) {
                    double dv[VW];
                    load_w<VW>(dinv, n, i0[c], dv);
#pragma unroll
                    for (int e = 0; e < VW; ++e)
                        o[e] = fma(dv[e], s[c * VW + e], o[e]);
                } else {
#pragma unroll
                    for (int e = 0; e < VW; ++e)
                        o[e] = o[e] + s[c * VW + e];
                }
            } else {
                load_w<VW>(w, n, i0[c], o);
#pragma unroll
                for (int e = 0; e < VW; ++e) {
                    o[e] = o[e] - s[c * VW + e];
                    ssq += o[e] * o[e];
                    mx = fmax(mx, fabs(o[e]));
                    s[c * VW + e] = o[e];        // kept for a hard step's re-dot
                }
            }
            store_w<VW>(w, n, i0[c], o);
        }
        if constexpr (ROLE == U_CGS2) {
            if (hard) {
                // Fig. 1 step 8 for this tile's rows: u_k += dec(V_k)^T w1
                // (rows >= n hold w1 = 0); one wave sum per vector, added
                // into the wave's slot in tile order
                for (int k = 0; k < j; ++k) {
                    const double sk = T::SCALED ? scales[k] : 1.0;
                    const uint8_t *Vk = V + (int64_t)k * ldb;
                    double acc = 0.0;
#pragma unroll
                    for (int c = 0; c < CH; ++c) {
                        double d[VW];
                        load_dec<F>(Vk, i0[c], n, sk, d);
#pragma unroll
                        for (int e = 0; e < VW; ++e)
                            acc = fma(d[e], s[c * VW + e], acc);
                    }
                    acc = wave_sum(acc);
                    if (lane == 0)
                        lp[k * NWAVE + wv] += acc;
                }
            }
        }
    }
    if constexpr (ROLE == U_SOLUTION || ROLE == U_COMBINE || ROLE == U_STEP1)
        return;
    // partial rows: the norms in rows 0 and 1; a hard step's first pass puts
    // the re-dot in rows 0..j-1 and the norms in rows j, j+1, its second
    // pass the norms in rows j+2, j+3
    int row = 0;
    if constexpr (ROLE == U_CGS2) {
        if (hard) {
            __syncthreads();
            for (int k = tid; k < j; k += BLK) {
                double a = lp[k * NWAVE];
#pragma unroll
                for (int w2 = 1; w2 < NWAVE; ++w2)
                    a += lp[k * NWAVE + w2];
                ra.part[(size_t)k * ra.stride + blockIdx.x] = a;
            }
            row = j;
        }
    }
    if constexpr (ROLE == U_HARD)
        row = j + 2;
    block_sum_max(ssq, mx);
    if (threadIdx.x == 0) {
        ra.part[(size_t)row * ra.stride + blockIdx.x] = ssq;
        ra.part[(size_t)(row + 1) * ra.stride + blockIdx.x] = mx;
    }
}

// ---------------------------------------------------------------------------
// Fused update and re-dot (Fig. 1 steps 5-8 for one basis pass):
//   w' = w - sum_k h_k dec(V_k);  u_k = sum_i dec(V_k)_i w'_i;  ||w'||, max|w'|.
// The re-dot needs every entry of w' of its rows, and w'_i needs every
// stored vector at row i, so each lane keeps the 8 bytes it loaded from
// each of the j vectors in registers (2 VGPRs per vector, j <= JM) and
// decodes them twice: once for the update, once for the dot.  The basis is
// read from HBM once instead of twice.  Partials as k_multidot with norms.
// ---------------------------------------------------------------------------

template <int F> struct Lane8;     // 8 bytes of a stored vector: LW entries
template <> struct Lane8<F_FP64> {
    static constexpr int LW = 1;
    __device__ static void dec(u32x2 q, double, double *d)
    {
        d[0] = __hiloint2double((int)q.y, (int)q.x);
    }
};
template <> struct Lane8<F_FP32> {
    static constexpr int LW = 2;
    __device__ static void dec(u32x2 q, double, double *d)
    {
        d[0] = (double)__uint_as_float(q.x);
        d[1] = (double)__uint_as_float(q.y);
    }
};
template <> struct Lane8<F_INT32> {
    static constexpr int LW = 2;
    __device__ static void dec(u32x2 q, double s, double *d)
    {
        d[0] = s * (double)(int32_t)q.x;
        d[1] = s * (double)(int32_t)q.y;
    }
};
template <int F> struct Lane8_16 {
    static constexpr int LW = 4;
    __device__ static void dec(u32x2 q, double s, double *d)
    {
        d[0] = Fmt16<F>::one(q.x & 0xFFFFu, s);
        d[1] = Fmt16<F>::one(q.x >> 16, s);
        d[2] = Fmt16<F>::one(q.y & 0xFFFFu, s);
        d[3] = Fmt16<F>::one(q.y >> 16, s);
    }
};
template <> struct Lane8<F_FP16> : Lane8_16<F_FP16> {};
template <> struct Lane8<F_BF16> : Lane8_16<F_BF16> {};
template <> struct Lane8<F_INT16> : Lane8_16<F_INT16> {};
template <> struct Lane8<F_FP16S> : Lane8_16<F_FP16S> {};
template <> struct Lane8<F_E4M3> {
    static constexpr int LW = 8;
    __device__ static void dec(u32x2 q, double s, double *d)
    {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            d[b] = dec_e4m3((q.x >> (8 * b)) & 0xFFu) * s;
            d[4 + b] = dec_e4m3((q.y >> (8 * b)) & 0xFFu) * s;
        }
    }
};

// Loads LW entries of w from i0 (entries >= n read as 0).
template <int LW>
__device__ __forceinline__ void load_wn(const double *__restrict__ w, int64_t n, int64_t i0,
                                        double *o)
{
    if constexpr (LW == 1) {
        o[0] = i0 < n ? w[i0] : 0.0;
    } else {
        load_w<LW>(w, n, i0, o);
    }
}
template <int LW>
__device__ __forceinline__ void store_wn(double *__restrict__ w, int64_t n, int64_t i0,
                                         const double *o)
{
    if constexpr (LW == 1) {
        if (i0 < n)
            w[i0] = o[0];
    } else {
        store_w<LW>(w, n, i0, o);
    }
}

constexpr int FUSED_JMAX = 104;     // largest j the fused pass takes

// Buffer resource word 3 for raw 32-bit accesses on gfx9-family parts.
constexpr int BUF_RSRC_W3 = 0x00020000;

template <int F, int JM>
__global__ __launch_bounds__(BLK) void k_update_redot(const uint8_t *__restrict__ V, int64_t ld,
                                                      const double *__restrict__ scales, int n,
                                                      int j, const double *__restrict__ coef,
                                                      double *__restrict__ w, RedArgs ra,
                                                      const DevState *st)
{
    if (st && st->done)
        return;
    using L = Lane8<F>;
    constexpr int LW = L::LW, KC = 8;
    constexpr int TILE = BLK * LW;
    constexpr bool SCALED = Fmt<F>::SCALED;
    constexpr uint32_t EB = fmt_bytes(F);
    const uint32_t ldb = (uint32_t)(ld * EB);
    __shared__ double wacc[NWAVE][JM];
    __shared__ double lh[JM], ls[JM];     // coefficients (0 beyond j) and scales
    for (int k = threadIdx.x; k < NWAVE * JM; k += BLK)
        (&wacc[0][0])[k] = 0.0;
    for (int k = threadIdx.x; k < JM; k += BLK) {
        lh[k] = k < j ? coef[k] : 0.0;
        ls[k] = (SCALED && k < j) ? scales[k] : 1.0;
    }
    __syncthreads();
    // The j stored vectors as one buffer of j*ldb bytes (the host checks that
    // JM*ldb fits in 32 bits): a load at or past the end returns 0, so the
    // vectors k >= j of the template's tile read as zero without a branch.
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)V, 0, (int)(j * ldb), BUF_RSRC_W3);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t ntiles = ((int64_t)n + TILE - 1) / TILE;
    double ssq = 0.0, mx = 0.0;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t i0 = tile * TILE + (int64_t)threadIdx.x * LW;
        // an opaque zero offset per tile: the JM coefficient and scale reads
        // stay inside the loop instead of being hoisted into 2*JM registers
        int z;
        asm volatile("s_mov_b32 %0, 0" : "=s"(z));
        const double *vh = lh + z, *vs = ls + z;
        // entries at or beyond n read as code 0: a chunk past n entirely, and
        // the tail of the chunk that straddles n
        uint64_t keep = 0ull;
        if (i0 < n)
            keep = i0 + LW <= n ? ~0ull : (1ull << (8 * EB * (n - i0))) - 1ull;
        const uint32_t voff = (uint32_t)((i0 < n ? i0 : 0) * EB);
        const uint32_t klo = (uint32_t)keep, khi = (uint32_t)(keep >> 32);
        u32x2 raw[JM];
#pragma unroll
        for (int k = 0; k < JM; ++k) {
            u32x2 q = __builtin_amdgcn_raw_buffer_load_b64(rs, voff + (uint32_t)k * ldb, 0, 0);
            q.x &= klo;
            q.y &= khi;
            raw[k] = q;
        }
        double wv[LW], sacc[LW];
        load_wn<LW>(w, n, i0, wv);
#pragma unroll
        for (int e = 0; e < LW; ++e)
            sacc[e] = 0.0;
        // update: s = sum_k h_k dec(V_k)   (h_k = 0 and V_k = 0 for k >= j)
#pragma unroll
        for (int k = 0; k < JM; ++k) {
            const double hk = vh[k];
            double d[LW];
            L::dec(raw[k], SCALED ? vs[k] : 1.0, d);
#pragma unroll
            for (int e = 0; e < LW; ++e)
                sacc[e] = fma(hk, d[e], sacc[e]);
            // decode in groups of 8: keeps decoded values from piling up
            if ((k & 7) == 7)
                __builtin_amdgcn_sched_barrier(0);
        }
        // only the raw bytes stay live into the re-dot (decoded again there)
#pragma unroll
        for (int k = 0; k < JM; ++k)
            asm volatile("" : "+v"(raw[k]));
#pragma unroll
        for (int e = 0; e < LW; ++e) {
            wv[e] = (i0 + e < n) ? wv[e] - sacc[e] : 0.0;
            ssq += wv[e] * wv[e];
            mx = fmax(mx, fabs(wv[e]));
        }
        store_wn<LW>(w, n, i0, wv);
        // re-dot of the updated rows, KC vectors per transposing reduction
#pragma unroll
        for (int kc = 0; kc < JM; kc += KC) {
            if (kc < j) {
                double acc[KC];
#pragma unroll
                for (int kk = 0; kk < KC; ++kk) {
                    double d[LW];
                    L::dec(raw[kc + kk], SCALED ? vs[kc + kk] : 1.0, d);
                    double a = 0.0;
#pragma unroll
                    for (int e = 0; e < LW; ++e)
                        a = fma(d[e], wv[e], a);
                    acc[kk] = a;
                }
                wave_transpose_sum<KC>(acc);
                if (lane < KC) {
                    const int k = kc + bitrev<KC>(lane);
                    if (k < j)
                        wacc[wave][k] += acc[0];
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < j; k += BLK) {
        double t = wacc[0][k];
#pragma unroll
        for (int q = 1; q < NWAVE; ++q)
            t += wacc[q][k];
        ra.part[(size_t)k * ra.stride + blockIdx.x] = t;
    }
    block_sum_max(ssq, mx);
    if (threadIdx.x == 0) {
        ra.part[(size_t)j * ra.stride + blockIdx.x] = ssq;
        ra.part[(size_t)(j + 1) * ra.stride + blockIdx.x] = mx;
    }
}

// ---------------------------------------------------------------------------
// Block-Jacobi right preconditioner with adaptive-precision storage (an
// extension: the paper discusses block-Jacobi preconditioners in Section 6;
// the selection rule is this project's own).  Block b covers the rows and
// columns [b*BS, min((b+1)*BS, n)); its inverse is stored in fp16, fp32 or
// fp64 (tag 16/32/64), in the array of that precision at b*BS*BS, row-major
// with row stride BS and zeros beyond the block's size.
// ---------------------------------------------------------------------------

// Gauss-Jordan inversion with partial pivoting, every operation a separate
// IEEE multiply, subtract or divide in a fixed order (the result is the same
// bits on any IEEE machine).  A ragged last block (sz < BS) is padded with
// identity rows and columns: padded rows are never pivots (their entries in
// the block's columns are 0) and elimination leaves them unchanged, so the
// top-left sz x sz of the result is the inverse of the block itself.
template <int BS>
__global__ __launch_bounds__(BLK) void k_bj_setup(int n, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci,
                                                  const double *__restrict__ val, int prec_min,
                                                  int8_t *__restrict__ tags,
                                                  double *__restrict__ x64,
                                                  float *__restrict__ x32,
                                                  uint16_t *__restrict__ x16,
                                                  unsigned *__restrict__ bad)
{
#pragma clang fp contract(off)
    const int nblk = (n + BS - 1) / BS;
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nblk; b += gridDim.x * blockDim.x) {
        const int i0 = b * BS;
        const int sz = min(BS, n - i0);
        double D[BS][BS], A0[BS][BS], X[BS][BS];
#pragma unroll
        for (int i = 0; i < BS; ++i)
#pragma unroll
            for (int k = 0; k < BS; ++k) {
                D[i][k] = (i == k && i >= sz) ? 1.0 : 0.0;
                X[i][k] = (i == k) ? 1.0 : 0.0;
            }
#pragma unroll
        for (int i = 0; i < BS; ++i) {
            if (i < sz) {
                for (int p = rp[i0 + i]; p < rp[i0 + i + 1]; ++p) {
                    const int c = ci[p] - i0;
                    const double a = val[p];
#pragma unroll
                    for (int k = 0; k < BS; ++k)
                        if (c == k && k < sz)
                            D[i][k] = a;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < BS; ++i)
#pragma unroll
            for (int k = 0; k < BS; ++k)
                A0[i][k] = D[i][k];
        bool singular = false;
#pragma unroll
        for (int c = 0; c < BS; ++c) {
            // pivot: the first row at or below c with the largest |entry|
            int r = c;
            double best = fabs(D[c][c]);
#pragma unroll
            for (int i = c + 1; i < BS; ++i)
                if (fabs(D[i][c]) > best) {
                    best = fabs(D[i][c]);
                    r = i;
                }
            if (best == 0.0)
                singular = true;
#pragma unroll
            for (int i = c + 1; i < BS; ++i) {
                if (i == r) {
#pragma unroll
                    for (int k = 0; k < BS; ++k) {
                        double t = D[c][k]; D[c][k] = D[i][k]; D[i][k] = t;
                        t = X[c][k]; X[c][k] = X[i][k]; X[i][k] = t;
                    }
                }
            }
            const double piv = D[c][c];
#pragma unroll
            for (int k = 0; k < BS; ++k) {
                D[c][k] = D[c][k] / piv;
                X[c][k] = X[c][k] / piv;
            }
#pragma unroll
            for (int i = 0; i < BS; ++i) {
                if (i == c)
                    continue;
                const double f = D[i][c];
#pragma unroll
                for (int k = 0; k < BS; ++k) {
                    const double pd = f * D[c][k];
                    D[i][k] = D[i][k] - pd;
                    const double px = f * X[c][k];
                    X[i][k] = X[i][k] - px;
                }
            }
        }
        if (singular) {
            *bad = 1u;
            tags[b] = 64;
            continue;
        }
        // kappa_1 = ||D_b||_1 ||D_b^-1||_1 over the block's own sz x sz
        double na = 0.0, nx = 0.0, mx = 0.0;
#pragma unroll
        for (int k = 0; k < BS; ++k) {
            double sa = 0.0, sx = 0.0;
#pragma unroll
            for (int i = 0; i < BS; ++i)
                if (i < sz && k < sz) {
                    sa = sa + fabs(A0[i][k]);
                    sx = sx + fabs(X[i][k]);
                    mx = fmax(mx, fabs(X[i][k]));
                }
            if (sa > na) na = sa;
            if (sx > nx) nx = sx;
        }
        const double kappa = na * nx;
        int pr = 64;
        if (prec_min <= 16 && kappa * 0x1p-11 <= 0.01 && mx <= 65504.0 && mx >= 0x1p-14)
            pr = 16;
        else if (prec_min <= 32 && kappa * 0x1p-24 <= 0.01 && mx <= 3.40282346638528859812e38 &&
                 mx >= 0x1p-126)
            pr = 32;
        tags[b] = (int8_t)pr;
        const size_t o = (size_t)b * BS * BS;
#pragma unroll
        for (int i = 0; i < BS; ++i)
#pragma unroll
            for (int k = 0; k < BS; ++k) {
                const double v = (i < sz && k < sz) ? X[i][k] : 0.0;
                if (pr == 16)
                    x16[o + i * BS + k] = (uint16_t)Fmt<F_FP16>::code(v, EncParam{1.0, 0});
                else if (pr == 32)
                    x32[o + i * BS + k] = (float)v;
                else
                    x64[o + i * BS + k] = v;
            }
    }
}

// Row i of the stored inverse of its block, widened to FP64.
__device__ __forceinline__ double bj_entry(int tag, size_t o, const double *__restrict__ x64,
                                           const float *__restrict__ x32,
                                           const uint16_t *__restrict__ x16)
{
    return tag == 16 ? dec_f16(x16[o]) : tag == 32 ? (double)x32[o] : x64[o];
}

// Fig. 1 steps 13-14 and 3 for block-Jacobi: v = w / t, stored as basis
// vector j through the accessor (rows up to ld, padding w = 0), and
// z = M^-1 v for the rows below n.  MODE 1 (no state): z = M^-1 w (or
// z += M^-1 w with accumulate), the kernel-level apply and the solution
// update.
__global__ __launch_bounds__(BLK) void k_bj_apply(int n, int64_t ldq, int bs,
                                                  const int8_t *__restrict__ tags,
                                                  const double *__restrict__ x64,
                                                  const float *__restrict__ x32,
                                                  const uint16_t *__restrict__ x16,
                                                  const double *__restrict__ w,
                                                  double *__restrict__ z, int accumulate,
                                                  const DevState *st, uint8_t *__restrict__ Q,
                                                  const double *__restrict__ qscale, int fmt,
                                                  int quant)
{
    double t = 1.0;
    EncParam ep{1.0, 0};
    if (st) {
        if (st->done)
            return;
        t = st->t;
        ep = param_from_scale(fmt, *qscale);
    }
    const int64_t rows = st ? ldq : n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (st)
            store_entry(fmt, Q, i, w[i] / t, ep);
        if (i >= n)
            continue;
        const int64_t b = i / bs, i0 = b * bs;
        const int sz = (int)min((int64_t)bs, (int64_t)n - i0);
        const int tag = tags[b];
        const size_t o = (size_t)b * bs * bs + (size_t)(i - i0) * bs;
        double s = 0.0;
        for (int l = 0; l < sz; ++l) {
            double v = st ? w[i0 + l] / t : w[i0 + l];
            if (quant)
                v = quantize(fmt, v, ep);
            s = fma(bj_entry(tag, o + l, x64, x32, x16), v, s);
        }
        z[i] = accumulate ? z[i] + s : s;
    }
}

// ---------------------------------------------------------------------------
// Modified Gram-Schmidt, one stored vector per launch (ablation of Fig. 1
// steps 5 and 8): launch k subtracts coef[k-1] dec(V_{k-1}) from w (k > 0)
// and forms block partials of dec(V_k)^T w with the updated w (k < j), or
// of ||w||^2 and max|w_i| (k = j).  A fold between launches turns the
// partials into coef[k].  j + 1 launches per pass instead of two basis
// passes: the cost of the sequential projections this variant studies.
// ---------------------------------------------------------------------------

template <int F>
__global__ __launch_bounds__(BLK) void k_mgs(const uint8_t *__restrict__ V, int64_t ld,
                                             const double *__restrict__ scales, int n, int k,
                                             int j, double *__restrict__ w,
                                             const double *__restrict__ coef, RedArgs ra,
                                             const DevState *st, int pass)
{
    if (st->done || (pass == 2 && !st->reorth))
        return;
    using T = Fmt<F>;
    constexpr int VW = T::VW;
    const int64_t ldb = ld * fmt_bytes(F);
    const double c = k > 0 ? coef[k - 1] : 0.0;
    const double sp = k > 0 ? scales[k - 1] : 1.0;
    const double sk = k < j ? scales[k] : 1.0;
    double acc = 0.0, mx = 0.0;
    const int64_t nch = ((int64_t)n + VW - 1) / VW;
    for (int64_t ch = blockIdx.x * (int64_t)BLK + threadIdx.x; ch < nch;
         ch += (int64_t)gridDim.x * BLK) {
        const int64_t i0 = ch * VW;               // i0 < n <= ld: the chunk is in the row
        double wv[VW], d[VW];
        load_w<VW>(w, n, i0, wv);                 // entries >= n read as 0
        if (k > 0) {
            T::dec(*(const u32x4 *)(V + (int64_t)(k - 1) * ldb + i0 * fmt_bytes(F)), sp, d);
#pragma unroll
            for (int e = 0; e < VW; ++e)
                wv[e] = wv[e] - c * d[e];
            store_w<VW>(w, n, i0, wv);            // entries >= n are not written
        }
        if (k < j) {
            T::dec(*(const u32x4 *)(V + (int64_t)k * ldb + i0 * fmt_bytes(F)), sk, d);
#pragma unroll
            for (int e = 0; e < VW; ++e)
                acc += d[e] * wv[e];              // padding codes decode to 0
        } else {
#pragma unroll
            for (int e = 0; e < VW; ++e) {
                acc += wv[e] * wv[e];
                mx = fmax(mx, fabs(wv[e]));
            }
        }
    }
    block_sum_max(acc, mx);
    if (threadIdx.x == 0) {
        ra.part[blockIdx.x] = acc;
        if (k == j)
            ra.part[(size_t)ra.stride + blockIdx.x] = mx;
    }
}

// ---------------------------------------------------------------------------
// One-block reductions of the producers' partials (fixed order: lane l sums
// blocks l, l+64, ... in turn, then a butterfly across the wave), followed
// by the scalar work that needs the totals.
// ---------------------------------------------------------------------------

// Roles (RR_* in the launch header):
//   RR_NB      ||b||: solve set-up
//   RR_SCALE   kernel-level encode: scale of a vector from max|v|
//   RR_NORM2   kernel-level SpMV: ||y||_2
//   RR_RESID   explicit residual: start of a restart cycle (Fig. 1 step 1)
//   RR_H       h = V^T w and omega (steps 4-5)
//   RR_U       u = V^T w, h_{j+1,j}, max|w|, and the test of step 7
//   RR_T2      after the re-orthogonalisation pass (steps 9-12)
//   RR_VALUES  kernel-level multi-dot
//   RR_NORMS   kernel-level update: ||w||_2, ||w||_inf
//   RR_MGS_H   MGS pass 1: one coefficient h_k into *out
//   RR_MGS_U   MGS pass 2: one coefficient u_k into *out
//   RR_MGS_T   end of MGS pass 1: as RR_U's scalars, from partials 0 and 1

// Block 0 does the scalars; block 1 + k folds value k (h_k, u_k or a
// kernel-level multi-dot value).
int reduce_grid(int role, int j)
{
    if (role == RR_H || role == RR_U || role == RR_VALUES || role == RR_UG)
        return 1 + (j > 0 ? j : 0);
    if (role == RR_HG)
        return 1 + 2 * (j > 0 ? j : 0);
    return 1;
}

__global__ __launch_bounds__(RBLK) void k_reduce(RedWs ws, int role, int nb_orth, int nb_spmv,
                                                 int j, DevState *st, StepArrays sa,
                                                 double *out, int fmt)
{
    if (role == RR_H || role == RR_U || role == RR_T2 || role >= RR_MGS_H) {
        if (st->done)
            return;
        if ((role == RR_T2 || role == RR_MGS_U) && !st->reorth)
            return;
    }
    if (role == RR_MGS_H || role == RR_MGS_U) {       // one value, one block
        const double a = block_fold(ws.orth, nb_orth, false);
        if (threadIdx.x == 0)
            *out = a;
        return;
    }
    const int tid = threadIdx.x;
    if (role == RR_HG && blockIdx.x > j) {
        // block 1 + j + k: g_k, mirrored into row and column j - 1 of G
        const int k = blockIdx.x - 1 - j;
        const double a = block_fold(ws.orth + (size_t)(j + 2 + k) * ws.stride, nb_orth, false);
        if (tid == 0) {
            const size_t ldg = (size_t)st->m + 1;
            sa.G[(size_t)(j - 1) * ldg + k] = a;
            sa.G[(size_t)k * ldg + (j - 1)] = a;
        }
        return;
    }
    if (role == RR_UG && blockIdx.x > 0) {
        // step 8 in Gram form: u_k = h_k - sum_l G_kl h_l (every step: the
        // test of step 7 is block 0's, and u is only read if it fired)
        __shared__ double prod[MAX_RESTART];
        const int k = blockIdx.x - 1;
        const size_t ldg = (size_t)st->m + 1;
        for (int l = tid; l < j; l += RBLK)
            prod[l] = sa.G[(size_t)k * ldg + l] * sa.h[l];
        __syncthreads();
        const double gh = block_fold(prod, j, false);
        if (tid == 0)
            sa.u[k] = sa.h[k] - gh;
        return;
    }
    // coefficients h_k / u_k / kernel-level values: block 1 + k folds value k
    if (blockIdx.x > 0) {
        const int k = blockIdx.x - 1;
        double *dst = (role == RR_H || role == RR_HG) ? sa.h : role == RR_U ? sa.u : out;
        const double a = block_fold(ws.orth + (size_t)k * ws.stride, nb_orth, false);
        if (tid == 0)
            dst[k] = a;
        return;
    }
    if (role == RR_VALUES)
        return;
    // the scalars (block 0): sum and max of a partial pair
    __shared__ double sv[2];
    const double *s0, *s1;
    int nb;
    if (role == RR_H || role == RR_HG) {
        s0 = ws.spmv;                                   // omega^2
        s1 = ws.spmv + ws.sstride;
        nb = nb_spmv;
    } else if (role == RR_U) {
        s0 = ws.orth + (size_t)j * ws.stride;           // ||w||^2, max|w_i|
        s1 = ws.orth + (size_t)(j + 1) * ws.stride;
        nb = nb_orth;
    } else if (role == RR_C2) {
        // the one-pass update's norms (rows 0, 1), or a hard step's second
        // pass (rows j+2, j+3, from its smaller grid)
        const int row = st->hard ? j + 2 : 0;
        s0 = ws.orth + (size_t)row * ws.stride;
        s1 = ws.orth + (size_t)(row + 1) * ws.stride;
        nb = st->hard ? min(nb_orth, HARD_BLOCKS) : nb_orth;
    } else if (role == RR_T2 || role == RR_NORMS || role == RR_MGS_T || role == RR_UG) {
        s0 = ws.orth;
        s1 = ws.orth + ws.stride;
        nb = nb_orth;
    } else {
        s0 = ws.spmv;
        s1 = ws.spmv + ws.sstride;
        nb = nb_spmv;
    }
    {
        const double a0 = block_fold(s0, nb, false);
        const double a1 = block_fold(s1, nb, true);
        if (tid == 0) {
            sv[0] = a0;
            sv[1] = a1;
        }
    }
    __syncthreads();
    switch (role) {
    case RR_NB:
        if (tid == 0) {
            const double nbv = sqrt(sv[0]);
            st->nb = nbv;
            st->tau_nb = st->tau_nb * nbv;
            if (!isfinite(nbv))
                st->nonfinite = 1;
        }
        break;
    case RR_SCALE:
        if (tid == 0)
            *out = make_param(fmt, sv[1]).scale;
        break;
    case RR_NORM2:
        if (tid == 0)
            *out = sqrt(sv[0]);
        break;
    case RR_NORMS:
        if (tid == 0 && out) {
            out[0] = sqrt(sv[0]);
            out[1] = sv[1];
        }
        break;
    case RR_RESID: {
        const double beta = sqrt(sv[0]);
        const int m = st->m;
        for (int i = tid; i < m + 2; i += RBLK)
            sa.g[i] = 0.0;
        __syncthreads();
        if (tid == 0) {
            st->jprev = st->jeff;
            st->beta = beta;
            st->rmax = sv[1];
            st->t = beta;
            st->done = 0;
            st->jeff = 0;
            st->reorth = 0;
            st->conv = 0;
            sa.g[0] = beta;
            if (!isfinite(beta))
                st->nonfinite = 1;
            sa.scales[0] = beta > 0.0 ? make_param(st->fmt, sv[1] / beta).scale : 1.0;
        }
        break;
    }
    case RR_H:
    case RR_HG:
        if (tid == 0)
            st->omega = sqrt(sv[0]);
        break;
    case RR_U:
    case RR_UG:
    case RR_MGS_T: {
        // Fig. 1 steps 6-7; without re-orthogonalisation the step ends here
        // (finish_step needs h, which the previous kernel stored, not u)
        const double t = sqrt(sv[0]);
        const bool ro = st->reorth_all || t < st->eta * st->omega;
        __syncthreads();
        if (tid == 0) {
            st->t = t;
            st->wmax = sv[1];
            st->reorth = ro ? 1 : 0;
        }
        __syncthreads();
        if (!ro)
            finish_step(st, sa, j, false, 0.0, 0.0);
        break;
    }
    case RR_T2:
        finish_step(st, sa, j, true, sqrt(sv[0]), sv[1]);
        break;
    case RR_C2:
        // the one-pass update's norms: with re-orthogonalisation the closing
        // norm against t1 (which the update stored), else the step's t.  A
        // hard step without re-orthogonalisation has its t and max|w| from
        // the second-pass kernel already.
        // The column was rotated by the update's column block.
        if (st->reorth) {
            finish_step(st, sa, j, true, sqrt(sv[0]), sv[1], true);
        } else {
            __syncthreads();
            if (tid == 0 && !st->hard) {
                st->t = sqrt(sv[0]);
                st->wmax = sv[1];
            }
            __syncthreads();
            finish_step(st, sa, j, false, 0.0, 0.0, true);
        }
        break;
    }
}

// ---------------------------------------------------------------------------
// Normalise and store through the accessor (Fig. 1 steps 13-14):
// v = w / t (IEEE division), v_out = v (FP64, the next SpMV input) and
// Q = enc(v) with the slot's scale.  Entries in [n, nst) are stored as 0.
// ---------------------------------------------------------------------------

template <int F>
__global__ __launch_bounds__(BLK) void k_normalize(const double *__restrict__ w, int n,
                                                   int64_t nst, double *__restrict__ v_out,
                                                   uint8_t *__restrict__ Q,
                                                   const double *__restrict__ scale_slot,
                                                   const double *__restrict__ tptr, double tval,
                                                   const DevState *st, int check_done, int fmt)
{
    if (check_done && st->done)
        return;
    using T = Fmt<F>;
    constexpr int VW = T::VW;
    const double t = tptr ? *tptr : tval;
    const EncParam p = param_from_scale(fmt, *scale_slot);
    const int64_t nchunks = (nst + VW - 1) / VW;
    for (int64_t c = blockIdx.x * (int64_t)BLK + threadIdx.x; c < nchunks;
         c += (int64_t)gridDim.x * BLK) {
        const int64_t i0 = c * VW;
        double v[VW];
        load_w<VW>(w, n, i0, v);
#pragma unroll
        for (int e = 0; e < VW; ++e)
            v[e] = v[e] / t;
        if (v_out)
            store_w<VW>(v_out, nst, i0, v);
        u32x4 q = T::enc(v, p);
        if (i0 + VW <= nst) {
            *(u32x4 *)(Q + i0 * fmt_bytes(F)) = q;
        } else {
            const uint8_t *qb = (const uint8_t *)&q;
            for (int64_t b = 0; b < (nst - i0) * fmt_bytes(F); ++b)
                Q[i0 * fmt_bytes(F) + b] = qb[b];
        }
    }
}

// Steps 13-14 of the previous Arnoldi step as a pass of their own, for
// matrices whose rows are long enough that dividing each gathered entry by t
// inside the next SpMV costs more than one extra sweep of v: v = w / t (IEEE
// division, the bits the gather forms), stored through the accessor, and
// written out as z = v, or z = dinv .* v for the Jacobi preconditioner (the
// product the gather forms, so that step 3 runs as the plain SpMV).
// Each thread owns NP pairs of consecutive entries, BLK pairs apart: every
// load and store of a wave is contiguous, and all NP loads are issued before
// the first division.
template <int F>
__device__ __forceinline__ void store_pair(uint8_t *__restrict__ Q, int64_t i, double a, double b,
                                           EncParam p)
{
    if constexpr (F == F_FP64) {
        f64x2 v = {a, b};
        *(f64x2 *)(Q + i * 8) = v;
    } else if constexpr (F == F_FP32) {
        u32x2 v = {__float_as_uint((float)a), __float_as_uint((float)b)};
        *(u32x2 *)(Q + i * 4) = v;
    } else if constexpr (F == F_INT32) {
        u32x2 v = {Fmt<F_INT32>::code(a, p), Fmt<F_INT32>::code(b, p)};
        *(u32x2 *)(Q + i * 4) = v;
    } else if constexpr (F == F_E4M3) {
        *(uint16_t *)(Q + i) = (uint16_t)(Fmt<F>::code(a, p) | (Fmt<F>::code(b, p) << 8));
    } else {
        *(uint32_t *)(Q + i * 2) = Fmt<F>::code(a, p) | (Fmt<F>::code(b, p) << 16);
    }
}

template <int F>
__global__ __launch_bounds__(BLK) void k_step_normalize(const double *__restrict__ w, int n,
                                                        int64_t ld, const double *__restrict__ dinv,
                                                        double *__restrict__ z,
                                                        uint8_t *__restrict__ Q,
                                                        const double *__restrict__ scale_slot,
                                                        const DevState *st)
{
    constexpr int NP = 4;
    if (st->done)
        return;
    const double t = st->t;
    const EncParam p = param_from_scale(F, *scale_slot);
    const int64_t npair = ld / 2;                         // ld is a multiple of 16
    for (int64_t base = blockIdx.x * (int64_t)(BLK * NP); base < npair;
         base += (int64_t)gridDim.x * BLK * NP) {
        f64x2 v[NP], d[NP];
#pragma unroll
        for (int u = 0; u < NP; ++u) {
            const int64_t q = base + u * BLK + threadIdx.x;
            const int64_t i = 2 * q;
            if (q < npair && i + 1 < n) {
                v[u] = *(const f64x2 *)(w + i);
            } else {
                v[u].x = q < npair && i < n ? w[i] : 0.0;  // entries >= n are 0
                v[u].y = 0.0;
            }
            if (dinv && q < npair)
                d[u] = *(const f64x2 *)(dinv + i);        // dinv holds 0 beyond n
        }
#pragma unroll
        for (int u = 0; u < NP; ++u) {
            const int64_t q = base + u * BLK + threadIdx.x;
            if (q >= npair)
                continue;
            const double a = v[u].x / t, b = v[u].y / t;
            store_pair<F>(Q, 2 * q, a, b, p);
            f64x2 o = {a, b};
            if (dinv) {
                o.x = d[u].x * a;
                o.y = d[u].y * b;
            }
            *(f64x2 *)(z + 2 * q) = o;
        }
    }
}

// The learned preconditioner in its stored form (CBG_PC_STENCIL): on an
// nx x ny x nz grid, row i's 27 slots carry float16 codes o (slot-major, row
// stride ld) and
//   z_i = dinv_i * (sum_p c_p w_(i + off_p)) / t,   c_p = [p = 13] + o_p,
// over the slots whose grid point exists, in slot order.  ST_STEP: w is the
// step's orthogonalised vector and t = h_{j+1,j}, so z = M^-1 v with v = w / t
// (one division per row instead of one per term; with all codes 0 this is
// the Jacobi pass's z bit for bit), and v_j = w / t is stored through the
// accessor for rows [0, ld) as in k_step_normalize (z written for all ld
// rows, 0 beyond n).  ST_PLAIN: z = M^-1 w and ST_ACC: z += M^-1 w (the
// solution update), both for rows < n only.
//
// A block takes a tile of BLK consecutive rows, one row per thread.  The
// tile's nine (dy, dz) neighbour lines of w, each BLK + 2 entries (dx = -1
// .. +1), are staged in LDS first: nine coalesced loads per thread, issued
// together with the row's 27 code loads, then one barrier.  The slot sums
// then read LDS only, so a wave has all of its global loads in flight at
// once instead of waiting on one plane of gathers after another.  Entries
// outside [0, n) are staged as 0; only absent slots (weight 0) read them.
enum { ST_STEP = 0, ST_PLAIN = 1, ST_ACC = 2 };
constexpr int ST_LINE = BLK + 2;

template <int F, int MODE, bool BUF>
__global__ __launch_bounds__(BLK) void k_stencil(const double *__restrict__ w, int n, int64_t ld,
                                                 int nx, int ny, int nz,
                                                 const uint16_t *__restrict__ codes,
                                                 const double *__restrict__ dinv,
                                                 double *__restrict__ z, uint8_t *__restrict__ Q,
                                                 const double *__restrict__ scale_slot,
                                                 const DevState *st)
{
    double t = 1.0;
    EncParam ep{1.0, 0};
    if constexpr (MODE == ST_STEP) {
        if (st->done)
            return;
        t = st->t;
        ep = param_from_scale(F, *scale_slot);
    }
    __shared__ double lw[9][ST_LINE];
    const int tid = threadIdx.x;
    const int64_t S = (int64_t)nx * ny;
    const int64_t ntiles = (ld + BLK - 1) / BLK;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t r0 = tile * BLK, i = r0 + tid;
        const bool live = i < n;
        // every load unconditional, so that all of them are in flight
        // together; values read for rows >= n or outside the grid only meet
        // weight 0
        const int64_t ic = min(i, (int64_t)n - 1);
        uint32_t cc[27];
        // the nine lines, 9 x ST_LINE entries, in flat order: entry f of
        // the staging goes to line f / ST_LINE, position f % ST_LINE
        constexpr int NLD = (9 * ST_LINE + BLK - 1) / BLK;
        double lv[NLD];
        if constexpr (BUF) {
            // buffer loads: the codes' slot offset in a scalar register
            // (one vector offset for all 27), and w's line entries outside
            // [0, n) returned as 0 by the buffer's range check
            const __amdgpu_buffer_rsrc_t rc =
                __builtin_amdgcn_make_buffer_rsrc((void *)codes, 0, (int)(27 * ld * 2), BUF_RSRC_W3);
            const __amdgpu_buffer_rsrc_t rw =
                __builtin_amdgcn_make_buffer_rsrc((void *)w, 0, (int)((int64_t)n * 8), BUF_RSRC_W3);
            const uint32_t vo = (uint32_t)ic * 2u;
#pragma unroll
            for (int p = 0; p < 27; ++p)
                cc[p] = __builtin_amdgcn_raw_buffer_load_b16(rc, vo, (int)(p * ld * 2), 0);
#pragma unroll
            for (int q = 0; q < NLD; ++q) {
                const int f = min(tid + q * BLK, 9 * ST_LINE - 1);
                const int k = f / ST_LINE, e = f - k * ST_LINE;
                const int64_t g = r0 + (k / 3 - 1) * S + (k % 3 - 1) * (int64_t)nx - 1 + e;
                lv[q] = __builtin_bit_cast(
                    double, __builtin_amdgcn_raw_buffer_load_b64(rw, (uint32_t)(g * 8), 0, 0));
            }
        } else {
            // indices clamped into the arrays
#pragma unroll
            for (int p = 0; p < 27; ++p)
                cc[p] = codes[(int64_t)p * ld + ic];
#pragma unroll
            for (int q = 0; q < NLD; ++q) {
                const int f = min(tid + q * BLK, 9 * ST_LINE - 1);
                const int k = f / ST_LINE, e = f - k * ST_LINE;
                const int64_t g = r0 + (k / 3 - 1) * S + (k % 3 - 1) * (int64_t)nx - 1 + e;
                lv[q] = w[min(max(g, (int64_t)0), (int64_t)n - 1)];
            }
        }
        __syncthreads();                            // lw free from the previous tile
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
            const int f = tid + q * BLK;
            if (f < 9 * ST_LINE)
                (&lw[0][0])[f] = lv[q];
        }
        // which of the three offsets along each axis exist for this row
        const uint32_t u = live ? (uint32_t)i : 0u, row = u / (uint32_t)nx;
        const int gx = (int)(u - row * (uint32_t)nx), gy = (int)(row % (uint32_t)ny),
                  gz = (int)(row / (uint32_t)ny);
        const uint32_t mx = 2u | (gx > 0 ? 1u : 0u) | (gx < nx - 1 ? 4u : 0u);
        const uint32_t my = 2u | (gy > 0 ? 1u : 0u) | (gy < ny - 1 ? 4u : 0u);
        const uint32_t mz = 2u | (gz > 0 ? 1u : 0u) | (gz < nz - 1 ? 4u : 0u);
        __syncthreads();                            // the lines are staged
        double s = 0.0;
#pragma unroll
        for (int p = 0; p < 27; ++p) {
            const int dz = p / 9 - 1, dy = (p / 3) % 3 - 1, dx = p % 3 - 1;
            const bool in = live && ((mx >> (dx + 1)) & (my >> (dy + 1)) & (mz >> (dz + 1)) & 1u);
            const double c = (p == 13 ? 1.0 : 0.0) + dec_f16(cc[p]);
            s = fma(in ? c : 0.0, lw[p / 3][tid + dx + 1], s);
        }
        if constexpr (MODE == ST_ACC) {
            if (live)
                z[i] = fma(dinv[i], s, z[i]);           // as x += dinv .* s
        } else if constexpr (MODE == ST_PLAIN) {
            if (live)
                z[i] = dinv[i] * s;
        } else if (i < ld) {
            z[i] = live ? dinv[i] * (s / t) : 0.0;      // dinv holds 0 beyond n
            store_entry(F, Q, i, live ? lw[4][tid + 1] / t : 0.0, ep);
        }
    }
}

// The accessor's load for the kernel-level API: v = dec(q) exactly.
template <int F>
__global__ __launch_bounds__(BLK) void k_decode(const uint8_t *__restrict__ Q, int n,
                                                const double *__restrict__ scale,
                                                double *__restrict__ v)
{
    using T = Fmt<F>;
    constexpr int VW = T::VW;
    const double s = T::SCALED ? *scale : 1.0;
    const int64_t nchunks = ((int64_t)n + VW - 1) / VW;
    for (int64_t c = blockIdx.x * (int64_t)BLK + threadIdx.x; c < nchunks;
         c += (int64_t)gridDim.x * BLK) {
        const int64_t i0 = c * VW;
        double d[VW];
        if (i0 + VW <= n) {
            u32x4 q = *(const u32x4 *)(Q + i0 * fmt_bytes(F));
            T::dec(q, s, d);
        } else {
            u32x4 q = {0u, 0u, 0u, 0u};
            uint8_t *qb = (uint8_t *)&q;
            for (int64_t b = 0; b < (n - i0) * fmt_bytes(F); ++b)
                qb[b] = Q[i0 * fmt_bytes(F) + b];
            T::dec(q, s, d);
        }
        store_w<VW>(v, n, i0, d);
    }
}

// Back substitution R y = g for the cycle's least-squares problem (Fig. 1
// step 17); R is the rotated Hessenberg matrix.  One wavefront, column
// oriented: y_i = g_i / R_ii, then g_k -= R_ki y_i for k < i in parallel.
__global__ __launch_bounds__(64) void k_backsolve(const DevState *st, StepArrays sa)
{
    __shared__ double gl[MAX_RESTART + 2];
    __shared__ double yi;
    const int jeff = st->jeff, m = st->m;
    for (int i = threadIdx.x; i < jeff; i += 64)
        gl[i] = sa.g[i];
    __syncthreads();
    for (int i = jeff - 1; i >= 0; --i) {
        if (threadIdx.x == 0) {
            yi = gl[i] / sa.H[(size_t)i * (m + 1) + i];
            sa.y[i] = yi;
        }
        __syncthreads();
        const double* Hi = sa.H + (size_t)i * (m + 1);
        for (int k = threadIdx.x; k < i; k += 64)
            gl[k] -= Hi[k] * yi;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------

static int grid_for(int64_t work_items, int per_block)
{
    int64_t g = (work_items + per_block - 1) / per_block;
    if (g < 1)
        g = 1;
    if (g > MAX_GRID)
        g = MAX_GRID;
    return (int)g;
}

// Launch shape of the CSR-stream SpMV from the mean row length: rows per
// block and the LDS product buffer (entries), sized so a block's products
// fit it at up to about 8, 32 and 64 entries per row.  A smaller buffer
// lets more blocks share a CU: on the 27-point stencil (26.6 per row) 64
// rows with 2048 entries run 15% faster than 128 rows with 4096.
int spmv_shape_of(int n, int64_t nnz)
{
    double avg = n > 0 ? (double)nnz / n : 1.0;
    if (avg <= 7.5) return SPMV_R256_C2K;
    if (avg <= 30.0) return SPMV_R64_C2K;
    if (avg <= 60.0) return SPMV_R64_C4K;
    return SPMV_R32_C4K;
}

int spmv_rows(int shape)
{
    switch (shape) {
    case SPMV_R256_C2K: return 256;
    case SPMV_R32_C4K: return 32;
    default: return 64;
    }
}

template <int RPB, int CAP>
static int spmv_shape(const SpmvArgs &a, hipStream_t s)
{
    int g = grid_for((a.ldy + RPB - 1) / RPB, 1);
    RedArgs ra{a.ws.spmv, a.ws.sstride};
#define CBG_SPMV_CASE(M)                                                                      \
    case M:                                                                                   \
        if (a.ev0)                                                                            \
            hipExtLaunchKernelGGL(k_spmv<RPB, CAP, M>, dim3(g), dim3(BLK), 0, s, a.ev0, a.ev1, \
                                  0, a.n, a.ldy, a.rp, a.ci, a.val, a.fval, a.x, a.dinv, a.b, \
                                  a.y, ra, a.role, a.st, (uint8_t *)a.Q, a.qscale, a.fmt);    \
        else                                                                                  \
            k_spmv<RPB, CAP, M><<<g, BLK, 0, s>>>(a.n, a.ldy, a.rp, a.ci, a.val, a.fval, a.x, \
                                                   a.dinv, a.b, a.y, ra, a.role, a.st,        \
                                                   (uint8_t *)a.Q, a.qscale, a.fmt);          \
        break;
    switch (a.mode) {
        CBG_SPMV_CASE(SP_PLAIN)
        CBG_SPMV_CASE(SP_JACOBI)
        CBG_SPMV_CASE(SP_RESID)
        CBG_SPMV_CASE(SP_FLOATVAL)
        CBG_SPMV_CASE(SP_ACCUM)
        CBG_SPMV_CASE(SP_STEP_PLAIN)
        CBG_SPMV_CASE(SP_STEP_JACOBI)
        CBG_SPMV_CASE(SP_STEP_FLOATVAL)
        CBG_SPMV_CASE(SP_STEP_PLAIN_Q)
        CBG_SPMV_CASE(SP_STEP_JACOBI_Q)
        CBG_SPMV_CASE(SP_STEP_FLOATVAL_Q)
    }
#undef CBG_SPMV_CASE
    return g;
}

template <int RPB, int CAP>
static int spmv_rp_shape(const SpmvArgs &a, hipStream_t s)
{
    int g = grid_for((a.ldy + RPB - 1) / RPB, 1);
    RedArgs ra{a.ws.spmv, a.ws.sstride};
#define CBG_SPMV_CASE(M)                                                                      \
    case M:                                                                                   \
        if (a.ev0)                                                                            \
            hipExtLaunchKernelGGL(k_spmv_rp<RPB, CAP, M>, dim3(g), dim3(BLK), 0, s, a.ev0,     \
                                  a.ev1, 0, a.n, a.ldy, a.rp, a.ci, a.val, a.fval, a.x,       \
                                  a.dinv, a.b, a.y, ra, a.role, a.st, (uint8_t *)a.Q,         \
                                  a.qscale, a.fmt);                                           \
        else                                                                                  \
            k_spmv_rp<RPB, CAP, M><<<g, BLK, 0, s>>>(a.n, a.ldy, a.rp, a.ci, a.val, a.fval,   \
                                                      a.x, a.dinv, a.b, a.y, ra, a.role, a.st, \
                                                      (uint8_t *)a.Q, a.qscale, a.fmt);        \
        break;
    switch (a.mode) {
        CBG_SPMV_CASE(SP_PLAIN)
        CBG_SPMV_CASE(SP_JACOBI)
        CBG_SPMV_CASE(SP_RESID)
        CBG_SPMV_CASE(SP_FLOATVAL)
        CBG_SPMV_CASE(SP_ACCUM)
        CBG_SPMV_CASE(SP_STEP_PLAIN)
        CBG_SPMV_CASE(SP_STEP_JACOBI)
        CBG_SPMV_CASE(SP_STEP_FLOATVAL)
        CBG_SPMV_CASE(SP_STEP_PLAIN_Q)
        CBG_SPMV_CASE(SP_STEP_JACOBI_Q)
        CBG_SPMV_CASE(SP_STEP_FLOATVAL_Q)
    }
#undef CBG_SPMV_CASE
    return g;
}

static int spmv_sell(const SpmvArgs &a, hipStream_t s)
{
    // long rows (more than 12 per row): up to SPMV_MAX_GRID blocks, which
    // measured 2% faster on the 27-point rows at 160^3; short rows keep
    // MAX_GRID (8192 blocks were 3% slower on the 7-point rows at 128^3,
    // the fold of their partials included)
    const int64_t nsy = (a.ldy + 63) / 64;
    const int g = (int)std::min<int64_t>(std::max<int64_t>((nsy + NWAVE - 1) / NWAVE, 1),
                                         a.sell_nt ? SPMV_MAX_GRID : MAX_GRID);
    RedArgs ra{a.ws.spmv, a.ws.sstride};
#define CBG_SELL_LAUNCH(M, NT, DX)                                                             \
    if (a.ev0)                                                                                 \
        hipExtLaunchKernelGGL(k_spmv_sell<M, NT, DX>, dim3(g), dim3(BLK), 0, s, a.ev0, a.ev1,  \
                              0, a.n, a.ldy, a.nslice, a.sp, a.sc, a.sd, a.sdiag, a.ndiag,     \
                              a.sv, a.x, a.dinv, a.b, a.y, ra, a.role, a.st, (uint8_t *)a.Q,   \
                              a.qscale, a.fmt);                                                \
    else                                                                                       \
        k_spmv_sell<M, NT, DX><<<g, BLK, 0, s>>>(a.n, a.ldy, a.nslice, a.sp, a.sc, a.sd,       \
                                                 a.sdiag, a.ndiag, a.sv, a.x, a.dinv, a.b,     \
                                                 a.y, ra, a.role, a.st, (uint8_t *)a.Q,        \
                                                 a.qscale, a.fmt);
#define CBG_SELL_CASE(M)                                                                       \
    case M:                                                                                    \
        if (a.sd) {                                                                            \
            if (a.sell_nt) {                                                                   \
                CBG_SELL_LAUNCH(M, true, true)                                                 \
            } else {                                                                           \
                CBG_SELL_LAUNCH(M, false, true)                                                \
            }                                                                                  \
        } else if (a.sell_nt) {                                                                \
            CBG_SELL_LAUNCH(M, true, false)                                                    \
        } else {                                                                               \
            CBG_SELL_LAUNCH(M, false, false)                                                   \
        }                                                                                      \
        break;
    switch (a.mode) {
        CBG_SELL_CASE(SP_PLAIN)
        CBG_SELL_CASE(SP_JACOBI)
        CBG_SELL_CASE(SP_RESID)
        CBG_SELL_CASE(SP_STEP_PLAIN)
        CBG_SELL_CASE(SP_STEP_JACOBI)
        CBG_SELL_CASE(SP_STEP_PLAIN_Q)
        CBG_SELL_CASE(SP_STEP_JACOBI_Q)
    }
#undef CBG_SELL_CASE
#undef CBG_SELL_LAUNCH
    return g;
}

bool sell_takes(int mode)
{
    const int base = mode & 7;
    return base == SP_PLAIN || base == SP_JACOBI || base == SP_RESID;
}

void launch_sell_ptr(int n, const int32_t *rp, int64_t nslice, int64_t *sp, hipStream_t s)
{
    k_sell_width<<<grid_for((nslice + NWAVE - 1) / NWAVE, 1), BLK, 0, s>>>(n, rp, nslice, sp);
    k_sell_scan<<<1, SCAN_BLK, 0, s>>>(nslice, sp);
}

int launch_sell_diag(int n, int64_t nslice, const int64_t *sp, const int32_t *sc, int32_t *diag,
                     uint8_t *sd, void *ws, hipStream_t s, int32_t *count_host)
{
    // ws: the hash table, the overflow flag and the count
    int32_t *hash = (int32_t *)ws;
    unsigned *full = (unsigned *)(hash + DIAG_HASH);
    int32_t *count = (int32_t *)(full + 1);
    k_fill_i32<<<grid_for(DIAG_HASH + 2, 256), 256, 0, s>>>(hash, DIAG_HASH + 2, DIAG_EMPTY);
    k_fill_i32<<<1, 64, 0, s>>>((int32_t *)full, 1, 0);
    const int g = grid_for((nslice + NWAVE - 1) / NWAVE, 1);
    k_diag_insert<<<g, BLK, 0, s>>>(n, nslice, sp, sc, hash, full);
    k_diag_collect<<<1, BLK, 0, s>>>(hash, full, diag, count);
    if (hipMemcpyAsync(count_host, count, sizeof(int32_t), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return -1;
    if (*count_host < 1 || *count_host > SELL_MAX_DIAG)
        return 1;
    k_diag_index<<<g, BLK, 0, s>>>(n, nslice, sp, sc, diag, *count_host, sd);
    return 0;
}

void launch_sell_fill(int n, const int32_t *rp, const int32_t *ci, const double *val,
                      int64_t nslice, const int64_t *sp, int32_t *sc, double *sv, hipStream_t s)
{
    k_sell_fill<<<grid_for((nslice + NWAVE - 1) / NWAVE, 1), BLK, 0, s>>>(n, rp, ci, val, nslice,
                                                                           sp, sc, sv);
}

int launch_spmv(const SpmvArgs &a, hipStream_t s)
{
    if (a.sp && sell_takes(a.mode))
        return spmv_sell(a, s);
    switch (a.sg) {
    case SPMV_R256_C2K: return spmv_shape<256, 2048>(a, s);
    case SPMV_R64_C2K: return spmv_shape<64, 2048>(a, s);
    case SPMV_R64_C4K: return spmv_shape<64, 4096>(a, s);
    case SPMV_RP64_C2K: return spmv_rp_shape<64, 2048>(a, s);
    default: return spmv_shape<32, 4096>(a, s);
    }
}

int spmv_grid(int shape, int64_t ldy)
{
    const int r = spmv_rows(shape);
    return grid_for((ldy + r - 1) / r, 1);
}

template <int F>
static int tile_elems() { return BLK * Fmt<F>::VW * Fmt<F>::CH; }

#define CBG_FMT_SWITCH(fmt, CALL)                  \
    switch (fmt) {                                 \
    case F_FP64: { constexpr int F = F_FP64; CALL; } break; \
    case F_FP32: { constexpr int F = F_FP32; CALL; } break; \
    case F_FP16: { constexpr int F = F_FP16; CALL; } break; \
    case F_BF16: { constexpr int F = F_BF16; CALL; } break; \
    case F_E4M3: { constexpr int F = F_E4M3; CALL; } break; \
    case F_INT32: { constexpr int F = F_INT32; CALL; } break; \
    case F_FP16S: { constexpr int F = F_FP16S; CALL; } break; \
    default: { constexpr int F = F_INT16; CALL; } break;    \
    }

int launch_bj_setup(int n, const int32_t *rp, const int32_t *ci, const double *val, int bs,
                    int prec_min, int8_t *tags, double *x64, float *x32, uint16_t *x16,
                    unsigned *bad, hipStream_t s)
{
    const int nblk = (n + bs - 1) / bs;
    const int g = grid_for(nblk, BLK);
#define CBG_BJ_CASE(B)                                                                      \
    case B:                                                                                 \
        k_bj_setup<B><<<g, BLK, 0, s>>>(n, rp, ci, val, prec_min, tags, x64, x32, x16, bad); \
        break;
    switch (bs) {
        CBG_BJ_CASE(1) CBG_BJ_CASE(2) CBG_BJ_CASE(3) CBG_BJ_CASE(4)
        CBG_BJ_CASE(5) CBG_BJ_CASE(6) CBG_BJ_CASE(7) CBG_BJ_CASE(8)
    default: return -1;
    }
#undef CBG_BJ_CASE
    return 0;
}

void launch_bj_apply(int n, int64_t ldq, int bs, const int8_t *tags, const double *x64,
                     const float *x32, const uint16_t *x16, const double *w, double *z,
                     int accumulate, const DevState *st, void *Q, const double *qscale, int fmt,
                     int quant, hipStream_t s)
{
    const int64_t rows = st ? ldq : n;
    k_bj_apply<<<grid_for(rows, BLK), BLK, 0, s>>>(n, ldq, bs, tags, x64, x32, x16, w, z,
                                                    accumulate, st, (uint8_t *)Q, qscale, fmt,
                                                    st ? quant : 0);
}

int orth_grid(int fmt, int64_t n)
{
    int tile = 0;
    CBG_FMT_SWITCH(fmt, (tile = tile_elems<F>()))
    return grid_for(n, tile);
}

// With events, the launch goes through hipExtLaunchKernelGGL, which records
// them at the kernel's own start and end (the interval a profiler reports).
void launch_multidot(const OrthArgs &a, hipStream_t s)
{
    int g = orth_grid(a.fmt, a.n);
    RedArgs ra{a.ws.orth, a.ws.stride};
    const uint8_t *V = (const uint8_t *)a.V;
#define CBG_MD(G)                                                                              \
    if (a.ev0) {                                                                               \
        CBG_FMT_SWITCH(a.fmt, (hipExtLaunchKernelGGL(k_multidot<F, G>, dim3(g), dim3(BLK), 0, s, \
                                                     a.ev0, a.ev1, 0, V, a.ld, a.scales, a.n,  \
                                                     a.j, a.w, ra, a.st, a.gated,              \
                                                     a.with_norms)))                           \
    } else {                                                                                   \
        CBG_FMT_SWITCH(a.fmt, (k_multidot<F, G><<<g, BLK, 0, s>>>(V, a.ld, a.scales, a.n, a.j,  \
                                                                   a.w, ra, a.st, a.gated,     \
                                                                   a.with_norms)))             \
    }
    if (a.gram) {
        CBG_MD(true)
    } else {
        CBG_MD(false)
    }
#undef CBG_MD
}

void launch_update(const OrthArgs &a, hipStream_t s)
{
    // the one-pass roles run one block more: the column block
    const bool onepass = a.role == U_CGS2 || a.role == U_HARD;
    const int g0 = orth_grid(a.fmt, a.n);
    const int g = (a.role == U_HARD ? min(g0, HARD_BLOCKS) : g0) + (onepass ? 1 : 0);
    RedArgs ra{a.ws.orth, a.ws.stride};
    const uint8_t *V = (const uint8_t *)a.V;
    StepArrays sa{};
    if (a.sa)
        sa = *(const StepArrays *)a.sa;
#define CBG_UPD(R)                                                                            \
    if (a.ev0) {                                                                              \
        CBG_FMT_SWITCH(a.fmt, (hipExtLaunchKernelGGL(k_update<F, R>, dim3(g), dim3(BLK), 0, s, \
                                                     a.ev0, a.ev1, 0, V, a.ld, a.scales, a.n, \
                                                     a.j, a.coef, a.wio, a.dinv, ra, a.st,    \
                                                     a.u, a.stw, a.G, sa, g0)))               \
    } else {                                                                                  \
        CBG_FMT_SWITCH(a.fmt, (k_update<F, R><<<g, BLK, 0, s>>>(V, a.ld, a.scales, a.n, a.j,   \
                                                                 a.coef, a.wio, a.dinv, ra,   \
                                                                 a.st, a.u, a.stw, a.G, sa,   \
                                                                 g0)))                        \
    }
    switch (a.role) {
    case U_PLAIN: CBG_UPD(U_PLAIN) break;
    case U_STEP1: CBG_UPD(U_STEP1) break;
    case U_STEP2: CBG_UPD(U_STEP2) break;
    case U_STEP1N: CBG_UPD(U_STEP1N) break;
    case U_CGS2: CBG_UPD(U_CGS2) break;
    case U_HARD: CBG_UPD(U_HARD) break;
    case U_SOLUTION: CBG_UPD(U_SOLUTION) break;
    default: CBG_UPD(U_COMBINE) break;
    }
#undef CBG_UPD
}

template <int F, int JM>
static void fused_launch(const OrthArgs &a, int g, const RedArgs &ra, const uint8_t *V,
                         hipStream_t s)
{
    if constexpr (F == F_E4M3 || (F == F_BF16 && JM > 48) ||
                  ((F == F_INT16 || F == F_FP16S) && JM > 80)) {
        return;              // not instantiated: beyond the format's fused range
    } else if (a.ev0) {
        hipExtLaunchKernelGGL(k_update_redot<F, JM>, dim3(g), dim3(BLK), 0, s, a.ev0, a.ev1, 0,
                              V, a.ld, a.scales, a.n, a.j, a.coef, a.wio, ra, a.st);
    } else {
        k_update_redot<F, JM><<<g, BLK, 0, s>>>(V, a.ld, a.scales, a.n, a.j, a.coef, a.wio, ra,
                                                a.st);
    }
}

template <int JM>
static void fused_shape(const OrthArgs &a, int g, const RedArgs &ra, const uint8_t *V,
                        hipStream_t s)
{
    CBG_FMT_SWITCH(a.fmt, (fused_launch<F, JM>(a, g, ra, V, s)))
}

// Largest j each format fuses at, from per-bucket timings on 128^3 (the
// fused pass against an update plus a multi-dot): beyond these the
// register tile drops the kernel to one wave per SIMD and two passes win.
int fused_jmax(int fmt)
{
    switch (fmt) {
    case F_BF16: return 48;
    case F_INT16: return 80;
    case F_FP16S: return 80;        // decoded like int16: one scale product per entry
    case F_E4M3: return 0;
    default: return FUSED_JMAX;
    }
}

// Whether launch_update_redot takes step j: within the format's fused range,
// and the template's vectors addressable with 32-bit buffer offsets.
bool fused_takes(int fmt, int64_t ld, int j)
{
    return j >= 1 && j <= fused_jmax(fmt) &&
           (double)FUSED_JMAX * (double)ld * fmt_bytes(fmt) < 2147483648.0;
}

int launch_update_redot(const OrthArgs &a, hipStream_t s)
{
    if (!fused_takes(a.fmt, a.ld, a.j))
        return 0;
    int lw = a.fmt == F_FP64 ? 1 : (a.fmt == F_FP32 || a.fmt == F_INT32) ? 2
             : a.fmt == F_E4M3 ? 8 : 4;
    const int g = grid_for(a.n, BLK * lw);
    RedArgs ra{a.ws.orth, a.ws.stride};
    const uint8_t *V = (const uint8_t *)a.V;
    if (a.j <= 16)
        fused_shape<16>(a, g, ra, V, s);
    else if (a.j <= 32)
        fused_shape<32>(a, g, ra, V, s);
    else if (a.j <= 48)
        fused_shape<48>(a, g, ra, V, s);
    else if (a.j <= 64)
        fused_shape<64>(a, g, ra, V, s);
    else if (a.j <= 80)
        fused_shape<80>(a, g, ra, V, s);
    else
        fused_shape<FUSED_JMAX>(a, g, ra, V, s);
    return g;
}

int launch_mgs(int fmt, const void *V, int64_t ld, const double *scales, int n, int k, int j,
               double *w, const double *coef, const RedWs &ws, const DevState *st, int pass,
               hipStream_t s)
{
    int g = 1;
    RedArgs ra{ws.orth, ws.stride};
    CBG_FMT_SWITCH(fmt, (g = grid_for(((int64_t)n + Fmt<F>::VW - 1) / Fmt<F>::VW, BLK),
                         k_mgs<F><<<g, BLK, 0, s>>>((const uint8_t *)V, ld, scales, n, k, j, w,
                                                    coef, ra, st, pass)))
    return g;
}

void launch_reduce(const RedWs &ws, int role, int nb_orth, int nb_spmv, int j, DevState *st,
                   const void *sa, double *out, int fmt, hipStream_t s)
{
    StepArrays a{};
    if (sa)
        a = *(const StepArrays *)sa;
    k_reduce<<<reduce_grid(role, j), RBLK, 0, s>>>(ws, role, nb_orth, nb_spmv, j, st, a, out,
                                                   fmt);
}

void launch_normalize(int fmt, const double *w, int n, int64_t nst, double *v_out, void *Q,
                      const double *scale_slot, const double *tptr, double tval,
                      const DevState *st, int check_done, hipStream_t s)
{
    int vw = fmt == F_FP64 ? 2 : (fmt == F_FP32 || fmt == F_INT32) ? 4 : fmt == F_E4M3 ? 16 : 8;
    int g = grid_for((nst + vw - 1) / vw, BLK);
    CBG_FMT_SWITCH(fmt, (k_normalize<F><<<g, BLK, 0, s>>>(w, n, nst, v_out, (uint8_t *)Q,
                                                           scale_slot, tptr, tval, st,
                                                           check_done, fmt)))
}

void launch_step_normalize(int fmt, const double *w, int n, int64_t ld, const double *dinv,
                           double *z, void *Q, const double *scale_slot, const DevState *st,
                           hipStream_t s)
{
    const int g = grid_for((ld / 2 + BLK * 4 - 1) / (BLK * 4), 1);
    CBG_FMT_SWITCH(fmt, (k_step_normalize<F><<<g, BLK, 0, s>>>(w, n, ld, dinv, z, (uint8_t *)Q,
                                                                scale_slot, st)))
}

void launch_stencil(int fmt, int mode, const double *w, int n, int64_t ld, const int32_t grid[3],
                    const uint16_t *codes, const double *dinv, double *z, void *Q,
                    const double *scale_slot, const DevState *st, hipStream_t s)
{
    // one tile per block (no block partials here): a block's loads, barrier
    // and sums are not serialised over several tiles, which measured about
    // 10% faster at 160^3 than 4096 blocks looping over 16,000 tiles
    const int g = (int)std::min<int64_t>(std::max<int64_t>((ld + BLK - 1) / BLK, 1), 65536);
    // buffer loads while the codes' byte range and w's fit the 32-bit
    // offsets of a buffer resource (ld below about 39.7 million)
    const bool buf = 27 * ld * 2 <= (int64_t)INT32_MAX - 16;
#define CBG_ST(B)                                                                              \
    if (mode == ST_STEP) {                                                                     \
        CBG_FMT_SWITCH(fmt, (k_stencil<F, ST_STEP, B><<<g, BLK, 0, s>>>(                       \
                                w, n, ld, grid[0], grid[1], grid[2], codes, dinv, z,           \
                                (uint8_t *)Q, scale_slot, st)))                                \
    } else if (mode == ST_PLAIN) {                                                             \
        k_stencil<F_FP64, ST_PLAIN, B><<<g, BLK, 0, s>>>(w, n, ld, grid[0], grid[1], grid[2],  \
                                                         codes, dinv, z, nullptr, nullptr,     \
                                                         nullptr);                             \
    } else {                                                                                   \
        k_stencil<F_FP64, ST_ACC, B><<<g, BLK, 0, s>>>(w, n, ld, grid[0], grid[1], grid[2],    \
                                                       codes, dinv, z, nullptr, nullptr,       \
                                                       nullptr);                               \
    }
    if (buf) {
        CBG_ST(true)
    } else {
        CBG_ST(false)
    }
#undef CBG_ST
}

void launch_decode(int fmt, const void *Q, int n, const double *scale, double *v, hipStream_t s)
{
    int vw = fmt == F_FP64 ? 2 : (fmt == F_FP32 || fmt == F_INT32) ? 4 : fmt == F_E4M3 ? 16 : 8;
    int g = grid_for(((int64_t)n + vw - 1) / vw, BLK);
    CBG_FMT_SWITCH(fmt, (k_decode<F><<<g, BLK, 0, s>>>((const uint8_t *)Q, n, scale, v)))
}

int launch_norm(const double *x, int64_t n, const RedWs &ws, hipStream_t s)
{
    int g = grid_for(n, BLK * 4);
    k_norm<<<g, BLK, 0, s>>>(x, n, RedArgs{ws.spmv, ws.sstride});
    return g;
}

void launch_init_state(DevState *st, int n, int m, int fmt, double tol, double eta,
                       int64_t maxiter, int reorth_all, hipStream_t s)
{
    k_init_state<<<1, 64, 0, s>>>(st, n, m, fmt, tol, eta, maxiter, reorth_all);
}

void launch_jacobi_setup(const SpmvArgs &a, int64_t ld, double *dinv, unsigned *bad,
                         hipStream_t s)
{
    if (a.sp && a.sd && a.sv) {
        const int g = (int)std::min<int64_t>(std::max<int64_t>((ld + BLK - 1) / BLK, 1), 65536);
        k_jacobi_setup_sell<<<g, BLK, 0, s>>>(a.n, ld, a.rp, a.sp, a.sd, a.sv, a.sdiag, a.ndiag,
                                              dinv, bad);
        return;
    }
    const int g = (int)std::min<int64_t>(std::max<int64_t>((ld + BLK / 32 - 1) / (BLK / 32), 1),
                                         65536);
    k_jacobi_setup<<<g, BLK, 0, s>>>(a.n, ld, a.rp, a.ci, a.val, dinv, bad);
}

__global__ void k_clear_flags(DevState *st, unsigned *bad)
{
    if (threadIdx.x == 0) {
        if (st)
            st->nonfinite = 0;
        if (bad)
            *bad = 0u;
    }
}

void launch_clear_flags(DevState *st, unsigned *bad, hipStream_t s)
{
    k_clear_flags<<<1, 64, 0, s>>>(st, bad);
}

// p[0 .. count) = 0 with a kernel (no memset node where a caller captures)
__global__ void k_fill_zero(double *p, int count)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        p[i] = 0.0;
}

void launch_fill_zero(double *p, int count, hipStream_t s)
{
    if (count > 0)
        k_fill_zero<<<grid_for(count, 256), 256, 0, s>>>(p, count);
}

void launch_backsolve(const DevState *st, const void *sa, hipStream_t s)
{
    k_backsolve<<<1, 64, 0, s>>>(st, *(const StepArrays *)sa);
}

size_t step_arrays_size() { return sizeof(StepArrays); }

void make_step_arrays(void *out, double *H, double *h, double *u, double *cs, double *sn,
                      double *g, double *y, double *hist, double *scales, int32_t *flags)
{
    StepArrays *a = (StepArrays *)out;
    a->H = H; a->h = h; a->u = u; a->cs = cs; a->sn = sn; a->g = g; a->y = y;
    a->hist = hist; a->scales = scales; a->flags = flags; a->G = nullptr;
}

void set_step_gram(void *sa, double *G) { ((StepArrays *)sa)->G = G; }

}  // namespace cbg
