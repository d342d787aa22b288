/*
 * CB-GMRES CPU oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Plain FP64 restarted GMRES with a compressed Krylov basis, written from
 * Aliaga et al., "Compressed Basis GMRES on High Performance GPUs":
 *   - the algorithm of Fig. 1 (Section 3): CGS orthogonalisation with
 *     conditional re-orthogonalisation, Givens-updated least squares, and an
 *     explicit residual at every restart;
 *   - the compressed basis of Section 4: V is stored in a reduced format and
 *     every read widens it to FP64 before any arithmetic (steps 5, 8, 17),
 *     every write (steps 13-14) compresses it;
 *   - the per-vector fixed-point scaling of Section 5.2.
 *
 * Where the paper is silent or garbled this file follows one reading, named
 * at the place it is used (R1 ... R18 in the design notes).
 *
 * Deliberately simple: no blocking, fusion or reordering beyond what the
 * algorithm states, except that reductions use a fixed order so results do
 * not depend on the thread count: sums over n entries are taken in blocks of
 * 1024 consecutive entries (each in index order), then the block sums in
 * block order.  OpenMP parallelises over rows and blocks only.
 */
#include "oracle.h"

#include <fenv.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define BLK 1024
/* eta = 1/sqrt(2), the nearest double (reading R1: the paper gives no value;
 * this is the classical Daniel-Gragg-Kaufman-Stewart threshold). */
#define ETA_DEFAULT 0.70710678118654752440

/* ------------------------------------------------------------------------- */
/* Storage formats (Section 5.2 plus the bf16 / e4m3 extensions).            */
/* ------------------------------------------------------------------------- */

/* A binary floating-point format: p significand bits (implicit bit
 * included), e bits of exponent, minimum normal exponent emin, bias 1-emin.
 * ieee: the all-ones exponent encodes inf/NaN (fp16, bf16); otherwise only
 * S.1111.111 is NaN (OCP E4M3FN). */
typedef struct { int p, ebits, emin, ieee; double maxfin; } ffmt;

static const ffmt F16  = {11, 5, -14, 1, 65504.0};
static const ffmt BF16 = {8, 8, -126, 1, 3.38953138925153547590470800371487866880e38};
static const ffmt E4M3 = {4, 4, -6, 0, 448.0};

int orc_format_bytes(int fmt)
{
    switch (fmt) {
    case ORC_FP64: return 8;
    case ORC_FP32: return 4;
    case ORC_FP16: return 2;
    case ORC_BF16: return 2;
    case ORC_E4M3: return 1;
    case ORC_INT32: return 4;
    case ORC_INT16: return 2;
    case ORC_FP16S: return 2;
    default: return 0;
    }
}

/* Round x to the nearest number with p significand bits and exponent at
 * least emin, ties to even (IEEE 754 roundTiesToEven), in one rounding.
 * The scaling by 2^(p-1-e) is exact, so the scaled value's fractional part is
 * the exact rounding remainder, and rint() in the default rounding mode
 * rounds it to the nearest integer with ties to even.  Overflow is left to
 * the caller. */
static double round_to_p(double x, int p, int emin)
{
    if (x == 0.0 || !isfinite(x))
        return x;
    int e = ilogb(x);
    if (e < emin)
        e = emin;                       /* subnormal range: fixed quantum */
    double q = rint(ldexp(x, p - 1 - e));
    return ldexp(q, e - p + 1);
}

/* Bit pattern of r, which must be exactly representable in F (or beyond its
 * largest finite value, which gives inf for IEEE formats and NaN for E4M3FN). */
static uint32_t float_bits(double r, const ffmt *F)
{
    int mb = F->p - 1;
    uint32_t sign = signbit(r) ? (1u << (F->ebits + mb)) : 0u;
    uint32_t emax_field = (1u << F->ebits) - 1u;
    double a = fabs(r);
    if (isnan(r))
        return sign | (emax_field << mb) | ((1u << mb) - 1u);
    if (a > F->maxfin) {
        if (F->ieee)
            return sign | (emax_field << mb);
        return sign | (emax_field << mb) | ((1u << mb) - 1u);
    }
    if (a == 0.0)
        return sign;
    int e = ilogb(a);
    if (e < F->emin)                    /* subnormal: a = mant * 2^(emin-mb) */
        return sign | (uint32_t)ldexp(a, mb - F->emin);
    uint32_t mant = (uint32_t)ldexp(a, mb - e) - (1u << mb);
    uint32_t ef = (uint32_t)(e - F->emin + 1);
    return sign | (ef << mb) | mant;
}

/* Value of bit pattern c in F, from the definition of the format. */
static double float_value(uint32_t c, const ffmt *F)
{
    int mb = F->p - 1;
    uint32_t mant = c & ((1u << mb) - 1u);
    uint32_t ef = (c >> mb) & ((1u << F->ebits) - 1u);
    int neg = (c >> (F->ebits + mb)) & 1u;
    uint32_t emax_field = (1u << F->ebits) - 1u;
    double v;
    if (F->ieee && ef == emax_field)
        v = mant ? NAN : INFINITY;
    else if (!F->ieee && ef == emax_field && mant == (1u << mb) - 1u)
        v = NAN;
    else if (ef == 0)
        v = ldexp((double)mant, F->emin - mb);
    else
        v = ldexp((double)(mant + (1u << mb)), (int)ef - (1 - F->emin) - mb);
    return neg ? -v : v;
}

/* Decode tables, filled once from float_value(). */
static double tab_f16[65536], tab_bf16[65536], tab_e4m3[256];

__attribute__((constructor)) static void build_tables(void)
{
    for (uint32_t c = 0; c < 65536u; ++c) {
        tab_f16[c] = float_value(c, &F16);
        tab_bf16[c] = float_value(c, &BF16);
    }
    for (uint32_t c = 0; c < 256u; ++c)
        tab_e4m3[c] = float_value(c, &E4M3);
}

static double max_abs(int64_t n, const double *v)
{
    double m = 0.0;
#pragma omp parallel for reduction(max : m) schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double a = fabs(v[i]);
        if (a > m)
            m = a;
    }
    return m;
}

int orc_encode(int fmt, int64_t n, const double *v, void *q, double *scale)
{
    if (n < 0 || orc_format_bytes(fmt) == 0 || (n > 0 && (!v || !q)) || !scale)
        return ORC_E_ARG;
    *scale = 1.0;
    switch (fmt) {
    case ORC_FP64: {
        double *o = (double *)q;
        for (int64_t i = 0; i < n; ++i)
            o[i] = v[i];
        break;
    }
    case ORC_FP32: {                    /* a plain cast: one RNE rounding */
        float *o = (float *)q;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            o[i] = (float)v[i];
        break;
    }
    case ORC_FP16:
    case ORC_BF16: {
        const ffmt *F = fmt == ORC_FP16 ? &F16 : &BF16;
        uint16_t *o = (uint16_t *)q;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            o[i] = (uint16_t)float_bits(round_to_p(v[i], F->p, F->emin), F);
        break;
    }
    case ORC_E4M3: {
        /* Per-vector power-of-two scale 2^k with max|v| * 2^-k in (224, 448],
         * so the largest entry lands in the top binade of E4M3 and nothing
         * overflows.  Scaling by 2^-k is exact. */
        double vinf = max_abs(n, v);
        int k = 0;
        if (vinf > 0.0) {
            k = ilogb(vinf) - 8;
            if (ldexp(vinf, -k) > 448.0)
                k += 1;
        }
        *scale = ldexp(1.0, k);
        uint8_t *o = (uint8_t *)q;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            o[i] = (uint8_t)float_bits(round_to_p(ldexp(v[i], -k), E4M3.p, E4M3.emin), &E4M3);
        break;
    }
    case ORC_FP16S: {
        /* float16 with a per-vector power-of-two scale 2^k, max|v| * 2^-k in
         * (32752, 65504]: the largest entry lands in the top binade and the
         * small entries stay clear of the subnormal range.  Scaling by 2^-k
         * is exact, so each entry is rounded once. */
        double vinf = max_abs(n, v);
        int k = 0;
        if (vinf > 0.0) {
            k = ilogb(vinf) - 15;
            if (ldexp(vinf, -k) > 65504.0)
                k += 1;
        }
        *scale = ldexp(1.0, k);
        uint16_t *o = (uint16_t *)q;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            o[i] = (uint16_t)float_bits(round_to_p(ldexp(v[i], -k), F16.p, F16.emin), &F16);
        break;
    }
    case ORC_INT32:
    case ORC_INT16: {
        /* Section 5.2: sigma = (||v||_inf / ||v||_2) / max_int for the raw
         * vector; the stored vector is the normalised one, so with
         * ||v||_2 = 1 this is sigma = ||v||_inf / max_int, and the entries
         * stored are the integers v_i / sigma (reading R4), rounded to
         * nearest with ties to even and clamped to [-max_int, max_int] (R5). */
        double M = fmt == ORC_INT32 ? 2147483647.0 : 32767.0;
        double vinf = max_abs(n, v);
        double sigma = vinf / M;
        *scale = sigma;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double t = sigma > 0.0 ? rint(v[i] / sigma) : 0.0;
            if (t > M) t = M;
            if (t < -M) t = -M;
            if (fmt == ORC_INT32)
                ((int32_t *)q)[i] = (int32_t)t;
            else
                ((int16_t *)q)[i] = (int16_t)t;
        }
        break;
    }
    }
    return 0;
}

/* Decode entries [i0, i1) of a stored vector into out[0 .. i1-i0). */
static void decode_range(int fmt, const void *q, double s, int64_t i0, int64_t i1, double *out)
{
    int64_t m = i1 - i0;
    switch (fmt) {
    case ORC_FP64: for (int64_t i = 0; i < m; ++i) out[i] = ((const double *)q)[i0 + i]; break;
    case ORC_FP32: for (int64_t i = 0; i < m; ++i) out[i] = (double)((const float *)q)[i0 + i]; break;
    case ORC_FP16: for (int64_t i = 0; i < m; ++i) out[i] = tab_f16[((const uint16_t *)q)[i0 + i]]; break;
    case ORC_BF16: for (int64_t i = 0; i < m; ++i) out[i] = tab_bf16[((const uint16_t *)q)[i0 + i]]; break;
    case ORC_E4M3: for (int64_t i = 0; i < m; ++i) out[i] = tab_e4m3[((const uint8_t *)q)[i0 + i]] * s; break;
    case ORC_INT32: for (int64_t i = 0; i < m; ++i) out[i] = s * (double)((const int32_t *)q)[i0 + i]; break;
    case ORC_INT16: for (int64_t i = 0; i < m; ++i) out[i] = s * (double)((const int16_t *)q)[i0 + i]; break;
    case ORC_FP16S: for (int64_t i = 0; i < m; ++i) out[i] = tab_f16[((const uint16_t *)q)[i0 + i]] * s; break;
    }
}

int orc_decode(int fmt, int64_t n, const void *q, double scale, double *out)
{
    if (n < 0 || orc_format_bytes(fmt) == 0 || (n > 0 && (!q || !out)))
        return ORC_E_ARG;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < (n + BLK - 1) / BLK; ++b) {
        int64_t i0 = b * BLK, i1 = i0 + BLK < n ? i0 + BLK : n;
        decode_range(fmt, q, scale, i0, i1, out + i0);
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Basic kernels: SpMV and fixed-order sums.                                 */
/* ------------------------------------------------------------------------- */

void orc_spmv(int32_t n, const int32_t *rp, const int32_t *ci, const double *val,
              const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p)
            s += val[p] * x[ci[p]];
        y[i] = s;
    }
}

/* y = P x where P has A's pattern and single-precision values (widened). */
static void spmv_f32vals(int32_t n, const int32_t *rp, const int32_t *ci, const float *val,
                         const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p)
            s += (double)val[p] * x[ci[p]];
        y[i] = s;
    }
}

static double sum_blocks(int64_t nb, const double *part)
{
    double s = 0.0;
    for (int64_t b = 0; b < nb; ++b)
        s += part[b];
    return s;
}

double orc_dot(int64_t n, const double *x, const double *y)
{
    int64_t nb = (n + BLK - 1) / BLK;
    double *part = (double *)malloc((size_t)(nb > 0 ? nb : 1) * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; ++b) {
        int64_t i1 = (b + 1) * BLK < n ? (b + 1) * BLK : n;
        double s = 0.0;
        for (int64_t i = b * BLK; i < i1; ++i)
            s += x[i] * y[i];
        part[b] = s;
    }
    double s = sum_blocks(nb, part);
    free(part);
    return s;
}

/* h_k = sum_i dec(Q_k)_i * w_i for k = 0..j-1, each sum in fixed block
 * order: the multi-dot V_j^T w of Fig. 1 steps 5 and 8 read through the
 * accessor. part: scratch of j*nb doubles. */
static void multidot(int fmt, int32_t j, void *const *Q, const double *sc, int64_t n,
                     const double *w, double *h, double *part)
{
    int64_t nb = (n + BLK - 1) / BLK;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; ++b) {
        double buf[BLK];
        int64_t i0 = b * BLK, i1 = i0 + BLK < n ? i0 + BLK : n;
        for (int32_t k = 0; k < j; ++k) {
            decode_range(fmt, Q[k], sc[k], i0, i1, buf);
            double s = 0.0;
            for (int64_t i = i0; i < i1; ++i)
                s += buf[i - i0] * w[i];
            part[(int64_t)k * nb + b] = s;
        }
    }
    for (int32_t k = 0; k < j; ++k)
        h[k] = sum_blocks(nb, part + (int64_t)k * nb);
}

/* out_i = sum_k c_k * dec(Q_k)_i (k in order) for k = 0..j-1: the product
 * V_j c of steps 5, 8 and 17, read through the accessor. */
static void basis_combine(int fmt, int32_t j, void *const *Q, const double *sc, int64_t n,
                          const double *c, double *out)
{
    int64_t nb = (n + BLK - 1) / BLK;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; ++b) {
        double buf[BLK], acc[BLK];
        int64_t i0 = b * BLK, i1 = i0 + BLK < n ? i0 + BLK : n;
        for (int64_t i = i0; i < i1; ++i)
            acc[i - i0] = 0.0;
        for (int32_t k = 0; k < j; ++k) {
            decode_range(fmt, Q[k], sc[k], i0, i1, buf);
            for (int64_t i = i0; i < i1; ++i)
                acc[i - i0] += c[k] * buf[i - i0];
        }
        for (int64_t i = i0; i < i1; ++i)
            out[i] = acc[i - i0];
    }
}

/* Modified Gram-Schmidt over the stored vectors (the ORC_V_MGS variant of
 * steps 5 and 8): for k = 0..j-1 in order, h_k = dec(Q_k)^T w in the fixed
 * block order of orc_dot, then w_i -= h_k dec(Q_k)_i.  buf: n doubles. */
static void mgs_pass(int fmt, int32_t j, void *const *Q, const double *sc, int64_t n,
                     double *w, double *h, double *buf)
{
    for (int32_t k = 0; k < j; ++k) {
        orc_decode(fmt, n, Q[k], sc[k], buf);
        h[k] = orc_dot(n, buf, w);
        const double hk = h[k];
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            w[i] = w[i] - hk * buf[i];
    }
}

/* ------------------------------------------------------------------------- */
/* Restarted CB-GMRES (Fig. 1).                                              */
/* ------------------------------------------------------------------------- */

/* ------------------------------------------------------------------------- */
/* Block-Jacobi with adaptive-precision storage (definition in oracle.h).     */
/* ------------------------------------------------------------------------- */

#define BJ_MAXB 8

/* X = D^-1 for the bs x bs row-major D (overwritten) by Gauss-Jordan
 * elimination with partial pivoting; every operation is a separate IEEE
 * multiply, subtract or divide in the order written.  -1 if a pivot is 0. */
static int gj_invert(int bs, double *D, double *X)
{
    for (int i = 0; i < bs; ++i)
        for (int k = 0; k < bs; ++k)
            X[i * bs + k] = (i == k) ? 1.0 : 0.0;
    for (int c = 0; c < bs; ++c) {
        int r = c;
        double best = fabs(D[c * bs + c]);
        for (int i = c + 1; i < bs; ++i)
            if (fabs(D[i * bs + c]) > best) {
                best = fabs(D[i * bs + c]);
                r = i;
            }
        if (best == 0.0)
            return -1;
        if (r != c)
            for (int k = 0; k < bs; ++k) {
                double t = D[c * bs + k]; D[c * bs + k] = D[r * bs + k]; D[r * bs + k] = t;
                t = X[c * bs + k]; X[c * bs + k] = X[r * bs + k]; X[r * bs + k] = t;
            }
        const double p = D[c * bs + c];
        for (int k = 0; k < bs; ++k) {
            D[c * bs + k] = D[c * bs + k] / p;
            X[c * bs + k] = X[c * bs + k] / p;
        }
        for (int i = 0; i < bs; ++i) {
            if (i == c)
                continue;
            const double f = D[i * bs + c];
            for (int k = 0; k < bs; ++k) {
                const double pd = f * D[c * bs + k];
                D[i * bs + k] = D[i * bs + k] - pd;
                const double px = f * X[c * bs + k];
                X[i * bs + k] = X[i * bs + k] - px;
            }
        }
    }
    return 0;
}

/* max over columns of the column's absolute sum (rows summed in order). */
static double norm1(int bs, const double *M)
{
    double best = 0.0;
    for (int k = 0; k < bs; ++k) {
        double s = 0.0;
        for (int i = 0; i < bs; ++i)
            s = s + fabs(M[i * bs + k]);
        if (s > best)
            best = s;
    }
    return best;
}

int orc_block_jacobi(int32_t n, const int32_t *rp, const int32_t *ci, const double *val,
                     int32_t bs, int32_t prec_min, double *vals, int8_t *prec)
{
    if (n < 0 || bs < 1 || bs > BJ_MAXB || (prec_min != 16 && prec_min != 32 && prec_min != 64) ||
        (n > 0 && (!rp || !ci || !val || !vals || !prec)))
        return ORC_E_ARG;
    fesetround(FE_TONEAREST);
    const int32_t nblk = (n + bs - 1) / bs;
    int bad = 0;
    for (int32_t b = 0; b < nblk; ++b) {
        const int32_t i0 = b * bs;
        const int sz = (n - i0 < bs) ? (int)(n - i0) : bs;
        double D[BJ_MAXB * BJ_MAXB], A0[BJ_MAXB * BJ_MAXB], X[BJ_MAXB * BJ_MAXB];
        for (int t = 0; t < sz * sz; ++t)
            D[t] = 0.0;
        for (int i = 0; i < sz; ++i)
            for (int32_t p = rp[i0 + i]; p < rp[i0 + i + 1]; ++p) {
                const int32_t c = ci[p];
                if (c >= i0 && c < i0 + sz)
                    D[i * sz + (c - i0)] = val[p];
            }
        memcpy(A0, D, sizeof(double) * (size_t)(sz * sz));
        double *out = vals + (size_t)b * bs * bs;
        for (int t = 0; t < bs * bs; ++t)
            out[t] = 0.0;
        if (gj_invert(sz, D, X) != 0) {
            bad = 1;
            prec[b] = 64;
            continue;
        }
        const double kappa = norm1(sz, A0) * norm1(sz, X);
        double mx = 0.0;
        for (int t = 0; t < sz * sz; ++t)
            if (fabs(X[t]) > mx)
                mx = fabs(X[t]);
        int pr = 64;
        if (prec_min <= 16 && kappa * ldexp(1.0, -11) <= 0.01 && mx <= 65504.0 &&
            mx >= ldexp(1.0, -14))
            pr = 16;
        else if (prec_min <= 32 && kappa * ldexp(1.0, -24) <= 0.01 &&
                 mx <= 3.40282346638528859811704183484516925e38 && mx >= ldexp(1.0, -126))
            pr = 32;
        prec[b] = (int8_t)pr;
        for (int i = 0; i < sz; ++i)
            for (int k = 0; k < sz; ++k) {
                const double x = X[i * sz + k];
                out[i * bs + k] = pr == 16 ? round_to_p(x, 11, -14)
                                : pr == 32 ? round_to_p(x, 24, -126) : x;
            }
    }
    return bad ? ORC_E_ARG : 0;
}

typedef struct {
    int kind;                 /* ORC_PC_* currently in force */
    double *dinv;             /* Jacobi, stencil: 1 / a_ii */
    const float *pv;          /* sparse: P values on A's pattern */
    int bs;                   /* block-Jacobi: block size */
    double *bj;               /* block-Jacobi: stored inverse values */
    const uint16_t *st;       /* stencil: float16 codes, slot-major */
    int32_t nx, ny, nz;       /* stencil: grid */
    int64_t st_ld;            /* stencil: slot stride */
} precond;

/* The stencil preconditioner of orc_opts (ORC_PC_STENCIL): row i at grid
 * point (x, y, z) sums its existing neighbours in slot order. */
static void apply_stencil(const precond *M, int32_t n, const double *v, double *z)
{
    const int64_t nx = M->nx, ny = M->ny, nz = M->nz;
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
        const int64_t x = i % nx, y = (i / nx) % ny, zz = i / (nx * ny);
        double s = 0.0;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (x + dx < 0 || x + dx >= nx || y + dy < 0 || y + dy >= ny ||
                        zz + dz < 0 || zz + dz >= nz)
                        continue;
                    const int p = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1);
                    const double c = (p == 13 ? 1.0 : 0.0) +
                                     tab_f16[M->st[(int64_t)p * M->st_ld + i]];
                    s = s + c * v[i + dz * nx * ny + dy * nx + dx];
                }
        z[i] = M->dinv[i] * s;
    }
}

/* z = M^{-1} v (Fig. 1 step 3 and step 17). */
static void apply_precond(const precond *M, int32_t n, const int32_t *rp, const int32_t *ci,
                          const double *v, double *z)
{
    if (M->kind == ORC_PC_JACOBI) {
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i)
            z[i] = M->dinv[i] * v[i];
    } else if (M->kind == ORC_PC_SPARSE) {
        spmv_f32vals(n, rp, ci, M->pv, v, z);
    } else if (M->kind == ORC_PC_STENCIL) {
        apply_stencil(M, n, v, z);
    } else if (M->kind == ORC_PC_BLOCK_JACOBI) {
        const int bs = M->bs;
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) {
            const int32_t i0 = i / bs * bs;
            const int sz = (n - i0 < bs) ? (int)(n - i0) : bs;
            const double *row = M->bj + (size_t)(i0 / bs) * bs * bs + (size_t)(i - i0) * bs;
            double s = 0.0;
            for (int l = 0; l < sz; ++l)
                s = s + row[l] * v[i0 + l];
            z[i] = s;
        }
    } else {
        memcpy(z, v, (size_t)n * sizeof(double));
    }
}

static int all_finite(int64_t n, const double *v)
{
    int ok = 1;
#pragma omp parallel for reduction(&& : ok) schedule(static)
    for (int64_t i = 0; i < n; ++i)
        ok = ok && isfinite(v[i]);
    return ok;
}

int orc_gmres(int32_t n, const int32_t *rp, const int32_t *ci, const double *val,
              const double *b, double *x, const orc_opts *opt, orc_result *res,
              double *hist, double *cycle_res, int32_t *cycle_len, double *dbg_V,
              double *dbg_H, int32_t *dbg_steps)
{
    if (!opt || !res)
        return ORC_E_ARG;
    memset(res, 0, sizeof(*res));
    const int32_t m = opt->restart;
    const int fmt = opt->format;
    const int bs = orc_format_bytes(fmt);
    if (n < 0 || m < 1 || bs == 0 || !(opt->tol >= 0.0) || opt->maxiter < 0 ||
        opt->precond < ORC_PC_NONE || opt->precond > ORC_PC_STENCIL ||
        (opt->variant & ~(ORC_V_SPMV_VHAT | ORC_V_ALWAYS_REORTH | ORC_V_MGS | ORC_V_GRAM |
                          ORC_V_ONEPASS)) != 0 ||
        ((opt->variant & ORC_V_MGS) && (opt->variant & ORC_V_GRAM)) ||
        ((opt->variant & ORC_V_ONEPASS) && !(opt->variant & ORC_V_GRAM)) ||
        (opt->precond == ORC_PC_SPARSE && !opt->p_val) ||
        (opt->precond == ORC_PC_STENCIL &&
         (!opt->p_stencil || opt->grid[0] < 1 || opt->grid[1] < 1 || opt->grid[2] < 1 ||
          (int64_t)opt->grid[0] * opt->grid[1] * opt->grid[2] != n || opt->st_ld < n)) ||
        (n > 0 && (!rp || !ci || !val || !b || !x))) {
        res->status = ORC_E_ARG;
        return ORC_E_ARG;
    }
    fesetround(FE_TONEAREST);
    if (dbg_steps)
        dbg_steps[0] = dbg_steps[1] = 0;
    if (n == 0) {                       /* empty system: nothing to solve */
        res->status = ORC_OK;
        return ORC_OK;
    }
    const double eta = opt->eta > 0.0 ? opt->eta : ETA_DEFAULT;
    const double tau = opt->tol;
    const int spmv_vhat = (opt->variant & ORC_V_SPMV_VHAT) != 0;
    const int always_reorth = (opt->variant & ORC_V_ALWAYS_REORTH) != 0;
    const int mgs = (opt->variant & ORC_V_MGS) != 0;
    const int gram = (opt->variant & ORC_V_GRAM) != 0;
    const int onepass = (opt->variant & ORC_V_ONEPASS) != 0;

    /* Fig. 1 works with ||b||_2 as the reference of the stop test (R8). */
    const double nb = sqrt(orc_dot(n, b, b));
    if (!isfinite(nb)) {
        res->status = ORC_E_NONFINITE;
        return ORC_E_NONFINITE;
    }
    if (nb == 0.0) {                    /* b = 0: the solution is x = 0 */
        memset(x, 0, (size_t)n * sizeof(double));
        res->status = ORC_OK;
        return ORC_OK;
    }

    precond M = {opt->precond, NULL, opt->p_val, 0, NULL, opt->p_stencil, opt->grid[0],
                 opt->grid[1], opt->grid[2], opt->st_ld};
    if (M.kind == ORC_PC_BLOCK_JACOBI) {
        M.bs = opt->pc_block > 0 ? opt->pc_block : 4;
        const int pmin = opt->pc_prec > 0 ? opt->pc_prec : 16;
        const int32_t nblk = (n + M.bs - 1) / M.bs;
        M.bj = (double *)malloc(sizeof(double) * (size_t)nblk * M.bs * M.bs);
        int8_t *pr = (int8_t *)malloc((size_t)nblk);
        const int rc = orc_block_jacobi(n, rp, ci, val, M.bs, pmin, M.bj, pr);
        free(pr);
        if (rc != 0) {
            free(M.bj);
            res->status = ORC_E_ARG;
            return ORC_E_ARG;
        }
    }
    if (M.kind == ORC_PC_JACOBI || M.kind == ORC_PC_STENCIL) {
        M.dinv = (double *)malloc((size_t)n * sizeof(double));
        int bad = 0;
        for (int32_t i = 0; i < n; ++i) {
            double d = 0.0;
            for (int32_t p = rp[i]; p < rp[i + 1]; ++p)
                if (ci[p] == i)
                    d = val[p];
            if (d == 0.0)
                bad = 1;
            M.dinv[i] = 1.0 / d;
        }
        if (bad) {
            free(M.dinv);
            res->status = ORC_E_ARG;
            return ORC_E_ARG;
        }
    }

    const int64_t nbk = ((int64_t)n + BLK - 1) / BLK;
    void **Q = (void **)malloc(sizeof(void *) * (size_t)(m + 1));
    double *sc = (double *)calloc((size_t)(m + 1), sizeof(double));
    for (int32_t k = 0; k <= m; ++k)
        Q[k] = malloc((size_t)n * (size_t)bs);
    double *r = (double *)malloc((size_t)n * sizeof(double));
    double *v = (double *)malloc((size_t)n * sizeof(double));
    double *z = (double *)malloc((size_t)n * sizeof(double));
    double *w = (double *)malloc((size_t)n * sizeof(double));
    double *s = (double *)malloc((size_t)n * sizeof(double));
    double *xprev = (double *)malloc((size_t)n * sizeof(double));
    double *part = (double *)malloc((size_t)(m + 1) * (size_t)nbk * sizeof(double));
    double *H = (double *)calloc((size_t)(m + 1) * (size_t)m, sizeof(double)); /* col-major */
    double *h = (double *)malloc((size_t)(m + 1) * sizeof(double));
    double *u = (double *)malloc((size_t)(m + 1) * sizeof(double));
    double *cs = (double *)malloc((size_t)(m + 1) * sizeof(double));
    double *sn = (double *)malloc((size_t)(m + 1) * sizeof(double));
    double *g = (double *)malloc((size_t)(m + 2) * sizeof(double));
    double *y = (double *)malloc((size_t)(m + 1) * sizeof(double));
    /* ORC_V_GRAM: G ((m+1) x (m+1), row-major, symmetric) and the decoded
     * newest stored vector */
    double *G = gram ? (double *)malloc((size_t)(m + 1) * (size_t)(m + 1) * sizeof(double)) : NULL;
    double *gv = gram ? (double *)malloc((size_t)n * sizeof(double)) : NULL;
    double *grow = gram ? (double *)malloc((size_t)(m + 1) * sizeof(double)) : NULL;
#define HH(i, jj) H[(size_t)(jj) * (size_t)(m + 1) + (size_t)(i)]   /* 0-based */

    int64_t it = 0;
    int status = ORC_NOT_CONVERGED;
    double rho_prev = INFINITY;
    int stagnant = 0;
    int64_t cycle = 0;
    double last_rec = NAN;

    for (;;) {
        /* Step 1 (and the restart of step 18): explicit residual r = b - A x. */
        orc_spmv(n, rp, ci, val, x, r);
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i)
            r[i] = b[i] - r[i];
        double rho = sqrt(orc_dot(n, r, r));
        if (cycle_res)
            cycle_res[cycle] = rho / nb;

        if (!isfinite(rho)) {
            if ((M.kind == ORC_PC_SPARSE || M.kind == ORC_PC_STENCIL) && opt->fallback &&
                cycle > 0) {
                /* plain CB-GMRES takes over from the last finite iterate */
                memcpy(x, xprev, (size_t)n * sizeof(double));
                M.kind = ORC_PC_NONE;
                res->fell_back = 1;
                stagnant = 0;
                rho_prev = INFINITY;
                continue;
            }
            status = ORC_E_NONFINITE;
            break;
        }
        if (rho <= tau * nb) {          /* stop test ||b - A x|| <= tau ||b|| */
            status = ORC_OK;
            break;
        }
        if (it >= opt->maxiter) {
            status = ORC_NOT_CONVERGED;
            break;
        }
        if ((M.kind == ORC_PC_SPARSE || M.kind == ORC_PC_STENCIL) && opt->fallback) {
            /* stagnation: explicit residual not below 0.99x its previous
             * value in two consecutive cycles */
            stagnant = rho > 0.99 * rho_prev ? stagnant + 1 : 0;
            if (stagnant >= 2) {
                M.kind = ORC_PC_NONE;
                res->fell_back = 1;
                stagnant = 0;
            }
        }
        rho_prev = rho;
        memcpy(xprev, x, (size_t)n * sizeof(double));
        res->restarts += 1;

        /* v = r / beta, stored through the accessor as V_1. */
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i)
            v[i] = r[i] / rho;
        orc_encode(fmt, n, v, Q[0], &sc[0]);
        int32_t nstored = 1;               /* basis vectors stored this cycle */
        for (int32_t i = 0; i < m + 2; ++i)
            g[i] = 0.0;
        g[0] = rho;
        memset(H, 0, (size_t)(m + 1) * (size_t)m * sizeof(double));

        int32_t meff = 0;
        for (int32_t j = 1; j <= m; ++j) {
            const int32_t jc = j - 1;            /* 0-based column */
            /* Step 3: w = A M^{-1} v, with v the FP64 vector of step 13
             * (reading R3: the accessor is named for steps 5, 8, 13-14 and
             * 17, not for step 3).  The SPMV_VHAT variant reads the stored
             * vector back through the accessor instead. */
            if (spmv_vhat)
                orc_decode(fmt, n, Q[jc], sc[jc], v);
            apply_precond(&M, n, rp, ci, v, z);
            orc_spmv(n, rp, ci, val, z, w);
            /* Step 4 */
            double omega = sqrt(orc_dot(n, w, w));
            /* Step 5: h = V_j^T w; w = w - V_j h, V_j widened from storage. */
            int brk;
            double t;
            if (onepass) {
                /* h and row jc of G, then u = h - G h and t1 by Pythagoras */
                multidot(fmt, j, Q, sc, n, w, h, part);
                orc_decode(fmt, n, Q[jc], sc[jc], gv);
                multidot(fmt, j, Q, sc, n, gv, grow, part);
                for (int32_t k = 0; k < j; ++k)
                    G[(size_t)jc * (m + 1) + k] = G[(size_t)k * (m + 1) + jc] = grow[k];
                double hh = 0.0, hu = 0.0;
                for (int32_t k = 0; k < j; ++k) {
                    double gh = 0.0;
                    for (int32_t l = 0; l < j; ++l)
                        gh += G[(size_t)k * (m + 1) + l] * h[l];
                    u[k] = h[k] - gh;
                }
                for (int32_t k = 0; k < j; ++k) {
                    hh += h[k] * h[k];
                    hu += h[k] * u[k];
                }
                /* below about (j+1) u64 omega^2 the difference is rounding
                 * alone: t1 is floored there, so that step 12 sees a w that
                 * lies numerically in span(V) as the breakdown it is */
                const double t1sq = omega * omega - hh - hu;
                const double floor2 = 4.0 * (j + 1) * 0x1p-53 * omega * omega;
                const double t1 = sqrt(t1sq > floor2 ? t1sq : floor2);
                const int ro = always_reorth || t1 < eta * omega;
                for (int32_t k = 0; k < j; ++k)
                    grow[k] = ro ? h[k] + u[k] : h[k];
                basis_combine(fmt, j, Q, sc, n, grow, s);
#pragma omp parallel for schedule(static)
                for (int32_t i = 0; i < n; ++i)
                    w[i] = w[i] - s[i];
                const double t2 = sqrt(orc_dot(n, w, w));
                if (ro) {
                    for (int32_t k = 0; k < j; ++k)
                        h[k] = h[k] + u[k];
                    res->reorths += 1;
                    brk = (t2 == 0.0) || (t2 < eta * t1);
                } else {
                    brk = (t2 == 0.0);
                }
                t = t2;
                goto column;
            }
            if (mgs) {
                mgs_pass(fmt, j, Q, sc, n, w, h, s);
            } else {
                multidot(fmt, j, Q, sc, n, w, h, part);
                basis_combine(fmt, j, Q, sc, n, h, s);
#pragma omp parallel for schedule(static)
                for (int32_t i = 0; i < n; ++i)
                    w[i] = w[i] - s[i];
            }
            if (gram) {
                /* row jc of G: dec(v^_k)^T dec(v^_jc), k = 0..jc, mirrored */
                orc_decode(fmt, n, Q[jc], sc[jc], gv);
                multidot(fmt, j, Q, sc, n, gv, grow, part);
                for (int32_t k = 0; k < j; ++k)
                    G[(size_t)jc * (m + 1) + k] = G[(size_t)k * (m + 1) + jc] = grow[k];
            }
            /* Step 6 */
            t = sqrt(orc_dot(n, w, w));
            if (always_reorth || t < eta * omega) {
                /* Steps 8-10: one more CGS (or MGS) pass. */
                if (mgs) {
                    mgs_pass(fmt, j, Q, sc, n, w, u, s);
                } else {
                    if (gram) {
                        /* V^T (w - V h) = V^T w - (V^T V) h = h - G h */
                        for (int32_t k = 0; k < j; ++k) {
                            double gh = 0.0;
                            for (int32_t l = 0; l < j; ++l)
                                gh += G[(size_t)k * (m + 1) + l] * h[l];
                            u[k] = h[k] - gh;
                        }
                    } else {
                        multidot(fmt, j, Q, sc, n, w, u, part);
                    }
                    basis_combine(fmt, j, Q, sc, n, u, s);
#pragma omp parallel for schedule(static)
                    for (int32_t i = 0; i < n; ++i)
                        w[i] = w[i] - s[i];
                }
                for (int32_t k = 0; k < j; ++k)
                    h[k] = h[k] + u[k];
                double t2 = sqrt(orc_dot(n, w, w));
                res->reorths += 1;
                /* Step 12, reading R2: taken literally the test would end
                 * every re-orthogonalised cycle; it is read as "the second
                 * pass again lost more than a factor eta", i.e. w lies
                 * numerically in span(V_j). */
                brk = (t2 == 0.0) || (t2 < eta * t);
                t = t2;
            } else {
                brk = (t == 0.0);
            }
        column:
            for (int32_t k = 0; k < j; ++k)
                HH(k, jc) = h[k];
            HH(j, jc) = t;
            if (dbg_H && cycle == 0)
                for (int32_t k = 0; k <= j; ++k)
                    dbg_H[(size_t)jc * (size_t)(m + 1) + (size_t)k] = HH(k, jc);

            /* Step 17, updated column by column (Section 3): apply the
             * previous rotations to the new column, then form rotation j.
             * Convention (R10): rho = sqrt(a^2 + b^2), c = a/rho, s = b/rho. */
            for (int32_t i = 0; i < jc; ++i) {
                double a0 = HH(i, jc), a1 = HH(i + 1, jc);
                HH(i, jc) = cs[i] * a0 + sn[i] * a1;
                HH(i + 1, jc) = -sn[i] * a0 + cs[i] * a1;
            }
            {
                double a = HH(jc, jc), bb = HH(j, jc);
                double rr = sqrt(a * a + bb * bb);
                if (rr > 0.0) {
                    cs[jc] = a / rr;
                    sn[jc] = bb / rr;
                } else {
                    cs[jc] = 1.0;
                    sn[jc] = 0.0;
                }
                HH(jc, jc) = rr;
                HH(j, jc) = 0.0;
                g[j] = -sn[jc] * g[jc];
                g[jc] = cs[jc] * g[jc];
            }
            it += 1;
            last_rec = fabs(g[j]) / nb;
            if (hist)
                hist[it - 1] = last_rec;
            meff = j;
            int finite = isfinite(omega) && isfinite(t) && isfinite(g[j]);
            int conv = fabs(g[j]) <= tau * nb;   /* recurrence residual (R7) */
            if (brk)
                res->breakdowns += 1;
            int last = brk || conv || it >= opt->maxiter || !finite || j == m;
            if (last && !(dbg_V && cycle == 0 && t > 0.0 && finite))
                break;
            /* Steps 13-14: v = w / h_{j+1,j} (IEEE division, R18), stored
             * through the accessor as column j+1. */
#pragma omp parallel for schedule(static)
            for (int32_t i = 0; i < n; ++i)
                v[i] = w[i] / t;
            orc_encode(fmt, n, v, Q[j], &sc[j]);
            nstored = j + 1;
            if (last)
                break;
        }
        if (dbg_V && cycle == 0) {
            for (int32_t k = 0; k < nstored; ++k)
                orc_decode(fmt, n, Q[k], sc[k], dbg_V + (size_t)k * (size_t)n);
            if (dbg_steps) {
                dbg_steps[0] = meff;
                dbg_steps[1] = nstored;
            }
        }

        /* Step 17: y = R^{-1} g by back substitution; x += M^{-1} V_m y. */
        for (int32_t i = meff - 1; i >= 0; --i) {
            double acc = g[i];
            for (int32_t k = i + 1; k < meff; ++k)
                acc -= HH(i, k) * y[k];
            y[i] = acc / HH(i, i);
        }
        if (cycle_len)
            cycle_len[cycle] = meff;
        basis_combine(fmt, meff, Q, sc, n, y, s);
        apply_precond(&M, n, rp, ci, s, z);
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i)
            x[i] = x[i] + z[i];
        cycle += 1;
    }
#undef HH

    /* true residual of the returned x */
    orc_spmv(n, rp, ci, val, x, r);
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i)
        r[i] = b[i] - r[i];
    res->true_rel_res = sqrt(orc_dot(n, r, r)) / nb;
    res->recurrence_rel_res = last_rec;
    res->iterations = it;
    res->status = status;
    if (status == ORC_OK && !all_finite(n, x))
        res->status = status = ORC_E_NONFINITE;

    for (int32_t k = 0; k <= m; ++k)
        free(Q[k]);
    free(Q); free(sc); free(r); free(v); free(z); free(w); free(s); free(xprev);
    free(part); free(H); free(h); free(u); free(cs); free(sn); free(g); free(y);
    free(G); free(gv); free(grow);
    free(M.dinv);
    free(M.bj);
    return status;
}

void orc_set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int orc_stencil_apply(int32_t n, const int32_t *rp, const int32_t *ci, const double *val,
                      const int32_t grid[3], const uint16_t *codes, int64_t st_ld,
                      const double *v, double *z)
{
    if (n < 0 || !grid || grid[0] < 1 || grid[1] < 1 || grid[2] < 1 ||
        (int64_t)grid[0] * grid[1] * grid[2] != n || st_ld < n ||
        (n > 0 && (!rp || !ci || !val || !codes || !v || !z)))
        return ORC_E_ARG;
    precond M = {ORC_PC_STENCIL, NULL, NULL, 0, NULL, codes, grid[0], grid[1], grid[2], st_ld};
    M.dinv = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    int bad = 0;
    for (int32_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p)
            if (ci[p] == i)
                d = val[p];
        if (d == 0.0)
            bad = 1;
        M.dinv[i] = 1.0 / d;
    }
    if (!bad)
        apply_stencil(&M, n, v, z);
    free(M.dinv);
    return bad ? ORC_E_ARG : 0;
}
