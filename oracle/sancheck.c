/*
 * Memory and undefined-behaviour check of the CPU oracle -- TEST
 * INFRASTRUCTURE ONLY.
 *
 * A driver that the test suite compiles together with oracle.c under
 * AddressSanitizer and UndefinedBehaviorSanitizer (gcc, host code only) and
 * runs: every storage format through encode/decode, the SpMV and the dot,
 * block-Jacobi set-up, and restarted CB-GMRES (Fig. 1) with every format,
 * every preconditioner and every variant bit, with and without the debug
 * outputs, on small seeded systems.  Inputs include zeros, a zero vector, a
 * vector with one entry and a row of length one.  Prints one line per case;
 * exits 1 if a call returns an unexpected status, so the sanitizers'
 * reports and the results are both checked.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

typedef struct {
    int32_t n, nnz;
    int32_t *rp, *ci;
    double *val;
} csr;

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;

/* splitmix64 (Steele, Lea, Flood 2014): uniform in [-1, 1) */
static double urand(void)
{
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-52 - 1.0;
}

/* 3D 7-point convection-diffusion on an nx x ny x nz grid (x fastest):
 * 6 + shift on the diagonal, -1 - c and -1 + c off it along x, -1 along y
 * and z; rows on the boundary drop the missing neighbours. */
static csr grid7(int nx, int ny, int nz, double c, double shift)
{
    csr A;
    A.n = nx * ny * nz;
    A.rp = malloc(sizeof(int32_t) * (A.n + 1));
    A.ci = malloc(sizeof(int32_t) * 7 * A.n);
    A.val = malloc(sizeof(double) * 7 * A.n);
    int32_t p = 0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int i = (z * ny + y) * nx + x;
                A.rp[i] = p;
                const int dz[7] = {-1, 0, 0, 0, 0, 0, 1}, dy[7] = {0, -1, 0, 0, 0, 1, 0},
                          dx[7] = {0, 0, -1, 0, 1, 0, 0};
                for (int k = 0; k < 7; ++k) {
                    const int xx = x + dx[k], yy = y + dy[k], zz = z + dz[k];
                    if (xx < 0 || xx >= nx || yy < 0 || yy >= ny || zz < 0 || zz >= nz)
                        continue;
                    A.ci[p] = (zz * ny + yy) * nx + xx;
                    A.val[p] = k == 3 ? 6.0 + shift : dx[k] < 0 ? -1.0 - c
                               : dx[k] > 0 ? -1.0 + c : -1.0;
                    ++p;
                }
            }
    A.rp[A.n] = p;
    A.nnz = p;
    return A;
}

static void csr_free(csr *A)
{
    free(A->rp);
    free(A->ci);
    free(A->val);
}

static int failures = 0;

static void expect(int ok, const char *what)
{
    printf("%s %s\n", ok ? "ok  " : "FAIL", what);
    if (!ok)
        ++failures;
}

static void check_formats(void)
{
    const int64_t lens[] = {0, 1, 1000};
    for (int fmt = ORC_FP64; fmt <= ORC_FP16S; ++fmt) {
        const int nb = orc_format_bytes(fmt);
        for (int t = 0; t < 3; ++t) {
            const int64_t n = lens[t];
            double *v = malloc(sizeof(double) * (n + 1));
            double *w = malloc(sizeof(double) * (n + 1));
            unsigned char *q = malloc((size_t)nb * (n + 1));
            for (int64_t i = 0; i < n; ++i)
                v[i] = (i % 7 == 0) ? 0.0 : urand() * ldexp(1.0, (int)(i % 9) - 4);
            double scale = 0.0;
            char what[96];
            int rc = orc_encode(fmt, n, v, q, &scale);
            int rd = orc_decode(fmt, n, q, scale, w);
            int finite = 1;
            for (int64_t i = 0; i < n; ++i)
                finite &= isfinite(w[i]) && (v[i] != 0.0 || w[i] == 0.0);
            snprintf(what, sizeof what, "encode/decode format %d n=%lld", fmt, (long long)n);
            expect(rc == ORC_OK && rd == ORC_OK && finite, what);
            /* a zero vector */
            for (int64_t i = 0; i < n; ++i)
                v[i] = 0.0;
            rc = orc_encode(fmt, n, v, q, &scale);
            rd = orc_decode(fmt, n, q, scale, w);
            int zero = 1;
            for (int64_t i = 0; i < n; ++i)
                zero &= w[i] == 0.0;
            snprintf(what, sizeof what, "zero vector format %d n=%lld", fmt, (long long)n);
            expect(rc == ORC_OK && rd == ORC_OK && zero, what);
            free(v);
            free(w);
            free(q);
        }
    }
    expect(orc_format_bytes(99) == 0, "unknown format has no width");
}

static void check_kernels(const csr *A)
{
    double *x = malloc(sizeof(double) * A->n), *y = malloc(sizeof(double) * A->n);
    for (int i = 0; i < A->n; ++i)
        x[i] = urand();
    orc_spmv(A->n, A->rp, A->ci, A->val, x, y);
    const double d = orc_dot(A->n, x, y);
    expect(isfinite(d), "spmv and dot");
    for (int bs = 1; bs <= 8; bs *= 2) {
        const int nblk = (A->n + bs - 1) / bs;
        double *vals = malloc(sizeof(double) * nblk * bs * bs);
        int8_t *prec = malloc(nblk);
        char what[64];
        snprintf(what, sizeof what, "block-Jacobi set-up bs=%d", bs);
        expect(orc_block_jacobi(A->n, A->rp, A->ci, A->val, bs, 16, vals, prec) == ORC_OK,
               what);
        free(vals);
        free(prec);
    }
    free(x);
    free(y);
}

static void check_gmres(const csr *A, int nx, int ny, int nz)
{
    double *b = malloc(sizeof(double) * A->n), *x = malloc(sizeof(double) * A->n);
    for (int i = 0; i < A->n; ++i)
        b[i] = urand();
    /* the sparse preconditioner: Jacobi's values on A's pattern */
    float *pv = malloc(sizeof(float) * A->nnz);
    for (int i = 0; i < A->n; ++i)
        for (int p = A->rp[i]; p < A->rp[i + 1]; ++p)
            pv[p] = A->ci[p] == i ? (float)(1.0 / A->val[p]) : 0.0f;
    /* the stored stencil form: small corrections on the slots */
    uint16_t *codes = malloc(sizeof(uint16_t) * 27 * (size_t)A->n);
    for (size_t k = 0; k < 27 * (size_t)A->n; ++k)
        codes[k] = (k % 5 == 0) ? 0x2000u : 0u;          /* float16 2^-7 */
    const int variants[] = {0, ORC_V_SPMV_VHAT, ORC_V_ALWAYS_REORTH, ORC_V_MGS, ORC_V_GRAM,
                            ORC_V_GRAM | ORC_V_ONEPASS};
    const int maxit = 300;
    double *hist = malloc(sizeof(double) * maxit), *cres = malloc(sizeof(double) * (maxit + 1));
    int32_t *clen = malloc(sizeof(int32_t) * maxit);
    const int m = 12;
    double *dV = malloc(sizeof(double) * (size_t)A->n * (m + 1));
    double *dH = malloc(sizeof(double) * (m + 1) * m);
    int32_t steps[2];
    for (int fmt = ORC_FP64; fmt <= ORC_FP16S; ++fmt)
        for (int pc = ORC_PC_NONE; pc <= ORC_PC_STENCIL; ++pc)
            for (int v = 0; v < 6; ++v) {
                if (v != 0 && pc != ORC_PC_NONE && fmt != ORC_FP16)
                    continue;            /* variants: every format without M, fp16 with each M */
                orc_opts o;
                memset(&o, 0, sizeof o);
                o.restart = m;
                o.format = fmt;
                o.tol = 1e-8;
                o.maxiter = maxit;
                o.precond = pc;
                o.p_val = pv;
                o.fallback = 1;
                o.variant = variants[v];
                o.p_stencil = codes;
                o.grid[0] = nx;
                o.grid[1] = ny;
                o.grid[2] = nz;
                o.st_ld = A->n;
                orc_result r;
                memset(x, 0, sizeof(double) * A->n);
                const int dbg = (fmt + pc + v) % 2 == 0;
                const int rc = orc_gmres(A->n, A->rp, A->ci, A->val, b, x, &o, &r, hist, cres,
                                         clen, dbg ? dV : NULL, dbg ? dH : NULL,
                                         dbg ? steps : NULL);
                char what[128];
                snprintf(what, sizeof what,
                         "gmres format %d precond %d variant %d: status %d, %lld steps, "
                         "res %.2e", fmt, pc, variants[v], rc, (long long)r.iterations,
                         r.true_rel_res);
                expect((rc == ORC_OK || rc == ORC_NOT_CONVERGED) && isfinite(r.true_rel_res),
                       what);
            }
    /* b = 0 and a one-unknown system */
    {
        orc_opts o;
        memset(&o, 0, sizeof o);
        o.restart = 5;
        o.format = ORC_FP16;
        o.tol = 1e-10;
        o.maxiter = 10;
        orc_result r;
        memset(b, 0, sizeof(double) * A->n);
        memset(x, 0, sizeof(double) * A->n);
        expect(orc_gmres(A->n, A->rp, A->ci, A->val, b, x, &o, &r, NULL, NULL, NULL, NULL, NULL,
                         NULL) == ORC_OK,
               "b = 0");
        const int32_t rp1[2] = {0, 1}, ci1[1] = {0};
        const double v1[1] = {4.0}, b1[1] = {2.0};
        double x1[1] = {0.0};
        expect(orc_gmres(1, rp1, ci1, v1, b1, x1, &o, &r, NULL, NULL, NULL, NULL, NULL, NULL) ==
                       ORC_OK &&
                   x1[0] == 0.5,
               "n = 1");
    }
    free(b);
    free(x);
    free(pv);
    free(codes);
    free(hist);
    free(cres);
    free(clen);
    free(dV);
    free(dH);
}

int main(void)
{
    orc_set_threads(2);
    check_formats();
    csr A = grid7(6, 5, 4, 0.3, 0.05);
    check_kernels(&A);
    check_gmres(&A, 6, 5, 4);
    csr_free(&A);
    printf("%s: %d failure(s)\n", failures ? "FAILED" : "PASSED", failures);
    return failures ? 1 : 0;
}
