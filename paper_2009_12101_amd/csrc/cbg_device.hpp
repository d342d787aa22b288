// Device-side building blocks of the gfx950 CB-GMRES library:
//   * storage-format traits: the accessor of Section 5.2 (decode to FP64 in
//     registers on every read, encode on every store);
//   * deterministic wave / block / grid reductions (no floating-point
//     atomics: results are bitwise reproducible run to run);
//   * the device state block that carries the scalars of Fig. 1 between
//     kernels so that the host synchronises only once per restart cycle.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cbg {

constexpr int BLK = 256;                 // threads per block (4 wave64)
constexpr int NWAVE = BLK / 64;
constexpr int MAX_RESTART = 512;
constexpr int MAX_GRID = 4096;           // upper bound on blocks of reducing kernels
constexpr int SPMV_MAX_GRID = 8192;      // the sliced-ELL SpMV's bound (its partials have rows of their own)

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// Storage formats.  Each thread of a tile owns CH chunks of VW consecutive
// entries; chunk c of thread t starts at tile_base + (c*BLK + t)*VW, so each
// chunk of the stored vector is one 16-byte load and a wave's load of one
// chunk index is contiguous.
// ---------------------------------------------------------------------------

enum { F_FP64 = 0, F_FP32 = 1, F_FP16 = 2, F_BF16 = 3, F_E4M3 = 4, F_INT32 = 5, F_INT16 = 6,
       F_FP16S = 7 };

__host__ __device__ constexpr int fmt_bytes(int f)
{
    return f == F_FP64 ? 8 : (f == F_FP32 || f == F_INT32) ? 4 : f == F_E4M3 ? 1 : 2;
}

// Round-to-nearest-even of |v| (an FP64 value) to a binary format with MB
// explicit mantissa bits, minimum normal exponent EMIN and exponent bias
// BIAS, returning the magnitude code.  Normal range: the fp64 exponent and
// mantissa fields, read as one integer, are rounded to MB mantissa bits by
// adding half an ulp minus one plus the kept LSB and shifting (a carry moves
// into the exponent, which is the correct result); the exponent is then
// rebiased.  Subnormal range: |v| * 2^(MB-EMIN) is exact and rint() rounds
// it to the nearest integer, ties to even.  Requires |v| <= the format's
// largest finite value.
template <int MB, int EMIN, int BIAS>
__device__ __forceinline__ uint32_t rne_code(double v)
{
    uint64_t a = (uint64_t)__double_as_longlong(v) & 0x7FFFFFFFFFFFFFFFull;
    int e = (int)(a >> 52) - 1023;
    if (e >= EMIN) {
        constexpr int SH = 52 - MB;
        uint64_t r = (a + ((1ull << (SH - 1)) - 1ull) + ((a >> SH) & 1ull)) >> SH;
        return (uint32_t)(r - ((uint64_t)(1023 - BIAS) << MB));
    }
    return (uint32_t)rint(ldexp(fabs(v), MB - EMIN));
}

__device__ __forceinline__ uint32_t sign_of(double v)
{
    return (uint32_t)((uint64_t)__double_as_longlong(v) >> 63);
}

__device__ __forceinline__ double dec_f16(uint32_t c)
{
    _Float16 h = __builtin_bit_cast(_Float16, (unsigned short)c);
    return (double)(float)h;
}
__device__ __forceinline__ double dec_bf16(uint32_t c) { return (double)__uint_as_float(c << 16); }
// e4m3 (OCP E4M3FN) code -> value: gfx950's fp8 conversion, exact for every
// finite code (each is a float); S.1111.111 is NaN, which the encoder never
// writes.
__device__ __forceinline__ double dec_e4m3(uint32_t c)
{
    return (double)__builtin_amdgcn_cvt_f32_fp8((int)c, 0);
}

// Encoding parameters of one stored vector, derived from its scale.
struct EncParam {
    double scale;   // e4m3, fp16s: 2^k ; int: sigma ; else 1
    int k;          // e4m3, fp16s exponent
};

template <int F> struct Fmt;

// VW entries per 16-byte chunk, CH chunks per thread and tile, KC stored
// vectors per multi-dot batch, UNR vectors in flight in the update loop.
template <> struct Fmt<F_FP64> {
    static constexpr int VW = 2, CH = 4, KC = 4, UNR = 2;
    static constexpr bool SCALED = false;
    __device__ static void dec(u32x4 q, double, double *d)
    {
        d[0] = __longlong_as_double(((uint64_t)q.y << 32) | q.x);
        d[1] = __longlong_as_double(((uint64_t)q.w << 32) | q.z);
    }
    __device__ static u32x4 enc(const double *v, EncParam)
    {
        uint64_t a = (uint64_t)__double_as_longlong(v[0]), b = (uint64_t)__double_as_longlong(v[1]);
        u32x4 q = {(uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32)};
        return q;
    }
};

template <> struct Fmt<F_FP32> {
    static constexpr int VW = 4, CH = 2, KC = 8, UNR = 4;
    static constexpr bool SCALED = false;
    __device__ static void dec(u32x4 q, double, double *d)
    {
        d[0] = (double)__uint_as_float(q.x); d[1] = (double)__uint_as_float(q.y);
        d[2] = (double)__uint_as_float(q.z); d[3] = (double)__uint_as_float(q.w);
    }
    __device__ static u32x4 enc(const double *v, EncParam)
    {
        // the hardware conversion rounds to nearest even: one rounding
        u32x4 q = {__float_as_uint((float)v[0]), __float_as_uint((float)v[1]),
                   __float_as_uint((float)v[2]), __float_as_uint((float)v[3])};
        return q;
    }
};

#ifndef CBG_KC16
#define CBG_KC16 4
#endif
#ifndef CBG_UNR16
#define CBG_UNR16 2
#endif
#ifndef CBG_CH16
#define CBG_CH16 2
#endif
template <int F> struct Fmt16 {
    static constexpr int VW = 8, CH = CBG_CH16, KC = CBG_KC16, UNR = CBG_UNR16;
    static constexpr bool SCALED = (F == F_INT16 || F == F_FP16S);
    __device__ static double one(uint32_t c, double s)
    {
        if constexpr (F == F_FP16) return dec_f16(c);
        else if constexpr (F == F_FP16S) return dec_f16(c) * s;   // s = 2^k: exact
        else if constexpr (F == F_BF16) return dec_bf16(c);
        else return s * (double)(int16_t)(uint16_t)c;
    }
    __device__ static void dec(u32x4 q, double s, double *d)
    {
        uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            d[2 * i] = one(w[i] & 0xFFFFu, s);
            d[2 * i + 1] = one(w[i] >> 16, s);
        }
    }
    __device__ static uint32_t code(double v, EncParam p)
    {
        if constexpr (F == F_FP16) return rne_code<10, -14, 15>(v) | (sign_of(v) << 15);
        else if constexpr (F == F_FP16S) {
            const double x = ldexp(v, -p.k);                           // exact
            return rne_code<10, -14, 15>(x) | (sign_of(x) << 15);
        } else if constexpr (F == F_BF16) return rne_code<7, -126, 127>(v) | (sign_of(v) << 15);
        else {
            double t = p.scale > 0.0 ? rint(v / p.scale) : 0.0;
            t = fmin(fmax(t, -32767.0), 32767.0);
            return (uint32_t)(uint16_t)(int16_t)t;
        }
    }
    __device__ static u32x4 enc(const double *v, EncParam p)
    {
        u32x4 q;
        q.x = code(v[0], p) | (code(v[1], p) << 16);
        q.y = code(v[2], p) | (code(v[3], p) << 16);
        q.z = code(v[4], p) | (code(v[5], p) << 16);
        q.w = code(v[6], p) | (code(v[7], p) << 16);
        return q;
    }
};
template <> struct Fmt<F_FP16> : Fmt16<F_FP16> {};
template <> struct Fmt<F_BF16> : Fmt16<F_BF16> {};
template <> struct Fmt<F_INT16> : Fmt16<F_INT16> {};
template <> struct Fmt<F_FP16S> : Fmt16<F_FP16S> {};

template <> struct Fmt<F_INT32> {
    static constexpr int VW = 4, CH = 2, KC = 8, UNR = 4;
    static constexpr bool SCALED = true;
    __device__ static void dec(u32x4 q, double s, double *d)
    {
        d[0] = s * (double)(int32_t)q.x; d[1] = s * (double)(int32_t)q.y;
        d[2] = s * (double)(int32_t)q.z; d[3] = s * (double)(int32_t)q.w;
    }
    __device__ static uint32_t code(double v, EncParam p)
    {
        double t = p.scale > 0.0 ? rint(v / p.scale) : 0.0;
        t = fmin(fmax(t, -2147483647.0), 2147483647.0);
        return (uint32_t)(int32_t)t;
    }
    __device__ static u32x4 enc(const double *v, EncParam p)
    {
        u32x4 q = {code(v[0], p), code(v[1], p), code(v[2], p), code(v[3], p)};
        return q;
    }
};

template <> struct Fmt<F_E4M3> {
    static constexpr int VW = 16, CH = 1, KC = 4, UNR = 2;
    static constexpr bool SCALED = true;
    __device__ static void dec(u32x4 q, double s, double *d)
    {
        // two codes per conversion (bytes 0-1, then 2-3, of each word);
        // s = 2^k, so the products are exact
        uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], false);
            const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], true);
            d[4 * i + 0] = (double)lo[0] * s;
            d[4 * i + 1] = (double)lo[1] * s;
            d[4 * i + 2] = (double)hi[0] * s;
            d[4 * i + 3] = (double)hi[1] * s;
        }
    }
    __device__ static uint32_t code(double v, EncParam p)
    {
        double x = ldexp(v, -p.k);                                     // exact
        return rne_code<3, -6, 7>(x) | (sign_of(x) << 7);
    }
    __device__ static u32x4 enc(const double *v, EncParam p)
    {
        uint32_t w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            w[i] = code(v[4 * i], p) | (code(v[4 * i + 1], p) << 8) |
                   (code(v[4 * i + 2], p) << 16) | (code(v[4 * i + 3], p) << 24);
        u32x4 q = {w[0], w[1], w[2], w[3]};
        return q;
    }
};

// Scale of a unit vector whose largest magnitude is vinf (Section 5.2 for
// the integer formats; the power-of-two rules for e4m3, max|v| 2^-k in
// (224, 448], and the scaled float16, max|v| 2^-k in (32752, 65504]).
__device__ inline EncParam make_param(int f, double vinf)
{
    EncParam p{1.0, 0};
    if (f == F_INT32)
        p.scale = vinf / 2147483647.0;
    else if (f == F_INT16)
        p.scale = vinf / 32767.0;
    else if (f == F_E4M3) {
        int k = 0;
        if (vinf > 0.0) {
            k = ilogb(vinf) - 8;
            if (ldexp(vinf, -k) > 448.0)
                k += 1;
        }
        p.k = k;
        p.scale = ldexp(1.0, k);
    } else if (f == F_FP16S) {
        int k = 0;
        if (vinf > 0.0) {
            k = ilogb(vinf) - 15;
            if (ldexp(vinf, -k) > 65504.0)
                k += 1;
        }
        p.k = k;
        p.scale = ldexp(1.0, k);
    }
    return p;
}

__device__ __forceinline__ EncParam param_from_scale(int f, double s)
{
    EncParam p{s, 0};
    if (f == F_E4M3 || f == F_FP16S)
        p.k = ilogb(s);
    return p;
}

// ---------------------------------------------------------------------------
// Deterministic reductions.
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
        x += __shfl_xor(x, d);
    return x;
}
__device__ __forceinline__ double wave_max(double x)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
        x = fmax(x, __shfl_xor(x, d));
    return x;
}

// Row i's diagonal entry (the last one in CSR order if stored twice, 0 if
// none), read by a half-wave (32 lanes) on the row's entries l, l + 32, ...
// and returned on every lane of it; `chunks` (the row's 32-entry chunks) is
// uniform over the wave.
__device__ __forceinline__ double hw_row_diag(int64_t i, int beg, int end, int chunks,
                                              const int32_t *__restrict__ ci,
                                              const double *__restrict__ val)
{
    const int lane = threadIdx.x & 31, half = threadIdx.x & 32;
    double d = 0.0;
    for (int q = 0; q < chunks; ++q) {
        const int p = beg + q * 32 + lane;
        const bool hit = p < end && ci[p] == i;
        const double v = hit ? val[p] : 0.0;
        const uint32_t mine = (uint32_t)(__ballot(hit) >> half);
        const double last = __shfl(v, half + (mine ? 31 - __clz(mine) : 0));
        if (mine)
            d = last;
    }
    return d;
}

// The value of lane (l xor P>>10) for an immediate ds_swizzle bit-mask
// pattern P (and-mask 31, or-mask 0, xor-mask P>>10: the partner within the
// lane's 32-lane half, no address arithmetic).
template <int P>
__device__ __forceinline__ double swizzle64(double v)
{
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), P);
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), P);
    return __hiloint2double(hi, lo);
}

// The value of lane (l xor d); d a power of two known after unrolling.
__device__ __forceinline__ double xor_lane(double v, int d)
{
    switch (d) {
    case 1: return swizzle64<(1 << 10) | 0x1F>(v);
    case 2: return swizzle64<(2 << 10) | 0x1F>(v);
    case 4: return swizzle64<(4 << 10) | 0x1F>(v);
    case 8: return swizzle64<(8 << 10) | 0x1F>(v);
    case 16: return swizzle64<(16 << 10) | 0x1F>(v);
    default: return __shfl_xor(v, d);
    }
}

// Reduce N per-lane values across the wave at once: N-1 exchanges halve the
// set each lane holds, then log2(64/N) exchanges finish the sums.  Lane l
// ends with (in a[0]) the wave total of index bitrev_N(l mod N).
template <int N>
__device__ __forceinline__ void wave_transpose_sum(double (&a)[N])
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1, cnt = N; cnt > 1; d <<= 1, cnt >>= 1) {
        const bool up = lane & d;
#pragma unroll
        for (int i = 0; i < cnt / 2; ++i) {
            // both candidates as register values: a select between two array
            // loads would otherwise become a load at a lane-dependent index,
            // which the backend emulates with compare/select chains
            double lo = a[i], hi = a[i + cnt / 2];
            asm volatile("" : "+v"(lo), "+v"(hi));
            const double send = up ? lo : hi;
            const double keep = up ? hi : lo;
            a[i] = keep + xor_lane(send, d);
        }
    }
#pragma unroll
    for (int d = N; d < 64; d <<= 1)
        a[0] += xor_lane(a[0], d);
}

template <int N>
__device__ __forceinline__ int bitrev(int l)
{
    int r = 0;
#pragma unroll
    for (int b = 1, o = N >> 1; b < N; b <<= 1, o >>= 1)
        if (l & b)
            r |= o;
    return r;
}

// Block partials of a reduction, value-major: value v of block b at
// part[v * stride + b].  A producer kernel writes its block's values with
// plain stores; a one-block reduce kernel launched after it (the kernel
// boundary makes the writes visible) folds them in block order.  No block
// waits for or fences against another, and the sums are bitwise
// reproducible.
struct RedArgs {
    double *part;
    int stride;          // >= the producer's grid size
};

// Block-level sum and max of one value per thread; result valid in thread 0.
__device__ inline void block_sum_max(double &s, double &m)
{
    __shared__ double ls[NWAVE], lm[NWAVE];
    s = wave_sum(s);
    m = wave_max(m);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        ls[w] = s;
        lm[w] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < NWAVE; ++i) {
            s += ls[i];
            m = fmax(m, lm[i]);
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Device state of one solve (the scalars of Fig. 1 and the cycle flags).
// ---------------------------------------------------------------------------
struct DevState {
    // constants
    double nb;          // ||b||_2
    double tau_nb;      // tol * ||b||_2
    double eta;
    int64_t maxiter;
    int32_t m, fmt;
    int32_t n, pad0;
    // counters over the whole solve
    int64_t it;         // Arnoldi steps taken
    int64_t reorths;
    int32_t breakdowns;
    int32_t nonfinite;  // a non-finite scalar appeared
    // current cycle
    int32_t done;       // cycle finished: later step kernels do nothing
    int32_t jeff;       // steps taken in this cycle
    int32_t jprev;      // steps taken in the previous cycle
    int32_t reorth_all; // re-orthogonalise on every step (CGS2 ablation)
    int32_t reorth;     // the current step re-orthogonalises
    int32_t conv;       // recurrence residual met the tolerance
    int32_t hard;       // the current step took the explicit form (t1 << omega)
    int32_t pad1;
    double beta;        // ||r||_2 at the cycle start
    double rmax;        // max |r_i| at the cycle start
    double omega;       // ||A M^-1 v||_2 (step 4)
    double t;           // h_{j+1,j}
    double wmax;        // ||w||_inf after the last orthogonalisation pass
    double last_rec;    // |g_{j+1}| / ||b||
    double carry;       // entry j-1 of the new Hessenberg column after the j-1 stored
                        // rotations (formed by the one-pass update's column block)
    double pad2[3];
};

}  // namespace cbg
