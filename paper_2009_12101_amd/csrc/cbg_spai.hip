// gfx950 kernels of the learned sparse-approximate-inverse preconditioner
// (an extension of the paper, which preconditions with scalar Jacobi,
// Section 6).  A per-row network 64 -> 64 -> 64 -> 32 (ReLU, bf16 weights,
// fp32 biases and accumulation on the MFMA units) maps features of row i of A
// to corrections of the Jacobi row: P_{i,c} = fl32((delta_{p,13} + O_{i,p}) /
// a_ii) on A's pattern, p the 27-point slot of (i, c).  Training minimises
// (1/|B|) sum_k ||A P v_k - v_k||^2 over Arnoldi vectors v_k with the
// project's own backward pass and Adam.
//
// MFMA: __builtin_amdgcn_mfma_f32_16x16x16bf16_1k, one wave per 16-row tile.
// Each layer is computed transposed, H^T = W^T X^T, so that the result's
// register layout (lane l holds rows 4(l/16)+r of column l%16) is exactly the
// B-operand layout of the next product: layers chain without data movement.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "../../include/cbgmres.h"
#include "cbg_device.hpp"
#include "cbg_launch.hpp"

namespace cbg {
namespace spai {

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int NF = 64, NH = 64, NO = 32, NSLOT = 27, CENTER = 13;
constexpr int NBR = 32;     // first neighbour-diagonal feature
// parameter vector: W1 (64x64) b1 (64) W2 (64x64) b2 (64) W3 (64x32) b3 (32)
constexpr int OW1 = 0, OB1 = OW1 + NF * NH, OW2 = OB1 + NH, OB2 = OW2 + NH * NH,
              OW3 = OB2 + NH, OB3 = OW3 + NH * NO, NPARAM = OB3 + NO;
// bf16 weights: W1, W2, W3 back to back
constexpr int QW1 = 0, QW2 = NF * NH, QW3 = QW2 + NH * NH, NWBF = QW3 + NH * NO;
static_assert(NPARAM == CBG_SPAI_NPARAM, "parameter count");
static_assert(NWBF == CBG_SPAI_NWEIGHT, "weight count");

__device__ __forceinline__ uint16_t bf16_of(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);        // round to nearest even (finite inputs)
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float f_of(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// fp64 -> bf16 in one rounding
__device__ __forceinline__ uint16_t bf16_of_d(double v)
{
    return (uint16_t)(rne_code<7, -126, 127>(v) | (sign_of(v) << 15));
}

__device__ __forceinline__ f32x4 mfma(s16x4 a, s16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// 27-point slot of entry (row, col) on an nx*ny*nz grid, or -1.
// Grid position of row i (x fastest); n < 2^31, so 32-bit arithmetic.
struct RowPos {
    int x, y;
};
__device__ __forceinline__ RowPos row_pos(int64_t i, int nx, int ny)
{
    const uint32_t u = (uint32_t)i, q = u / (uint32_t)nx;
    return {(int)(u - q * (uint32_t)nx), (int)(q % (uint32_t)ny)};
}

// Slot (0..26, 13 = the diagonal) of column c in row i on an nx x ny x nz
// grid, or -1 if c is not one of i's 27 stencil neighbours.  A neighbour is
// at offset d = c - i = dz nx ny + dy nx + dx with dx, dy, dz in {-1, 0, 1}
// and its x, y inside the grid (then its z is too, as 0 <= c < n); since
// grid points and indices correspond one to one, a triple that passes these
// tests is the column's true offset.  For nx, ny >= 3 the ranges of d for
// dz = -1, 0, 1 (and then of d - dz nx ny for dy) are disjoint, so the
// triple follows from comparisons; smaller grids try the nine (dz, dy).
__device__ __forceinline__ int slot_at(RowPos r, int64_t i, int64_t c, int nx, int ny)
{
    const int64_t d = c - i, S = (int64_t)nx * ny;
    auto check = [&](int64_t dz, int64_t dy) -> int {
        const int64_t dx = d - dz * S - dy * nx;
        if (dx < -1 || dx > 1)
            return -1;
        const int64_t x = r.x + dx, y = r.y + dy;
        if (x < 0 || x >= nx || y < 0 || y >= ny)
            return -1;
        return (int)((dz + 1) * 9 + (dy + 1) * 3 + (dx + 1));
    };
    if (nx >= 3 && ny >= 3) {
        const int64_t zb = S - nx - 1;            // |d| >= zb only for dz = +-1
        const int64_t dz = d >= zb ? 1 : (d <= -zb ? -1 : 0);
        const int64_t rem = d - dz * S;
        const int64_t dy = rem >= nx - 1 ? 1 : (rem <= -(nx - 1) ? -1 : 0);
        return check(dz, dy);
    }
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy) {
            const int s = check(dz, dy);
            if (s >= 0)
                return s;
        }
    return -1;
}

// Row kernels: a half-wave (32 lanes) per row, HWR rows per 256-thread
// block, lane l on the row's entries l, l + 32, ...: a row's indices and
// values are read as one contiguous run, its outputs written the same way.
// Loops that contain a barrier run the same number of times in every
// half-wave of the block (the block's largest chunk count).
constexpr int HWR = 8;

// Largest number of 32-entry chunks over the block's rows (block-uniform
// call).
__device__ __forceinline__ int block_chunks(int chunks)
{
    __shared__ int m[HWR];
    const int g = threadIdx.x >> 5;
    if ((threadIdx.x & 31) == 0)
        m[g] = chunks;
    __syncthreads();
    int r = 0;
#pragma unroll
    for (int k = 0; k < HWR; ++k)
        r = max(r, m[k]);
    __syncthreads();
    return r;
}

// The diagonal of A (0 where a row stores none).
__global__ __launch_bounds__(256) void k_diag(int n, const int32_t *__restrict__ rp,
                                              const int32_t *__restrict__ ci,
                                              const double *__restrict__ val,
                                              double *__restrict__ diag)
{
    const int g = threadIdx.x >> 5, lane = threadIdx.x & 31;
    for (int64_t base = (int64_t)blockIdx.x * HWR; base < n; base += (int64_t)gridDim.x * HWR) {
        const int64_t i = base + g;
        const bool live = i < n;
        const int beg = live ? rp[i] : 0, end = live ? rp[i + 1] : 0;
        const int ch = (end - beg + 31) / 32;
        const int chunks = max(ch, __shfl_xor(ch, 32));          // uniform over the wave
        const double d = hw_row_diag(i, beg, end, chunks, ci, val);
        if (live && lane == 0)
            diag[i] = d;
    }
}

// Orders a wave's LDS accesses across its lanes (its half-waves keep their
// rows in LDS regions of their own, so no block barrier is needed).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int SL_B = 9;                 // entries per batch of the sliced-ELL row walks

// The diagonal from A's sliced-ELL copy with one-byte diagonal indices: a
// lane per row walks the row's CSR-length prefix of the index bytes and
// reads the value of the last entry at offset 0 only (the last in CSR order,
// as k_diag; 0 where a row stores none).
__global__ __launch_bounds__(256) void k_diag_sell(int n, const int32_t *__restrict__ rp,
                                                   const int64_t *__restrict__ sp,
                                                   const uint8_t *__restrict__ sd,
                                                   const double *__restrict__ sv,
                                                   const int32_t *__restrict__ sdiag, int ndiag,
                                                   double *__restrict__ diag)
{
    __shared__ int32_t ldg[CBG_SELL_MAX_DIAG];
    for (int t = threadIdx.x; t < ndiag; t += blockDim.x)
        ldg[t] = sdiag[t];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t sl = i / 64, beg = sp[sl];
        const int width = (int)((sp[sl + 1] - beg) / 64);
        const int len = rp[i + 1] - rp[i];
        int64_t hit = -1;
        for (int k0 = 0; k0 < len; k0 += SL_B) {
            uint32_t dx[SL_B];
#pragma unroll
            for (int u = 0; u < SL_B; ++u)
                dx[u] = sd[beg + (int64_t)min(k0 + u, width - 1) * 64 + (i & 63)];
#pragma unroll
            for (int u = 0; u < SL_B; ++u)
                if (k0 + u < len && ldg[dx[u]] == 0)
                    hit = beg + (int64_t)(k0 + u) * 64 + (i & 63);
        }
        diag[i] = hit >= 0 ? sv[hit] : 0.0;
    }
}

// Features of each row: f_p = fl32(a_{i,c(p)} / a_ii) and f_{32+p} =
// fl32(a_{c(p),c(p)} / a_ii) on present slots, f_27 = fl32((a_ii -
// sum_{c != i} |a_ic|) / a_ii) with the sum in CSR order, the rest 0; all
// rounded to bf16.  The entries' terms go through the half-wave's own LDS
// region; one lane adds them in CSR order.  (Columns are unique within a
// row, so each slot is written at most once.)
__global__ __launch_bounds__(256) void k_features(int n, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci,
                                                  const double *__restrict__ val, int nx, int ny,
                                                  const double *__restrict__ diag,
                                                  uint16_t *__restrict__ feat,
                                                  unsigned *__restrict__ bad)
{
    __shared__ double loff[HWR][32];
    __shared__ uint32_t lfw[HWR][NF / 2];
    const int g = threadIdx.x >> 5, lane = threadIdx.x & 31;
    uint16_t *lf = (uint16_t *)lfw[g];
    for (int64_t i = (int64_t)blockIdx.x * HWR + g; i < n; i += (int64_t)gridDim.x * HWR) {
        const int beg = rp[i], end = rp[i + 1];
        const double d = diag[i];
        const RowPos rpos = row_pos(i, nx, ny);
        lfw[g][lane] = 0u;
        wave_sync();
        double off = 0.0;
        for (int p0 = beg; p0 < end; p0 += 32) {
            const int p = p0 + lane;
            const bool in = p < end;
            const int64_t c = in ? ci[p] : -1;
            const double a = in ? val[p] : 0.0;
            loff[g][lane] = (in && c != i) ? fabs(a) : 0.0;
            const int s = in ? slot_at(rpos, i, c, nx, ny) : -1;
            if (s >= 0) {
                lf[s] = bf16_of((float)(a / d));
                lf[NBR + s] = bf16_of((float)(diag[c] / d));
            }
            wave_sync();
            if (lane == 0) {
                const int m = min(32, end - p0);
                for (int k = 0; k < m; ++k)
                    off += loff[g][k];
            }
            wave_sync();
        }
        if (lane == 0) {
            const double margin = (d - off) / d;
            if (!(d != 0.0) || !isfinite(margin))
                *bad = 1u;
            lf[27] = bf16_of((float)margin);
        }
        wave_sync();
        ((uint32_t *)(feat + i * NF))[lane] = lfw[g][lane];
        wave_sync();
    }
}

// The same features from A's sliced-ELL copy with one-byte diagonal indices
// (the same values and bits): one wave per 64-row slice, lane = row.  The
// copy keeps each row's entries in CSR order, so the lane adds the
// off-diagonal sum in that order; entries past the row's CSR length are
// padding and skipped.  A batch's values and indices are loaded together
// (indices clamped into the slice), then the neighbours' diagonals.  Each
// lane assembles its row's 64 features in an LDS row of its own (odd word
// stride: the 64 rows sit in distinct banks); the wave then writes two rows
// per store.
constexpr int FS_LD = NF / 2 + 1;       // LDS row stride in 32-bit words

__global__ __launch_bounds__(256) void k_features_sell(
    int n, int64_t nslice, const int32_t *__restrict__ rp, const int64_t *__restrict__ sp,
    const uint8_t *__restrict__ sd, const double *__restrict__ sv,
    const int32_t *__restrict__ sdiag, int ndiag, int nx, int ny,
    const double *__restrict__ diag, uint16_t *__restrict__ feat, unsigned *__restrict__ bad)
{
    __shared__ int32_t ldg[CBG_SELL_MAX_DIAG];
    __shared__ uint32_t lf[4][64 * FS_LD];
    for (int t = threadIdx.x; t < ndiag; t += blockDim.x)
        ldg[t] = sdiag[t];
    __syncthreads();
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t *my = lf[wv] + lane * FS_LD;
    uint16_t *myh = (uint16_t *)my;
    for (int64_t sl = (int64_t)blockIdx.x * 4 + wv; sl < nslice; sl += (int64_t)gridDim.x * 4) {
        const int64_t i = sl * 64 + lane;
        const bool live = i < n;
        const int64_t ic = live ? i : (int64_t)n - 1;
        for (int q = 0; q < NF / 2; ++q)
            my[q] = 0u;
        const int64_t beg = sp[sl];
        const int width = (int)((sp[sl + 1] - beg) / 64);
        const int len = live ? rp[i + 1] - rp[i] : 0;
        const double d = diag[ic];
        const RowPos rpos = row_pos(ic, nx, ny);
        double off = 0.0;
        for (int k0 = 0; k0 < width; k0 += SL_B) {
            double a[SL_B];
            int64_t c[SL_B];
#pragma unroll
            for (int u = 0; u < SL_B; ++u) {
                const int64_t e = beg + (int64_t)min(k0 + u, width - 1) * 64 + lane;
                a[u] = sv[e];
                c[u] = ic + ldg[sd[e]];
            }
            double dc[SL_B];
#pragma unroll
            for (int u = 0; u < SL_B; ++u)
                dc[u] = diag[min(max(c[u], (int64_t)0), (int64_t)n - 1)];
#pragma unroll
            for (int u = 0; u < SL_B; ++u) {
                if (k0 + u >= len)
                    continue;
                if (c[u] != ic)
                    off += fabs(a[u]);
                const int s = slot_at(rpos, ic, c[u], nx, ny);
                if (s >= 0) {
                    myh[s] = bf16_of((float)(a[u] / d));
                    myh[NBR + s] = bf16_of((float)(dc[u] / d));
                }
            }
        }
        if (live) {
            const double margin = (d - off) / d;
            if (!(d != 0.0) || !isfinite(margin))
                *bad = 1u;
            myh[27] = bf16_of((float)margin);
        }
        wave_sync();
        for (int q = 0; q < 32; ++q) {
            const int r = 2 * q + (lane >> 5);
            const int64_t row = sl * 64 + r;
            if (row < n)
                ((uint32_t *)(feat + row * NF))[lane & 31] = lf[wv][r * FS_LD + (lane & 31)];
        }
        wave_sync();
    }
}

// Weights staged in LDS transposed (out-major) so that an A operand
// (4 consecutive k of one output row) is one 8-byte read.
struct WeightsLds {
    uint16_t w1t[NH * NF];   // [out 64][in 64]
    uint16_t w2t[NH * NH];   // [out 64][in 64]
    uint16_t w3t[NO * NH];   // [out 32][in 64]
    float b1[NH], b2[NH], b3[NO];
};

__device__ void stage_weights(WeightsLds &L, const uint16_t *__restrict__ wq,
                              const float *__restrict__ prm)
{
    for (int e = threadIdx.x; e < NF * NH; e += blockDim.x) {
        const int in = e / NH, out = e % NH;
        L.w1t[out * NF + in] = wq[QW1 + e];
    }
    for (int e = threadIdx.x; e < NH * NH; e += blockDim.x) {
        const int in = e / NH, out = e % NH;
        L.w2t[out * NH + in] = wq[QW2 + e];
    }
    for (int e = threadIdx.x; e < NH * NO; e += blockDim.x) {
        const int in = e / NO, out = e % NO;
        L.w3t[out * NH + in] = wq[QW3 + e];
    }
    for (int e = threadIdx.x; e < NH; e += blockDim.x) {
        L.b1[e] = prm[OB1 + e];
        L.b2[e] = prm[OB2 + e];
    }
    for (int e = threadIdx.x; e < NO; e += blockDim.x)
        L.b3[e] = prm[OB3 + e];
    __syncthreads();
}

__device__ __forceinline__ s16x4 lds4(const uint16_t *p)
{
    const uint2 v = *(const uint2 *)p;
    s16x4 r;
    r[0] = (short)(v.x & 0xFFFF);
    r[1] = (short)(v.x >> 16);
    r[2] = (short)(v.y & 0xFFFF);
    r[3] = (short)(v.y >> 16);
    return r;
}

__device__ __forceinline__ s16x4 relu_bf16(f32x4 c)
{
    s16x4 r;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        r[q] = (short)bf16_of(fmaxf(c[q], 0.0f));
    return r;
}

// Forward pass of 16-row tiles: O (n x 32 fp32); optionally the bf16 hidden
// activations H1, H2 (n x 64) for the backward pass.
__global__ __launch_bounds__(256) void k_forward(int n, const uint16_t *__restrict__ feat,
                                                 const uint16_t *__restrict__ wq,
                                                 const float *__restrict__ prm,
                                                 float *__restrict__ O, uint16_t *__restrict__ H1,
                                                 uint16_t *__restrict__ H2)
{
    __shared__ WeightsLds L;
    stage_weights(L, wq, prm);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int col = lane & 15, kq = (lane >> 4) * 4;      // lane's column; first of its 4 k
    const int64_t ntile = ((int64_t)n + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * nw + wave; tile < ntile;
         tile += (int64_t)gridDim.x * nw) {
        const int64_t row = tile * 16 + col;              // this lane's row in the B layout
        const bool live = row < n;
        // layer 1: H1^T (64 x 16) = W1^T (64 x 64) F^T (64 x 16)
        s16x4 fb[NF / 16];
#pragma unroll
        for (int ks = 0; ks < NF / 16; ++ks) {
            if (live) {
                const uint2 v = *(const uint2 *)(feat + row * NF + ks * 16 + kq);
                fb[ks][0] = (short)(v.x & 0xFFFF);
                fb[ks][1] = (short)(v.x >> 16);
                fb[ks][2] = (short)(v.y & 0xFFFF);
                fb[ks][3] = (short)(v.y >> 16);
            } else {
                fb[ks] = s16x4{0, 0, 0, 0};
            }
        }
        s16x4 h1[4];
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            f32x4 c;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                c[q] = L.b1[ot * 16 + kq + q];
#pragma unroll
            for (int ks = 0; ks < NF / 16; ++ks)
                c = mfma(lds4(&L.w1t[(ot * 16 + col) * NF + ks * 16 + kq]), fb[ks], c);
            h1[ot] = relu_bf16(c);
        }
        // layer 2: H2^T (64 x 16) = W2^T (64 x 64) H1^T
        s16x4 h2[4];
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            f32x4 c;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                c[q] = L.b2[ot * 16 + kq + q];
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
                c = mfma(lds4(&L.w2t[(ot * 16 + col) * NH + ks * 16 + kq]), h1[ks], c);
            h2[ot] = relu_bf16(c);
        }
        // layer 3: O^T (32 x 16) = W3^T (32 x 64) H2^T
#pragma unroll
        for (int ot = 0; ot < 2; ++ot) {
            f32x4 c;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                c[q] = L.b3[ot * 16 + kq + q];
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
                c = mfma(lds4(&L.w3t[(ot * 16 + col) * NH + ks * 16 + kq]), h2[ks], c);
            if (live)
                *(f32x4 *)(O + row * NO + ot * 16 + kq) = c;
        }
        if (live && H1) {
#pragma unroll
            for (int ot = 0; ot < 4; ++ot) {
                uint2 a = {(uint32_t)(uint16_t)h1[ot][0] | ((uint32_t)(uint16_t)h1[ot][1] << 16),
                           (uint32_t)(uint16_t)h1[ot][2] | ((uint32_t)(uint16_t)h1[ot][3] << 16)};
                uint2 b = {(uint32_t)(uint16_t)h2[ot][0] | ((uint32_t)(uint16_t)h2[ot][1] << 16),
                           (uint32_t)(uint16_t)h2[ot][2] | ((uint32_t)(uint16_t)h2[ot][3] << 16)};
                *(uint2 *)(H1 + row * NH + ot * 16 + kq) = a;
                *(uint2 *)(H2 + row * NH + ot * 16 + kq) = b;
            }
        }
    }
}

// P on A's pattern from the network output (a half-wave per row).
__global__ __launch_bounds__(256) void k_assemble(int n, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci,
                                                  const double *__restrict__ val, int nx, int ny,
                                                  const float *__restrict__ O,
                                                  float *__restrict__ pval)
{
    const int g = threadIdx.x >> 5, lane = threadIdx.x & 31;
    for (int64_t base = (int64_t)blockIdx.x * HWR; base < n; base += (int64_t)gridDim.x * HWR) {
        const int64_t i = base + g;
        const bool live = i < n;
        const int beg = live ? rp[i] : 0, end = live ? rp[i + 1] : 0;
        const int ch = (end - beg + 31) / 32;
        const int chunks = max(ch, __shfl_xor(ch, 32));
        const double d = hw_row_diag(i, beg, end, chunks, ci, val);
        const RowPos rpos = row_pos(live ? i : 0, nx, ny);
        for (int q = 0; q < chunks; ++q) {
            const int p = beg + q * 32 + lane;
            if (p < end) {
                const int s = slot_at(rpos, i, ci[p], nx, ny);
                double v = 0.0;
                if (s >= 0)
                    v = ((s == CENTER ? 1.0 : 0.0) + (double)O[i * NO + s]) / d;
                pval[p] = (float)v;
            }
        }
    }
}

// float16 code of an fp32 value: one rounding to nearest even; magnitudes
// from 65520 up become infinity, NaN the quiet NaN.
__device__ __forceinline__ uint16_t f16_code(float f)
{
    const double v = (double)f;
    if (!(fabs(v) < 65520.0))
        return (uint16_t)(v != v ? 0x7E00u : (0x7C00u | (sign_of(v) << 15)));
    return (uint16_t)(rne_code<10, -14, 15>(v) | (sign_of(v) << 15));
}

// The stored form's codes: on the slots present in A's row the float16 code
// of O[i][slot], 0 on the others and on rows in [n, ld); slot-major with row
// stride ld.  A block takes PK_ROWS consecutive rows: each half-wave walks
// PK_ROWS / 8 of them (one entry per lane) and puts the row's codes in LDS,
// slot-major; the block then writes each slot's run of PK_ROWS codes with
// one 4-byte store per two rows.
constexpr int PK_ROWS = 128;
constexpr int PK_LD = PK_ROWS + 2;      // LDS row stride: a half-wave's 27 slots in 27 banks

__global__ __launch_bounds__(256) void k_stencil_pack(int n, int64_t ld,
                                                      const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ ci, int nx,
                                                      int ny, const float *__restrict__ O,
                                                      uint16_t *__restrict__ codes)
{
    __shared__ uint32_t lcw[NSLOT * PK_LD / 2];
    uint16_t *lc = (uint16_t *)lcw;
    const int g = threadIdx.x >> 5, lane = threadIdx.x & 31;
    for (int64_t base = (int64_t)blockIdx.x * PK_ROWS; base < ld;
         base += (int64_t)gridDim.x * PK_ROWS) {
        for (int e = threadIdx.x; e < NSLOT * PK_LD / 2; e += blockDim.x)
            lcw[e] = 0u;
        __syncthreads();
        for (int r = g; r < PK_ROWS && base + r < n; r += HWR) {
            const int64_t i = base + r;
            const int beg = rp[i], end = rp[i + 1];
            const RowPos rpos = row_pos(i, nx, ny);
            for (int p = beg + lane; p < end; p += 32) {
                const int sl = slot_at(rpos, i, ci[p], nx, ny);
                if (sl >= 0)
                    lc[sl * PK_LD + r] = f16_code(O[i * NO + sl]);
            }
        }
        __syncthreads();
        // ld is even and base a multiple of PK_ROWS: every pair starts 4-byte aligned
        for (int e = threadIdx.x; e < NSLOT * (PK_ROWS / 2); e += blockDim.x) {
            const int sl = e / (PK_ROWS / 2), r = 2 * (e - sl * (PK_ROWS / 2));
            const int64_t i = base + r;
            if (i < ld)
                *(uint32_t *)(codes + (int64_t)sl * ld + i) = lcw[(sl * PK_LD + r) / 2];
        }
        __syncthreads();
    }
}

// The stored form's codes from the sliced-ELL copy with diagonal indices
// (the same codes): one wave per 64-row slice, lane = row, the row's slots
// marked in an LDS block of the wave's own (slot-major, 64 rows), then each
// slot's 64 codes written as one run.  Slices past the copy's (rows up to
// ld) are written as 0.
__global__ __launch_bounds__(256) void k_stencil_pack_sell(
    int n, int64_t ld, int64_t nslice, const int32_t *__restrict__ rp,
    const int64_t *__restrict__ sp, const uint8_t *__restrict__ sd,
    const int32_t *__restrict__ sdiag, int ndiag, int nx, int ny, const float *__restrict__ O,
    uint16_t *__restrict__ codes)
{
    __shared__ int32_t ldg[CBG_SELL_MAX_DIAG];
    __shared__ uint16_t lc[4][NSLOT * 64];
    for (int t = threadIdx.x; t < ndiag; t += blockDim.x)
        ldg[t] = sdiag[t];
    __syncthreads();
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint16_t *mine = lc[wv];
    const int64_t nsl_ld = ld / 64;                      // ld is a multiple of 256
    for (int64_t sl = (int64_t)blockIdx.x * 4 + wv; sl < nsl_ld; sl += (int64_t)gridDim.x * 4) {
        for (int s = 0; s < NSLOT; ++s)
            mine[s * 64 + lane] = 0;
        wave_sync();
        if (sl < nslice) {
            const int64_t i = sl * 64 + lane;
            const bool live = i < n;
            const int64_t ic = live ? i : (int64_t)n - 1;
            const int64_t beg = sp[sl];
            const int width = (int)((sp[sl + 1] - beg) / 64);
            const int len = live ? rp[i + 1] - rp[i] : 0;
            const RowPos rpos = row_pos(ic, nx, ny);
            for (int k0 = 0; k0 < width; k0 += SL_B) {
                int sl_of[SL_B];
                float o[SL_B];
#pragma unroll
                for (int u = 0; u < SL_B; ++u) {
                    const int64_t e = beg + (int64_t)min(k0 + u, width - 1) * 64 + lane;
                    sl_of[u] = slot_at(rpos, ic, ic + ldg[sd[e]], nx, ny);
                }
#pragma unroll
                for (int u = 0; u < SL_B; ++u)
                    o[u] = O[ic * NO + max(sl_of[u], 0)];
#pragma unroll
                for (int u = 0; u < SL_B; ++u)
                    if (k0 + u < len && sl_of[u] >= 0)
                        mine[sl_of[u] * 64 + lane] = f16_code(o[u]);
            }
        }
        wave_sync();
        for (int s = 0; s < NSLOT; ++s)
            codes[(int64_t)s * ld + sl * 64 + lane] = mine[s * 64 + lane];
        wave_sync();
    }
}

// dL/dO (bf16, n x 32) from dL/dP: dO_{i,p} = dP_{i,c(p)} / a_ii (a
// half-wave per row; the row's 32 slots assembled in LDS).
__global__ __launch_bounds__(256) void k_grad_o(int n, const int32_t *__restrict__ rp,
                                                const int32_t *__restrict__ ci,
                                                const double *__restrict__ val, int nx, int ny,
                                                const double *__restrict__ dP,
                                                uint16_t *__restrict__ dO)
{
    __shared__ uint16_t lg[HWR][NO];
    const int g = threadIdx.x >> 5, lane = threadIdx.x & 31;
    for (int64_t base = (int64_t)blockIdx.x * HWR; base < n; base += (int64_t)gridDim.x * HWR) {
        const int64_t i = base + g;
        const bool live = i < n;
        const int beg = live ? rp[i] : 0, end = live ? rp[i + 1] : 0;
        const int chunks = block_chunks((end - beg + 31) / 32);
        const double d = hw_row_diag(i, beg, end, chunks, ci, val);
        const RowPos rpos = row_pos(live ? i : 0, nx, ny);
        lg[g][lane] = 0;
        __syncthreads();
        for (int q = 0; q < chunks; ++q) {
            const int p = beg + q * 32 + lane;
            if (p < end) {
                const int s = slot_at(rpos, i, ci[p], nx, ny);
                if (s >= 0)
                    lg[g][s] = bf16_of_d(dP[p] / d);
            }
        }
        __syncthreads();
        if (live)
            dO[i * NO + lane] = lg[g][lane];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Batched sparse products over K <= 32 vectors stored row-major (n x K):
// a 32-lane group per row, lane k for vector k.
// ---------------------------------------------------------------------------
enum { MM_PV = 0, MM_AY_MINUS_V = 1, MM_ATR = 2 };

template <int MODE>
__global__ __launch_bounds__(256) void k_spmm(int n, int K, const int32_t *__restrict__ rp,
                                              const int32_t *__restrict__ ci,
                                              const double *__restrict__ val,
                                              const float *__restrict__ fval,
                                              const double *__restrict__ X,
                                              const uint16_t *__restrict__ Vh,
                                              double *__restrict__ Y, double scale,
                                              double *__restrict__ part)
{
    const int k = threadIdx.x & 31, grp = threadIdx.x >> 5, ngrp = blockDim.x >> 5;
    double ssq = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * ngrp + grp; i < n; i += (int64_t)gridDim.x * ngrp) {
        if (k >= K)
            continue;
        double s = 0.0;
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            const int64_t c = ci[p];
            if constexpr (MODE == MM_PV) {
                const _Float16 h = __builtin_bit_cast(_Float16, Vh[c * K + k]);
                s = fma((double)fval[p], (double)(float)h, s);
            } else {
                s = fma(val[p], X[c * K + k], s);
            }
        }
        if constexpr (MODE == MM_AY_MINUS_V) {
            const _Float16 h = __builtin_bit_cast(_Float16, Vh[i * K + k]);
            s = s - (double)(float)h;
            ssq += s * s;
        }
        if constexpr (MODE == MM_ATR)
            s *= scale;
        Y[i * K + k] = s;
    }
    if constexpr (MODE == MM_AY_MINUS_V) {
        double m = 0.0;
        block_sum_max(ssq, m);
        if (threadIdx.x == 0)
            part[blockIdx.x] = ssq;
    }
}

// dP_e = sum_k G[row(e)][k] * v_k[col(e)] on A's pattern.
__global__ __launch_bounds__(256) void k_sddmm(int n, int K, const int32_t *__restrict__ rp,
                                               const int32_t *__restrict__ ci,
                                               const double *__restrict__ G,
                                               const uint16_t *__restrict__ Vh,
                                               double *__restrict__ dP)
{
    const int k = threadIdx.x & 31, grp = threadIdx.x >> 5, ngrp = blockDim.x >> 5;
    for (int64_t i = (int64_t)blockIdx.x * ngrp + grp; i < n; i += (int64_t)gridDim.x * ngrp) {
        const double g = k < K ? G[i * K + k] : 0.0;
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            const int64_t c = ci[p];
            double t = 0.0;
            if (k < K) {
                const _Float16 h = __builtin_bit_cast(_Float16, Vh[c * K + k]);
                t = g * (double)(float)h;
            }
#pragma unroll
            for (int d = 16; d >= 1; d >>= 1)
                t += __shfl_xor(t, d, 32);
            if (k == 0)
                dP[p] = t;
        }
    }
}

// *loss (+)= scale * sum of the block partials, folded in block order.
__global__ void k_loss_fold(const double *__restrict__ part, int nb, double scale, int accumulate,
                            double *__restrict__ loss)
{
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x)
        s += part[b];
    double m = 0.0;
    block_sum_max(s, m);
    if (threadIdx.x == 0)
        *loss = (accumulate ? *loss : 0.0) + s * scale;
}

// ---------------------------------------------------------------------------
// Backward pass.  Per 16-row tile: dH2^T = W3 dO^T and dH1^T = W2 dH2^T on
// the MFMA units (masked by the ReLU, rounded to bf16), then the weight
// gradients dW3 = H2^T dO, dW2 = H1^T dH2, dW1 = F^T dH1 as MFMA products
// over the tile's rows (operands transposed through LDS), accumulated per
// wave across tiles; bias gradients are column sums.  Each block writes its
// NPARAM partial gradients; k_grad_fold sums blocks in order.
// ---------------------------------------------------------------------------

struct BackLds {
    uint16_t w3[NH * NO];    // W3 as stored: [hidden 64][out 32]
    uint16_t w2[NH * NH];    // W2 as stored: [in 64][out 64]
};

struct TileLds {             // one wave's 16-row tile, row-major
    uint16_t f[16 * NF], h1[16 * NH], h2[16 * NH], dO[16 * NO], dh2[16 * NH], dh1[16 * NH];
};

__device__ __forceinline__ s16x4 col4(const uint16_t *t, int ld, int r0, int c)
{
    s16x4 r;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        r[q] = (short)t[(r0 + q) * ld + c];
    return r;
}

__global__ __launch_bounds__(256) void k_backward(int n, const uint16_t *__restrict__ feat,
                                                  const uint16_t *__restrict__ H1,
                                                  const uint16_t *__restrict__ H2,
                                                  const uint16_t *__restrict__ dO,
                                                  const uint16_t *__restrict__ wq,
                                                  float *__restrict__ part)
{
    __shared__ BackLds W;
    __shared__ TileLds T[4];
    __shared__ float red[4][NPARAM / 4 + 1];   // wave-level staging of one quarter
    for (int e = threadIdx.x; e < NH * NO; e += blockDim.x)
        W.w3[e] = wq[QW3 + e];
    for (int e = threadIdx.x; e < NH * NH; e += blockDim.x)
        W.w2[e] = wq[QW2 + e];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int col = lane & 15, kq = (lane >> 4) * 4;
    TileLds &t = T[wave];
    f32x4 gw3[4][2], gw2[4][4], gw1[NF / 16][4];   // [row tile of W][col tile of W]
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
            gw3[a][b] = f32x4{0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
            gw2[a][b] = f32x4{0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < NF / 16; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
            gw1[a][b] = f32x4{0, 0, 0, 0};
    float gb1 = 0.0f, gb2 = 0.0f, gb3 = 0.0f;   // lane c: column c
    const int64_t ntile = ((int64_t)n + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * nw + wave; tile < ntile;
         tile += (int64_t)gridDim.x * nw) {
        const int64_t r0 = tile * 16;
        // stage the tile's inputs (rows beyond n read as 0)
        for (int e = lane; e < 16 * NF; e += 64) {
            const int64_t r = r0 + e / NF;
            t.f[e] = r < n ? feat[r * NF + e % NF] : 0;
        }
        for (int e = lane; e < 16 * NO; e += 64) {
            const int64_t r = r0 + e / NO;
            t.dO[e] = r < n ? dO[r * NO + e % NO] : 0;
        }
        for (int e = lane; e < 16 * NH; e += 64) {
            const int64_t r = r0 + e / NH;
            t.h1[e] = r < n ? H1[r * NH + e % NH] : 0;
            t.h2[e] = r < n ? H2[r * NH + e % NH] : 0;
        }
        __builtin_amdgcn_wave_barrier();
        // B operand dO^T: lane holds dO[row col][o = ks*16 + kq .. +3]
        s16x4 ob[2];
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
            ob[ks] = lds4(&t.dO[col * NO + ks * 16 + kq]);
        // dH2^T (64 x 16) = W3 (64 x 32) dO^T; mask, bf16, keep and stage
        s16x4 dh2[4];
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            f32x4 c = {0, 0, 0, 0};
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
                c = mfma(lds4(&W.w3[(ot * 16 + col) * NO + ks * 16 + kq]), ob[ks], c);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int h = ot * 16 + kq + q;
                const float m = f_of(t.h2[col * NH + h]) > 0.0f ? c[q] : 0.0f;
                dh2[ot][q] = (short)bf16_of(m);
                t.dh2[col * NH + h] = (uint16_t)dh2[ot][q];
            }
        }
        // dH1^T (64 x 16) = W2 (64 x 64) dH2^T; mask, bf16, stage
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            f32x4 c = {0, 0, 0, 0};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
                c = mfma(lds4(&W.w2[(ot * 16 + col) * NH + ks * 16 + kq]), dh2[ks], c);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int h = ot * 16 + kq + q;
                const float m = f_of(t.h1[col * NH + h]) > 0.0f ? c[q] : 0.0f;
                t.dh1[col * NH + h] = bf16_of(m);
            }
        }
        __builtin_amdgcn_wave_barrier();
        // weight gradients over the tile's 16 rows: D (M x N) += A (M x 16 rows)
        // B (16 rows x N), A[i][k] = X[row k][i], B[k][j] = Y[row k][j]
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                gw3[a][b] = mfma(col4(t.h2, NH, kq, a * 16 + col), col4(t.dO, NO, kq, b * 16 + col),
                                 gw3[a][b]);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                gw2[a][b] = mfma(col4(t.h1, NH, kq, a * 16 + col),
                                 col4(t.dh2, NH, kq, b * 16 + col), gw2[a][b]);
#pragma unroll
        for (int a = 0; a < NF / 16; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                gw1[a][b] = mfma(col4(t.f, NF, kq, a * 16 + col),
                                 col4(t.dh1, NH, kq, b * 16 + col), gw1[a][b]);
        // bias gradients: column sums of dO, dH2, dH1 over the tile (lane c
        // owns columns c, c+64 of each)
        for (int q = 0; q < 16; ++q) {
            if (lane < NO)
                gb3 += f_of(t.dO[q * NO + lane]);
            gb2 += f_of(t.dh2[q * NH + lane]);
            gb1 += f_of(t.dh1[q * NH + lane]);
        }
        __builtin_amdgcn_wave_barrier();
    }
    // per-block partials in parameter order, folded over the 4 waves in LDS
    // (fixed wave order) one quarter of the parameters at a time
    auto emit = [&](int q0, int q1) {
        // each wave writes its sums for the parameters in [q0, q1): every
        // parameter is held by exactly one lane of every wave
        float *mine = red[wave];
        // gw3: D[i][j] with i = hidden (a*16 + 4(l/16)+r), j = out (b*16 + col)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int e = OW3 + (a * 16 + kq + r) * NO + b * 16 + col;
                    if (e >= q0 && e < q1)
                        mine[e - q0] = gw3[a][b][r];
                }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int e = OW2 + (a * 16 + kq + r) * NH + b * 16 + col;
                    if (e >= q0 && e < q1)
                        mine[e - q0] = gw2[a][b][r];
                }
#pragma unroll
        for (int a = 0; a < NF / 16; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int e = OW1 + (a * 16 + kq + r) * NH + b * 16 + col;
                    if (e >= q0 && e < q1)
                        mine[e - q0] = gw1[a][b][r];
                }
        {
            int e = OB3 + lane;
            if (lane < NO && e >= q0 && e < q1)
                mine[e - q0] = gb3;
            e = OB2 + lane;
            if (e >= q0 && e < q1)
                mine[e - q0] = gb2;
            e = OB1 + lane;
            if (e >= q0 && e < q1)
                mine[e - q0] = gb1;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < q1 - q0; e += blockDim.x) {
            float s = red[0][e];
            for (int w = 1; w < nw; ++w)
                s += red[w][e];
            part[(size_t)blockIdx.x * NPARAM + q0 + e] = s;
        }
        __syncthreads();
    };
    constexpr int QS = NPARAM / 4;
    emit(0, QS);
    emit(QS, 2 * QS);
    emit(2 * QS, 3 * QS);
    emit(3 * QS, NPARAM);
}

// grad[e] (+)= sum over blocks of part[b][e] (fixed block order, fp64).
__global__ void k_grad_fold(const float *__restrict__ part, int nb, int accumulate,
                            double *__restrict__ grad)
{
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < NPARAM; e += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b)
            s += (double)part[(size_t)b * NPARAM + e];
        grad[e] = (accumulate ? grad[e] : 0.0) + s;
    }
}

// Adam (Kingma and Ba, 2015) on the fp32 master parameters: moments and
// parameters are formed in FP64 (no contraction) and stored rounded to fp32;
// c1 = 1 - beta1^t and c2 = 1 - beta2^t come from the host.  The bf16
// weights are refreshed as the round-to-nearest-even of the new masters.
__global__ void k_adam(float *__restrict__ prm, float *__restrict__ m1, float *__restrict__ m2,
                       uint16_t *__restrict__ wq, const double *__restrict__ grad, double lr,
                       double b1, double b2, double eps, double c1, double c2)
{
#pragma clang fp contract(off)
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < NPARAM; e += gridDim.x * blockDim.x) {
        const double g = grad[e];
        const float m = (float)(b1 * (double)m1[e] + (1.0 - b1) * g);
        const float v = (float)(b2 * (double)m2[e] + (1.0 - b2) * g * g);
        m1[e] = m;
        m2[e] = v;
        const double mh = (double)m / c1;
        const double vh = (double)v / c2;
        const float p = (float)((double)prm[e] - lr * mh / (sqrt(vh) + eps));
        prm[e] = p;
        int q = -1;
        if (e >= OW1 && e < OB1)
            q = QW1 + (e - OW1);
        else if (e >= OW2 && e < OB2)
            q = QW2 + (e - OW2);
        else if (e >= OW3 && e < OB3)
            q = QW3 + (e - OW3);
        if (q >= 0)
            wq[q] = bf16_of(p);
    }
}

// bf16 weights from the fp32 masters (round to nearest even).
__global__ void k_round_weights(const float *__restrict__ prm, uint16_t *__restrict__ wq)
{
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < NWBF; e += gridDim.x * blockDim.x) {
        const int p = e < QW2 ? OW1 + e : e < QW3 ? OW2 + (e - QW2) : OW3 + (e - QW3);
        wq[e] = bf16_of(prm[p]);
    }
}

// Values of A^T on A's pattern (structurally symmetric A): t_val[p] of
// entry (i, c) is a_ci, found by binary search in row c; a missing mirror
// entry sets *bad.
__global__ __launch_bounds__(256) void k_transpose_values(int n, const int32_t *__restrict__ rp,
                                                          const int32_t *__restrict__ ci,
                                                          const double *__restrict__ val,
                                                          double *__restrict__ tval,
                                                          unsigned *__restrict__ bad)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            const int c = ci[p];
            int lo = rp[c], hi = rp[c + 1] - 1;
            double v = 0.0;
            bool found = false;
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                const int cm = ci[mid];
                if (cm == i) {
                    v = val[mid];
                    found = true;
                    break;
                }
                if (cm < i)
                    lo = mid + 1;
                else
                    hi = mid - 1;
            }
            if (!found)
                *bad = 1u;
            tval[p] = v;
        }
    }
}

// out (n x K, row-major fp16) from K FP64 vectors V[(first + k*stride)*ld ..];
// one rounding to nearest even; magnitudes from 65520 up become infinity.
__global__ __launch_bounds__(256) void k_pack(const double *__restrict__ V, int64_t ld, int n,
                                              int K, int first, int stride,
                                              uint16_t *__restrict__ out)
{
    const int64_t total = (int64_t)n * K;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / K;
        const int k = (int)(e % K);
        const double v = V[(int64_t)(first + (int64_t)k * stride) * ld + i];
        uint32_t c = fabs(v) >= 65520.0 ? 0x7C00u : rne_code<10, -14, 15>(v);
        out[e] = (uint16_t)(c | (sign_of(v) << 15));
    }
}

}  // namespace spai
}  // namespace cbg

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
using namespace cbg;
using namespace cbg::spai;

namespace {

constexpr size_t SALIGN = 256;
constexpr int MAXB_ROW = 4096;     // grid cap of the row-parallel kernels
constexpr int MAXB_BACK = 512;     // grid cap of the backward pass (partials)

size_t salign(size_t x) { return (x + SALIGN - 1) / SALIGN * SALIGN; }

struct SpaiWs {
    unsigned *bad;
    double *diag;
    double *dinv;          // 1 / a_ii on cbg_basis_ld(n) rows (stencil apply)
    double *lpart;
    float *gpart;
    uint16_t *feat, *h1, *h2, *dO;
    float *O, *pval;
    double *X0, *X1, *dP;
};

SpaiWs carve_spai(void *ws, int64_t n, int64_t nnz, int64_t K, size_t *total)
{
    uint8_t *base = (uint8_t *)ws;
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        void *p = base ? base + off : nullptr;
        off = salign(off + bytes);
        return p;
    };
    SpaiWs s;
    s.bad = (unsigned *)take(sizeof(unsigned));
    s.diag = (double *)take(8 * (size_t)n);
    s.dinv = (double *)take(8 * (size_t)((n + 255) / 256 * 256));
    s.lpart = (double *)take(sizeof(double) * MAXB_ROW);
    s.gpart = (float *)take(sizeof(float) * (size_t)MAXB_BACK * NPARAM);
    s.feat = (uint16_t *)take(2 * (size_t)n * NF);
    s.h1 = (uint16_t *)take(2 * (size_t)n * NH);
    s.h2 = (uint16_t *)take(2 * (size_t)n * NH);
    s.dO = (uint16_t *)take(2 * (size_t)n * NO);
    s.O = (float *)take(4 * (size_t)n * NO);
    s.pval = (float *)take(4 * (size_t)nnz);
    s.X0 = (double *)take(8 * (size_t)n * K);
    s.X1 = (double *)take(8 * (size_t)n * K);
    s.dP = (double *)take(8 * (size_t)nnz);
    if (total)
        *total = off;
    return s;
}

bool a16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

bool csr_ok(const cbg_csr *A)
{
    return A && A->n >= 0 && A->nnz >= 0 && A->nnz <= INT32_MAX &&
           (A->n == 0 || (A->row_ptr && (A->nnz == 0 || (A->col_idx && A->val))));
}

// A carries a whole sliced-ELL copy with one-byte diagonal indices
bool sell_dix_of(const cbg_csr *A)
{
    return A->sell_ptr && A->sell_val && A->sell_dix && A->sell_diag && A->sell_ndiag >= 1 &&
           A->sell_ndiag <= CBG_SELL_MAX_DIAG && A->sell_entries >= A->nnz &&
           A->sell_entries % 64 == 0;
}

bool grid_ok(const cbg_csr *A, const int32_t *grid)
{
    return grid && grid[0] > 0 && grid[1] > 0 && grid[2] > 0 &&
           (int64_t)grid[0] * grid[1] * grid[2] == A->n;
}

int row_grid(int64_t rows) { return (int)std::min<int64_t>(std::max<int64_t>((rows + 255) / 256, 1), MAXB_ROW); }
int group_grid(int64_t rows) { return (int)std::min<int64_t>(std::max<int64_t>((rows + 7) / 8, 1), MAXB_ROW); }
int tile_grid(int64_t n, int cap) { return (int)std::min<int64_t>(std::max<int64_t>((n + 63) / 64, 1), cap); }

int slice_grid(int64_t n)
{
    return (int)std::min<int64_t>(std::max<int64_t>(((n + 63) / 64 + 3) / 4, 1), 65536);
}

// The diagonal, from the sliced-ELL copy when A carries one
void enqueue_diag(const cbg_csr *A, double *diag, hipStream_t s)
{
    if (sell_dix_of(A)) {
        const int g = (int)std::min<int64_t>(std::max<int64_t>(((int64_t)A->n + 255) / 256, 1),
                                             65536);
        hipLaunchKernelGGL(k_diag_sell, dim3(g), dim3(256), 0, s, A->n, A->row_ptr,
                           A->sell_ptr, A->sell_dix, A->sell_val, A->sell_diag, A->sell_ndiag,
                           diag);
    } else {
        hipLaunchKernelGGL(k_diag, dim3(group_grid(A->n)), dim3(256), 0, s, A->n, A->row_ptr,
                           A->col_idx, A->val, diag);
    }
}

// The features, from the sliced-ELL copy when A carries one
void enqueue_features(const cbg_csr *A, const int32_t grid[3], const double *diag, uint16_t *feat,
                      unsigned *bad, hipStream_t s)
{
    if (sell_dix_of(A)) {
        hipLaunchKernelGGL(k_features_sell, dim3(slice_grid(A->n)), dim3(256), 0, s, A->n,
                           (int64_t)(A->n + 63) / 64, A->row_ptr, A->sell_ptr, A->sell_dix,
                           A->sell_val, A->sell_diag, A->sell_ndiag, grid[0], grid[1], diag,
                           feat, bad);
    } else {
        hipLaunchKernelGGL(k_features, dim3(group_grid(A->n)), dim3(256), 0, s, A->n,
                           A->row_ptr, A->col_idx, A->val, grid[0], grid[1], diag, feat, bad);
    }
}

size_t ws_need(int64_t n, int64_t nnz, int64_t K)
{
    size_t t = 0;
    carve_spai(nullptr, n, nnz, K, &t);
    return t;
}

#define SP_TRY(x)                           \
    do {                                    \
        const hipError_t e_ = (x);          \
        if (e_ != hipSuccess) {             \
            cbg::note_hip_error(e_, __LINE__); \
            (void)hipGetLastError();        \
            return CBG_E_HIP;               \
        }                                   \
    } while (0)

int ws_check(void *ws, size_t ws_bytes, int64_t n, int64_t nnz, int64_t K)
{
    if (!ws || ((uintptr_t)ws & (SALIGN - 1)) || ws_bytes < ws_need(n, nnz, K))
        return CBG_E_WORKSPACE;
    return CBG_OK;
}

// Reads and clears the device flag (synchronous).
int read_flag(unsigned *bad, hipStream_t s, unsigned *out)
{
    SP_TRY(hipMemcpyAsync(out, bad, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    SP_TRY(hipStreamSynchronize(s));
    return CBG_OK;
}

void enqueue_forward(int64_t n, const uint16_t *feat, const uint16_t *w, const float *prm, float *O,
                     uint16_t *h1, uint16_t *h2, hipStream_t s)
{
    hipLaunchKernelGGL(k_forward, dim3(tile_grid(n, 2048)), dim3(256), 0, s, (int)n, feat, w, prm,
                       O, h1, h2);
}

int enqueue_grad_p(const cbg_csr *A, const double *tval, const float *pval, int K,
                   const uint16_t *V, double scale, double *loss, int accumulate, double *dP,
                   const SpaiWs &W, hipStream_t s)
{
    const int gb = group_grid(A->n);
    hipLaunchKernelGGL(k_spmm<MM_PV>, dim3(gb), dim3(256), 0, s, A->n, K, A->row_ptr, A->col_idx,
                       A->val, pval, (const double *)nullptr, V, W.X0, 1.0, (double *)nullptr);
    hipLaunchKernelGGL(k_spmm<MM_AY_MINUS_V>, dim3(gb), dim3(256), 0, s, A->n, K, A->row_ptr,
                       A->col_idx, A->val, (const float *)nullptr, (const double *)W.X0, V, W.X1,
                       1.0, W.lpart);
    hipLaunchKernelGGL(k_loss_fold, dim3(1), dim3(256), 0, s, (const double *)W.lpart, gb, scale,
                       accumulate, loss);
    hipLaunchKernelGGL(k_spmm<MM_ATR>, dim3(gb), dim3(256), 0, s, A->n, K, A->row_ptr, A->col_idx,
                       tval, (const float *)nullptr, (const double *)W.X1, V, W.X0, 2.0 * scale,
                       (double *)nullptr);
    hipLaunchKernelGGL(k_sddmm, dim3(gb), dim3(256), 0, s, A->n, K, A->row_ptr, A->col_idx,
                       (const double *)W.X0, V, dP);
    SP_TRY(hipGetLastError());
    return CBG_OK;
}

int enqueue_backward(int64_t n, const uint16_t *feat, const uint16_t *h1, const uint16_t *h2,
                     const uint16_t *dO, const uint16_t *w, double *grad, int accumulate,
                     const SpaiWs &W, hipStream_t s)
{
    const int nb = tile_grid(n, MAXB_BACK);
    hipLaunchKernelGGL(k_backward, dim3(nb), dim3(256), 0, s, (int)n, feat, h1, h2, dO, w,
                       W.gpart);
    hipLaunchKernelGGL(k_grad_fold, dim3((NPARAM + 255) / 256), dim3(256), 0, s,
                       (const float *)W.gpart, nb, accumulate, grad);
    SP_TRY(hipGetLastError());
    return CBG_OK;
}

}  // namespace

extern "C" {

size_t cbg_spai_workspace_bytes(int32_t n, int64_t nnz, int32_t K)
{
    if (n < 0 || nnz < 0 || K < 0 || K > CBG_SPAI_MAX_K)
        return 0;
    return ws_need(n, nnz, K);
}

int cbg_spai_features(const cbg_csr *A, const int32_t grid[3], uint16_t *feat, void *ws,
                      size_t ws_bytes, void *stream)
{
    if (!csr_ok(A) || !grid_ok(A, grid) || (A->n > 0 && !a16(feat)) || !feat)
        return CBG_E_ARG;
    int e = ws_check(ws, ws_bytes, A->n, A->nnz, 0);
    if (e)
        return e;
    if (A->n == 0)
        return CBG_OK;
    hipStream_t s = (hipStream_t)stream;
    SpaiWs W = carve_spai(ws, A->n, A->nnz, 0, nullptr);
    SP_TRY(hipMemsetAsync(W.bad, 0, sizeof(unsigned), s));
    enqueue_diag(A, W.diag, s);
    enqueue_features(A, grid, (const double *)W.diag, feat, W.bad, s);
    SP_TRY(hipGetLastError());
    unsigned bad = 0;
    if ((e = read_flag(W.bad, s, &bad)))
        return e;
    return bad ? CBG_E_NONFINITE : CBG_OK;
}

int cbg_mlp_forward(int32_t n, const uint16_t *feat, const uint16_t *weights, const float *params,
                    float *out, uint16_t *h1, uint16_t *h2, void *stream)
{
    if (n < 0 || (n > 0 && (!feat || !weights || !params || !out)) || !a16(feat) || !a16(out) ||
        !a16(h1) || !a16(h2) || ((h1 == nullptr) != (h2 == nullptr)) || !a16(weights) ||
        !a16(params))
        return CBG_E_ARG;
    if (n == 0)
        return CBG_OK;
    enqueue_forward(n, feat, weights, params, out, h1, h2, (hipStream_t)stream);
    SP_TRY(hipGetLastError());
    return CBG_OK;
}

int cbg_spai_assemble(const cbg_csr *A, const int32_t grid[3], const float *out, float *p_val,
                      void *stream)
{
    if (!csr_ok(A) || !grid_ok(A, grid) || (A->n > 0 && (!out || !p_val)))
        return CBG_E_ARG;
    if (A->n == 0)
        return CBG_OK;
    hipLaunchKernelGGL(k_assemble, dim3(group_grid(A->n)), dim3(256), 0, (hipStream_t)stream, A->n,
                       A->row_ptr, A->col_idx, A->val, grid[0], grid[1], out, p_val);
    SP_TRY(hipGetLastError());
    return CBG_OK;
}

int cbg_learned_build(const cbg_csr *A, const int32_t grid[3], const uint16_t *weights,
                      const float *params, float *p_val, void *ws, size_t ws_bytes, void *stream)
{
    if (!csr_ok(A) || !grid_ok(A, grid) || (A->n > 0 && (!weights || !params || !p_val)) ||
        !a16(weights) || !a16(params))
        return CBG_E_ARG;
    int e = ws_check(ws, ws_bytes, A->n, A->nnz, 0);
    if (e)
        return e;
    if (A->n == 0)
        return CBG_OK;
    hipStream_t s = (hipStream_t)stream;
    SpaiWs W = carve_spai(ws, A->n, A->nnz, 0, nullptr);
    SP_TRY(hipMemsetAsync(W.bad, 0, sizeof(unsigned), s));
    enqueue_diag(A, W.diag, s);
    enqueue_features(A, grid, (const double *)W.diag, W.feat, W.bad, s);
    enqueue_forward(A->n, W.feat, weights, params, W.O, nullptr, nullptr, s);
    hipLaunchKernelGGL(k_assemble, dim3(group_grid(A->n)), dim3(256), 0, s, A->n, A->row_ptr,
                       A->col_idx, A->val, grid[0], grid[1], (const float *)W.O, p_val);
    SP_TRY(hipGetLastError());
    unsigned bad = 0;
    if ((e = read_flag(W.bad, s, &bad)))
        return e;
    return bad ? CBG_E_NONFINITE : CBG_OK;
}

int cbg_learned_build_stencil(const cbg_csr *A, const int32_t grid[3], const uint16_t *weights,
                              const float *params, uint16_t *p_stencil, void *ws,
                              size_t ws_bytes, void *stream)
{
    if (!csr_ok(A) || !grid_ok(A, grid) || (A->n > 0 && (!weights || !params || !p_stencil)) ||
        !a16(weights) || !a16(params) || !a16(p_stencil))
        return CBG_E_ARG;
    int e = ws_check(ws, ws_bytes, A->n, A->nnz, 0);
    if (e)
        return e;
    if (A->n == 0)
        return CBG_OK;
    hipStream_t s = (hipStream_t)stream;
    SpaiWs W = carve_spai(ws, A->n, A->nnz, 0, nullptr);
    const int64_t ld = cbg_basis_ld(A->n);
    SP_TRY(hipMemsetAsync(W.bad, 0, sizeof(unsigned), s));
    enqueue_diag(A, W.diag, s);
    enqueue_features(A, grid, (const double *)W.diag, W.feat, W.bad, s);
    enqueue_forward(A->n, W.feat, weights, params, W.O, nullptr, nullptr, s);
    if (sell_dix_of(A)) {
        hipLaunchKernelGGL(k_stencil_pack_sell, dim3(slice_grid(ld)), dim3(256), 0, s, A->n, ld,
                           (int64_t)(A->n + 63) / 64, A->row_ptr, A->sell_ptr, A->sell_dix,
                           A->sell_diag, A->sell_ndiag, grid[0], grid[1], (const float *)W.O,
                           p_stencil);
    } else {
        const int gp = (int)std::min<int64_t>((ld + PK_ROWS - 1) / PK_ROWS, MAXB_ROW);
        hipLaunchKernelGGL(k_stencil_pack, dim3(std::max(gp, 1)), dim3(256), 0, s, A->n, ld,
                           A->row_ptr, A->col_idx, grid[0], grid[1], (const float *)W.O,
                           p_stencil);
    }
    SP_TRY(hipGetLastError());
    unsigned bad = 0;
    if ((e = read_flag(W.bad, s, &bad)))
        return e;
    return bad ? CBG_E_NONFINITE : CBG_OK;
}

int cbg_stencil_apply(const cbg_csr *A, const int32_t grid[3], const uint16_t *p_stencil,
                      const double *v, double *z, void *ws, size_t ws_bytes, void *stream)
{
    if (!csr_ok(A) || !grid_ok(A, grid) || (A->n > 0 && (!p_stencil || !v || !z)) ||
        !a16(p_stencil))
        return CBG_E_ARG;
    int e = ws_check(ws, ws_bytes, A->n, A->nnz, 0);
    if (e)
        return e;
    if (A->n == 0)
        return CBG_OK;
    hipStream_t s = (hipStream_t)stream;
    SpaiWs W = carve_spai(ws, A->n, A->nnz, 0, nullptr);
    const int64_t ld = cbg_basis_ld(A->n);
    SP_TRY(hipMemsetAsync(W.bad, 0, sizeof(unsigned), s));
    SpmvArgs am{};
    am.n = A->n;
    am.rp = A->row_ptr;
    am.ci = A->col_idx;
    am.val = A->val;
    if (sell_dix_of(A)) {
        am.sp = A->sell_ptr;
        am.sv = A->sell_val;
        am.sd = A->sell_dix;
        am.sdiag = A->sell_diag;
        am.ndiag = A->sell_ndiag;
    }
    launch_jacobi_setup(am, ld, W.dinv, W.bad, s);
    launch_stencil(F_FP64, 1, v, A->n, ld, grid, p_stencil, W.dinv, z, nullptr, nullptr, nullptr,
                   s);
    SP_TRY(hipGetLastError());
    unsigned bad = 0;
    if ((e = read_flag(W.bad, s, &bad)))
        return e;
    return bad ? CBG_E_ARG : CBG_OK;
}

int cbg_csr_transpose_values(const cbg_csr *A, double *t_val, void *ws, size_t ws_bytes,
                             void *stream)
{
    if (!csr_ok(A) || (A->nnz > 0 && !t_val))
        return CBG_E_ARG;
    int e = ws_check(ws, ws_bytes, A->n, A->nnz, 0);
    if (e)
        return e;
    if (A->n == 0)
        return CBG_OK;
    hipStream_t s = (hipStream_t)stream;
    SpaiWs W = carve_spai(ws, A->n, A->nnz, 0, nullptr);
    SP_TRY(hipMemsetAsync(W.bad, 0, sizeof(unsigned), s));
    hipLaunchKernelGGL(k_transpose_values, dim3(row_grid(A->n)), dim3(256), 0, s, A->n,
                       A->row_ptr, A->col_idx, A->val, t_val, W.bad);
    SP_TRY(hipGetLastError());
    unsigned bad = 0;
    if ((e = read_flag(W.bad, s, &bad)))
        return e;
    return bad ? CBG_E_UNSUPPORTED : CBG_OK;
}

int cbg_spai_pack(const double *V, int64_t ld, int32_t n, int32_t K, int32_t first,
                  int32_t stride, uint16_t *out, void *stream)
{
    if (n < 0 || K < 0 || K > CBG_SPAI_MAX_K || first < 0 || stride < 1 || ld < n ||
        (n > 0 && K > 0 && (!V || !out)))
        return CBG_E_ARG;
    if (n == 0 || K == 0)
        return CBG_OK;
    const int64_t total = (int64_t)n * K;
    hipLaunchKernelGGL(k_pack, dim3(row_grid(total)), dim3(256), 0, (hipStream_t)stream, V, ld, n,
                       K, first, stride, out);
    SP_TRY(hipGetLastError());
    return CBG_OK;
}

int cbg_spai_grad_p(const cbg_csr *A, const double *t_val, const float *p_val, int32_t K,
                    const uint16_t *V, double scale, double *loss, int32_t accumulate,
                    double *dP, void *ws, size_t ws_bytes, void *stream)
{
    if (!csr_ok(A) || K < 1 || K > CBG_SPAI_MAX_K || !loss ||
        (A->n > 0 && (!t_val || !p_val || !V || !dP)) || !isfinite(scale))
        return CBG_E_ARG;
    int e = ws_check(ws, ws_bytes, A->n, A->nnz, K);
    if (e)
        return e;
    hipStream_t s = (hipStream_t)stream;
    SpaiWs W = carve_spai(ws, A->n, A->nnz, K, nullptr);
    return enqueue_grad_p(A, t_val, p_val, K, V, scale, loss, accumulate, dP, W, s);
}

int cbg_spai_grad_o(const cbg_csr *A, const int32_t grid[3], const double *dP, uint16_t *dO,
                    void *stream)
{
    if (!csr_ok(A) || !grid_ok(A, grid) || (A->n > 0 && (!dP || !dO)) || !a16(dO))
        return CBG_E_ARG;
    if (A->n == 0)
        return CBG_OK;
    hipLaunchKernelGGL(k_grad_o, dim3(group_grid(A->n)), dim3(256), 0, (hipStream_t)stream, A->n,
                       A->row_ptr, A->col_idx, A->val, grid[0], grid[1], dP, dO);
    SP_TRY(hipGetLastError());
    return CBG_OK;
}

int cbg_mlp_backward(int32_t n, const uint16_t *feat, const uint16_t *h1, const uint16_t *h2,
                     const uint16_t *dO, const uint16_t *weights, double *grad,
                     int32_t accumulate, void *ws, size_t ws_bytes, void *stream)
{
    if (n < 0 || !grad || !weights || (n > 0 && (!feat || !h1 || !h2 || !dO)))
        return CBG_E_ARG;
    int e = ws_check(ws, ws_bytes, n, 0, 0);
    if (e)
        return e;
    SpaiWs W = carve_spai(ws, n, 0, 0, nullptr);
    return enqueue_backward(n, feat, h1, h2, dO, weights, grad, accumulate, W,
                            (hipStream_t)stream);
}

int cbg_spai_loss_grad(const cbg_csr *A, const double *t_val, const int32_t grid[3],
                       const uint16_t *feat, const uint16_t *weights, const float *params,
                       int32_t K, const uint16_t *V, double scale, double *loss, double *grad,
                       int32_t accumulate, void *ws, size_t ws_bytes, void *stream)
{
    if (!csr_ok(A) || !grid_ok(A, grid) || K < 1 || K > CBG_SPAI_MAX_K || !loss || !grad ||
        !weights || !params || (A->n > 0 && (!t_val || !feat || !V)) || !a16(feat) ||
        !a16(weights) || !a16(params) || !isfinite(scale))
        return CBG_E_ARG;
    int e = ws_check(ws, ws_bytes, A->n, A->nnz, K);
    if (e)
        return e;
    hipStream_t s = (hipStream_t)stream;
    SpaiWs W = carve_spai(ws, A->n, A->nnz, K, nullptr);
    if (A->n == 0) {
        hipLaunchKernelGGL(k_loss_fold, dim3(1), dim3(256), 0, s, (const double *)W.lpart, 0, 0.0,
                           accumulate, loss);
        hipLaunchKernelGGL(k_grad_fold, dim3((NPARAM + 255) / 256), dim3(256), 0, s,
                           (const float *)W.gpart, 0, accumulate, grad);
        SP_TRY(hipGetLastError());
        return CBG_OK;
    }
    enqueue_forward(A->n, feat, weights, params, W.O, W.h1, W.h2, s);
    hipLaunchKernelGGL(k_assemble, dim3(group_grid(A->n)), dim3(256), 0, s, A->n, A->row_ptr,
                       A->col_idx, A->val, grid[0], grid[1], (const float *)W.O, W.pval);
    if ((e = enqueue_grad_p(A, t_val, W.pval, K, V, scale, loss, accumulate, W.dP, W, s)))
        return e;
    hipLaunchKernelGGL(k_grad_o, dim3(group_grid(A->n)), dim3(256), 0, s, A->n, A->row_ptr,
                       A->col_idx, A->val, grid[0], grid[1], (const double *)W.dP, W.dO);
    return enqueue_backward(A->n, feat, W.h1, W.h2, W.dO, weights, grad, accumulate, W, s);
}

int cbg_spai_round_weights(const float *params, uint16_t *weights, void *stream)
{
    if (!params || !weights)
        return CBG_E_ARG;
    hipLaunchKernelGGL(k_round_weights, dim3((NWBF + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, params, weights);
    SP_TRY(hipGetLastError());
    return CBG_OK;
}

int cbg_adam_step(float *params, float *m1, float *m2, uint16_t *weights, const double *grad,
                  int64_t t, double lr, double beta1, double beta2, double eps, void *stream)
{
    if (!params || !m1 || !m2 || !weights || !grad || t < 1 || !(lr > 0) || !(beta1 >= 0) ||
        !(beta1 < 1) || !(beta2 >= 0) || !(beta2 < 1) || !(eps > 0))
        return CBG_E_ARG;
    const double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
    hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       params, m1, m2, weights, grad, lr, beta1, beta2, eps, c1, c2);
    SP_TRY(hipGetLastError());
    return CBG_OK;
}

}  // extern "C"
