// C ABI of the library: argument checks, workspace carving and the restart
// loop of Fig. 1 (Section 3).  Every step of the loop runs in the kernels of
// cbg_kernels.hip; this file only enqueues them, reads the device state once
// per restart cycle, and applies the host-side decisions (stop, restart,
// preconditioner fallback).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <vector>

#include "../../include/cbgmres.h"
#include "cbg_device.hpp"
#include "cbg_launch.hpp"

using namespace cbg;

namespace {

constexpr size_t ALIGN = 256;
constexpr int BJ_MAX = 8;          // largest block-Jacobi block size
constexpr double ETA_DEFAULT = 0.70710678118654752440;   // 1/sqrt(2), nearest double

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

bool valid_format(int f) { return f >= CBG_FP64 && f <= CBG_FP16S; }

// the preconditioners whose explicit-residual checks may drop them (M = I)
bool droppable(int pc) { return pc == CBG_PC_SPARSE || pc == CBG_PC_STENCIL; }

bool has_dix(const cbg_csr *A)
{
    return A->sell_dix && A->sell_diag && A->sell_ndiag >= 1 &&
           A->sell_ndiag <= CBG_SELL_MAX_DIAG;
}

bool has_sell(const cbg_csr *A)
{
    return A->sell_ptr && A->sell_val && (A->sell_col || has_dix(A));
}

// the sliced-ELL fields all set or all absent (columns as indices or as
// diagonal indices), and the entry count plausible
bool sell_ok(const cbg_csr *A)
{
    const bool any = A->sell_ptr || A->sell_col || A->sell_val || A->sell_dix || A->sell_diag;
    if (!any)
        return true;
    if ((A->sell_dix || A->sell_diag) && !has_dix(A))
        return false;
    return has_sell(A) && A->sell_entries >= A->nnz && A->sell_entries % 64 == 0;
}

// A's arrays into an SpMV argument block, with the sliced-ELL copy when
// present (rows longer than 12 entries on average stream it past the caches)
void set_matrix(SpmvArgs &a, const cbg_csr *A)
{
    a.rp = A->row_ptr;
    a.ci = A->col_idx;
    a.val = A->val;
    if (has_sell(A)) {
        a.sp = A->sell_ptr;
        a.sc = A->sell_col;
        a.sv = A->sell_val;
        if (has_dix(A)) {
            a.sd = A->sell_dix;
            a.sdiag = A->sell_diag;
            a.ndiag = A->sell_ndiag;
        }
        a.nslice = ((int64_t)A->n + 63) / 64;
        a.sell_nt = A->sell_entries > 12 * (int64_t)A->n;
    }
}

int64_t basis_ld(int32_t n) { return ((int64_t)n + 255) / 256 * 256; }

size_t red_bytes(int jmax)
{
    return align_up((size_t)(jmax + 2) * MAX_GRID * sizeof(double)) +
           align_up((size_t)2 * SPMV_MAX_GRID * sizeof(double));
}

// Carves a workspace front to back; records the total size.
struct Carver {
    uint8_t *base;
    size_t off = 0;
    explicit Carver(void *p) : base((uint8_t *)p) {}
    template <class T> T *take(size_t count)
    {
        T *p = base ? (T *)(base + off) : nullptr;
        off = align_up(off + count * sizeof(T));
        return p;
    }
};

RedWs carve_red(Carver &c, int jmax, int rows = 0)
{
    RedWs r;
    r.stride = MAX_GRID;
    r.sstride = SPMV_MAX_GRID;
    r.orth = c.take<double>((size_t)(rows > 0 ? rows : jmax + 2) * MAX_GRID);
    r.spmv = c.take<double>((size_t)2 * SPMV_MAX_GRID);
    return r;
}

struct SolveWs {
    size_t v_off, scales_off;   // byte offsets of V and scales in the workspace
    DevState *st;
    uint8_t *V;
    double *scales, *w0, *w1, *z, *v, *dinv, *xprev;
    int8_t *bj_tags;               // block-Jacobi: per-block storage precision
    double *bj64;                  // and the inverted blocks by precision
    float *bj32;
    uint16_t *bj16;
    double *H, *h, *u, *cs, *sn, *g, *y, *hist, *G;
    int32_t *flags;
    unsigned *bad;
    RedWs red;
};

SolveWs carve_solve(void *ws, int32_t n, int32_t m, int fmt, int pc, size_t *total)
{
    Carver c(ws);
    SolveWs s;
    const int64_t ld = basis_ld(n);
    s.st = c.take<DevState>(1);
    s.v_off = c.off;
    s.V = c.take<uint8_t>((size_t)(m + 1) * ld * fmt_bytes(fmt));
    s.scales_off = c.off;
    s.scales = c.take<double>(m + 1);
    s.w0 = c.take<double>(ld);   // the step's w and the previous step's w
    s.w1 = c.take<double>(ld);   // alternate between these two buffers
    const bool bj = pc == CBG_PC_BLOCK_JACOBI, stc = pc == CBG_PC_STENCIL;
    s.z = c.take<double>(pc == CBG_PC_SPARSE || bj || stc ? ld : 1);
    s.v = c.take<double>(bj || stc ? 1 : ld);   // v_j from the separate normalising pass
    s.dinv = c.take<double>(pc == CBG_PC_JACOBI || stc ? ld : 1);
    s.xprev = c.take<double>(pc == CBG_PC_SPARSE || stc ? ld : 1);
    // sized for the largest block size: ceil(n/bs) bs^2 <= n BJ_MAX + BJ_MAX^2
    const size_t bjv = bj ? (size_t)n * BJ_MAX + BJ_MAX * BJ_MAX : 1;
    s.bj_tags = c.take<int8_t>(bj ? (size_t)n + 1 : 1);
    s.bj64 = c.take<double>(bjv);
    s.bj32 = c.take<float>(bjv);
    s.bj16 = c.take<uint16_t>(bjv);
    s.H = c.take<double>((size_t)(m + 1) * m);
    s.h = c.take<double>(m + 1);
    s.u = c.take<double>(m + 1);
    s.cs = c.take<double>(m + 1);
    s.sn = c.take<double>(m + 1);
    s.g = c.take<double>(m + 2);
    s.y = c.take<double>(m + 1);
    s.hist = c.take<double>(m);
    s.flags = c.take<int32_t>(m);
    s.bad = c.take<unsigned>(1);
    s.G = c.take<double>((size_t)(m + 1) * (m + 1));
    // partial rows: h_k, two norms, and the Gram row g_k in rows j + 2 + k
    s.red = carve_red(c, m + 1, 2 * (m + 1) + 2);
    if (total)
        *total = c.off;
    return s;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

#define HIP_TRY(x)                              \
    do {                                        \
        const hipError_t e_ = (x);              \
        if (e_ != hipSuccess) {                 \
            note_hip_error(e_, __LINE__);       \
            (void)hipGetLastError();            \
            return CBG_E_HIP;                   \
        }                                       \
    } while (0)

// Algorithmic HBM bytes (what each kernel must move at least).
struct ByteModel {
    double n, nnz, bs;
    double sell = 0.0;      // entries of the sliced-ELL copy the SpMV reads (0: CSR)
    double sell_eb = 12.0;  // bytes per entry: value and column (9 with diagonal indices)
    // CSR (values, column indices, row pointers), or the sliced-ELL copy
    // (values, columns, slice offsets), the gathered input and the output
    // vector
    double spmv() const
    {
        return sell > 0.0 ? sell_eb * sell + 8.0 * (std::floor((n + 63.0) / 64.0) + 1.0) + 16.0 * n
                          : 12.0 * nnz + 4.0 * (n + 1) + 16.0 * n;
    }
    // the Arnoldi-step SpMV also stores the previous basis vector
    double spmv_step() const { return spmv() + n * bs; }
    double dot(int j) const { return j * n * bs + 8.0 * n; }
    double upd(int j) const { return j * n * bs + 16.0 * n; }
};

// Profiling events of one cycle: per step, start/end of the four
// basis-streaming launches (dot, update, re-dot, re-update) and of the SpMV
// with A, recorded by hipExtLaunchKernelGGL at each kernel's own start and
// end.
// Event pairs for the timed launches of a cycle: five launch slots per step.
// The events are created once per host thread and device, grown to the
// longest cycle asked for, and kept until the process ends (creating m x 10
// of them for every solve took about half a millisecond at m = 200).
struct CycleEvents {
    hipEvent_t *ev = nullptr;
    int create(int m)
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess)
            return CBG_E_HIP;
        static thread_local std::vector<std::vector<hipEvent_t>> pools;
        if ((int)pools.size() <= dev)
            pools.resize((size_t)dev + 1);
        std::vector<hipEvent_t> &p = pools[(size_t)dev];
        const size_t need = (size_t)m * 10;
        p.reserve(need);
        while (p.size() < need) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess)
                return CBG_E_HIP;
            p.push_back(e);
        }
        ev = p.data();
        return 0;
    }
    hipEvent_t at(int j, int k, int edge) const { return ev[((size_t)(j - 1) * 5 + k) * 2 + edge]; }
};

// Steps of a cycle are enqueued in chunks; after each chunk the cycle's done
// flag is copied to pinned host memory behind an event. The host reads the
// flag of the chunk before the one just enqueued, so one chunk always stays
// queued and the device never waits on the host, while a cycle that ends
// early (recurrence residual met, breakdown) leaves at most two chunks of
// launches that find the cycle finished and return at once.
constexpr int STEP_CHUNK = 16;

struct DoneWatch {
    hipEvent_t ev[2] = {nullptr, nullptr};
    int32_t *flag = nullptr;        // pinned: one slot per chunk of a cycle
    bool ok = false;
    int pending = -1;               // chunk whose event and flag are unread
    int create()
    {
        // the pinned slots are per host thread and live until the process ends
        static thread_local int32_t *slots = nullptr;
        if (!slots && hipHostMalloc((void **)&slots, sizeof(int32_t) * 2,
                                    hipHostMallocDefault) != hipSuccess) {
            slots = nullptr;
            (void)hipGetLastError();
            return 0;               // no pinned memory: every step is enqueued
        }
        for (auto &e : ev)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
                return CBG_E_HIP;
        flag = slots;
        ok = true;
        return 0;
    }
    // Called before the step that opens chunk k (k >= 1). Returns 1 when the
    // cycle was already finished by the end of chunk k - 2, so the caller
    // stops enqueueing; a negative value is a HIP error.
    int boundary(int k, const int32_t *done_dev, hipStream_t s)
    {
        if (!ok)
            return 0;
        const int slot = k & 1;
        if (hipMemcpyAsync(flag + slot, done_dev, sizeof(int32_t), hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipEventRecord(ev[slot], s) != hipSuccess)
            return -1;
        int stop = 0;
        if (pending >= 0) {
            if (hipEventSynchronize(ev[pending & 1]) != hipSuccess)
                return -1;
            stop = flag[pending & 1] != 0;
        }
        pending = k;
        return stop;
    }
    void reset() { pending = -1; }
    ~DoneWatch()
    {
        for (auto &e : ev)
            if (e)
                (void)hipEventDestroy(e);
    }
};

}  // namespace

// The failing HIP call's error code and source line, per host thread, for
// cbg_last_hip_error.
namespace {
thread_local int g_hip_err = 0, g_hip_line = 0;
}
void cbg::note_hip_error(hipError_t e, int line)
{
    g_hip_err = (int)e;
    g_hip_line = line;
}

extern "C" {

const char *cbg_strerror(int status)
{
    switch (status) {
    case CBG_OK: return "converged";
    case CBG_NOT_CONVERGED: return "iteration limit reached before the tolerance";
    case CBG_E_ARG: return "invalid argument";
    case CBG_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case CBG_E_HIP: return "HIP runtime error";
    case CBG_E_NONFINITE: return "non-finite value in the input or during the solve";
    case CBG_E_UNSUPPORTED: return "unsupported request";
    default: return "unknown status";
    }
}

int cbg_last_hip_error(int *line, const char **name)
{
    if (line)
        *line = g_hip_line;
    if (name)
        *name = g_hip_err ? hipGetErrorName((hipError_t)g_hip_err) : "hipSuccess";
    return g_hip_err;
}

int64_t cbg_basis_ld(int32_t n) { return n < 0 ? 0 : basis_ld(n); }

size_t cbg_workspace_bytes(int32_t n, int32_t restart, int32_t format, int32_t precond)
{
    if (n < 0 || restart < 1 || restart > CBG_MAX_RESTART || !valid_format(format) ||
        precond < CBG_PC_NONE || precond > CBG_PC_STENCIL)
        return 0;
    size_t total = 0;
    carve_solve(nullptr, n, restart, format, precond, &total);
    return total;
}

int cbg_workspace_basis(int32_t n, int32_t restart, int32_t format, int32_t precond,
                        size_t *basis_offset, size_t *scales_offset)
{
    if (n < 0 || restart < 1 || restart > CBG_MAX_RESTART || !valid_format(format) ||
        precond < CBG_PC_NONE || precond > CBG_PC_STENCIL || !basis_offset ||
        !scales_offset)
        return CBG_E_ARG;
    const SolveWs w = carve_solve(nullptr, n, restart, format, precond, nullptr);
    *basis_offset = w.v_off;
    *scales_offset = w.scales_off;
    return CBG_OK;
}

size_t cbg_kernel_workspace_bytes(int32_t n, int32_t j)
{
    if (n < 0 || j < 0 || j > CBG_MAX_RESTART + 1)
        return 0;
    return red_bytes(j);
}

int cbgmres_solve(const cbg_csr *A, const double *b, double *x, const cbg_opts *opt,
                  void *workspace, size_t ws_bytes, void *stream, cbg_result *res,
                  double *hist_out, int64_t hist_len)
{
    const double t_start = now_s();
    if (!res)
        return CBG_E_ARG;
    memset(res, 0, sizeof(*res));
    auto fail = [&](int code) {
        res->status = code;
        res->seconds = now_s() - t_start;
        return code;
    };
    if (!A || !opt || !sell_ok(A))
        return fail(CBG_E_ARG);
    const int32_t n = A->n, m = opt->restart;
    const int fmt = opt->format, pc0 = opt->precond;
    if (n < 0 || A->nnz < 0 || m < 1 || m > CBG_MAX_RESTART || !valid_format(fmt) ||
        !(opt->tol >= 0.0) || !isfinite(opt->tol) || opt->maxiter < 0 || pc0 < CBG_PC_NONE ||
        pc0 > CBG_PC_STENCIL || (hist_len > 0 && !hist_out) || hist_len < 0 ||
        (opt->flags & ~CBG_FLAG_ALL) != 0 ||
        (~opt->flags & (CBG_FLAG_NORMALISE_PASS | CBG_FLAG_NORMALISE_GATHER)) == 0 ||
        // the two-pass Gram form excludes the other forms of steps 5-10
        ((opt->flags & CBG_FLAG_TWO_PASS) &&
         (opt->flags & (CBG_FLAG_EXPLICIT_REDOT | CBG_FLAG_MGS))))
        return fail(CBG_E_ARG);
    const int bj_bs = opt->pc_block > 0 ? opt->pc_block : 4;
    const int bj_prec = opt->pc_prec > 0 ? opt->pc_prec : 16;
    if (pc0 == CBG_PC_BLOCK_JACOBI &&
        (bj_bs > BJ_MAX || (bj_prec != 16 && bj_prec != 32 && bj_prec != 64)))
        return fail(CBG_E_ARG);
    if (n > 0 && (!A->row_ptr || !A->col_idx || !A->val || !b || !x || !aligned16(b) ||
                  !aligned16(x) || (A->nnz > 0 && (!A->col_idx || !A->val))))
        return fail(CBG_E_ARG);
    if (pc0 == CBG_PC_SPARSE && n > 0 && !opt->p_val)
        return fail(CBG_E_ARG);
    if (pc0 == CBG_PC_STENCIL &&
        (opt->grid[0] < 1 || opt->grid[1] < 1 || opt->grid[2] < 1 ||
         (int64_t)opt->grid[0] * opt->grid[1] * opt->grid[2] != n ||
         (n > 0 && (!opt->p_stencil || !aligned16(opt->p_stencil)))))
        return fail(CBG_E_ARG);
    if (n == 0)
        return fail(CBG_OK);
    size_t need = 0;
    carve_solve(nullptr, n, m, fmt, pc0, &need);
    if (!workspace || ((uintptr_t)workspace & (ALIGN - 1)) || ws_bytes < need)
        return fail(CBG_E_WORKSPACE);

    hipStream_t s = (hipStream_t)stream;
    SolveWs W = carve_solve(workspace, n, m, fmt, pc0, nullptr);
    const int64_t ld = basis_ld(n);
    const size_t vbytes = (size_t)ld * fmt_bytes(fmt);
    const double eta = opt->eta > 0.0 ? opt->eta : ETA_DEFAULT;
    const int sg = spmv_shape_of(n, A->nnz);
    const bool prof_all = (opt->flags & CBG_FLAG_PROFILE) != 0;
    const bool prof = prof_all || (opt->flags & CBG_FLAG_PROFILE_DOT) != 0;
    const bool prof_spmv = (opt->flags & CBG_FLAG_PROFILE_SPMV) != 0;
    // the steps whose launches carry events: all, or every CBG_PROFILE_STRIDE-th
    // step of the solve; ev_on[j] marks them in the current cycle
    const int64_t prof_stride = (opt->flags & CBG_FLAG_PROFILE_SAMPLED) ? CBG_PROFILE_STRIDE : 1;
    int64_t step_no = 0;
    std::vector<char> ev_on((size_t)m + 1, 0);
    // launch slots k of a step: 0 multi-dot, 1 update (or fused update +
    // re-dot), 2 re-dot multi-dot, 3 re-orthogonalising update
    auto profiled = [&](int k) { return prof_all || k % 2 == 0; };
    const bool fuse = (opt->flags & CBG_FLAG_NO_FUSE) == 0;
    // ablations of the Arnoldi step
    const int vhat = (opt->flags & CBG_FLAG_SPMV_VHAT) ? 1 : 0;
    const int reorth_all = (opt->flags & CBG_FLAG_ALWAYS_REORTH) ? 1 : 0;
    const bool mgs = (opt->flags & CBG_FLAG_MGS) != 0;
    // step 8 in Gram form unless the explicit re-dot is asked for
    const bool gram = !mgs && (opt->flags & CBG_FLAG_EXPLICIT_REDOT) == 0;
    // steps 5-10 in one update unless the two-pass Gram form is asked for
    const bool onepass = gram && (opt->flags & CBG_FLAG_TWO_PASS) == 0;
    if (mgs && (prof || prof_spmv))
        return fail(CBG_E_UNSUPPORTED);     // event timing covers the CGS kernels only
    if (vhat && pc0 == CBG_PC_STENCIL)
        return fail(CBG_E_UNSUPPORTED);     // the stencil pass reads the FP64 v only
    // steps 13-14 in a pass of their own, or inside the next SpMV's gather:
    // one division per row against one per nonzero, so long rows favour the
    // pass; with Jacobi the pass also forms dinv .* v once, where the gather
    // reads dinv per nonzero
    const bool norm_pass = !vhat && pc0 != CBG_PC_BLOCK_JACOBI &&
        ((opt->flags & CBG_FLAG_NORMALISE_PASS) != 0 ||
         ((opt->flags & CBG_FLAG_NORMALISE_GATHER) == 0 &&
          ((double)A->nnz > 12.0 * n || pc0 == CBG_PC_JACOBI)));
    // steps whose update and re-dot share one basis pass
    auto fused = [&](int j) { return !gram && fuse && fused_takes(fmt, basis_ld(n), j); };
    ByteModel bm{(double)n, (double)A->nnz, (double)fmt_bytes(fmt)};
    if (has_sell(A)) {
        bm.sell = (double)A->sell_entries;
        bm.sell_eb = has_dix(A) ? 9.0 : 12.0;
    }

    std::vector<unsigned char> sa_buf(step_arrays_size());
    void *sa = sa_buf.data();
    make_step_arrays(sa, W.H, W.h, W.u, W.cs, W.sn, W.g, W.y, W.hist, W.scales, W.flags);
    set_step_gram(sa, W.G);

    // set-up: initialise the state, ||b||
    const int nb_orth = orth_grid(fmt, n);
    launch_clear_flags(nullptr, W.bad, s);
    launch_init_state(W.st, n, m, fmt, opt->tol, eta, opt->maxiter, reorth_all, s);
    {
        const int g = launch_norm(b, n, W.red, s);
        launch_reduce(W.red, RR_NB, 0, g, 0, W.st, sa, nullptr, fmt, s);
    }
    int pc = pc0;
    if (pc == CBG_PC_JACOBI || pc == CBG_PC_STENCIL) {
        SpmvArgs am{};
        am.n = n;
        set_matrix(am, A);
        launch_jacobi_setup(am, ld, W.dinv, W.bad, s);
    }
    const int bj_nblk = (n + bj_bs - 1) / bj_bs;
    std::vector<int8_t> bj_tags;
    if (pc == CBG_PC_BLOCK_JACOBI) {
        launch_bj_setup(n, A->row_ptr, A->col_idx, A->val, bj_bs, bj_prec, W.bj_tags, W.bj64,
                        W.bj32, W.bj16, W.bad, s);
        bj_tags.resize(bj_nblk);
        HIP_TRY(hipMemcpyAsync(bj_tags.data(), W.bj_tags, bj_nblk, hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipGetLastError());

    DevState hs;
    unsigned bad = 0;
    HIP_TRY(hipMemcpyAsync(&hs, W.st, sizeof(hs), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&bad, W.bad, sizeof(bad), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (bad)
        return fail(CBG_E_ARG);
    // bytes of one block-Jacobi apply's inverse values (a row reads its block row)
    double bj_bytes = 0.0;
    for (int b = 0; b < (int)bj_tags.size(); ++b) {
        const int sz = std::min(bj_bs, n - b * bj_bs);
        bj_bytes += (double)sz * sz * (bj_tags[b] / 8);
    }
    if (!isfinite(hs.nb))
        return fail(CBG_E_NONFINITE);
    if (hs.nb == 0.0) {                       // b = 0: the solution is x = 0
        HIP_TRY(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), s));
        HIP_TRY(hipStreamSynchronize(s));
        return fail(CBG_OK);
    }
    const double nb = hs.nb;

    CycleEvents evs;
    if ((prof || prof_spmv) && evs.create(m) != 0)
        return fail(CBG_E_HIP);
    DoneWatch watch;
    if (watch.create() != 0)
        return fail(CBG_E_HIP);
    int jl = m;                         // steps enqueued in the cycle that ran last

    std::vector<double> cyc_hist(m);
    std::vector<int32_t> cyc_flags(m);
    int64_t hist_n = 0;
    int status = CBG_NOT_CONVERGED;
    double rho_prev = INFINITY, rho = NAN;
    int stagnant = 0;
    int64_t cycles = 0;
    double model_bytes = 0.0;
    bool prev_cycle = false;
    int prev_pc = pc;

    for (;;) {
        // Fig. 1 step 1 / step 18: explicit residual r = b - A x into w,
        // ||r|| and max|r_i|; resets the cycle state.
        {
            SpmvArgs a{};
            a.n = n; a.ldy = ld; set_matrix(a, A);
            a.x = x; a.b = b; a.y = W.w0; a.ws = W.red; a.mode = 2 /*SP_RESID*/;
            a.role = 2 /*SR_FREE*/; a.sg = sg; a.st = W.st;
            const int g = launch_spmv(a, s);
            launch_reduce(W.red, RR_RESID, 0, g, 0, W.st, sa, nullptr, fmt, s);
            model_bytes += bm.spmv() + 8.0 * n;
        }
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(&hs, W.st, sizeof(hs), hipMemcpyDeviceToHost, s));
        if (prev_cycle) {
            HIP_TRY(hipMemcpyAsync(cyc_hist.data(), W.hist, sizeof(double) * m,
                                   hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(cyc_flags.data(), W.flags, sizeof(int32_t) * m,
                                   hipMemcpyDeviceToHost, s));
        }
        HIP_TRY(hipStreamSynchronize(s));

        if (prev_cycle) {
            // account for the cycle that just ended
            const int jeff = hs.jprev;
            if (prof) {
                // every launch of the cycle is timed, including the ones that
                // found the cycle finished (they move no bytes)
                for (int j = 1; j <= jl; ++j) {
                    if (!ev_on[j])
                        continue;
                    const bool ro = j <= jeff && (cyc_flags[j - 1] & 1);
                    for (int k = 0; k < 4; ++k) {
                        if ((k == 2 && (fused(j) || gram)) || (k == 3 && onepass) ||
                            !profiled(k))
                            continue;            // no separate re-dot launch, or not timed
                        float ms;
                        HIP_TRY(hipEventElapsedTime(&ms, evs.at(j, k, 0), evs.at(j, k, 1)));
                        const bool work = j <= jeff && (k < 3 || ro);
                        const double by = !work ? 0.0
                                          : k == 0 && gram ? bm.dot(j) + n * bm.bs
                                          : (k % 2 == 0) ? bm.dot(j) : bm.upd(j);
                        res->prof_orth_ms += ms;
                        res->prof_orth_bytes += by;
                        res->prof_orth_launches += 1;
                        if (k % 2 == 0) {
                            res->prof_dot_ms += ms;
                            res->prof_dot_bytes += by;
                            res->prof_dot_launches += 1;
                        } else if (k == 1 && fused(j)) {
                            res->prof_fused_ms += ms;
                            res->prof_fused_bytes += by;
                            res->prof_fused_launches += 1;
                        }
                    }
                }
            }
            if (prof_spmv) {
                // the step SpMV: the plain product when a pass formed M^-1 v,
                // else the gather variant, which also stores v_j
                const bool gather = !norm_pass && prev_pc != CBG_PC_STENCIL &&
                                    prev_pc != CBG_PC_SPARSE && prev_pc != CBG_PC_BLOCK_JACOBI;
                for (int j = 1; j <= jl; ++j) {
                    if (!ev_on[j])
                        continue;
                    float ms;
                    HIP_TRY(hipEventElapsedTime(&ms, evs.at(j, 4, 0), evs.at(j, 4, 1)));
                    res->prof_spmv_ms += ms;
                    res->prof_spmv_bytes +=
                        j <= jeff ? (gather ? bm.spmv_step() : bm.spmv()) : 0.0;
                    res->prof_spmv_launches += 1;
                }
            }
            for (int j = 1; j <= jeff; ++j) {
                const bool ro = cyc_flags[j - 1] & 1;
                if (cyc_flags[j - 1] & 4)
                    res->explicit_steps += 1;
                if (hist_n < hist_len)
                    hist_out[hist_n] = cyc_hist[j - 1];
                ++hist_n;
                // MGS pass: w read j + 1 times and written j times, each
                // stored vector read twice
                const double b_mgs = 2.0 * j * n * bm.bs + (2.0 * j + 1.0) * 8.0 * n;
                double b_step = bm.spmv_step() + (mgs ? b_mgs : bm.dot(j) + bm.upd(j));
                if (prev_pc == CBG_PC_JACOBI) b_step += 8.0 * n;
                if (prev_pc == CBG_PC_SPARSE) b_step += 8.0 * A->nnz + 4.0 * (n + 1) + 16.0 * n;
                // the stencil pass in place of the normalising one: codes
                // (27 x 2 bytes), dinv, and z written and read
                if (prev_pc == CBG_PC_STENCIL) b_step += 62.0 * n + 16.0 * n;
                if (prev_pc == CBG_PC_BLOCK_JACOBI) b_step += bj_bytes + 16.0 * n;
                if (norm_pass && prev_pc != CBG_PC_STENCIL)
                    b_step += 16.0 * n;  // v written by the pass, read by the SpMV
                if (!fused(j) && !mgs && !gram)
                    b_step += bm.dot(j);             // the separate re-dot pass
                if (gram)
                    b_step += n * bm.bs;             // the newest vector's tile for G
                if (ro && !onepass) b_step += mgs ? b_mgs : bm.upd(j);
                // a hard step of the one-pass form: the re-dot pass, and the
                // second update if it re-orthogonalised
                if (onepass && (cyc_flags[j - 1] & 4))
                    b_step += j * n * bm.bs + (ro ? bm.upd(j) : 0.0);
                model_bytes += b_step;
            }
            model_bytes += jeff * n * bm.bs + 16.0 * n;     // solution update
        }

        rho = hs.beta;
        if (hs.nonfinite || !isfinite(rho)) {
            if (droppable(pc) && opt->fallback && cycles > 0) {
                // plain CB-GMRES takes over from the last finite iterate
                HIP_TRY(hipMemcpyAsync(x, W.xprev, (size_t)n * sizeof(double),
                                       hipMemcpyDeviceToDevice, s));
                pc = CBG_PC_NONE;
                res->fell_back = 1;
                stagnant = 0;
                rho_prev = INFINITY;
                prev_cycle = false;
                launch_clear_flags(W.st, nullptr, s);
                continue;
            }
            status = CBG_E_NONFINITE;
            break;
        }
        if (rho <= hs.tau_nb) {
            status = CBG_OK;
            break;
        }
        if (hs.it >= opt->maxiter) {
            status = CBG_NOT_CONVERGED;
            break;
        }
        if (droppable(pc) && opt->fallback) {
            stagnant = rho > 0.99 * rho_prev ? stagnant + 1 : 0;
            if (stagnant >= 2) {
                pc = CBG_PC_NONE;
                res->fell_back = 1;
                stagnant = 0;
            }
        }
        rho_prev = rho;
        if (droppable(pc) && opt->fallback)
            HIP_TRY(hipMemcpyAsync(W.xprev, x, (size_t)n * sizeof(double),
                                   hipMemcpyDeviceToDevice, s));
        cycles += 1;
        prev_cycle = true;
        prev_pc = pc;

        // The residual r sits in w0 with t = beta; step 1's SpMV forms
        // v_1 = r / beta and stores it as basis vector 1.
        double *cur = W.w0, *nxt = W.w1;
        watch.reset();
        jl = m;
        for (int j = 1; j <= m; ++j) {
            if (j > 1 && (j - 1) % STEP_CHUNK == 0) {
                const int w = watch.boundary((j - 1) / STEP_CHUNK, &W.st->done, s);
                if (w < 0)
                    return fail(CBG_E_HIP);
                if (w > 0) {
                    jl = j - 1;
                    break;
                }
            }
            // steps 13-14 of the previous step (v_j = w / t, stored as basis
            // vector j) fused with steps 3-4: w = A M^-1 v_j, omega
            void *slot = W.V + (size_t)(j - 1) * vbytes;
            int nb_spmv;
            ev_on[j] = step_no++ % prof_stride == 0 ? 1 : 0;
            hipEvent_t sev0 = prof_spmv && ev_on[j] ? evs.at(j, 4, 0) : nullptr;
            hipEvent_t sev1 = prof_spmv && ev_on[j] ? evs.at(j, 4, 1) : nullptr;
            if (pc == CBG_PC_STENCIL) {
                // v_j = w / t stored, z = M^-1 v_j in one pass; then w = A z
                launch_stencil(fmt, 0, cur, n, ld, opt->grid, opt->p_stencil, W.dinv, W.z, slot,
                               W.scales + (j - 1), W.st, s);
                SpmvArgs b2{};
                b2.n = n; b2.ldy = ld; set_matrix(b2, A);
                b2.x = W.z; b2.y = nxt; b2.ws = W.red; b2.mode = 0 /*SP_PLAIN*/;
                b2.role = 1 /*SR_STEP*/; b2.sg = sg; b2.st = W.st;
                b2.ev0 = sev0; b2.ev1 = sev1;
                nb_spmv = launch_spmv(b2, s);
            } else if (pc == CBG_PC_BLOCK_JACOBI) {
                // v_j = w / t stored, z = M^-1 v_j; then w = A z, omega
                launch_bj_apply(n, ld, bj_bs, W.bj_tags, W.bj64, W.bj32, W.bj16, cur, W.z, 0,
                                W.st, slot, W.scales + (j - 1), fmt, vhat, s);
                SpmvArgs b2{};
                b2.n = n; b2.ldy = ld; set_matrix(b2, A);
                b2.x = W.z; b2.y = nxt; b2.ws = W.red; b2.mode = 0 /*SP_PLAIN*/;
                b2.role = 1 /*SR_STEP*/; b2.sg = sg; b2.st = W.st;
                b2.ev0 = sev0; b2.ev1 = sev1;
                nb_spmv = launch_spmv(b2, s);
            } else if (pc == CBG_PC_SPARSE) {
                SpmvArgs a{};
                a.n = n; a.ldy = ld; a.rp = A->row_ptr; a.ci = A->col_idx; a.fval = opt->p_val;
                a.y = W.z; a.ws = W.red; a.role = 0 /*SR_NONE*/; a.sg = sg; a.st = W.st;
                if (norm_pass) {
                    launch_step_normalize(fmt, cur, n, ld, nullptr, W.v, slot, W.scales + (j - 1),
                                          W.st, s);
                    a.x = W.v; a.mode = 3 /*SP_FLOATVAL*/;
                } else {
                    a.x = cur; a.mode = (vhat << 4) | 8 | 3 /*SP_STEP_FLOATVAL*/;
                    a.Q = slot; a.qscale = W.scales + (j - 1); a.fmt = fmt;
                }
                launch_spmv(a, s);
                SpmvArgs b2{};
                b2.n = n; b2.ldy = ld; set_matrix(b2, A);
                b2.x = W.z; b2.y = nxt; b2.ws = W.red; b2.mode = 0 /*SP_PLAIN*/;
                b2.role = 1 /*SR_STEP*/; b2.sg = sg; b2.st = W.st;
                b2.ev0 = sev0; b2.ev1 = sev1;
                nb_spmv = launch_spmv(b2, s);
            } else {
                SpmvArgs a{};
                a.n = n; a.ldy = ld; set_matrix(a, A);
                a.dinv = W.dinv; a.y = nxt; a.ws = W.red; a.role = 1 /*SR_STEP*/;
                a.sg = sg; a.st = W.st;
                const int base = pc == CBG_PC_JACOBI ? 1 /*SP_JACOBI*/ : 0 /*SP_PLAIN*/;
                if (norm_pass) {
                    // z = M^-1 v_j formed by the pass: step 3 is the plain SpMV
                    launch_step_normalize(fmt, cur, n, ld, pc == CBG_PC_JACOBI ? W.dinv : nullptr,
                                          W.v, slot, W.scales + (j - 1), W.st, s);
                    a.x = W.v; a.mode = 0 /*SP_PLAIN*/;
                } else {
                    a.x = cur; a.mode = (vhat << 4) | 8 | base;
                    a.Q = slot; a.qscale = W.scales + (j - 1); a.fmt = fmt;
                }
                a.ev0 = sev0; a.ev1 = sev1;
                nb_spmv = launch_spmv(a, s);
            }
            if (mgs) {
                // steps 5-12 by modified Gram-Schmidt: omega, then one launch
                // and one fold per stored vector, per pass
                launch_reduce(W.red, RR_H, 0, nb_spmv, 0, W.st, sa, nullptr, fmt, s);
                for (int pass = 1; pass <= 2; ++pass) {
                    double *coef = pass == 1 ? W.h : W.u;
                    for (int k = 0; k <= j; ++k) {
                        const int g = launch_mgs(fmt, W.V, ld, W.scales, n, k, j, nxt, coef,
                                                 W.red, W.st, pass, s);
                        const int role = k < j ? (pass == 1 ? RR_MGS_H : RR_MGS_U)
                                               : (pass == 1 ? RR_MGS_T : RR_T2);
                        launch_reduce(W.red, role, g, 0, j, W.st, sa, k < j ? coef + k : nullptr,
                                      fmt, s);
                    }
                }
                double *t = cur;
                cur = nxt;
                nxt = t;
                continue;
            }
            OrthArgs o{};
            o.fmt = fmt; o.V = W.V; o.ld = ld; o.scales = W.scales; o.n = n; o.j = j;
            o.w = nxt; o.wio = nxt; o.ws = W.red; o.st = W.st; o.gated = 1;
            auto timed = [&](int k) {
                const bool on = prof && profiled(k) && ev_on[j];
                o.ev0 = on ? evs.at(j, k, 0) : nullptr;
                o.ev1 = on ? evs.at(j, k, 1) : nullptr;
            };
            // step 5: h = V^T w ; w -= V h
            timed(0);
            o.gram = gram ? 1 : 0;
            launch_multidot(o, s);
            o.gram = 0;
            launch_reduce(W.red, gram ? RR_HG : RR_H, nb_orth, nb_spmv, j, W.st, sa, nullptr,
                          fmt, s);
            o.coef = W.h; o.role = 1 /*U_STEP1*/;
            timed(1);
            if (onepass) {
                // u = h - G h and steps 5-10 in one update with h + u or h;
                // a hard step's explicit second pass (nothing otherwise);
                // the close
                o.role = 6 /*U_CGS2*/; o.u = W.u; o.stw = W.st; o.G = W.G; o.sa = sa;
                launch_update(o, s);
                o.role = 7 /*U_HARD*/;
                o.ev0 = o.ev1 = nullptr;        // the events belong to the update above
                launch_update(o, s);
                launch_reduce(W.red, RR_C2, nb_orth, 0, j, W.st, sa, nullptr, fmt, s);
                double *t = cur;
                cur = nxt;
                nxt = t;
                continue;
            }
            if (gram) {
                // steps 6-8: ||w||, the test of step 7, u = h - G h
                o.role = 5 /*U_STEP1N*/;
                launch_update(o, s);
                launch_reduce(W.red, RR_UG, nb_orth, 0, j, W.st, sa, nullptr, fmt, s);
            } else if (fused(j)) {
                // steps 5-8 in one basis pass: w -= V h, then ||w||, max|w|
                // and u = V^T w of the updated rows
                const int nb_u = launch_update_redot(o, s);
                launch_reduce(W.red, RR_U, nb_u, 0, j, W.st, sa, nullptr, fmt, s);
            } else {
                launch_update(o, s);
                // steps 6-8: ||w||, the test of step 7, and u = V^T w in one pass
                o.with_norms = 1;
                timed(2);
                launch_multidot(o, s);
                launch_reduce(W.red, RR_U, nb_orth, 0, j, W.st, sa, nullptr, fmt, s);
            }
            // steps 8-12 (no work unless step 7 asked for it)
            o.coef = W.u; o.role = 2 /*U_STEP2*/;
            timed(3);
            launch_update(o, s);
            launch_reduce(W.red, RR_T2, nb_orth, 0, j, W.st, sa, nullptr, fmt, s);
            double *t = cur;
            cur = nxt;
            nxt = t;
        }
        HIP_TRY(hipGetLastError());
        // step 17: y = R^-1 g ; x += M^-1 V y
        launch_backsolve(W.st, sa, s);
        {
            OrthArgs o{};
            o.fmt = fmt; o.V = W.V; o.ld = ld; o.scales = W.scales; o.n = n; o.j = 0;
            o.coef = W.y; o.ws = W.red; o.st = W.st;
            if (pc == CBG_PC_BLOCK_JACOBI) {
                o.role = 4 /*U_COMBINE*/;       // z = V y
                o.wio = W.z;
                launch_update(o, s);
                launch_bj_apply(n, ld, bj_bs, W.bj_tags, W.bj64, W.bj32, W.bj16, W.z, x, 1,
                                nullptr, nullptr, nullptr, fmt, 0, s);   // x += M^-1 z
            } else if (pc == CBG_PC_STENCIL) {
                o.role = 4 /*U_COMBINE*/;       // z = V y
                o.wio = W.z;
                launch_update(o, s);
                launch_stencil(fmt, 2, W.z, n, ld, opt->grid, opt->p_stencil, W.dinv, x, nullptr,
                               nullptr, nullptr, s);   // x += M^-1 z
            } else if (pc == CBG_PC_SPARSE) {
                o.role = 4 /*U_COMBINE*/;       // z = V y
                o.wio = W.z;
                launch_update(o, s);
                SpmvArgs a{};                   // x += P z
                a.n = n; a.ldy = n; a.rp = A->row_ptr; a.ci = A->col_idx; a.fval = opt->p_val;
                a.x = W.z; a.y = x; a.ws = W.red; a.mode = 4 /*SP_ACCUM*/; a.role = 0;
                a.sg = sg; a.st = nullptr;
                launch_spmv(a, s);
            } else {
                o.role = 3 /*U_SOLUTION*/;      // x += dinv .* (V y)  or  x += V y
                o.dinv = pc == CBG_PC_JACOBI ? W.dinv : nullptr;
                o.wio = x;
                launch_update(o, s);
            }
        }
        HIP_TRY(hipGetLastError());
    }

    res->status = status;
    res->iterations = hs.it;
    res->restarts = cycles;
    res->reorths = hs.reorths;
    res->breakdowns = hs.breakdowns;
    res->true_rel_res = rho / nb;
    res->recurrence_rel_res = hs.last_rec;
    res->model_bytes = model_bytes;
    res->seconds = now_s() - t_start;
    return status;
}

// ------------------------------------------------------------------------
// Kernel-level entry points.
// ------------------------------------------------------------------------

static bool kernel_ws_ok(void *ws, size_t ws_bytes, int j)
{
    return ws && ((uintptr_t)ws & (ALIGN - 1)) == 0 && ws_bytes >= red_bytes(j);
}

static RedWs kernel_red(void *ws, int j)
{
    Carver c(ws);
    return carve_red(c, j);
}

int cbg_encode(int32_t format, const double *v, int32_t n, void *q, double *scale, void *ws,
               size_t ws_bytes, void *stream)
{
    if (!valid_format(format) || n < 0 || !scale || (n > 0 && (!v || !q)) || !aligned16(v) ||
        !aligned16(q))
        return CBG_E_ARG;
    if (!kernel_ws_ok(ws, ws_bytes, 0))
        return CBG_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    RedWs r = kernel_red(ws, 0);
    const int g = launch_norm(v, n, r, s);
    launch_reduce(r, RR_SCALE, 0, g, 0, nullptr, nullptr, scale, format, s);
    if (n > 0)
        launch_normalize(format, v, n, n, nullptr, q, scale, nullptr, 1.0, nullptr, 0, s);
    HIP_TRY(hipGetLastError());
    return CBG_OK;
}

int cbg_decode(int32_t format, const void *q, const double *scale, int32_t n, double *v,
               void *stream)
{
    if (!valid_format(format) || n < 0 || !scale || (n > 0 && (!v || !q)) || !aligned16(v) ||
        !aligned16(q))
        return CBG_E_ARG;
    if (n > 0)
        launch_decode(format, q, n, scale, v, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return CBG_OK;
}

int cbg_spmv(const cbg_csr *A, const double *x, double *y, double *norm2, void *ws,
             size_t ws_bytes, void *stream)
{
    if (!A || A->n < 0 || A->nnz < 0 || !sell_ok(A) ||
        (A->n > 0 && (!A->row_ptr || !x || !y || (A->nnz > 0 && (!A->col_idx || !A->val)))))
        return CBG_E_ARG;
    if (norm2 && !kernel_ws_ok(ws, ws_bytes, 0))
        return CBG_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (A->n == 0) {
        if (norm2)
            HIP_TRY(hipMemsetAsync(norm2, 0, sizeof(double), s));
        return CBG_OK;
    }
    SpmvArgs a{};
    a.n = A->n; a.ldy = A->n; set_matrix(a, A); a.x = x;
    a.y = y; a.mode = 0; a.sg = spmv_shape_of(A->n, A->nnz);
    a.role = norm2 ? 2 /*SR_FREE*/ : 0;
    if (norm2)
        a.ws = kernel_red(ws, 0);
    const int g = launch_spmv(a, s);
    if (norm2)
        launch_reduce(a.ws, RR_NORM2, 0, g, 0, nullptr, nullptr, norm2, 0, s);
    HIP_TRY(hipGetLastError());
    return CBG_OK;
}

int cbg_sell_ptr(const cbg_csr *A, int64_t *sell_ptr, int64_t *entries, void *stream)
{
    if (!A || A->n < 0 || A->nnz < 0 || !sell_ptr || !entries || ((uintptr_t)sell_ptr & 7) ||
        (A->n > 0 && !A->row_ptr))
        return CBG_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    const int64_t nslice = ((int64_t)A->n + 63) / 64;
    *entries = 0;
    if (nslice == 0) {
        HIP_TRY(hipMemsetAsync(sell_ptr, 0, sizeof(int64_t), s));
        HIP_TRY(hipStreamSynchronize(s));
        return CBG_OK;
    }
    launch_sell_ptr(A->n, A->row_ptr, nslice, sell_ptr, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(entries, sell_ptr + nslice, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return CBG_OK;
}

int cbg_sell_diag(const cbg_csr *A, int32_t *sell_diag, uint8_t *sell_dix, int32_t *ndiag,
                  void *ws, size_t ws_bytes, void *stream)
{
    if (!A || A->n < 0 || !ndiag || !sell_diag || (A->n > 0 && (!A->sell_ptr || !A->sell_col ||
                                                                !sell_dix)))
        return CBG_E_ARG;
    if (!kernel_ws_ok(ws, ws_bytes, 0))
        return CBG_E_WORKSPACE;
    *ndiag = 0;
    const int64_t nslice = ((int64_t)A->n + 63) / 64;
    if (nslice == 0)
        return CBG_OK;
    int32_t count = 0;
    const int rc = launch_sell_diag(A->n, nslice, A->sell_ptr, A->sell_col, sell_diag, sell_dix,
                                    ws, (hipStream_t)stream, &count);
    HIP_TRY(hipGetLastError());
    if (rc < 0)
        return CBG_E_HIP;
    *ndiag = count;
    return rc == 0 ? CBG_OK : CBG_E_UNSUPPORTED;
}

int cbg_sell_fill(const cbg_csr *A, const int64_t *sell_ptr, int32_t *sell_col, double *sell_val,
                  void *stream)
{
    if (!A || A->n < 0 || A->nnz < 0 || !sell_ptr ||
        (A->n > 0 && (!A->row_ptr || !sell_col || !sell_val ||
                      (A->nnz > 0 && (!A->col_idx || !A->val)))))
        return CBG_E_ARG;
    const int64_t nslice = ((int64_t)A->n + 63) / 64;
    if (nslice == 0)
        return CBG_OK;
    launch_sell_fill(A->n, A->row_ptr, A->col_idx, A->val, nslice, sell_ptr, sell_col, sell_val,
                     (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return CBG_OK;
}

static bool basis_args_ok(int32_t format, const void *V, int64_t ld, const double *scales,
                          int32_t n, int32_t j)
{
    return valid_format(format) && n >= 0 && j >= 0 && j <= CBG_MAX_RESTART + 1 && ld >= n &&
           ld % 16 == 0 && (j == 0 || n == 0 || (V && scales && aligned16(V)));
}

int cbg_multidot(int32_t format, const void *V, int64_t ld, const double *scales, int32_t n,
                 int32_t j, const double *w, double *h, void *ws, size_t ws_bytes, void *stream)
{
    if (!basis_args_ok(format, V, ld, scales, n, j) || (j > 0 && !h) ||
        (n > 0 && (!w || !aligned16(w))))
        return CBG_E_ARG;
    if (!kernel_ws_ok(ws, ws_bytes, j))
        return CBG_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (j == 0)
        return CBG_OK;
    if (n == 0) {
        HIP_TRY(hipMemsetAsync(h, 0, sizeof(double) * j, s));
        return CBG_OK;
    }
    OrthArgs o{};
    o.fmt = format; o.V = V; o.ld = ld; o.scales = scales; o.n = n; o.j = j; o.w = w;
    o.ws = kernel_red(ws, j);
    launch_multidot(o, s);
    launch_reduce(o.ws, RR_VALUES, orth_grid(format, n), 0, j, nullptr, nullptr, h, format, s);
    HIP_TRY(hipGetLastError());
    return CBG_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------
// The multi-dot without a workspace argument: its block partials live in a
// fixed device array of this library, one per GPU (each device holds its own
// copy at its own address, found once per device with hipGetSymbolAddress).
// ------------------------------------------------------------------------

namespace {

// the workspace layout of the kernel-level calls at the largest j: j + 2
// rows of multi-dot partials, then the SpMV's two rows
constexpr int NOALLOC_ROWS = CBG_NOALLOC_MAX_J + 4;
constexpr size_t NOALLOC_DOUBLES = (size_t)NOALLOC_ROWS * MAX_GRID;
__device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int NOALLOC_MAX_DEVICES = 64;
double *g_scratch_ptr[NOALLOC_MAX_DEVICES];
std::mutex g_scratch_mu;

// This device's copy of `scratch` (a device address; the array's name in
// host code is only a host-side stand-in), or nullptr after a HIP error.
double *scratch_on_current_device()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            note_hip_error(e, __LINE__);
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[dev] = (double *)p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

int cbg_multidot_noalloc(int32_t format, const void *V, int64_t ld, const double *scales,
                         int32_t n, int32_t j, const double *w, double *h, void *stream)
{
    if (!basis_args_ok(format, V, ld, scales, n, j) || (j > 0 && !h) ||
        (n > 0 && (!w || !aligned16(w))))
        return CBG_E_ARG;
    if (j > CBG_NOALLOC_MAX_J)
        return CBG_E_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    if (j == 0)
        return CBG_OK;
    if (n == 0) {
        launch_fill_zero(h, j, s);
        HIP_TRY(hipGetLastError());
        return CBG_OK;
    }
    double *base = scratch_on_current_device();
    if (!base)
        return CBG_E_HIP;
    OrthArgs o{};
    o.fmt = format; o.V = V; o.ld = ld; o.scales = scales; o.n = n; o.j = j; o.w = w;
    o.ws.orth = base;          // rows 0 .. j-1: the block partials of h
    o.ws.spmv = base + (size_t)(j + 2) * MAX_GRID;
    o.ws.stride = MAX_GRID;
    o.ws.sstride = MAX_GRID;            // no SpMV here
    launch_multidot(o, s);
    launch_reduce(o.ws, RR_VALUES, orth_grid(format, n), 0, j, nullptr, nullptr, h, format, s);
    HIP_TRY(hipGetLastError());
    return CBG_OK;
}

int cbg_update(int32_t format, const void *V, int64_t ld, const double *scales, int32_t n,
               int32_t j, const double *h, double *w, double *norms, void *ws, size_t ws_bytes,
               void *stream)
{
    if (!basis_args_ok(format, V, ld, scales, n, j) || (j > 0 && !h) ||
        (n > 0 && (!w || !aligned16(w))))
        return CBG_E_ARG;
    if (!kernel_ws_ok(ws, ws_bytes, 0))
        return CBG_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        if (norms)
            HIP_TRY(hipMemsetAsync(norms, 0, 2 * sizeof(double), s));
        return CBG_OK;
    }
    OrthArgs o{};
    o.fmt = format; o.V = V; o.ld = ld; o.scales = scales; o.n = n; o.j = j; o.coef = h;
    o.wio = w; o.role = 0 /*U_PLAIN*/; o.ws = kernel_red(ws, 0);
    launch_update(o, s);
    if (norms)
        launch_reduce(o.ws, RR_NORMS, orth_grid(format, n), 0, 0, nullptr, nullptr, norms, format,
                      s);
    HIP_TRY(hipGetLastError());
    return CBG_OK;
}

int cbg_update_redot(int32_t format, const void *V, int64_t ld, const double *scales, int32_t n,
                     int32_t j, const double *h, double *w, double *u, double *norms, void *ws,
                     size_t ws_bytes, void *stream)
{
    if (!basis_args_ok(format, V, ld, scales, n, j) || j < 1 || !h || !u || !norms ||
        (n > 0 && (!w || !aligned16(w))))
        return CBG_E_ARG;
    if (!kernel_ws_ok(ws, ws_bytes, j))
        return CBG_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        HIP_TRY(hipMemsetAsync(u, 0, sizeof(double) * j, s));
        HIP_TRY(hipMemsetAsync(norms, 0, 2 * sizeof(double), s));
        return CBG_OK;
    }
    OrthArgs o{};
    o.fmt = format; o.V = V; o.ld = ld; o.scales = scales; o.n = n; o.j = j; o.coef = h;
    o.wio = w; o.w = w; o.ws = kernel_red(ws, j);
    int nb = launch_update_redot(o, s);
    if (nb == 0) {
        // beyond the register tile: the same arithmetic in two passes
        o.role = 0 /*U_PLAIN*/;
        launch_update(o, s);
        o.with_norms = 1;
        launch_multidot(o, s);
        nb = orth_grid(format, n);
    }
    launch_reduce(o.ws, RR_VALUES, nb, 0, j, nullptr, nullptr, u, format, s);
    RedWs tail = o.ws;                  // ||w||^2 and max|w| follow the j values
    tail.orth += (size_t)j * tail.stride;
    launch_reduce(tail, RR_NORMS, nb, 0, 0, nullptr, nullptr, norms, format, s);
    HIP_TRY(hipGetLastError());
    return CBG_OK;
}

int cbg_block_jacobi_setup(const cbg_csr *A, int32_t bs, int32_t prec_min, int8_t *tags,
                           double *x64, float *x32, uint16_t *x16, void *ws, size_t ws_bytes,
                           void *stream)
{
    if (!A || A->n < 0 || bs < 1 || bs > BJ_MAX ||
        (prec_min != 16 && prec_min != 32 && prec_min != 64) ||
        (A->n > 0 && (!A->row_ptr || !tags || !x64 || !x32 || !x16 ||
                      (A->nnz > 0 && (!A->col_idx || !A->val)))))
        return CBG_E_ARG;
    if (!kernel_ws_ok(ws, ws_bytes, 0))
        return CBG_E_WORKSPACE;
    if (A->n == 0)
        return CBG_OK;
    hipStream_t s = (hipStream_t)stream;
    unsigned *bad = (unsigned *)ws;
    HIP_TRY(hipMemsetAsync(bad, 0, sizeof(unsigned), s));
    launch_bj_setup(A->n, A->row_ptr, A->col_idx, A->val, bs, prec_min, tags, x64, x32, x16,
                    bad, s);
    HIP_TRY(hipGetLastError());
    unsigned hb = 0;
    HIP_TRY(hipMemcpyAsync(&hb, bad, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return hb ? CBG_E_ARG : CBG_OK;
}

int cbg_block_jacobi_apply(int32_t n, int32_t bs, const int8_t *tags, const double *x64,
                           const float *x32, const uint16_t *x16, const double *v, double *z,
                           void *stream)
{
    if (n < 0 || bs < 1 || bs > BJ_MAX ||
        (n > 0 && (!tags || !x64 || !x32 || !x16 || !v || !z)))
        return CBG_E_ARG;
    if (n == 0)
        return CBG_OK;
    launch_bj_apply(n, n, bs, tags, x64, x32, x16, v, z, 0, nullptr, nullptr, nullptr, 0, 0,
                    (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return CBG_OK;
}

}  // extern "C"
