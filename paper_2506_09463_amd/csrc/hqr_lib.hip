// hqr_lib.hip -- libhqr: the C ABI declared in include/hqr.h and its host
// dispatch.  One translation unit: the kernels live in the included headers.
#include "hqr.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>

#include "hqr_device.hpp"
#include "hqr_small.hpp"
#include "hqr_blocked.hpp"
#include "hqr_cqr.hpp"
#include "hqr_batched.hpp"
#include "hqr_wg.hpp"

#include <numeric>
#include <vector>

namespace hqr {

// ------------------------------------------------------------- profiling
// Optional per-kernel-class timing: while active, every launch is bracketed
// by a pair of HIP events recorded on the launch's own stream.
enum KClass {
    K_SMALL, K_PANEL, K_VTX, K_TFACTOR, K_WSOLVE, K_UPDATE, K_DIAG, K_TRSV, K_RESNORM, K_FILL,
    K_GRAM1, K_GRAM2, K_GRED, K_CQR_CHOL, K_CQR_FINISH, K_NVTX, K_BATCHED, K_REFINE, K_NCLASS
};
static const char *kclass_name[K_NCLASS] = {"small_lsq", "panel_col", "vtx", "tfactor", "wsolve",
                                            "update", "diag_check", "trsv", "resnorm", "fill",
                                            "cqr_gram1", "cqr_gram2", "gram_reduce", "cqr_chol",
                                            "cqr_finish", "narrow_vtx", "batched_lsq", "refine"};
struct ProfRec {
    int cls;
    hipEvent_t e0, e1;
};
struct ProfState {
    bool on = false;
    ProfRec *recs = nullptr;
    size_t n = 0, cap = 0;
    hipEvent_t *pool = nullptr;
    size_t pool_n = 0, pool_used = 0;
};
static ProfState g_prof;

static hipEvent_t prof_event()
{
    if (g_prof.pool_used == g_prof.pool_n) {
        size_t nn = g_prof.pool_n ? 2 * g_prof.pool_n : 1024;
        hipEvent_t *np = (hipEvent_t *)realloc(g_prof.pool, nn * sizeof(hipEvent_t));
        if (!np) return nullptr;
        g_prof.pool = np;
        for (size_t i = g_prof.pool_n; i < nn; ++i)
            if (hipEventCreate(&g_prof.pool[i]) != hipSuccess) g_prof.pool[i] = nullptr;
        g_prof.pool_n = nn;
    }
    return g_prof.pool[g_prof.pool_used++];
}

static hipEvent_t prof_begin(hipStream_t s)
{
    if (!g_prof.on) return nullptr;
    hipEvent_t e = prof_event();
    if (e) (void)hipEventRecord(e, s);
    return e;
}

static void prof_end(int cls, hipEvent_t e0, hipStream_t s)
{
    if (!g_prof.on || !e0) return;
    hipEvent_t e1 = prof_event();
    if (!e1) return;
    (void)hipEventRecord(e1, s);
    if (g_prof.n == g_prof.cap) {
        size_t nc = g_prof.cap ? 2 * g_prof.cap : 1024;
        ProfRec *nr = (ProfRec *)realloc(g_prof.recs, nc * sizeof(ProfRec));
        if (!nr) return;
        g_prof.recs = nr;
        g_prof.cap = nc;
    }
    g_prof.recs[g_prof.n++] = ProfRec{cls, e0, e1};
}

#define HQR_LAUNCH(cls, kern, grid, block, shmem, stream, ...)                     \
    do {                                                                           \
        hipEvent_t e0_ = prof_begin(stream);                                       \
        hipLaunchKernelGGL(kern, grid, block, shmem, stream, __VA_ARGS__);         \
        prof_end(cls, e0_, stream);                                                \
    } while (0)

// ------------------------------------------------- one-workgroup variants
typedef void (*wg_batched_fn)(const WgDesc *, int, int *, int *);
typedef void (*wg_single_fn)(WgDesc, int *);
struct WgVariant {
    const char *name;
    int nt, qm, per_cu;
    wg_batched_fn batched;
    wg_single_fn single;
    int64_t max_rows, max_x;
};

template <int NT, int QM>
static WgVariant make_wg(const char *name)
{
    const int per_cu = (int)std::max<size_t>(1, (160 * 1024) / sizeof(WgShared<NT, QM>));
    return WgVariant{name, NT, QM, std::min(per_cu, 2), wg_batched_kernel<NT, QM>, wg_single_kernel<NT, QM>,
                     wg_max_rows<NT, QM>(), wg_max_x<NT, QM>()};
}

static const WgVariant *wg_variants(int *count)
{
    static const WgVariant v[] = {
        make_wg<64, 2>("wg64x2"),   // m <= 128, one wave
        make_wg<64, 4>("wg64x4"),   // m <= 256, one wave
        make_wg<128, 1>("wg128x1"), // m <= 128
        make_wg<256, 1>("wg256x1"), // m <= 256
        make_wg<128, 4>("wg128x4"), // m <= 512
        make_wg<256, 2>("wg256x2"), // m <= 512
        make_wg<256, 4>("wg256x4"), // m <= 1024
    };
    *count = (int)(sizeof(v) / sizeof(v[0]));
    return v;
}

static bool wg_fits(const WgVariant &v, int64_t m, int64_t n, int64_t nrhs)
{
    return m <= v.max_rows && n * nrhs <= v.max_x;
}

// Tuning rules (first match wins): op HQR_TUNE_SINGLE picks the path of one
// problem (-1 = the blocked multi-kernel path, else a variant index), op
// HQR_TUNE_BATCHED the variant of a batched launch from the batch's largest
// m and n.  Without a matching rule: single problems with n <= 128 and
// batches use the smallest variant that holds them.
struct TuneRule {
    int op;
    int64_t mlo, mhi, nlo, nhi;
    int prec, choice;
};
static std::vector<TuneRule> g_rules;

static int tune_lookup(int op, int64_t m, int64_t n, int prec)
{
    for (const TuneRule &r : g_rules)
        if (r.op == op && r.prec == prec && m >= r.mlo && m <= r.mhi && n >= r.nlo && n <= r.nhi) return r.choice;
    return -2;
}

static const WgVariant *pick_wg_single(int64_t m, int64_t n, int64_t nrhs)
{
    int cnt = 0;
    const WgVariant *v = wg_variants(&cnt);
    const int c = tune_lookup(HQR_TUNE_SINGLE, m, n, HQR_PREC_FP64);
    if (c == -1) return nullptr;
    if (c >= 0 && c < cnt && wg_fits(v[c], m, n, nrhs)) return &v[c];
    if (n > 128) return nullptr;
    for (int i = 0; i < cnt; ++i)
        if (wg_fits(v[i], m, n, nrhs)) return &v[i];
    return nullptr;
}

// Batched launches use only the variants with BATCH_NT threads: with the
// thread count fixed, the rows each thread holds (QM) change no arithmetic
// (row-to-thread map, reduction trees and tile order depend on NT alone), so
// an instance's result does not depend on the rest of the batch.  Whether an
// instance goes to the one-workgroup kernel also depends on its own shape
// only: m <= BATCH_WG_ROWS and n * nrhs within the smallest staging area.
constexpr int BATCH_NT = 256;
constexpr int64_t BATCH_WG_ROWS = 1024;

static bool batch_variant(const WgVariant &v) { return v.nt == BATCH_NT; }

static bool batch_wg_fits(int64_t m, int64_t n, int64_t nrhs)
{
    int cnt = 0;
    const WgVariant *v = wg_variants(&cnt);
    int64_t xmin = INT64_MAX;
    for (int i = 0; i < cnt; ++i)
        if (batch_variant(v[i])) xmin = std::min(xmin, v[i].max_x);
    return m <= BATCH_WG_ROWS && n * nrhs <= xmin;
}

static const WgVariant *pick_wg_batched(int64_t mmax, int64_t nmax)
{
    int cnt = 0;
    const WgVariant *v = wg_variants(&cnt);
    const int c = tune_lookup(HQR_TUNE_BATCHED, mmax, nmax, HQR_PREC_FP64);
    if (c >= 0 && c < cnt && batch_variant(v[c]) && v[c].max_rows >= mmax) return &v[c];
    const WgVariant *best = nullptr;
    for (int i = 0; i < cnt; ++i)
        if (batch_variant(v[i]) && v[i].max_rows >= mmax && (!best || v[i].max_rows < best->max_rows)) best = &v[i];
    return best;
}

static int launch_wg_single(const WgVariant *v, const WgDesc &d, int *info, hipStream_t s)
{
    HQR_LAUNCH(K_SMALL, v->single, dim3(1), dim3(v->nt), 0, s, d, info);
    return hipGetLastError() == hipSuccess ? 0 : HQR_EDEVICE;
}

// ------------------------------------------------------------- small path
typedef void (*small_fn)(SmallArgs);
struct SmallCfg {
    int nw, rw, q;
    small_fn fn;
    size_t static_lds;
};

template <int NW, int RW, int Q>
static SmallCfg make_small()
{
    const size_t st = sizeof(double) * (2 * NW * (Q * 64 + 2) + 2 * Q * 64 + NW + Q * 64 + 2 * NW * RW) + 16;
    return SmallCfg{NW, RW, Q, small_lsq_kernel<NW, RW, Q>, st};
}

static const SmallCfg *small_configs(int *count)
{
    static SmallCfg cfgs[] = {
        make_small<4, 16, 1>(),  // m <= 64,  n+nrhs <= 64
        make_small<8, 16, 2>(),  // m <= 128, n+nrhs <= 128
        make_small<16, 16, 2>(), // m <= 256, n+nrhs <= 128
    };
    *count = (int)(sizeof(cfgs) / sizeof(cfgs[0]));
    return cfgs;
}

static constexpr size_t LDS_LIMIT = 160 * 1024;

static const SmallCfg *pick_small(int64_t m, int64_t n, int64_t nrhs)
{
    if (m > 256 || n + nrhs > 128 || n == 0) return nullptr;
    int cnt = 0;
    const SmallCfg *c = small_configs(&cnt);
    for (int i = 0; i < cnt; ++i) {
        if (m > (int64_t)c[i].nw * c[i].rw || n + nrhs > 64 * c[i].q) continue;
        if (c[i].static_lds + small_dyn_lds((int)m, (int)n, (int)nrhs) > LDS_LIMIT) continue;
        return &c[i];
    }
    return nullptr;
}

static hipError_t launch_small(const SmallCfg *cfg, SmallArgs a, hipStream_t s)
{
    a.ldl = small_ldl(a.m);
    const size_t dyn = small_dyn_lds(a.m, a.n, a.nrhs);
    (void)hipFuncSetAttribute((const void *)cfg->fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    HQR_LAUNCH(K_SMALL, cfg->fn, dim3(1), dim3(cfg->nw * 64), dyn, s, a);
    return hipGetLastError();
}

// ------------------------------------------------------------ large path
struct Plan {
    int64_t m, n, nrhs;
    int nchunk;      // panel row chunks for the first panel (upper bound)
    int nxpad;       // row stride of W partials
    int nsplit_max;
    int nblk;        // triangular blocks
    int ngroups;     // CholeskyQR row groups of the first panel (upper bound)
    int npanels;
    int nb;          // panel width (<= NB)
    bool f32;        // trailing-update contractions in FP32
};

static int64_t rup(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

static Plan make_plan(int64_t m, int64_t n, int64_t nrhs, int nb = NB, bool f32 = false)
{
    Plan p;
    p.nb = nb;
    p.f32 = f32;
    p.m = m;
    p.n = n;
    p.nrhs = nrhs;
    p.nchunk = (int)((m + PC_ROWS - 1) / PC_ROWS);
    p.nxpad = (int)rup(NB + n + nrhs, 128);
    p.nsplit_max = 16;
    p.nblk = (int)((n + 63) / 64);
    p.ngroups = (int)((m + CQR_ROWS - 1) / CQR_ROWS);
    p.npanels = (int)((n + nb - 1) / nb);
    return p;
}

struct Work {
    double *xbuf, *pbuf, *wpart, *T, *wp;
    double *wpart2, *T2, *wp2;            // second set for the look-ahead stream
    int *flags;
    int *iscratch;
    double *gpart, *r1, *r1inv, *winv, *q1top;
    double *G, *xn;                          // reduced Gram; W = T^T V^T C of the look-ahead (transposed)
    double *borig, *rvec, *gvec, *mstat_d;   // mixed precision: original B, residual, A^T r, ||dx||
    int *mstat;                              // mixed precision: [first converged step, stagnation, run]
    unsigned long long *mask, *mask_all;
    int *pflag;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static size_t work_bytes(const Plan &p, Work *w, char *base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *ptr = base ? base + off : nullptr;
        off += align256(bytes);
        return ptr;
    };
    char *x = take(sizeof(double) * 2 * (size_t)p.nchunk * PW);
    char *pb = take(sizeof(double) * 2 * NB);
    char *wpart = take(sizeof(double) * (size_t)p.nsplit_max * NB * p.nxpad);
    char *T = take(sizeof(double) * NB * NB);
    char *wp = take(sizeof(double) * NB * (size_t)p.nxpad);
    char *wpart2 = take(sizeof(double) * (size_t)p.nsplit_max * NB * p.nxpad);
    char *T2 = take(sizeof(double) * NB * NB);
    char *wp2 = take(sizeof(double) * NB * (size_t)p.nxpad);
    char *fl = take(sizeof(int) * (size_t)std::max(p.nblk, 1));
    char *is = take(sizeof(int) * 64);
    char *gp = take(sizeof(double) * (size_t)p.ngroups * NB * NB);
    char *r1 = take(sizeof(double) * NB * NB);
    char *r1i = take(sizeof(double) * NB * NB);
    char *wi = take(sizeof(double) * NB * NB);
    char *mk = take(sizeof(unsigned long long) * (size_t)p.ngroups);
    char *pf = take(sizeof(int) * (size_t)std::max(p.npanels, 1));
    char *bo = take(sizeof(double) * (size_t)p.m * (size_t)std::max<int64_t>(p.nrhs, 1));
    char *rv = take(sizeof(double) * (size_t)std::max<int64_t>(p.m, 1));
    char *gv = take(sizeof(double) * (size_t)std::max<int64_t>(p.m, 1));
    char *msd = take(sizeof(double) * 64);
    char *ms = take(sizeof(int) * 64);
    char *q1 = take(sizeof(double) * NB * NB);
    char *gg = take(sizeof(double) * NB * NB);
    char *xn = take(sizeof(double) * NB * NB);
    char *ma = take(sizeof(unsigned long long));
    if (w) {
        w->q1top = (double *)q1;
        w->G = (double *)gg;
        w->xn = (double *)xn;
        w->borig = (double *)bo;
        w->rvec = (double *)rv;
        w->gvec = (double *)gv;
        w->mstat_d = (double *)msd;
        w->mstat = (int *)ms;
        w->mask_all = (unsigned long long *)ma;
        w->gpart = (double *)gp;
        w->r1 = (double *)r1;
        w->r1inv = (double *)r1i;
        w->winv = (double *)wi;
        w->mask = (unsigned long long *)mk;
        w->pflag = (int *)pf;
        w->xbuf = (double *)x;
        w->pbuf = (double *)pb;
        w->wpart = (double *)wpart;
        w->T = (double *)T;
        w->wp = (double *)wp;
        w->wpart2 = (double *)wpart2;
        w->T2 = (double *)T2;
        w->wp2 = (double *)wp2;
        w->flags = (int *)fl;
        w->iscratch = (int *)is;
    }
    return off;
}

static int pick_nsplit(int64_t rows, int ntiles, int nsplit_max)
{
    int want = (int)std::max<int64_t>(1, (512 + ntiles - 1) / std::max(ntiles, 1));
    int cap = (int)std::max<int64_t>(1, rows / 256);
    return std::max(1, std::min(std::min(want, cap), nsplit_max));
}

#define HQR_CK(call)                                   \
    do {                                               \
        if ((call) != hipSuccess) return HQR_EDEVICE;  \
    } while (0)

// Buffers one trailing update works in.
struct TrailBufs {
    double *wpart, *T, *wp;
};

// Apply the compact-WY block of panel (c0, bw) to trailing A columns
// [c0+bw+aoff, c0+bw+aoff+ncA) and all nB columns of B.  With have_t the
// panel's T is already in tb.T; otherwise it is formed from V^T V.
// With ev_first: the first `first_cols` A columns (at most 64) are updated by
// a launch of their own, ev_first is recorded on s after it, and the rest
// follows (ev_first is recorded at the end when there is nothing to split).
// vtx_wg_cap > 0 bounds the V^T C grid (fewer row splits), leaving CUs free
// for work on another stream.
static int apply_panel_block(const Plan &pl, const TrailBufs &tb, double *A, int64_t lda, double *B, int64_t ldb,
                             const double *up, int c0, int bw, int aoff, int ncA, int nB, bool have_t,
                             hipStream_t s, bool f32 = false, int first_cols = 0, hipEvent_t ev_first = nullptr,
                             int vtx_wg_cap = 0)
{
    const int64_t rows = pl.m - c0;
    VtxArgs v;
    v.A = A;
    v.lda = lda;
    v.B = B;
    v.ldb = ldb;
    v.up = up;
    v.m = pl.m;
    v.c0 = c0;
    v.bw = bw;
    v.ncA = ncA;
    v.nB = nB;
    v.aoff = aoff;
    v.with_v = have_t ? 0 : 1;
    const int vcols = have_t ? 0 : bw;
    v.nx = vcols + ncA + nB;
    v.nxpad = pl.nxpad;
    const int ntiles = (v.nx + VTX_COLS - 1) / VTX_COLS;
    // narrow updates (at most 64 columns, the next panel's on the critical
    // path): more row splits with a compact partial layout (row stride 128),
    // within the space the wide layout reserves
    const bool narrow = (ncA + nB) <= 64 && v.nx <= VTX_COLS;
    if (narrow) v.nxpad = VTX_COLS;
    const int nsplit = narrow ? std::max(1, std::min<int>((int)std::min<int64_t>(64, rows / 128),
                                                           pl.nsplit_max * pl.nxpad / VTX_COLS))
                              : pick_nsplit(rows, ntiles,
                                            vtx_wg_cap > 0 ? std::max(1, std::min(pl.nsplit_max, vtx_wg_cap / ntiles))
                                                           : pl.nsplit_max);
    v.split_rows = rup((rows + nsplit - 1) / nsplit, KC);
    const int nsplit_eff = (int)((rows + v.split_rows - 1) / v.split_rows);
    v.wpart = tb.wpart;
    const dim3 vg(ntiles, nsplit_eff);
    if (v.with_v) {
        if (f32)
            HQR_LAUNCH(K_VTX, (vtx_kernel<true, true>), vg, dim3(256), 0, s, v);
        else
            HQR_LAUNCH(K_VTX, (vtx_kernel<false, true>), vg, dim3(256), 0, s, v);
    } else {
        if (f32)
            HQR_LAUNCH(K_VTX, (vtx_kernel<true, false>), vg, dim3(256), 0, s, v);
        else
            HQR_LAUNCH(K_VTX, (vtx_kernel<false, false>), vg, dim3(256), 0, s, v);
    }
    HQR_CK(hipGetLastError());

    if (!have_t) {
        TArgs t;
        t.A = A;
        t.lda = lda;
        t.up = up;
        t.c0 = c0;
        t.bw = bw;
        t.wpart = tb.wpart;
        t.nsplit = nsplit_eff;
        t.nxpad = v.nxpad;
        t.T = tb.T;
        HQR_LAUNCH(K_TFACTOR, tfactor_kernel, dim3(1), dim3(256), 0, s, t);
        HQR_CK(hipGetLastError());
    }

    const int ncols = ncA + nB;
    if (ncols == 0) {
        if (ev_first) HQR_CK(hipEventRecord(ev_first, s));
        return 0;
    }
    WArgs wa;
    wa.wpart = tb.wpart;
    wa.nsplit = nsplit_eff;
    wa.nxpad = v.nxpad;
    wa.xoff = vcols;
    wa.ncols = ncols;
    wa.bw = bw;
    wa.T = tb.T;
    wa.wp = tb.wp;
    if (narrow)
        HQR_LAUNCH(K_WSOLVE, wsolve_narrow_kernel, dim3((ncols + WSN_COLS - 1) / WSN_COLS), dim3(256), 0, s, wa);
    else
        HQR_LAUNCH(K_WSOLVE, wsolve_kernel, dim3((ncols + WS_COLS - 1) / WS_COLS), dim3(256), 0, s, wa);
    HQR_CK(hipGetLastError());

    UpdArgs u;
    u.A = A;
    u.lda = lda;
    u.B = B;
    u.ldb = ldb;
    u.up = up;
    u.m = pl.m;
    u.c0 = c0;
    u.bw = bw;
    u.ncA = ncA;
    u.nB = nB;
    u.aoff = aoff;
    u.xoff = vcols;
    u.wp = tb.wp;
    u.nxpad = v.nxpad;
    const bool split = ev_first && !narrow && first_cols > 0 && first_cols <= NB && first_cols < ncA;
    if (split) {
        UpdArgs uf = u;
        uf.ncA = first_cols;
        uf.nB = 0;
        const dim3 ug((unsigned)((rows + 63) / 64));
        if (f32)
            HQR_LAUNCH(K_UPDATE, update_narrow_kernel<true>, ug, dim3(256), 0, s, uf);
        else
            HQR_LAUNCH(K_UPDATE, update_narrow_kernel<false>, ug, dim3(256), 0, s, uf);
        HQR_CK(hipGetLastError());
        HQR_CK(hipEventRecord(ev_first, s));
        u.ncA -= first_cols;
        u.aoff += first_cols;
        u.xoff += first_cols;
    }
    const int ncols_u = u.ncA + u.nB;
    if (narrow) {
        const dim3 ug((unsigned)((rows + 63) / 64));
        if (f32)
            HQR_LAUNCH(K_UPDATE, update_narrow_kernel<true>, ug, dim3(256), 0, s, u);
        else
            HQR_LAUNCH(K_UPDATE, update_narrow_kernel<false>, ug, dim3(256), 0, s, u);
    } else {
        const dim3 ug((unsigned)((rows + UPD_TILE - 1) / UPD_TILE), (ncols_u + UPD_TILE - 1) / UPD_TILE);
        if (f32)
            HQR_LAUNCH(K_UPDATE, update_kernel<true>, ug, dim3(256), 0, s, u);
        else
            HQR_LAUNCH(K_UPDATE, update_kernel<false>, ug, dim3(256), 0, s, u);
    }
    HQR_CK(hipGetLastError());
    if (ev_first && !split) HQR_CK(hipEventRecord(ev_first, s));
    return 0;
}

// Panel factorization by one launch per pivot (exact loop order).
static int panel_percol(const Plan &pl, const Work &w, double *A, int64_t lda, double *up, int c0, int bw,
                        hipStream_t s)
{
    PanelArgs pa;
    pa.A = A;
    pa.lda = lda;
    pa.m = pl.m;
    pa.c0 = c0;
    pa.bw = bw;
    pa.nchunk = (int)((pl.m - c0 + PC_ROWS - 1) / PC_ROWS);
    pa.up = up;
    pa.xbuf = w.xbuf;
    pa.pbuf = w.pbuf;
    for (int k = 0; k <= bw; ++k) {
        pa.k = k;
        HQR_LAUNCH(K_PANEL, panel_col_kernel, dim3(pa.nchunk), dim3(256), 0, s, pa);
        HQR_CK(hipGetLastError());
    }
    return 0;
}

// Sum of `parts` 64 x 64 partials in w.gpart into out (fixed order); with the
// pass-1 masks ORed into w.mask_all.  Skipped for a flagged panel when flag
// is given.
static int launch_gred(const Plan &, const Work &w, int parts, double *out, bool with_mask, const int *flag,
                       hipStream_t s)
{
    GredArgs gr;
    gr.gpart = w.gpart;
    gr.ngroups = parts;
    gr.G = out;
    gr.mask = w.mask;
    gr.mask_all = w.mask_all;
    gr.with_mask = with_mask ? 1 : 0;
    gr.flag = flag;
    HQR_LAUNCH(K_GRED, gram_reduce_kernel, dim3(NB * NB / 64), dim3(256), 0, s, gr);
    HQR_CK(hipGetLastError());
    return 0;
}

static int launch_chol(const Plan &pl, const Work &w, double *A, int64_t lda, double *up, int c0, int bw, int pidx,
                       int pass, double *Tout, hipStream_t s)
{
    CholArgs c;
    c.A = A;
    c.lda = lda;
    c.m = pl.m;
    c.c0 = c0;
    c.bw = bw;
    c.pass = pass;
    c.G = w.G;
    c.mask_all = w.mask_all;
    c.r1 = w.r1;
    c.r1inv = w.r1inv;
    c.q1top = w.q1top;
    c.winv = w.winv;
    c.T = Tout;
    c.up = up;
    c.flag = w.pflag + pidx;
    c.tstamp = nullptr;
    HQR_LAUNCH(K_CQR_CHOL, cqr_chol_kernel, dim3(1), dim3(256), 0, s, c);
    HQR_CK(hipGetLastError());
    return 0;
}

// Panel (c0, bw) by CholeskyQR2 + reconstruction, bottom rows not yet
// finished.  With upd, the previous panel (start cp, width NB; W = T^T V^T C
// transposed in w.xn) is first applied to this panel's columns.
static int panel_passes(const Plan &pl, const Work &w, double *A, int64_t lda, double *up, int c0, int bw, int pidx,
                        double *Tout, bool upd, int cp, hipStream_t s)
{
    const int64_t rbase = upd ? cp : c0;
    const int parts = (int)((pl.m - c0 + 63) / 64);
    int *flag = w.pflag + pidx;
    Gram1Args g;
    g.A = A;
    g.lda = lda;
    g.m = pl.m;
    g.c0 = c0;
    g.bw = bw;
    g.upd = upd ? 1 : 0;
    g.cp = cp;
    g.up = up;
    g.Wt = w.xn;
    g.gpart = w.gpart;
    g.mask = w.mask;
    g.flag = flag;
    HQR_LAUNCH(K_GRAM1, cqr_gram1_kernel, dim3((unsigned)((pl.m - rbase + 63) / 64)), dim3(256), 0, s, g);
    HQR_CK(hipGetLastError());
    int rc = launch_gred(pl, w, parts, w.G, true, flag, s);
    if (!rc) rc = launch_chol(pl, w, A, lda, up, c0, bw, pidx, 1, Tout, s);
    if (rc) return rc;
    Gram2Args g2;
    g2.A = A;
    g2.lda = lda;
    g2.m = pl.m;
    g2.c0 = c0;
    g2.bw = bw;
    g2.r1inv = w.r1inv;
    g2.q1top = w.q1top;
    g2.gpart = w.gpart;
    g2.flag = flag;
    HQR_LAUNCH(K_GRAM2, cqr_gram2_kernel, dim3((unsigned)parts), dim3(256), 0, s, g2);
    HQR_CK(hipGetLastError());
    rc = launch_gred(pl, w, parts, w.G, false, flag, s);
    if (!rc) rc = launch_chol(pl, w, A, lda, up, c0, bw, pidx, 2, Tout, s);
    return rc;
}

// Bottom rows of panel (c0, bw): V_bot = A_bot W^{-1} (nothing when flagged).
static int launch_finish(const Plan &pl, const Work &w, double *A, int64_t lda, int c0, int bw, int pidx,
                         hipStream_t s)
{
    const int64_t mp = pl.m - c0;
    if (mp <= bw) return 0;
    FinArgs f;
    f.A = A;
    f.lda = lda;
    f.m = pl.m;
    f.c0 = c0;
    f.bw = bw;
    f.winv = w.winv;
    f.flag = w.pflag + pidx;
    HQR_LAUNCH(K_CQR_FINISH, cqr_finish_kernel, dim3((unsigned)((mp - bw + 63) / 64)), dim3(256), 0, s, f);
    HQR_CK(hipGetLastError());
    return 0;
}

// Look-ahead: finish panel (c0, NB)'s V and write the partials of X = V^T C
// for the next panel's nc columns (summed into w.xn by launch_gred).
static int launch_narrow_vtx(const Plan &pl, const Work &w, double *A, int64_t lda, const double *up, int c0, int nc,
                             int pidx, hipStream_t s)
{
    NarrowArgs a;
    a.A = A;
    a.lda = lda;
    a.m = pl.m;
    a.c0 = c0;
    a.nc = nc;
    a.up = up;
    a.winv = w.winv;
    a.flag = w.pflag + pidx;
    a.gpart = w.gpart;
    const int parts = (int)((pl.m - c0 + 63) / 64);
    HQR_LAUNCH(K_NVTX, narrow_vtx_kernel, dim3((unsigned)parts), dim3(256), 0, s, a);
    HQR_CK(hipGetLastError());
    return 0;
}

// Panel factorization by CholeskyQR2 + Householder reconstruction (the exact
// loop when the device flags the panel), bottom rows finished.  Leaves T (for
// the stored vectors) in Tout.
static int panel_cqr(const Plan &pl, const Work &w, double *A, int64_t lda, double *up, int c0, int bw, int pidx,
                     double *Tout, hipStream_t s)
{
    int rc = panel_passes(pl, w, A, lda, up, c0, bw, pidx, Tout, false, 0, s);
    if (!rc) rc = launch_finish(pl, w, A, lda, c0, bw, pidx, s);
    return rc;
}

enum PanelMode { PANEL_CQR = 0, PANEL_PERCOL = 1, PANEL_EXACT = 2 };

static int panel_mode()
{
    const char *e = getenv("HQR_PANEL");
    if (!e) return PANEL_CQR;
    if (!strcmp(e, "percol")) return PANEL_PERCOL;
    if (!strcmp(e, "exact")) return PANEL_EXACT;
    return PANEL_CQR;
}

// Side stream and events for the look-ahead (one per device, created on first
// use, default priority).
struct SideStream {
    int device = -1;
    hipStream_t stream = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};
static SideStream g_side[16];

static SideStream *side_stream()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16) return nullptr;
    SideStream &ss = g_side[dev];
    if (ss.device != dev) {
        if (hipStreamCreateWithFlags(&ss.stream, hipStreamNonBlocking) != hipSuccess) return nullptr;
        // the events only order the two streams of one device: no timing and
        // no system-scope fence (kernel boundaries already release to the device)
        for (auto &e : ss.ev)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming | hipEventDisableSystemFence) != hipSuccess)
                return nullptr;
        ss.device = dev;
    }
    return &ss;
}

static bool lookahead_enabled()
{
    const char *e = getenv("HQR_LOOKAHEAD");
    return !(e && e[0] == '0');
}

// Blocked factorization; B (nB columns) rides along as trailing columns.
//
// With look-ahead (default), panel p+1 is factored on the caller's stream
// while the rest of panel p's trailing update runs on a side stream:
//   main: P(p) -> [a] -> N(p) (next panel's columns) -> P(p+1) -> wait r(p) -> N(p+1) -> ...
//   side: wait a -> R(p): V^T C and W for all later columns and B, the
//         update of panel p+2's columns -> [r(p)] -> the update of the rest
// r(p) marks all that N(p+1) reads, so N(p+1) and P(p+2) overlap the bulk
// of R(p)'s update.  N and R use separate W buffers; T alternates between
// two buffers by panel parity (P(p+2) is issued after main has waited for
// r(p), which follows R(p)'s last read of T).
static int factor_blocked(const Plan &pl, const Work &w, double *A, int64_t lda, double *up, double *B, int64_t ldb,
                          int nB, hipStream_t s)
{
    const int64_t n = pl.n;
    const int mode = panel_mode();
    const bool have_t = (mode != PANEL_PERCOL);
    if (have_t) {
        // exact-only mode: every panel flagged up front
        HQR_LAUNCH(K_FILL, fill_int_kernel, dim3(1), dim3(256), 0, s, w.pflag, mode == PANEL_EXACT ? 1 : 0,
                   (int64_t)pl.npanels);
        HQR_CK(hipGetLastError());
    }
    SideStream *ss = (lookahead_enabled() && pl.npanels > 1) ? side_stream() : nullptr;
    const TrailBufs bufN{w.wpart, nullptr, w.wp};
    const TrailBufs bufR{w.wpart2, nullptr, w.wp2};
    double *Tbuf[2] = {w.T, w.T2};
    auto do_panel = [&](int64_t c0, int bw, int pidx) -> int {
        if (mode == PANEL_PERCOL) return panel_percol(pl, w, A, lda, up, (int)c0, bw, s);
        return panel_cqr(pl, w, A, lda, up, (int)c0, bw, pidx, Tbuf[pidx & 1], s);
    };
    if (!ss) {
        for (int64_t c0 = 0; c0 < n; c0 += pl.nb) {
            const int bw = (int)std::min<int64_t>(pl.nb, n - c0);
            const int pidx = (int)(c0 / pl.nb);
            int rc = do_panel(c0, bw, pidx);
            if (rc) return rc;
            const int ncA = (int)(n - c0 - bw);
            TrailBufs b = bufN;
            b.T = Tbuf[pidx & 1];
            if (ncA + nB > 0) {
                rc = apply_panel_block(pl, b, A, lda, B, ldb, up, (int)c0, bw, 0, ncA, nB, have_t, s, pl.f32);
                if (rc) return rc;
            }
        }
        return 0;
    }
    hipEvent_t ev_a = ss->ev[0], ev_r = ss->ev[1], ev_join = ss->ev[2], ev_fork = ss->ev[3];
    // side stream starts after everything already on the caller's stream
    HQR_CK(hipEventRecord(ev_fork, s));
    HQR_CK(hipStreamWaitEvent(ss->stream, ev_fork, 0));
    bool pending_r = false;
    if (have_t && !pl.f32) {
        // Fused chain on the caller's stream, per panel p:
        //   [wait R(p-1)] -> narrow_vtx(p): V(p) finished, X = V^T C for the
        //   next panel's columns (or finish(p) for the last panel) -> [a] ->
        //   passes of panel p+1, the first applying N(p) = (V, T^T X)
        // side: wait a -> R(p) (all later columns and B) -> [r(p)]
        const int bw0 = (int)std::min<int64_t>(pl.nb, n);
        int rc = panel_passes(pl, w, A, lda, up, 0, bw0, 0, Tbuf[0], false, 0, s);
        if (rc) return rc;
        for (int64_t c0 = 0; c0 < n; c0 += pl.nb) {
            const int bw = (int)std::min<int64_t>(pl.nb, n - c0);
            const int pidx = (int)(c0 / pl.nb);
            const int64_t c1 = c0 + bw;
            const int bw1 = (int)std::min<int64_t>(pl.nb, std::max<int64_t>(0, n - c1));
            const int ncR = (int)std::max<int64_t>(0, n - c1 - bw1);
            TrailBufs br = bufR;
            br.T = Tbuf[pidx & 1];
            if (pending_r) HQR_CK(hipStreamWaitEvent(s, ev_r, 0));
            rc = (bw1 > 0) ? launch_narrow_vtx(pl, w, A, lda, up, (int)c0, bw1, pidx, s)
                           : launch_finish(pl, w, A, lda, (int)c0, bw, pidx, s);
            if (rc) return rc;
            HQR_CK(hipEventRecord(ev_a, s));
            HQR_CK(hipStreamWaitEvent(ss->stream, ev_a, 0));
            // R(p): the columns of panel p+2 first, then r(p) (all that
            // narrow_vtx(p+1) reads), then the rest of the columns and B
            if (ncR + nB > 0) {
                // late panels, where the main chain is the longer one: V^T C
                // on at most half the CUs so the chain's kernels find free ones
                rc = apply_panel_block(pl, br, A, lda, B, ldb, up, (int)c0, bw, bw1, ncR, nB, true, ss->stream, false,
                                       std::min(ncR, (int)pl.nb), ev_r, (ncR + nB <= 2048) ? 128 : 0);
                if (rc) return rc;
            } else {
                HQR_CK(hipEventRecord(ev_r, ss->stream));
            }
            if (bw1 > 0) {
                XwArgs xa;
                xa.gpart = w.gpart;
                xa.parts = (int)((pl.m - c0 + 63) / 64);
                xa.T = Tbuf[pidx & 1];
                xa.Wt = w.xn;
                HQR_LAUNCH(K_GRED, xw_reduce_kernel, dim3(NB), dim3(256), 0, s, xa);
                HQR_CK(hipGetLastError());
                if (!rc)
                    rc = panel_passes(pl, w, A, lda, up, (int)c1, bw1, pidx + 1, Tbuf[(pidx + 1) & 1], true, (int)c0,
                                      s);
                if (rc) return rc;
            }
            pending_r = true;
        }
        HQR_CK(hipEventRecord(ev_join, ss->stream));
        HQR_CK(hipStreamWaitEvent(s, ev_join, 0));
        return 0;
    }
    int rc = do_panel(0, (int)std::min<int64_t>(pl.nb, n), 0);
    if (rc) return rc;
    for (int64_t c0 = 0; c0 < n; c0 += pl.nb) {
        const int bw = (int)std::min<int64_t>(pl.nb, n - c0);
        const int pidx = (int)(c0 / pl.nb);
        const int64_t c1 = c0 + bw;                       // next panel
        const int bw1 = (int)std::min<int64_t>(pl.nb, std::max<int64_t>(0, n - c1));
        const int ncR = (int)std::max<int64_t>(0, n - c1 - bw1);
        TrailBufs bn = bufN, br = bufR;
        bn.T = br.T = Tbuf[pidx & 1];
        // main: wait for r(p-1) (R(p-1) has updated the next panel's
        // columns); issued before R(p) re-records ev_r
        if (pending_r) HQR_CK(hipStreamWaitEvent(s, ev_r, 0));
        // R(p) on the side stream: columns beyond the next panel, and B; the
        // columns of panel p+2 first, then r(p), then the rest and B
        HQR_CK(hipEventRecord(ev_a, s));
        HQR_CK(hipStreamWaitEvent(ss->stream, ev_a, 0));
        if (ncR + nB > 0) {
            rc = apply_panel_block(pl, br, A, lda, B, ldb, up, (int)c0, bw, bw1, ncR, nB, have_t, ss->stream, pl.f32,
                                   std::min(ncR, (int)pl.nb), ev_r);
            if (rc) return rc;
        } else {
            HQR_CK(hipEventRecord(ev_r, ss->stream));
        }
        // main: N(p), then P(p+1)
        if (bw1 > 0) {
            rc = apply_panel_block(pl, bn, A, lda, B, ldb, up, (int)c0, bw, 0, bw1, 0, have_t, s, pl.f32);
            if (rc) return rc;
            rc = do_panel(c1, bw1, pidx + 1);
            if (rc) return rc;
        }
        pending_r = true;
    }
    // join: the caller's stream waits for the last side-stream work
    HQR_CK(hipEventRecord(ev_join, ss->stream));
    HQR_CK(hipStreamWaitEvent(s, ev_join, 0));
    return 0;
}

static int backsolve_blocked(const Plan &pl, const Work &w, const double *A, int64_t lda, double *B, int64_t ldb,
                             int nrhs, int *info, hipStream_t s, bool trans = false)
{
    HQR_LAUNCH(K_DIAG, diag_check_kernel, dim3(1), dim3(256), 0, s, A, lda, pl.n, info);
    HQR_CK(hipGetLastError());
    for (int c = 0; c < nrhs; c += TRSV_MAXRHS) {
        HQR_LAUNCH(K_FILL, fill_int_kernel, dim3(1), dim3(256), 0, s, w.flags, 0, (int64_t)pl.nblk);
        HQR_CK(hipGetLastError());
        TrsvArgs t;
        t.A = A;
        t.lda = lda;
        t.B = B + (size_t)c * ldb;
        t.ldb = ldb;
        t.n = pl.n;
        t.nrhs = std::min(TRSV_MAXRHS, nrhs - c);
        t.flags = w.flags;
        t.info = info;
        t.epoch = 1;
        t.spin_limit = 20000000L;
        if (t.nrhs == 1) {
            if (trans)
                HQR_LAUNCH(K_TRSV, (trsv_kernel<true, 1>), dim3(pl.nblk), dim3(256), 0, s, t);
            else
                HQR_LAUNCH(K_TRSV, (trsv_kernel<false, 1>), dim3(pl.nblk), dim3(256), 0, s, t);
        } else {
            if (trans)
                HQR_LAUNCH(K_TRSV, (trsv_kernel<true, TRSV_MAXRHS>), dim3(pl.nblk), dim3(256), 0, s, t);
            else
                HQR_LAUNCH(K_TRSV, (trsv_kernel<false, TRSV_MAXRHS>), dim3(pl.nblk), dim3(256), 0, s, t);
        }
        HQR_CK(hipGetLastError());
    }
    return 0;
}

struct WorkGuard {
    void *ptr = nullptr;
    hipStream_t s = nullptr;
    ~WorkGuard()
    {
        if (ptr) (void)hipFreeAsync(ptr, s);
    }
};

static int get_work(const Plan &pl, void *work, int64_t lwork, hipStream_t s, WorkGuard &g, Work *w)
{
    const size_t need = work_bytes(pl, nullptr, nullptr);
    char *base = (char *)work;
    if (!base) {
        if (hipMallocAsync((void **)&base, need, s) != hipSuccess) return HQR_ENOMEM;
        g.ptr = base;
        g.s = s;
    } else if (lwork < (int64_t)need) {
        return HQR_ENOMEM;
    }
    work_bytes(pl, w, base);
    return 0;
}

// The FP64 path: small problems in one register-resident workgroup, larger
// ones by the blocked factorization, then residual norms and back-substitution.
static int lsq_fp64(int64_t m, int64_t n, int64_t nrhs, double *A, int64_t lda, double *up, double *B, int64_t ldb,
                    double *resnorm, void *work, int64_t lwork, int *info, hipStream_t s)
{
    if (n == 0) {
        HQR_LAUNCH(K_FILL, fill_int_kernel, dim3(1), dim3(64), 0, s, info, 0, (int64_t)1);
        HQR_CK(hipGetLastError());
        if (resnorm && nrhs > 0) {
            HQR_LAUNCH(K_RESNORM, resnorm_kernel, dim3((unsigned)nrhs), dim3(256), 0, s, (const double *)B, ldb,
                       (int64_t)0, m, resnorm);
            HQR_CK(hipGetLastError());
        }
        return 0;
    }
    if (const WgVariant *v = pick_wg_single(m, n, nrhs)) {
        if (nrhs == 0) {
            HQR_LAUNCH(K_FILL, fill_int_kernel, dim3(1), dim3(64), 0, s, info, 0, (int64_t)1);
            HQR_CK(hipGetLastError());
        }
        const WgDesc d{m, n, nrhs, lda, ldb, A, B, up, resnorm, 0, WG_FACTOR | (nrhs > 0 ? WG_SOLVE : 0)};
        return launch_wg_single(v, d, info, s);
    }
    Plan pl = make_plan(m, n, nrhs);
    WorkGuard g;
    Work w;
    int rc = get_work(pl, work, lwork, s, g, &w);
    if (rc) return rc;
    HQR_LAUNCH(K_FILL, fill_int_kernel, dim3(1), dim3(64), 0, s, info, 0, (int64_t)1);
    HQR_CK(hipGetLastError());
    rc = factor_blocked(pl, w, A, lda, up, B, ldb, (int)nrhs, s);
    if (rc) return rc;
    if (nrhs == 0) return 0;
    if (resnorm) {
        HQR_LAUNCH(K_RESNORM, resnorm_kernel, dim3((unsigned)nrhs), dim3(256), 0, s, (const double *)B, ldb, n, m,
                   resnorm);
        HQR_CK(hipGetLastError());
    }
    return backsolve_blocked(pl, w, A, lda, B, ldb, (int)nrhs, info, s);
}

// Mixed precision: FP32 trailing contractions in the factorization, then
// corrections of the semi-normal equations with FP64 residuals:
//   r = b - A0 x,  g = A0^T r,  R^T z = g,  R dx = z,  x += dx
// (A0 = the unmodified FP64 matrix, R = the factor's triangle).  A run of
// max_iter steps is enqueued; the stream is synchronized once at the end to
// read the convergence record and, without convergence, the FP64 path is
// run on the restored inputs (info gets HQR_INFO_NOCONV).
// Corrections of the semi-normal equations for every right-hand side:
// x (in B[0:n]) += dx until converged (see csne_update_kernel), with FP64
// residuals of A0 against the original right-hand sides in w.borig and
// triangular solves with R (upper triangle of A).  Reports the largest
// first-converged step and whether every column converged.
static int mixed_refine(const Plan &pl, const Work &w, const double *A, int64_t lda, double *B, int64_t ldb,
                        int64_t nrhs, double *resnorm, double tol, int max_iter, const double *A0, int64_t lda0,
                        hipStream_t s, int *first, bool *converged)
{
    const int64_t m = pl.m, n = pl.n;
    *first = 0;
    *converged = true;
    for (int64_t c = 0; c < nrhs; ++c) {
        double *x = B + (size_t)c * ldb;
        const double *b0 = w.borig + (size_t)c * m;
        HQR_LAUNCH(K_FILL, fill_int_kernel, dim3(1), dim3(64), 0, s, w.mstat, 0, (int64_t)4);
        HQR_CK(hipGetLastError());
        for (int it = 0; it < max_iter; ++it) {
            HQR_LAUNCH(K_REFINE, resid_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, A0, lda0, b0,
                       (const double *)x, w.rvec, m, n);
            HQR_LAUNCH(K_REFINE, gemvt_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, A0, lda0,
                       (const double *)w.rvec, w.gvec, m, n);
            HQR_CK(hipGetLastError());
            int rc = backsolve_blocked(pl, w, A, lda, w.gvec, std::max<int64_t>(n, 1), 1, w.iscratch, s, true);
            if (rc) return rc;
            rc = backsolve_blocked(pl, w, A, lda, w.gvec, std::max<int64_t>(n, 1), 1, w.iscratch, s, false);
            if (rc) return rc;
            HQR_LAUNCH(K_REFINE, csne_update_kernel, dim3(1), dim3(1024), 0, s, x, (const double *)w.gvec, n, tol,
                       it, w.mstat, w.mstat_d);
            HQR_CK(hipGetLastError());
        }
        if (resnorm) {
            HQR_LAUNCH(K_REFINE, resid_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, A0, lda0, b0,
                       (const double *)x, w.rvec, m, n);
            HQR_LAUNCH(K_RESNORM, resnorm_kernel, dim3(1), dim3(256), 0, s, (const double *)w.rvec,
                       std::max<int64_t>(m, 1), (int64_t)0, m, resnorm + c);
            HQR_CK(hipGetLastError());
        }
        int st[4] = {0, 0, 0, 0};
        HQR_CK(hipMemcpyAsync(st, w.mstat, sizeof(st), hipMemcpyDeviceToHost, s));
        HQR_CK(hipStreamSynchronize(s));
        if (st[0] == 0 || st[1]) *converged = false;
        *first = std::max(*first, st[0]);
    }
    return 0;
}

static int write_iters(int *iters, int v, hipStream_t s)
{
    if (!iters) return 0;
    HQR_CK(hipMemcpyAsync(iters, &v, sizeof(int), hipMemcpyHostToDevice, s));
    HQR_CK(hipStreamSynchronize(s));
    return 0;
}

// Mixed precision: FP32 trailing contractions in the factorization, then
// corrections of the semi-normal equations with FP64 residuals:
//   r = b - A0 x,  g = A0^T r,  R^T z = g,  R dx = z,  x += dx
// (A0 = the unmodified FP64 matrix, R = the factor's triangle).  A run of
// max_iter steps is enqueued; the stream is synchronized once per right-hand
// side to read the convergence record and, without convergence, the FP64
// path is run on the restored inputs (info gets HQR_INFO_NOCONV).
static int lsq_mixed(int64_t m, int64_t n, int64_t nrhs, double *A, int64_t lda, double *up, double *B,
                     int64_t ldb, double *resnorm, const hqr_opts *opt, const double *A0, int64_t lda0, void *work,
                     int64_t lwork, int *info, int *iters, hipStream_t s)
{
    const double tol = (opt && opt->tol > 0.0) ? opt->tol : 1e-13;
    const int max_iter = (opt && opt->max_iter >= 0) ? opt->max_iter : 10;
    const int nb = (n <= 256) ? 16 : NB;
    Plan pl = make_plan(m, n, nrhs, nb, true);
    WorkGuard g;
    Work w;
    int rc = get_work(pl, work, lwork, s, g, &w);
    if (rc) return rc;
    HQR_CK(hipMemcpy2DAsync(w.borig, sizeof(double) * m, B, sizeof(double) * ldb, sizeof(double) * m, nrhs,
                            hipMemcpyDeviceToDevice, s));
    HQR_LAUNCH(K_FILL, fill_int_kernel, dim3(1), dim3(64), 0, s, info, 0, (int64_t)1);
    HQR_CK(hipGetLastError());
    rc = factor_blocked(pl, w, A, lda, up, B, ldb, (int)nrhs, s);
    if (rc) return rc;
    rc = backsolve_blocked(pl, w, A, lda, B, ldb, (int)nrhs, info, s);
    if (rc) return rc;
    int first = 0;
    bool converged = true;
    rc = mixed_refine(pl, w, A, lda, B, ldb, nrhs, resnorm, tol, max_iter, A0, lda0, s, &first, &converged);
    if (rc) return rc;
    int hinfo = 0;
    HQR_CK(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, s));
    HQR_CK(hipStreamSynchronize(s));
    if (!converged && hinfo == 0) {
        // FP64 fallback on the restored inputs: the same call as precision FP64
        HQR_CK(hipMemcpy2DAsync(A, sizeof(double) * lda, A0, sizeof(double) * lda0, sizeof(double) * m, n,
                                hipMemcpyDeviceToDevice, s));
        HQR_CK(hipMemcpy2DAsync(B, sizeof(double) * ldb, w.borig, sizeof(double) * m, sizeof(double) * m, nrhs,
                                hipMemcpyDeviceToDevice, s));
        rc = lsq_fp64(m, n, nrhs, A, lda, up, B, ldb, resnorm, nullptr, 0, info, s);
        if (rc) return rc;
        hinfo = HQR_INFO_NOCONV;
        HQR_CK(hipMemcpyAsync(info, &hinfo, sizeof(int), hipMemcpyHostToDevice, s));
        first = max_iter;
        HQR_CK(hipStreamSynchronize(s));
    }
    return write_iters(iters, first, s);
}

} // namespace hqr

using namespace hqr;


// ------------------------------------------------------------ batched path
namespace hqr {

// Pinned staging buffer for the descriptor upload; `ready` fences reuse.
struct Staging {
    void *host = nullptr;
    size_t bytes = 0;
    hipEvent_t ready = nullptr;
};
static Staging g_stage;

static int stage_upload(const void *src, size_t bytes, void *dst, hipStream_t s)
{
    if (g_stage.ready) HQR_CK(hipEventSynchronize(g_stage.ready));
    if (g_stage.bytes < bytes) {
        if (g_stage.host) (void)hipHostFree(g_stage.host);
        g_stage.host = nullptr;
        g_stage.bytes = 0;
        if (hipHostMalloc(&g_stage.host, bytes, hipHostMallocDefault) != hipSuccess) return HQR_ENOMEM;
        g_stage.bytes = bytes;
    }
    if (!g_stage.ready) HQR_CK(hipEventCreateWithFlags(&g_stage.ready, hipEventDisableTiming));
    memcpy(g_stage.host, src, bytes);
    HQR_CK(hipMemcpyAsync(dst, g_stage.host, bytes, hipMemcpyHostToDevice, s));
    HQR_CK(hipEventRecord(g_stage.ready, s));
    return 0;
}

static int num_cus()
{
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 256;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    }
    return cus;
}

} // namespace hqr

extern "C" int64_t hqr_batched_workspace_size(int count)
{
    if (count < 0) return -1;
    return (int64_t)(align256(sizeof(BatchDesc) * (size_t)std::max(count, 1)) + 256);
}

static int lsq_batched_impl(int count, const int64_t *m, const int64_t *n, const int64_t *nrhs, double *const *A,
                            const int64_t *lda, double *const *up, double *const *B, const int64_t *ldb,
                            double *const *resnorm, const int *factored, int *info, void *work, int64_t lwork,
                            hipStream_t stream)
{
    if (count < 0) return -1;
    if (count == 0) return 0;
    if (!m) return -2;
    if (!n) return -3;
    if (!nrhs) return -4;
    if (!A) return -5;
    if (!lda) return -6;
    if (!up) return -7;
    if (!B) return -8;
    if (!ldb) return -9;
    if (!info) return -11;
    std::vector<BatchDesc> d((size_t)count);
    std::vector<double> cost((size_t)count);
    int max_ntot = 0;
    for (int i = 0; i < count; ++i) {
        if (m[i] < 0 || m[i] > BATCH_MAX_ROWS) return -2;
        if (n[i] < 0 || n[i] > m[i]) return -3;
        if (nrhs[i] < 0 || n[i] + nrhs[i] > BATCH_MAX_COLS) return -4;
        if (lda[i] < std::max<int64_t>(1, m[i])) return -6;
        if (ldb[i] < std::max<int64_t>(1, m[i])) return -9;
        if (n[i] > 0 && (!A[i] || !up[i])) return -5;
        if (nrhs[i] > 0 && !B[i]) return -8;
        d[i] = BatchDesc{m[i], n[i], nrhs[i], lda[i], ldb[i], A[i], B[i], up[i], resnorm ? resnorm[i] : nullptr, i,
                         (factored && factored[i]) ? 0 : 1};
        const double mm = (double)m[i], nn = (double)n[i];
        cost[i] = 2.0 * mm * nn * nn - 2.0 / 3.0 * nn * nn * nn + 4.0 * mm * nn * (double)nrhs[i] + mm;
        max_ntot = std::max<int>(max_ntot, (int)(n[i] + nrhs[i]));
    }
    // The one-workgroup blocked kernel takes every instance the chosen variant
    // holds; the rest (more rows, or n * nrhs beyond its staging area) go to
    // the streaming kernel in a second launch.  Each group runs longest
    // first; ties keep caller order, so the order depends on shapes only.
    std::vector<char> fits((size_t)count);
    int64_t mmax = 0, nmax = 0;
    for (int i = 0; i < count; ++i) {
        fits[i] = batch_wg_fits(m[i], n[i], nrhs[i]) ? 1 : 0;
        if (fits[i]) {
            mmax = std::max(mmax, m[i]);
            nmax = std::max(nmax, n[i]);
        }
    }
    const WgVariant *var = pick_wg_batched(mmax, nmax);
    std::vector<int> order((size_t)count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (fits[a] != fits[b]) return fits[a] > fits[b];
        return cost[a] > cost[b];
    });
    int nwg = 0;
    while (nwg < count && fits[order[nwg]]) ++nwg;
    std::vector<BatchDesc> sorted((size_t)count);
    for (int i = 0; i < count; ++i) sorted[i] = d[order[i]];
    static_assert(sizeof(WgDesc) == sizeof(BatchDesc), "descriptor layouts share the staging buffer");
    std::vector<WgDesc> wsorted((size_t)nwg);
    for (int i = 0; i < nwg; ++i) {
        const BatchDesc &b = sorted[i];
        wsorted[i] = WgDesc{b.m, b.n, b.nrhs, b.lda, b.ldb, b.A, b.B, b.up, b.resnorm, b.index,
                            (b.factor ? WG_FACTOR : 0) | WG_SOLVE};
    }

    const size_t need = (size_t)hqr_batched_workspace_size(count);
    WorkGuard g;
    char *base = (char *)work;
    if (!base) {
        if (hipMallocAsync((void **)&base, need, stream) != hipSuccess) return HQR_ENOMEM;
        g.ptr = base;
        g.s = stream;
    } else if (lwork < (int64_t)need) {
        return HQR_ENOMEM;
    }
    char *dbase = base;
    int *head = (int *)(base + align256(sizeof(BatchDesc) * (size_t)count));
    // one host image: WgDesc entries, then BatchDesc entries
    std::vector<char> img(sizeof(BatchDesc) * (size_t)count);
    memcpy(img.data(), wsorted.data(), sizeof(WgDesc) * (size_t)nwg);
    memcpy(img.data() + sizeof(WgDesc) * (size_t)nwg, sorted.data() + nwg, sizeof(BatchDesc) * (size_t)(count - nwg));
    int rc = stage_upload(img.data(), img.size(), dbase, stream);
    if (rc) return rc;
    HQR_LAUNCH(K_FILL, fill_int_kernel, dim3(1), dim3(64), 0, stream, head, 0, (int64_t)2);
    HQR_CK(hipGetLastError());
    if (nwg > 0) {
        const int grid = std::min(nwg, var->per_cu * num_cus());
        HQR_LAUNCH(K_BATCHED, var->batched, dim3(grid), dim3(var->nt), 0, stream, (const WgDesc *)dbase, nwg, head,
                   info);
        HQR_CK(hipGetLastError());
    }
    if (nwg < count) {
        BatchArgs a;
        a.desc = (const BatchDesc *)(dbase + sizeof(WgDesc) * (size_t)nwg);
        a.count = count - nwg;
        a.head = head + 1;
        a.info = info;
        a.max_ntot = max_ntot;
        const int grid = std::min(count - nwg, 2 * num_cus());
        HQR_LAUNCH(K_BATCHED, batched_lsq_kernel, dim3(grid), dim3(1024), 0, stream, a);
        HQR_CK(hipGetLastError());
    }
    return 0;
}

extern "C" int qr_lsq_solve_batched(int count, const int64_t *m, const int64_t *n, const int64_t *nrhs,
                                    double *const *A, const int64_t *lda, double *const *up, double *const *B,
                                    const int64_t *ldb, double *const *resnorm, int *info, void *work,
                                    int64_t lwork, hipStream_t stream)
{
    return lsq_batched_impl(count, m, n, nrhs, A, lda, up, B, ldb, resnorm, nullptr, info, work, lwork, stream);
}

extern "C" int qr_lsq_batched_mixed(int count, const int64_t *m, const int64_t *n, const int64_t *nrhs,
                                    double *const *A, const int64_t *lda, double *const *up, double *const *B,
                                    const int64_t *ldb, double *const *resnorm, const int *factored, int *info,
                                    void *work, int64_t lwork, hipStream_t stream)
{
    if (!factored) return -11;
    return lsq_batched_impl(count, m, n, nrhs, A, lda, up, B, ldb, resnorm, factored, info, work, lwork, stream);
}

extern "C" {

int64_t hqr_workspace_size(int64_t m, int64_t n, int64_t nrhs, int precision)
{
    if (m < 0) return -1;
    if (n < 0 || n > m) return -2;
    if (nrhs < 0) return -3;
    if (precision != HQR_PREC_FP64 && precision != HQR_PREC_MIXED) return -4;
    Plan pl = (precision == HQR_PREC_MIXED) ? make_plan(m, n, nrhs, (n <= 256) ? 16 : NB, true) : make_plan(m, n, nrhs);
    return (int64_t)work_bytes(pl, nullptr, nullptr);
}

int qr_factor(int64_t m, int64_t n, double *A, int64_t lda, double *up, void *work, int64_t lwork, int *info,
              hipStream_t stream)
{
    if (m < 0) return -1;
    if (n < 0 || n > m) return -2;
    if (lda < std::max<int64_t>(1, m)) return -4;
    if (!info) return -8;
    if (n > 0 && !A) return -3;
    if (n > 0 && !up) return -5;
    if (m > INT32_MAX / 2 || n > INT32_MAX / 2) return HQR_ENOTSUP;
    if (n == 0) {
        HQR_LAUNCH(K_FILL, fill_int_kernel, dim3(1), dim3(64), 0, stream, info, 0, (int64_t)1);
        return hipGetLastError() == hipSuccess ? 0 : HQR_EDEVICE;
    }
    if (const WgVariant *v = pick_wg_single(m, n, 0)) {
        HQR_LAUNCH(K_FILL, fill_int_kernel, dim3(1), dim3(64), 0, stream, info, 0, (int64_t)1);
        HQR_CK(hipGetLastError());
        const WgDesc d{m, n, 0, lda, std::max<int64_t>(1, m), A, nullptr, up, nullptr, 0, WG_FACTOR};
        return launch_wg_single(v, d, info, stream);
    }
    Plan pl = make_plan(m, n, 0);
    WorkGuard g;
    Work w;
    int rc = get_work(pl, work, lwork, stream, g, &w);
    if (rc) return rc;
    HQR_LAUNCH(K_FILL, fill_int_kernel, dim3(1), dim3(64), 0, stream, info, 0, (int64_t)1);
    HQR_CK(hipGetLastError());
    return factor_blocked(pl, w, A, lda, up, nullptr, 1, 0, stream);
}

int qr_apply_qt(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *up, double *B,
                int64_t ldb, void *work, int64_t lwork, hipStream_t stream)
{
    if (m < 0) return -1;
    if (n < 0 || n > m) return -2;
    if (nrhs < 0) return -3;
    if (lda < std::max<int64_t>(1, m)) return -5;
    if (ldb < std::max<int64_t>(1, m)) return -8;
    if (n == 0 || nrhs == 0) return 0;
    if (!A) return -4;
    if (!up) return -6;
    if (!B) return -7;
    if (m > INT32_MAX / 2 || n > INT32_MAX / 2 || nrhs > INT32_MAX / 4) return HQR_ENOTSUP;
    if (const WgVariant *v = pick_wg_single(m, n, nrhs)) {
        const WgDesc d{m, n, nrhs, lda, ldb, const_cast<double *>(A), B, const_cast<double *>(up), nullptr, 0, 0};
        return launch_wg_single(v, d, nullptr, stream);
    }
    Plan pl = make_plan(m, n, nrhs);
    WorkGuard g;
    Work w;
    int rc = get_work(pl, work, lwork, stream, g, &w);
    if (rc) return rc;
    for (int64_t c0 = 0; c0 < n; c0 += NB) {
        const int bw = (int)std::min<int64_t>(NB, n - c0);
        rc = apply_panel_block(pl, TrailBufs{w.wpart, w.T, w.wp}, const_cast<double *>(A), lda, B, ldb, up, (int)c0, bw, 0, 0, (int)nrhs, false, stream);
        if (rc) return rc;
    }
    return 0;
}

int qr_backsolve(int64_t n, int64_t nrhs, const double *A, int64_t lda, double *B, int64_t ldb, int *info,
                 hipStream_t stream)
{
    if (n < 0) return -1;
    if (nrhs < 0) return -2;
    if (lda < std::max<int64_t>(1, n)) return -4;
    if (ldb < std::max<int64_t>(1, n)) return -6;
    if (!info) return -7;
    if (n > 0 && nrhs > 0) {
        if (!A) return -3;
        if (!B) return -5;
    }
    if (n > INT32_MAX / 2) return HQR_ENOTSUP;
    if (n == 0 || nrhs == 0) {
        HQR_LAUNCH(K_FILL, fill_int_kernel, dim3(1), dim3(64), 0, stream, info, 0, (int64_t)1);
        return hipGetLastError() == hipSuccess ? 0 : HQR_EDEVICE;
    }
    Plan pl = make_plan(n, n, nrhs);
    WorkGuard g;
    Work w;
    int rc = get_work(pl, nullptr, 0, stream, g, &w);
    if (rc) return rc;
    return backsolve_blocked(pl, w, A, lda, B, ldb, (int)nrhs, info, stream);
}

int qr_lsq_solve(int64_t m, int64_t n, int64_t nrhs, double *A, int64_t lda, double *up, double *B, int64_t ldb,
                 double *resnorm, const hqr_opts *opt, const double *A_orig, int64_t lda_orig, void *work,
                 int64_t lwork, int *info, int *iters, hipStream_t stream)
{
    if (m < 0) return -1;
    if (n < 0 || n > m) return -2;
    if (nrhs < 0) return -3;
    if (lda < std::max<int64_t>(1, m)) return -5;
    if (ldb < std::max<int64_t>(1, m)) return -8;
    if (!info) return -15;
    const int prec = opt ? opt->precision : HQR_PREC_FP64;
    if (prec != HQR_PREC_FP64 && prec != HQR_PREC_MIXED) return -10;
    if (n > 0) {
        if (!A) return -4;
        if (!up) return -6;
    }
    if (nrhs > 0 && !B) return -7;
    if (prec == HQR_PREC_MIXED) {
        if (!A_orig) return -11;
        if (lda_orig < std::max<int64_t>(1, m)) return -12;
        if (m > INT32_MAX / 2 || n > INT32_MAX / 2 || nrhs > INT32_MAX / 4) return HQR_ENOTSUP;
        if (iters) {
            HQR_LAUNCH(K_FILL, fill_int_kernel, dim3(1), dim3(64), 0, stream, iters, 0, (int64_t)1);
            HQR_CK(hipGetLastError());
        }
        if (n == 0 || nrhs == 0) {
            HQR_LAUNCH(K_FILL, fill_int_kernel, dim3(1), dim3(64), 0, stream, info, 0, (int64_t)1);
            return hipGetLastError() == hipSuccess ? 0 : HQR_EDEVICE;
        }
        return lsq_mixed(m, n, nrhs, A, lda, up, B, ldb, resnorm, opt, A_orig, lda_orig, work, lwork, info, iters,
                         stream);
    }
    (void)A_orig;
    (void)lda_orig;
    if (m > INT32_MAX / 2 || n > INT32_MAX / 2 || nrhs > INT32_MAX / 4) return HQR_ENOTSUP;
    if (iters) {
        HQR_LAUNCH(K_FILL, fill_int_kernel, dim3(1), dim3(64), 0, stream, iters, 0, (int64_t)1);
        HQR_CK(hipGetLastError());
    }
    return lsq_fp64(m, n, nrhs, A, lda, up, B, ldb, resnorm, work, lwork, info, stream);
}

int qr_lsq_refine(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *up, double *B,
                  int64_t ldb, double *resnorm, const hqr_opts *opt, const double *A_orig, int64_t lda_orig,
                  void *work, int64_t lwork, int *info, int *iters, hipStream_t stream)
{
    if (m < 0) return -1;
    if (n < 0 || n > m) return -2;
    if (nrhs < 0) return -3;
    if (lda < std::max<int64_t>(1, m)) return -5;
    if (ldb < std::max<int64_t>(1, m)) return -8;
    if (!info) return -15;
    if (n > 0 && !A) return -4;
    if (n > 0 && !up) return -6;
    if (nrhs > 0 && !B) return -7;
    if (n > 0 && !A_orig) return -11;
    if (lda_orig < std::max<int64_t>(1, m)) return -12;
    if (m > INT32_MAX / 2 || n > INT32_MAX / 2 || nrhs > INT32_MAX / 4) return HQR_ENOTSUP;
    HQR_LAUNCH(K_FILL, fill_int_kernel, dim3(1), dim3(64), 0, stream, info, 0, (int64_t)1);
    HQR_CK(hipGetLastError());
    if (iters) {
        HQR_LAUNCH(K_FILL, fill_int_kernel, dim3(1), dim3(64), 0, stream, iters, 0, (int64_t)1);
        HQR_CK(hipGetLastError());
    }
    if (n == 0 || nrhs == 0) return 0;
    const double tol = (opt && opt->tol > 0.0) ? opt->tol : 1e-13;
    const int max_iter = (opt && opt->max_iter >= 0) ? opt->max_iter : 10;
    Plan pl = make_plan(m, n, nrhs, NB, true);
    WorkGuard g;
    Work w;
    int rc = get_work(pl, work, lwork, stream, g, &w);
    if (rc) return rc;
    HQR_CK(hipMemcpy2DAsync(w.borig, sizeof(double) * m, B, sizeof(double) * ldb, sizeof(double) * m, nrhs,
                            hipMemcpyDeviceToDevice, stream));
    rc = qr_apply_qt(m, n, nrhs, A, lda, up, B, ldb, nullptr, 0, stream);
    if (rc) return rc;
    rc = backsolve_blocked(pl, w, A, lda, B, ldb, (int)nrhs, info, stream);
    if (rc) return rc;
    int first = 0;
    bool converged = true;
    rc = mixed_refine(pl, w, A, lda, B, ldb, nrhs, resnorm, tol, max_iter, A_orig, lda_orig, stream, &first,
                      &converged);
    if (rc) return rc;
    int hinfo = 0;
    HQR_CK(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, stream));
    HQR_CK(hipStreamSynchronize(stream));
    if (!converged && hinfo == 0) {
        // FP64 solve from a copy of A_orig; the stored factorization is kept
        double *A2 = nullptr;
        if (hipMallocAsync((void **)&A2, sizeof(double) * (size_t)m * (size_t)n, stream) != hipSuccess)
            return HQR_ENOMEM;
        WorkGuard g2;
        g2.ptr = A2;
        g2.s = stream;
        double *up2 = nullptr;
        if (hipMallocAsync((void **)&up2, sizeof(double) * (size_t)n, stream) != hipSuccess) return HQR_ENOMEM;
        WorkGuard g3;
        g3.ptr = up2;
        g3.s = stream;
        HQR_CK(hipMemcpy2DAsync(A2, sizeof(double) * m, A_orig, sizeof(double) * lda_orig, sizeof(double) * m, n,
                                hipMemcpyDeviceToDevice, stream));
        HQR_CK(hipMemcpy2DAsync(B, sizeof(double) * ldb, w.borig, sizeof(double) * m, sizeof(double) * m, nrhs,
                                hipMemcpyDeviceToDevice, stream));
        rc = lsq_fp64(m, n, nrhs, A2, m, up2, B, ldb, resnorm, nullptr, 0, info, stream);
        if (rc) return rc;
        HQR_CK(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, stream));
        HQR_CK(hipStreamSynchronize(stream));
        hinfo |= HQR_INFO_NOCONV;
        HQR_CK(hipMemcpyAsync(info, &hinfo, sizeof(int), hipMemcpyHostToDevice, stream));
        HQR_CK(hipStreamSynchronize(stream));
        first = max_iter;
    }
    return write_iters(iters, first, stream);
}

int hqr_tune_set(int op, int64_t m_lo, int64_t m_hi, int64_t n_lo, int64_t n_hi, int precision, int choice)
{
    if (op != HQR_TUNE_SINGLE && op != HQR_TUNE_BATCHED) return -1;
    if (m_lo < 0) return -2;
    if (m_hi < m_lo) return -3;
    if (n_lo < 0) return -4;
    if (n_hi < n_lo) return -5;
    if (precision != HQR_PREC_FP64 && precision != HQR_PREC_MIXED) return -6;
    int cnt = 0;
    (void)wg_variants(&cnt);
    if (choice < (op == HQR_TUNE_SINGLE ? -1 : 0) || choice >= cnt) return -7;
    if (op == HQR_TUNE_BATCHED && !batch_variant(wg_variants(&cnt)[choice])) return -7;
    g_rules.push_back(TuneRule{op, m_lo, m_hi, n_lo, n_hi, precision, choice});
    return 0;
}

int hqr_tune_clear(void)
{
    g_rules.clear();
    return 0;
}

int hqr_tune_variants(void)
{
    int cnt = 0;
    (void)wg_variants(&cnt);
    return cnt;
}

const char *hqr_tune_variant_name(int i)
{
    int cnt = 0;
    const WgVariant *v = wg_variants(&cnt);
    return (i >= 0 && i < cnt) ? v[i].name : nullptr;
}

int hqr_profile_begin(void)
{
    g_prof.on = true;
    g_prof.n = 0;
    g_prof.pool_used = 0;
    return 0;
}

int hqr_profile_end(int nclass, double *ms, int64_t *count)
{
    if (nclass < 0) return -1;
    g_prof.on = false;
    for (int c = 0; c < nclass; ++c) {
        if (ms) ms[c] = 0.0;
        if (count) count[c] = 0;
    }
    int rc = 0;
    for (size_t i = 0; i < g_prof.n; ++i) {
        const ProfRec &r = g_prof.recs[i];
        if (hipEventSynchronize(r.e1) != hipSuccess) {
            rc = HQR_EDEVICE;
            continue;
        }
        float t = 0.0f;
        if (hipEventElapsedTime(&t, r.e0, r.e1) != hipSuccess) {
            rc = HQR_EDEVICE;
            continue;
        }
        if (r.cls < nclass) {
            if (ms) ms[r.cls] += (double)t;
            if (count) count[r.cls] += 1;
        }
    }
    g_prof.n = 0;
    g_prof.pool_used = 0;
    return rc ? rc : (int)K_NCLASS;
}

const char *hqr_profile_class(int cls)
{
    return (cls >= 0 && cls < (int)K_NCLASS) ? kclass_name[cls] : "";
}

const char *hqr_status_string(int status)
{
    switch (status) {
    case 0: return "success";
    case HQR_ENOMEM: return "workspace too small or allocation failed";
    case HQR_EDEVICE: return "a HIP call failed";
    case HQR_ENOTSUP: return "shape or option combination not supported";
    case HQR_INFO_TIMEOUT: return "a bounded cross-workgroup wait expired";
    case HQR_INFO_NOCONV: return "refinement did not converge; FP64 fallback used";
    default: break;
    }
    if (status < 0 && status > -100) return "invalid argument";
    if (status > 0) return "zero diagonal entry of R (info = k+1)";
    return "unknown status";
}

const char *hqr_version(void) { return "hqr-mi355x 0.1 (gfx950)"; }

} // extern "C"
