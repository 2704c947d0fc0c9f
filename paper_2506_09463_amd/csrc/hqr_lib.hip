// hqr_lib.hip -- libhqr: the C ABI declared in include/hqr.h and its host
// dispatch.  The kernels live in their own translation units (k_*.hip), each
// exporting launch functions declared in hqr_args.hpp.
#include "hqr.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "hqr_args.hpp"

namespace hqr {

// ------------------------------------------------------------- profiling
// Optional per-kernel-class timing: while active, every launch is bracketed
// by a pair of HIP events recorded on the launch's own stream.
static const char *kclass_name[K_NCLASS] = {"small_lsq", "panel_col", "vtx", "tfactor", "wsolve",
                                            "update", "diag_check", "trsv", "resnorm", "fill",
                                            "cqr_gram1", "cqr_gram2", "gram_reduce", "cqr_chol",
                                            "cqr_finish", "narrow_vtx", "batched_lsq", "refine", "tsqr"};
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

hipEvent_t prof_begin(hipStream_t s)
{
    if (!g_prof.on) return nullptr;
    hipEvent_t e = prof_event();
    if (e) (void)hipEventRecord(e, s);
    return e;
}

void prof_end(int cls, hipEvent_t e0, hipStream_t s)
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


// ------------------------------------------------- one-workgroup variants
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
    return k_wg_single(v, s, d, info) == hipSuccess ? 0 : HQR_EDEVICE;
}

// Panel factorization: CholeskyQR2 + reconstruction (default), one launch
// per pivot, the exact one-workgroup loop for every panel, or a TSQR panel
// + reconstruction for every panel (HQR_PANEL=percol|exact|tsqr; the TSQR
// panel also by HQR_OPT_TSQR_PANEL).
enum PanelMode { PANEL_CQR = 0, PANEL_PERCOL = 1, PANEL_EXACT = 2, PANEL_TSQR = 3 };

static int panel_mode()
{
    const char *e = getenv("HQR_PANEL");
    if (!e) return PANEL_CQR;
    if (!strcmp(e, "percol")) return PANEL_PERCOL;
    if (!strcmp(e, "exact")) return PANEL_EXACT;
    if (!strcmp(e, "tsqr")) return PANEL_TSQR;
    return PANEL_CQR;
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
    bool no_side;    // no look-ahead side stream (one stream only)
    bool tsqr;       // TSQR panels (workspace for the tree included)
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
    p.no_side = false;
    p.tsqr = panel_mode() == PANEL_TSQR;
    return p;
}

// Levels of a panel's TSQR tree: level 0 is the panel (mp rows), level l + 1
// stacks the bw x bw R factors of level l's blocks of at most
// TSQR_LEAF_ROWS rows; the last level is one block.
struct TsqrGeom {
    int nlev;
    int64_t rows[TSQR_MAX_LEVELS], nblk[TSQR_MAX_LEVELS];
};

static bool tsqr_geometry(int64_t mp, int bw, TsqrGeom &g)
{
    g.nlev = 0;
    int64_t rows = mp;
    for (;;) {
        if (g.nlev == TSQR_MAX_LEVELS) return false;
        const int64_t nblk = std::max<int64_t>(1, (rows + TSQR_LEAF_ROWS - 1) / TSQR_LEAF_ROWS);
        g.rows[g.nlev] = rows;
        g.nblk[g.nlev] = nblk;
        ++g.nlev;
        if (nblk == 1) return true;
        rows = nblk * bw;
    }
}

struct Work {
    double *xbuf, *pbuf, *wpart, *T, *wp;
    double *wpart2, *T2, *wp2;            // second set for the look-ahead stream
    double *xpub;                            // back-substitution: published x, [TRSV_MAXRHS][n]
    int *iscratch;
    double *gpart, *r1, *r1inv, *winv, *q1top;
    double *G, *xn;                          // reduced Gram; W = T^T V^T C of the look-ahead (transposed)
    double *borig, *rvec, *gvec, *mstat_d;   // refinement: original B, residuals, A^T r, previous ||dx||
    int *mstat;                              // refinement: [nrhs][4] column states, active count, verdict
    unsigned long long *mask, *mask_all;
    int *pflag;
    // TSQR panels: level 0's Q (m x NB), the stacked R and Q of levels >= 1,
    // the blocks' pivots, descriptors, queue heads and an unused info slot
    double *tq0 = nullptr;
    double *tstack[TSQR_MAX_LEVELS] = {}, *tqs[TSQR_MAX_LEVELS] = {}, *tup[TSQR_MAX_LEVELS] = {};
    WgDesc *tdesc[TSQR_MAX_LEVELS] = {};
    int *theads = nullptr, *tinfo = nullptr;
    double *tsign = nullptr;
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
    char *fl = take(sizeof(double) * TRSV_MAXRHS * (size_t)std::max<int64_t>(p.n, 1));
    char *is = take(sizeof(int) * 64);
    char *gp = take(sizeof(double) * (size_t)p.ngroups * NB * NB);
    char *r1 = take(sizeof(double) * NB * NB);
    char *r1i = take(sizeof(double) * NB * NB);
    char *wi = take(sizeof(double) * NB * NB);
    char *mk = take(sizeof(unsigned long long) * (size_t)p.ngroups);
    char *pf = take(sizeof(int) * (size_t)std::max(p.npanels, 1));
    char *bo = take(sizeof(double) * (size_t)p.m * (size_t)std::max<int64_t>(p.nrhs, 1));
    const size_t nr = (size_t)std::max<int64_t>(p.nrhs, 1);
    char *rv = take(sizeof(double) * (size_t)std::max<int64_t>(p.m, 1) * nr);
    char *gv = take(sizeof(double) * (size_t)std::max<int64_t>(p.n, 1) * nr);
    char *msd = take(sizeof(double) * nr);
    char *ms = take(sizeof(int) * (4 * nr + 2));
    char *q1 = take(sizeof(double) * NB * NB);
    char *gg = take(sizeof(double) * NB * NB);
    char *xn = take(sizeof(double) * NB * NB);
    char *ma = take(sizeof(unsigned long long));
    if (p.tsqr) {
        TsqrGeom g;
        tsqr_geometry(p.m, NB, g);
        char *q0 = take(sizeof(double) * (size_t)p.m * NB);
        char *st[TSQR_MAX_LEVELS] = {}, *qs[TSQR_MAX_LEVELS] = {}, *tu[TSQR_MAX_LEVELS] = {}, *td[TSQR_MAX_LEVELS] = {};
        for (int l = 0; l < g.nlev; ++l) {
            if (l > 0) {
                st[l] = take(sizeof(double) * (size_t)g.rows[l] * NB);
                qs[l] = take(sizeof(double) * (size_t)g.rows[l] * NB);
            }
            tu[l] = take(sizeof(double) * (size_t)g.nblk[l] * NB);
            td[l] = take(sizeof(WgDesc) * 2 * (size_t)g.nblk[l]);
        }
        char *th = take(sizeof(int) * 2 * TSQR_MAX_LEVELS);
        char *ti = take(sizeof(int) * 64);
        char *tsg = take(sizeof(double) * NB);
        if (w) {
            w->tq0 = (double *)q0;
            for (int l = 0; l < TSQR_MAX_LEVELS; ++l) {
                w->tstack[l] = (double *)st[l];
                w->tqs[l] = (double *)qs[l];
                w->tup[l] = (double *)tu[l];
                w->tdesc[l] = (WgDesc *)td[l];
            }
            w->theads = (int *)th;
            w->tinfo = (int *)ti;
            w->tsign = (double *)tsg;
        }
    }
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
        w->xpub = (double *)fl;
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
                             int vtx_wg_cap = 0, bool apply_q = false)
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
    HQR_CK(k_vtx(f32, v.with_v != 0, vg, s, v));

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
        HQR_CK(k_tfactor(s, t));
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
    wa.tmode = apply_q ? 1 : 0;
    HQR_CK(k_wsolve(narrow, dim3(narrow ? (ncols + WSN_COLS - 1) / WSN_COLS : (ncols + WS_COLS - 1) / WS_COLS), s,
                    wa));

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
        HQR_CK(k_update(true, f32, ug, s, uf));
        HQR_CK(hipEventRecord(ev_first, s));
        u.ncA -= first_cols;
        u.aoff += first_cols;
        u.xoff += first_cols;
    }
    const int ncols_u = u.ncA + u.nB;
    if (narrow) {
        const dim3 ug((unsigned)((rows + 63) / 64));
        HQR_CK(k_update(true, f32, ug, s, u));
    } else {
        const dim3 ug((unsigned)((rows + UPD_TILE - 1) / UPD_TILE), (ncols_u + UPD_TILE - 1) / UPD_TILE);
        HQR_CK(k_update(false, f32, ug, s, u));
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
        HQR_CK(k_panel_col(dim3(pa.nchunk), s, pa));
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
    HQR_CK(k_gram_reduce(s, gr));
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
    HQR_CK(k_cqr_chol(s, c));
    return 0;
}

// Panel (c0, bw) by CholeskyQR2 + reconstruction, bottom rows not yet
// finished.  With upd, the previous panel (start cp, width NB; W = T^T V^T C
// transposed in w.xn) is first applied to this panel's columns.
// TSQR panel (c0, bw) after CholeskyQR pass 1 (which has applied the
// previous panel's update and flagged exact zero tails): the tree's block
// factorizations bottom-up, the explicit Q top-down, then the panel := Q D
// and the first factor := D R for the second pass.  Every launch is empty or
// returns at once for a panel flagged 1 (read on the device).
static int num_cus();

static int tsqr_panel(const Plan &pl, const Work &w, double *A, int64_t lda, int c0, int bw, int pidx,
                      hipStream_t s)
{
    TsqrGeom g;
    if (!tsqr_geometry(pl.m - c0, bw, g)) return HQR_ENOTSUP;
    TsqrArgs a;
    a.flag = w.pflag + pidx;
    a.bw = bw;
    a.nlev = g.nlev;
    a.heads = w.theads;
    double *Ap = A + (size_t)c0 * lda + c0;
    for (int l = 0; l < g.nlev; ++l) {
        TsqrLevel &L = a.lev[l];
        L.rows = g.rows[l];
        L.nblk = g.nblk[l];
        L.base = L.rows / L.nblk;
        L.rem = L.rows % L.nblk;
        L.X = (l == 0) ? Ap : w.tstack[l];
        L.ldx = (l == 0) ? lda : L.rows;
        L.Q = (l == 0) ? w.tq0 : w.tqs[l];
        L.ldq = (l == 0) ? pl.m : L.rows;
        L.up = w.tup[l];
        L.fdesc = w.tdesc[l];
        L.adesc = w.tdesc[l] + L.nblk;
    }
    HQR_CK(k_tsqr_desc(s, a));
    auto batched = [&](int l, const WgDesc *desc, int *head) -> int {
        const TsqrLevel &L = a.lev[l];
        const WgVariant *v = pick_wg_batched(L.base + (L.rem > 0 ? 1 : 0), bw);
        if (!v) return HQR_ENOTSUP;
        const int grid = (int)std::min<int64_t>(L.nblk, (int64_t)v->per_cu * num_cus());
        HQR_CK(k_wg_batched(v, grid, s, desc, (int)L.nblk, head, w.tinfo));
        return 0;
    };
    const int top = g.nlev - 1;
    for (int l = 0; l <= top; ++l) {
        int rc = batched(l, a.lev[l].fdesc, a.heads + 2 * l);
        if (rc) return rc;
        if (l < top) HQR_CK(k_tsqr_gather(s, a, l));
    }
    HQR_CK(k_eye(s, a.lev[top].Q, a.lev[top].ldq, a.lev[top].rows, bw));
    int rc = batched(top, a.lev[top].adesc, a.heads + 2 * top + 1);
    if (rc) return rc;
    for (int l = top - 1; l >= 0; --l) {
        HQR_CK(k_tsqr_scatter(s, a, l));
        rc = batched(l, a.lev[l].adesc, a.heads + 2 * l + 1);
        if (rc) return rc;
    }
    HQR_CK(k_tsqr_final(s, a, Ap, lda, w.r1, w.r1inv, w.tsign));
    return 0;
}

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
    HQR_CK(k_cqr_gram1(dim3((unsigned)((pl.m - rbase + 63) / 64)), s, g));
    int rc = launch_gred(pl, w, parts, w.G, true, flag, s);
    if (!rc) rc = launch_chol(pl, w, A, lda, up, c0, bw, pidx, 1, Tout, s);
    if (!rc && pl.tsqr) rc = tsqr_panel(pl, w, A, lda, c0, bw, pidx, s);
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
    HQR_CK(k_cqr_gram2(dim3((unsigned)parts), s, g2));
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
    HQR_CK(k_cqr_finish(dim3((unsigned)((mp - bw + 63) / 64)), s, f));
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
    HQR_CK(k_narrow_vtx(dim3((unsigned)parts), s, a));
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

// Per caller stream (and device): the look-ahead's side stream with its
// events, and the pinned staging buffer of the batched descriptor upload.
// Created on first use and kept for the process; a solve on stream s only
// ever touches s's context, so solves on different streams neither share
// events nor serialize their look-ahead work.  Calls on ONE stream from
// several host threads must be serialized by the caller (as any stream use).
struct StreamCtx {
    int device = -1;
    hipStream_t caller = nullptr;
    hipStream_t side = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    void *stage = nullptr;       // pinned host staging buffer
    size_t stage_bytes = 0;
    hipEvent_t stage_ready = nullptr;
};
constexpr int MAX_STREAM_CTX = 256;
static StreamCtx g_ctx[MAX_STREAM_CTX];
static int g_nctx = 0;
static std::mutex g_ctx_mu;

static StreamCtx *stream_ctx(hipStream_t caller)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_ctx_mu);
    for (int i = 0; i < g_nctx; ++i)
        if (g_ctx[i].device == dev && g_ctx[i].caller == caller) return &g_ctx[i];
    if (g_nctx == MAX_STREAM_CTX) return nullptr;
    StreamCtx &c = g_ctx[g_nctx];
    if (hipStreamCreateWithFlags(&c.side, hipStreamNonBlocking) != hipSuccess) return nullptr;
    // the events only order the two streams of one device: no timing and
    // no system-scope fence (kernel boundaries already release to the device)
    for (auto &e : c.ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming | hipEventDisableSystemFence) != hipSuccess)
            return nullptr;
    if (hipEventCreateWithFlags(&c.stage_ready, hipEventDisableTiming) != hipSuccess) return nullptr;
    c.device = dev;
    c.caller = caller;
    ++g_nctx;
    return &c;
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
        HQR_CK(k_fill_int(s, w.pflag, mode == PANEL_EXACT ? 1 : 0,
                   (int64_t)pl.npanels));
        HQR_CK(hipGetLastError());
    }
    StreamCtx *ss = (lookahead_enabled() && pl.npanels > 1 && !pl.no_side) ? stream_ctx(s) : nullptr;
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
    HQR_CK(hipStreamWaitEvent(ss->side, ev_fork, 0));
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
            HQR_CK(hipStreamWaitEvent(ss->side, ev_a, 0));
            // R(p): the columns of panel p+2 first, then r(p) (all that
            // narrow_vtx(p+1) reads), then the rest of the columns and B
            if (ncR + nB > 0) {
                // late panels, where the main chain is the longer one: V^T C
                // on at most half the CUs so the chain's kernels find free ones
                rc = apply_panel_block(pl, br, A, lda, B, ldb, up, (int)c0, bw, bw1, ncR, nB, true, ss->side, false,
                                       std::min(ncR, (int)pl.nb), ev_r, (ncR + nB <= 2048) ? 128 : 0);
                if (rc) return rc;
            } else {
                HQR_CK(hipEventRecord(ev_r, ss->side));
            }
            if (bw1 > 0) {
                XwArgs xa;
                xa.gpart = w.gpart;
                xa.parts = (int)((pl.m - c0 + 63) / 64);
                xa.T = Tbuf[pidx & 1];
                xa.Wt = w.xn;
                HQR_CK(k_xw_reduce(s, xa));
                if (!rc)
                    rc = panel_passes(pl, w, A, lda, up, (int)c1, bw1, pidx + 1, Tbuf[(pidx + 1) & 1], true, (int)c0,
                                      s);
                if (rc) return rc;
            }
            pending_r = true;
        }
        HQR_CK(hipEventRecord(ev_join, ss->side));
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
        HQR_CK(hipStreamWaitEvent(ss->side, ev_a, 0));
        if (ncR + nB > 0) {
            rc = apply_panel_block(pl, br, A, lda, B, ldb, up, (int)c0, bw, bw1, ncR, nB, have_t, ss->side, pl.f32,
                                   std::min(ncR, (int)pl.nb), ev_r);
            if (rc) return rc;
        } else {
            HQR_CK(hipEventRecord(ev_r, ss->side));
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
    HQR_CK(hipEventRecord(ev_join, ss->side));
    HQR_CK(hipStreamWaitEvent(s, ev_join, 0));
    return 0;
}

static int backsolve_blocked(const Plan &pl, const Work &w, const double *A, int64_t lda, double *B, int64_t ldb,
                             int nrhs, int *info, hipStream_t s, bool trans = false, const int *active = nullptr)
{
    HQR_CK(k_diag_check(s, A, lda, pl.n, info));
    for (int c = 0; c < nrhs; c += TRSV_MAXRHS) {
        TrsvArgs t;
        t.A = A;
        t.lda = lda;
        t.B = B + (size_t)c * ldb;
        t.ldb = ldb;
        t.n = pl.n;
        t.nrhs = std::min(TRSV_MAXRHS, nrhs - c);
        HQR_CK(k_fill_int(s, (int *)w.xpub, TRSV_EMPTY_WORD, 2 * pl.n * (int64_t)t.nrhs));
        t.xpub = w.xpub;
        t.info = info;
        t.spin_limit = 20000000L;
        t.active = active;
        HQR_CK(k_trsv(trans, t.nrhs, dim3(pl.nblk), s, t));
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

// B <- Q^T B (transpose) or Q B with the stored reflectors in (A, up).  With
// skip, B's column j is only touched by the panels that start at or before
// column j: B then starts as leading columns of the identity, and no
// reflector k > j changes column j of the identity (its vector is zero in
// rows 0..k-1).
static int apply_stored(const Plan &pl, const Work &w, const double *A, int64_t lda, const double *up, double *B,
                        int64_t ldb, int64_t nrhs, bool transpose, bool skip, hipStream_t s)
{
    const int64_t m = pl.m, n = pl.n;
    if (n == 0 || nrhs == 0) return 0;
    if (const WgVariant *v = pick_wg_single(m, n, nrhs)) {
        const int64_t fl = (transpose ? 0 : WG_APPLY_Q) | (skip ? WG_QSKIP : 0);
        const WgDesc d{m, n, nrhs, lda, ldb, const_cast<double *>(A), B, const_cast<double *>(up), nullptr, 0, fl};
        return launch_wg_single(v, d, nullptr, s);
    }
    const int npan = (int)((n + NB - 1) / NB);
    for (int q = 0; q < npan; ++q) {
        const int p = transpose ? q : npan - 1 - q;
        const int64_t c0 = (int64_t)p * NB;
        const int bw = (int)std::min<int64_t>(NB, n - c0);
        const int64_t j0 = skip ? c0 : 0;
        if (nrhs <= j0) continue;
        int rc = apply_panel_block(pl, TrailBufs{w.wpart, w.T, w.wp}, const_cast<double *>(A), lda,
                                   B + (size_t)j0 * ldb, ldb, up, (int)c0, bw, 0, 0, (int)(nrhs - j0), false, s,
                                   false, 0, nullptr, 0, !transpose);
        if (rc) return rc;
    }
    return 0;
}

// The FP64 path: small problems in one register-resident workgroup, larger
// ones by the blocked factorization, then residual norms and back-substitution.
static int lsq_fp64(int64_t m, int64_t n, int64_t nrhs, double *A, int64_t lda, double *up, double *B, int64_t ldb,
                    double *resnorm, void *work, int64_t lwork, int *info, hipStream_t s, bool side = true,
                    bool tsqr = false)
{
    if (n == 0) {
        HQR_CK(k_fill_int(s, info, 0, (int64_t)1));
        HQR_CK(hipGetLastError());
        if (resnorm && nrhs > 0) {
            HQR_CK(k_resnorm(dim3((unsigned)nrhs), s, B, ldb, 0, m, resnorm));
        }
        return 0;
    }
    if (const WgVariant *v = pick_wg_single(m, n, nrhs)) {
        if (nrhs == 0) {
            HQR_CK(k_fill_int(s, info, 0, (int64_t)1));
            HQR_CK(hipGetLastError());
        }
        const WgDesc d{m, n, nrhs, lda, ldb, A, B, up, resnorm, 0, WG_FACTOR | (nrhs > 0 ? WG_SOLVE : 0)};
        return launch_wg_single(v, d, info, s);
    }
    Plan pl = make_plan(m, n, nrhs);
    pl.no_side = !side;
    pl.tsqr = pl.tsqr || tsqr;
    WorkGuard g;
    Work w;
    int rc = get_work(pl, work, lwork, s, g, &w);
    if (rc) return rc;
    HQR_CK(k_fill_int(s, info, 0, (int64_t)1));
    rc = factor_blocked(pl, w, A, lda, up, B, ldb, (int)nrhs, s);
    if (rc) return rc;
    if (nrhs == 0) return 0;
    if (resnorm) {
        HQR_CK(k_resnorm(dim3((unsigned)nrhs), s, B, ldb, n, m, resnorm));
    }
    return backsolve_blocked(pl, w, A, lda, B, ldb, (int)nrhs, info, s);
}

// Refinement of every right-hand side with the semi-normal equations
// (RefineArgs): max_iter steps are enqueued; a column that converges or fails
// freezes and, once none is left, the remaining launches return at once.  The
// verdict kernel then writes iters and verdict (1: every column converged),
// and with or_info ORs HQR_INFO_NOCONV into info when not.  Residual norms
// ||b - A0 x|| go to resnorm.  Nothing here waits on the host.
static int mixed_refine(const Plan &pl, const Work &w, const double *A, int64_t lda, double *B, int64_t ldb,
                        int64_t nrhs, double *resnorm, double tol, int max_iter, const double *A0, int64_t lda0,
                        hipStream_t s, int *info, int *iters, bool or_info)
{
    RefineArgs r;
    r.A0 = A0;
    r.lda0 = lda0;
    r.borig = w.borig;
    r.X = B;
    r.ldx = ldb;
    r.rvec = w.rvec;
    r.gvec = w.gvec;
    r.m = pl.m;
    r.n = pl.n;
    r.nrhs = (int)nrhs;
    r.tol = tol;
    r.max_iter = max_iter;
    r.stat = w.mstat;
    r.dxprev = w.mstat_d;
    r.active = w.mstat + 4 * nrhs;
    int *verdict = w.mstat + 4 * nrhs + 1;
    HQR_CK(k_refine_init(s, r));
    const int64_t ldg = std::max<int64_t>(pl.n, 1);
    for (int it = 0; it < max_iter; ++it) {
        HQR_CK(k_resid(false, s, r));
        HQR_CK(k_gemvt(s, r));
        int rc = backsolve_blocked(pl, w, A, lda, w.gvec, ldg, (int)nrhs, w.iscratch, s, true, r.active);
        if (rc) return rc;
        rc = backsolve_blocked(pl, w, A, lda, w.gvec, ldg, (int)nrhs, w.iscratch, s, false, r.active);
        if (rc) return rc;
        HQR_CK(k_csne_update(s, r, it));
    }
    if (resnorm) {
        HQR_CK(k_resid(true, s, r));
        HQR_CK(k_resnorm(dim3((unsigned)nrhs), s, w.rvec, std::max<int64_t>(pl.m, 1), 0, pl.m, resnorm));
    }
    HQR_CK(k_refine_verdict(s, r, verdict, info, iters, or_info));
    return 0;
}

// Reads the refinement verdict back (one synchronization of the stream).
static int read_verdict(const Work &w, int64_t nrhs, hipStream_t s, bool *converged)
{
    int v = 0;
    HQR_CK(hipMemcpyAsync(&v, w.mstat + 4 * nrhs + 1, sizeof(int), hipMemcpyDeviceToHost, s));
    HQR_CK(hipStreamSynchronize(s));
    *converged = v != 0;
    return 0;
}

static bool no_fallback(const hqr_opts *opt) { return opt && (opt->flags & HQR_OPT_NO_FALLBACK); }
static bool tsqr_opt(const hqr_opts *opt) { return opt && (opt->flags & HQR_OPT_TSQR_PANEL); }

// Mixed precision: FP32 trailing contractions in the factorization, FP64
// back-substitution, then the refinement above.  Without HQR_OPT_NO_FALLBACK
// the stream is synchronized once to read the verdict and, without
// convergence, the FP64 path runs on the restored inputs and
// HQR_INFO_NOCONV is ORed into the info it reports.  With it nothing waits
// on the host: HQR_INFO_NOCONV is ORed into info on the device and x is the
// last iterate.
static int lsq_mixed(int64_t m, int64_t n, int64_t nrhs, double *A, int64_t lda, double *up, double *B,
                     int64_t ldb, double *resnorm, const hqr_opts *opt, const double *A0, int64_t lda0, void *work,
                     int64_t lwork, int *info, int *iters, hipStream_t s)
{
    const double tol = (opt && opt->tol > 0.0) ? opt->tol : 1e-13;
    const int max_iter = (opt && opt->max_iter >= 0) ? opt->max_iter : 10;
    const bool async = no_fallback(opt);
    const int nb = (n <= 256) ? 16 : NB;
    Plan pl = make_plan(m, n, nrhs, nb, true);
    pl.tsqr = pl.tsqr || tsqr_opt(opt);
    WorkGuard g;
    Work w;
    int rc = get_work(pl, work, lwork, s, g, &w);
    if (rc) return rc;
    HQR_CK(hipMemcpy2DAsync(w.borig, sizeof(double) * m, B, sizeof(double) * ldb, sizeof(double) * m, nrhs,
                            hipMemcpyDeviceToDevice, s));
    HQR_CK(k_fill_int(s, info, 0, (int64_t)1));
    rc = factor_blocked(pl, w, A, lda, up, B, ldb, (int)nrhs, s);
    if (rc) return rc;
    rc = backsolve_blocked(pl, w, A, lda, B, ldb, (int)nrhs, info, s);
    if (rc) return rc;
    rc = mixed_refine(pl, w, A, lda, B, ldb, nrhs, resnorm, tol, max_iter, A0, lda0, s, info, iters, async);
    if (rc || async) return rc;
    bool converged = true;
    rc = read_verdict(w, nrhs, s, &converged);
    if (rc || converged) return rc;
    // FP64 fallback on the restored inputs: the same call as precision FP64,
    // then the flag ORed into whatever info that call reports
    HQR_CK(hipMemcpy2DAsync(A, sizeof(double) * lda, A0, sizeof(double) * lda0, sizeof(double) * m, n,
                            hipMemcpyDeviceToDevice, s));
    HQR_CK(hipMemcpy2DAsync(B, sizeof(double) * ldb, w.borig, sizeof(double) * m, sizeof(double) * m, nrhs,
                            hipMemcpyDeviceToDevice, s));
    rc = lsq_fp64(m, n, nrhs, A, lda, up, B, ldb, resnorm, nullptr, 0, info, s, true, tsqr_opt(opt));
    if (rc) return rc;
    HQR_CK(k_or_int(s, info, HQR_INFO_NOCONV));
    return 0;
}

} // namespace hqr

using namespace hqr;


// ------------------------------------------------------------ batched path
namespace hqr {

// Descriptor upload through the caller stream's pinned staging buffer; the
// buffer's `stage_ready` event fences its reuse by the next call on that
// stream.
static int stage_upload(const void *src, size_t bytes, void *dst, hipStream_t s)
{
    StreamCtx *c = stream_ctx(s);
    if (!c) return HQR_EDEVICE;
    HQR_CK(hipEventSynchronize(c->stage_ready));
    if (c->stage_bytes < bytes) {
        if (c->stage) (void)hipHostFree(c->stage);
        c->stage = nullptr;
        c->stage_bytes = 0;
        if (hipHostMalloc(&c->stage, bytes, hipHostMallocDefault) != hipSuccess) return HQR_ENOMEM;
        c->stage_bytes = bytes;
    }
    memcpy(c->stage, src, bytes);
    HQR_CK(hipMemcpyAsync(dst, c->stage, bytes, hipMemcpyHostToDevice, s));
    HQR_CK(hipEventRecord(c->stage_ready, s));
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
    HQR_CK(k_fill_int(stream, head, 0, (int64_t)2));
    HQR_CK(hipGetLastError());
    if (nwg > 0) {
        int occ = tune_lookup(HQR_TUNE_OCCUPANCY, mmax, nmax, HQR_PREC_FP64);
        occ = (occ >= 1) ? std::min(occ, var->per_cu) : std::min(var->per_cu, 2);
        const int grid = std::min(nwg, occ * num_cus());
        HQR_CK(k_wg_batched(var, grid, stream, (const WgDesc *)dbase, nwg, head, info));
    }
    if (nwg < count) {
        BatchArgs a;
        a.desc = (const BatchDesc *)(dbase + sizeof(WgDesc) * (size_t)nwg);
        a.count = count - nwg;
        a.head = head + 1;
        a.info = info;
        a.max_ntot = max_ntot;
        const int grid = std::min(count - nwg, 2 * num_cus());
        HQR_CK(k_batched_lsq(dim3(grid), stream, a));
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

int64_t hqr_workspace_size_opts(int64_t m, int64_t n, int64_t nrhs, const hqr_opts *opt)
{
    const int precision = opt ? opt->precision : HQR_PREC_FP64;
    const int64_t base = hqr_workspace_size(m, n, nrhs, precision);
    if (base < 0 || !tsqr_opt(opt)) return base;
    Plan pl = (precision == HQR_PREC_MIXED) ? make_plan(m, n, nrhs, (n <= 256) ? 16 : NB, true) : make_plan(m, n, nrhs);
    pl.tsqr = true;
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
        HQR_CK(k_fill_int(stream, info, 0, (int64_t)1));
        return hipGetLastError() == hipSuccess ? 0 : HQR_EDEVICE;
    }
    if (const WgVariant *v = pick_wg_single(m, n, 0)) {
        HQR_CK(k_fill_int(stream, info, 0, (int64_t)1));
        HQR_CK(hipGetLastError());
        const WgDesc d{m, n, 0, lda, std::max<int64_t>(1, m), A, nullptr, up, nullptr, 0, WG_FACTOR};
        return launch_wg_single(v, d, info, stream);
    }
    Plan pl = make_plan(m, n, 0);
    WorkGuard g;
    Work w;
    int rc = get_work(pl, work, lwork, stream, g, &w);
    if (rc) return rc;
    HQR_CK(k_fill_int(stream, info, 0, (int64_t)1));
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
    Plan pl = make_plan(m, n, nrhs);
    WorkGuard g;
    Work w;
    if (!pick_wg_single(m, n, nrhs)) {
        const int rc = get_work(pl, work, lwork, stream, g, &w);
        if (rc) return rc;
    }
    return apply_stored(pl, w, A, lda, up, B, ldb, nrhs, true, false, stream);
}

int qr_apply_q(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *up, double *B,
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
    Plan pl = make_plan(m, n, nrhs);
    WorkGuard g;
    Work w;
    if (!pick_wg_single(m, n, nrhs)) {
        const int rc = get_work(pl, work, lwork, stream, g, &w);
        if (rc) return rc;
    }
    return apply_stored(pl, w, A, lda, up, B, ldb, nrhs, false, false, stream);
}

int qr_form_q(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, const double *up, double *Q,
              int64_t ldq, void *work, int64_t lwork, hipStream_t stream)
{
    if (m < 0) return -1;
    if (n < 0 || n > m) return -2;
    if (k < 0 || k > m) return -3;
    if (lda < std::max<int64_t>(1, m)) return -5;
    if (ldq < std::max<int64_t>(1, m)) return -8;
    if (k == 0) return 0;
    if (!Q) return -7;
    if (n > 0 && !A) return -4;
    if (n > 0 && !up) return -6;
    if (m > INT32_MAX / 2 || k > INT32_MAX / 4) return HQR_ENOTSUP;
    HQR_CK(k_eye(stream, Q, ldq, m, k));
    if (n == 0) return 0;
    Plan pl = make_plan(m, n, k);
    WorkGuard g;
    Work w;
    if (!pick_wg_single(m, n, k)) {
        const int rc = get_work(pl, work, lwork, stream, g, &w);
        if (rc) return rc;
    }
    return apply_stored(pl, w, A, lda, up, Q, ldq, k, false, true, stream);
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
        HQR_CK(k_fill_int(stream, info, 0, (int64_t)1));
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
            HQR_CK(k_fill_int(stream, iters, 0, (int64_t)1));
            HQR_CK(hipGetLastError());
        }
        if (n == 0 || nrhs == 0) {
            HQR_CK(k_fill_int(stream, info, 0, (int64_t)1));
            return hipGetLastError() == hipSuccess ? 0 : HQR_EDEVICE;
        }
        return lsq_mixed(m, n, nrhs, A, lda, up, B, ldb, resnorm, opt, A_orig, lda_orig, work, lwork, info, iters,
                         stream);
    }
    (void)A_orig;
    (void)lda_orig;
    if (m > INT32_MAX / 2 || n > INT32_MAX / 2 || nrhs > INT32_MAX / 4) return HQR_ENOTSUP;
    if (iters) {
        HQR_CK(k_fill_int(stream, iters, 0, (int64_t)1));
        HQR_CK(hipGetLastError());
    }
    return lsq_fp64(m, n, nrhs, A, lda, up, B, ldb, resnorm, work, lwork, info, stream, true, tsqr_opt(opt));
}

// ------------------------------------------- entry point without allocation
// qr_lsq_solve_static works in `scratch`, a device array of the library's
// own (one per GPU, held until the process ends).  Host code never uses the
// array's name as an address: its device address is looked up once per
// device with hipGetSymbolAddress, on the first call on that device (with
// the device current), and kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[HQR_STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static void *g_scratch_ptr[MAX_DEVICES];
static std::mutex g_scratch_mu;

static int scratch_address(void **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return HQR_EDEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HQR_EDEVICE;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

int qr_lsq_solve_static(int64_t m, int64_t n, int64_t nrhs, double *A, int64_t lda, double *up, double *B,
                        int64_t ldb, double *resnorm, int *info, hipStream_t stream)
{
    if (m < 0) return -1;
    if (n < 0 || n > m) return -2;
    if (nrhs < 0) return -3;
    if (lda < std::max<int64_t>(1, m)) return -5;
    if (ldb < std::max<int64_t>(1, m)) return -8;
    if (!info) return -10;
    if (n > 0) {
        if (!A) return -4;
        if (!up) return -6;
    }
    if (nrhs > 0 && !B) return -7;
    if (m > INT32_MAX / 2 || n > INT32_MAX / 2 || nrhs > INT32_MAX / 4) return HQR_ENOTSUP;
    const int64_t need = hqr_workspace_size(m, n, nrhs, HQR_PREC_FP64);
    if (need < 0) return (int)need;
    if (need > (int64_t)HQR_STATIC_SCRATCH_BYTES) return HQR_ENOMEM;
    void *p = nullptr;
    const int rc = scratch_address(&p);
    if (rc) return rc;
    return lsq_fp64(m, n, nrhs, A, lda, up, B, ldb, resnorm, p, (int64_t)HQR_STATIC_SCRATCH_BYTES, info, stream,
                    false);
}

// ------------------------------------- equality-constrained least squares
// Pieces of the LSE workspace: C^T, its up, A^T, the reduced problem's up,
// info words, then one region shared by the sub-steps in turn (each
// sub-step's own workspace, at most the largest of them).
struct LseParts {
    double *ct, *upc, *at, *upr;
    int *ints;
    char *sub;
    int64_t sub_bytes;
};

static int64_t lse_sub_bytes(int64_t m, int64_t n, int64_t p)
{
    int64_t s = 0;
    if (p > 0) {
        s = std::max(s, hqr_workspace_size(n, p, 0, HQR_PREC_FP64));
        s = std::max(s, hqr_workspace_size(n, p, std::max<int64_t>(m, 1), HQR_PREC_FP64));
        s = std::max(s, hqr_workspace_size(p, p, 1, HQR_PREC_FP64));
    }
    if (n - p > 0) s = std::max(s, hqr_workspace_size(m, n - p, 1, HQR_PREC_FP64));
    return s;
}

static size_t lse_bytes(int64_t m, int64_t n, int64_t p, LseParts *lp, char *base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *ptr = base ? base + off : nullptr;
        off += align256(std::max<size_t>(bytes, 1));
        return ptr;
    };
    char *ct = take(sizeof(double) * (size_t)n * (size_t)p);
    char *upc = take(sizeof(double) * (size_t)p);
    char *at = take(sizeof(double) * (size_t)n * (size_t)m);
    char *upr = take(sizeof(double) * (size_t)(n - p));
    char *ints = take(sizeof(int) * 4);
    const int64_t sb = lse_sub_bytes(m, n, p);
    char *sub = take((size_t)sb);
    if (lp) *lp = LseParts{(double *)ct, (double *)upc, (double *)at, (double *)upr, (int *)ints, sub, sb};
    return off;
}

int64_t hqr_lse_workspace_size(int64_t m, int64_t n, int64_t p)
{
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (p < 0 || p > n || m < n - p) return -3;
    return (int64_t)lse_bytes(m, n, p, nullptr, nullptr);
}

int qr_lse_solve(int64_t m, int64_t n, int64_t p, double *A, int64_t lda, double *C, int64_t ldc, double *b,
                 const double *d, double *x, void *work, int64_t lwork, int *info, hipStream_t stream)
{
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (p < 0 || p > n || m < n - p) return -3;
    if (lda < std::max<int64_t>(1, m)) return -5;
    if (ldc < std::max<int64_t>(1, p)) return -7;
    if (!info) return -13;
    if (n > 0 && m > 0 && !A) return -4;
    if (p > 0 && !C) return -6;
    if (p > 0 && !d) return -9;
    if (m > 0 && !b) return -8;
    if (n > 0 && !x) return -10;
    if (m > INT32_MAX / 4 || n > INT32_MAX / 4) return HQR_ENOTSUP;
    HQR_CK(k_fill_int(stream, info, 0, (int64_t)1));
    if (n == 0) return 0;
    const size_t need = lse_bytes(m, n, p, nullptr, nullptr);
    WorkGuard g;
    char *base = (char *)work;
    if (!base) {
        if (hipMallocAsync((void **)&base, need, stream) != hipSuccess) return HQR_ENOMEM;
        g.ptr = base;
        g.s = stream;
    } else if (lwork < (int64_t)need) {
        return HQR_ENOMEM;
    }
    LseParts lp;
    lse_bytes(m, n, p, &lp, base);
    int *info_c = lp.ints, *info_r = lp.ints + 1;
    HQR_CK(k_fill_int(stream, lp.ints, 0, (int64_t)4));
    int rc = 0;
    if (p > 0) {
        // 1. C^T = Q [R; 0]
        HQR_CK(k_transpose(stream, C, ldc, lp.ct, n, p, n));
        rc = qr_factor(n, p, lp.ct, n, lp.upc, lp.sub, lp.sub_bytes, lp.ints + 2, stream);
        if (rc) return rc;
        // 2. R^T y1 = d, y1 in x[0:p]
        HQR_CK(k_copy_vec(stream, d, x, p));
        Plan pb = make_plan(p, p, 1);
        Work wb;
        WorkGuard gb;
        rc = get_work(pb, lp.sub, lp.sub_bytes, stream, gb, &wb);
        if (!rc) rc = backsolve_blocked(pb, wb, lp.ct, n, x, std::max<int64_t>(p, 1), 1, info_c, stream, true);
        if (rc) return rc;
        // 3. A Q = (Q^T A^T)^T, written over A
        if (m > 0) {
            HQR_CK(k_transpose(stream, A, lda, lp.at, n, m, n));
            rc = qr_apply_qt(n, p, m, lp.ct, n, lp.upc, lp.at, n, lp.sub, lp.sub_bytes, stream);
            if (rc) return rc;
            HQR_CK(k_transpose(stream, lp.at, n, A, lda, n, m));
            // 4. b -= (A Q)[:, 0:p] y1
            HQR_CK(k_gemv_sub(stream, A, lda, x, b, m, p));
        }
    }
    // 5. the reduced least-squares problem on (A Q)[:, p:n]; y2 in x[p:n]
    if (n - p > 0) {
        rc = lsq_fp64(m, n - p, 1, A + (size_t)p * lda, lda, lp.upr, b, std::max<int64_t>(m, 1), nullptr, lp.sub,
                      lp.sub_bytes, info_r, stream);
        if (rc) return rc;
        HQR_CK(k_copy_vec(stream, b, x + p, n - p));
    }
    // 6. x = Q [y1; y2]
    if (p > 0) {
        rc = qr_apply_q(n, p, 1, lp.ct, n, lp.upc, x, std::max<int64_t>(n, 1), lp.sub, lp.sub_bytes, stream);
        if (rc) return rc;
    }
    HQR_CK(k_lse_info(stream, info, info_c, info_r, p));
    return 0;
}

// ------------------------------------------------ Cholesky and its update
int hqr_cholesky(int64_t n, double *S, int64_t lds, void *work, int64_t lwork, int *info, hipStream_t stream)
{
    if (n < 0) return -1;
    if (lds < std::max<int64_t>(1, n)) return -3;
    if (!info) return -6;
    if (n > 0 && !S) return -2;
    if (n > INT32_MAX / 4) return HQR_ENOTSUP;
    HQR_CK(k_fill_int(stream, info, 0, (int64_t)1));
    if (n == 0) return 0;
    const size_t need = sizeof(double) * 64 * 64;
    WorkGuard g;
    double *rinv = (double *)work;
    if (!rinv) {
        if (hipMallocAsync((void **)&rinv, need, stream) != hipSuccess) return HQR_ENOMEM;
        g.ptr = rinv;
        g.s = stream;
    } else if (lwork < (int64_t)need) {
        return HQR_ENOMEM;
    }
    for (int64_t k0 = 0; k0 < n; k0 += 64) {
        const int bw = (int)std::min<int64_t>(64, n - k0);
        HQR_CK(k_chol_block(stream, S, lds, n, k0, bw, rinv, info));
    }
    return 0;
}

int hqr_chol_update(int64_t n, double *R, int64_t ldr, double *v, hipStream_t stream)
{
    if (n < 0) return -1;
    if (ldr < std::max<int64_t>(1, n)) return -3;
    if (n > 0 && !R) return -2;
    if (n > 0 && !v) return -4;
    if (n > 4096) return HQR_ENOTSUP;
    if (n == 0) return 0;
    HQR_CK(k_chol_update(stream, R, ldr, v, n));
    return 0;
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
    HQR_CK(k_fill_int(stream, info, 0, (int64_t)1));
    if (iters) HQR_CK(k_fill_int(stream, iters, 0, (int64_t)1));
    if (n == 0 || nrhs == 0) return 0;
    const double tol = (opt && opt->tol > 0.0) ? opt->tol : 1e-13;
    const int max_iter = (opt && opt->max_iter >= 0) ? opt->max_iter : 10;
    const bool async = no_fallback(opt);
    Plan pl = make_plan(m, n, nrhs, NB, true);
    WorkGuard g;
    Work w;
    int rc = get_work(pl, work, lwork, stream, g, &w);
    if (rc) return rc;
    HQR_CK(hipMemcpy2DAsync(w.borig, sizeof(double) * m, B, sizeof(double) * ldb, sizeof(double) * m, nrhs,
                            hipMemcpyDeviceToDevice, stream));
    rc = apply_stored(pl, w, A, lda, up, B, ldb, nrhs, true, false, stream);
    if (rc) return rc;
    rc = backsolve_blocked(pl, w, A, lda, B, ldb, (int)nrhs, info, stream);
    if (rc) return rc;
    rc = mixed_refine(pl, w, A, lda, B, ldb, nrhs, resnorm, tol, max_iter, A_orig, lda_orig, stream, info, iters,
                      async);
    if (rc || async) return rc;
    bool converged = true;
    rc = read_verdict(w, nrhs, stream, &converged);
    if (rc || converged) return rc;
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
    HQR_CK(k_or_int(stream, info, HQR_INFO_NOCONV));
    return 0;
}

int hqr_tune_set(int op, int64_t m_lo, int64_t m_hi, int64_t n_lo, int64_t n_hi, int precision, int choice)
{
    if (op != HQR_TUNE_SINGLE && op != HQR_TUNE_BATCHED && op != HQR_TUNE_OCCUPANCY) return -1;
    if (m_lo < 0) return -2;
    if (m_hi < m_lo) return -3;
    if (n_lo < 0) return -4;
    if (n_hi < n_lo) return -5;
    if (precision != HQR_PREC_FP64 && precision != HQR_PREC_MIXED) return -6;
    int cnt = 0;
    (void)wg_variants(&cnt);
    if (op == HQR_TUNE_OCCUPANCY) {
        if (choice < 1 || choice > 8) return -7;
    } else {
        if (choice < (op == HQR_TUNE_SINGLE ? -1 : 0) || choice >= cnt) return -7;
        if (op == HQR_TUNE_BATCHED && !batch_variant(wg_variants(&cnt)[choice])) return -7;
    }
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
