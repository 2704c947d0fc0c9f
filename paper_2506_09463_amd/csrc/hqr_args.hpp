// hqr_args.hpp -- the interface between libhqr's host dispatch and its
// kernels: tile constants, the argument structures every kernel takes, and
// the host-side launch functions each kernel translation unit defines.
// (The kernels themselves live in hqr_blocked.hpp, hqr_cqr.hpp, hqr_wg.hpp
// and hqr_batched.hpp, each compiled in its own translation unit.)
#pragma once

#include "hqr.h"
#include "hqr_device.hpp"

namespace hqr {

constexpr int NB = 64;          // panel width

constexpr int PC_ROWS = 128;    // rows per workgroup in panel_col_kernel

constexpr int PW = NB + 2;      // partial vector: dots, max|x|, #nonzero

constexpr int KC = 32;          // rows per LDS chunk in vtc_kernel

// ------------------------------------------------------------------ panel
struct PanelArgs {
    double *A;
    int64_t lda;
    int64_t m;        // rows of A
    int c0;           // first column (and pivot row) of the panel
    int bw;           // panel width (<= NB)
    int k;            // launch index 0..bw
    int nchunk;       // workgroups (row chunks of PC_ROWS rows from c0)
    double *up;       // global up array (output for columns c0..c0+bw)
    double *xbuf;     // [2][nchunk][PW] partials
    double *pbuf;     // [2][NB] pivot rows
};

// ----------------------------------------------------- W = V^T X (partials)
// X columns: [0, bw) = V itself (gives G = V^T V), then ncA trailing columns
// of A starting at column c0+bw, then nB columns of B.
struct VtxArgs {
    const double *A;
    int64_t lda;
    const double *B;
    int64_t ldb;
    const double *up;
    int64_t m;
    int c0, bw;
    int ncA, nB;          // trailing A columns, B columns
    int aoff;             // first trailing A column is c0 + bw + aoff
    int nx;               // bw + ncA + nB
    int nxpad;            // row stride of the partial buffers
    int64_t split_rows;   // rows per split (multiple of KC)
    int with_v;           // include the bw V columns as X columns
    double *wpart;        // [nsplit][NB][nxpad]
};

// grid: (ceil(nx/128), nsplit); 256 threads.  Output tile: 64 reflectors x
// 128 X columns over the rows of one split.  Wave w owns reflector rows
// [16w, 16w+16) and all eight 16-column tiles.  Row chunks of KC rows are
// staged in LDS ([row][col]); the next chunk is prefetched into registers
// while the current one is multiplied.
constexpr int VTX_COLS = 128;

// ------------------------------------------------- T from G = V^T V and tau
// One workgroup.  tau_k = -1/(up_k R_kk) (0 for identity reflectors);
// T[j][j] = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] G[0:j, j].
struct TArgs {
    const double *A;
    int64_t lda;
    const double *up;
    int c0, bw;
    const double *wpart; // partials holding G in columns [0, bw)
    int nsplit, nxpad;
    double *T;           // [NB][NB] row-major T[i][j]
};

// ------------------------------------------------ W' = T^T (sum of partials)
// grid: ceil(ncols/64) over the X columns that get updated (offset xoff).
struct WArgs {
    const double *wpart;
    int nsplit, nxpad;
    int xoff, ncols;      // updated X columns [xoff, xoff+ncols)
    int bw;
    const double *T;
    double *wp;           // [NB][nxpad] row-major, same column indexing
    int tmode;            // 0: W' = T^T X (applying Q^T), 1: W' = T X (applying Q)
};

// grid: ceil(ncols/WS_COLS); 256 threads, WS_COLS columns per workgroup.
constexpr int WS_COLS = 16;

// Narrow form (at most 64 columns, many row splits): 4 columns per
// workgroup, thread (row i, column c) sums its partials 16 at a time.
constexpr int WSN_COLS = 4;

// ---------------------------------------------------------- X <- X - V W'
// grid: (ceil(rows/64), ceil(ncols/64)); 256 threads.  Tile 64 rows x 64
// columns, computed transposed (D' = W'^T V^T) so each accumulator register
// maps to 16 consecutive rows of one column.
struct UpdArgs {
    double *A;
    int64_t lda;
    double *B;
    int64_t ldb;
    const double *up;
    int64_t m;
    int c0, bw;
    int ncA, nB;          // updated A columns start at c0+bw+aoff; then B columns
    int aoff;
    int xoff;             // X index of the first updated column in wp
    const double *wp;     // [NB][nxpad]
    int nxpad;
};

// grid: (ceil(rows/128), ceil(ncols/128)); 256 threads.  Wave (wr, wc)
// owns rows [128 bx + 64 wr, +64) x columns [128 by + 64 wc, +64) and keeps
// that 64 x 64 block of X^T in 16 MFMA accumulators.  The fragments of W'
// and V are read straight from global memory (L2): each fragment load is
// four 128-byte segments.
constexpr int UPD_TILE = 128;

// Blocked back-substitution R X = B[0:n].  Row blocks of 64; workgroup b
// owns row block nblk-1-b, so every block it waits for belongs to a
// workgroup dispatched before it.  A block is published by storing its x
// values into xpub, whose slots hold the TRSV_EMPTY pattern until then: each
// value is its own flag, so a consumer's poll is the read of the data.  The
// wait is bounded: on expiry the kernel records HQR_INFO_TIMEOUT.
struct TrsvArgs {
    const double *A;
    int64_t lda;
    double *B;
    int64_t ldb;
    int64_t n;
    int nrhs;
    double *xpub;    // [nrhs][n], every slot TRSV_EMPTY on entry
    int *info;       // read: nonzero -> nothing to do; written on timeout
    long spin_limit;
    const int *active; // optional: nothing to do when *active == 0
};

constexpr int TRSV_MAXRHS = 8;
// A signalling NaN with a nonzero payload, the same 32-bit word twice (so the
// integer fill writes it).  Arithmetic returns only quiet NaNs, and a value
// that matched the pattern would be published as the default quiet NaN, so a
// slot that differs from it holds its block's final value.
constexpr unsigned long long TRSV_EMPTY = 0x7FF47FF47FF47FF4ull;
constexpr int TRSV_EMPTY_WORD = 0x7FF47FF4;

// Refinement of least-squares solutions with the semi-normal equations,
// every right-hand side at once (column c: x = X[0:n, c], original b =
// borig[:, c]):  r = b - A0 x,  g = A0^T r,  R^T z = g,  R dx = z,  x += dx.
// Per column stat[4c .. 4c+3] = {first converged step (1-based, 0 = not yet),
// failed, consecutive stalls, frozen}; a frozen column's x no longer changes.
// *active counts the columns still refining: every refinement kernel returns
// at once when it reaches 0.
struct RefineArgs {
    const double *A0;  // unmodified FP64 A (m x n)
    int64_t lda0;
    const double *borig; // m x nrhs, leading dimension m
    double *X;         // x in rows 0..n-1
    int64_t ldx;
    double *rvec;      // m x nrhs residuals, leading dimension m
    double *gvec;      // n x nrhs: A0^T r, then z, then dx (leading dimension n)
    int64_t m, n;
    int nrhs;
    double tol;        // converged when ||dx|| <= tol ||x||
    int max_iter;
    int *stat;         // [nrhs][4]
    double *dxprev;    // [nrhs] ||dx|| of the previous step
    int *active;
};

// A correction that stops shrinking is accepted as converged only at or
// below this fraction of ||x||.  Corrections that no longer shrink are the
// rounding noise of the iteration's fixed point, whose distance to the
// least-squares solution is of the same size (measured on MI355X at
// kappa = 1e6: stall level 4e-12..2e-11, solution error 0.5..1.4 times it),
// so the floor keeps the solution error below the 1e-10 relative target
// with a margin of about 3.  Above it the run counts as failed.
constexpr double REFINE_STALL_FLOOR = 3e-11;

constexpr int CQR_ROWS = 64;           // rows per workgroup in the Gram kernels

constexpr double CQR_RATIO = 1e-15;    // smallest accepted pivot^2 / G_kk

constexpr int LD65 = NB + 1;

// --------------------------------------- Gram partials (with the update)
// Pass 1, workgroup t owns rows rbase + 64t .. +63 (rbase = cp with the
// update, c0 without).  With `upd` it first applies the previous panel's
// compact-WY block to this panel's columns: C -= V W with W = T^T X, X = V^T C
// reduced over all rows (narrow_vtx_kernel + xw_reduce_kernel), V the
// previous panel's reflectors (rows from cp, width NB).  Then the rows at or
// below c0 give a Gram partial Z^T Z of the panel and its zero-tail mask.
struct Gram1Args {
    double *A;
    int64_t lda;
    int64_t m;
    int c0, bw;               // panel whose Gram is formed
    int upd, cp;              // apply the previous panel (start cp, width NB) first
    const double *up;         // stored up (the previous panel's part is read)
    const double *Wt;         // [NB][NB] W = T^T V^T C of the previous panel, transposed (upd)
    double *gpart;            // [tiles][NB][NB]
    unsigned long long *mask; // [tiles]
    const int *flag;
};

// --------------------------------------------------- pass-2 Gram partials
// Workgroup t: Q1 = A_p R1^{-1} on rows c0 + 64t .. +63 and its Gram partial;
// workgroup 0 also keeps the top bw x bw block of Q1.
struct Gram2Args {
    const double *A;
    int64_t lda;
    int64_t m;
    int c0, bw;
    const double *r1inv;
    double *q1top;
    double *gpart;
    const int *flag;
};

// ----------------------------------------------- partial Gram reduction
// G[e] = sum_q gpart[q][e] in a fixed order: 64 workgroups of 256 threads;
// thread (entry e, quarter g4) sums q = g4, g4+4, ..; quarters added 0..3.
// Workgroup 0 also ORs the zero-tail masks.
struct GredArgs {
    const double *gpart;
    int ngroups;
    double *G;
    const unsigned long long *mask;
    unsigned long long *mask_all;
    int with_mask;
    const int *flag;                     // nullptr: always run
};

// --------------------------------------------------------- Cholesky kernel
struct CholArgs {
    double *A;
    int64_t lda;
    int64_t m;
    int c0, bw;
    int pass;
    const double *G;                    // reduced Gram
    const unsigned long long *mask_all; // ORed zero-tail masks (pass 1)
    double *r1;         // [NB][NB]  (pass 1 out, pass 2 in)
    double *r1inv;      // [NB][NB]  (pass 1 out, pass 2 in)
    const double *q1top; // [NB][NB] (pass 2 in) top bw x bw block of A_p R1^{-1}
    double *winv;       // [NB][NB]  (pass 2 out) R^{-1} U^{-1} diag(up)
    double *T;          // [NB][NB]  (pass 2 out) T for the stored vectors
    double *up;         // global up (pass 2 out)
    int *flag;
    long long *tstamp;  // optional per-phase timestamps (thread 0), may be null
};

// ---------------------------------- bottom rows: Y_bot * diag(up) (standalone)
struct FinArgs {
    double *A;
    int64_t lda;
    int64_t m;
    int c0, bw;
    const double *winv;
    const int *flag;
};

// --------------------------- next panel's V^T C, finishing this panel's V
// For the look-ahead: panel p (start c0, width NB) has just been factored;
// its bottom rows still hold A_bot and become V_bot = A_bot W^{-1} here
// (unless the panel was flagged: the exact loop stored V itself).
// Workgroup t (rows c0 + 64t .. +63) writes its V rows back and the partial
// V_t^T C_t for the next panel's nc columns C (summed by gram_reduce_kernel;
// cqr_gram1_kernel applies the block).
struct NarrowArgs {
    double *A;
    int64_t lda;
    int64_t m;
    int c0, nc;
    const double *up;
    const double *winv;
    const int *flag;
    double *gpart;            // [tiles][NB][NB] out
};

// --------------------------------------------- W = T^T X for the look-ahead
// Workgroup j: column j of X = sum of the transposed partials of
// narrow_vtx_kernel (fixed order: thread (i, g4) sums q = g4, g4 + 4, ..;
// the quarters added 0..3), then column j of W = T^T X (T upper triangular,
// W[i][j] = sum_{l <= i} T[l][i] X[l][j]; thread (i, g4) takes l in
// [16 g4, 16 g4 + 16), the quarters added 0..3), stored transposed
// (Wt[j][i]).  Under 64 VGPRs, so it can start beside two bulk waves per SIMD.
struct XwArgs {
    const double *gpart;      // [parts][NB][NB], [q][j][i]
    int parts;
    const double *T;          // [NB][NB] row-major
    double *Wt;               // [NB][NB] out, Wt[j][i] = W[i][j]
};

constexpr int WG_P = 16;    // panel width

constexpr int WG_LD = 17;   // LDS row stride (doubles) of V and T

constexpr int WG_PIPE = 4;  // default 16-row blocks whose loads the trailing update issues together

// WG_FACTOR: factor A (B's columns ride along: Q^T B); without it A and up
// hold a stored factorization, which is applied to B: Q^T B, or Q B with
// WG_APPLY_Q (WG_QSKIP: B starts as leading columns of the identity, so
// panel p leaves B's columns before its first column untouched).  WG_SOLVE:
// residual norms and back-substitution after Q^T B.
enum : int64_t { WG_FACTOR = 1, WG_SOLVE = 2, WG_APPLY_Q = 4, WG_QSKIP = 8 };

struct WgDesc {
    int64_t m, n, nrhs, lda, ldb;
    double *A;
    double *B;       // may be null when nrhs == 0
    double *up;
    double *resnorm; // may be null
    int64_t index;   // info slot
    int64_t flags;   // WG_FACTOR | WG_SOLVE
};

struct BatchDesc {
    int64_t m, n, nrhs, lda, ldb;
    double *A;
    double *B;
    double *up;
    double *resnorm; // may be null
    int64_t index;   // position in the caller's arrays (info slot)
    int64_t factor;  // 1: factor A (B fused); 0: A, up hold a stored factorization
};

struct BatchArgs {
    const BatchDesc *desc;
    int count;
    int *head;       // zero on entry
    int *info;       // [count], caller order
    int max_ntot;    // largest n + nrhs in the batch (<= BATCH_MAX_COLS)
};

// ---------------------------------------------------------------- TSQR
// One level of the TSQR tree of a panel (bw columns): `rows` rows of X
// (column-major, leading dimension ldx) in nblk row blocks, block i of
// base + (i < rem) rows starting at row i * base + min(i, rem).  Level 0 is
// the panel itself; level l + 1 stacks the bw x bw R factors of level l's
// blocks (block i at rows i * bw).  Q (ldq) receives the level's explicit
// orthonormal factor, up the blocks' reflector pivots (64 per block), fdesc
// and adesc the one-workgroup descriptors that factor the blocks and apply
// their reflectors.
constexpr int TSQR_MAX_LEVELS = 8;
constexpr int64_t TSQR_LEAF_ROWS = 1024;   // rows per block at most (one-workgroup limit)

struct TsqrLevel {
    int64_t rows, nblk, base, rem;
    double *X;
    int64_t ldx;
    double *Q;
    int64_t ldq;
    double *up;
    WgDesc *fdesc;
    WgDesc *adesc;
};

struct TsqrArgs {
    int *flag;          // the panel's flag: 1 (exact zero tail) skips the panel
    int bw, nlev;
    TsqrLevel lev[TSQR_MAX_LEVELS];
    int *heads;         // 2 * nlev queue heads, zeroed by the descriptor kernel
};

// first row and row count of block i of a level
__host__ __device__ inline int64_t tsqr_block_start(const TsqrLevel &L, int64_t i)
{
    return i * L.base + (i < L.rem ? i : L.rem);
}
__host__ __device__ inline int64_t tsqr_block_rows(const TsqrLevel &L, int64_t i)
{
    return L.base + (i < L.rem ? 1 : 0);
}

constexpr int BATCH_MAX_ROWS = 4096;

constexpr int BATCH_MAX_COLS = 2048;

constexpr int BATCH_NW = 16;

// ------------------------------------------------------------ profiling
// Kernel classes of the optional per-launch event timing (hqr_profile_*).
enum KClass {
    K_SMALL, K_PANEL, K_VTX, K_TFACTOR, K_WSOLVE, K_UPDATE, K_DIAG, K_TRSV, K_RESNORM, K_FILL,
    K_GRAM1, K_GRAM2, K_GRED, K_CQR_CHOL, K_CQR_FINISH, K_NVTX, K_BATCHED, K_REFINE, K_TSQR, K_NCLASS
};
// Defined in hqr_lib.hip: while timing is on, every launch is bracketed by a
// pair of HIP events recorded on the launch's own stream.
hipEvent_t prof_begin(hipStream_t s);
void prof_end(int cls, hipEvent_t e0, hipStream_t s);

#define HQR_LAUNCH(cls, kern, grid, block, shmem, stream, ...)                     \
    do {                                                                           \
        hipEvent_t e0_ = ::hqr::prof_begin(stream);                                \
        hipLaunchKernelGGL(kern, grid, block, shmem, stream, __VA_ARGS__);         \
        ::hqr::prof_end(cls, e0_, stream);                                         \
    } while (0)

// ------------------------------------------------- launch functions
// Each returns hipGetLastError() after the launch.

// hqr_blocked.hpp (k_blocked.hip)
hipError_t k_panel_col(dim3 grid, hipStream_t s, const PanelArgs &a);
hipError_t k_vtx(bool f32, bool with_v, dim3 grid, hipStream_t s, const VtxArgs &a);
hipError_t k_tfactor(hipStream_t s, const TArgs &a);
hipError_t k_wsolve(bool narrow, dim3 grid, hipStream_t s, const WArgs &a);
hipError_t k_update(bool narrow, bool f32, dim3 grid, hipStream_t s, const UpdArgs &a);
hipError_t k_diag_check(hipStream_t s, const double *A, int64_t lda, int64_t n, int *info);
hipError_t k_trsv(bool trans, int nrhs, dim3 grid, hipStream_t s, const TrsvArgs &a);
hipError_t k_resnorm(dim3 grid, hipStream_t s, const double *B, int64_t ldb, int64_t n, int64_t m, double *out);
hipError_t k_fill_int(hipStream_t s, int *p, int v, int64_t count);
hipError_t k_or_int(hipStream_t s, int *p, int v);
hipError_t k_eye(hipStream_t s, double *Q, int64_t ldq, int64_t m, int64_t k);
hipError_t k_refine_init(hipStream_t s, const RefineArgs &a);
hipError_t k_resid(bool all, hipStream_t s, const RefineArgs &a);
hipError_t k_gemvt(hipStream_t s, const RefineArgs &a);
hipError_t k_csne_update(hipStream_t s, const RefineArgs &a, int step);
hipError_t k_refine_verdict(hipStream_t s, const RefineArgs &a, int *verdict, int *info, int *iters, bool or_info);

// hqr_cqr.hpp (k_cqr.hip)
hipError_t k_cqr_gram1(dim3 grid, hipStream_t s, const Gram1Args &a);
hipError_t k_cqr_gram2(dim3 grid, hipStream_t s, const Gram2Args &a);
hipError_t k_gram_reduce(hipStream_t s, const GredArgs &a);
hipError_t k_cqr_chol(hipStream_t s, const CholArgs &a);
hipError_t k_cqr_finish(dim3 grid, hipStream_t s, const FinArgs &a);
hipError_t k_narrow_vtx(dim3 grid, hipStream_t s, const NarrowArgs &a);
hipError_t k_xw_reduce(hipStream_t s, const XwArgs &a);

// hqr_wg.hpp (k_wg.hip): one-workgroup kernel variants "wgNTxQM" (NT
// threads holding QM rows each)
struct WgVariant {
    const char *name;
    int nt, qm, pipe;
    int per_cu;         // workgroups per CU the LDS allows
    int64_t max_rows, max_x;
    int index;          // position in wg_variants()
};
const WgVariant *wg_variants(int *count);
hipError_t k_wg_single(const WgVariant *v, hipStream_t s, const WgDesc &d, int *info);
hipError_t k_wg_batched(const WgVariant *v, int grid, hipStream_t s, const WgDesc *desc, int count, int *head,
                        int *info);

// hqr_tsqr.hpp (k_tsqr.hip)
hipError_t k_tsqr_desc(hipStream_t s, const TsqrArgs &a);
hipError_t k_tsqr_gather(hipStream_t s, const TsqrArgs &a, int l);
hipError_t k_tsqr_scatter(hipStream_t s, const TsqrArgs &a, int l);
// D R and the identity into r1 / r1inv, the signs D into sign; then the
// panel := Q D (two launches)
hipError_t k_tsqr_final(hipStream_t s, const TsqrArgs &a, double *Ap, int64_t lda, double *r1, double *r1inv,
                        double *sign);


// hqr_lse.hpp (k_lse.hip)
hipError_t k_transpose(hipStream_t s, const double *in, int64_t ldi, double *out, int64_t ldo, int64_t rows,
                       int64_t cols);
hipError_t k_gemv_sub(hipStream_t s, const double *M, int64_t ldm, const double *y, double *b, int64_t m,
                      int64_t p);
hipError_t k_copy_vec(hipStream_t s, const double *src, double *dst, int64_t n);
hipError_t k_lse_info(hipStream_t s, int *info, const int *info_c, const int *info_r, int64_t p);

// hqr_chol.hpp (k_chol.hip): one 64-column block step of the Cholesky
// factorization (diagonal block, block row, trailing update); the rank-one
// update (n <= 4096)
hipError_t k_chol_block(hipStream_t s, double *S, int64_t lds, int64_t n, int64_t k0, int bw, double *rinv,
                        int *info);
hipError_t k_chol_update(hipStream_t s, double *R, int64_t ldr, double *v, int64_t n);

// hqr_batched.hpp (k_batched.hip)
hipError_t k_batched_lsq(dim3 grid, hipStream_t s, const BatchArgs &a);

} // namespace hqr
