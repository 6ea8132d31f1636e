// Kernel argument blocks and launchers of libmsb (internal).
#pragma once

#include "common.h"

namespace msb {

enum { EPI_PLAIN = 0, EPI_MV = 1, EPI_MV_Y = 2, EPI_SV = 3, EPI_MVN = 5, EPI_SV2 = 7 };
// epilogues that write partials (EPI_MVN: EPI_MV without the <r~, out> term,
// which a sparse list supplies)
__host__ __device__ constexpr bool epi_dots(int e) { return e == EPI_MV || e == EPI_MVN; }

// A per-right-hand-side complex coefficient in device memory: the value for
// rhs r is *(const double2 *)(p + r * stride).
struct CoefRef {
    const char *p = nullptr;
    long stride = 0;
};
__device__ inline double2 ld(const CoefRef &c, int rhs) {
    return *(const double2 *)(c.p + (long)rhs * c.stride);
}

template <typename T>
struct DslashArgs {
    const C<T> *in = nullptr;
    C<T> *out = nullptr;
    const C<T> *U = nullptr;   // [4][3][3][V]
    Geom g{};
    T diag = 0, ef = 1, eb = 1, bc = -1;
    int g5out = 0;
    T scale = 1, sigma0 = 0;
    const double *sigma0_rhs = nullptr;  // if set: per-rhs sigma0 (overrides sigma0)
    const C<T> *v = nullptr;   // EPI_MV*: + sigma0 * v
    const C<T> *rt = nullptr;  // EPI_MV: partials of <rt, out>
    double *part = nullptr;    // [rhs][PMAX][ps]
    long ps = NBMAX;           // partial row stride
    int nsb = 0;               // site blocks (set by the launcher)
    int per = 0;               // blocks per XCD in the flattened grid (set by the launcher)
    int sstride = 0;           // site-loop stride (set by the launcher)
    int nrhs = 0;
    int nch = 0;               // chunked stencil: 64-site chunks (set by the launcher)
    int tsc = 0;               // chunked stencil: chunks per t-slice, 0 if not whole
    int per_t = 0;             // chunked stencil: blocks per XCD (per rounded up to tsc)
    CoefRef ycoef;             // EPI_MV_Y: coefficient of the Mv output
    double2 *y = nullptr;      // EPI_MV_Y accumulator (always FP64)
    const C<T> *w = nullptr;   // EPI_SV2: subtracted from the output
    long w_rs = 0;
    Gate gate{};
    // element strides between right-hand sides (0: 12 V)
    long in_rs = 0, out_rs = 0, v_rs = 0, rt_rs = 0, y_rs = 0;
};

// One block per (256-site block, right-hand side); the launcher sets nsb, per
// and nrhs.
template <typename T>
void launch_dslash(hipStream_t st, DslashArgs<T> a, int nrhs, int epi, bool g5in);
// Timing of the next launch_dslash on this host thread: its kernel is
// dispatched with start and stop events that the dispatch itself records
// (no event packets of their own on the stream around it).  stencil_timing_
// taken() reports, and clears, whether a launch consumed the pair.
void stencil_timing_arm(hipEvent_t start, hipEvent_t stop);
bool stencil_timing_taken();

// Launch geometry of the site-block stencil: sets nsb, nrhs, per and sstride
// and returns the number of (virtual) blocks, 8 per, so that block p runs on
// XCD p % 8.
template <typename T>
inline long dslash_prepare(DslashArgs<T> &a, int nrhs) {
    a.nsb = (a.g.V + BLOCK - 1) / BLOCK;
    a.nrhs = nrhs;
    const long G = (long)a.nsb * nrhs;
    a.per = (int)((G + 7) / 8);
    a.sstride = 1 << 30;
    return 8L * a.per;
}

// Batches of at least this many right-hand sides use the chunked stencil,
// which stages the links of 64 sites in LDS once for all of them.
constexpr int CHUNK_MIN_RHS = 4;
constexpr int CHUNK = 64;
// Launch geometry of the chunked stencil (blocks = 8 per_t).
template <typename T>
inline long dslash_chunk_prepare(DslashArgs<T> &a, int nrhs) {
    a.nrhs = nrhs;
    a.nch = (a.g.V + CHUNK - 1) / CHUNK;
    a.per = (a.nch + 7) / 8;
    const int sites_t = a.g.Lx * a.g.Ly * a.g.Lz;
    a.tsc = (sites_t % CHUNK == 0) ? sites_t / CHUNK : 0;
    a.per_t = a.tsc ? ((a.per + a.tsc - 1) / a.tsc) * a.tsc : a.per;
    a.sstride = 1 << 30;
    return 8L * a.per_t;
}

// link force: pairs (c, p, q), the gradient of sum c Re <p, D(mu) q>
struct LinkPair {
    const double2 *p = nullptr, *q = nullptr;
    long p_rs = 0, q_rs = 0;   // element strides between right-hand sides (0: 12 V)
    double c = 0;
    int g5p = 0;               // use gamma5 p instead of p
};
constexpr int MAX_PAIRS = 4;
struct LinkForceArgs {
    Geom g{};
    double ef = 1, eb = 1, bc = -1;
    int npair = 0, nrhs = 1;
    LinkPair pairs[MAX_PAIRS];
    double2 *G = nullptr;      // [4][3][3][V], accumulated (+=)
};
void launch_link_force(hipStream_t st, const LinkForceArgs &a);
// Per block of 256 links (U [4][3][3][V], 4V links), the largest Gershgorin
// bound max_k (Re M_kk + sum_{l != k} |M_kl|) of M = U^+ U over its links: an
// upper bound of ||U||_2^2 (exactly 1 up to rounding for unitary links).
// blockmax: device [nblk], nblk = ceil(4V / 256).
void launch_link_gershgorin(hipStream_t st, const double2 *U, int V, double *blockmax);
inline int link_gershgorin_blocks(int V) { return (4 * V + 255) / 256; }

// ---- vector kernels ------------------------------------------------------
template <typename T>
struct VecArgs {
    long n = 0;                 // elements (complex) per vector = 12 V
    int l = 0;                  // MR degree (vectors R_0..R_l, U_0..U_l)
    int nshift = 0;             // shifts per rhs in the shift arrays
    C<T> *R = nullptr;          // [rhs][l+1][n]
    C<T> *U = nullptr;          // [rhs][l+1][n]
    C<T> *W = nullptr;          // [rhs][nshift][l+1][n]  (pass 1)
    double2 *X = nullptr;       // [rhs][nshift][n] shift solutions, FP64 (pass 1)
    double2 *XH = nullptr;      // [rhs][n] seed solution, FP64 (reliable updates)
    const C<T> *rt = nullptr;   // [rhs][n] shadow residual
    double *part = nullptr;
    long ps = NBMAX;            // partial row stride
    const SeedState *seed = nullptr;
    const StepCoef *sc = nullptr;   // [rhs][NSMAX]
    const MRCoef *mc = nullptr;     // [rhs][NSMAX]
    CoefRef beta, alpha;
    CoefRef gam;                // gamma_1 at gam, gamma_i at gam.p + (i-1)*16
    int partials = 1;
    Gate gate{};
    // deferred single pass
    C<T> *Bm = nullptr;         // [rhs][2l+2][n] the outer iteration's basis
    C<T> *W0 = nullptr;         // [rhs][nshift][n] u^s_0 of every shift
    const DeferCoef *dc = nullptr;  // [rhs][NSMAX]
    // pseudo-double pass: an Mv output is written to the store only, and is
    // read from there (not from R / U) until its first update; index -1: none
    const C<T> *r_src = nullptr;
    long r_src_rs = 0;
    int r_src_i = -1;
    const C<T> *u_src = nullptr;
    long u_src_rs = 0;
    int u_src_i = -1;
    // the MR step of the pseudo-double pass and of the deferred single pass
    // (mr_dyn = 1): r_L and u_L, L the BiCG steps the outer iteration
    // completed, are read from the iteration's store slots (slot t at
    // st_base + rhs * st_rs + t n) unless a step updated them since: r_L
    // always (its first update would be step L's r-update), u_L unless step
    // L made its u-step before a gamma breakdown
    const C<T> *st_base = nullptr;
    long st_rs = 0;
    int mr_dyn = 0;
};

// Basis form of the seed (MSB_SEED_BASIS, FP64): the vectors of the basis
// kernels.  Vector b of the outer iteration's basis (see SeedBasis) of right-
// hand side r is at bv[b] + r * brs[b].
template <typename T>
struct BasisArgs {
    long n = 0;
    int l = 0;
    Gate gate{};
    const C<T> *bv[NBB] = {};
    long brs[NBB] = {};
    const SeedBasis *sb = nullptr;    // [rhs]
    const SeedState *seed = nullptr;
    double *part = nullptr;
    long ps = NBMAX;
    // axpy: dst = x - c y with c per right-hand side; ||dst||^2 into partial
    // row prow when prow >= 0
    C<T> *dst = nullptr;
    long dst_rs = 0;
    const C<T> *x = nullptr;
    long x_rs = 0;
    const C<T> *y = nullptr;
    long y_rs = 0;
    CoefRef c{};
    int prow = -1;
    // r_0 from the basis: the first nbu basis vectors, ||r_0||^2 into row 3
    int nbu = 0;
    // MR update: r_0 and u_0 written over B_0 and B_1; <r~, r_0> (rt, or left
    // at zero for the sparse list) and ||r_0||^2 into rows 0..2
    C<T> *R0 = nullptr;
    C<T> *U0 = nullptr;
    long r0_rs = 0, u0_rs = 0;
    const C<T> *rt = nullptr;
    // MR update with a sparse r~ (wu set): <r~, r_0> from r_0 at the list's
    // entries (into rows 0, 1), the next outer iteration's beta from it
    // (seed_w[rhs].beta_spec) and u_0 = r_0 - beta u_0 into wu ([rhs][n])
    C<T> *wu = nullptr;
    SeedState *seed_w = nullptr;
    const long *sp_idx = nullptr;     // [rhs][sp_max]
    const double2 *sp_val = nullptr;  // [rhs][sp_max]
    const int *sp_cnt = nullptr;      // [rhs], at most SPARSE_MAX
    int sp_max = 0;
};
void launch_basis_axpy(hipStream_t, const BasisArgs<double> &, int nrhs, int nblk);
// replay of the double pass in basis form: r_0, u_0 after outer iteration
// m from the basis with the coefficients of sc_basis_replay (sb[rhs].r[0],
// u[0], over the first sb[rhs].nbu basis vectors), written over B_0, B_1
void launch_basis_combine(hipStream_t, const BasisArgs<double> &, int nrhs, int nblk);
void launch_basis_r0norm(hipStream_t, const BasisArgs<double> &, int nrhs, int nblk);
void launch_basis_gram(hipStream_t, const BasisArgs<double> &, int nrhs, int nblk);
void launch_basis_mr_update(hipStream_t, const BasisArgs<double> &, int nrhs, int nblk);
// sparse r~: <r~, r_0> after the MR step and the next iteration's beta, from
// the basis before the MR update (one block per right-hand side)
void launch_basis_spec(hipStream_t, const BasisArgs<double> &, int nrhs);

// mode: 0 u_0..u_j, 1 u_j only, 2 u_0..u_{j-1} (see seed_u_body)
template <typename T> void launch_seed_u(hipStream_t, const VecArgs<T> &, int j, int nrhs, int nblk, int mode = 0);
// fused: the r-update also applies the step's deferred u_0..u_{j-1} update
template <typename T>
void launch_r_update(hipStream_t, const VecArgs<T> &, int j, bool shifts, bool xh, int nrhs, int nblk,
                     bool fused = false);
template <typename T> void launch_gram(hipStream_t, const VecArgs<T> &, int nrhs, int nblk);
template <typename T> void launch_mr_update(hipStream_t, const VecArgs<T> &, bool shifts, bool xh, int nrhs, int nblk);
// reliable update: r_0 = b - v (v = S x in FP64), partials <rt, r_0>, ||r_0||^2
// (optionally y += c v with c from yc)
template <typename T> void launch_rel_update(hipStream_t, const VecArgs<T> &, const double2 *b, const double2 *v,
                                             double2 *y, CoefRef yc, int nrhs, int nblk);

// deferred single pass: B_0 <- r_0, B_1 <- u_0 at the start of an outer
// iteration; once per iteration, u^s_0 and x^s of every active shift from B
template <typename T> void launch_snapshot(hipStream_t, const VecArgs<T> &, int nrhs, int nblk);
template <typename T> void launch_defer_update(hipStream_t, const VecArgs<T> &, int nrhs, int nblk);

// pseudo-double pass: y += sum over outer iterations m0 .. m0+mc-1 of this
// storage chunk of cu V^u_{m,j} + cr V^r_{m,j} (replay coefficients, step flags)
// and, when rel is given, crel S x_m of the reliable updates.
// V: [rhs][chunk slots][2l][n] (v_rs between rhs); rel: [chunk slots][rhs][n]
// FP64 (rel_ms between slots).
template <typename T>
void launch_pstore_sum(hipStream_t, double2 *y, const C<T> *V, long v_rs, const double2 *rel, long rel_ms,
                       const ReplayStep *rs, const ReplayOuter *ro, int Mcap, int l, int m0, int mc, long n,
                       int nrhs, int nblk);

// small utility kernels
template <typename T>
void launch_convert_in(hipStream_t, C<T> *dst, const double2 *src, long n, long dst_stride,
                       long src_stride, int nrhs);
template <typename T>
void launch_convert_out(hipStream_t, double2 *dst, const C<T> *src, long n, long dst_stride,
                        long src_stride, int nrhs);
template <typename T>
void launch_zero(hipStream_t, C<T> *dst, long n, long stride, int nrhs);

// sparse shadow residual: index list of the nonzero entries of v ([nrhs] rows
// of n at stride rs), at most spmax per row, in index order.  Returns the
// largest row count (the list is written only when it is <= spmax), or -1 on
// a HIP error.  work: nrhs * nb ints.  Synchronises the stream.
int sparse_list(hipStream_t, const double2 *v, long n, long rs, int nrhs, int spmax, long *idx, double2 *val,
                int *cnt, int *work, int nb, bool fp32 = false);
struct SparseDotArgs {
    const long *idx = nullptr;      // [nrhs][spmax]
    const double2 *val = nullptr;   // [nrhs][spmax]
    const int *cnt = nullptr;       // [nrhs]
    int spmax = 0;
    const void *x = nullptr;        // the vector dotted with r~, rhs stride x_rs (elements)
    long x_rs = 0;
    int fp32 = 0;                   // x holds float2 (mixed precision)
    const double2 *b = nullptr;     // set: dot with b - v instead (FP64, rhs stride x_rs)
    const double2 *v = nullptr;
    double *part = nullptr;
    long ps = 0;
    Gate gate{};
};
void launch_sparse_dot(hipStream_t, const SparseDotArgs &, int nrhs);
template <typename T>
void launch_dot_partials(hipStream_t, const C<T> *x, const C<T> *y, long n, double *part, long ps,
                         int nrhs, int nblk, Gate gate);
template <typename T>
void launch_diffnorm_partials(hipStream_t, const C<T> *x, const C<T> *y, long n, long sx, long sy,
                              double *part, long ps, int nrhs, int nblk);
// y[rhs] = sum_s w[rhs][s] X[rhs][s]   (X stride n per shift, nshift per rhs)
void launch_ysum(hipStream_t, double2 *y, const double2 *X, const double *w, long n, int nshift,
                 int nrhs, int nblk);
// per (rhs, shift): Re <eta_r, x_rs> and Re <z_rs, x_rs> partials into
// out[((rhs * ns + s) * 2 + k) * nblk + block]
void launch_shift_dots(hipStream_t, const double2 *eta, const double2 *X, const double2 *Z, long n, int ns,
                       int nrhs, int nblk, double *out);
// R[rhs] = b[rhs] - t[rhs] (b rows b_rs apart, t and R rows n apart),
// partial slot 0 = ||R||^2
void launch_residual(hipStream_t, double2 *R, const double2 *b, long b_rs, const double2 *t, long n,
                     double *part, long ps, int nrhs, int nblk);
// y[rhs] = c[rhs] * b[rhs]
void launch_yinit(hipStream_t, double2 *y, const double2 *b, const double2 *c, long n, int nrhs,
                  int nblk);
// out = b + gamma5 w   (overlap), or out = s * w
void launch_overlap_out(hipStream_t, double2 *out, const double2 *b, const double2 *w, long V,
                        int nrhs, int overlap, double s, int nblk);
// vector axpy with a host scalar: y += a * x over n complex
void launch_axpy_host(hipStream_t, double2 *y, const double2 *x, double2 a, long n, int nblk);

// ---- scalar (single block per rhs) kernels --------------------------------
struct ScalarArgs {
    SeedState *seed = nullptr;
    ShiftState *sh = nullptr;       // [rhs][NSMAX]
    StepCoef *sc = nullptr;
    MRCoef *mc = nullptr;
    TapeStep *tape = nullptr;       // [rhs][max_steps]
    double2 *tape_gam = nullptr;    // [rhs][max_outer][LMAX]
    TapeOuter *tape_outer = nullptr;  // [rhs][max_outer]
    const double *part = nullptr;
    long ps = NBMAX;                // partial row stride
    int nblk = 0;                   // blocks that wrote the partials consumed
    int nblk2 = 0;                  // blocks of the second partial source
    int l = 0;
    int j = 0;
    int record = 0;                 // record the tape (double-pass)
    StepCoef *sc_hist = nullptr;    // deferred: [rhs][LMAX][NSMAX] every step's shift coefficients
    DeferCoef *dc = nullptr;        // deferred: [rhs][NSMAX] the iteration's coefficients
    int shadow = 0;                 // init: ||r~|| from partial row 5 (r~ other than b)
    // basis form (MSB_SEED_BASIS)
    int basis = 0;
    int spec = 0;                   // the MR update forms the next u_0 update (sparse r~)
    double norm_a = 0;              // an upper bound of ||S|| (2-norm)
    SeedBasis *sb = nullptr;        // [rhs]
};

void launch_sc_init(hipStream_t, const ScalarArgs &, int nrhs);
void launch_sc_beta(hipStream_t, const ScalarArgs &, int nrhs);
void launch_sc_alpha(hipStream_t, const ScalarArgs &, int nrhs);
void launch_sc_mr(hipStream_t, const ScalarArgs &, int nrhs);
void launch_sc_conv(hipStream_t, const ScalarArgs &, int nrhs);
void launch_sc_rel(hipStream_t, const ScalarArgs &, int nrhs);
void launch_sc_defer(hipStream_t, const ScalarArgs &, int nrhs);
void launch_sc_basis(hipStream_t, const ScalarArgs &, int nrhs);
// Replay of the double pass in basis form: outer iteration m's recorded step
// coefficients and MR coefficients (rs [rhs][Mcap][l], ro [rhs][Mcap]) as the
// combined coefficients of r_0 and u_0 after the iteration (sb[rhs])
struct BasisReplayArgs {
    const ReplayStep *rs = nullptr;
    const ReplayOuter *ro = nullptr;
    int Mcap = 0, l = 0, m = 0;
    SeedBasis *sb = nullptr;
};
void launch_sc_basis_replay(hipStream_t, const BasisReplayArgs &, int nrhs);
void launch_sc_exh(hipStream_t, const ScalarArgs &, int nrhs);

// ---- persistent execution --------------------------------------------------
// The stages of a solve, recorded as a table of operations that one
// cooperative launch executes in order, with a grid-wide barrier between
// consecutive operations.  Each operation is split into virtual blocks (the
// blocks its own launch would have had); resident block b takes the virtual
// blocks b, b + P, b + 2P, ... (P, the resident grid, is a multiple of 8, so
// a virtual block stays on the XCD its own launch would have used).
enum OpKind : int {
    OP_DS = 1,        // stencil in the iteration's precision (blob: DslashArgs<T>)
    OP_DS64,          // FP64 stencil of a reliable update (blob: DslashArgs<double>)
    OP_SEED_U,        // blob: VecArgs<T>
    OP_R_UPDATE,
    OP_GRAM,
    OP_MR_UPDATE,
    OP_REL_UPDATE,
    OP_SC_BETA,       // blob: ScalarArgs
    OP_SC_ALPHA,
    OP_SC_MR,
    OP_SC_REL,
    OP_SC_CONV,
    OP_SC_DEFER,      // per-stage launches only (the deferred single pass)
    OP_SC_BASIS,      // per-stage launches only (the basis form of the seed)
    OP_SC_EXH,
};
constexpr int POP_BLOB = 512;
struct alignas(16) POp {
    int kind = 0;
    int cls = 0;                 // timing class
    int epi = 0;                 // OP_DS, OP_DS64
    int j = 0;                   // OP_SEED_U, OP_R_UPDATE: BiCG step
    int shifts = 0;              // OP_R_UPDATE, OP_MR_UPDATE: update the shift vectors
    int nvb = 0;                 // virtual blocks
    int nblk = 0;                // vector ops: element blocks per right-hand side
    int pad = 0;
    const double2 *b = nullptr;  // OP_REL_UPDATE operands
    const double2 *v = nullptr;
    double2 *y = nullptr;
    CoefRef yc{};
    alignas(16) unsigned char blob[POP_BLOB];
};
constexpr int PERSIST_CLASSES = 8;
constexpr int PERSIST_GROUP = 32;      // blocks per first-level barrier group
constexpr int PERSIST_MAX_GROUPS = 64; // per XCD
// Barrier and timing state of a persistent launch (zeroed before it).
struct PersistCtl {
    unsigned long long bar;                              // XCD arrivals (one per XCD in use)
    int abort;                                           // set when a wait exceeds its bound
    int pad;
    unsigned long long ticks[PERSIST_CLASSES];           // wall-clock ticks per timing class
    unsigned long long execs[PERSIST_CLASSES];           // operations executed per class
    unsigned long long xbar[8], xrel[8];                 // per XCD: group arrivals, release
    unsigned long long gbar[8 * PERSIST_MAX_GROUPS];     // per group: block arrivals
    unsigned long long grel[8 * PERSIST_MAX_GROUPS];     // per group: release
    unsigned long long xcount[8];                        // census: blocks found on each XCD
    unsigned long long census;                           // census: blocks counted
};
struct PersistArgs {
    const POp *ops = nullptr;
    int nops = 0;                // operations per iteration of the table
    int iters = 1;               // repetitions of the table
    int loop = 0;                // 1: stop after a repetition when no seed runs
    const SeedState *seed = nullptr;
    int nrhs = 0;
    int timing = 0;              // record per-class stage times
    PersistCtl *ctl = nullptr;
};
// Largest co-resident grid of the persistent kernel of MR degree l (a
// multiple of 8; 0 when l is outside 1..PERSIST_LMAX).
constexpr int PERSIST_LMAX = 6;
template <typename T> int persistent_grid(int device, int l);
template <typename T> hipError_t launch_persistent(hipStream_t st, const PersistArgs &pa, int grid, int l);

}  // namespace msb
