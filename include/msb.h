/*
 * msb.h -- multi-shift BiCGstab(l) for the overlap operator at nonzero
 * chemical potential, on AMD Instinct MI355X (gfx950).
 *
 * The library evaluates the partial-fraction expansion (PFE)
 *
 *     f(A) b  ~  y = sum_s w_s (A + sigma_s)^{-1} b,          (Eq. 1.2)
 *
 * for A = a (gamma5 D_w(mu))^2 with one Krylov space for all shifts
 * (shift invariance, Section 1), in the single-pass form, the double-pass
 * form of Section 2 (option 1 after Eq. 2.2; Section 5) and the
 * pseudo-double-pass form (option 2 after Eq. 2.2), and
 * from it sign(H) b and the overlap operator D_ov = 1 + gamma5 sign(H)
 * (Eq. 1.1).  D_w(mu): the Wilson stencil, mu entering as e^{+-mu} on the
 * time links:
 *
 *   (D psi)(x) = (4+m) psi(x)
 *     - 1/2 sum_nu b_nu(x)   (1-gamma_nu) e^{+mu d_nu4} U_nu(x)     psi(x+nu)
 *     - 1/2 sum_nu b_nu(x-nu)(1+gamma_nu) e^{-mu d_nu4} U_nu(x-nu)^+ psi(x-nu)
 *
 * with b_4 = bc_t on the links from t = Lt-1 to t = 0 and 1 elsewhere, and
 * chiral gamma matrices gamma_k = [[0,-i sigma_k],[i sigma_k,0]],
 * gamma_4 = [[0,1],[1,0]], gamma5 = diag(1,1,-1,-1).
 *
 * Layouts (all complex numbers are interleaved (re, im) pairs of doubles,
 * i.e. complex128):
 *   site     s = x + Lx*(y + Ly*(z + Lz*t))
 *   spinor   [nrhs][k][V], k = 3*spin + colour (12 per site)
 *   links    [nu][a][b][V], nu = 0..3 for x, y, z, t; U_nu(x)_{ab}
 *
 * Ownership: every vector and link pointer is a DEVICE pointer owned by the
 * caller; the library never keeps one after a call returns (links are copied
 * into the context by msb_create).  The library owns its workspace (seed
 * vectors, shift vectors, reduction partials, scalar state, the double-pass
 * tape) and grows it on demand.  Host arrays (shifts, weights, info arrays)
 * are read or written during the call only.
 *
 * Streams: every call is ordered on the context's stream (a hipStream_t given
 * at creation or by msb_set_stream; NULL = the default stream).  Calls that
 * fill msb_solve_info or host gradient arrays synchronise that stream before
 * returning.
 *
 * Errors: every entry point returns an msb_status; no C++ exception crosses
 * the boundary.  Invalid arguments are rejected with MSB_ERR_ARG before any
 * work is queued.  msb_last_error() gives the calling thread's message for
 * its last non-zero status.
 */
#ifndef MSB_H
#define MSB_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MSB_OK = 0,
    MSB_ERR_ARG = 1,        /* invalid argument; nothing was launched          */
    MSB_ERR_HIP = 2,        /* a HIP runtime call failed                        */
    MSB_ERR_OOM = 3,        /* workspace allocation failed                      */
    MSB_NOT_CONVERGED = 4,  /* max_outer reached; y and info are still filled   */
    MSB_BREAKDOWN = 5,      /* BiCG/MR/shift breakdown; partial y is returned   */
    MSB_REDUCED_ACCURACY = 6 /* MSB_MIXED without MSB_REFINE: every shift met tol
                               on its recursive (FP32-updated) residual and the
                               seed's residual was recomputed in FP64, but the
                               shifts' FP64 true residuals are not shown to be
                               <= tol (they stall near eps_32 times the
                               condition number of A + sigma_s); y and info are
                               filled.  MSB_REFINE (pass 1) checks and
                               corrects every shift in FP64 instead.        */
} msb_status;

/* flags for wilson_apply */
#define MSB_G5_LEFT   1     /* out = gamma5 D in                                */
#define MSB_NEG_MU    2     /* use -mu instead of mu                            */
#define MSB_DAGGER    4     /* out = D^+ in  (= gamma5 D(-mu) gamma5 in)        */
/* flags for the solvers */
#define MSB_MIXED     8     /* FP32 stencil / vectors, FP64 reductions + scalars */
#define MSB_PERSISTENT 16   /* whole solve in one cooperative launch (batched)   */
#define MSB_OVERLAP   32    /* pfe_sign_apply: out = b + gamma5 sign(H) b        */
#define MSB_ADJOINT   64    /* solve with A^+ = A(-mu) (used by the backward)    */
#define MSB_DEFERRED  256   /* pass 1: shift vectors updated once per outer
                               iteration from its 2l+2 seed basis vectors (only
                               u^s_0 and x^s kept per shift)                   */
#define MSB_OP_WILSON 512   /* mshift_bicgstabl: A = a D_w(mu) (one stencil per
                               Mv) instead of a (gamma5 D_w)^2.  Wilson masses
                               differ by a shift, D_w(m + sigma) = D_w(m) +
                               sigma, so with a = 1 and sigma_s = m_s - m (m the
                               context's mass) the single pass's x_shifts are
                               the propagators of every mass from one Krylov
                               space.  Not with MSB_ADJOINT, pfe_sign_apply or
                               pfe_sign_backward (which need the Hermitian
                               kernel H = gamma5 D_w).                          */
#define MSB_SEED_BASIS 1024 /* pass 2, 3, or 1 with MSB_DEFERRED (FP64, not
                               MSB_MIXED or MSB_PERSISTENT):
                               the seed's BiCG steps of Section 2 update only
                               the two vectors the step's Mv reads; every
                               other r_i, u_i of the outer iteration is kept
                               as coefficients on its 2l+2 basis vectors (r_0,
                               u_0 and the Mv outputs) and formed from them
                               for the MR step; the double pass's replay
                               likewise.  Same iterates up to rounding, fewer
                               vector passes per outer iteration (about 2/3
                               of them at l = 4); + nrhs * n * 32 bytes of
                               workspace.                                     */
#define MSB_REFINE    128   /* pass 1: after the solve, the FP64 true residual of
                               every shift; shifts above tol get refinement
                               solves (A + sigma_s) d = r_s, x_s += d (<= 3
                               rounds) -- what makes MSB_MIXED reach tol      */

typedef struct msb_ctx msb_ctx;

typedef struct {
    int dims[4];            /* Lx, Ly, Lz, Lt (each >= 1)                        */
    double mass;            /* Wilson mass m: diagonal term 4 + m                */
    double mu;              /* chemical potential (e^{+mu} on forward t hops)    */
    int bc_t;               /* time boundary: -1 antiperiodic, +1 periodic       */
} msb_lattice;

/* Solve report.  All pointer members are optional caller-owned HOST arrays of
 * length nrhs * n_shift (index rhs * n_shift + s, shifts in caller order). */
typedef struct {
    int status;             /* the call's msb_status                             */
    int outer_iters;        /* max over right-hand sides of outer iterations M   */
    int bicg_steps;         /* max over RHS of BiCG steps (2 Mv each)           */
    long long mv_count;     /* total applications of A + sigma_0 (all RHS)       */
    long long dot_count;    /* inner products in the paper's counting            */
    long long axpy_count;   /* vector updates (y <- a x + y) actually executed    */
    int reliable_updates;   /* mixed precision: FP64 residual recomputations     */
    double bytes_model;     /* algorithmic HBM bytes of the call                 */
    int *shift_iters;       /* out: M_s, outer iterations until shift s froze    */
    double *shift_resid;    /* out: final collinear residual estimate            */
    double *shift_true_resid; /* out (pass 1 only): ||b-(A+sigma_s)x_s||/||b||   */
    const int *force_iters; /* in, test hook: freeze shift s after exactly
                               force_iters[...] outer iterations (no early exit) */
    int refined_shifts;     /* out (MSB_REFINE): (rhs, shift) refinement solves   */
    const void *shadow;     /* in, mshift_bicgstabl: DEVICE [nrhs][12][V]
                               complex128 shadow residual r~ of BiCGstab(l)
                               (any vector with <r~, b> != 0; NULL: r~ = b).
                               A point source with r~ = b breaks down under
                               MSB_OP_WILSON (D_w's hops change the site
                               parity); a random r~ avoids it.               */
    int stored_iters;       /* out (pass = 3): outer iterations whose Mv outputs
                               were kept in the store; those after them were
                               regenerated (see msb_set_store_limit); -1 for
                               the other passes                             */
} msb_solve_info;

/* Create a context on the current HIP device.  links: device pointer to
 * [4][3][3][V] complex128 gauge links (copied; FP64 and FP32 internal copies).
 * stream: hipStream_t (may be NULL). */
int msb_create(msb_ctx **ctx, const msb_lattice *lat, const void *links,
               void *stream);
void msb_destroy(msb_ctx *ctx);
int msb_set_stream(msb_ctx *ctx, void *stream);
const char *msb_last_error(void);

/* Neuberger PFE of x^{-1/2} (Fig. 1 caption): theta_s = pi (s - 1/2)/(2n),
 * sigma_s = tan^2 theta_s, w_s = 1/(n cos^2 theta_s), s = 1..n.  Host arrays
 * of length n. */
int msb_neuberger_pfe(int n, double *sigma, double *weight);

/* Power-iteration estimate of lambda_max(D^+ D) from the device start vector
 * start [12][V] complex128: Rayleigh quotient after iters normalised steps.
 * The scale convention of the solvers is a_scale = 1 / (1.01 * rho). */
int msb_spectral_radius(msb_ctx *ctx, const void *start, int iters, double *rho);

/* Device memory the pseudo-double pass (pass = 3) of this context may use
 * for its store of Mv outputs, in bytes; 0 (the default): whatever can be
 * allocated.  The store grows by chunks of 8 outer iterations; once the next
 * chunk would pass the limit (or cannot be allocated), no further iteration
 * is stored: the first pass continues as the double pass's first pass (the
 * seed's state at that iteration is kept), and after the sweep y is
 * completed by replaying the remaining iterations from that state (Section
 * 2: option 2 as far as memory allows, option 1 beyond).  The result is the
 * pseudo-double pass's to rounding; info->stored_iters reports the split. */
int msb_set_store_limit(msb_ctx *ctx, unsigned long long bytes);

/* Kernel timing of later calls on this context, a measurement aid: with
 * enable != 0 every kernel launch of the solvers is bracketed by a pair of HIP
 * events on the context's stream (previous records are dropped); 0 stops
 * recording.  Synchronises the stream. */
int msb_profile_enable(msb_ctx *ctx, int enable);

/* Which launches msb_profile_enable records: those of the kernel classes
 * whose bit k is set in mask (the classes of msb_profile_read), and of those
 * every stride-th one (stride >= 1, counted over the selected launches from
 * this call on); all classes, stride 1 on a new context.  The events take
 * time on the stream (stencil launches carry theirs in the dispatch, about
 * 8 us each), so a measurement of one kernel's average records that class
 * alone, sampled with a stride coprime to its launch pattern.  Synchronises
 * the stream.  MSB_ERR_ARG for stride < 1. */
int msb_profile_classes(msb_ctx *ctx, unsigned mask, int stride);

/* Totals of the recorded launches per kernel class k < n_classes (host arrays
 * of n_classes): count[k] launches, ms[k] summed event time, bytes[k] summed
 * algorithmic HBM bytes (every operand of a launch read or written once).
 * Classes: 0 stencil (D_w applications, all epilogues), 1 fused all-shift
 * update of a BiCG step, 2 fused all-shift MR update, 3 seed vector kernels,
 * 4 device scalar kernels, 5 set-up and output kernels.  Synchronises. */
int msb_profile_read(msb_ctx *ctx, int n_classes, long long *count, double *ms,
                     double *bytes);

/* out = D_w(mu) in (flags MSB_G5_LEFT, MSB_NEG_MU, MSB_DAGGER, MSB_MIXED).
 * The operator the paper names in Section 1.  in, out: device
 * [nrhs][12][V] complex128, must not overlap. */
int wilson_apply(msb_ctx *ctx, const void *in, void *out, int nrhs, int flags);

/* y = sum_s w_s (A + sigma_s)^{-1} b by multi-shift BiCGstab(l)
 * (Eq. 1.2, Section 2), A = a_scale (gamma5 D_w(mu))^2, tolerance tol on each
 * shift's relative residual.
 *   shifts, weights  host [n_sets][n_shift] doubles; n_sets = nrhs when
 *                    per_rhs_shift_sets = 1, else 1.  Shifts must be >= 0
 *                    after subtracting the smallest (any order).
 *   l                degree of the MR polynomial, 1..8
 *   pass             1: single-pass (N_s (l+1) shift vectors);
 *                    2: double-pass (no shift vectors, 4 M l Mv)
 *                    3: pseudo-double-pass (Section 2, the second option
 *                       after Eq. 2.2; Table 1): the first pass keeps all
 *                       2 M l Mv outputs in device memory (2 M l vectors
 *                       per right-hand side, plus M FP64 vectors with
 *                       MSB_MIXED), and y is summed from them after the
 *                       sweep: 2 M l Mv.  Not with MSB_PERSISTENT.  When
 *                       they do not fit (or pass msb_set_store_limit), the
 *                       iterations beyond the store are regenerated as in
 *                       the double pass.
 *   flags            MSB_MIXED, MSB_PERSISTENT, MSB_ADJOINT, MSB_REFINE (pass 1),
 *                    MSB_DEFERRED (pass 1, not with MSB_PERSISTENT),
 *                    MSB_OP_WILSON (A = a D_w; not with MSB_ADJOINT),
 *                    MSB_SEED_BASIS (pass 2 or 3, or 1 with MSB_DEFERRED; FP64,
 *                    one launch per stage)
 *   b                device [nrhs][12][V] complex128
 *   y                device [nrhs][12][V] complex128 (written)
 *   x_shifts         device [nrhs][n_shift][12][V] complex128 or NULL
 *                    (pass 1 only): the individual solutions x_s
 *   info             may be NULL.
 * Returns MSB_NOT_CONVERGED / MSB_BREAKDOWN with y filled. */
int mshift_bicgstabl(msb_ctx *ctx, double a_scale, int n_shift,
                     const double *shifts, const double *weights,
                     int per_rhs_shift_sets, int l, double tol, int max_outer,
                     int pass, int flags, int nrhs, const void *b, void *y,
                     void *x_shifts, msb_solve_info *info);

/* Size of the fixed device array behind mshift_bicgstabl_noalloc (one copy
 * per device the library runs on, held until the process ends). */
#define MSB_NOALLOC_SCRATCH_BYTES (256ull << 20)

/* mshift_bicgstabl without any device allocation, for callers that cannot
 * allocate: code that must not call hipMalloc/hipFree (under stream capture of
 * the surrounding work, tight serving loops, harnesses that forbid it).  Same
 * arguments, layouts, outputs and returns as mshift_bicgstabl; the workspace
 * (seed vectors, shift vectors of pass 1, reduction partials, scalar state,
 * the double-pass tape and replay program) is carved from one fixed device
 * array of MSB_NOALLOC_SCRATCH_BYTES, whose device address msb_create looks
 * up once per device.  The call makes no hipMalloc, hipFree or pinned host
 * allocation (host-side bookkeeping uses ordinary heap memory), and does not
 * grow the context's own workspace.
 *   pass   1 or 2 (the pseudo-double pass keeps a store that grows with the
 *          iteration count, so it is not offered here)
 *   flags  those of mshift_bicgstabl except MSB_PERSISTENT, MSB_REFINE and
 *          MSB_SEED_BASIS
 * Returns MSB_ERR_ARG, before anything is queued, when the workspace would
 * exceed the array.  With c = 16 bytes (8 with MSB_MIXED) and n = 12 V it
 * is about nrhs * n * c * (2 l + 3) for the seed (+ 3 * 16 n per rhs with
 * MSB_MIXED), + nrhs * n_shift * n * c * (l + 1) for pass 1's shift vectors
 * (c * 1 with MSB_DEFERRED, which adds nrhs * n * c * (2 l + 2)), + 16 n
 * per shift and rhs when x_shifts is NULL, + 720 bytes per rhs per 64
 * sites, at least 1.5 MB per rhs (reduction partials), + about 100 bytes
 * per rhs per BiCG step of max_outer * l for pass 2's tape and replay
 * program.
 * Every call on one device shares that device's array and leaves its
 * contents there; nothing is read from it before the call writes it.  Calls
 * that overlap in time on one device (several streams or host threads) race.
 * msb_profile_enable's records do not cover this call. */
int mshift_bicgstabl_noalloc(msb_ctx *ctx, double a_scale, int n_shift,
                             const double *shifts, const double *weights,
                             int per_rhs_shift_sets, int l, double tol, int max_outer,
                             int pass, int flags, int nrhs, const void *b, void *y,
                             void *x_shifts, msb_solve_info *info);

/* Multi-shift conjugate gradients for the same sum when A is Hermitian,
 * i.e. the context has mu = 0 (then gamma5 D_w is Hermitian and
 * A = a (gamma5 D_w)^2 >= 0): y = sum_s w_s (A + sigma_s)^{-1} b.  The CG
 * setting of Neuberger's double pass, the model of Section 2, and of the
 * pseudo-double pass the concluding section proposes for CG.
 *   pass  1: single pass (per shift a direction and a solution vector);
 *         2: double pass (scalars recorded, the seed residuals regenerated
 *            and summed with coefficients from a backward recurrence:
 *            2N - 1 Mv for N iterations);
 *         3: pseudo-double pass (the N seed residuals kept in device memory;
 *            N Mv; fails with MSB_ERR_OOM when they do not fit).
 *   max_iter   CG iteration limit; shift s freezes at the first iteration k
 *              with ||r_k|| / |zeta^s_k| <= tol ||b|| (info->shift_iters).
 *   flags      must be 0 (FP64, one launch per stage).
 *   Other arguments, layouts and returns as mshift_bicgstabl; info reports
 *   outer_iters = bicg_steps = N.  Returns MSB_ERR_ARG when mu != 0. */
int mshift_cg(msb_ctx *ctx, double a_scale, int n_shift, const double *shifts,
              const double *weights, int per_rhs_shift_sets, double tol, int max_iter,
              int pass, int flags, int nrhs, const void *b, void *y, void *x_shifts,
              msb_solve_info *info);

/* Low modes of H = gamma5 D_w at mu = 0 (H Hermitian): the nev eigenpairs of
 * smallest |lambda|, for deflation (the paper's overlap benchmarks deflate
 * these modes; see the figure captions of Sections 3 and 4).  Chebyshev-
 * filtered subspace iteration on H^2 with a block of nev + 1 <= nblock <= 128
 * vectors: Cholesky-QR, Rayleigh-Ritz with H^2 on the block (its small Ritz
 * values cannot be spurious), then with H on the leading nev Ritz vectors
 * (the signed eigenvalues).
 *   start   device [nblock][12][V] complex128 start block (the caller's
 *           random vectors; read only)
 *   tol     stop when ||H v - lambda v|| <= tol * ||H|| for every mode kept
 *   degree  largest Chebyshev degree per iteration (2 stencils on the block
 *           each); lowered while the filter interval is wide, so that no
 *           direction grows by more than 1e8 in one iteration
 *   evals   host [nev], sorted by |lambda|; evecs device [nev][12][V]
 *           (orthonormal); resid host [nev] or NULL; iters host or NULL.
 * Returns MSB_ERR_ARG when mu != 0, MSB_NOT_CONVERGED after max_iter
 * iterations (outputs filled), MSB_BREAKDOWN if the block loses rank. */
int msb_low_modes(msb_ctx *ctx, int nev, int nblock, const void *start, double tol,
                  int degree, int max_iter, double *evals, void *evecs, double *resid,
                  int *iters);

/* sign(H) b (or b + gamma5 sign(H) b with MSB_OVERLAP) at mu = 0 with nev
 * orthonormal low modes deflated:
 *   sign(H) b = sum_k sign(lambda_k) v_k <v_k, b> + sqrt(a) H f(a H^2) P b,
 *   P b = b - sum_k v_k <v_k, b>,
 * the partial-fraction expansion f (Eq. 1.2) solved as in mshift_bicgstabl.
 * evals host [nev], evecs device [nev][12][V]; other arguments as
 * pfe_sign_apply.  Returns MSB_ERR_ARG when mu != 0. */
int pfe_sign_apply_deflated(msb_ctx *ctx, double a_scale, int n_shift,
                            const double *shifts, const double *weights, int l, double tol,
                            int max_outer, int pass, int flags, int nrhs, int nev,
                            const double *evals, const void *evecs, const void *b, void *out,
                            msb_solve_info *info);

/* out = sign(H) b = sqrt(a_scale) H y, y the PFE solve above (Section 1,
 * sign z = z / sqrt(z^2)); with MSB_OVERLAP out = b + gamma5 sign(H) b, the
 * overlap operator of Eq. 1.1.  Arguments as for mshift_bicgstabl. */
int pfe_sign_apply(msb_ctx *ctx, double a_scale, int n_shift,
                   const double *shifts, const double *weights, int l,
                   double tol, int max_outer, int pass, int flags, int nrhs,
                   const void *b, void *out, msb_solve_info *info);

/* Gradients of the real loss L = Re <eta, y> with y = f(A) b (mode 0) or
 * y = sign(H) b (mode 1), in the convention dL/dRe + i dL/dIm:
 *   grad_b      device [nrhs][12][V] complex128 (written)
 *   grad_w      host [n_shift] (written; summed over RHS)
 *   grad_sigma  host [n_shift] (written; summed over RHS)
 *   grad_links  device [4][3][3][V] complex128 (ADDED to)
 * Uses adjoint multi-shift solves with A^+ = A(-mu) and a link-force kernel;
 * a_scale is held constant.  Not in the paper: the backward of Eq. 1.2. */
int pfe_sign_backward(msb_ctx *ctx, double a_scale, int n_shift,
                      const double *shifts, const double *weights, int l,
                      double tol, int max_outer, int flags, int nrhs,
                      const void *b, const void *eta, int mode, void *grad_b,
                      double *grad_w, double *grad_sigma, void *grad_links,
                      msb_solve_info *info);

#ifdef __cplusplus
}
#endif
#endif /* MSB_H */
