// Library context and host-side solver entry points (internal).
#pragma once

#include <string>
#include <vector>

#include "common.h"
#include "kernels.h"


namespace msb {

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

// A caller-provided block of device memory that ensure() carves workspace
// from instead of allocating (the no-allocation entry point): bump
// allocation in 256-byte steps, never freed, an error once it is full.
struct Arena {
    char *base = nullptr;
    size_t cap = 0;
    size_t used = 0;
};

struct Ctx {
    Geom g{};
    double mass = 0, mu = 0;
    int bc_t = -1;
    hipStream_t stream = nullptr;
    int device = 0;
    double2 *U64 = nullptr;    // links, FP64 copy [4][3][3][V]
    float2 *U32 = nullptr;     // links, FP32 copy
    // workspace, grown on demand and kept for later calls
    DevBuf ws_R, ws_U, ws_tmp, ws_W, ws_X, ws_rt, ws_b, ws_y, ws_part, ws_seed, ws_shift, ws_sc,
        ws_mc, ws_tape, ws_tape_gam, ws_tape_outer, ws_replay, ws_replay_outer, ws_wts, ws_sig0,
        ws_cb, ws_aux1, ws_aux2, ws_aux3, ws_aux4, ws_bX, ws_bZ, ws_by, ws_beta, ws_bA, ws_bB, ws_bdots,
        ws_ops, ws_pctl, ws_rX, ws_rX2, ws_ry, ws_rB, ws_rR, ws_rt1, ws_rt2, ws_rsig, ws_rw, ws_Bm, ws_schist,
        ws_dc, ws_cg_r, ws_cg_p, ws_cg_w, ws_cg_P, ws_cg_seed, ws_cg_shift, ws_cg_coef, ws_cg_tape, ws_cg_c,
        ws_cg_n, ws_eY, ws_eW, ws_eZ, ws_eP, ws_eS, ws_eG, ws_sp;
    int pgrid[32] = {};        // co-resident grid of the persistent kernel, per (precision, l)
    // pseudo-double passes: stored Mv outputs (and reliable-update Mv
    // outputs) of BiCGstab(l), or stored residuals of CG, in chunks, kept for
    // later calls
    std::vector<DevBuf> pstore, prel;
    DevBuf ws_ones;
    void *host_pinned = nullptr;
    size_t host_pinned_bytes = 0;
    // set for the duration of a no-allocation call: device workspace comes
    // from the arena and host staging from ordinary (pageable) heap memory
    Arena *arena = nullptr;
    std::vector<char> host_heap;
    // kernel timing (msb_profile_enable): HIP event pairs around launches
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    struct Rec {
        int cls;
        double bytes;
        hipEvent_t e0, e1;
    };
    std::vector<Rec> recs;
    // stage times measured inside a persistent launch (wall clock per class);
    // pending: bytes not yet attached
    struct SRec {
        int cls;
        long long count;
        double ms, bytes;
        bool pending = true;
    };
    std::vector<SRec> srecs;
    double bytes_acc = 0;      // algorithmic bytes of the current call
};

// kernel classes of the timing hook
enum { CL_STENCIL = 0, CL_SHIFT = 1, CL_SHIFT_MR = 2, CL_SEED = 3, CL_SCALAR = 4, CL_OTHER = 5,
       CL_COUNT = 6 };

// Scope that records a HIP event pair around the launches inside it (when
// profiling) and adds the launch's algorithmic bytes to the call's model.
struct Prof {
    Ctx *c;
    int cls;
    double bytes;
    hipEvent_t e0 = nullptr;
    Prof(Ctx *c_, int cls_, double bytes_);
    ~Prof();
};
int profile_enable(Ctx *c, bool on);
int profile_read(Ctx *c, int ncls, long long *count, double *ms, double *bytes);

// All solver parameters of one call (shifts and weights already expanded to
// one set per right-hand side).
struct SolveParams {
    double a_scale = 1;
    int n_shift = 0;
    std::vector<double> shifts;    // [nrhs][n_shift]
    std::vector<double> weights;   // [nrhs][n_shift]
    int l = 1;
    double tol = 1e-8;
    std::vector<double> tol_rhs;       // optional per-rhs tolerance (overrides tol)
    int max_outer = 1000;
    int pass = 1;
    bool mixed = false;
    bool neg_mu = false;
    bool persistent = false;           // one cooperative launch per pass
    bool refine = false;               // pass 1: refine shifts above tol (true residual)
    bool deferred = false;             // pass 1: shift vectors updated once per outer iteration
    bool op_wilson = false;            // A = a D_w(mu) instead of a (g5 D_w(mu))^2
    int nrhs = 1;
    const int *force_iters = nullptr;   // [nrhs][n_shift] or null
    const double2 *shadow = nullptr;    // [nrhs][12V] shadow residual r~, or null (r~ = b)
};

struct SolveReport {
    int status = 0;
    int outer_max = 0, steps_max = 0;
    long long mv = 0, dots = 0, axpys = 0;
    int reliable = 0;
    double bytes_model = 0;
    std::vector<int> shift_iters;
    std::vector<double> shift_resid;
    std::vector<double> shift_true_resid;
    std::vector<int> rhs_outer;
    int refined = 0;                   // (rhs, shift) refinement solves
};

// status-returning helpers; on failure they record a message
int set_error(int status, const std::string &msg);
int hip_check(hipError_t e, const char *what);
// grow b to at least `bytes` (hipMalloc, or carved from c->arena when set)
int ensure(Ctx *c, DevBuf &b, size_t bytes);

int ctx_create(Ctx *c, const int dims[4], double mass, double mu, int bc_t, const void *links,
               hipStream_t stream);
void ctx_destroy(Ctx *c);

int apply_wilson(Ctx *c, const double2 *in, double2 *out, int nrhs, int flags);
int spectral_radius(Ctx *c, const double2 *start, int iters, double *rho);
int solve_mshift(Ctx *c, const SolveParams &P, const double2 *b, double2 *y, double2 *x_shifts,
                 bool want_true_resid, SolveReport *rep);
// multi-shift CG (A Hermitian: mu = 0); P.max_outer is the iteration limit,
// P.l is unused
int solve_cg(Ctx *c, const SolveParams &P, const double2 *b, double2 *y, double2 *x_shifts, SolveReport *rep);
// low modes of H = gamma5 D_w (mu = 0) by Chebyshev-filtered subspace
// iteration on H^2 with a block of m vectors from `start` ([m][12V])
int low_modes(Ctx *c, int nev, int m, const double2 *start, double tol, int degree, int max_iter, double *evals,
              double2 *evecs, double *resid, int *iters);
// sign(H) b (or the overlap) with the given orthonormal low modes deflated
int sign_apply_deflated(Ctx *c, const SolveParams &P, int nev, const double *evals, const double2 *evecs,
                        const double2 *b, double2 *out, bool overlap, SolveReport *rep);
// the no-allocation entry point: the device scratch array's address is looked
// up once per device (at context creation) and the solve's workspace is
// carved from it
int noalloc_setup(int device);
int solve_noalloc(Ctx *c, const SolveParams &P, const double2 *b, double2 *y, double2 *x_shifts, bool want_true,
                  SolveReport *rep);
int sign_apply(Ctx *c, const SolveParams &P, const double2 *b, double2 *out, bool overlap,
               SolveReport *rep);
int sign_backward(Ctx *c, const SolveParams &P, const double2 *b, const double2 *eta, int mode,
                  double2 *grad_b, double *grad_w, double *grad_sigma, double2 *grad_links,
                  SolveReport *rep);

}  // namespace msb
