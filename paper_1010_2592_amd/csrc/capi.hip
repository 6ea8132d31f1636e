// The extern "C" boundary of libmsb: argument validation and marshalling
// only; all arithmetic happens in the kernels behind msb::solve_mshift and
// friends.  No C++ exception crosses this boundary.
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "msb.h"
#include "ctx.h"

namespace msb {
const char *last_error_msg();
}

struct msb_ctx {
    msb::Ctx c;
};

namespace {

using msb::set_error;

int arg_error(const std::string &m) { return set_error(MSB_ERR_ARG, m); }

bool finite_array(const double *p, long n) {
    for (long i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// Common validation and expansion of the solver arguments.
int make_params(msb_ctx *ctx, double a_scale, int n_shift, const double *shifts, const double *weights,
                int per_rhs, int l, double tol, int max_outer, int pass, int flags, int nrhs,
                const char *who, msb::SolveParams *P) {
    const std::string w(who);
    if (!ctx) return arg_error(w + ": null context");
    if (!(a_scale > 0.0) || !std::isfinite(a_scale)) return arg_error(w + ": a_scale must be finite and > 0");
    if (n_shift < 1 || n_shift > msb::NSMAX)
        return arg_error(w + ": n_shift must be in 1.." + std::to_string(msb::NSMAX));
    if (!shifts || !weights) return arg_error(w + ": shifts and weights are required");
    if (per_rhs != 0 && per_rhs != 1) return arg_error(w + ": per_rhs_shift_sets must be 0 or 1");
    if (l < 1 || l > msb::LMAX) return arg_error(w + ": l must be in 1.." + std::to_string(msb::LMAX));
    if (!(tol > 0.0) || !std::isfinite(tol)) return arg_error(w + ": tol must be finite and > 0");
    if (max_outer < 1 || (long)max_outer * l > (1L << 24)) return arg_error(w + ": max_outer out of range");
    if (pass < 1 || pass > 3) return arg_error(w + ": pass must be 1, 2 or 3");
    if (pass == 3 && (flags & MSB_PERSISTENT))
        return arg_error(w + ": pass = 3 runs with one launch per stage, not MSB_PERSISTENT");
    if (nrhs < 1 || nrhs > 4096) return arg_error(w + ": nrhs must be in 1..4096");
    if (flags & ~(MSB_MIXED | MSB_PERSISTENT | MSB_ADJOINT | MSB_OVERLAP | MSB_REFINE | MSB_DEFERRED |
                  MSB_OP_WILSON | MSB_SEED_BASIS))
        return arg_error(w + ": unknown flag bits");
    if ((flags & MSB_SEED_BASIS) && pass == 1 && !(flags & MSB_DEFERRED))
        return arg_error(w + ": MSB_SEED_BASIS needs pass = 2 or 3, or pass = 1 with MSB_DEFERRED (the per-step "
                             "shift updates read every r_i of every step)");
    if ((flags & MSB_SEED_BASIS) && (flags & (MSB_MIXED | MSB_PERSISTENT)))
        return arg_error(w + ": MSB_SEED_BASIS runs in FP64 with one launch per stage (not MSB_MIXED, "
                             "MSB_PERSISTENT)");
    if ((flags & MSB_OP_WILSON) && (flags & MSB_ADJOINT))
        return arg_error(w + ": MSB_OP_WILSON (A = a D_w) has no MSB_ADJOINT form");
    if ((flags & MSB_DEFERRED) && pass != 1)
        return arg_error(w + ": MSB_DEFERRED is a form of the single pass (pass = 1)");
    if ((flags & MSB_DEFERRED) && (flags & MSB_PERSISTENT))
        return arg_error(w + ": MSB_DEFERRED runs with one launch per stage, not MSB_PERSISTENT");
    if ((flags & MSB_REFINE) && pass != 1)
        return arg_error(w + ": MSB_REFINE needs pass = 1 (the double pass keeps no shift solutions)");
    if ((flags & MSB_PERSISTENT) && l > msb::PERSIST_LMAX)
        return arg_error(w + ": MSB_PERSISTENT needs l <= " + std::to_string(msb::PERSIST_LMAX));
    const long nsets = per_rhs ? nrhs : 1;
    if (!finite_array(shifts, nsets * n_shift) || !finite_array(weights, nsets * n_shift))
        return arg_error(w + ": shifts and weights must be finite");
    P->a_scale = a_scale;
    P->n_shift = n_shift;
    P->l = l;
    P->tol = tol;
    P->max_outer = max_outer;
    P->pass = pass;
    P->mixed = (flags & MSB_MIXED) != 0;
    P->neg_mu = (flags & MSB_ADJOINT) != 0;
    P->persistent = (flags & MSB_PERSISTENT) != 0;
    P->refine = (flags & MSB_REFINE) != 0;
    P->deferred = (flags & MSB_DEFERRED) != 0;
    P->op_wilson = (flags & MSB_OP_WILSON) != 0;
    P->seed_basis = (flags & MSB_SEED_BASIS) != 0;
    P->nrhs = nrhs;
    P->shifts.resize((size_t)nrhs * n_shift);
    P->weights.resize((size_t)nrhs * n_shift);
    for (int r = 0; r < nrhs; ++r) {
        const long src = per_rhs ? (long)r * n_shift : 0;
        for (int s = 0; s < n_shift; ++s) {
            P->shifts[(size_t)r * n_shift + s] = shifts[src + s];
            P->weights[(size_t)r * n_shift + s] = weights[src + s];
        }
    }
    return MSB_OK;
}

void fill_info(msb_solve_info *info, const msb::SolveReport &R, int nrhs, int n_shift, int status) {
    if (!info) return;
    info->status = status;
    info->outer_iters = R.outer_max;
    info->bicg_steps = R.steps_max;
    info->mv_count = R.mv;
    info->dot_count = R.dots;
    info->axpy_count = R.axpys;
    info->reliable_updates = R.reliable;
    info->bytes_model = R.bytes_model;
    info->refined_shifts = R.refined;
    info->stored_iters = R.stored_iters;
    const size_t m = (size_t)nrhs * n_shift;
    if (info->shift_iters && R.shift_iters.size() == m)
        std::memcpy(info->shift_iters, R.shift_iters.data(), m * sizeof(int));
    if (info->shift_resid && R.shift_resid.size() == m)
        std::memcpy(info->shift_resid, R.shift_resid.data(), m * sizeof(double));
    if (info->shift_true_resid && R.shift_true_resid.size() == m)
        std::memcpy(info->shift_true_resid, R.shift_true_resid.data(), m * sizeof(double));
}

int finish(int rc, const msb::SolveReport &R, msb_solve_info *info, int nrhs, int n_shift, int flags) {
    if (rc != MSB_OK) {
        if (info) info->status = rc;
        return rc;
    }
    int st = R.status;
    // mixed precision without the per-shift FP64 check: the shifts' true
    // residuals are not shown to meet tol
    if (st == MSB_OK && (flags & MSB_MIXED) && !(flags & MSB_REFINE)) st = MSB_REDUCED_ACCURACY;
    if (st == MSB_ERR_ARG) set_error(MSB_ERR_ARG, "right-hand side with a non-finite norm");
    else if (st == MSB_NOT_CONVERGED) set_error(st, "max_outer reached before every shift converged");
    else if (st == MSB_BREAKDOWN) set_error(st, "breakdown of the BiCG, MR or shift recurrence");
    else if (st == MSB_REDUCED_ACCURACY)
        set_error(st, "mixed precision without MSB_REFINE: the shifts' FP64 residuals are not checked");
    fill_info(info, R, nrhs, n_shift, st);
    return st;
}

}  // namespace

extern "C" {

const char *msb_last_error(void) { return msb::last_error_msg(); }

int msb_create(msb_ctx **out, const msb_lattice *lat, const void *links, void *stream) {
    if (!out || !lat || !links) return arg_error("msb_create: null argument");
    *out = nullptr;
    long V = 1;
    for (int d = 0; d < 4; ++d) {
        if (lat->dims[d] < 1) return arg_error("msb_create: dims must be >= 1");
        V *= lat->dims[d];
    }
    if (V > (1L << 26)) return arg_error("msb_create: volume too large (max 2^26 sites)");
    if (lat->bc_t != 1 && lat->bc_t != -1) return arg_error("msb_create: bc_t must be +1 or -1");
    if (!std::isfinite(lat->mass) || !std::isfinite(lat->mu)) return arg_error("msb_create: mass and mu must be finite");
    msb_ctx *x = new (std::nothrow) msb_ctx;
    if (!x) return set_error(MSB_ERR_OOM, "msb_create: out of host memory");
    int rc = msb::ctx_create(&x->c, lat->dims, lat->mass, lat->mu, lat->bc_t, links, (hipStream_t)stream);
    // the no-allocation entry point's scratch array on this device
    if (!rc) rc = msb::noalloc_setup(x->c.device);
    if (rc) {
        msb::ctx_destroy(&x->c);
        delete x;
        return rc;
    }
    *out = x;
    return MSB_OK;
}

void msb_destroy(msb_ctx *ctx) {
    if (!ctx) return;
    msb::ctx_destroy(&ctx->c);
    delete ctx;
}

int msb_set_stream(msb_ctx *ctx, void *stream) {
    if (!ctx) return arg_error("msb_set_stream: null context");
    ctx->c.stream = (hipStream_t)stream;
    return MSB_OK;
}

int msb_neuberger_pfe(int n, double *sigma, double *weight) {
    if (n < 1 || !sigma || !weight) return arg_error("msb_neuberger_pfe: need n >= 1 and output arrays");
    const double pi = 3.14159265358979323846;
    for (int s = 1; s <= n; ++s) {
        const double th = pi * (s - 0.5) / (2.0 * n);
        const double t = std::tan(th), c = std::cos(th);
        sigma[s - 1] = t * t;
        weight[s - 1] = 1.0 / (n * c * c);
    }
    return MSB_OK;
}

int msb_spectral_radius(msb_ctx *ctx, const void *start, int iters, double *rho) {
    if (!ctx || !start || !rho) return arg_error("msb_spectral_radius: null argument");
    if (iters < 1) return arg_error("msb_spectral_radius: iters must be >= 1");
    return msb::spectral_radius(&ctx->c, (const double2 *)start, iters, rho);
}

int msb_set_store_limit(msb_ctx *ctx, unsigned long long bytes) {
    if (!ctx) return arg_error("msb_set_store_limit: null context");
    ctx->c.store_limit = (size_t)bytes;
    return MSB_OK;
}

int msb_profile_enable(msb_ctx *ctx, int enable) {
    if (!ctx) return arg_error("msb_profile_enable: null context");
    return msb::profile_enable(&ctx->c, enable != 0);
}

int msb_profile_classes(msb_ctx *ctx, unsigned mask, int stride) {
    if (!ctx) return arg_error("msb_profile_classes: null context");
    if (stride < 1) return arg_error("msb_profile_classes: stride must be >= 1");
    return msb::profile_classes(&ctx->c, mask, stride);
}

int msb_profile_read(msb_ctx *ctx, int n_classes, long long *count, double *ms, double *bytes) {
    if (!ctx || !count || !ms || !bytes || n_classes < 1) return arg_error("msb_profile_read: bad argument");
    return msb::profile_read(&ctx->c, n_classes, count, ms, bytes);
}

int wilson_apply(msb_ctx *ctx, const void *in, void *out, int nrhs, int flags) {
    if (!ctx || !in || !out) return arg_error("wilson_apply: null argument");
    if (in == out) return arg_error("wilson_apply: in and out must not overlap");
    if (nrhs < 1) return arg_error("wilson_apply: nrhs must be >= 1");
    if (flags & ~(MSB_G5_LEFT | MSB_NEG_MU | MSB_DAGGER | MSB_MIXED)) return arg_error("wilson_apply: unknown flag bits");
    return msb::apply_wilson(&ctx->c, (const double2 *)in, (double2 *)out, nrhs, flags);
}

int mshift_bicgstabl(msb_ctx *ctx, double a_scale, int n_shift, const double *shifts,
                     const double *weights, int per_rhs_shift_sets, int l, double tol, int max_outer,
                     int pass, int flags, int nrhs, const void *b, void *y, void *x_shifts,
                     msb_solve_info *info) {
    msb::SolveParams P;
    int rc = make_params(ctx, a_scale, n_shift, shifts, weights, per_rhs_shift_sets, l, tol, max_outer,
                         pass, flags & ~MSB_OVERLAP, nrhs, "mshift_bicgstabl", &P);
    if (rc) return rc;
    if (!b || !y) return arg_error("mshift_bicgstabl: b and y are required");
    if (x_shifts && pass != 1) return arg_error("mshift_bicgstabl: x_shifts needs pass = 1");
    if (flags & MSB_OVERLAP) return arg_error("mshift_bicgstabl: MSB_OVERLAP applies to pfe_sign_apply");
    P.force_iters = info ? info->force_iters : nullptr;
    P.shadow = info ? (const double2 *)info->shadow : nullptr;
    msb::SolveReport R;
    const bool want_true = info && info->shift_true_resid && pass == 1;
    rc = msb::solve_mshift(&ctx->c, P, (const double2 *)b, (double2 *)y, (double2 *)x_shifts, want_true, &R);
    return finish(rc, R, info, nrhs, n_shift, flags);
}

int mshift_bicgstabl_noalloc(msb_ctx *ctx, double a_scale, int n_shift, const double *shifts,
                             const double *weights, int per_rhs_shift_sets, int l, double tol, int max_outer,
                             int pass, int flags, int nrhs, const void *b, void *y, void *x_shifts,
                             msb_solve_info *info) {
    msb::SolveParams P;
    int rc = make_params(ctx, a_scale, n_shift, shifts, weights, per_rhs_shift_sets, l, tol, max_outer,
                         pass, flags & ~MSB_OVERLAP, nrhs, "mshift_bicgstabl_noalloc", &P);
    if (rc) return rc;
    if (pass != 1 && pass != 2) return arg_error("mshift_bicgstabl_noalloc: pass must be 1 or 2");
    if (flags & (MSB_PERSISTENT | MSB_REFINE | MSB_SEED_BASIS))
        return arg_error("mshift_bicgstabl_noalloc: MSB_PERSISTENT, MSB_REFINE and MSB_SEED_BASIS are not offered");
    if (!b || !y) return arg_error("mshift_bicgstabl_noalloc: b and y are required");
    if (x_shifts && pass != 1) return arg_error("mshift_bicgstabl_noalloc: x_shifts needs pass = 1");
    if (flags & MSB_OVERLAP) return arg_error("mshift_bicgstabl_noalloc: MSB_OVERLAP applies to pfe_sign_apply");
    P.force_iters = info ? info->force_iters : nullptr;
    P.shadow = info ? (const double2 *)info->shadow : nullptr;
    msb::SolveReport R;
    const bool want_true = info && info->shift_true_resid && pass == 1;
    rc = msb::solve_noalloc(&ctx->c, P, (const double2 *)b, (double2 *)y, (double2 *)x_shifts, want_true, &R);
    return finish(rc, R, info, nrhs, n_shift, flags);
}

int mshift_cg(msb_ctx *ctx, double a_scale, int n_shift, const double *shifts, const double *weights,
              int per_rhs_shift_sets, double tol, int max_iter, int pass, int flags, int nrhs, const void *b,
              void *y, void *x_shifts, msb_solve_info *info) {
    msb::SolveParams P;
    if (flags != 0) return arg_error("mshift_cg: no flags apply (FP64, one launch per stage)");
    int rc = make_params(ctx, a_scale, n_shift, shifts, weights, per_rhs_shift_sets, 1, tol, max_iter, pass, 0,
                         nrhs, "mshift_cg", &P);
    if (rc) return rc;
    if (ctx->c.mu != 0.0) return arg_error("mshift_cg: needs mu = 0 (A Hermitian); use mshift_bicgstabl");
    if (!b || !y) return arg_error("mshift_cg: b and y are required");
    if (x_shifts && pass != 1) return arg_error("mshift_cg: x_shifts needs pass = 1");
    P.force_iters = info ? info->force_iters : nullptr;
    msb::SolveReport R;
    rc = msb::solve_cg(&ctx->c, P, (const double2 *)b, (double2 *)y, (double2 *)x_shifts, &R);
    return finish(rc, R, info, nrhs, n_shift, flags);
}

int msb_low_modes(msb_ctx *ctx, int nev, int nblock, const void *start, double tol, int degree, int max_iter,
                  double *evals, void *evecs, double *resid, int *iters) {
    if (!ctx) return arg_error("msb_low_modes: null context");
    if (ctx->c.mu != 0.0) return arg_error("msb_low_modes: needs mu = 0 (H Hermitian)");
    if (nev < 1 || nblock < nev + 1 || nblock > 128)
        return arg_error("msb_low_modes: need 1 <= nev < nblock <= 128");
    if (!start || !evals || !evecs) return arg_error("msb_low_modes: start, evals and evecs are required");
    if (!(tol > 0.0) || !std::isfinite(tol)) return arg_error("msb_low_modes: tol must be finite and > 0");
    if (degree < 1 || degree > 1000 || max_iter < 0) return arg_error("msb_low_modes: degree in 1..1000, max_iter >= 0");
    return msb::low_modes(&ctx->c, nev, nblock, (const double2 *)start, tol, degree, max_iter, evals,
                          (double2 *)evecs, resid, iters);
}

int pfe_sign_apply_deflated(msb_ctx *ctx, double a_scale, int n_shift, const double *shifts, const double *weights,
                            int l, double tol, int max_outer, int pass, int flags, int nrhs, int nev,
                            const double *evals, const void *evecs, const void *b, void *out,
                            msb_solve_info *info) {
    if (flags & MSB_OP_WILSON) return arg_error("pfe_sign_apply_deflated: needs A = a H^2, not MSB_OP_WILSON");
    msb::SolveParams P;
    int rc = make_params(ctx, a_scale, n_shift, shifts, weights, 0, l, tol, max_outer, pass, flags, nrhs,
                         "pfe_sign_apply_deflated", &P);
    if (rc) return rc;
    if (ctx->c.mu != 0.0) return arg_error("pfe_sign_apply_deflated: needs mu = 0 (orthonormal low modes of H)");
    if (nev < 1 || !evals || !evecs) return arg_error("pfe_sign_apply_deflated: nev >= 1 with evals and evecs");
    if (!finite_array(evals, nev)) return arg_error("pfe_sign_apply_deflated: evals must be finite");
    if (!b || !out) return arg_error("pfe_sign_apply_deflated: b and out are required");
    if (flags & MSB_ADJOINT) return arg_error("pfe_sign_apply_deflated: MSB_ADJOINT does not apply");
    P.force_iters = info ? info->force_iters : nullptr;
    msb::SolveReport R;
    rc = msb::sign_apply_deflated(&ctx->c, P, nev, evals, (const double2 *)evecs, (const double2 *)b,
                                  (double2 *)out, (flags & MSB_OVERLAP) != 0, &R);
    return finish(rc, R, info, nrhs, n_shift, flags);
}

int pfe_sign_apply(msb_ctx *ctx, double a_scale, int n_shift, const double *shifts,
                   const double *weights, int l, double tol, int max_outer, int pass, int flags,
                   int nrhs, const void *b, void *out, msb_solve_info *info) {
    msb::SolveParams P;
    if (flags & MSB_OP_WILSON) return arg_error("pfe_sign_apply: the sign function needs A = a H^2, not MSB_OP_WILSON");
    int rc = make_params(ctx, a_scale, n_shift, shifts, weights, 0, l, tol, max_outer, pass, flags, nrhs,
                         "pfe_sign_apply", &P);
    if (rc) return rc;
    if (!b || !out) return arg_error("pfe_sign_apply: b and out are required");
    P.force_iters = info ? info->force_iters : nullptr;
    msb::SolveReport R;
    rc = msb::sign_apply(&ctx->c, P, (const double2 *)b, (double2 *)out, (flags & MSB_OVERLAP) != 0, &R);
    return finish(rc, R, info, nrhs, n_shift, flags);
}

int pfe_sign_backward(msb_ctx *ctx, double a_scale, int n_shift, const double *shifts,
                      const double *weights, int l, double tol, int max_outer, int flags, int nrhs,
                      const void *b, const void *eta, int mode, void *grad_b, double *grad_w,
                      double *grad_sigma, void *grad_links, msb_solve_info *info) {
    msb::SolveParams P;
    if (flags & (MSB_OVERLAP | MSB_ADJOINT | MSB_OP_WILSON))
        return arg_error("pfe_sign_backward: only MSB_MIXED applies");
    int rc = make_params(ctx, a_scale, n_shift, shifts, weights, 0, l, tol, max_outer, 1, flags, nrhs,
                         "pfe_sign_backward", &P);
    if (rc) return rc;
    if (!b || !eta || !grad_b || !grad_w || !grad_sigma || !grad_links)
        return arg_error("pfe_sign_backward: b, eta and every gradient output are required");
    if (mode != 0 && mode != 1) return arg_error("pfe_sign_backward: mode must be 0 (f(A)b) or 1 (sign)");
    P.force_iters = info ? info->force_iters : nullptr;
    msb::SolveReport R;
    rc = msb::sign_backward(&ctx->c, P, (const double2 *)b, (const double2 *)eta, mode, (double2 *)grad_b,
                            grad_w, grad_sigma, (double2 *)grad_links, &R);
    return finish(rc, R, info, nrhs, n_shift, flags);
}

}  // extern "C"
