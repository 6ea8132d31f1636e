// Multi-shift conjugate gradients for a Hermitian A -- the overlap kernel
// A = a (gamma5 D_w)^2 at mu = 0, where gamma5 D_w is Hermitian -- in the
// single-pass form, Neuberger's double-pass form (which Section 2 of the
// paper takes as the model for its BiCGstab(l) variants) and the
// pseudo-double-pass form proposed for CG in the paper's concluding section.
//
// Seed: CG on S = A + sigma_0 (sigma_0 = min_s sigma_s), x0 = 0, r_0 = p_0 = b:
//   alpha_k = (r_k, r_k) / (p_k, S p_k),  r_{k+1} = r_k - alpha_k S p_k,
//   beta_k = (r_{k+1}, r_{k+1}) / (r_k, r_k),  p_{k+1} = r_{k+1} + beta_k p_k.
// Shift s (sigma' = sigma_s - sigma_0): collinear residual r_k / zeta_k with
// zeta_k = R_k(-sigma') from the seed's residual polynomial,
//   zeta_{k+1} = (1 + d_k + alpha_k sigma') zeta_k - d_k zeta_{k-1},
//   d_k = alpha_k beta_{k-1} / alpha_{k-1},
//   alpha^s_k = alpha_k zeta_k / zeta_{k+1},  beta^s_k = beta_k (zeta_k / zeta_{k+1})^2,
//   x^s += alpha^s_k p^s_k,  p^s_{k+1} = r_{k+1} / zeta_{k+1} + beta^s_k p^s_k.
// The single pass keeps p^s and x^s per shift; its p^s update is deferred
// into the next iteration's r-update pass (p^s_k from r_k, which that pass
// reads anyway).  The double pass records alpha_k and beta_k, forms on the
// host c_i = sum_s w_s e^s_i / zeta^s_i with e^s_{M_s-1} = alpha^s_{M_s-1},
// e^s_i = alpha^s_i + beta^s_i e^s_{i+1}, and regenerates r_i to sum
// y = sum_i c_i r_i; the pseudo-double pass stores r_i in the first pass.
// Everything runs in FP64 with device-side scalars; the host synchronises
// once every CG_SYNC iterations.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "ctx.h"

namespace msb {

namespace {

#define CG_HIPCHK(x)                                       \
    do {                                                   \
        int rc_ = hip_check((x), #x);                      \
        if (rc_) return rc_;                               \
    } while (0)
#define CG_CHK(x)                                          \
    do {                                                   \
        int rc_ = (x);                                     \
        if (rc_) return rc_;                               \
    } while (0)

constexpr int CG_SYNC = 16;       // iterations between host checks of the run flags
constexpr int CG_CHUNK = 32;      // pseudo-double pass: residuals per storage chunk

struct CGSeed {
    double rr, alpha, beta, alpha_prev, beta_prev, bnorm, tol;
    int run, k, max_iter, forced, nact, status, mv, dots;
    int act[NSMAX];
};
struct CGShift {
    double sp, zeta, zeta_prev, zeta_next, alpha_s, beta_s, res;
    int active, iters, force, pad;
};
// per active shift of the current iteration, read by the vector pass
struct CGCoef {
    double inv_zeta;   // 1 / zeta_k
    double beta_s;     // beta^s_{k-1}
    double alpha_s;    // alpha^s_k
    int s, first;
};

struct CGArgs {
    CGSeed *seed = nullptr;
    CGShift *sh = nullptr;
    CGCoef *coef = nullptr;
    double *part = nullptr;
    long ps = 0;
    int nblk_ds = 0, nblk_v = 0;   // partial counts of the stencil and vector passes
    double *tape_a = nullptr, *tape_b = nullptr;   // [rhs][max_iter] (double and pseudo-double pass)
    int tape_stride = 0;
};

__device__ inline const double *cg_row(const CGArgs &a, int rhs, int row) {
    return a.part + (size_t)rhs * PMAX * a.ps + (size_t)row * a.ps;
}

// ||b||, run flags
__global__ __launch_bounds__(BLOCK) void k_cg_init(CGArgs a) {
    const int rhs = blockIdx.x;
    CGSeed &S = a.seed[rhs];
    const double nb2 = block_sum(cg_row(a, rhs, 2), a.nblk_v);
    if (threadIdx.x != 0) return;
    S.bnorm = sqrt(nb2);
    S.rr = nb2;
    S.k = 0;
    S.mv = 0;
    S.dots = 0;
    S.alpha_prev = 1.0;
    S.beta_prev = 0.0;
    S.status = isfinite(nb2) ? S_OK : S_ERR_ARG;
    S.run = (nb2 > 0.0 && isfinite(nb2) && S.nact > 0) ? 1 : 0;
    if (!S.run) {
        for (int q = 0; q < S.nact; ++q) {
            CGShift &H = a.sh[(size_t)rhs * NSMAX + S.act[q]];
            H.active = 0;
            H.iters = 0;
            H.res = 0.0;
        }
        S.nact = 0;
    }
}

// alpha_k from (p_k, S p_k); each active shift's zeta_{k+1} and alpha^s_k
__global__ __launch_bounds__(BLOCK) void k_cg_alpha(CGArgs a) {
    const int rhs = blockIdx.x;
    CGSeed &S = a.seed[rhs];
    if (!S.run) return;
    const double pw = block_sum(cg_row(a, rhs, 0), a.nblk_ds);
    if (threadIdx.x != 0) return;
    S.mv += 1;
    S.dots += 1;
    if (!(pw > 0.0) || !isfinite(pw)) {
        S.status = S_BREAKDOWN;
        S.run = 0;
        for (int q = 0; q < S.nact; ++q) a.sh[(size_t)rhs * NSMAX + S.act[q]].iters = S.k;
        return;
    }
    const double alpha = S.rr / pw;
    const double d = S.k > 0 ? alpha * S.beta_prev / S.alpha_prev : 0.0;
    S.alpha = alpha;
    if (a.tape_a) a.tape_a[(size_t)rhs * a.tape_stride + S.k] = alpha;
    for (int q = 0; q < S.nact; ++q) {
        CGShift &H = a.sh[(size_t)rhs * NSMAX + S.act[q]];
        const double zn = (1.0 + d + alpha * H.sp) * H.zeta - d * H.zeta_prev;
        H.zeta_next = zn;
        H.alpha_s = alpha * H.zeta / zn;
        CGCoef &c = a.coef[(size_t)rhs * NSMAX + q];
        c.inv_zeta = 1.0 / H.zeta;
        c.beta_s = H.beta_s;
        c.alpha_s = H.alpha_s;
        c.s = S.act[q];
        c.first = S.k == 0 ? 1 : 0;
    }
}

// beta_k from ||r_{k+1}||^2; shift beta^s_k, residuals, freezing, termination
__global__ __launch_bounds__(BLOCK) void k_cg_beta(CGArgs a) {
    const int rhs = blockIdx.x;
    CGSeed &S = a.seed[rhs];
    if (!S.run) return;
    const double rrn = block_sum(cg_row(a, rhs, 3), a.nblk_v);
    if (threadIdx.x != 0) return;
    S.dots += 1;
    const double beta = rrn / S.rr;
    if (a.tape_b) a.tape_b[(size_t)rhs * a.tape_stride + S.k] = beta;
    int nact = 0;
    for (int q = 0; q < S.nact; ++q) {
        const int s = S.act[q];
        CGShift &H = a.sh[(size_t)rhs * NSMAX + s];
        const double zn = H.zeta_next;
        H.beta_s = beta * (H.zeta / zn) * (H.zeta / zn);
        H.zeta_prev = H.zeta;
        H.zeta = zn;
        H.res = sqrt(rrn) / fabs(zn) / S.bnorm;
        const bool done = S.forced ? (S.k + 1 >= H.force) : (H.res <= FREEZE_FRAC * S.tol);
        if (done || !isfinite(H.res)) {
            H.active = 0;
            H.iters = S.k + 1;
            if (!isfinite(H.res)) S.status = S_BREAKDOWN;
        } else {
            S.act[nact++] = s;
        }
    }
    S.nact = nact;
    S.alpha_prev = S.alpha;
    S.beta_prev = beta;
    S.beta = beta;
    S.rr = rrn;
    S.k += 1;
    if (nact == 0) {
        S.run = 0;
    } else if (S.k >= S.max_iter) {
        S.run = 0;
        if (S.status == S_OK) S.status = S_NOT_CONVERGED;
        for (int q = 0; q < nact; ++q) a.sh[(size_t)rhs * NSMAX + S.act[q]].iters = S.k;
    }
}

struct CGVec {
    const CGSeed *seed = nullptr;
    const CGCoef *coef = nullptr;
    double2 *r = nullptr, *p = nullptr;
    const double2 *w = nullptr;
    double2 *P = nullptr, *X = nullptr;   // shift directions and solutions [rhs][s][n]
    int nshift = 0;
    double2 *store = nullptr;             // pseudo-double pass: slot for r_{k+1} ([rhs] stride store_rs)
    long store_rs = 0;
    const double2 *rk = nullptr;          // pseudo-double pass: where r_k is read ([rhs] stride rk_rs;
    long rk_rs = 0;                       // null: r), r_{k+1} then going to the store slot only
    double *part = nullptr;
    long ps = 0;
    long n = 0;
};

// r_{k+1} = r_k - alpha_k w and ||r_{k+1}||^2; with SHIFTS every active shift's
// p^s_k = r_k / zeta_k + beta^s_{k-1} p^s_{k-1} (p^s_0 = r_0) and
// x^s += alpha^s_k p^s_k; with STORE r_{k+1} goes to the store slot instead of
// r (r_k read from rk when set: the previous slot).
template <bool SHIFTS, bool STORE>
__global__ __launch_bounds__(BLOCK) void k_cg_r(CGVec a) {
    const int rhs = blockIdx.y;
    const CGSeed &S = a.seed[rhs];
    if (!S.run) return;
    const long n = a.n;
    const double alpha = S.alpha;
    double2 *r = a.r + (size_t)rhs * n;
    const double2 *rin = (STORE && a.rk) ? a.rk + (size_t)rhs * a.rk_rs : r;
    const double2 *w = a.w + (size_t)rhs * n;
    const int nact = SHIFTS ? S.nact : 0;
    const CGCoef *cf = a.coef + (size_t)rhs * NSMAX;
    double part[1] = {0.0};
    for (long e = (long)blockIdx.x * BLOCK + threadIdx.x; e < n; e += (long)gridDim.x * BLOCK) {
        const double2 ro = rin[e];
        const double2 rn = csub(ro, cscale(w[e], alpha));
        if (STORE) a.store[(size_t)rhs * a.store_rs + e] = rn;
        else r[e] = rn;
        part[0] += rn.x * rn.x + rn.y * rn.y;
        if (SHIFTS) {
            for (int q = 0; q < nact; ++q) {
                const CGCoef c = cf[q];
                const size_t off = ((size_t)rhs * a.nshift + c.s) * n + e;
                const double2 pk = c.first ? ro : cadd(cscale(ro, c.inv_zeta), cscale(a.P[off], c.beta_s));
                a.P[off] = pk;
                a.X[off] = cadd(a.X[off], cscale(pk, c.alpha_s));
            }
        }
    }
    block_reduce_store<1>(part, a.part + (size_t)rhs * PMAX * a.ps + 3 * a.ps + blockIdx.x, a.ps);
}

// p_{k+1} = r_{k+1} + beta_k p_k
__global__ __launch_bounds__(BLOCK) void k_cg_p(CGVec a) {
    const int rhs = blockIdx.y;
    const CGSeed &S = a.seed[rhs];
    if (!S.run) return;
    const long n = a.n;
    const double beta = S.beta;
    double2 *p = a.p + (size_t)rhs * n;
    const double2 *r = a.rk ? a.rk + (size_t)rhs * a.rk_rs : a.r + (size_t)rhs * n;   // rk: r_{k+1}'s slot
    for (long e = (long)blockIdx.x * BLOCK + threadIdx.x; e < n; e += (long)gridDim.x * BLOCK)
        p[e] = cadd(r[e], cscale(p[e], beta));
}

// double pass, replay step k (right-hand sides with k + 1 < N_r):
// r_{k+1} = r_k - alpha_k w, y += c_{k+1} r_{k+1}, p_{k+1} = r_{k+1} + beta_k p_k
struct CGReplay {
    double2 *r = nullptr, *p = nullptr, *y = nullptr;
    const double2 *w = nullptr;
    const double *tape_a = nullptr, *tape_b = nullptr, *cc = nullptr;
    const int *nr = nullptr;
    int tape_stride = 0, c_stride = 0, k = 0;
    long n = 0;
};
__global__ __launch_bounds__(BLOCK) void k_cg_replay(CGReplay a) {
    const int rhs = blockIdx.y;
    if (a.k + 1 >= a.nr[rhs]) return;
    const long n = a.n;
    const double alpha = a.tape_a[(size_t)rhs * a.tape_stride + a.k];
    const double beta = a.tape_b[(size_t)rhs * a.tape_stride + a.k];
    const double c = a.cc[(size_t)rhs * a.c_stride + a.k + 1];
    double2 *r = a.r + (size_t)rhs * n, *p = a.p + (size_t)rhs * n, *y = a.y + (size_t)rhs * n;
    const double2 *w = a.w + (size_t)rhs * n;
    for (long e = (long)blockIdx.x * BLOCK + threadIdx.x; e < n; e += (long)gridDim.x * BLOCK) {
        const double2 rn = csub(r[e], cscale(w[e], alpha));
        r[e] = rn;
        y[e] = cadd(y[e], cscale(rn, c));
        p[e] = cadd(rn, cscale(p[e], beta));
    }
}

// pseudo-double pass: y += sum over the chunk's stored r_i (1 <= i < N_r) of c_i r_i
struct CGSum {
    double2 *y = nullptr;
    const double2 *store = nullptr;   // [rhs][CG_CHUNK][n]
    const double *cc = nullptr;
    const int *nr = nullptr;
    int c_stride = 0, i0 = 0;
    long n = 0;
};
__global__ __launch_bounds__(BLOCK) void k_cg_sum(CGSum a) {
    const int rhs = blockIdx.y;
    const long n = a.n;
    const int nr = a.nr[rhs];
    const double *c = a.cc + (size_t)rhs * a.c_stride;
    const double2 *V = a.store + (size_t)rhs * CG_CHUNK * n;
    double2 *y = a.y + (size_t)rhs * n;
    for (long e = (long)blockIdx.x * BLOCK + threadIdx.x; e < n; e += (long)gridDim.x * BLOCK) {
        double2 acc = y[e];
        for (int q = 0; q < CG_CHUNK; ++q) {
            const int i = a.i0 + q;
            if (i >= 1 && i < nr) acc = cadd(acc, cscale(V[(size_t)q * n + e], c[i]));
        }
        y[e] = acc;
    }
}

DslashArgs<double> cg_ds_args(const Ctx *c, bool g5out) {
    DslashArgs<double> a;
    a.U = c->U64;
    a.g = c->g;
    a.diag = 4.0 + c->mass;
    a.ef = std::exp(c->mu);
    a.eb = std::exp(-c->mu);
    a.bc = (double)c->bc_t;
    a.g5out = g5out ? 1 : 0;
    return a;
}

// c_i, i < N, with sum_s w_s x^s = sum_i c_i r_i (the double pass's backward
// recurrence over the recorded seed scalars)
void cg_coefficients(const double *alpha, const double *beta, int N, int ns, const double *sp, const double *w,
                     const int *M, double *c) {
    std::fill(c, c + N, 0.0);
    std::vector<double> z, as, bs;
    for (int s = 0; s < ns; ++s) {
        const int Ms = std::min(M[s], N);
        if (Ms <= 0) continue;
        z.assign(Ms + 1, 0.0);
        as.assign(Ms, 0.0);
        bs.assign(Ms, 0.0);
        z[0] = 1.0;
        double zprev = 1.0;
        for (int k = 0; k < Ms; ++k) {
            const double d = k > 0 ? alpha[k] * beta[k - 1] / alpha[k - 1] : 0.0;
            const double zn = (1.0 + d + alpha[k] * sp[s]) * z[k] - d * zprev;
            as[k] = alpha[k] * z[k] / zn;
            bs[k] = beta[k] * (z[k] / zn) * (z[k] / zn);
            zprev = z[k];
            z[k + 1] = zn;
        }
        double e = as[Ms - 1];
        c[Ms - 1] += w[s] * e / z[Ms - 1];
        for (int i = Ms - 2; i >= 0; --i) {
            e = as[i] + bs[i] * e;
            c[i] += w[s] * e / z[i];
        }
    }
}

}  // namespace

int solve_cg(Ctx *c, const SolveParams &P, const double2 *b, double2 *y, double2 *xs_out, SolveReport *rep) {
    hipStream_t st = c->stream;
    const int V = c->g.V;
    const long n = 12L * V;
    const int nrhs = P.nrhs, ns = P.n_shift;
    const int max_iter = P.max_outer;
    const bool pass1 = P.pass == 1, pass3 = P.pass == 3;
    const int nbd = (V + CHUNK - 1) / CHUNK;
    const int nbv = nblocks_for(n);
    const long ps = part_stride(c->g);
    const double nd = (double)n, Vd = (double)V, cB = 16.0;
    c->bytes_acc = 0;

    CG_CHK(ensure(c, c->ws_cg_r, (size_t)nrhs * n * sizeof(double2)));
    CG_CHK(ensure(c, c->ws_cg_p, (size_t)nrhs * n * sizeof(double2)));
    CG_CHK(ensure(c, c->ws_tmp, (size_t)nrhs * n * sizeof(double2)));
    CG_CHK(ensure(c, c->ws_cg_w, (size_t)nrhs * n * sizeof(double2)));
    CG_CHK(ensure(c, c->ws_part, (size_t)nrhs * PMAX * ps * sizeof(double)));
    CG_CHK(ensure(c, c->ws_cg_seed, (size_t)nrhs * sizeof(CGSeed)));
    CG_CHK(ensure(c, c->ws_cg_shift, (size_t)nrhs * NSMAX * sizeof(CGShift)));
    CG_CHK(ensure(c, c->ws_cg_coef, (size_t)nrhs * NSMAX * sizeof(CGCoef)));
    CG_CHK(ensure(c, c->ws_sig0, (size_t)nrhs * sizeof(double)));
    CG_CHK(ensure(c, c->ws_wts, (size_t)nrhs * ns * sizeof(double)));
    double2 *r = (double2 *)c->ws_cg_r.p, *p = (double2 *)c->ws_cg_p.p, *tmp = (double2 *)c->ws_tmp.p;
    double2 *w = (double2 *)c->ws_cg_w.p;
    double *part = (double *)c->ws_part.p;
    CGSeed *seed = (CGSeed *)c->ws_cg_seed.p;
    CGShift *sh = (CGShift *)c->ws_cg_shift.p;
    double2 *Pv = nullptr, *X = nullptr;
    if (pass1) {
        CG_CHK(ensure(c, c->ws_cg_P, (size_t)nrhs * ns * n * sizeof(double2)));
        Pv = (double2 *)c->ws_cg_P.p;
        if (xs_out) {
            X = xs_out;
        } else {
            CG_CHK(ensure(c, c->ws_X, (size_t)nrhs * ns * n * sizeof(double2)));
            X = (double2 *)c->ws_X.p;
        }
    }
    double *tape_a = nullptr, *tape_b = nullptr;
    if (!pass1) {
        CG_CHK(ensure(c, c->ws_cg_tape, (size_t)2 * nrhs * max_iter * sizeof(double)));
        tape_a = (double *)c->ws_cg_tape.p;
        tape_b = tape_a + (size_t)nrhs * max_iter;
    }

    // host-side initial state
    std::vector<CGSeed> hs(nrhs);
    std::vector<CGShift> hsh((size_t)nrhs * NSMAX);
    std::vector<double> sig0(nrhs);
    for (int rr = 0; rr < nrhs; ++rr) {
        const double *sg = &P.shifts[(size_t)rr * ns];
        sig0[rr] = *std::min_element(sg, sg + ns);
        CGSeed &S = hs[rr];
        std::memset(&S, 0, sizeof(S));
        S.tol = P.tol;
        S.max_iter = max_iter;
        S.forced = P.force_iters ? 1 : 0;
        S.nact = ns;
        for (int s = 0; s < ns; ++s) {
            S.act[s] = s;
            CGShift &H = hsh[(size_t)rr * NSMAX + s];
            std::memset(&H, 0, sizeof(H));
            H.sp = sg[s] - sig0[rr];
            H.zeta = 1.0;
            H.zeta_prev = 1.0;
            H.res = INFINITY;
            H.active = 1;
            H.force = P.force_iters ? P.force_iters[(size_t)rr * ns + s] : 0;
        }
    }
    CG_HIPCHK(hipMemcpyAsync(seed, hs.data(), nrhs * sizeof(CGSeed), hipMemcpyHostToDevice, st));
    CG_HIPCHK(hipMemcpyAsync(sh, hsh.data(), hsh.size() * sizeof(CGShift), hipMemcpyHostToDevice, st));
    CG_HIPCHK(hipMemcpyAsync(c->ws_sig0.p, sig0.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st));
    CG_HIPCHK(hipMemcpyAsync(c->ws_wts.p, P.weights.data(), (size_t)nrhs * ns * sizeof(double),
                             hipMemcpyHostToDevice, st));

    CGArgs ca;
    ca.seed = seed;
    ca.sh = sh;
    ca.coef = (CGCoef *)c->ws_cg_coef.p;
    ca.part = part;
    ca.ps = ps;
    ca.nblk_ds = nbd;
    ca.nblk_v = nbv;
    ca.tape_a = tape_a;
    ca.tape_b = tape_b;
    ca.tape_stride = max_iter;
    {
        Prof pr(c, CL_OTHER, nrhs * nd * cB * (pass1 ? 3.0 + ns : 3.0));
        CG_HIPCHK(hipMemcpyAsync(r, b, (size_t)nrhs * n * sizeof(double2), hipMemcpyDeviceToDevice, st));
        CG_HIPCHK(hipMemcpyAsync(p, b, (size_t)nrhs * n * sizeof(double2), hipMemcpyDeviceToDevice, st));
        if (pass1) launch_zero<double>(st, X, (long)nrhs * ns * n, 0, 1);
        launch_dot_partials<double>(st, b, b, n, part, ps, nrhs, nbv, Gate{});
    }
    {
        Prof pr(c, CL_SCALAR, 0);
        hipLaunchKernelGGL(k_cg_init, dim3(nrhs), dim3(BLOCK), 0, st, ca);
    }
    CG_HIPCHK(hipGetLastError());

    // Mv: w = a g5 D (g5 D p) + sigma0 p with (p, w) partials
    Gate g_run;
    g_run.flag = &seed[0].run;
    g_run.flag_stride = (long)sizeof(CGSeed) / (long)sizeof(int);
    g_run.need = 1;
    DslashArgs<double> d1 = cg_ds_args(c, true);
    d1.in = p;
    d1.out = tmp;
    d1.gate = g_run;
    DslashArgs<double> d2 = cg_ds_args(c, true);
    d2.in = tmp;
    d2.out = w;
    d2.v = p;
    d2.rt = p;
    d2.scale = P.a_scale;
    d2.sigma0_rhs = (const double *)c->ws_sig0.p;
    d2.part = part;
    d2.ps = ps;
    d2.gate = g_run;
    const double ds_plain = nrhs * 24 * cB * Vd + 36 * cB * Vd;
    const double ds_mv = nrhs * 48 * cB * Vd + 36 * cB * Vd;
    CGVec vv;
    vv.seed = seed;
    vv.coef = ca.coef;
    vv.r = r;
    vv.p = p;
    vv.w = w;
    vv.P = Pv;
    vv.X = X;
    vv.nshift = ns;
    vv.part = part;
    vv.ps = ps;
    vv.n = n;

    const long store_rs = (long)CG_CHUNK * n;
    for (int k = 0; k < max_iter; ++k) {
        CGVec vp = vv;   // the p-update's arguments (pass 3: r_{k+1} from its slot)
        {
            Prof pr(c, CL_STENCIL, ds_plain);
            launch_dslash<double>(st, d1, nrhs, EPI_PLAIN, false);
        }
        {
            Prof pr(c, CL_STENCIL, ds_mv);
            launch_dslash<double>(st, d2, nrhs, EPI_MV, false);
        }
        {
            Prof pr(c, CL_SCALAR, 0);
            hipLaunchKernelGGL(k_cg_alpha, dim3(nrhs), dim3(BLOCK), 0, st, ca);
        }
        {
            CGVec v1 = vv;
            if (pass3) {
                // r_{k+1} is written to its slot only; r_k is read from slot k
                // (r_0 = b from r)
                const int slot = k + 1;
                const int ch = slot / CG_CHUNK;
                while ((int)c->pstore.size() <= ch) c->pstore.push_back(DevBuf{});
                CG_CHK(ensure(c, c->pstore[ch], (size_t)nrhs * store_rs * sizeof(double2)));
                v1.store = (double2 *)c->pstore[ch].p + (size_t)(slot % CG_CHUNK) * n;
                v1.store_rs = store_rs;
                if (k >= 1) {
                    v1.rk = (const double2 *)c->pstore[k / CG_CHUNK].p + (size_t)(k % CG_CHUNK) * n;
                    v1.rk_rs = store_rs;
                }
                vp.rk = v1.store;
                vp.rk_rs = store_rs;
            }
            // upper bound: every shift active (the byte model of the solve)
            Prof pr(c, pass1 ? CL_SHIFT : CL_SEED,
                    nrhs * nd * (3.0 * cB + (pass1 ? ns * 4.0 * cB : 0.0)));
            dim3 g(nbv, nrhs);
            if (pass1) hipLaunchKernelGGL((k_cg_r<true, false>), g, dim3(BLOCK), 0, st, v1);
            else if (pass3) hipLaunchKernelGGL((k_cg_r<false, true>), g, dim3(BLOCK), 0, st, v1);
            else hipLaunchKernelGGL((k_cg_r<false, false>), g, dim3(BLOCK), 0, st, v1);
        }
        {
            Prof pr(c, CL_SCALAR, 0);
            hipLaunchKernelGGL(k_cg_beta, dim3(nrhs), dim3(BLOCK), 0, st, ca);
        }
        {
            Prof pr(c, CL_SEED, nrhs * nd * 3.0 * cB);
            hipLaunchKernelGGL(k_cg_p, dim3(nbv, nrhs), dim3(BLOCK), 0, st, vp);
        }
        CG_HIPCHK(hipGetLastError());
        if ((k + 1) % CG_SYNC == 0 || k + 1 == max_iter) {
            std::vector<CGSeed> cur(nrhs);
            CG_HIPCHK(hipStreamSynchronize(st));
            CG_HIPCHK(hipMemcpy(cur.data(), seed, nrhs * sizeof(CGSeed), hipMemcpyDeviceToHost));
            bool any = false;
            for (int q = 0; q < nrhs; ++q) any = any || cur[q].run;
            if (!any) break;
        }
    }

    // results of the first pass
    std::vector<CGSeed> fs(nrhs);
    std::vector<CGShift> fsh((size_t)nrhs * NSMAX);
    CG_HIPCHK(hipStreamSynchronize(st));
    CG_HIPCHK(hipMemcpy(fs.data(), seed, nrhs * sizeof(CGSeed), hipMemcpyDeviceToHost));
    CG_HIPCHK(hipMemcpy(fsh.data(), sh, fsh.size() * sizeof(CGShift), hipMemcpyDeviceToHost));
    rep->status = S_OK;
    rep->outer_max = 0;
    rep->steps_max = 0;
    rep->mv = 0;
    rep->dots = 0;
    rep->reliable = 0;
    rep->shift_iters.assign((size_t)nrhs * ns, 0);
    rep->shift_resid.assign((size_t)nrhs * ns, 0.0);
    rep->rhs_outer.assign(nrhs, 0);
    std::vector<int> Nr(nrhs, 0);
    for (int q = 0; q < nrhs; ++q) {
        const CGSeed &S = fs[q];
        int status = S.status;
        if (S.run) status = S_NOT_CONVERGED;
        rep->status = std::max(rep->status, status);
        rep->outer_max = std::max(rep->outer_max, S.k);
        rep->steps_max = rep->outer_max;
        rep->rhs_outer[q] = S.k;
        rep->mv += S.mv;
        rep->dots += S.dots;
        for (int s = 0; s < ns; ++s) {
            const CGShift &H = fsh[(size_t)q * NSMAX + s];
            const int it = H.active ? S.k : H.iters;
            rep->shift_iters[(size_t)q * ns + s] = it;
            rep->shift_resid[(size_t)q * ns + s] = H.res;
            Nr[q] = std::max(Nr[q], it);
        }
    }

    if (pass1) {
        Prof pr(c, CL_OTHER, nrhs * nd * (ns * cB + 16.0));
        launch_ysum(st, y, X, (const double *)c->ws_wts.p, n, ns, nrhs, nbv);
        CG_HIPCHK(hipGetLastError());
    } else {
        // coefficients of the seed residuals
        int Nmax = 1;
        for (int q = 0; q < nrhs; ++q) Nmax = std::max(Nmax, Nr[q]);
        std::vector<double> ta((size_t)nrhs * max_iter), tb((size_t)nrhs * max_iter);
        CG_HIPCHK(hipMemcpy(ta.data(), tape_a, ta.size() * sizeof(double), hipMemcpyDeviceToHost));
        CG_HIPCHK(hipMemcpy(tb.data(), tape_b, tb.size() * sizeof(double), hipMemcpyDeviceToHost));
        std::vector<double> cc((size_t)nrhs * Nmax, 0.0), spv(ns), wv(ns);
        std::vector<int> Ms(ns);
        std::vector<double2> c0(nrhs);
        for (int q = 0; q < nrhs; ++q) {
            for (int s = 0; s < ns; ++s) {
                spv[s] = fsh[(size_t)q * NSMAX + s].sp;
                wv[s] = P.weights[(size_t)q * ns + s];
                Ms[s] = rep->shift_iters[(size_t)q * ns + s];
            }
            if (Nr[q] > 0)
                cg_coefficients(&ta[(size_t)q * max_iter], &tb[(size_t)q * max_iter], Nr[q], ns, spv.data(),
                                wv.data(), Ms.data(), &cc[(size_t)q * Nmax]);
            c0[q] = double2{cc[(size_t)q * Nmax], 0.0};
        }
        CG_CHK(ensure(c, c->ws_cg_c, cc.size() * sizeof(double)));
        CG_CHK(ensure(c, c->ws_cg_n, (size_t)nrhs * sizeof(int)));
        CG_CHK(ensure(c, c->ws_cb, (size_t)nrhs * sizeof(double2)));
        CG_HIPCHK(hipMemcpy(c->ws_cg_c.p, cc.data(), cc.size() * sizeof(double), hipMemcpyHostToDevice));
        CG_HIPCHK(hipMemcpy(c->ws_cg_n.p, Nr.data(), nrhs * sizeof(int), hipMemcpyHostToDevice));
        CG_HIPCHK(hipMemcpy(c->ws_cb.p, c0.data(), nrhs * sizeof(double2), hipMemcpyHostToDevice));
        {
            Prof pr(c, CL_OTHER, nrhs * nd * 32.0);
            launch_yinit(st, y, b, (const double2 *)c->ws_cb.p, n, nrhs, nbv);
        }
        if (pass3) {
            // y += sum_{i >= 1} c_i r_i over the stored residuals
            for (int i0 = 0; i0 < Nmax; i0 += CG_CHUNK) {
                CGSum a;
                a.y = y;
                a.store = (const double2 *)c->pstore[i0 / CG_CHUNK].p;
                a.cc = (const double *)c->ws_cg_c.p;
                a.nr = (const int *)c->ws_cg_n.p;
                a.c_stride = Nmax;
                a.i0 = i0;
                a.n = n;
                Prof pr(c, CL_OTHER, nrhs * nd * (32.0 + CG_CHUNK * cB));
                hipLaunchKernelGGL(k_cg_sum, dim3(nbv, nrhs), dim3(BLOCK), 0, st, a);
            }
        } else {
            // regenerate r_1 .. r_{N-1} with the recorded scalars
            {
                Prof pr(c, CL_OTHER, nrhs * nd * 4.0 * cB);
                CG_HIPCHK(hipMemcpyAsync(r, b, (size_t)nrhs * n * sizeof(double2), hipMemcpyDeviceToDevice, st));
                CG_HIPCHK(hipMemcpyAsync(p, b, (size_t)nrhs * n * sizeof(double2), hipMemcpyDeviceToDevice, st));
            }
            CGReplay ra;
            ra.r = r;
            ra.p = p;
            ra.y = y;
            ra.w = w;
            ra.tape_a = tape_a;
            ra.tape_b = tape_b;
            ra.cc = (const double *)c->ws_cg_c.p;
            ra.nr = (const int *)c->ws_cg_n.p;
            ra.tape_stride = max_iter;
            ra.c_stride = Nmax;
            ra.n = n;
            DslashArgs<double> e1 = d1, e2 = d2;
            e2.rt = nullptr;
            e2.part = nullptr;
            for (int k = 0; k + 1 < Nmax; ++k) {
                Gate gk;
                gk.flag = (const int *)c->ws_cg_n.p;
                gk.flag_stride = 1;
                gk.need = k + 2;
                e1.gate = gk;
                e2.gate = gk;
                int nr_k = 0;
                for (int q = 0; q < nrhs; ++q) nr_k += (k + 1 < Nr[q]) ? 1 : 0;
                {
                    Prof pr(c, CL_STENCIL, nr_k * 24 * cB * Vd + 36 * cB * Vd);
                    launch_dslash<double>(st, e1, nrhs, EPI_PLAIN, false);
                }
                {
                    Prof pr(c, CL_STENCIL, nr_k * 36 * cB * Vd + 36 * cB * Vd);
                    launch_dslash<double>(st, e2, nrhs, EPI_SV, false);
                }
                ra.k = k;
                {
                    Prof pr(c, CL_SEED, nr_k * nd * 7.0 * cB);
                    hipLaunchKernelGGL(k_cg_replay, dim3(nbv, nrhs), dim3(BLOCK), 0, st, ra);
                }
                CG_HIPCHK(hipGetLastError());
                rep->mv += nr_k;
            }
        }
        CG_HIPCHK(hipGetLastError());
    }
    CG_HIPCHK(hipStreamSynchronize(st));
    rep->bytes_model = c->bytes_acc;
    return 0;
}

}  // namespace msb
