// Device bodies of the scalar stages of multi-shift BiCGstab(l), one block
// per right-hand side (see scalar.hip for the recurrences).  Shared by the
// one-launch-per-stage kernels and the persistent kernel.
#pragma once
#include "common.h"
#include "kernels.h"

namespace msb {
namespace dev {

__device__ inline double2 cpowi_neg(double sp, int i) {
    // (-sp)^i for integer i >= 0
    double p = 1.0;
    for (int k = 0; k < i; ++k) p *= -sp;
    return d2(p, 0.0);
}

__device__ inline const double *prow(const ScalarArgs &a, int rhs) {
    return a.part + (size_t)rhs * PMAX * a.ps;
}

// the sums of partial rows 0, 1, 2 (re, im of an inner product, a squared
// norm) in one pass, bitwise those of three block_sum calls
__device__ inline void sum3(const double *row, long ps, int n, double &s0, double &s1, double &s2) {
    const int rows[3] = {0, 1, 2};
    double o[3];
    block_sum_rows<3>(row, ps, rows, 3, n, o);
    s0 = o[0];
    s1 = o[1];
    s2 = o[2];
}

__device__ __forceinline__ void sc_init_body(const ScalarArgs &a, int rhs) {
    SeedState &S = a.seed[rhs];
    const double *row = prow(a, rhs);
    const double re = block_sum(row, a.nblk);
    const double im = block_sum(row + a.ps, a.nblk);
    const double nb2 = block_sum(row + 2 * a.ps, a.nblk);
    const double rt2 = a.shadow ? block_sum(row + 5 * a.ps, a.nblk) : nb2;
    if (threadIdx.x == 0) {
        S.rho1 = d2(re, im);
        S.bnorm = sqrt(nb2);
        S.rtnorm = sqrt(rt2);
        S.rnorm0 = S.bnorm;
        S.rnorm_j = S.bnorm;
        S.rho0 = d2(1, 0);
        S.alpha = d2(0, 0);
        S.omega = d2(1, 0);
        S.beta = d2(0, 0);
        for (int i = 0; i < LMAX; ++i) S.gam[i] = d2(0, 0);
        S.bicg_on = 1;
        S.l_eff = 0;
        S.l_mr = 0;
        S.broken = S.exhausted = S.partial = 0;
        S.m = S.n = 0;
        S.status = S_OK;
        S.mv = S.dots = S.axpys = S.reliable = 0;
        S.rel = 0;
        S.rmax = S.bnorm;
        S.beta_spec = d2(NAN, NAN);
        S.wu_ready = 0;
        for (int i = 0; i < LMAX; ++i) S.step_flag[i] = 0;
        S.nact = 0;
        for (int s = 0; s < S.nshift; ++s) {
            if (a.sh[(size_t)rhs * NSMAX + s].active) S.act[S.nact++] = s;
        }
        S.dots = 0;
        S.run = (S.bnorm > 0.0 && S.nact > 0 && isfinite(S.bnorm)) ? 1 : 0;
        if (!isfinite(S.bnorm)) S.status = S_ERR_ARG;
        if (!(S.bnorm > 0.0) || !isfinite(S.bnorm)) {
            for (int s = 0; s < S.nshift; ++s) {
                ShiftState &H = a.sh[(size_t)rhs * NSMAX + s];
                H.active = 0;
                H.iters = 0;
                H.res = 0.0;
            }
            S.nact = 0;
        }
    }
}

__device__ __forceinline__ void sc_beta_body(const ScalarArgs &a, int rhs) {
    SeedState &S = a.seed[rhs];
    if (!S.run || !S.bicg_on) return;
    const int j = a.j;
    const double *row = prow(a, rhs);
    double re, im, rj2;
    sum3(row, a.ps, a.nblk, re, im, rj2);
    double r02 = 0.0;
    if (j >= 1) r02 = block_sum(row + 3 * a.ps, a.nblk2);
    if (threadIdx.x != 0) return;
    if (j == 0) S.wu_ready = 0;
    // basis form: ||r_0|| exists only where sc_exh found that the test could
    // fire; elsewhere it cannot (||r_0|| >= ||r_{j-1}|| / ||S||^(j-1))
    const bool have_r0 = !a.basis || S.exh_check;
    if (j >= 1 && have_r0) S.rnorm0 = sqrt(r02);
    if (j >= 1 && have_r0 && !S.forced && S.nact > 0) {
        // Krylov space exhausted: every active shift already meets its
        // tolerance after the previous step's r-update
        double mn = 1e308;
        for (int q = 0; q < S.nact; ++q) {
            const ShiftState &H = a.sh[(size_t)rhs * NSMAX + S.act[q]];
            if (!H.active) continue;
            const double sc = cmod(cmul(H.zeta, H.psi));
            mn = sc < mn ? sc : mn;
        }
        if (S.rnorm0 <= FREEZE_FRAC * S.tol * S.bnorm * mn) {
            S.exhausted = 1;
            S.bicg_on = 0;
            S.l_eff = j;
            return;
        }
    }
    if (j == 0) S.rho0 = cneg(cmul(S.omega, S.rho0));
    const double2 rho1 = d2(re, im);
    S.dots += 1;
    if ((rho1.x == 0.0 && rho1.y == 0.0) || !cfinite(rho1) ||
        cabsd(rho1) <= BREAK_REL * S.rtnorm * sqrt(rj2)) {
        S.broken = 1;
        S.bicg_on = 0;
        S.l_eff = j;
        return;
    }
    const double2 beta = cdiv(cmul(S.alpha, rho1), S.rho0);
    if (j == 0 && a.spec) {
        // the MR update already made u_0 = r_0 - beta u_0 with this beta
        S.wu_ready = (beta.x == S.beta_spec.x && beta.y == S.beta_spec.y) ? 1 : 0;
        S.beta_spec = d2(NAN, NAN);
    }
    S.rho0 = rho1;
    S.beta = beta;
    S.step_beta[j] = beta;
    S.step_flag[j] = 1;
    if (a.record && S.n < S.max_steps) {
        TapeStep &t = a.tape[(size_t)rhs * S.max_steps + S.n];
        t.beta = beta;
        t.alpha = d2(0, 0);
        t.flag = 0;
    }
}

__device__ __forceinline__ void sc_alpha_body(const ScalarArgs &a, int rhs) {
    SeedState &S = a.seed[rhs];
    if (!S.run || !S.bicg_on) return;
    const int j = a.j;
    const double *row = prow(a, rhs);
    double re, im, u2;
    sum3(row, a.ps, a.nblk, re, im, u2);
    __shared__ int ok;
    __shared__ double2 sh_alpha, sh_beta;
    if (threadIdx.x == 0) {
        const double2 gam = d2(re, im);
        S.dots += 1;
        S.mv += 1;
        ok = 1;
        if ((gam.x == 0.0 && gam.y == 0.0) || !cfinite(gam) ||
            cabsd(gam) <= BREAK_REL * S.rtnorm * sqrt(u2)) {
            S.broken = 1;
            S.partial = 1;
            S.bicg_on = 0;
            S.l_eff = j;
            if (a.record && S.n < S.max_steps) a.tape[(size_t)rhs * S.max_steps + S.n].flag = 1;
            ok = 0;
        } else {
            const double2 alpha = cdiv(S.rho0, gam);
            S.alpha = alpha;
            S.step_alpha[j] = alpha;
            S.step_flag[j] = 2;
            if (a.record && S.n < S.max_steps) {
                TapeStep &t = a.tape[(size_t)rhs * S.max_steps + S.n];
                t.alpha = alpha;
                t.flag = 2;
            }
        }
        sh_alpha = S.alpha;
        sh_beta = S.beta;
    }
    __syncthreads();
    if (!ok) return;
    const double2 alpha = sh_alpha, beta = sh_beta;
    const int nact = S.nact;
    for (int q = threadIdx.x; q < nact; q += BLOCK) {
        const int s = S.act[q];
        ShiftState &H = a.sh[(size_t)rhs * NSMAX + s];
        StepCoef &c = a.sc[(size_t)rhs * NSMAX + q];
        c.s = s;
        if (!H.active) {
            c.live = 0;
            continue;
        }
        const double2 z = H.zeta, zp = H.zeta_prev, pp = H.pi_prev, ps = H.psi;
        const double sp = H.sp;
        const double2 pi_n = csub(z, cmul(beta, pp));
        const double2 step = cscale(cmul(alpha, pi_n), sp);
        const double2 z_next = cadd(z, step);
        // zeta_{n+1} not finite or cancelled to rounding: the shifted
        // recurrence has no next iterate (broken); |zeta_{n+1} psi| beyond
        // ZETA_MAX: converged
        const bool brk = !cfinite(z_next) || cmod(z_next) < ZETA_MIN ||
                         cmod(z_next) <= BREAK_REL * (cmod(z) + cmod(step));
        if (brk || !(cmod(z_next) * cmod(ps) <= ZETA_MAX)) {
            H.active = 0;
            H.broken = brk ? 1 : 0;
            H.stopped = 1;
            H.iters = S.m;
            c.live = 0;
            continue;
        }
        const double2 alpha_s = cdiv(cmul(alpha, z), z_next);
        const double2 rz = cdiv(zp, z);
        const double2 beta_s = cmul(beta, cmul(rz, rz));
        const double2 kap = cdiv(d2(1, 0), cmul(z, ps));
        const double2 kap_next = cdiv(d2(1, 0), cmul(z_next, ps));
        c.kap = kap;
        c.beta_s = beta_s;
        c.alpha_s = alpha_s;
        c.a1 = cdiv(csub(kap, kap_next), alpha_s);
        c.a2 = cdiv(cmul(kap_next, alpha), alpha_s);
        c.sp = sp;
        c.live = 1;
        H.zeta_prev = z;
        H.zeta = z_next;
        H.pi_prev = pi_n;
    }
    if (a.sc_hist) {
        // deferred single pass: keep every step's coefficients of the iteration
        __syncthreads();
        for (int q = threadIdx.x; q < nact; q += BLOCK)
            a.sc_hist[((size_t)rhs * LMAX + j) * NSMAX + q] = a.sc[(size_t)rhs * NSMAX + q];
    }
    if (threadIdx.x == 0) {
        S.mv += 1;
        S.n += 1;
        S.l_eff = j + 1;
    }
}

__device__ __forceinline__ void sc_mr_body(const ScalarArgs &a, int rhs) {
    SeedState &S = a.seed[rhs];
    if (!S.run) return;
    const int l = a.l;
    const int L = S.exhausted ? 0 : S.l_eff;
    __shared__ double2 G[LMAX][LMAX];
    __shared__ double2 cvec[LMAX];
    __shared__ double2 g[LMAX];
    // the Cholesky factor and the forward-substitution vector, used by
    // thread 0 alone: in LDS, since indexed at run time they would otherwise
    // live in scratch memory, whose dependent accesses dominated the kernel
    __shared__ double2 Lm[LMAX][LMAX];
    __shared__ double2 zz[LMAX];
    __shared__ int lmr_sh;
    const double *row = prow(a, rhs);
    // pair index of (i, k), i <= k, in the gram kernel's order over 0..l
    auto pidx = [l](int i, int k) {
        int p = 0;
        for (int ii = 0; ii < i; ++ii) p += l + 1 - ii;
        return p + (k - i);
    };
    // the pairs (i, k) in the Gram kernel's order, 4 pairs (8 partial rows)
    // per pass over the partials (more would cost the persistent kernel, which
    // inlines this body, an occupancy step)
    constexpr int NB = 4;
    int pi_[NB], pk_[NB], rows[2 * NB];
    int cnt = 0;
    for (int i = 0; i <= L; ++i) {
        for (int k = (i == 0 ? 1 : i); k <= L; ++k) {
            pi_[cnt] = i;
            pk_[cnt] = k;
            rows[2 * cnt] = 2 * pidx(i, k);
            rows[2 * cnt + 1] = 2 * pidx(i, k) + 1;
            ++cnt;
            const bool last = i == L && k == L;
            if (cnt == NB || last) {
                double sums[2 * NB];
                block_sum_rows<2 * NB>(row, a.ps, rows, 2 * cnt, a.nblk, sums);
                if (threadIdx.x == 0) {
                    for (int q = 0; q < cnt; ++q) {
                        const double re = sums[2 * q], im = sums[2 * q + 1];
                        if (pi_[q] == 0) {
                            cvec[pk_[q] - 1] = d2(re, -im);   // <r_k, r_0> = conj(<r_0, r_k>)
                        } else {
                            G[pi_[q] - 1][pk_[q] - 1] = d2(re, im);
                            G[pk_[q] - 1][pi_[q] - 1] = d2(re, -im);
                        }
                    }
                }
                cnt = 0;
            }
        }
    }
    if (threadIdx.x == 0) {
        int n = L;
        int kok = n;
        if (n > 0) {
            double dmax = 0.0;
            for (int i = 0; i < n; ++i) dmax = G[i][i].x > dmax ? G[i][i].x : dmax;
            for (int i = 0; i < n; ++i) {
                double d = G[i][i].x;
                for (int p = 0; p < i; ++p) d -= cabs2(Lm[i][p]);
                if (!(d > CHOL_REL * dmax)) {
                    kok = i;
                    break;
                }
                const double dd = sqrt(d);
                Lm[i][i] = d2(dd, 0.0);
                for (int r = i + 1; r < n; ++r) {
                    double2 acc = G[r][i];
                    for (int p = 0; p < i; ++p) acc = csub(acc, cmul(Lm[r][p], cconj(Lm[i][p])));
                    Lm[r][i] = cscale(acc, 1.0 / dd);
                }
            }
        }
        n = kok;
        for (int i = 0; i < n; ++i) {
            double2 acc = cvec[i];
            for (int p = 0; p < i; ++p) acc = csub(acc, cmul(Lm[i][p], zz[p]));
            zz[i] = cscale(acc, 1.0 / Lm[i][i].x);
        }
        for (int i = n - 1; i >= 0; --i) {
            double2 acc = zz[i];
            for (int p = i + 1; p < n; ++p) acc = csub(acc, cmul(cconj(Lm[p][i]), g[p]));
            g[i] = cscale(acc, 1.0 / Lm[i][i].x);
        }
        for (int i = n; i < LMAX; ++i) g[i] = d2(0, 0);
        for (int i = 0; i < LMAX; ++i) S.gam[i] = g[i];
        S.l_mr = n;
        lmr_sh = n;
        if (L >= 1) S.dots += L * (L + 3) / 2;
        if (!S.exhausted) {
            if (n < l) S.broken = 1;
            if (n == l) S.omega = g[l - 1];
        }
        if (a.record && S.m < S.max_outer) {
            for (int i = 0; i < LMAX; ++i) a.tape_gam[((size_t)rhs * S.max_outer + S.m) * LMAX + i] = g[i];
        }
    }
    __syncthreads();
    const int lm = lmr_sh;
    for (int q = threadIdx.x; q < S.nact; q += BLOCK) {
        const int s = S.act[q];
        ShiftState &H = a.sh[(size_t)rhs * NSMAX + s];
        MRCoef &c = a.mc[(size_t)rhs * NSMAX + q];
        c.s = s;
        for (int k = 0; k < LMAX; ++k) c.kc[k] = d2(0, 0);
        c.inv_q = d2(1, 0);
        if (!H.active || lm == 0) {
            c.live = 0;
            continue;
        }
        const double sp = H.sp;
        double2 qs = d2(1, 0);
        double qterms = 1.0;
        for (int i = 1; i <= lm; ++i) {
            const double2 t = cmul(g[i - 1], cpowi_neg(sp, i));
            qs = csub(qs, t);
            qterms += cmod(t);
        }
        const bool brk = !cfinite(qs) || cmod(qs) < ZETA_MIN || cmod(qs) <= BREAK_REL * qterms;
        if (brk || !(cmod(H.zeta) * cmod(H.psi) * cmod(qs) <= ZETA_MAX)) {
            H.active = 0;
            H.broken = brk ? 1 : 0;
            H.stopped = 1;
            H.iters = S.m;
            c.live = 0;
            continue;
        }
        const double2 inv_q = cdiv(d2(1, 0), qs);
        const double2 kap = cdiv(d2(1, 0), cmul(H.zeta, H.psi));
        for (int k = 0; k < lm; ++k) {
            double2 acc = d2(0, 0);
            for (int i = k + 1; i <= lm; ++i) acc = cadd(acc, cmul(g[i - 1], cpowi_neg(sp, i - 1 - k)));
            c.kc[k] = cmul(kap, cmul(acc, inv_q));
        }
        c.inv_q = inv_q;
        c.live = 1;
        H.psi = cmul(H.psi, qs);
    }
}

// Mixed precision: decide whether the outer iteration ends with a reliable
// update r_0 = b - S x (FP64): when ||r_0|| has dropped below 0.1 of its
// largest value since the last one, when any shift would freeze on the
// recursively updated residual, or when the Krylov space looks exhausted.
__device__ __forceinline__ void sc_rel_body(const ScalarArgs &a, int rhs) {
    SeedState &S = a.seed[rhs];
    if (!S.run || !S.mixed) return;
    const double r02 = block_sum(prow(a, rhs) + 2 * a.ps, a.nblk);
    if (threadIdx.x != 0) return;
    const double rn = sqrt(r02);
    if (rn > S.rmax) S.rmax = rn;
    bool freeze = false;
    for (int q = 0; q < S.nact; ++q) {
        const ShiftState &H = a.sh[(size_t)rhs * NSMAX + S.act[q]];
        if (!H.active) continue;
        const bool due = S.forced ? (S.m + 1 >= H.force) : (rn / (cmod(cmul(H.zeta, H.psi)) * S.bnorm) <= FREEZE_FRAC * S.tol);
        freeze = freeze || due;
    }
    S.rel = (rn <= 0.1 * S.rmax || freeze || S.exhausted) ? 1 : 0;
}

__device__ __forceinline__ void sc_conv_body(const ScalarArgs &a, int rhs) {
    SeedState &S = a.seed[rhs];
    if (!S.run) return;
    const double *row = prow(a, rhs);
    double re, im, r02;
    sum3(row, a.ps, a.nblk, re, im, r02);
    __shared__ double rn;
    if (threadIdx.x == 0) {
        rn = sqrt(r02);
        S.rnorm0 = rn;
        S.rho1 = d2(re, im);
        if (a.record && S.m < S.max_outer) {
            TapeOuter &o = a.tape_outer[(size_t)rhs * S.max_outer + S.m];
            o.l_eff = S.l_eff;
            o.l_mr = S.exhausted ? 0 : S.l_mr;
            o.partial = S.partial;
            o.exhausted = S.exhausted;
            o.rel = S.rel;
        }
        if (S.rel) {
            S.reliable += 1;
            S.rmax = rn;
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < S.nact; q += BLOCK) {
        ShiftState &H = a.sh[(size_t)rhs * NSMAX + S.act[q]];
        if (!H.active) continue;
        const double res = rn / (cmod(cmul(H.zeta, H.psi)) * S.bnorm);
        H.res = res;
        bool done = S.forced ? (S.m + 1 >= H.force) : (res <= FREEZE_FRAC * S.tol);
        // an exhausted Krylov space ends the solve; in mixed precision the
        // residual was just recomputed in FP64, so a shift that still misses
        // its tolerance is reported as not converged
        if (S.exhausted && !S.mixed) done = true;
        if (done) {
            H.active = 0;
            H.iters = S.m + 1;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int nact = 0, anybroken = 0;
        for (int s = 0; s < S.nshift; ++s) {
            const ShiftState &H = a.sh[(size_t)rhs * NSMAX + s];
            if (H.active) S.act[nact++] = s;
            anybroken |= H.broken;
        }
        S.nact = nact;
        S.m += 1;
        S.rel = 0;
        const bool stop = (nact == 0) || S.broken || S.exhausted || (S.m >= S.max_outer);
        if (stop) {
            S.run = 0;
            if (nact > 0) {
                S.status = S.broken ? S_BREAKDOWN : S_NOT_CONVERGED;
                for (int q = 0; q < nact; ++q) a.sh[(size_t)rhs * NSMAX + S.act[q]].iters = S.m;
            } else {
                S.status = anybroken ? S_BREAKDOWN : S_OK;
            }
        }
        S.bicg_on = 1;
        S.l_eff = 0;
        S.l_mr = 0;
        S.partial = 0;
        for (int i = 0; i < LMAX; ++i) S.step_flag[i] = 0;
    }
}

// Deferred single pass: every active shift's update over the outer iteration
// that just ended, as coefficients on the iteration's basis (see DeferCoef).
// One work-item per shift replays the iteration on coefficient vectors: the
// seed's r_i, u_i exactly as the vector kernels updated them (the recorded
// beta, alpha and step flags), and the shift's u^s_i and x^s increment by the
// recurrences of the per-step form (the recorded step coefficients of every
// step and the MR coefficients).  Vectors no step defined are zero, as the
// per-step form multiplies their stale contents by zero coefficients.
__device__ __forceinline__ void sc_defer_body(const ScalarArgs &a, int rhs) {
    SeedState &S = a.seed[rhs];
    if (!S.run) return;
    const int l = a.l, nb = 2 * l + 2, self = nb;
    for (int q = threadIdx.x; q < S.nact; q += BLOCK) {
        DeferCoef &d = a.dc[(size_t)rhs * NSMAX + q];
        d.s = S.act[q];
        double2 R[LMAX + 1][NDEF], U[LMAX + 1][NDEF], w[LMAX + 1][NDEF], dx[NDEF];
        for (int i = 0; i <= l; ++i)
            for (int b = 0; b <= nb; ++b) R[i][b] = U[i][b] = w[i][b] = d2(0, 0);
        for (int b = 0; b <= nb; ++b) dx[b] = d2(0, 0);
        R[0][0] = d2(1, 0);
        U[0][1] = d2(1, 0);
        w[0][self] = d2(1, 0);
        bool live = true;
        for (int j = 0; j < l; ++j) {
            const int flag = S.step_flag[j];
            if (flag == 0) break;
            const double2 beta = S.step_beta[j];
            for (int i = 0; i <= j; ++i)
                for (int b = 0; b <= nb; ++b) U[i][b] = csub(R[i][b], cmul(beta, U[i][b]));
            for (int b = 0; b <= nb; ++b) U[j + 1][b] = d2(0, 0);
            U[j + 1][2 + 2 * j] = d2(1, 0);
            if (flag == 1) break;
            const StepCoef c = a.sc_hist[((size_t)rhs * LMAX + j) * NSMAX + q];
            if (live && c.live) {
                for (int i = 0; i <= j; ++i)
                    for (int b = 0; b <= nb; ++b) w[i][b] = csub(cmul(c.kap, R[i][b]), cmul(c.beta_s, w[i][b]));
                for (int b = 0; b <= nb; ++b) dx[b] = cfma(c.alpha_s, w[0][b], dx[b]);
                for (int b = 0; b <= nb; ++b)
                    w[j + 1][b] = csub(cadd(cmul(c.a1, R[j][b]), cmul(c.a2, U[j + 1][b])), cscale(w[j][b], c.sp));
            } else {
                live = false;
            }
            const double2 alpha = S.step_alpha[j];
            for (int i = 0; i <= j; ++i)
                for (int b = 0; b <= nb; ++b) R[i][b] = csub(R[i][b], cmul(alpha, U[i + 1][b]));
            for (int b = 0; b <= nb; ++b) R[j + 1][b] = d2(0, 0);
            R[j + 1][3 + 2 * j] = d2(1, 0);
        }
        const MRCoef &m = a.mc[(size_t)rhs * NSMAX + q];
        if (live && m.live) {
            for (int k = 0; k < l; ++k)
                for (int b = 0; b <= nb; ++b) dx[b] = cfma(m.kc[k], R[k][b], dx[b]);
            for (int b = 0; b <= nb; ++b) {
                double2 u0 = w[0][b];
                for (int i = 1; i <= l; ++i) u0 = csub(u0, cmul(S.gam[i - 1], w[i][b]));
                w[0][b] = cmul(u0, m.inv_q);
            }
        }
        // a shift whose recurrences stopped this iteration keeps the part
        // applied before: the per-step form updated it until then
        for (int b = 0; b < NDEF; ++b) {
            d.cu[b] = b <= nb ? w[0][b] : d2(0, 0);
            d.cx[b] = b <= nb ? dx[b] : d2(0, 0);
        }
        d.live = 1;
    }
}

// The seed's step recurrences of this outer iteration (the steps it completed,
// step_flag), replayed on the coefficients of its basis: r_i and u_i as sums
// over B (see SeedBasis), R[i][b] and U[i][b].  Steps in the order and with
// the arithmetic of the explicit form: u_i = r_i - beta u_i (i <= j),
// u_{j+1} = S u_j, then r_i = r_i - alpha u_{i+1} (i <= j), r_{j+1} = S r_j.
// The recurrences act on each basis index b alone: one work-item per b
// (column b of R and U).
// STEP(j, flag, beta, alpha) gives step j's flag and coefficients.
template <typename STEP>
__device__ inline void basis_replay_col(const STEP &step, int l, int b, double2 (*R)[NBB], double2 (*U)[NBB]) {
    for (int i = 0; i <= l; ++i) R[i][b] = U[i][b] = d2(0, 0);
    if (b == 0) R[0][0] = d2(1, 0);
    if (b == 1) U[0][1] = d2(1, 0);
    for (int j = 0; j < l; ++j) {
        int flag;
        double2 beta, alpha;
        step(j, flag, beta, alpha);
        if (flag == 0) break;
        for (int i = 0; i <= j; ++i) U[i][b] = csub(R[i][b], cmul(beta, U[i][b]));
        if (b == 2 + 2 * j) U[j + 1][b] = d2(1, 0);
        if (flag == 1) break;
        for (int i = 0; i <= j; ++i) R[i][b] = csub(R[i][b], cmul(alpha, U[i + 1][b]));
        if (b == 3 + 2 * j) R[j + 1][b] = d2(1, 0);
    }
}
__device__ inline void seed_basis_replay_col(const SeedState &S, int l, int b, double2 (*R)[NBB],
                                             double2 (*U)[NBB]) {
    basis_replay_col(
        [&](int j, int &flag, double2 &beta, double2 &alpha) {
            flag = S.step_flag[j];
            beta = S.step_beta[j];
            alpha = S.step_alpha[j];
        },
        l, b, R, U);
}

// Basis form, before the MR step: every r_i and u_i of the outer iteration as
// coefficients on its basis.
__device__ __forceinline__ void sc_basis_body(const ScalarArgs &a, int rhs) {
    const SeedState &S = a.seed[rhs];
    if (!S.run) return;
    __shared__ double2 R[LMAX + 1][NBB], U[LMAX + 1][NBB];
    const int b = threadIdx.x;
    if (b >= NBB) return;
    seed_basis_replay_col(S, a.l, b, R, U);
    SeedBasis &B = a.sb[rhs];
    for (int i = 0; i <= LMAX; ++i) {
        B.r[i][b] = i <= a.l ? R[i][b] : d2(0, 0);
        B.u[i][b] = i <= a.l ? U[i][b] : d2(0, 0);
    }
}

// Replay of the double pass in basis form, after outer iteration m's steps:
// the recorded steps replayed on the basis coefficients, then the recorded
// MR step, r_0 - sum_i gamma_i r_i and u_0 - sum_i gamma_i u_i (i <= lm),
// with the arithmetic of the first pass's MR update.
__device__ __forceinline__ void sc_basis_replay_body(const BasisReplayArgs &a, int rhs) {
    __shared__ double2 R[LMAX + 1][NBB], U[LMAX + 1][NBB];
    const ReplayStep *rs = a.rs + ((size_t)rhs * a.Mcap + a.m) * a.l;
    const ReplayOuter &ro = a.ro[(size_t)rhs * a.Mcap + a.m];
    const int b = threadIdx.x;
    if (b >= NBB) return;
    basis_replay_col(
        [&](int j, int &flag, double2 &beta, double2 &alpha) {
            flag = rs[j].flag;
            beta = rs[j].beta;
            alpha = rs[j].alpha;
        },
        a.l, b, R, U);
    const int lm = ro.lm < a.l ? ro.lm : a.l;
    double2 vr = R[0][b], vu = U[0][b];
    for (int i = 1; i <= lm; ++i) {
        vr = csub(vr, cmul(ro.gam[i - 1], R[i][b]));
        vu = csub(vu, cmul(ro.gam[i - 1], U[i][b]));
    }
    SeedBasis &B = a.sb[rhs];
    B.r[0][b] = vr;
    B.u[0][b] = vu;
    if (b == 0) {
        int le = 0;
        while (le < a.l && rs[le].flag == 2) ++le;
        B.nbu = (rs[0].flag == 0 && ro.lm == 0) ? 0 : 2 * le + 2;
    }
}

// Basis form, before step j >= 1: could the exhaustion test of this step
// fire?  It reads ||r_0|| after step j-1, which the basis form does not
// form; but then r_{j-1} = S^(j-1) r_0 (the steps keep r_{i+1} = S r_i), so
// ||r_0|| >= ||r_{j-1}|| / ||S||^(j-1), with norm_a an upper bound of ||S||.
// Where ||r_{j-1}|| (partial row 4, from the step's r-update) is within
// twice that factor of the test's threshold, exh_check is set and r_0's
// coefficients are written for the kernel that forms it; otherwise the test
// cannot fire and is left out.
__device__ __forceinline__ void sc_exh_body(const ScalarArgs &a, int rhs) {
    SeedState &S = a.seed[rhs];
    if (!S.run || !S.bicg_on) {
        if (threadIdx.x == 0) S.exh_check = 0;
        return;
    }
    const int j = a.j;
    const double *row = prow(a, rhs);
    const double rj1 = sqrt(block_sum(row + 4 * a.ps, a.nblk2));
    __shared__ int check;
    __shared__ double2 R[LMAX + 1][NBB], U[LMAX + 1][NBB];
    if (threadIdx.x == 0) {
        check = 0;
        if (!S.forced && S.nact > 0) {
            double mn = 1e308;
            for (int q = 0; q < S.nact; ++q) {
                const ShiftState &H = a.sh[(size_t)rhs * NSMAX + S.act[q]];
                if (!H.active) continue;
                const double sc = cmod(cmul(H.zeta, H.psi));
                mn = sc < mn ? sc : mn;
            }
            double fac = 2.0;
            for (int k = 0; k < j - 1; ++k) fac *= a.norm_a;
            if (rj1 <= fac * FREEZE_FRAC * S.tol * S.bnorm * mn) check = 1;
        }
        S.exh_check = check;
    }
    __syncthreads();
    if (!check) return;
    const int b = threadIdx.x;
    if (b >= NBB) return;
    seed_basis_replay_col(S, a.l, b, R, U);
    a.sb[rhs].r[0][b] = R[0][b];
}

}  // namespace dev
}  // namespace msb
