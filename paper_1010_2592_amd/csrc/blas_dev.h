// Device bodies of the streaming vector stages of multi-shift BiCGstab(l)
// (see blas.hip for what each computes).  bx and gx are the element block and
// the number of element blocks, rhs the right-hand side: the one-launch-per-
// stage kernels pass blockIdx.x, gridDim.x and blockIdx.y, the persistent
// kernel its virtual block coordinates.
#pragma once
#include "common.h"
#include "kernels.h"

namespace msb {
namespace dev {

template <typename T>
__device__ __forceinline__ C<T> cvt(double2 z) { return to_c<T>(z); }

// Where seed vector r_i / u_i of right-hand side rhs is read: its row of R / U
// (base already offset to the right-hand side), or the store of the
// pseudo-double pass for the one vector named by r_src_i / u_src_i.
template <typename T>
__device__ __forceinline__ const C<T> *rsrc(const VecArgs<T> &a, const C<T> *R, int i, int rhs, long n) {
    return i == a.r_src_i ? a.r_src + (size_t)rhs * a.r_src_rs : R + (size_t)i * n;
}
template <typename T>
__device__ __forceinline__ const C<T> *usrc(const VecArgs<T> &a, const C<T> *U, int i, int rhs, long n) {
    return i == a.u_src_i ? a.u_src + (size_t)rhs * a.u_src_rs : U + (size_t)i * n;
}

// The MR step's view of the seed vectors (see VecArgs::mr_dyn): with mr_dyn
// the store redirect follows the device's count of completed BiCG steps L,
// otherwise the fixed r_src_i / u_src_i; lm is the number of MR terms the
// scalar stage applied (terms beyond it are not read).
template <typename T>
struct MRView {
    int ri = -1, ui = -1, lm = 0;
    const C<T> *rp = nullptr, *up = nullptr;
};
template <typename T>
__device__ __forceinline__ MRView<T> mr_view(const VecArgs<T> &a, int rhs, int lmax) {
    MRView<T> v;
    v.lm = lmax;
    if (!a.mr_dyn) {
        v.ri = a.r_src_i;
        v.ui = a.u_src_i;
        v.rp = a.r_src ? a.r_src + (size_t)rhs * a.r_src_rs : nullptr;
        v.up = a.u_src ? a.u_src + (size_t)rhs * a.u_src_rs : nullptr;
        return v;
    }
    const SeedState &S = a.seed[rhs];
    const int L = S.l_eff;
    v.lm = S.l_mr < lmax ? S.l_mr : lmax;
    if (L >= 1) {
        const C<T> *base = a.st_base + (size_t)rhs * a.st_rs;
        v.ri = L;
        v.rp = base + (size_t)(2 * L - 1) * a.n;
        if (L >= a.l || S.step_flag[L] == 0) {
            v.ui = L;
            v.up = base + (size_t)(2 * L - 2) * a.n;
        }
    }
    return v;
}

// ---------------------------------------------------------------------------
// u_i = r_i - beta u_i for i in [I0, I1]: MODE 0 all of 0..J (the BiCG step's
// direction update), MODE 1 only u_J (the one the step's Mv needs; the others
// then follow in the fused r-update), MODE 2 only u_0..u_{J-1} (completes a
// step that ended after its Mv of u_J).
template <typename T, int J, int MODE = 0>
__device__ __forceinline__ void seed_u_body(const VecArgs<T> &a, int bx, int gx, int rhs) {
    constexpr int I0 = (MODE == 1) ? J : 0;
    constexpr int I1 = (MODE == 2) ? J - 1 : J;
    if (!gate_open(a.gate, rhs)) return;
    const long n = a.n;
    const C<T> beta = cvt<T>(ld(a.beta, rhs));
    C<T> *R = a.R + (size_t)rhs * (a.l + 1) * n;
    C<T> *U = a.U + (size_t)rhs * (a.l + 1) * n;
    for (long e = (long)bx * BLOCK + threadIdx.x; e < n; e += (long)gx * BLOCK) {
#pragma unroll
        for (int i = I0; i <= I1; ++i) {
            const C<T> r = rsrc(a, R, i, rhs, n)[e];
            const C<T> u = usrc(a, U, i, rhs, n)[e];
            U[i * n + e] = csub(r, cmul(beta, u));
        }
    }
}

// r_i -= alpha u_{i+1}, i = 0..J.  FU (fused): the step's direction update of
// u_0..u_{J-1} (u_i = r_i - beta u_i, deferred from before the Mv, which
// needs only u_J) is done here on the same pass, with the same arithmetic:
// u_0..u_{J-1} are read once, updated in registers and written back.
template <typename T, int J, bool SHIFTS, bool XH, bool FU = false>
__device__ __forceinline__ void r_update_body(const VecArgs<T> &a, int bx, int gx, int rhs) {
    if (!gate_open(a.gate, rhs)) return;
    const long n = a.n;
    const double2 alpha_d = ld(a.alpha, rhs);
    const C<T> alpha = cvt<T>(alpha_d);
    C<T> *R = a.R + (size_t)rhs * (a.l + 1) * n;
    C<T> *U = a.U + (size_t)rhs * (a.l + 1) * n;
    const C<T> beta = FU ? cvt<T>(ld(a.beta, rhs)) : mk<T>(0, 0);
    const int nact = SHIFTS ? a.seed[rhs].nact : 0;
    const StepCoef *sc = SHIFTS ? a.sc + (size_t)rhs * NSMAX : nullptr;
    double part[1] = {0.0};
    for (long e = (long)bx * BLOCK + threadIdx.x; e < n; e += (long)gx * BLOCK) {
        C<T> r[J + 1], u1[J + 1];
        C<T> u0n = mk<T>(0, 0);
#pragma unroll
        for (int i = 0; i <= J; ++i) r[i] = rsrc(a, R, i, rhs, n)[e];
        if (FU && J >= 1) {
            // u_i (i < J) = r_i - beta u_i; u1[i] = u_{i+1}
#pragma unroll
            for (int i = 0; i < J; ++i) {
                const C<T> un = csub(r[i], cmul(beta, usrc(a, U, i, rhs, n)[e]));
                U[i * n + e] = un;
                if (i == 0) u0n = un;
                else u1[i - 1] = un;
            }
            u1[J - 1] = usrc(a, U, J, rhs, n)[e];
            u1[J] = usrc(a, U, J + 1, rhs, n)[e];
        } else {
#pragma unroll
            for (int i = 0; i <= J; ++i) u1[i] = usrc(a, U, i + 1, rhs, n)[e];
        }
        if (SHIFTS) {
            for (int q = 0; q < nact; ++q) {
                const StepCoef c = sc[q];
                if (!c.live) continue;
                const C<T> kap = cvt<T>(c.kap), bs = cvt<T>(c.beta_s), as = cvt<T>(c.alpha_s);
                const C<T> a1 = cvt<T>(c.a1), a2 = cvt<T>(c.a2);
                const T sp = (T)c.sp;
                C<T> *W = a.W + ((size_t)rhs * a.nshift + c.s) * (a.l + 1) * n;
                double2 *X = a.X + ((size_t)rhs * a.nshift + c.s) * n;
                C<T> w[J + 2];
#pragma unroll
                for (int i = 0; i <= J; ++i) w[i] = csub(cmul(kap, r[i]), cmul(bs, W[i * n + e]));
                X[e] = cfma(c.alpha_s, d2((double)w[0].x, (double)w[0].y), X[e]);
                (void)as;
                w[J + 1] = csub(cadd(cmul(a1, r[J]), cmul(a2, u1[J])), cscale(w[J], sp));
#pragma unroll
                for (int i = 0; i <= J + 1; ++i) W[i * n + e] = w[i];
            }
        }
        if (XH) {
            // seed solution x += alpha u_0, accumulated in FP64
            const C<T> u0 = (FU && J >= 1) ? u0n : usrc(a, U, 0, rhs, n)[e];
            double2 *xh = a.XH + (size_t)rhs * n;
            xh[e] = cfma(alpha_d, d2((double)u0.x, (double)u0.y), xh[e]);
        }
#pragma unroll
        for (int i = 0; i <= J; ++i) {
            const C<T> rn = csub(r[i], cmul(alpha, u1[i]));
            R[i * n + e] = rn;
            if (i == 0) part[0] += (double)rn.x * rn.x + (double)rn.y * rn.y;
        }
    }
    if (a.partials)
        block_reduce_store<1>(part, a.part + (size_t)rhs * PMAX * a.ps + 3 * a.ps + bx, a.ps);
}

template <typename T, int L>
__device__ __forceinline__ void gram_body(const VecArgs<T> &a, int bx, int gx, int rhs) {
    if (!gate_open(a.gate, rhs)) return;
    constexpr int NP = (L + 1) * (L + 2) / 2;
    const long n = a.n;
    const C<T> *R = a.R + (size_t)rhs * (a.l + 1) * n;
    const MRView<T> mv = mr_view(a, rhs, L);
    double acc[2 * NP];
#pragma unroll
    for (int p = 0; p < 2 * NP; ++p) acc[p] = 0.0;
    for (long e = (long)bx * BLOCK + threadIdx.x; e < n; e += (long)gx * BLOCK) {
        C<T> r[L + 1];
#pragma unroll
        for (int i = 0; i <= L; ++i) r[i] = (i == mv.ri ? mv.rp : R + (size_t)i * n)[e];
        int p = 0;
#pragma unroll
        for (int i = 0; i <= L; ++i)
#pragma unroll
            for (int k = i; k <= L; ++k) {
                // conj(r_i) r_k
                acc[2 * p] += (double)r[i].x * r[k].x + (double)r[i].y * r[k].y;
                acc[2 * p + 1] += (double)r[i].x * r[k].y - (double)r[i].y * r[k].x;
                ++p;
            }
    }
    block_reduce_store<2 * NP>(acc, a.part + (size_t)rhs * PMAX * a.ps + bx, a.ps);
}

template <typename T, int L, bool SHIFTS, bool XH>
__device__ __forceinline__ void mr_update_body(const VecArgs<T> &a, int bx, int gx, int rhs) {
    if (!gate_open(a.gate, rhs)) return;
    const long n = a.n;
    C<T> *R = a.R + (size_t)rhs * (a.l + 1) * n;
    C<T> *U = a.U + (size_t)rhs * (a.l + 1) * n;
    const C<T> *rt = a.rt ? a.rt + (size_t)rhs * n : nullptr;
    C<T> g[L + 1];
    double2 gd[L + 1];
#pragma unroll
    for (int i = 1; i <= L; ++i) {
        CoefRef c = a.gam;
        c.p += (i - 1) * sizeof(double2);
        gd[i] = ld(c, rhs);
        g[i] = cvt<T>(gd[i]);
    }
    const int nact = SHIFTS ? a.seed[rhs].nact : 0;
    const MRCoef *mc = SHIFTS ? a.mc + (size_t)rhs * NSMAX : nullptr;
    const MRView<T> mv = mr_view(a, rhs, L);
    const int lm = mv.lm;     // terms applied (zero coefficients beyond)
    double part[3] = {0.0, 0.0, 0.0};
    for (long e = (long)bx * BLOCK + threadIdx.x; e < n; e += (long)gx * BLOCK) {
        C<T> r[L + 1];
#pragma unroll
        for (int i = 0; i <= L; ++i) r[i] = i <= lm ? (i == mv.ri ? mv.rp : R + (size_t)i * n)[e] : mk<T>(0, 0);
        if (SHIFTS) {
            for (int q = 0; q < nact; ++q) {
                const MRCoef &c = mc[q];
                if (!c.live) continue;
                C<T> *W = a.W + ((size_t)rhs * a.nshift + c.s) * (a.l + 1) * n;
                double2 *X = a.X + ((size_t)rhs * a.nshift + c.s) * n;
                double2 x = X[e];
#pragma unroll
                for (int k = 0; k < L; ++k) x = cfma(c.kc[k], d2((double)r[k].x, (double)r[k].y), x);
                X[e] = x;
                C<T> w0 = W[e];
#pragma unroll
                for (int i = 1; i <= L; ++i) w0 = csub(w0, cmul(g[i], W[i * n + e]));
                W[e] = cmul(w0, cvt<T>(c.inv_q));
            }
        }
        if (XH) {
            // seed solution x += sum_i gamma_i r_{i-1}, accumulated in FP64
            double2 *xh = a.XH + (size_t)rhs * n;
            double2 x = xh[e];
#pragma unroll
            for (int i = 1; i <= L; ++i) x = cfma(gd[i], d2((double)r[i - 1].x, (double)r[i - 1].y), x);
            xh[e] = x;
        }
        C<T> r0 = r[0];
#pragma unroll
        for (int i = 1; i <= L; ++i) r0 = csub(r0, cmul(g[i], r[i]));
        R[e] = r0;
        C<T> u0 = (0 == mv.ui ? mv.up : U)[e];
#pragma unroll
        for (int i = 1; i <= L; ++i)
            if (i <= lm) u0 = csub(u0, cmul(g[i], (i == mv.ui ? mv.up : U + (size_t)i * n)[e]));
        U[e] = u0;
        if (a.partials) {
            if (rt) {
                const C<T> t = rt[e];
                part[0] += (double)t.x * r0.x + (double)t.y * r0.y;
                part[1] += (double)t.x * r0.y - (double)t.y * r0.x;
            }
            part[2] += (double)r0.x * r0.x + (double)r0.y * r0.y;
        }
    }
    if (a.partials)
        block_reduce_store<3>(part, a.part + (size_t)rhs * PMAX * a.ps + bx, a.ps);
}

// r_0 = b - v in FP64 (v = S x), stored in the iteration's precision;
// partials of <rt, r_0> and ||r_0||^2 from the FP64 value
template <typename T>
__device__ __forceinline__ void rel_update_body(const VecArgs<T> &a, const double2 *b, const double2 *v,                                                       double2 *y, CoefRef yc, int bx, int gx, int rhs) {
    if (!gate_open(a.gate, rhs)) return;
    const long n = a.n;
    C<T> *R = a.R + (size_t)rhs * (a.l + 1) * n;
    const C<T> *rt = a.rt ? a.rt + (size_t)rhs * n : nullptr;   // null: sparse r~, dot taken afterwards
    const double2 *br = b + (size_t)rhs * n, *vr = v + (size_t)rhs * n;
    double2 *yr = y ? y + (size_t)rhs * n : nullptr;
    const double2 c = y ? ld(yc, rhs) : d2(0, 0);
    double p[3] = {0.0, 0.0, 0.0};
    for (long e = (long)bx * BLOCK + threadIdx.x; e < n; e += (long)gx * BLOCK) {
        const double2 ve = vr[e];
        const double2 r0 = csub(br[e], ve);
        R[e] = to_c<T>(r0);
        if (yr) yr[e] = cfma(c, ve, yr[e]);
        if (rt) {
            const C<T> t = rt[e];
            p[0] += (double)t.x * r0.x + (double)t.y * r0.y;
            p[1] += (double)t.x * r0.y - (double)t.y * r0.x;
        }
        p[2] += r0.x * r0.x + r0.y * r0.y;
    }
    block_reduce_store<3>(p, a.part + (size_t)rhs * PMAX * a.ps + bx, a.ps);
}

// ---------------------------------------------------------------------------
// Basis form of the seed (MSB_SEED_BASIS, FP64).  Vector b of the basis of
// right-hand side rhs, element e.
__device__ __forceinline__ double2 bvec(const BasisArgs<double> &a, int b, int rhs, long e) {
    return a.bv[b][(size_t)rhs * a.brs[b] + e];
}

// dst = x - c y (the direction update u_j = r_j - beta u_j before the step's
// first Mv, the residual update r_j = r_j - alpha u_{j+1} before its second),
// ||dst||^2 into partial row prow
__device__ __forceinline__ void basis_axpy_body(const BasisArgs<double> &a, int bx, int gx, int rhs) {
    if (!gate_open(a.gate, rhs)) return;
    const long n = a.n;
    const double2 c = ld(a.c, rhs);
    const double2 *x = a.x + (size_t)rhs * a.x_rs, *y = a.y + (size_t)rhs * a.y_rs;
    double2 *d = a.dst + (size_t)rhs * a.dst_rs;
    double part[1] = {0.0};
    for (long e = (long)bx * BLOCK + threadIdx.x; e < n; e += (long)gx * BLOCK) {
        const double2 v = csub(x[e], cmul(c, y[e]));
        d[e] = v;
        part[0] += v.x * v.x + v.y * v.y;
    }
    if (a.prow >= 0)
        block_reduce_store<1>(part, a.part + (size_t)rhs * PMAX * a.ps + (size_t)a.prow * a.ps + bx, a.ps);
}

// ||r_0||^2 into partial row 3, r_0 formed from the first nbu basis vectors
// with the coefficients sc_exh wrote (gated on its check)
__device__ __forceinline__ void basis_r0norm_body(const BasisArgs<double> &a, int bx, int gx, int rhs) {
    if (!gate_open(a.gate, rhs)) return;
    __shared__ double2 cf[NBB];
    for (int b = threadIdx.x; b < NBB; b += BLOCK) cf[b] = a.sb[rhs].r[0][b];
    __syncthreads();
    const long n = a.n;
    const int nbu = a.nbu;
    double part[1] = {0.0};
    for (long e = (long)bx * BLOCK + threadIdx.x; e < n; e += (long)gx * BLOCK) {
        double2 r = d2(0, 0);
        for (int b = 0; b < nbu; ++b)
            if (b != 1) r = cfma(cf[b], bvec(a, b, rhs, e), r);   // no r_i holds u_0 (B_1)
        part[0] += r.x * r.x + r.y * r.y;
    }
    block_reduce_store<1>(part, a.part + (size_t)rhs * PMAX * a.ps + 3 * a.ps + bx, a.ps);
}

// Basis vectors the MR step reads: those of the L = l_eff steps the outer
// iteration completed (r_i and u_i, i <= L, lie in B_0 .. B_{2L+1})
__device__ __forceinline__ int basis_used(const SeedState &S) { return 2 * S.l_eff + 2; }

// The MR step's Gram matrix, conj(r_i) r_k for 0 <= i <= k <= L in the order
// of the explicit form's partials, each r_i formed in registers from the
// basis with the coefficients of sc_basis.  B_1 = u_0 is not read: the steps
// add multiples of u_0 to the u_i only (r_i - alpha u_{i+1} with i + 1 >= 1,
// and u_i for i >= 1 never takes up u_0), so its coefficient in every r_i is
// exactly zero.
template <int L>
__device__ __forceinline__ void basis_gram_body(const BasisArgs<double> &a, int bx, int gx, int rhs) {
    if (!gate_open(a.gate, rhs)) return;
    constexpr int NP = (L + 1) * (L + 2) / 2;
    constexpr int NBL = 2 * L + 2;
    __shared__ double2 cr[L + 1][NBL];
    for (int k = threadIdx.x; k < (L + 1) * NBL; k += BLOCK) cr[k / NBL][k % NBL] = a.sb[rhs].r[k / NBL][k % NBL];
    __syncthreads();
    const int nbu = basis_used(a.seed[rhs]);
    const long n = a.n;
    double acc[2 * NP];
#pragma unroll
    for (int p = 0; p < 2 * NP; ++p) acc[p] = 0.0;
    for (long e = (long)bx * BLOCK + threadIdx.x; e < n; e += (long)gx * BLOCK) {
        // the coefficients are read from LDS in every pass: kept in registers
        // across the loop they would take (L+1)(2L+2) complex registers
        asm volatile("" ::: "memory");
        double2 B[NBL];
#pragma unroll
        for (int b = 0; b < NBL; ++b) B[b] = (b < nbu && b != 1) ? bvec(a, b, rhs, e) : d2(0, 0);
        double2 r[L + 1];
#pragma unroll
        for (int i = 0; i <= L; ++i) {
            double2 v = d2(0, 0);
#pragma unroll
            for (int b = 0; b < NBL; ++b)
                if (b != 1) v = cfma(cr[i][b], B[b], v);
            r[i] = v;
        }
        int p = 0;
#pragma unroll
        for (int i = 0; i <= L; ++i)
#pragma unroll
            for (int k = i; k <= L; ++k) {
                acc[2 * p] += r[i].x * r[k].x + r[i].y * r[k].y;
                acc[2 * p + 1] += r[i].x * r[k].y - r[i].y * r[k].x;
                ++p;
            }
    }
    block_reduce_store<2 * NP>(acc, a.part + (size_t)rhs * PMAX * a.ps + bx, a.ps);
}

// The MR update: r_0 = r_0 - sum_i gamma_i r_i and u_0 = u_0 - sum_i gamma_i u_i
// (i = 1 .. l_mr), formed from the basis with the combined coefficients and
// written over B_0 and B_1; partials <r~, r_0> (rows 0, 1; left at zero for
// the sparse list) and ||r_0||^2 (row 2)
template <int L>
__device__ __forceinline__ void basis_mr_update_body(const BasisArgs<double> &a, int bx, int gx, int rhs) {
    if (!gate_open(a.gate, rhs)) return;
    constexpr int NBL = 2 * L + 2;
    const SeedState &S = a.seed[rhs];
    __shared__ double2 c_r[NBL], c_u[NBL];
    if (threadIdx.x < NBL) {
        const int b = threadIdx.x;
        const SeedBasis &SB = a.sb[rhs];
        const int lm = S.l_mr < L ? S.l_mr : L;
        double2 vr = SB.r[0][b], vu = SB.u[0][b];
        for (int i = 1; i <= lm; ++i) {
            vr = csub(vr, cmul(S.gam[i - 1], SB.r[i][b]));
            vu = csub(vu, cmul(S.gam[i - 1], SB.u[i][b]));
        }
        c_r[b] = vr;
        c_u[b] = vu;
    }
    __syncthreads();
    const int nbu = basis_used(S);
    const long n = a.n;
    double2 *R0 = a.R0 + (size_t)rhs * a.r0_rs, *U0 = a.U0 + (size_t)rhs * a.u0_rs;
    const double2 *rt = a.rt ? a.rt + (size_t)rhs * n : nullptr;
    double part[3] = {0.0, 0.0, 0.0};
    // with the sparse r~ (basis_spec_body, before this kernel: r_0 and u_0
    // are overwritten here): <r~, r_0> into rows 0, 1 and the next outer
    // iteration's first direction update with its beta
    double2 *WU = a.wu ? a.wu + (size_t)rhs * n : nullptr;
    const double2 bspec = S.beta_spec;
    if (WU && bx == 0 && threadIdx.x == 0) {
        part[0] = S.spec_rho1.x;
        part[1] = S.spec_rho1.y;
    }
    for (long e = (long)bx * BLOCK + threadIdx.x; e < n; e += (long)gx * BLOCK) {
        asm volatile("" ::: "memory");   // coefficients from LDS in every pass (as in the Gram kernel)
        double2 B[NBL];
#pragma unroll
        for (int b = 0; b < NBL; ++b) B[b] = b < nbu ? bvec(a, b, rhs, e) : d2(0, 0);
        double2 r0 = d2(0, 0), u0 = d2(0, 0);
#pragma unroll
        for (int b = 0; b < NBL; ++b) {
            r0 = cfma(c_r[b], B[b], r0);
            u0 = cfma(c_u[b], B[b], u0);
        }
        R0[e] = r0;
        U0[e] = u0;
        if (WU) WU[e] = csub(r0, cmul(bspec, u0));
        if (rt) {
            const double2 t = rt[e];
            part[0] += t.x * r0.x + t.y * r0.y;
            part[1] += t.x * r0.y - t.y * r0.x;
        }
        part[2] += r0.x * r0.x + r0.y * r0.y;
    }
    block_reduce_store<3>(part, a.part + (size_t)rhs * PMAX * a.ps + bx, a.ps);
}

// Basis form with a sparse r~, after the MR step's coefficients and before
// the MR update overwrites r_0 and u_0: r_0 after the MR step at the list's
// entries (the MR update's combined coefficients), <r~, r_0>, and the next
// outer iteration's beta = alpha rho_1 / rho_0 with rho_0 <- -omega rho_0
// (as its first step will find it), into seed_w[rhs] (one block per rhs).
template <int L>
__device__ __forceinline__ void basis_spec_body(const BasisArgs<double> &a, int rhs) {
    if (!gate_open(a.gate, rhs)) return;
    constexpr int NBL = 2 * L + 2;
    const SeedState &S = a.seed[rhs];
    __shared__ double2 c_r[NBL];
    __shared__ double2 rk[SPARSE_MAX];
    if (threadIdx.x < NBL) {
        const int b = threadIdx.x;
        const SeedBasis &SB = a.sb[rhs];
        const int lm = S.l_mr < L ? S.l_mr : L;
        double2 vr = SB.r[0][b];
        for (int i = 1; i <= lm; ++i) vr = csub(vr, cmul(S.gam[i - 1], SB.r[i][b]));
        c_r[b] = vr;
    }
    __syncthreads();
    const int nbu = basis_used(S);
    const int nk = a.sp_cnt[rhs];
    if ((int)threadIdx.x < nk) {
        const long e = a.sp_idx[(size_t)rhs * a.sp_max + threadIdx.x];
        double2 r0 = d2(0, 0);
        for (int b = 0; b < nbu; ++b) r0 = cfma(c_r[b], bvec(a, b, rhs, e), r0);
        rk[threadIdx.x] = r0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double p0 = 0.0, p1 = 0.0;
        for (int k = 0; k < nk; ++k) {
            const double2 t = a.sp_val[(size_t)rhs * a.sp_max + k], o = rk[k];
            p0 += t.x * o.x + t.y * o.y;
            p1 += t.x * o.y - t.y * o.x;
        }
        const double2 rho0 = cneg(cmul(S.omega, S.rho0));
        a.seed_w[rhs].spec_rho1 = d2(p0, p1);
        a.seed_w[rhs].beta_spec = cdiv(cmul(S.alpha, d2(p0, p1)), rho0);
    }
}

// Replay of the double pass in basis form: r_0 and u_0 after the outer
// iteration, written over B_0 and B_1 (no partial sums: the replay takes no
// inner products)
template <int L>
__device__ __forceinline__ void basis_combine_body(const BasisArgs<double> &a, int bx, int gx, int rhs) {
    if (!gate_open(a.gate, rhs)) return;
    constexpr int NBL = 2 * L + 2;
    const SeedBasis &SB = a.sb[rhs];
    __shared__ double2 c_r[NBL], c_u[NBL];
    if (threadIdx.x < NBL) {
        c_r[threadIdx.x] = SB.r[0][threadIdx.x];
        c_u[threadIdx.x] = SB.u[0][threadIdx.x];
    }
    __syncthreads();
    const int nbu = SB.nbu;
    const long n = a.n;
    double2 *R0 = a.R0 + (size_t)rhs * a.r0_rs, *U0 = a.U0 + (size_t)rhs * a.u0_rs;
    for (long e = (long)bx * BLOCK + threadIdx.x; e < n; e += (long)gx * BLOCK) {
        asm volatile("" ::: "memory");   // coefficients from LDS in every pass
        double2 B[NBL];
#pragma unroll
        for (int b = 0; b < NBL; ++b) B[b] = b < nbu ? bvec(a, b, rhs, e) : d2(0, 0);
        double2 r0 = d2(0, 0), u0 = d2(0, 0);
#pragma unroll
        for (int b = 0; b < NBL; ++b) {
            r0 = cfma(c_r[b], B[b], r0);
            u0 = cfma(c_u[b], B[b], u0);
        }
        R0[e] = r0;
        U0[e] = u0;
    }
}

}  // namespace dev
}  // namespace msb
