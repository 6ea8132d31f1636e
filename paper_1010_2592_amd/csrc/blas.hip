// Streaming vector kernels of multi-shift BiCGstab(l) for gfx950.
//
// All of them are elementwise over the 12 V complex numbers of a spinor (one
// block row per right-hand side, grid-stride over elements), so they are
// bound by HBM bandwidth; each one reads its operands once, fuses every
// update that uses the same operands, and reduces inner products with a fixed
// shuffle tree (deterministic, FP64 accumulation) into per-block partials.
//
//   seed_u     u_i <- r_i - beta u_i,  i = 0..j          (BiCG part, step j)
//   r_update   r_i <- r_i - alpha u_{i+1}, i = 0..j, partial ||r_0||^2, and
//              -- single-pass only -- every active shift in the same sweep:
//                u^s_i <- kappa_n r_i - beta^s u^s_i           (i <= j)
//                x^s   <- x^s + alpha^s u^s_0
//                u^s_{j+1} <- a1 r_j + a2 u_{j+1} - sigma' u^s_j
//              (r_i here is the value before the seed update; a1, a2 encode
//              (kappa_n r_j^old - kappa_{n+1} r_j^new) / alpha^s)
//   gram       <r_i, r_k>, 0 <= i <= k <= l (MR normal equations)
//   mr_update  r_0 <- r_0 - sum gamma_i r_i, u_0 <- u_0 - sum gamma_i u_i,
//              partials <rt, r_0>, ||r_0||^2, and per active shift:
//                x^s   <- x^s + sum_k kappa c^s_k r_k
//                u^s_0 <- (u^s_0 - sum_i gamma_i u^s_i) / q^s
//
// The seed vectors are loaded once per element and reused for every shift;
// this is the paper's sum_s M_s l (0.5 l + 4.5) extra axpys (Section 2)
// executed as one pass over the shift vectors per BiCG step and per MR step.
#include "common.h"
#include "kernels.h"

namespace msb {

namespace {

template <typename T>
__device__ __forceinline__ C<T> cvt(double2 z) { return to_c<T>(z); }

// ---------------------------------------------------------------------------
template <typename T, int J>
__global__ __launch_bounds__(BLOCK) void k_seed_u(VecArgs<T> a) {
    const int rhs = blockIdx.y;
    if (!gate_open(a.gate, rhs)) return;
    const long n = a.n;
    const C<T> beta = cvt<T>(ld(a.beta, rhs));
    C<T> *R = a.R + (size_t)rhs * (a.l + 1) * n;
    C<T> *U = a.U + (size_t)rhs * (a.l + 1) * n;
    for (long e = (long)blockIdx.x * BLOCK + threadIdx.x; e < n; e += (long)gridDim.x * BLOCK) {
#pragma unroll
        for (int i = 0; i <= J; ++i) {
            const C<T> r = R[i * n + e];
            const C<T> u = U[i * n + e];
            U[i * n + e] = csub(r, cmul(beta, u));
        }
    }
}

template <typename T, int J, bool SHIFTS, bool XH>
__global__ __launch_bounds__(BLOCK) void k_r_update(VecArgs<T> a) {
    const int rhs = blockIdx.y;
    if (!gate_open(a.gate, rhs)) return;
    const long n = a.n;
    const double2 alpha_d = ld(a.alpha, rhs);
    const C<T> alpha = cvt<T>(alpha_d);
    C<T> *R = a.R + (size_t)rhs * (a.l + 1) * n;
    const C<T> *U = a.U + (size_t)rhs * (a.l + 1) * n;
    const int nact = SHIFTS ? a.seed[rhs].nact : 0;
    const StepCoef *sc = SHIFTS ? a.sc + (size_t)rhs * NSMAX : nullptr;
    double part[1] = {0.0};
    for (long e = (long)blockIdx.x * BLOCK + threadIdx.x; e < n; e += (long)gridDim.x * BLOCK) {
        C<T> r[J + 1], u1[J + 1];
#pragma unroll
        for (int i = 0; i <= J; ++i) {
            r[i] = R[i * n + e];
            u1[i] = U[(i + 1) * n + e];
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
            const C<T> u0 = U[e];
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
        block_reduce_store<1>(part, a.part + (size_t)rhs * PMAX * a.ps + 3 * a.ps + blockIdx.x, a.ps);
}

template <typename T, int L>
__global__ __launch_bounds__(BLOCK) void k_gram(VecArgs<T> a) {
    const int rhs = blockIdx.y;
    if (!gate_open(a.gate, rhs)) return;
    constexpr int NP = (L + 1) * (L + 2) / 2;
    const long n = a.n;
    const C<T> *R = a.R + (size_t)rhs * (a.l + 1) * n;
    double acc[2 * NP];
#pragma unroll
    for (int p = 0; p < 2 * NP; ++p) acc[p] = 0.0;
    for (long e = (long)blockIdx.x * BLOCK + threadIdx.x; e < n; e += (long)gridDim.x * BLOCK) {
        C<T> r[L + 1];
#pragma unroll
        for (int i = 0; i <= L; ++i) r[i] = R[i * n + e];
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
    block_reduce_store<2 * NP>(acc, a.part + (size_t)rhs * PMAX * a.ps + blockIdx.x, a.ps);
}

template <typename T, int L, bool SHIFTS, bool XH>
__global__ __launch_bounds__(BLOCK) void k_mr_update(VecArgs<T> a) {
    const int rhs = blockIdx.y;
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
    double part[3] = {0.0, 0.0, 0.0};
    for (long e = (long)blockIdx.x * BLOCK + threadIdx.x; e < n; e += (long)gridDim.x * BLOCK) {
        C<T> r[L + 1];
#pragma unroll
        for (int i = 0; i <= L; ++i) r[i] = R[i * n + e];
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
        C<T> u0 = U[e];
#pragma unroll
        for (int i = 1; i <= L; ++i) u0 = csub(u0, cmul(g[i], U[i * n + e]));
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
        block_reduce_store<3>(part, a.part + (size_t)rhs * PMAX * a.ps + blockIdx.x, a.ps);
}

// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_convert_in(C<T> *dst, const double2 *src, long n, long ds, long ss) {
    const int rhs = blockIdx.y;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        dst[rhs * ds + e] = to_c<T>(src[rhs * ss + e]);
}

template <typename T>
__global__ void k_convert_out(double2 *dst, const C<T> *src, long n, long ds, long ss) {
    const int rhs = blockIdx.y;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const C<T> z = src[rhs * ss + e];
        dst[rhs * ds + e] = d2((double)z.x, (double)z.y);
    }
}

template <typename T>
__global__ void k_zero(C<T> *dst, long n, long stride) {
    const int rhs = blockIdx.y;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        dst[rhs * stride + e] = mk<T>(0, 0);
}

// partials: slot 0,1 = <x, y>, slot 2 = ||y||^2
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_dot(const C<T> *x, const C<T> *y, long n, double *part, long ps, Gate gate) {
    const int rhs = blockIdx.y;
    if (!gate_open(gate, rhs)) return;
    double p[3] = {0.0, 0.0, 0.0};
    const C<T> *xr = x + (size_t)rhs * n, *yr = y + (size_t)rhs * n;
    for (long e = (long)blockIdx.x * BLOCK + threadIdx.x; e < n; e += (long)gridDim.x * BLOCK) {
        const C<T> a = xr[e], b = yr[e];
        p[0] += (double)a.x * b.x + (double)a.y * b.y;
        p[1] += (double)a.x * b.y - (double)a.y * b.x;
        p[2] += (double)b.x * b.x + (double)b.y * b.y;
    }
    block_reduce_store<3>(p, part + (size_t)rhs * PMAX * ps + blockIdx.x, ps);
}

// partial slot 0 = ||x - y||^2
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_diffnorm(const C<T> *x, const C<T> *y, long n, long sx, long sy,
                                                    double *part, long ps) {
    const int rhs = blockIdx.y;
    double p[1] = {0.0};
    const C<T> *xr = x + (size_t)rhs * sx, *yr = y + (size_t)rhs * sy;
    for (long e = (long)blockIdx.x * BLOCK + threadIdx.x; e < n; e += (long)gridDim.x * BLOCK) {
        const C<T> a = xr[e], b = yr[e];
        const double dx = (double)a.x - b.x, dy = (double)a.y - b.y;
        p[0] += dx * dx + dy * dy;
    }
    block_reduce_store<1>(p, part + (size_t)rhs * PMAX * ps + blockIdx.x, ps);
}

__global__ void k_ysum(double2 *y, const double2 *X, const double *w, long n, int ns) {
    const int rhs = blockIdx.y;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        double2 acc = d2(0, 0);
        for (int s = 0; s < ns; ++s) {
            const double2 z = X[((size_t)rhs * ns + s) * n + e];
            const double ws = w[rhs * ns + s];
            acc.x += ws * z.x;
            acc.y += ws * z.y;
        }
        y[(size_t)rhs * n + e] = acc;
    }
}

// r_0 = b - v in FP64 (v = S x), stored in the iteration's precision;
// partials of <rt, r_0> and ||r_0||^2 from the FP64 value
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_rel_update(VecArgs<T> a, const double2 *b, const double2 *v,
                                                      double2 *y, CoefRef yc) {
    const int rhs = blockIdx.y;
    if (!gate_open(a.gate, rhs)) return;
    const long n = a.n;
    C<T> *R = a.R + (size_t)rhs * (a.l + 1) * n;
    const C<T> *rt = a.rt + (size_t)rhs * n;
    const double2 *br = b + (size_t)rhs * n, *vr = v + (size_t)rhs * n;
    double2 *yr = y ? y + (size_t)rhs * n : nullptr;
    const double2 c = y ? ld(yc, rhs) : d2(0, 0);
    double p[3] = {0.0, 0.0, 0.0};
    for (long e = (long)blockIdx.x * BLOCK + threadIdx.x; e < n; e += (long)gridDim.x * BLOCK) {
        const double2 ve = vr[e];
        const double2 r0 = csub(br[e], ve);
        R[e] = to_c<T>(r0);
        if (yr) yr[e] = cfma(c, ve, yr[e]);
        const C<T> t = rt[e];
        p[0] += (double)t.x * r0.x + (double)t.y * r0.y;
        p[1] += (double)t.x * r0.y - (double)t.y * r0.x;
        p[2] += r0.x * r0.x + r0.y * r0.y;
    }
    block_reduce_store<3>(p, a.part + (size_t)rhs * PMAX * a.ps + blockIdx.x, a.ps);
}

__global__ __launch_bounds__(BLOCK) void k_shift_dots(const double2 *eta, const double2 *X, const double2 *Z, long n,
                                                      int ns, double *out) {
    const int rs = blockIdx.y;            // rhs * ns + s
    const int rhs = rs / ns;
    const double2 *e = eta + (size_t)rhs * n, *x = X + (size_t)rs * n, *z = Z + (size_t)rs * n;
    double p[2] = {0.0, 0.0};
    for (long i = (long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (long)gridDim.x * BLOCK) {
        const double2 xv = x[i], ev = e[i], zv = z[i];
        p[0] += ev.x * xv.x + ev.y * xv.y;
        p[1] += zv.x * xv.x + zv.y * xv.y;
    }
    block_reduce_store<2>(p, out + (size_t)rs * 2 * gridDim.x + blockIdx.x, gridDim.x);
}

__global__ void k_yinit(double2 *y, const double2 *b, const double2 *c, long n) {
    const int rhs = blockIdx.y;
    const double2 cc = c[rhs];
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        y[(size_t)rhs * n + e] = cmul(cc, b[(size_t)rhs * n + e]);
}

__global__ void k_overlap_out(double2 *out, const double2 *b, const double2 *w, long V, int overlap, double s) {
    const int rhs = blockIdx.y;
    const long n = 12 * V;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const size_t i = (size_t)rhs * n + e;
        double2 z = cscale(w[i], s);
        if (overlap) {
            const int spin = (int)(e / V) / 3;
            if (spin >= 2) z = cneg(z);
            z = cadd(b[i], z);
        }
        out[i] = z;
    }
}

__global__ void k_axpy_host(double2 *y, const double2 *x, double2 a, long n) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        y[e] = cfma(a, x[e], y[e]);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
void launch_seed_u(hipStream_t st, const VecArgs<T> &a, int j, int nrhs, int nblk) {
    dim3 g(nblk, nrhs), b(BLOCK);
    switch (j) {
#define C_(J) case J: hipLaunchKernelGGL((k_seed_u<T, J>), g, b, 0, st, a); break;
        C_(0) C_(1) C_(2) C_(3) C_(4) C_(5) C_(6) C_(7)
#undef C_
    }
}

template <typename T, bool SH, bool XH>
static void r_update_j(hipStream_t st, const VecArgs<T> &a, int j, dim3 g, dim3 b) {
    switch (j) {
#define C_(J) case J: hipLaunchKernelGGL((k_r_update<T, J, SH, XH>), g, b, 0, st, a); break;
        C_(0) C_(1) C_(2) C_(3) C_(4) C_(5) C_(6) C_(7)
#undef C_
    }
}

template <typename T>
void launch_r_update(hipStream_t st, const VecArgs<T> &a, int j, bool shifts, bool xh, int nrhs, int nblk) {
    dim3 g(nblk, nrhs), b(BLOCK);
    if (shifts) {
        if (xh) r_update_j<T, true, true>(st, a, j, g, b);
        else r_update_j<T, true, false>(st, a, j, g, b);
    } else {
        if (xh) r_update_j<T, false, true>(st, a, j, g, b);
        else r_update_j<T, false, false>(st, a, j, g, b);
    }
}

template <typename T>
void launch_gram(hipStream_t st, const VecArgs<T> &a, int nrhs, int nblk) {
    dim3 g(nblk, nrhs), b(BLOCK);
    switch (a.l) {
#define C_(L) case L: hipLaunchKernelGGL((k_gram<T, L>), g, b, 0, st, a); break;
        C_(1) C_(2) C_(3) C_(4) C_(5) C_(6) C_(7) C_(8)
#undef C_
    }
}

template <typename T, bool SH, bool XH>
static void mr_update_l(hipStream_t st, const VecArgs<T> &a, dim3 g, dim3 b) {
    switch (a.l) {
#define C_(L) case L: hipLaunchKernelGGL((k_mr_update<T, L, SH, XH>), g, b, 0, st, a); break;
        C_(1) C_(2) C_(3) C_(4) C_(5) C_(6) C_(7) C_(8)
#undef C_
    }
}

template <typename T>
void launch_mr_update(hipStream_t st, const VecArgs<T> &a, bool shifts, bool xh, int nrhs, int nblk) {
    dim3 g(nblk, nrhs), b(BLOCK);
    if (shifts) {
        if (xh) mr_update_l<T, true, true>(st, a, g, b);
        else mr_update_l<T, true, false>(st, a, g, b);
    } else {
        if (xh) mr_update_l<T, false, true>(st, a, g, b);
        else mr_update_l<T, false, false>(st, a, g, b);
    }
}

template <typename T>
void launch_rel_update(hipStream_t st, const VecArgs<T> &a, const double2 *b, const double2 *v, double2 *y,
                       CoefRef yc, int nrhs, int nblk) {
    hipLaunchKernelGGL((k_rel_update<T>), dim3(nblk, nrhs), dim3(BLOCK), 0, st, a, b, v, y, yc);
}

template <typename T>
void launch_convert_in(hipStream_t st, C<T> *dst, const double2 *src, long n, long ds, long ss, int nrhs) {
    hipLaunchKernelGGL((k_convert_in<T>), dim3(nblocks_for(n), nrhs), dim3(BLOCK), 0, st, dst, src, n, ds, ss);
}
template <typename T>
void launch_convert_out(hipStream_t st, double2 *dst, const C<T> *src, long n, long ds, long ss, int nrhs) {
    hipLaunchKernelGGL((k_convert_out<T>), dim3(nblocks_for(n), nrhs), dim3(BLOCK), 0, st, dst, src, n, ds, ss);
}
template <typename T>
void launch_zero(hipStream_t st, C<T> *dst, long n, long stride, int nrhs) {
    hipLaunchKernelGGL((k_zero<T>), dim3(nblocks_for(n), nrhs), dim3(BLOCK), 0, st, dst, n, stride);
}
template <typename T>
void launch_dot_partials(hipStream_t st, const C<T> *x, const C<T> *y, long n, double *part, long ps,
                         int nrhs, int nblk, Gate gate) {
    hipLaunchKernelGGL((k_dot<T>), dim3(nblk, nrhs), dim3(BLOCK), 0, st, x, y, n, part, ps, gate);
}
template <typename T>
void launch_diffnorm_partials(hipStream_t st, const C<T> *x, const C<T> *y, long n, long sx, long sy,
                              double *part, long ps, int nrhs, int nblk) {
    hipLaunchKernelGGL((k_diffnorm<T>), dim3(nblk, nrhs), dim3(BLOCK), 0, st, x, y, n, sx, sy, part, ps);
}
void launch_ysum(hipStream_t st, double2 *y, const double2 *X, const double *w, long n, int ns, int nrhs, int nblk) {
    hipLaunchKernelGGL(k_ysum, dim3(nblk, nrhs), dim3(BLOCK), 0, st, y, X, w, n, ns);
}
void launch_yinit(hipStream_t st, double2 *y, const double2 *b, const double2 *c, long n, int nrhs, int nblk) {
    hipLaunchKernelGGL(k_yinit, dim3(nblk, nrhs), dim3(BLOCK), 0, st, y, b, c, n);
}
void launch_overlap_out(hipStream_t st, double2 *out, const double2 *b, const double2 *w, long V, int nrhs,
                        int overlap, double s, int nblk) {
    hipLaunchKernelGGL(k_overlap_out, dim3(nblk, nrhs), dim3(BLOCK), 0, st, out, b, w, V, overlap, s);
}
void launch_shift_dots(hipStream_t st, const double2 *eta, const double2 *X, const double2 *Z, long n, int ns,
                       int nrhs, int nblk, double *out) {
    hipLaunchKernelGGL(k_shift_dots, dim3(nblk, nrhs * ns), dim3(BLOCK), 0, st, eta, X, Z, n, ns, out);
}

void launch_axpy_host(hipStream_t st, double2 *y, const double2 *x, double2 a, long n, int nblk) {
    hipLaunchKernelGGL(k_axpy_host, dim3(nblk), dim3(BLOCK), 0, st, y, x, a, n);
}

#define INST(T)                                                                                  \
    template void launch_seed_u<T>(hipStream_t, const VecArgs<T> &, int, int, int);              \
    template void launch_r_update<T>(hipStream_t, const VecArgs<T> &, int, bool, bool, int, int); \
    template void launch_gram<T>(hipStream_t, const VecArgs<T> &, int, int);                     \
    template void launch_mr_update<T>(hipStream_t, const VecArgs<T> &, bool, bool, int, int);    \
    template void launch_rel_update<T>(hipStream_t, const VecArgs<T> &, const double2 *, const double2 *, double2 *, CoefRef, int, int); \
    template void launch_convert_in<T>(hipStream_t, C<T> *, const double2 *, long, long, long, int); \
    template void launch_convert_out<T>(hipStream_t, double2 *, const C<T> *, long, long, long, int); \
    template void launch_zero<T>(hipStream_t, C<T> *, long, long, int);                          \
    template void launch_dot_partials<T>(hipStream_t, const C<T> *, const C<T> *, long, double *, long, int, int, Gate); \
    template void launch_diffnorm_partials<T>(hipStream_t, const C<T> *, const C<T> *, long, long, long, double *, long, int, int);
INST(double)
INST(float)
#undef INST

}  // namespace msb
