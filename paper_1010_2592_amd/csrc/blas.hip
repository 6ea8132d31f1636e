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
#include <vector>

#include "blas_dev.h"

namespace msb {

namespace {

using namespace dev;

template <typename T, int J, int MODE>
__global__ __launch_bounds__(BLOCK) void k_seed_u(VecArgs<T> a) {
    seed_u_body<T, J, MODE>(a, blockIdx.x, gridDim.x, blockIdx.y);
}

template <typename T, int J, bool SHIFTS, bool XH, bool FU>
__global__ __launch_bounds__(BLOCK) void k_r_update(VecArgs<T> a) {
    r_update_body<T, J, SHIFTS, XH, FU>(a, blockIdx.x, gridDim.x, blockIdx.y);
}

template <typename T, int L>
__global__ __launch_bounds__(BLOCK) void k_gram(VecArgs<T> a) { gram_body<T, L>(a, blockIdx.x, gridDim.x, blockIdx.y); }

template <typename T, int L, bool SHIFTS, bool XH>
__global__ __launch_bounds__(BLOCK) void k_mr_update(VecArgs<T> a) {
    mr_update_body<T, L, SHIFTS, XH>(a, blockIdx.x, gridDim.x, blockIdx.y);
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_rel_update(VecArgs<T> a, const double2 *b, const double2 *v, double2 *y,
                                                      CoefRef yc) {
    rel_update_body<T>(a, b, v, y, yc, blockIdx.x, gridDim.x, blockIdx.y);
}

// ---------------------------------------------------------------------------
// Deferred single pass.
// snapshot: B_0 <- r_0, B_1 <- u_0 at the start of an outer iteration.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_snapshot(VecArgs<T> a) {
    const int rhs = blockIdx.y;
    if (!gate_open(a.gate, rhs)) return;
    const long n = a.n;
    const C<T> *R = a.R + (size_t)rhs * (a.l + 1) * n;
    const C<T> *U = a.U + (size_t)rhs * (a.l + 1) * n;
    C<T> *B = a.Bm + (size_t)rhs * (2 * a.l + 2) * n;
    for (long e = (long)blockIdx.x * BLOCK + threadIdx.x; e < n; e += (long)gridDim.x * BLOCK) {
        B[e] = R[e];
        B[n + e] = U[e];
    }
}

// defer_update: per element, the 2L + 2 basis values are loaded once and every
// active shift's u^s_0 (iteration precision) and x^s (FP64) are rewritten:
// the shift vectors cross HBM twice per outer iteration instead of
// (l + 1)(l + 4) times.
template <typename T, int L>
__global__ __launch_bounds__(BLOCK) void k_defer_update(VecArgs<T> a) {
    const int rhs = blockIdx.y;
    if (!gate_open(a.gate, rhs)) return;
    constexpr int NB = 2 * L + 2;
    const long n = a.n;
    const int nact = a.seed[rhs].nact;
    const C<T> *B = a.Bm + (size_t)rhs * NB * n;
    const DeferCoef *dc = a.dc + (size_t)rhs * NSMAX;
    // one shift's update of element e from its loaded u^s_0 and x^s
    auto upd = [&](const DeferCoef &d, const C<T> (&b)[NB], long e, C<T> u0, double2 x0) {
        const double2 u0d = d2((double)u0.x, (double)u0.y);
        C<T> un = cmul(cvt<T>(d.cu[NB]), u0);
        double2 xn = cfma(d.cx[NB], u0d, x0);
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            un = cfma(cvt<T>(d.cu[k]), b[k], un);
            xn = cfma(d.cx[k], d2((double)b[k].x, (double)b[k].y), xn);
        }
        a.W0[((size_t)rhs * a.nshift + d.s) * n + e] = un;
        a.X[((size_t)rhs * a.nshift + d.s) * n + e] = xn;
    };
    // basis vectors this outer iteration wrote (r_0, u_0, then the Mv outputs
    // of the steps it made): the slots after them hold whatever an earlier
    // call left, which zero coefficients must not meet (0 * NaN)
    int nbw = 2;
    for (int j = 0; j < L; ++j) {
        const int f = a.seed[rhs].step_flag[j];
        if (f >= 1) nbw = 3 + 2 * j;
        if (f == 2) nbw = 4 + 2 * j;
        if (f < 2) break;
    }
    for (long e = (long)blockIdx.x * BLOCK + threadIdx.x; e < n; e += (long)gridDim.x * BLOCK) {
        C<T> b[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) b[k] = k < nbw ? B[k * n + e] : mk<T>(0, 0);
        // two shifts at a time: their four loads issue together (every
        // shift's vectors exist; a shift that stopped is loaded, not written)
        int q = 0;
        for (; q + 1 < nact; q += 2) {
            const DeferCoef &d0 = dc[q], &d1 = dc[q + 1];
            const size_t o0 = ((size_t)rhs * a.nshift + d0.s) * n + e, o1 = ((size_t)rhs * a.nshift + d1.s) * n + e;
            const C<T> u0 = a.W0[o0], u1 = a.W0[o1];
            const double2 x0 = a.X[o0], x1 = a.X[o1];
            if (d0.live) upd(d0, b, e, u0, x0);
            if (d1.live) upd(d1, b, e, u1, x1);
        }
        if (q < nact) {
            const DeferCoef &d = dc[q];
            if (d.live) {
                const size_t o = ((size_t)rhs * a.nshift + d.s) * n + e;
                upd(d, b, e, a.W0[o], a.X[o]);
            }
        }
    }
}

// pseudo-double pass: the stored Mv outputs of one storage chunk, weighted
// by the transposed sweep's coefficients, added to y (FP64)
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_pstore_sum(double2 *y, const C<T> *V, long v_rs, const double2 *rel,
                                                      long rel_ms, const ReplayStep *rs, const ReplayOuter *ro,
                                                      int Mcap, int l, int m0, int mc, long n) {
    const int rhs = blockIdx.y;
    const C<T> *Vr = V + (size_t)rhs * v_rs;
    const double2 *relr = rel ? rel + (size_t)rhs * n : nullptr;
    const ReplayStep *rsr = rs + (size_t)rhs * Mcap * l;
    const ReplayOuter *ror = ro + (size_t)rhs * Mcap;
    double2 *yr = y + (size_t)rhs * n;
    for (long e = (long)blockIdx.x * BLOCK + threadIdx.x; e < n; e += (long)gridDim.x * BLOCK) {
        double2 acc = yr[e];
        for (int mm = 0; mm < mc; ++mm) {
            const int m = m0 + mm;
            for (int j = 0; j < l; ++j) {
                const ReplayStep &q = rsr[(size_t)m * l + j];
                if (q.flag >= 1) {
                    const C<T> v = Vr[((size_t)mm * 2 * l + 2 * j) * n + e];
                    acc = cfma(q.cu, d2((double)v.x, (double)v.y), acc);
                }
                if (q.flag >= 2) {
                    const C<T> v = Vr[((size_t)mm * 2 * l + 2 * j + 1) * n + e];
                    acc = cfma(q.cr, d2((double)v.x, (double)v.y), acc);
                }
            }
            if (relr && ror[m].rel) acc = cfma(ror[m].crel, relr[(size_t)mm * rel_ms + e], acc);
        }
        yr[e] = acc;
    }
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

__global__ __launch_bounds__(BLOCK) void k_residual(double2 *R, const double2 *b, long b_rs, const double2 *t, long n,
                                                    double *part, long ps) {
    const int rhs = blockIdx.y;
    const double2 *br = b + (size_t)rhs * b_rs, *tr = t + (size_t)rhs * n;
    double2 *Rr = R + (size_t)rhs * n;
    double p[1] = {0.0};
    for (long e = (long)blockIdx.x * BLOCK + threadIdx.x; e < n; e += (long)gridDim.x * BLOCK) {
        const double2 r = csub(br[e], tr[e]);
        Rr[e] = r;
        p[0] += r.x * r.x + r.y * r.y;
    }
    block_reduce_store<1>(p, part + (size_t)rhs * PMAX * ps + blockIdx.x, ps);
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

// basis form of the seed (FP64)
__global__ __launch_bounds__(BLOCK) void k_basis_axpy(BasisArgs<double> a) {
    basis_axpy_body(a, blockIdx.x, gridDim.x, blockIdx.y);
}
__global__ __launch_bounds__(BLOCK) void k_basis_r0norm(BasisArgs<double> a) {
    basis_r0norm_body(a, blockIdx.x, gridDim.x, blockIdx.y);
}
template <int L>
__global__ __launch_bounds__(BLOCK) void k_basis_gram(BasisArgs<double> a) {
    basis_gram_body<L>(a, blockIdx.x, gridDim.x, blockIdx.y);
}
template <int L>
__global__ __launch_bounds__(BLOCK) void k_basis_mr_update(BasisArgs<double> a) {
    basis_mr_update_body<L>(a, blockIdx.x, gridDim.x, blockIdx.y);
}
template <int L>
__global__ __launch_bounds__(64) void k_basis_spec(BasisArgs<double> a) {
    basis_spec_body<L>(a, blockIdx.x);
}
template <int L>
__global__ __launch_bounds__(BLOCK) void k_basis_combine(BasisArgs<double> a) {
    basis_combine_body<L>(a, blockIdx.x, gridDim.x, blockIdx.y);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T, int MODE>
static void seed_u_j(hipStream_t st, const VecArgs<T> &a, int j, dim3 g, dim3 b) {
    switch (j) {
#define C_(J) case J: hipLaunchKernelGGL((k_seed_u<T, J, MODE>), g, b, 0, st, a); break;
        C_(0) C_(1) C_(2) C_(3) C_(4) C_(5) C_(6) C_(7)
#undef C_
    }
}

template <typename T>
void launch_seed_u(hipStream_t st, const VecArgs<T> &a, int j, int nrhs, int nblk, int mode) {
    dim3 g(nblk, nrhs), b(BLOCK);
    if (mode == 1) seed_u_j<T, 1>(st, a, j, g, b);
    else if (mode == 2) {
        if (j >= 1) seed_u_j<T, 2>(st, a, j, g, b);
    } else seed_u_j<T, 0>(st, a, j, g, b);
}

template <typename T, bool SH, bool XH, bool FU>
static void r_update_j(hipStream_t st, const VecArgs<T> &a, int j, dim3 g, dim3 b) {
    switch (j) {
#define C_(J) case J: hipLaunchKernelGGL((k_r_update<T, J, SH, XH, FU>), g, b, 0, st, a); break;
        C_(0) C_(1) C_(2) C_(3) C_(4) C_(5) C_(6) C_(7)
#undef C_
    }
}

template <typename T, bool FU>
static void r_update_f(hipStream_t st, const VecArgs<T> &a, int j, bool shifts, bool xh, dim3 g, dim3 b) {
    if (shifts) {
        if (xh) r_update_j<T, true, true, FU>(st, a, j, g, b);
        else r_update_j<T, true, false, FU>(st, a, j, g, b);
    } else {
        if (xh) r_update_j<T, false, true, FU>(st, a, j, g, b);
        else r_update_j<T, false, false, FU>(st, a, j, g, b);
    }
}

template <typename T>
void launch_r_update(hipStream_t st, const VecArgs<T> &a, int j, bool shifts, bool xh, int nrhs, int nblk,
                     bool fused) {
    dim3 g(nblk, nrhs), b(BLOCK);
    if (fused && j >= 1) r_update_f<T, true>(st, a, j, shifts, xh, g, b);
    else r_update_f<T, false>(st, a, j, shifts, xh, g, b);
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
void launch_snapshot(hipStream_t st, const VecArgs<T> &a, int nrhs, int nblk) {
    hipLaunchKernelGGL((k_snapshot<T>), dim3(nblk, nrhs), dim3(BLOCK), 0, st, a);
}

template <typename T>
void launch_defer_update(hipStream_t st, const VecArgs<T> &a, int nrhs, int nblk) {
    dim3 g(nblk, nrhs), b(BLOCK);
    switch (a.l) {
#define C_(L) case L: hipLaunchKernelGGL((k_defer_update<T, L>), g, b, 0, st, a); break;
        C_(1) C_(2) C_(3) C_(4) C_(5) C_(6) C_(7) C_(8)
#undef C_
    }
}

template <typename T>
void launch_pstore_sum(hipStream_t st, double2 *y, const C<T> *V, long v_rs, const double2 *rel, long rel_ms,
                       const ReplayStep *rs, const ReplayOuter *ro, int Mcap, int l, int m0, int mc, long n,
                       int nrhs, int nblk) {
    hipLaunchKernelGGL((k_pstore_sum<T>), dim3(nblk, nrhs), dim3(BLOCK), 0, st, y, V, v_rs, rel, rel_ms, rs, ro,
                       Mcap, l, m0, mc, n);
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
void launch_residual(hipStream_t st, double2 *R, const double2 *b, long b_rs, const double2 *t, long n,
                     double *part, long ps, int nrhs, int nblk) {
    hipLaunchKernelGGL(k_residual, dim3(nblk, nrhs), dim3(BLOCK), 0, st, R, b, b_rs, t, n, part, ps);
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

// ---------------------------------------------------------------------------
// Sparse shadow residual.  When every right-hand side's r~ has at most SPMAX
// nonzero entries (a point source with r~ = b has one), the dots <r~, v> of
// the Mv epilogue and of the MR update are taken from an index list instead
// of a full read of r~.  One wavefront per (block range, rhs): count, then
// write each nonzero at its rank in index order, so the list is the same on
// every run.
__global__ __launch_bounds__(64) void k_nnz_count(const double2 *__restrict__ v, long n, long rs, int *__restrict__ cnt,
                                                  int nb) {
    const int b = blockIdx.x, rhs = blockIdx.y, lane = threadIdx.x;
    const long len = (n + nb - 1) / nb, e0 = (long)b * len;
    const long e1 = e0 + len < n ? e0 + len : n;
    const double2 *x = v + (size_t)rhs * rs;
    int c = 0;
    for (long e = e0; e < e1; e += 64) {
        const long k = e + lane;
        bool nz = false;
        if (k < e1) {
            const double2 z = x[k];
            nz = z.x != 0.0 || z.y != 0.0;
        }
        c += __popcll(__ballot(nz));
    }
    if (lane == 0) cnt[(size_t)rhs * nb + b] = c;
}

__global__ __launch_bounds__(64) void k_nnz_collect(const double2 *__restrict__ v, long n, long rs,
                                                    const int *__restrict__ off, int nb, long *__restrict__ idx,
                                                    double2 *__restrict__ val, int spmax, int fp32) {
    const int b = blockIdx.x, rhs = blockIdx.y, lane = threadIdx.x;
    const long len = (n + nb - 1) / nb, e0 = (long)b * len;
    const long e1 = e0 + len < n ? e0 + len : n;
    const double2 *x = v + (size_t)rhs * rs;
    int c = off[(size_t)rhs * nb + b];
    const unsigned long long below = (1ull << lane) - 1ull;
    for (long e = e0; e < e1; e += 64) {
        const long k = e + lane;
        bool nz = false;
        double2 z{0.0, 0.0};
        if (k < e1) {
            z = x[k];
            nz = z.x != 0.0 || z.y != 0.0;
        }
        const unsigned long long m = __ballot(nz);
        if (nz) {
            const int pos = c + __popcll(m & below);
            if (pos < spmax) {
                idx[(size_t)rhs * spmax + pos] = k;
                // mixed precision: the value of the FP32 copy of r~ the dense path reads
                val[(size_t)rhs * spmax + pos] = fp32 ? double2{(double)(float)z.x, (double)(float)z.y} : z;
            }
        }
        c += __popcll(m);
    }
}

// <r~, x> of each open rhs from the list, written over column 0 of partial
// slots 0 (re) and 1 (im); the kernel that produced x left those slots zero.
// X: the element type of x (double2, or float2 for mixed precision, each
// product formed in FP64 as the dense epilogues do).  With DIFF, x = b - v
// for FP64 b and v (the reliable update's residual before its rounding).
template <typename X, bool DIFF>
__global__ __launch_bounds__(64) void k_sparse_dot(SparseDotArgs a, int nrhs) {
    const int rhs = blockIdx.x * 64 + threadIdx.x;
    if (rhs >= nrhs || !gate_open(a.gate, rhs)) return;
    double p0 = 0.0, p1 = 0.0;
    const int nk = a.cnt[rhs];
    for (int k = 0; k < nk; ++k) {
        const double2 t = a.val[(size_t)rhs * a.spmax + k];
        const long e = a.idx[(size_t)rhs * a.spmax + k];
        double2 o;
        if (DIFF) {
            o = csub(a.b[(size_t)rhs * a.x_rs + e], a.v[(size_t)rhs * a.x_rs + e]);
        } else {
            const X z = reinterpret_cast<const X *>(a.x)[(size_t)rhs * a.x_rs + e];
            o = double2{(double)z.x, (double)z.y};
        }
        p0 += t.x * o.x + t.y * o.y;
        p1 += t.x * o.y - t.y * o.x;
    }
    double *row = a.part + (size_t)rhs * PMAX * a.ps;
    row[0] = p0;
    row[a.ps] = p1;
}

int sparse_list(hipStream_t st, const double2 *v, long n, long rs, int nrhs, int spmax, long *idx, double2 *val,
                int *cnt, int *work, int nb, bool fp32) {
    hipLaunchKernelGGL(k_nnz_count, dim3(nb, nrhs), dim3(64), 0, st, v, n, rs, work, nb);
    if (hipGetLastError() != hipSuccess) return -1;
    std::vector<int> h((size_t)nrhs * nb), off((size_t)nrhs * nb), tot(nrhs, 0);
    if (hipStreamSynchronize(st) != hipSuccess) return -1;
    if (hipMemcpy(h.data(), work, h.size() * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return -1;
    int worst = 0;
    for (int r = 0; r < nrhs; ++r) {
        for (int b = 0; b < nb; ++b) {
            off[(size_t)r * nb + b] = tot[r];
            tot[r] += h[(size_t)r * nb + b];
        }
        worst = tot[r] > worst ? tot[r] : worst;
    }
    if (worst > spmax) return worst;
    if (hipMemcpy(work, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) return -1;
    if (hipMemcpy(cnt, tot.data(), nrhs * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) return -1;
    hipLaunchKernelGGL(k_nnz_collect, dim3(nb, nrhs), dim3(64), 0, st, v, n, rs, work, nb, idx, val, spmax,
                       fp32 ? 1 : 0);
    if (hipGetLastError() != hipSuccess) return -1;
    return worst;
}

void launch_sparse_dot(hipStream_t st, const SparseDotArgs &a, int nrhs) {
    const dim3 g((nrhs + 63) / 64), b(64);
    if (a.b) hipLaunchKernelGGL((k_sparse_dot<double2, true>), g, b, 0, st, a, nrhs);
    else if (a.fp32) hipLaunchKernelGGL((k_sparse_dot<float2, false>), g, b, 0, st, a, nrhs);
    else hipLaunchKernelGGL((k_sparse_dot<double2, false>), g, b, 0, st, a, nrhs);
}

#define INST(T)                                                                                  \
    template void launch_seed_u<T>(hipStream_t, const VecArgs<T> &, int, int, int, int);                \
    template void launch_r_update<T>(hipStream_t, const VecArgs<T> &, int, bool, bool, int, int, bool); \
    template void launch_gram<T>(hipStream_t, const VecArgs<T> &, int, int);                     \
    template void launch_snapshot<T>(hipStream_t, const VecArgs<T> &, int, int);                 \
    template void launch_pstore_sum<T>(hipStream_t, double2 *, const C<T> *, long, const double2 *, long, \
                                       const ReplayStep *, const ReplayOuter *, int, int, int, int, long, int, int); \
    template void launch_defer_update<T>(hipStream_t, const VecArgs<T> &, int, int);             \
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

void launch_basis_axpy(hipStream_t st, const BasisArgs<double> &a, int nrhs, int nblk) {
    hipLaunchKernelGGL(k_basis_axpy, dim3(nblk, nrhs), dim3(BLOCK), 0, st, a);
}
void launch_basis_r0norm(hipStream_t st, const BasisArgs<double> &a, int nrhs, int nblk) {
    hipLaunchKernelGGL(k_basis_r0norm, dim3(nblk, nrhs), dim3(BLOCK), 0, st, a);
}
void launch_basis_gram(hipStream_t st, const BasisArgs<double> &a, int nrhs, int nblk) {
    dim3 g(nblk, nrhs), b(BLOCK);
    switch (a.l) {
#define C_(L) case L: hipLaunchKernelGGL((k_basis_gram<L>), g, b, 0, st, a); break;
        C_(1) C_(2) C_(3) C_(4) C_(5) C_(6) C_(7) C_(8)
#undef C_
    }
}
void launch_basis_mr_update(hipStream_t st, const BasisArgs<double> &a, int nrhs, int nblk) {
    dim3 g(nblk, nrhs), b(BLOCK);
    switch (a.l) {
#define C_(L) case L: hipLaunchKernelGGL((k_basis_mr_update<L>), g, b, 0, st, a); break;
        C_(1) C_(2) C_(3) C_(4) C_(5) C_(6) C_(7) C_(8)
#undef C_
    }
}
void launch_basis_spec(hipStream_t st, const BasisArgs<double> &a, int nrhs) {
    switch (a.l) {
#define C_(L) case L: hipLaunchKernelGGL((k_basis_spec<L>), dim3(nrhs), dim3(64), 0, st, a); break;
        C_(1) C_(2) C_(3) C_(4) C_(5) C_(6) C_(7) C_(8)
#undef C_
    }
}
void launch_basis_combine(hipStream_t st, const BasisArgs<double> &a, int nrhs, int nblk) {
    dim3 g(nblk, nrhs), b(BLOCK);
    switch (a.l) {
#define C_(L) case L: hipLaunchKernelGGL((k_basis_combine<L>), g, b, 0, st, a); break;
        C_(1) C_(2) C_(3) C_(4) C_(5) C_(6) C_(7) C_(8)
#undef C_
    }
}

}  // namespace msb
