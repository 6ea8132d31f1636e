// Low modes of H = gamma5 D_w at mu = 0 and the sign function with those
// modes deflated.
//
// The paper's overlap benchmarks deflate the eigenvalues of H of smallest
// modulus (the numbers deflated are given with Figs. 1, 3 and 4): with
// eigenpairs (lambda_k, v_k), k < K,
//   sign(H) b = sum_k sign(lambda_k) v_k <v_k, b> + sqrt(a) H f(a H^2) P b,
//   P b = b - sum_k v_k <v_k, b>,
// so the partial-fraction expansion f only sees the spectrum of H^2 above
// lambda_K^2.  At mu = 0 H is Hermitian and the v_k are orthonormal (the
// mu != 0 case needs left and right eigenvectors and is not treated).
//
// Eigensolver: Chebyshev-filtered subspace iteration on H^2 with a block of
// m >= K + 1 vectors.
//  * Filter: T_d((H^2 - e)/h), the degree-d Chebyshev polynomial of [c, hi]
//    (c the block's largest Ritz value of H^2, hi a rigorous bound of the
//    spectrum), which damps the modes above c and keeps those below.  The
//    degree is capped so that no direction grows by more than 1e8 relative to
//    the damped interval, which keeps the block numerically full rank.
//  * Orthonormalisation: Cholesky-QR twice (a shifted Cholesky-QR first when
//    the plain Cholesky factorisation fails).
//  * Rayleigh-Ritz with H^2 first: H^2 is positive semi-definite and the
//    wanted modes are its smallest, so its Ritz values converge from above
//    and cannot be spurious.  (Rayleigh-Ritz with the indefinite H on a
//    subspace that is not yet invariant produces small Ritz values from
//    mixtures of +lambda and -lambda modes.)  Then Rayleigh-Ritz with H
//    inside the leading K Ritz vectors of H^2 gives the signed eigenpairs.
// The tall-skinny products (X^H Y over 12 V rows, X Q) are the library's own
// HBM-bound kernels; the m x m problems (Cholesky, triangular inverse,
// Hermitian eigenproblems) are solved on the host in FP64.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "ctx.h"
#include "smallla.h"

namespace msb {

namespace {

using sla::cplx;

#define E_HIPCHK(x)                                        \
    do {                                                   \
        int rc_ = hip_check((x), #x);                      \
        if (rc_) return rc_;                               \
    } while (0)
#define E_CHK(x)                                           \
    do {                                                   \
        int rc_ = (x);                                     \
        if (rc_) return rc_;                               \
    } while (0)

constexpr int TM = 32;             // vectors per tile side of the block kernels
constexpr int TE = 64;             // elements (complex) per tile
constexpr int GRAM_BLOCKS = 1024;  // blocks of the Gram kernel (partials per entry)
constexpr int QG = 8;              // row group of the combine kernel

// Partial Gram matrix of two blocks of at most TM vectors:
//   part[(i + j * TM) * nblk + blockIdx.x] = sum over this block's elements of conj(X_i[e]) Y_j[e]
// for i < m1, j < m2.  A tile holds TE elements of every vector in LDS; each
// thread accumulates a 4 x 4 patch of the (padded) TM x TM result over a
// quarter of the tile (rows ib + 8a, columns jb + 8b); the four quarters are
// added at the end in a fixed order.
__global__ __launch_bounds__(BLOCK) void k_gram(const double2 *__restrict__ X, int m1, const double2 *__restrict__ Y,
                                                int m2, long n, double2 *__restrict__ part, int nblk) {
    __shared__ double2 sm[2 * TM * (TE + 1)];
    double2 *xs = sm, *ys = sm + TM * (TE + 1);
    const int t = threadIdx.x, ib = t & 7, jb = (t >> 3) & 7, q = t >> 6;
    const int e = t & 63, v0 = t >> 6;
    for (int k = t; k < 2 * TM * (TE + 1); k += BLOCK) sm[k] = double2{0.0, 0.0};
    __syncthreads();
    double2 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = double2{0.0, 0.0};
    const long ntile = (n + TE - 1) / TE;
    for (long tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const long idx = tile * TE + e;
        const bool in = idx < n;
        for (int v = v0; v < m1; v += 4) xs[v * (TE + 1) + e] = in ? X[(size_t)v * n + idx] : double2{0.0, 0.0};
        for (int v = v0; v < m2; v += 4) ys[v * (TE + 1) + e] = in ? Y[(size_t)v * n + idx] : double2{0.0, 0.0};
        __syncthreads();
#pragma unroll 4
        for (int k = q * (TE / 4); k < (q + 1) * (TE / 4); ++k) {
            double2 xv[4], yv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) xv[a] = xs[(ib + 8 * a) * (TE + 1) + k];
#pragma unroll
            for (int b = 0; b < 4; ++b) yv[b] = ys[(jb + 8 * b) * (TE + 1) + k];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    acc[a][b].x += xv[a].x * yv[b].x + xv[a].y * yv[b].y;
                    acc[a][b].y += xv[a].x * yv[b].y - xv[a].y * yv[b].x;
                }
        }
        __syncthreads();
    }
    // add the four quarters (reusing the tile storage: 4 * TM * TM <= 2 * TM * (TE + 1))
    double2 *red = sm;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) red[q * TM * TM + (ib + 8 * a) + (jb + 8 * b) * TM] = acc[a][b];
    __syncthreads();
    for (int k = t; k < TM * TM; k += BLOCK) {
        const int i = k % TM, j = k / TM;
        if (i >= m1 || j >= m2) continue;
        double2 s = red[k];
        for (int w = 1; w < 4; ++w) s = cadd(s, red[w * TM * TM + k]);
        part[(size_t)k * nblk + blockIdx.x] = s;
    }
}

// C[i + j * ldc] = sum_b part[(i + j * TM) * nblk + b]; one block per entry
__global__ __launch_bounds__(BLOCK) void k_gram_sum(const double2 *__restrict__ part, int nblk, int m1,
                                                    double2 *__restrict__ C, int ldc) {
    const int i = blockIdx.x % m1, j = blockIdx.x / m1;
    const double2 *p = part + (size_t)(i + j * TM) * nblk;
    double s[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += BLOCK) {
        s[0] += p[b].x;
        s[1] += p[b].y;
    }
    block_reduce_store<2>(s, reinterpret_cast<double *>(C + i + (size_t)j * ldc), 1);
}

// Z_j[e] = sum_{i < m1} X_i[e] Q[i + j * ldq] + beta Z_j[e] for j < m2 (m1, m2
// <= TM, Q already scaled by alpha).  Each thread keeps the m1 values of its
// element in registers (in row groups of QG), Q sits in LDS.  Z must not
// alias X.
__global__ __launch_bounds__(BLOCK) void k_combine(const double2 *__restrict__ X, int m1,
                                                   const double2 *__restrict__ Q, int ldq, int m2, long n,
                                                   double2 *__restrict__ Z, double alpha, double beta) {
    __shared__ double2 qs[TM * TM];
    for (int k = threadIdx.x; k < TM * TM; k += BLOCK) {
        const int i = k % TM, j = k / TM;
        qs[k] = (i < m1 && j < m2) ? cscale(Q[i + (size_t)j * ldq], alpha) : double2{0.0, 0.0};
    }
    __syncthreads();
    for (long e = (long)blockIdx.x * BLOCK + threadIdx.x; e < n; e += (long)gridDim.x * BLOCK) {
        double2 x[TM];
#pragma unroll
        for (int g = 0; g < TM / QG; ++g)
            if (g * QG < m1) {
#pragma unroll
                for (int r = 0; r < QG; ++r) {
                    const int i = g * QG + r;
                    x[i] = i < m1 ? X[(size_t)i * n + e] : double2{0.0, 0.0};
                }
            }
        for (int j = 0; j < m2; ++j) {
            double2 acc = beta != 0.0 ? cscale(Z[(size_t)j * n + e], beta) : double2{0.0, 0.0};
#pragma unroll
            for (int g = 0; g < TM / QG; ++g)
                if (g * QG < m1) {
#pragma unroll
                    for (int r = 0; r < QG; ++r) {
                        const double2 qv = qs[g * QG + r + j * TM];
                        const double2 xv = x[g * QG + r];
                        acc.x += xv.x * qv.x - xv.y * qv.y;
                        acc.y += xv.x * qv.y + xv.y * qv.x;
                    }
                }
            Z[(size_t)j * n + e] = acc;
        }
    }
}

// partial sums of ||W_i - theta_i Y_i||^2, one row of nblk per vector i
__global__ __launch_bounds__(BLOCK) void k_resid(const double2 *W, const double2 *Y, const double *theta, long n,
                                                 double *part, int nblk) {
    const int i = blockIdx.y;
    const double t = theta[i];
    const double2 *w = W + (size_t)i * n, *y = Y + (size_t)i * n;
    double p[1] = {0.0};
    for (long e = (long)blockIdx.x * BLOCK + threadIdx.x; e < n; e += (long)gridDim.x * BLOCK) {
        const double2 d = csub(w[e], cscale(y[e], t));
        p[0] += d.x * d.x + d.y * d.y;
    }
    block_reduce_store<1>(p, part + (size_t)i * nblk + blockIdx.x, 1);
}

// small host <-> device copies: finish the stream's work, then a synchronous
// copy (asynchronous copies with pageable host memory are avoided)
int to_host(hipStream_t st, void *dst, const void *src, size_t bytes) {
    E_HIPCHK(hipStreamSynchronize(st));
    E_HIPCHK(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
    return 0;
}
int to_dev(hipStream_t st, void *dst, const void *src, size_t bytes) {
    E_HIPCHK(hipStreamSynchronize(st));
    E_HIPCHK(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    return 0;
}

// G (host, m1 x m2 column-major) = X^H Y for blocks X [m1][n], Y [m2][n];
// Cd is device scratch of m1 * m2 complex
int gram(Ctx *c, const double2 *X, int m1, const double2 *Y, int m2, long n, double2 *Cd, std::vector<cplx> &G) {
    hipStream_t st = c->stream;
    const long ntile = (n + TE - 1) / TE;
    const int nblk = (int)std::min<long>(ntile, GRAM_BLOCKS);
    E_CHK(ensure(c, c->ws_eG, (size_t)TM * TM * nblk * sizeof(double2)));
    double2 *part = (double2 *)c->ws_eG.p;
    for (int i0 = 0; i0 < m1; i0 += TM)
        for (int j0 = 0; j0 < m2; j0 += TM) {
            const int b1 = std::min(TM, m1 - i0), b2 = std::min(TM, m2 - j0);
            hipLaunchKernelGGL(k_gram, dim3(nblk), dim3(BLOCK), 0, st, X + (size_t)i0 * n, b1, Y + (size_t)j0 * n,
                               b2, n, part, nblk);
            hipLaunchKernelGGL(k_gram_sum, dim3(b1 * b2), dim3(BLOCK), 0, st, part, nblk, b1,
                               Cd + i0 + (size_t)j0 * m1, m1);
        }
    E_HIPCHK(hipGetLastError());
    G.resize((size_t)m1 * m2);
    return to_host(st, G.data(), Cd, G.size() * sizeof(double2));
}

// Z [m2][n] = alpha X Q + beta Z for X [m1][n] and Q (m1 x m2, column-major,
// device); Z must not alias X
int combine(Ctx *c, const double2 *X, int m1, const double2 *Qd, int m2, long n, double2 *Z, double alpha,
            double beta) {
    hipStream_t st = c->stream;
    const int nb = nblocks_for(n);
    for (int j0 = 0; j0 < m2; j0 += TM)
        for (int i0 = 0; i0 < m1; i0 += TM) {
            const int b1 = std::min(TM, m1 - i0), b2 = std::min(TM, m2 - j0);
            hipLaunchKernelGGL(k_combine, dim3(nb), dim3(BLOCK), 0, st, X + (size_t)i0 * n, b1,
                               Qd + i0 + (size_t)j0 * m1, m1, b2, n, Z + (size_t)j0 * n, alpha,
                               i0 == 0 ? beta : 1.0);
        }
    E_HIPCHK(hipGetLastError());
    return 0;
}

DslashArgs<double> h_args(const Ctx *c, const double2 *in, double2 *out) {
    DslashArgs<double> a;
    a.U = c->U64;
    a.g = c->g;
    a.diag = 4.0 + c->mass;
    a.ef = std::exp(c->mu);
    a.eb = std::exp(-c->mu);
    a.bc = (double)c->bc_t;
    a.g5out = 1;
    a.in = in;
    a.out = out;
    return a;
}

}  // namespace

int low_modes(Ctx *c, int nev, int m, const double2 *start, double tol, int degree, int max_iter, double *evals,
              double2 *evecs, double *resid, int *iters_out) {
    hipStream_t st = c->stream;
    const long n = 12L * c->g.V;
    const int nbv = nblocks_for(n);
    // upper bound of the spectrum of H^2 = D^+ D: the filter must damp every
    // mode above its interval, so the bound has to be rigorous -- a power
    // iteration's Rayleigh quotient lies below lambda_max.  Each direction's
    // forward and backward hops are orthogonal projectors times unitary links
    // (norm <= 1, e^{|mu|} on the time links), so ||D|| <= |4 + m| + 3 + e^{|mu|}.
    const double dnorm = std::fabs(4.0 + c->mass) + 3.0 + std::exp(std::fabs(c->mu));
    const double hi = dnorm * dnorm;
    const size_t blk = (size_t)m * n * sizeof(double2);
    E_CHK(ensure(c, c->ws_eY, blk));
    E_CHK(ensure(c, c->ws_eW, blk));
    E_CHK(ensure(c, c->ws_eZ, blk));
    E_CHK(ensure(c, c->ws_eP, blk));
    E_CHK(ensure(c, c->ws_eS, (size_t)m * m * sizeof(double2) + (size_t)m * sizeof(double) + 256));
    E_CHK(ensure(c, c->ws_part, (size_t)m * nbv * sizeof(double)));
    double2 *Y = (double2 *)c->ws_eY.p, *W = (double2 *)c->ws_eW.p, *Z = (double2 *)c->ws_eZ.p,
            *Pv = (double2 *)c->ws_eP.p;
    double2 *Sd = (double2 *)c->ws_eS.p;
    double *Td = (double *)(Sd + (size_t)m * m);
    double *part = (double *)c->ws_part.p;
    E_HIPCHK(hipMemcpyAsync(Y, start, blk, hipMemcpyDeviceToDevice, st));

    std::vector<cplx> G;
    // B <- B R for the block B [m][n] and R (m x m, host): through Z, then swap
    auto rotate = [&](double2 *&B, const std::vector<cplx> &R) -> int {
        E_CHK(to_dev(st, Sd, R.data(), R.size() * sizeof(double2)));
        E_CHK(combine(c, B, m, Sd, m, n, Z, 1.0, 0.0));
        std::swap(B, Z);
        return 0;
    };
    // Y <- Y R^{-1} with R^H R = Y^H Y: twice, or three times with a shifted
    // first factorisation when the plain one fails (shift from Fukaya et al.'s
    // shifted Cholesky-QR: 11 (n m + m (m + 1)) u ||G||)
    auto orth = [&]() -> int {
        int passes = 2;
        for (int pass = 0; pass < passes; ++pass) {
            E_CHK(gram(c, Y, m, Y, m, n, Sd, G));
            std::vector<cplx> R = G;
            if (!sla::cholesky_upper(R, m)) {
                if (passes == 3) return set_error(S_BREAKDOWN, "low_modes: the block lost rank (Cholesky-QR failed)");
                double tr = 0.0;
                for (int j = 0; j < m; ++j) tr += G[j + (size_t)j * m].real();
                const double shift = 11.0 * ((double)n * m + (double)m * (m + 1)) * 1.1102230246251565e-16 * tr;
                R = G;
                for (int j = 0; j < m; ++j) R[j + (size_t)j * m] += shift;
                if (!sla::cholesky_upper(R, m))
                    return set_error(S_BREAKDOWN, "low_modes: the block lost rank (shifted Cholesky-QR failed)");
                passes = 3;
            }
            sla::upper_inverse(R, m);
            E_CHK(rotate(Y, R));
        }
        return 0;
    };
    // Rayleigh-Ritz with H^2 on the block, then with H on its leading nev Ritz
    // vectors; afterwards Y, W = H Y hold the Ritz vectors (the first nev ordered
    // by |theta|), mu2 the Ritz values of H^2 (ascending), res the residuals
    // ||H y_j - theta_j y_j|| of the first nev
    std::vector<double> theta(nev), res(nev), mu2(m);
    auto rayleigh_ritz = [&]() -> int {
        {
            DslashArgs<double> a = h_args(c, Y, W);
            launch_dslash<double>(st, a, m, EPI_PLAIN, false);
        }
        std::vector<cplx> G2, G1, Q2, Q1;
        E_CHK(gram(c, W, m, W, m, n, Sd, G2));
        E_CHK(gram(c, Y, m, W, m, n, Sd, G1));
        if (sla::heev_jacobi(G2, m, mu2, Q2) < 0)
            return set_error(S_BREAKDOWN, "low_modes: Rayleigh-Ritz (H^2) eigensolver did not converge");
        const int k = nev;
        // S = Q2k^H G1 Q2k, Hermitian part
        std::vector<cplx> T((size_t)m * k, cplx(0.0)), S((size_t)k * k, cplx(0.0));
        for (int j = 0; j < k; ++j)
            for (int l = 0; l < m; ++l) {
                const cplx q = Q2[l + (size_t)j * m];
                for (int i = 0; i < m; ++i) T[i + (size_t)j * m] += G1[i + (size_t)l * m] * q;
            }
        for (int j = 0; j < k; ++j)
            for (int i = 0; i < k; ++i) {
                cplx s = 0.0;
                for (int l = 0; l < m; ++l) s += std::conj(Q2[l + (size_t)i * m]) * T[l + (size_t)j * m];
                S[i + (size_t)j * k] = s;
            }
        for (int j = 0; j < k; ++j)
            for (int i = 0; i <= j; ++i) {
                const cplx h = 0.5 * (S[i + (size_t)j * k] + std::conj(S[j + (size_t)i * k]));
                S[i + (size_t)j * k] = h;
                S[j + (size_t)i * k] = std::conj(h);
            }
        std::vector<double> th;
        if (sla::heev_jacobi(S, k, th, Q1) < 0)
            return set_error(S_BREAKDOWN, "low_modes: Rayleigh-Ritz (H) eigensolver did not converge");
        std::vector<int> ord(k);
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return std::fabs(th[x]) < std::fabs(th[y]); });
        // R = [Q2k Q1 (ordered) | Q2 columns k..m-1]
        std::vector<cplx> R((size_t)m * m, cplx(0.0));
        for (int j = 0; j < k; ++j) {
            theta[j] = th[ord[j]];
            for (int l = 0; l < k; ++l) {
                const cplx q = Q1[l + (size_t)ord[j] * k];
                for (int i = 0; i < m; ++i) R[i + (size_t)j * m] += Q2[i + (size_t)l * m] * q;
            }
        }
        for (int j = k; j < m; ++j) std::copy(&Q2[(size_t)j * m], &Q2[(size_t)j * m] + m, &R[(size_t)j * m]);
        E_CHK(rotate(Y, R));
        E_CHK(rotate(W, R));
        // residuals of the first nev
        E_CHK(to_dev(st, Td, theta.data(), nev * sizeof(double)));
        hipLaunchKernelGGL(k_resid, dim3(nbv, nev), dim3(BLOCK), 0, st, W, Y, Td, n, part, nbv);
        E_HIPCHK(hipGetLastError());
        std::vector<double> pr((size_t)nev * nbv);
        E_CHK(to_host(st, pr.data(), part, pr.size() * sizeof(double)));
        for (int j = 0; j < nev; ++j) {
            double s2 = 0.0;
            for (int q = 0; q < nbv; ++q) s2 += pr[(size_t)j * nbv + q];
            res[j] = std::sqrt(s2);
        }
        return 0;
    };

    E_CHK(orth());
    E_CHK(rayleigh_ritz());
    const double scale = std::sqrt(hi);   // |lambda| bound of H
    const double grow_max = std::acosh(1e8);
    int it = 0;
    for (; it < max_iter; ++it) {
        bool done = true;
        for (int j = 0; j < nev; ++j) done = done && res[j] <= tol * scale;
        if (done) break;
        // damp [c, hi] with c the block's largest Ritz value of H^2
        const double c2 = std::min(std::max(mu2[m - 1], 0.0), 0.5 * hi);
        const double e = 0.5 * (hi + c2), hw = 0.5 * (hi - c2);
        // degree cap: T_d(e / hw) (the growth at lambda = 0) at most 1e8
        const int dcap = std::max(1, (int)std::floor(grow_max / std::acosh(e / hw)));
        const int deg = std::min(degree, dcap);
        // Chebyshev recurrence on the block: Yp = Y_{j-1}, Yc = Y_j
        double2 *Yp = Pv, *Yc = Y, *Yn = Z;
        for (int d = 1; d <= deg; ++d) {
            DslashArgs<double> a1 = h_args(c, Yc, W);          // W = H Y_j
            launch_dslash<double>(st, a1, m, EPI_PLAIN, false);
            DslashArgs<double> a2 = h_args(c, W, Yn);          // Y_{j+1} = s H W + s0 Y_j (- Y_{j-1})
            a2.v = Yc;
            a2.scale = (d == 1 ? 1.0 : 2.0) / hw;
            a2.sigma0 = -(d == 1 ? 1.0 : 2.0) * e / hw;
            if (d > 1) a2.w = Yp;                             // the subtraction in the epilogue
            launch_dslash<double>(st, a2, m, d > 1 ? EPI_SV2 : EPI_SV, false);
            E_HIPCHK(hipGetLastError());
            double2 *t = Yp;
            Yp = Yc;
            Yc = Yn;
            Yn = t;
        }
        // the filtered block is Yc; the other two buffers become the scratch
        Y = Yc;
        Pv = Yp;
        Z = Yn;
        E_CHK(orth());
        E_CHK(rayleigh_ritz());
    }
    for (int j = 0; j < nev; ++j) {
        evals[j] = theta[j];
        if (resid) resid[j] = res[j];
    }
    if (iters_out) *iters_out = it;
    E_HIPCHK(hipMemcpyAsync(evecs, Y, (size_t)nev * n * sizeof(double2), hipMemcpyDeviceToDevice, st));
    E_HIPCHK(hipStreamSynchronize(st));
    bool done = true;
    for (int j = 0; j < nev; ++j) done = done && res[j] <= tol * scale;
    return done ? 0 : set_error(S_NOT_CONVERGED, "low_modes: max_iter reached before every mode met tol");
}

int sign_apply_deflated(Ctx *c, const SolveParams &P, int nev, const double *evals, const double2 *evecs,
                        const double2 *b, double2 *out, bool overlap, SolveReport *rep) {
    hipStream_t st = c->stream;
    const int V = c->g.V;
    const long n = 12L * V;
    const int nrhs = P.nrhs;
    const int nbv = nblocks_for(n);
    E_CHK(ensure(c, c->ws_eS, (size_t)nev * nrhs * sizeof(double2) + 256));
    E_CHK(ensure(c, c->ws_eY, (size_t)nrhs * n * sizeof(double2)));   // P b, then sign(H) b
    E_CHK(ensure(c, c->ws_eW, (size_t)nrhs * n * sizeof(double2)));   // H y
    double2 *cd = (double2 *)c->ws_eS.p;
    double2 *pb = (double2 *)c->ws_eY.p, *hy = (double2 *)c->ws_eW.p;
    // c = V^H b (nev x nrhs), P b = b - V c
    std::vector<cplx> cb;
    E_CHK(gram(c, evecs, nev, b, nrhs, n, cd, cb));
    E_HIPCHK(hipMemcpyAsync(pb, b, (size_t)nrhs * n * sizeof(double2), hipMemcpyDeviceToDevice, st));
    E_CHK(combine(c, evecs, nev, cd, nrhs, n, pb, -1.0, 1.0));
    // y = f(A) P b
    E_CHK(ensure(c, c->ws_y, (size_t)nrhs * n * sizeof(double2)));
    double2 *yy = (double2 *)c->ws_y.p;
    E_CHK(solve_mshift(c, P, pb, yy, nullptr, false, rep));
    // sign part: sqrt(a) H y + V (sign(lambda) c)
    {
        DslashArgs<double> a = h_args(c, yy, hy);
        launch_dslash<double>(st, a, nrhs, EPI_PLAIN, false);
    }
    double2 *sg = overlap ? pb : out;
    launch_overlap_out(st, sg, b, hy, V, nrhs, 0, std::sqrt(P.a_scale), nbv);
    for (int r = 0; r < nrhs; ++r)
        for (int k = 0; k < nev; ++k) {
            const double s = evals[k] > 0 ? 1.0 : (evals[k] < 0 ? -1.0 : 0.0);
            cb[(size_t)k + (size_t)r * nev] *= s;
        }
    E_CHK(to_dev(st, cd, cb.data(), cb.size() * sizeof(double2)));
    E_CHK(combine(c, evecs, nev, cd, nrhs, n, sg, 1.0, 1.0));
    if (overlap) launch_overlap_out(st, out, b, sg, V, nrhs, 1, 1.0, nbv);
    E_HIPCHK(hipGetLastError());
    E_HIPCHK(hipStreamSynchronize(st));
    return 0;
}

}  // namespace msb
