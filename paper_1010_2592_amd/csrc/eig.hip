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
// m >= K + 1 vectors.  Each iteration applies T_d((H^2 - e)/h), the degree-d
// Chebyshev polynomial of the interval [c, hi] (c the block's largest Ritz
// value of H^2, hi an upper bound of the spectrum from the power iteration),
// which damps the modes above c and keeps those below; then Cholesky-QR twice
// and Rayleigh-Ritz with H itself (so the Ritz pairs are eigenpairs of H,
// either sign).  The block products are plain tall-skinny GEMMs (rocBLAS), the
// small factorisations rocSOLVER; the Chebyshev steps are the library's own
// stencils on the whole block (chunked form) and one vector pass.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "ctx.h"

namespace msb {

namespace {

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
#define E_BLAS(x)                                                                       \
    do {                                                                                \
        rocblas_status s_ = (x);                                                        \
        if (s_ != rocblas_status_success)                                               \
            return set_error(S_ERR_HIP, std::string(#x) + ": rocBLAS/rocSOLVER status " + \
                                            std::to_string((int)s_));                   \
    } while (0)

int blas_handle(Ctx *c, rocblas_handle *h) {
    if (!c->blas) {
        rocblas_handle nh = nullptr;
        E_BLAS(rocblas_create_handle(&nh));
        c->blas = nh;
    }
    *h = (rocblas_handle)c->blas;
    E_BLAS(rocblas_set_stream(*h, c->stream));
    return 0;
}

inline rocblas_double_complex *zc(double2 *p) { return reinterpret_cast<rocblas_double_complex *>(p); }
inline const rocblas_double_complex *zc(const double2 *p) {
    return reinterpret_cast<const rocblas_double_complex *>(p);
}

// C (m1 x m2, column-major) = X^H Y for blocks X [m1][n], Y [m2][n]
int gram(rocblas_handle h, const double2 *X, int m1, const double2 *Y, int m2, long n, double2 *C) {
    const rocblas_double_complex one{1.0, 0.0}, zero{0.0, 0.0};
    E_BLAS(rocblas_zgemm(h, rocblas_operation_conjugate_transpose, rocblas_operation_none, m1, m2, (int)n, &one,
                         zc(X), (int)n, zc(Y), (int)n, &zero, zc(C), m1));
    return 0;
}
// Z [m2][n] = alpha X Q + beta Z, X [m1][n], Q (m1 x m2, column-major)
int combine(rocblas_handle h, const double2 *X, int m1, const double2 *Q, int m2, long n, double2 *Z,
            double alpha, double beta) {
    const rocblas_double_complex al{alpha, 0.0}, be{beta, 0.0};
    E_BLAS(rocblas_zgemm(h, rocblas_operation_none, rocblas_operation_none, (int)n, m2, m1, &al, zc(X), (int)n,
                         zc(Q), m1, &be, zc(Z), (int)n));
    return 0;
}

// z -= y over n complex (Chebyshev three-term step)
__global__ __launch_bounds__(BLOCK) void k_sub(double2 *z, const double2 *y, long n) {
    for (long e = (long)blockIdx.x * BLOCK + threadIdx.x; e < n; e += (long)gridDim.x * BLOCK)
        z[e] = csub(z[e], y[e]);
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

void eig_release(Ctx *c) {
    if (c->blas) (void)rocblas_destroy_handle((rocblas_handle)c->blas);
    c->blas = nullptr;
}

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
    rocblas_handle h;
    E_CHK(blas_handle(c, &h));
    const size_t blk = (size_t)m * n * sizeof(double2);
    E_CHK(ensure(c->ws_eY, blk));
    E_CHK(ensure(c->ws_eW, blk));
    E_CHK(ensure(c->ws_eZ, blk));
    E_CHK(ensure(c->ws_eP, blk));
    E_CHK(ensure(c->ws_eS, (size_t)m * m * sizeof(double2) + (size_t)3 * m * sizeof(double) + 64));
    E_CHK(ensure(c->ws_part, (size_t)m * nbv * sizeof(double)));
    double2 *Y = (double2 *)c->ws_eY.p, *W = (double2 *)c->ws_eW.p, *Z = (double2 *)c->ws_eZ.p,
            *Pv = (double2 *)c->ws_eP.p;
    double2 *S = (double2 *)c->ws_eS.p;
    double *D = (double *)(S + (size_t)m * m), *E = D + m, *T = E + m;
    rocblas_int *dinfo = (rocblas_int *)(T + m);
    double *part = (double *)c->ws_part.p;
    E_HIPCHK(hipMemcpyAsync(Y, start, blk, hipMemcpyDeviceToDevice, st));

    // Y <- Y U^{-1} with U^H U = Y^H Y, twice
    auto orth = [&]() -> int {
        for (int pass = 0; pass < 2; ++pass) {
            E_CHK(gram(h, Y, m, Y, m, n, S));
            E_BLAS(rocsolver_zpotrf(h, rocblas_fill_upper, m, zc(S), m, dinfo));
            rocblas_int info = 0;
            E_CHK(to_host(st, &info, dinfo, sizeof(info)));
            if (info != 0) return set_error(S_BREAKDOWN, "low_modes: the block lost rank (Cholesky-QR failed)");
            const rocblas_double_complex one{1.0, 0.0};
            E_BLAS(rocblas_ztrsm(h, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none,
                                 rocblas_diagonal_non_unit, (int)n, m, &one, zc(S), m, zc(Y), (int)n));
        }
        return 0;
    };
    // Rayleigh-Ritz with H: Y <- Y Q, W <- H Y, ordered by |theta|
    std::vector<double> theta(m), res(m);
    std::vector<double2> Qh((size_t)m * m), Qs((size_t)m * m);
    auto rayleigh_ritz = [&]() -> int {
        {
            DslashArgs<double> a = h_args(c, Y, W);
            launch_dslash<double>(st, a, m, EPI_PLAIN, false);
        }
        E_CHK(gram(h, Y, m, W, m, n, S));
        E_BLAS(rocsolver_zheevd(h, rocblas_evect_original, rocblas_fill_upper, m, zc(S), m, D, E, dinfo));
        rocblas_int info = 0;
        std::vector<double> th(m);
        E_CHK(to_host(st, &info, dinfo, sizeof(info)));
        E_CHK(to_host(st, th.data(), D, m * sizeof(double)));
        E_CHK(to_host(st, Qh.data(), S, Qh.size() * sizeof(double2)));
        if (info != 0) return set_error(S_BREAKDOWN, "low_modes: Rayleigh-Ritz eigensolver did not converge");
        std::vector<int> ord(m);
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return std::fabs(th[x]) < std::fabs(th[y]); });
        for (int j = 0; j < m; ++j) {
            theta[j] = th[ord[j]];
            std::copy(&Qh[(size_t)ord[j] * m], &Qh[(size_t)ord[j] * m] + m, &Qs[(size_t)j * m]);
        }
        E_CHK(to_dev(st, S, Qs.data(), Qs.size() * sizeof(double2)));
        E_CHK(combine(h, Y, m, S, m, n, Z, 1.0, 0.0));
        std::swap(Y, Z);
        E_CHK(combine(h, W, m, S, m, n, Z, 1.0, 0.0));
        std::swap(W, Z);
        // residuals ||H y_j - theta_j y_j||
        E_CHK(to_dev(st, T, theta.data(), m * sizeof(double)));
        hipLaunchKernelGGL(k_resid, dim3(nbv, m), dim3(BLOCK), 0, st, W, Y, T, n, part, nbv);
        E_HIPCHK(hipGetLastError());
        std::vector<double> pr((size_t)m * nbv);
        E_CHK(to_host(st, pr.data(), part, pr.size() * sizeof(double)));
        for (int j = 0; j < m; ++j) {
            double s2 = 0.0;
            for (int q = 0; q < nbv; ++q) s2 += pr[(size_t)j * nbv + q];
            res[j] = std::sqrt(s2);
        }
        return 0;
    };

    E_CHK(orth());
    E_CHK(rayleigh_ritz());
    const double scale = std::sqrt(hi);   // |lambda| bound of H
    int it = 0;
    for (; it < max_iter; ++it) {
        bool done = true;
        for (int j = 0; j < nev; ++j) done = done && res[j] <= tol * scale;
        if (done) break;
        // damp [c, hi] with c the block's largest Ritz value of H^2
        double c2 = 0.0;
        for (int j = 0; j < m; ++j) c2 = std::max(c2, theta[j] * theta[j]);
        c2 = std::min(c2, 0.5 * hi);
        const double e = 0.5 * (hi + c2), hw = 0.5 * (hi - c2);
        // Chebyshev recurrence on Y (the current block): P = Y_{j-1}, Y = Y_j
        double2 *Yp = Pv, *Yc = Y, *Yn = Z;
        for (int d = 1; d <= degree; ++d) {
            DslashArgs<double> a1 = h_args(c, Yc, W);          // W = H Y_j
            launch_dslash<double>(st, a1, m, EPI_PLAIN, false);
            DslashArgs<double> a2 = h_args(c, W, Yn);          // Y_{j+1} = s H W + s0 Y_j (- Y_{j-1})
            a2.v = Yc;
            a2.scale = (d == 1 ? 1.0 : 2.0) / hw;
            a2.sigma0 = -(d == 1 ? 1.0 : 2.0) * e / hw;
            launch_dslash<double>(st, a2, m, EPI_SV, false);
            if (d > 1) hipLaunchKernelGGL(k_sub, dim3(nbv), dim3(BLOCK), 0, st, Yn, Yp, (long)m * n);
            E_HIPCHK(hipGetLastError());
            double2 *t = Yp;
            Yp = Yc;
            Yc = Yn;
            Yn = t;
        }
        // the filtered block is Yc; keep the buffers Y, Z, P distinct
        if (Yc != Y) E_HIPCHK(hipMemcpyAsync(Y, Yc, blk, hipMemcpyDeviceToDevice, st));
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
    rocblas_handle h;
    E_CHK(blas_handle(c, &h));
    E_CHK(ensure(c->ws_eS, (size_t)nev * nrhs * sizeof(double2) + 64));
    E_CHK(ensure(c->ws_eY, (size_t)nrhs * n * sizeof(double2)));   // P b, then sign(H) b
    E_CHK(ensure(c->ws_eW, (size_t)nrhs * n * sizeof(double2)));   // y, then H y
    double2 *cb = (double2 *)c->ws_eS.p;
    double2 *pb = (double2 *)c->ws_eY.p, *y = (double2 *)c->ws_eW.p;
    // c = V^H b, P b = b - V c
    E_CHK(gram(h, evecs, nev, b, nrhs, n, cb));
    E_HIPCHK(hipMemcpyAsync(pb, b, (size_t)nrhs * n * sizeof(double2), hipMemcpyDeviceToDevice, st));
    E_CHK(combine(h, evecs, nev, cb, nrhs, n, pb, -1.0, 1.0));
    // y = f(A) P b
    E_CHK(ensure(c->ws_y, (size_t)nrhs * n * sizeof(double2)));
    double2 *yy = (double2 *)c->ws_y.p;
    E_CHK(solve_mshift(c, P, pb, yy, nullptr, false, rep));
    // sign part: sqrt(a) H y + V (sign(lambda) c)
    {
        DslashArgs<double> a = h_args(c, yy, y);
        launch_dslash<double>(st, a, nrhs, EPI_PLAIN, false);
    }
    double2 *sg = overlap ? pb : out;
    launch_overlap_out(st, sg, b, y, V, nrhs, 0, std::sqrt(P.a_scale), nbv);
    std::vector<double2> ch((size_t)nev * nrhs);
    E_CHK(to_host(st, ch.data(), cb, ch.size() * sizeof(double2)));
    for (int r = 0; r < nrhs; ++r)
        for (int k = 0; k < nev; ++k) {
            const double s = evals[k] > 0 ? 1.0 : (evals[k] < 0 ? -1.0 : 0.0);
            double2 &z = ch[(size_t)r * nev + k];
            z = double2{s * z.x, s * z.y};
        }
    E_CHK(to_dev(st, cb, ch.data(), ch.size() * sizeof(double2)));
    E_CHK(combine(h, evecs, nev, cb, nrhs, n, sg, 1.0, 1.0));
    if (overlap) launch_overlap_out(st, out, b, sg, V, nrhs, 1, 1.0, nbv);
    E_HIPCHK(hipGetLastError());
    E_HIPCHK(hipStreamSynchronize(st));
    return 0;
}

}  // namespace msb
