// Small dense complex linear algebra on the host (matrices of order <= a few
// dozen): the Rayleigh-Ritz and Cholesky-QR steps of the low-mode eigensolver
// reduce the tall block products to m x m problems, which are solved here in
// FP64 in microseconds instead of through device library calls.
//
// Storage: column-major, A[i + j * m].  Plain C++ (no HIP), so the same header
// builds on the host side of the library and in a CPU-only check program.
#pragma once

#include <algorithm>
#include <cmath>
#include <complex>
#include <numeric>
#include <vector>

namespace msb {
namespace sla {

using cplx = std::complex<double>;

// G = R^H R for Hermitian positive definite G; R (upper triangular) replaces
// G, the strict lower triangle is zeroed.  Returns false when a pivot is not
// positive (G numerically singular).
inline bool cholesky_upper(std::vector<cplx> &G, int m) {
    for (int j = 0; j < m; ++j) {
        double d = G[j + (size_t)j * m].real();
        for (int k = 0; k < j; ++k) d -= std::norm(G[k + (size_t)j * m]);
        if (!(d > 0.0)) return false;
        const double rjj = std::sqrt(d);
        G[j + (size_t)j * m] = rjj;
        for (int c = j + 1; c < m; ++c) {
            cplx s = G[j + (size_t)c * m];
            for (int k = 0; k < j; ++k) s -= std::conj(G[k + (size_t)j * m]) * G[k + (size_t)c * m];
            G[j + (size_t)c * m] = s / rjj;
        }
    }
    for (int j = 0; j < m; ++j)
        for (int i = j + 1; i < m; ++i) G[i + (size_t)j * m] = 0.0;
    return true;
}

// R <- R^{-1} for upper triangular R with nonzero diagonal (back substitution
// column by column; the inverse is upper triangular too).
inline void upper_inverse(std::vector<cplx> &R, int m) {
    std::vector<cplx> X((size_t)m * m, cplx(0.0));
    for (int j = 0; j < m; ++j) {
        // solve R x = e_j for x (column j of the inverse), x_i = 0 for i > j
        for (int i = j; i >= 0; --i) {
            cplx s = (i == j) ? cplx(1.0) : cplx(0.0);
            for (int k = i + 1; k <= j; ++k) s -= R[i + (size_t)k * m] * X[k + (size_t)j * m];
            X[i + (size_t)j * m] = s / R[i + (size_t)i * m];
        }
    }
    R.swap(X);
}

// Eigen-decomposition of a Hermitian matrix by cyclic Jacobi rotations:
// A = Q diag(w) Q^H, w ascending, Q unitary (columns are the eigenvectors).
// A is overwritten.  Each rotation first rotates the phase of a_pq away
// (a diagonal unitary), then zeroes the now real off-diagonal entry with the
// symmetric Schur rotation.  Returns the number of sweeps, or -1 when the
// off-diagonal part did not fall below the rounding level.
inline int heev_jacobi(std::vector<cplx> &A, int m, std::vector<double> &w, std::vector<cplx> &Q) {
    auto at = [&](int i, int j) -> cplx & { return A[i + (size_t)j * m]; };
    Q.assign((size_t)m * m, cplx(0.0));
    for (int i = 0; i < m; ++i) Q[i + (size_t)i * m] = 1.0;
    for (int i = 0; i < m; ++i) at(i, i) = at(i, i).real();
    double fro = 0.0;
    for (const cplx &z : A) fro += std::norm(z);
    fro = std::sqrt(fro);
    int sweeps = 0;
    const int max_sweeps = 60;
    for (; sweeps < max_sweeps; ++sweeps) {
        double off = 0.0;
        for (int j = 0; j < m; ++j)
            for (int i = 0; i < j; ++i) off += std::norm(at(i, j));
        if (std::sqrt(2.0 * off) <= 1e-15 * fro || fro == 0.0) break;
        for (int p = 0; p < m - 1; ++p)
            for (int q = p + 1; q < m; ++q) {
                const cplx g = at(p, q);
                const double ag = std::abs(g);
                if (ag == 0.0) continue;
                const cplx ph = g / ag;                    // e^{i phi}
                const double app = at(p, p).real(), aqq = at(q, q).real();
                const double tau = (aqq - app) / (2.0 * ag);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                // G = diag(1, e^{-i phi}) [[c, s], [-s, c]] on columns (p, q)
                const cplx gqp = -s * std::conj(ph), gqq = c * std::conj(ph);
                for (int k = 0; k < m; ++k) {     // A <- A G
                    const cplx akp = at(k, p), akq = at(k, q);
                    at(k, p) = c * akp + gqp * akq;
                    at(k, q) = s * akp + gqq * akq;
                }
                for (int k = 0; k < m; ++k) {     // A <- G^H A
                    const cplx apk = at(p, k), aqk = at(q, k);
                    at(p, k) = c * apk + std::conj(gqp) * aqk;
                    at(q, k) = s * apk + std::conj(gqq) * aqk;
                }
                at(p, q) = 0.0;
                at(q, p) = 0.0;
                at(p, p) = at(p, p).real();
                at(q, q) = at(q, q).real();
                for (int k = 0; k < m; ++k) {     // Q <- Q G
                    const cplx qkp = Q[k + (size_t)p * m], qkq = Q[k + (size_t)q * m];
                    Q[k + (size_t)p * m] = c * qkp + gqp * qkq;
                    Q[k + (size_t)q * m] = s * qkp + gqq * qkq;
                }
            }
    }
    std::vector<int> ord(m);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return at(x, x).real() < at(y, y).real(); });
    std::vector<cplx> Qs((size_t)m * m);
    w.resize(m);
    for (int j = 0; j < m; ++j) {
        w[j] = at(ord[j], ord[j]).real();
        std::copy(&Q[(size_t)ord[j] * m], &Q[(size_t)ord[j] * m] + m, &Qs[(size_t)j * m]);
    }
    Q.swap(Qs);
    return sweeps < max_sweeps ? sweeps : -1;
}

}  // namespace sla
}  // namespace msb
