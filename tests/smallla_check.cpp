// Reads "op m" and an m x m complex matrix (column-major, re im pairs) from
// stdin; prints the result of the small dense routine of the library's
// eigensolver: chol -> R (upper, R^H R = A) or FAIL; inv -> R^{-1} of the
// upper triangle of A; eig -> eigenvalues, then Q (column-major).
#include <cstdio>
#include <cstring>
#include <vector>

#include "smallla.h"

using msb::sla::cplx;

int main() {
    char op[16];
    int m;
    if (std::scanf("%15s %d", op, &m) != 2 || m < 1) return 2;
    std::vector<cplx> A((size_t)m * m);
    for (auto &z : A) {
        double re, im;
        if (std::scanf("%lf %lf", &re, &im) != 2) return 2;
        z = cplx(re, im);
    }
    auto dump = [&](const std::vector<cplx> &M) {
        for (const cplx &z : M) std::printf("%.17g %.17g\n", z.real(), z.imag());
    };
    if (!std::strcmp(op, "chol")) {
        if (!msb::sla::cholesky_upper(A, m)) {
            std::printf("FAIL\n");
            return 0;
        }
        dump(A);
    } else if (!std::strcmp(op, "inv")) {
        msb::sla::upper_inverse(A, m);
        dump(A);
    } else if (!std::strcmp(op, "eig")) {
        std::vector<double> w;
        std::vector<cplx> Q;
        const int sweeps = msb::sla::heev_jacobi(A, m, w, Q);
        std::printf("%d\n", sweeps);
        for (double x : w) std::printf("%.17g\n", x);
        dump(Q);
    } else {
        return 2;
    }
    return 0;
}
