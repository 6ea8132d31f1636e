// Device-side scalar work of multi-shift BiCGstab(l): one block per
// right-hand side, FP64 throughout.  Keeping these steps on the device means
// the host never waits on an inner product inside an outer iteration: the
// vector kernels read the coefficients these kernels write, and a right-hand
// side that has stopped (or whose BiCG part has ended early) gates every later
// launch off through its SeedState flags.
//
// Seed (BiCGstab(l), x0 = 0, shadow residual b):
//   j = 0: rho0 <- -omega rho0
//   rho1 = <rt, r_j>, beta = alpha rho1 / rho0, rho0 = rho1
//   gamma = <rt, u_{j+1}>, alpha = rho0 / gamma
//   MR: G g = c by Cholesky, G_ik = <r_i, r_k>, c_i = <r_i, r_0>, omega = g_l
// Shifts (sigma' = sigma_s - sigma_0; zeta_n = R_n(-sigma'), pi_n = P_n(-sigma'),
// psi = product of the MR polynomials at -sigma'):
//   pi_n = zeta_n - beta_n pi_{n-1},  zeta_{n+1} = zeta_n + alpha_n sigma' pi_n
//   alpha^s = alpha zeta_n / zeta_{n+1},  beta^s = beta (zeta_{n-1} / zeta_n)^2
//   kappa_n = 1 / (zeta_n psi)
//   MR: q^s = 1 - sum_i g_i (-sigma')^i,
//       c^s_k = (1/q^s) sum_{i>k} g_i (-sigma')^{i-1-k},  psi <- psi q^s
// Convergence at the end of each outer iteration: shift s freezes when
// ||r_0|| / (|zeta psi| ||b||) <= tol (its outer-iteration count is the
// paper's M_s, Section 2); the iteration stops when no shift is left.
#include "scalar_dev.h"

namespace msb {

namespace {

using namespace dev;

__global__ __launch_bounds__(BLOCK) void sc_init(ScalarArgs a) { sc_init_body(a, blockIdx.x); }
__global__ __launch_bounds__(BLOCK) void sc_beta(ScalarArgs a) { sc_beta_body(a, blockIdx.x); }
__global__ __launch_bounds__(BLOCK) void sc_alpha(ScalarArgs a) { sc_alpha_body(a, blockIdx.x); }
__global__ __launch_bounds__(BLOCK) void sc_mr(ScalarArgs a) { sc_mr_body(a, blockIdx.x); }
__global__ __launch_bounds__(BLOCK) void sc_rel(ScalarArgs a) { sc_rel_body(a, blockIdx.x); }
__global__ __launch_bounds__(BLOCK) void sc_conv(ScalarArgs a) { sc_conv_body(a, blockIdx.x); }
__global__ __launch_bounds__(BLOCK) void sc_defer(ScalarArgs a) { sc_defer_body(a, blockIdx.x); }
__global__ __launch_bounds__(BLOCK) void sc_basis(ScalarArgs a) { sc_basis_body(a, blockIdx.x); }
__global__ __launch_bounds__(BLOCK) void sc_exh(ScalarArgs a) { sc_exh_body(a, blockIdx.x); }
__global__ __launch_bounds__(64) void sc_basis_replay(BasisReplayArgs a) { sc_basis_replay_body(a, blockIdx.x); }

}  // namespace

void launch_sc_init(hipStream_t st, const ScalarArgs &a, int nrhs) {
    hipLaunchKernelGGL(sc_init, dim3(nrhs), dim3(BLOCK), 0, st, a);
}
void launch_sc_beta(hipStream_t st, const ScalarArgs &a, int nrhs) {
    hipLaunchKernelGGL(sc_beta, dim3(nrhs), dim3(BLOCK), 0, st, a);
}
void launch_sc_alpha(hipStream_t st, const ScalarArgs &a, int nrhs) {
    hipLaunchKernelGGL(sc_alpha, dim3(nrhs), dim3(BLOCK), 0, st, a);
}
void launch_sc_mr(hipStream_t st, const ScalarArgs &a, int nrhs) {
    hipLaunchKernelGGL(sc_mr, dim3(nrhs), dim3(BLOCK), 0, st, a);
}
void launch_sc_rel(hipStream_t st, const ScalarArgs &a, int nrhs) {
    hipLaunchKernelGGL(sc_rel, dim3(nrhs), dim3(BLOCK), 0, st, a);
}
void launch_sc_conv(hipStream_t st, const ScalarArgs &a, int nrhs) {
    hipLaunchKernelGGL(sc_conv, dim3(nrhs), dim3(BLOCK), 0, st, a);
}
void launch_sc_defer(hipStream_t st, const ScalarArgs &a, int nrhs) {
    hipLaunchKernelGGL(sc_defer, dim3(nrhs), dim3(BLOCK), 0, st, a);
}
void launch_sc_basis(hipStream_t st, const ScalarArgs &a, int nrhs) {
    hipLaunchKernelGGL(sc_basis, dim3(nrhs), dim3(BLOCK), 0, st, a);
}
void launch_sc_exh(hipStream_t st, const ScalarArgs &a, int nrhs) {
    hipLaunchKernelGGL(sc_exh, dim3(nrhs), dim3(BLOCK), 0, st, a);
}
void launch_sc_basis_replay(hipStream_t st, const BasisReplayArgs &a, int nrhs) {
    hipLaunchKernelGGL(sc_basis_replay, dim3(nrhs), dim3(64), 0, st, a);
}

}  // namespace msb
