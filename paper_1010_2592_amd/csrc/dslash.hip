// Wilson-Dirac stencil with chemical potential, D_w(mu), for gfx950.
//
//   (D psi)(x) = (4+m) psi(x)
//     - 1/2 sum_nu b_nu(x)   (1 - gamma_nu) e^{+mu d_nu4} U_nu(x)     psi(x+nu)
//     - 1/2 sum_nu b_nu(x-nu)(1 + gamma_nu) e^{-mu d_nu4} U_nu(x-nu)^+ psi(x-nu)
//
// The operator the paper names in Section 1; chiral gamma matrices.  One
// work-item per lattice site and right-hand side.  Each hop loads the neighbour's 12 complex components (coalesced SoA
// planes), projects them to a two-component half spinor with (1 -/+ gamma),
// multiplies the half spinor by the 3x3 link, and reconstructs the lower spin
// components from the upper ones.  The kernel is HBM-bound (about 1.4 flop
// per byte in FP64), so it never touches the matrix cores.
//
// Epilogues (fused so that the output is written once and never re-read):
//   EPI_PLAIN  out = scale * [gamma5] D in
//   EPI_MV     out = scale * gamma5 D in + sigma0 * v, and per-block partials
//              of <rt, out> and ||out||^2 (the next BiCG inner product)
//   EPI_MV_Y   as EPI_MV without partials, plus y += c * out (double-pass
//              accumulation of the Mv outputs)
//   EPI_SV     out = scale * gamma5 D in + sigma0 * v, nothing else
//   EPI_SV2    as EPI_SV minus w (the Chebyshev three-term step of the
//              low-mode eigensolver: out = scale gamma5 D in + sigma0 v - w)
//   EPI_MVN    as EPI_MV without reading rt (partials of
//              <rt, out> left zero; the solver adds them from a sparse list
//              of rt's nonzero entries)
// Which operands exist is a compile-time property of the mode: run-time null
// checks inside the unrolled epilogue made the compiler keep every epilogue
// load live at once and spill.
#include <hip/hip_ext.h>

#include "stencil_dev.h"

namespace msb {

namespace {

using namespace dev;

template <typename T, int EPI, bool G5IN>
__global__ __launch_bounds__(BLOCK) void dslash_kernel(DslashArgs<T> a) {
    dslash_body<T, EPI, G5IN>(a, blockIdx.x);
}

// wavefronts per block of the chunked stencil: 4 (FP64: two blocks per CU by
// the 74 KB of staged links and by registers; FP32: three, 96 chunks resident
// per XCD, whose z-t checkerboard reads overlap in L2 better than those of
// one 12-wavefront block per CU, 2863 against 2690 GB/s on 16^3x32 with 12
// right-hand sides)
template <typename T> constexpr int chunk_waves() { return 4; }

template <typename T, int EPI, bool G5IN>
__global__ __launch_bounds__(64 * chunk_waves<T>()) void dslash_chunk_kernel(DslashArgs<T> a) {
    dslash_chunk<T, EPI, G5IN, chunk_waves<T>()>(a, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Link force: gradient of sum_pairs c Re <p, D(mu) q> with respect to the
// links (the unconstrained complex gradient, dL/dRe + i dL/dIm).  U_nu(x)
// enters (D q)(x) through the forward hop and (D q)(x+nu) through the
// backward hop, hence with
//   M1_ab = sum_alpha conj(p(x)_{alpha a})    [(1 - gamma_nu) q(x+nu)]_{alpha b}
//   M2_ab = sum_alpha conj(p(x+nu)_{alpha a}) [(1 + gamma_nu) q(x)]_{alpha b}
//   G_nu(x) += -c b_nu(x)/2 (e^{mu d_nu4} conj(M1) + e^{-mu d_nu4} M2^T).
// One work-item per site; it accumulates all pairs and right-hand sides of
// the launch before its single read-modify-write of the 36 link entries.
template <int NU, int SGN>
__device__ __forceinline__ void proj_full(const double2 *__restrict__ q, long rs, int V, int s, bool g5,
                                          double2 (&out)[4][3]) {
    using P = Proj<NU, SGN>;
    double2 h[2][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double2 q0 = q[(0 + c) * V + s], q1 = q[(3 + c) * V + s];
        double2 qa = q[(3 * P::P0 + c) * V + s], qb = q[(3 * P::P1 + c) * V + s];
        if (g5) {
            if (P::P0 >= 2) qa = cneg(qa);
            if (P::P1 >= 2) qb = cneg(qb);
        }
        h[0][c] = cadd(q0, mulcode<P::C0>(qa));
        h[1][c] = cadd(q1, mulcode<P::C1>(qb));
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        out[0][c] = h[0][c];
        out[1][c] = h[1][c];
        out[2][c] = mulcode<P::D2>(h[P::Q2][c]);
        out[3][c] = mulcode<P::D3>(h[P::Q3][c]);
    }
    (void)rs;
}

template <int NU>
__device__ __forceinline__ void force_dir(const LinkForceArgs &a, int s, int sf, double bnu, double2 *G) {
    const int V = a.g.V;
    const long nv = 12L * V;
    double2 M1[3][3], M2[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) M1[i][j] = M2[i][j] = d2(0, 0);
    for (int k = 0; k < a.npair; ++k) {
        const LinkPair &pr = a.pairs[k];
        for (int r = 0; r < a.nrhs; ++r) {
            const double2 *p = pr.p + (size_t)r * (pr.p_rs ? pr.p_rs : nv);
            const double2 *q = pr.q + (size_t)r * (pr.q_rs ? pr.q_rs : nv);
            const double c = pr.c;
            double2 pr1[4][3], pr2[4][3];
            proj_full<NU, -1>(q, 0, V, sf, false, pr1);      // (1 - gamma) q(x+nu)
            proj_full<NU, +1>(q, 0, V, s, false, pr2);       // (1 + gamma) q(x)
#pragma unroll
            for (int al = 0; al < 4; ++al) {
#pragma unroll
                for (int ia = 0; ia < 3; ++ia) {
                    double2 px = p[(3 * al + ia) * V + s];
                    double2 pf = p[(3 * al + ia) * V + sf];
                    if (pr.g5p && al >= 2) {
                        px = cneg(px);
                        pf = cneg(pf);
                    }
                    px = cscale(px, c);
                    pf = cscale(pf, c);
#pragma unroll
                    for (int ib = 0; ib < 3; ++ib) {
                        M1[ia][ib] = cadd(M1[ia][ib], cmulc(px, pr1[al][ib]));
                        M2[ia][ib] = cadd(M2[ia][ib], cmulc(pf, pr2[al][ib]));
                    }
                }
            }
        }
    }
    const double ef = (NU == 3) ? a.ef : 1.0, eb = (NU == 3) ? a.eb : 1.0;
    const double f = -0.5 * bnu;
#pragma unroll
    for (int ia = 0; ia < 3; ++ia)
#pragma unroll
        for (int ib = 0; ib < 3; ++ib) {
            double2 *gp = G + ((size_t)NU * 9 + 3 * ia + ib) * V + s;
            const double2 add = cscale(cadd(cscale(cconj(M1[ia][ib]), ef), cscale(M2[ib][ia], eb)), f);
            *gp = cadd(*gp, add);
        }
}

__global__ __launch_bounds__(BLOCK) void link_force_kernel(LinkForceArgs a) {
    const int V = a.g.V, Lx = a.g.Lx, Ly = a.g.Ly, Lz = a.g.Lz, Lt = a.g.Lt;
    for (int s = blockIdx.x * BLOCK + threadIdx.x; s < V; s += gridDim.x * BLOCK) {
        const int x = s % Lx;
        const int r1 = s / Lx;
        const int yy = r1 % Ly;
        const int r2 = r1 / Ly;
        const int z = r2 % Lz;
        const int t = r2 / Lz;
        const int sxy = Lx * Ly, sxyz = Lx * Ly * Lz;
        force_dir<0>(a, s, (x == Lx - 1) ? s - (Lx - 1) : s + 1, 1.0, a.G);
        force_dir<1>(a, s, (yy == Ly - 1) ? s - (Ly - 1) * Lx : s + Lx, 1.0, a.G);
        force_dir<2>(a, s, (z == Lz - 1) ? s - (Lz - 1) * sxy : s + sxy, 1.0, a.G);
        force_dir<3>(a, s, (t == Lt - 1) ? s - (Lt - 1) * sxyz : s + sxyz, (t == Lt - 1) ? a.bc : 1.0, a.G);
    }
}

}  // namespace

namespace {
thread_local hipEvent_t t_start = nullptr, t_stop = nullptr;
thread_local bool t_taken = false;

// one stencil dispatch, with the armed timing events if any
template <typename T>
void dispatch(void (*kernel)(DslashArgs<T>), dim3 grid, dim3 block, hipStream_t st, const DslashArgs<T> &a) {
    if (t_start) {
        hipExtLaunchKernelGGL(kernel, grid, block, 0, st, t_start, t_stop, 0, a);
        t_start = t_stop = nullptr;
        t_taken = true;
    } else {
        hipLaunchKernelGGL(kernel, grid, block, 0, st, a);
    }
}
}  // namespace

void stencil_timing_arm(hipEvent_t start, hipEvent_t stop) {
    t_start = start;
    t_stop = stop;
    t_taken = false;
}

bool stencil_timing_taken() {
    const bool k = t_taken;
    t_start = t_stop = nullptr;
    t_taken = false;
    return k;
}

template <typename T>
void launch_dslash(hipStream_t st, DslashArgs<T> a, int nrhs, int epi, bool g5in) {
    if (nrhs >= CHUNK_MIN_RHS) {
        dim3 grid((unsigned)dslash_chunk_prepare(a, nrhs)), block(64 * chunk_waves<T>());
#define MSB_DS(E, G5) dispatch<T>(dslash_chunk_kernel<T, E, G5>, grid, block, st, a)
        if (g5in) {
            if (epi == EPI_PLAIN) MSB_DS(EPI_PLAIN, true);
            else if (epi == EPI_MV) MSB_DS(EPI_MV, true);
            else if (epi == EPI_SV) MSB_DS(EPI_SV, true);
            else if (epi == EPI_SV2) MSB_DS(EPI_SV2, true);
            else if (epi == EPI_MVN) MSB_DS(EPI_MVN, true);
            else MSB_DS(EPI_MV_Y, true);
        } else {
            if (epi == EPI_PLAIN) MSB_DS(EPI_PLAIN, false);
            else if (epi == EPI_MV) MSB_DS(EPI_MV, false);
            else if (epi == EPI_SV) MSB_DS(EPI_SV, false);
            else if (epi == EPI_SV2) MSB_DS(EPI_SV2, false);
            else if (epi == EPI_MVN) MSB_DS(EPI_MVN, false);
            else MSB_DS(EPI_MV_Y, false);
        }
#undef MSB_DS
        return;
    }
    dim3 grid((unsigned)dslash_prepare(a, nrhs)), block(BLOCK);
#define MSB_DS(E, G5) dispatch<T>(dslash_kernel<T, E, G5>, grid, block, st, a)
    if (g5in) {
        if (epi == EPI_PLAIN) MSB_DS(EPI_PLAIN, true);
        else if (epi == EPI_MV) MSB_DS(EPI_MV, true);
        else if (epi == EPI_SV) MSB_DS(EPI_SV, true);
        else if (epi == EPI_SV2) MSB_DS(EPI_SV2, true);
        else if (epi == EPI_MVN) MSB_DS(EPI_MVN, true);
        else MSB_DS(EPI_MV_Y, true);
    } else {
        if (epi == EPI_PLAIN) MSB_DS(EPI_PLAIN, false);
        else if (epi == EPI_MV) MSB_DS(EPI_MV, false);
        else if (epi == EPI_SV) MSB_DS(EPI_SV, false);
        else if (epi == EPI_SV2) MSB_DS(EPI_SV2, false);
        else if (epi == EPI_MVN) MSB_DS(EPI_MVN, false);
        else MSB_DS(EPI_MV_Y, false);
    }
#undef MSB_DS
}

template void launch_dslash<double>(hipStream_t, DslashArgs<double>, int, int, bool);

namespace {
__global__ __launch_bounds__(256) void k_link_gershgorin(const double2 *U, int V, double *blockmax) {
    __shared__ double red[256];
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    double g = 0.0;
    if (idx < 4L * V) {
        const int nu = (int)(idx / V), s = (int)(idx % V);
        double2 u[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) u[i][j] = U[((size_t)nu * 9 + 3 * i + j) * V + s];
        for (int k = 0; k < 3; ++k) {
            double row = 0.0;
            for (int l = 0; l < 3; ++l) {
                double2 m = d2(0, 0);
                for (int i = 0; i < 3; ++i) m = cadd(m, cmulc(u[i][k], u[i][l]));   // conj(u_ik) u_il
                row += (l == k) ? m.x : sqrt(m.x * m.x + m.y * m.y);
            }
            g = row > g ? row : g;
        }
    }
    red[threadIdx.x] = g;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x + w] > red[threadIdx.x] ? red[threadIdx.x + w]
                                                                                        : red[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) blockmax[blockIdx.x] = red[0];
}
}  // namespace

void launch_link_gershgorin(hipStream_t st, const double2 *U, int V, double *blockmax) {
    hipLaunchKernelGGL(k_link_gershgorin, dim3(link_gershgorin_blocks(V)), dim3(256), 0, st, U, V, blockmax);
}

void launch_link_force(hipStream_t st, const LinkForceArgs &a) {
    const int nb = nblocks_for(a.g.V);
    hipLaunchKernelGGL(link_force_kernel, dim3(nb), dim3(BLOCK), 0, st, a);
}
template void launch_dslash<float>(hipStream_t, DslashArgs<float>, int, int, bool);

}  // namespace msb
