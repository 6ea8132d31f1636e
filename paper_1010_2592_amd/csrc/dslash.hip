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
// Which operands exist is a compile-time property of the mode: run-time null
// checks inside the unrolled epilogue made the compiler keep every epilogue
// load live at once and spill.
#include "common.h"
#include "kernels.h"

namespace msb {

namespace {

// multiply by one of {+1, -1, +i, -i}
template <int CODE, typename Z>
__device__ __forceinline__ Z mulcode(Z z) {
    if constexpr (CODE == 0) return z;
    else if constexpr (CODE == 1) return cneg(z);
    else if constexpr (CODE == 2) return ctimes_i(z);
    else return ctimes_mi(z);
}

constexpr int ONE = 0, NEG = 1, I = 2, MI = 3;

// Spin projection (1 + SGN gamma_NU) psi = (h0, h1, D2 h_Q2, D3 h_Q3) with
// h0 = psi_0 + C0 psi_P0, h1 = psi_1 + C1 psi_P1 (chiral basis).
template <int NU, int SGN> struct Proj;
template <> struct Proj<0, -1> { static constexpr int P0 = 3, C0 = I, P1 = 2, C1 = I, Q2 = 1, D2 = MI, Q3 = 0, D3 = MI; };
template <> struct Proj<0, +1> { static constexpr int P0 = 3, C0 = MI, P1 = 2, C1 = MI, Q2 = 1, D2 = I, Q3 = 0, D3 = I; };
template <> struct Proj<1, -1> { static constexpr int P0 = 3, C0 = ONE, P1 = 2, C1 = NEG, Q2 = 1, D2 = NEG, Q3 = 0, D3 = ONE; };
template <> struct Proj<1, +1> { static constexpr int P0 = 3, C0 = NEG, P1 = 2, C1 = ONE, Q2 = 1, D2 = ONE, Q3 = 0, D3 = NEG; };
template <> struct Proj<2, -1> { static constexpr int P0 = 2, C0 = I, P1 = 3, C1 = MI, Q2 = 0, D2 = MI, Q3 = 1, D3 = I; };
template <> struct Proj<2, +1> { static constexpr int P0 = 2, C0 = MI, P1 = 3, C1 = I, Q2 = 0, D2 = I, Q3 = 1, D3 = MI; };
template <> struct Proj<3, -1> { static constexpr int P0 = 2, C0 = NEG, P1 = 3, C1 = NEG, Q2 = 0, D2 = NEG, Q3 = 1, D3 = NEG; };
template <> struct Proj<3, +1> { static constexpr int P0 = 2, C0 = ONE, P1 = 3, C1 = ONE, Q2 = 0, D2 = ONE, Q3 = 1, D3 = ONE; };

// Load spin component `sp` (3 colours) of site `s`; with G5IN the lower two
// spins are negated (gamma5 applied on the fly).
template <typename T, bool G5IN>
__device__ __forceinline__ void load_spin(const C<T> *__restrict__ in, int V, int s, int sp, C<T> (&c)[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        C<T> z = in[(3 * sp + a) * V + s];
        if (G5IN && sp >= 2) z = cneg(z);
        c[a] = z;
    }
}

// acc += f * (1 + SGN gamma_NU) Umat psi(sn), Umat = U_NU(sl) (DAG=false) or
// U_NU(sl)^+ (DAG=true)
template <typename T, int NU, int SGN, bool DAG, bool G5IN>
__device__ __forceinline__ void hop(C<T> (&acc)[4][3], const C<T> *__restrict__ in,
                                   const C<T> *__restrict__ U, int V, int sn, int sl, T f) {
    using P = Proj<NU, SGN>;
    C<T> h[2][3];
    {
        C<T> p0[3], p1[3], q0[3], q1[3];
        load_spin<T, G5IN>(in, V, sn, 0, p0);
        load_spin<T, G5IN>(in, V, sn, 1, p1);
        load_spin<T, G5IN>(in, V, sn, P::P0, q0);
        load_spin<T, G5IN>(in, V, sn, P::P1, q1);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            h[0][a] = cadd(p0[a], mulcode<P::C0>(q0[a]));
            h[1][a] = cadd(p1[a], mulcode<P::C1>(q1[a]));
        }
    }
    const C<T> *Un = U + (size_t)NU * 9 * V + sl;
    C<T> g[2][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        C<T> u0, u1, u2;
        if (!DAG) {
            u0 = Un[(3 * a + 0) * V];
            u1 = Un[(3 * a + 1) * V];
            u2 = Un[(3 * a + 2) * V];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                C<T> r = cmul(u0, h[i][0]);
                r = cfma(u1, h[i][1], r);
                r = cfma(u2, h[i][2], r);
                g[i][a] = r;
            }
        } else {
            // (U^+)_{ab} = conj(U_{ba})
            u0 = Un[(0 * 3 + a) * V];
            u1 = Un[(1 * 3 + a) * V];
            u2 = Un[(2 * 3 + a) * V];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                C<T> r = cmulc(u0, h[i][0]);
                r = cadd(r, cmulc(u1, h[i][1]));
                r = cadd(r, cmulc(u2, h[i][2]));
                g[i][a] = r;
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        acc[0][a] = cadd(acc[0][a], cscale(g[0][a], f));
        acc[1][a] = cadd(acc[1][a], cscale(g[1][a], f));
        acc[2][a] = cadd(acc[2][a], cscale(mulcode<P::D2>(g[P::Q2][a]), f));
        acc[3][a] = cadd(acc[3][a], cscale(mulcode<P::D3>(g[P::Q3][a]), f));
    }
}

// One block per (256-site block, right-hand side).  The flattened grid is
// padded to a multiple of 8 and mapped XCD-aware: hardware block p runs on
// XCD p % 8, which here owns the contiguous logical range
// [(p % 8) per, (p % 8 + 1) per); inside it the right-hand side varies fastest,
// so the 12 sources of one site block run back to back on one XCD and share
// its L2 copy of the links and of the neighbouring planes.
template <typename T, int EPI, bool G5IN>
__global__ __launch_bounds__(BLOCK) void dslash_kernel(DslashArgs<T> a) {
    const int p = blockIdx.x;
    const int L = (p & 7) * a.per + (p >> 3);
    if (L >= a.nsb * a.nrhs) return;
    const int sblk = L / a.nrhs;
    const int rhs = L - sblk * a.nrhs;
    if (!gate_open(a.gate, rhs)) return;
    const int V = a.g.V, Lx = a.g.Lx, Ly = a.g.Ly, Lz = a.g.Lz, Lt = a.g.Lt;
    const long nv = 12L * V;
    const C<T> *__restrict__ in = a.in + (size_t)rhs * (a.in_rs ? a.in_rs : nv);
    C<T> *__restrict__ out = a.out + (size_t)rhs * (a.out_rs ? a.out_rs : nv);
    const C<T> *__restrict__ U = a.U;
    const C<T> *__restrict__ v = a.v ? a.v + (size_t)rhs * (a.v_rs ? a.v_rs : nv) : nullptr;
    const C<T> *__restrict__ rt = a.rt ? a.rt + (size_t)rhs * (a.rt_rs ? a.rt_rs : nv) : nullptr;
    double2 *__restrict__ y = a.y ? a.y + (size_t)rhs * (a.y_rs ? a.y_rs : nv) : nullptr;
    C<T> yc = mk<T>(0, 0);
    if (EPI == EPI_MV_Y) yc = to_c<T>(ld(a.ycoef, rhs));
    const T sig0 = a.sigma0_rhs ? (T)a.sigma0_rhs[rhs] : a.sigma0;
    double part[3] = {0.0, 0.0, 0.0};
    // a.sstride exceeds V, so the loop body runs at most once; keeping it a
    // loop with a run-time bound stops the compiler from hoisting every load
    // of the eight hops at once (which needs more than 256 VGPRs and spills)
    for (int s = sblk * BLOCK + threadIdx.x; s < V; s += a.sstride) {
        const int sxy = Lx * Ly, sxyz = Lx * Ly * Lz;
        const int x = s % Lx;
        const int r1 = s / Lx;
        const int yy = r1 % Ly;
        const int r2 = r1 / Ly;
        const int z = r2 % Lz;
        const int t = r2 / Lz;
        C<T> acc[4][3];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[i][c] = mk<T>(0, 0);

        int sf, sb;
        sf = (x == Lx - 1) ? s - (Lx - 1) : s + 1;
        sb = (x == 0) ? s + (Lx - 1) : s - 1;
        hop<T, 0, -1, false, G5IN>(acc, in, U, V, sf, s, (T)1);
        hop<T, 0, +1, true, G5IN>(acc, in, U, V, sb, sb, (T)1);
        sf = (yy == Ly - 1) ? s - (Ly - 1) * Lx : s + Lx;
        sb = (yy == 0) ? s + (Ly - 1) * Lx : s - Lx;
        hop<T, 1, -1, false, G5IN>(acc, in, U, V, sf, s, (T)1);
        hop<T, 1, +1, true, G5IN>(acc, in, U, V, sb, sb, (T)1);
        sf = (z == Lz - 1) ? s - (Lz - 1) * sxy : s + sxy;
        sb = (z == 0) ? s + (Lz - 1) * sxy : s - sxy;
        hop<T, 2, -1, false, G5IN>(acc, in, U, V, sf, s, (T)1);
        hop<T, 2, +1, true, G5IN>(acc, in, U, V, sb, sb, (T)1);
        sf = (t == Lt - 1) ? s - (Lt - 1) * sxyz : s + sxyz;
        sb = (t == 0) ? s + (Lt - 1) * sxyz : s - sxyz;
        const T ff = (t == Lt - 1) ? a.ef * a.bc : a.ef;
        const T fb = (t == 0) ? a.eb * a.bc : a.eb;
        hop<T, 3, -1, false, G5IN>(acc, in, U, V, sf, s, ff);
        hop<T, 3, +1, true, G5IN>(acc, in, U, V, sb, sb, fb);

        // out = scale * [gamma5] ((4+m) psi(x) - acc / 2), formed in place
#pragma unroll
        for (int sp = 0; sp < 4; ++sp) {
            C<T> ps[3];
            load_spin<T, G5IN>(in, V, s, sp, ps);
            const T sg = ((a.g5out && sp >= 2) ? (T)-1 : (T)1) * a.scale;
#pragma unroll
            for (int c = 0; c < 3; ++c)
                acc[sp][c] = cscale(csub(cscale(ps[c], a.diag), cscale(acc[sp][c], (T)0.5)), sg);
        }
#pragma unroll
        for (int sp = 0; sp < 4; ++sp) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int k = 3 * sp + c;
                C<T> o = acc[sp][c];
                if (EPI != EPI_PLAIN) o = cadd(o, cscale(v[k * V + s], sig0));
                out[k * V + s] = o;
                if (EPI == EPI_MV) {
                    const C<T> r = rt[k * V + s];
                    part[0] += (double)r.x * o.x + (double)r.y * o.y;
                    part[1] += (double)r.x * o.y - (double)r.y * o.x;
                    part[2] += (double)o.x * o.x + (double)o.y * o.y;
                }
                if (EPI == EPI_MV_Y) {
                    double2 yv = y[k * V + s];
                    yv.x += (double)yc.x * o.x - (double)yc.y * o.y;
                    yv.y += (double)yc.x * o.y + (double)yc.y * o.x;
                    y[k * V + s] = yv;
                }
            }
        }
    }
    if (EPI == EPI_MV)
        block_reduce_store<3>(part, a.part + (size_t)rhs * PMAX * a.ps + sblk, a.ps);
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

template <typename T>
void launch_dslash(hipStream_t st, DslashArgs<T> a, int nrhs, int epi, bool g5in) {
    a.nsb = (a.g.V + BLOCK - 1) / BLOCK;
    a.nrhs = nrhs;
    const long G = (long)a.nsb * nrhs;
    a.per = (int)((G + 7) / 8);
    a.sstride = 1 << 30;
    dim3 grid((unsigned)(8L * a.per)), block(BLOCK);
#define MSB_DS(E, G5) hipLaunchKernelGGL((dslash_kernel<T, E, G5>), grid, block, 0, st, a)
    if (g5in) {
        if (epi == EPI_PLAIN) MSB_DS(EPI_PLAIN, true);
        else if (epi == EPI_MV) MSB_DS(EPI_MV, true);
        else if (epi == EPI_SV) MSB_DS(EPI_SV, true);
        else MSB_DS(EPI_MV_Y, true);
    } else {
        if (epi == EPI_PLAIN) MSB_DS(EPI_PLAIN, false);
        else if (epi == EPI_MV) MSB_DS(EPI_MV, false);
        else if (epi == EPI_SV) MSB_DS(EPI_SV, false);
        else MSB_DS(EPI_MV_Y, false);
    }
#undef MSB_DS
}

template void launch_dslash<double>(hipStream_t, DslashArgs<double>, int, int, bool);

void launch_link_force(hipStream_t st, const LinkForceArgs &a) {
    const int nb = nblocks_for(a.g.V);
    hipLaunchKernelGGL(link_force_kernel, dim3(nb), dim3(BLOCK), 0, st, a);
}
template void launch_dslash<float>(hipStream_t, DslashArgs<float>, int, int, bool);

}  // namespace msb
