// Device body of the Wilson-Dirac stencil D_w(mu) (see dslash.hip for the
// operator and the epilogues).  Shared by the one-launch-per-stage kernels and
// by the persistent kernel, which calls dslash_body for each of its virtual
// blocks.
#pragma once
#include "common.h"
#include "kernels.h"

namespace msb {
namespace dev {

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

// acc += f * [(1 + SGN gamma_NU) reconstruction of] Umat h for a projected
// half-spinor h (h0, h1); Umat = U (DAG=false) or U^+ (DAG=true), where entry
// (a, b) of U is Ub[(3 a + b) us]: the link in global memory (us = V) or
// staged in LDS (us = CHUNK).
template <typename T, int NU, int SGN, bool DAG>
__device__ __forceinline__ void hop_h(C<T> (&acc)[4][3], const C<T> (&h)[2][3], const C<T> *__restrict__ Ub, int us,
                                      T f) {
    using P = Proj<NU, SGN>;
    C<T> g[2][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        C<T> u0, u1, u2;
        if (!DAG) {
            u0 = Ub[(3 * a + 0) * us];
            u1 = Ub[(3 * a + 1) * us];
            u2 = Ub[(3 * a + 2) * us];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                C<T> r = cmul(u0, h[i][0]);
                r = cfma(u1, h[i][1], r);
                r = cfma(u2, h[i][2], r);
                g[i][a] = r;
            }
        } else {
            // (U^+)_{ab} = conj(U_{ba})
            u0 = Ub[(0 * 3 + a) * us];
            u1 = Ub[(1 * 3 + a) * us];
            u2 = Ub[(2 * 3 + a) * us];
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

// acc += f * (1 + SGN gamma_NU) Umat psi(sn), psi loaded here (one spin at a
// time; used by the persistent kernel's stencil).
template <typename T, int NU, int SGN, bool DAG, bool G5IN>
__device__ __forceinline__ void hop(C<T> (&acc)[4][3], const C<T> *__restrict__ in,
                                   const C<T> *__restrict__ Ub, int us, int V, int sn, T f) {
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
    hop_h<T, NU, SGN, DAG>(acc, h, Ub, us, f);
}

// Element k (= 3 spin + colour) of site s: base in + k V is the same for the
// whole wavefront and the site offset is a 32-bit unsigned index, so each
// component load takes a scalar base and one vector offset per site.
template <typename E>
__device__ __forceinline__ E &elem(E *__restrict__ p, int k, int V, int s) {
    return (p + (size_t)k * (unsigned)V)[(unsigned)s];
}
// UB = false: the plain signed index k V + s (the site-block kernel's form,
// which the compiler schedules in fewer registers there)
template <bool UB, typename E>
__device__ __forceinline__ E &elem_at(E *__restrict__ p, int k, int V, int s) {
    if constexpr (UB) return elem(p, k, V, s);
    else return p[k * V + s];
}

// An operand read once per sweep (v, w, r~, y): with UB (the chunked form) streamed
// past L2, like the output, so that it does not evict neighbour spinors.
template <bool UB, typename E>
__device__ __forceinline__ E ld_stream(const E *__restrict__ p, int k, int V, int s) {
    if constexpr (UB) {
        const E &q = elem(p, k, V, s);
        E r;
        r.x = __builtin_nontemporal_load(&q.x);
        r.y = __builtin_nontemporal_load(&q.y);
        return r;
    } else {
        return p[k * V + s];
    }
}

// The 12 components of psi(s) ([gamma5] applied: lower spins negated).
template <typename T, bool G5IN>
__device__ __forceinline__ void load_site(const C<T> *__restrict__ in, int V, int s, C<T> (&b)[12]) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        C<T> z = elem(in, k, V, s);
        if (G5IN && k >= 6) z = cneg(z);
        b[k] = z;
    }
}

// h = the two independent spins of (1 + SGN gamma_NU) psi
template <typename T, int NU, int SGN>
__device__ __forceinline__ void project(const C<T> (&b)[12], C<T> (&h)[2][3]) {
    using P = Proj<NU, SGN>;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        h[0][a] = cadd(b[a], mulcode<P::C0>(b[3 * P::P0 + a]));
        h[1][a] = cadd(b[3 + a], mulcode<P::C1>(b[3 * P::P1 + a]));
    }
}

// Where a hop finds its link: in global memory ([4][3][3][V], entry stride V)
// or staged in LDS for a 64-site chunk ([8 hops][9][CHUNK], stride CHUNK).
template <typename T>
struct GlobalLinks {
    static constexpr bool staged = false;
    const C<T> *U;
    int V;
    __device__ __forceinline__ const C<T> *at(int nu, int bwd, int sl, int) const {
        (void)bwd;
        return U + (size_t)nu * 9 * V + sl;
    }
    __device__ __forceinline__ int stride() const { return V; }
};
template <typename T>
struct LdsLinks {
    static constexpr bool staged = true;
    const C<T> *L;
    int base;   // first site of the chunk
    __device__ __forceinline__ const C<T> *at(int nu, int bwd, int, int s) const {
        return L + (2 * nu + bwd) * 9 * CHUNK + (s - base);
    }
    __device__ __forceinline__ int stride() const { return CHUNK; }
};

// Lx = 16 in the chunked form: the 16 lanes of each row of a wavefront hold
// one periodic x-line, so a site's x-neighbour values are in the lanes next
// to it.  x_rotate replaces each lane's half spinor with that of lane
// (i + 1) mod 16 (FWD) or (i - 1) mod 16 of its row (DPP row rotate), which
// is bitwise the projection the lane would have formed from the neighbour's
// loaded spinor, without its twelve loads.
template <bool FWD>
__device__ __forceinline__ int row_rot(int v) {
    return __builtin_amdgcn_update_dpp(0, v, FWD ? 0x12F : 0x121, 0xF, 0xF, false);
}
__device__ __forceinline__ double row_rot_d(double v, bool fwd) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return fwd ? __hiloint2double(row_rot<true>(hi), row_rot<true>(lo))
               : __hiloint2double(row_rot<false>(hi), row_rot<false>(lo));
}
__device__ __forceinline__ float row_rot_d(float v, bool fwd) {
    return __int_as_float(fwd ? row_rot<true>(__float_as_int(v)) : row_rot<false>(__float_as_int(v)));
}
template <typename T, bool FWD>
__device__ __forceinline__ void x_rotate(C<T> (&h)[2][3]) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) h[i][c] = mk<T>(row_rot_d(h[i][c].x, FWD), row_rot_d(h[i][c].y, FWD));
}

// Order of the hop sum, chosen by the parity of z + t at the first site of
// the site's aligned 64-site group (order_parity below).  Even
// sites start from the diagonal term, -2 (4+m) psi(x), add the hops x-, x+,
// y-, y+, z-, z+, t-, t+ and scale the sum by -scale/2; odd sites add z-, z+,
// t-, t+, x-, x+, y-, y+ and form scale ((4+m) psi(x) - sum/2) at the end.
// A chunk's spinors are read by the chunk itself (its x and y hops and its
// centre) and by the z and t neighbour chunks, which have the other parity:
// an even chunk reads its own data first and then its neighbours', an odd
// chunk its neighbours' first and then its own, so co-resident chunks that
// sweep a right-hand side together read each line within a short stretch of
// the sweep, while it is still in the XCD's L2.  Every stencil form uses the
// same per-site order, so all of them give the same bits.

// The parity that picks a site's order: that of z + t at the first site of
// its aligned 64-site group.  Every form runs its wavefronts over such groups
// (chunks, and the four wavefronts of a 256-site block), so the choice is
// uniform over a wavefront and the branch on it is a scalar one: a per-lane
// choice made the waves that straddle a z-t plane (Lx Ly not a multiple of
// 64) run both orders.  Where Lx Ly is a multiple of 64 this is the site's
// own parity.
__device__ __forceinline__ int order_parity(const Geom &g, int s) {
    const int zt = (s & ~63) / (g.Lx * g.Ly);
    return __builtin_amdgcn_readfirstlane((zt % g.Lz + zt / g.Lz) & 1);
}

// m2d = -2 (4+m): acc = m2d psi(x).  No multiply-add may absorb this product
// (the forms must round it alike wherever it is inlined).
template <typename T>
__device__ __forceinline__ void diag_start_spin(C<T> (&acc)[3], const C<T> (&b)[3], T m2d) {
#pragma clang fp contract(off)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] = mk<T>(b[c].x * m2d, b[c].y * m2d);
}
template <typename T>
__device__ __forceinline__ void diag_start(C<T> (&acc)[4][3], const C<T> (&b)[12], T m2d) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) {
        const C<T> bs[3] = {b[3 * sp], b[3 * sp + 1], b[3 * sp + 2]};
        diag_start_spin<T>(acc[sp], bs, m2d);
    }
}
// even sites: out = (-scale/2 [gamma5]) acc
template <typename T>
__device__ __forceinline__ void even_finish(C<T> (&acc)[4][3], T scale, int g5out) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) {
        const T f = ((g5out && sp >= 2) ? (T)0.5 : (T)-0.5) * scale;
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[sp][c] = cscale(acc[sp][c], f);
    }
}
// odd sites: out = scale [gamma5] ((4+m) psi(x) - acc / 2)
template <typename T>
__device__ __forceinline__ void odd_finish_spin(C<T> (&acc)[3], const C<T> (&b)[3], T diag, T sg) {
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] = cscale(csub(cscale(b[c], diag), cscale(acc[c], (T)0.5)), sg);
}
template <typename T>
__device__ __forceinline__ void odd_finish(C<T> (&acc)[4][3], const C<T> (&b)[12], T diag, T scale, int g5out) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) {
        const C<T> bs[3] = {b[3 * sp], b[3 * sp + 1], b[3 * sp + 2]};
        odd_finish_spin<T>(acc[sp], bs, diag, ((g5out && sp >= 2) ? (T)-1 : (T)1) * scale);
    }
}

// The Wilson operator at site s with the links read from global memory
// ([4][3][3][V]; the site-block and persistent forms): one hop at a time,
// since two gather buffers would cost the site-block kernel an occupancy
// step.  Leaves scale [gamma5] D [gamma5] psi(s) in acc.
template <typename T, bool G5IN>
__device__ __forceinline__ void wilson_site_global(const DslashArgs<T> &a, const C<T> *__restrict__ U,
                                                   const C<T> *__restrict__ in, int s, C<T> (&acc)[4][3]) {
    const int V = a.g.V, Lx = a.g.Lx, Ly = a.g.Ly, Lz = a.g.Lz, Lt = a.g.Lt;
    const int sxy = Lx * Ly, sxyz = Lx * Ly * Lz;
    const int x = s % Lx;
    const int r1 = s / Lx;
    const int yy = r1 % Ly;
    const int r2 = r1 / Ly;
    const int z = r2 % Lz;
    const int t = r2 / Lz;
    const T ff = (t == Lt - 1) ? a.ef * a.bc : a.ef;
    const T fb = (t == 0) ? a.eb * a.bc : a.eb;
    auto hx = [&]() __attribute__((always_inline)) {
        const int sf = (x == Lx - 1) ? s - (Lx - 1) : s + 1;
        const int sb = (x == 0) ? s + (Lx - 1) : s - 1;
        hop<T, 0, -1, false, G5IN>(acc, in, U + s, V, V, sf, (T)1);
        hop<T, 0, +1, true, G5IN>(acc, in, U + sb, V, V, sb, (T)1);
    };
    auto hy = [&]() __attribute__((always_inline)) {
        const int sf = (yy == Ly - 1) ? s - (Ly - 1) * Lx : s + Lx;
        const int sb = (yy == 0) ? s + (Ly - 1) * Lx : s - Lx;
        hop<T, 1, -1, false, G5IN>(acc, in, U + (size_t)9 * V + s, V, V, sf, (T)1);
        hop<T, 1, +1, true, G5IN>(acc, in, U + (size_t)9 * V + sb, V, V, sb, (T)1);
    };
    auto hz = [&]() __attribute__((always_inline)) {
        const int sf = (z == Lz - 1) ? s - (Lz - 1) * sxy : s + sxy;
        const int sb = (z == 0) ? s + (Lz - 1) * sxy : s - sxy;
        hop<T, 2, -1, false, G5IN>(acc, in, U + (size_t)18 * V + s, V, V, sf, (T)1);
        hop<T, 2, +1, true, G5IN>(acc, in, U + (size_t)18 * V + sb, V, V, sb, (T)1);
    };
    auto ht = [&]() __attribute__((always_inline)) {
        const int sf = (t == Lt - 1) ? s - (Lt - 1) * sxyz : s + sxyz;
        const int sb = (t == 0) ? s + (Lt - 1) * sxyz : s - sxyz;
        hop<T, 3, -1, false, G5IN>(acc, in, U + (size_t)27 * V + s, V, V, sf, ff);
        hop<T, 3, +1, true, G5IN>(acc, in, U + (size_t)27 * V + sb, V, V, sb, fb);
    };
    C<T> b[12];
    if (order_parity(a.g, s)) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[i][c] = mk<T>(0, 0);
        hz(); ht(); hx(); hy();
        load_site<T, G5IN>(in, V, s, b);
        odd_finish<T>(acc, b, a.diag, a.scale, a.g5out);
    } else {
        load_site<T, G5IN>(in, V, s, b);
        diag_start<T>(acc, b, (T)-2 * a.diag);
        hx(); hy(); hz(); ht();
        even_finish<T>(acc, a.scale, a.g5out);
    }
}

// The stencil and its epilogue for sites s0, s0 + sstride, ... < V of one
// right-hand side.  sstride exceeds V, so the loop body runs at most once;
// keeping it a loop with a run-time bound (and every address derived from s)
// stops the compiler from hoisting loads out of the caller's loop over
// right-hand sides.  With links in LDS the neighbours are gathered two hops
// ahead: while hop k is multiplied, the spinors of hops k + 1 and k + 2 are
// in flight (two 12-component buffers), in the parity order above.
template <typename T, int EPI, bool G5IN, typename LK>
__device__ __forceinline__ void dslash_sites(const DslashArgs<T> &a, const LK &lk, const C<T> *__restrict__ in,
                                             C<T> *__restrict__ out, const C<T> *__restrict__ v,
                                             const C<T> *__restrict__ rt, double2 *__restrict__ y, C<T> yc,
                                             T sig0, const C<T> *__restrict__ wsub,
                                             int s0, double (&part)[3]) {
    const int V = a.g.V;
    for (int s = s0; s < V; s += a.sstride) {
    C<T> acc[4][3];
    if constexpr (!LK::staged) {
        wilson_site_global<T, G5IN>(a, lk.U, in, s, acc);
    } else {
    const int Lx = a.g.Lx, Ly = a.g.Ly, Lz = a.g.Lz, Lt = a.g.Lt;
    const int sxy = Lx * Ly, sxyz = Lx * Ly * Lz;
    const int x = s % Lx;
    const int r1 = s / Lx;
    const int yy = r1 % Ly;
    const int r2 = r1 / Ly;
    const int z = r2 % Lz;
    const int t = r2 / Lz;
    const int us = lk.stride();
    const T ff = (t == Lt - 1) ? a.ef * a.bc : a.ef;
    const T fb = (t == 0) ? a.eb * a.bc : a.eb;
    const int xf = (x == Lx - 1) ? s - (Lx - 1) : s + 1;
    const int xb = (x == 0) ? s + (Lx - 1) : s - 1;
    const int yf = (yy == Ly - 1) ? s - (Ly - 1) * Lx : s + Lx;
    const int yb = (yy == 0) ? s + (Ly - 1) * Lx : s - Lx;
    const int zf = (z == Lz - 1) ? s - (Lz - 1) * sxy : s + sxy;
    const int zb = (z == 0) ? s + (Lz - 1) * sxy : s - sxy;
    const int tf = (t == Lt - 1) ? s - (Lt - 1) * sxyz : s + sxyz;
    const int tb = (t == 0) ? s + (Lt - 1) * sxyz : s - sxyz;
    C<T> bA[12], bB[12], h[2][3];
    if (order_parity(a.g, s) && Lx == 16) {
        // odd, x from the neighbouring lanes: z, t, x, y, the centre loaded
        // during the t hops and kept for the diagonal term
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[i][c] = mk<T>(0, 0);
        load_site<T, G5IN>(in, V, zf, bA);
        load_site<T, G5IN>(in, V, zb, bB);
        project<T, 2, -1>(bA, h);
        load_site<T, G5IN>(in, V, tf, bA);
        hop_h<T, 2, -1, false>(acc, h, lk.at(2, 0, s, s), us, (T)1);
        project<T, 2, +1>(bB, h);
        load_site<T, G5IN>(in, V, tb, bB);
        hop_h<T, 2, +1, true>(acc, h, lk.at(2, 1, zb, s), us, (T)1);
        project<T, 3, -1>(bA, h);
        load_site<T, G5IN>(in, V, s, bA);    // the centre
        hop_h<T, 3, -1, false>(acc, h, lk.at(3, 0, s, s), us, ff);
        project<T, 3, +1>(bB, h);
        load_site<T, G5IN>(in, V, yf, bB);
        hop_h<T, 3, +1, true>(acc, h, lk.at(3, 1, tb, s), us, fb);
        project<T, 0, -1>(bA, h);
        x_rotate<T, true>(h);
        hop_h<T, 0, -1, false>(acc, h, lk.at(0, 0, s, s), us, (T)1);
        project<T, 0, +1>(bA, h);
        x_rotate<T, false>(h);
        hop_h<T, 0, +1, true>(acc, h, lk.at(0, 1, xb, s), us, (T)1);
        project<T, 1, -1>(bB, h);
        load_site<T, G5IN>(in, V, yb, bB);
        hop_h<T, 1, -1, false>(acc, h, lk.at(1, 0, s, s), us, (T)1);
        project<T, 1, +1>(bB, h);
        hop_h<T, 1, +1, true>(acc, h, lk.at(1, 1, yb, s), us, (T)1);
        odd_finish<T>(acc, bA, a.diag, a.scale, a.g5out);
    } else if (order_parity(a.g, s)) {
        // odd: z, t, x, y, then the centre
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[i][c] = mk<T>(0, 0);
        load_site<T, G5IN>(in, V, zf, bA);
        load_site<T, G5IN>(in, V, zb, bB);
        project<T, 2, -1>(bA, h);
        load_site<T, G5IN>(in, V, tf, bA);
        hop_h<T, 2, -1, false>(acc, h, lk.at(2, 0, s, s), us, (T)1);
        project<T, 2, +1>(bB, h);
        load_site<T, G5IN>(in, V, tb, bB);
        hop_h<T, 2, +1, true>(acc, h, lk.at(2, 1, zb, s), us, (T)1);
        project<T, 3, -1>(bA, h);
        load_site<T, G5IN>(in, V, xf, bA);
        hop_h<T, 3, -1, false>(acc, h, lk.at(3, 0, s, s), us, ff);
        project<T, 3, +1>(bB, h);
        load_site<T, G5IN>(in, V, xb, bB);
        hop_h<T, 3, +1, true>(acc, h, lk.at(3, 1, tb, s), us, fb);
        project<T, 0, -1>(bA, h);
        load_site<T, G5IN>(in, V, yf, bA);
        hop_h<T, 0, -1, false>(acc, h, lk.at(0, 0, s, s), us, (T)1);
        project<T, 0, +1>(bB, h);
        load_site<T, G5IN>(in, V, yb, bB);
        hop_h<T, 0, +1, true>(acc, h, lk.at(0, 1, xb, s), us, (T)1);
        project<T, 1, -1>(bA, h);
        load_site<T, G5IN>(in, V, s, bA);    // the centre, for the diagonal term
        hop_h<T, 1, -1, false>(acc, h, lk.at(1, 0, s, s), us, (T)1);
        project<T, 1, +1>(bB, h);
        hop_h<T, 1, +1, true>(acc, h, lk.at(1, 1, yb, s), us, (T)1);
        odd_finish<T>(acc, bA, a.diag, a.scale, a.g5out);
    } else {
        // even: the centre, x, y, z, t
        if (Lx == 16) {
            // x from the neighbouring lanes (the centre's projections)
            load_site<T, G5IN>(in, V, s, bB);
            load_site<T, G5IN>(in, V, yf, bA);
            diag_start<T>(acc, bB, (T)-2 * a.diag);
            project<T, 0, -1>(bB, h);
            x_rotate<T, true>(h);
            hop_h<T, 0, -1, false>(acc, h, lk.at(0, 0, s, s), us, (T)1);
            project<T, 0, +1>(bB, h);
            load_site<T, G5IN>(in, V, yb, bB);
            x_rotate<T, false>(h);
            hop_h<T, 0, +1, true>(acc, h, lk.at(0, 1, xb, s), us, (T)1);
        } else {
            C<T> cc[12];
            load_site<T, G5IN>(in, V, s, cc);
            load_site<T, G5IN>(in, V, xf, bA);
            load_site<T, G5IN>(in, V, xb, bB);
            diag_start<T>(acc, cc, (T)-2 * a.diag);
            project<T, 0, -1>(bA, h);
            load_site<T, G5IN>(in, V, yf, bA);
            hop_h<T, 0, -1, false>(acc, h, lk.at(0, 0, s, s), us, (T)1);
            project<T, 0, +1>(bB, h);
            load_site<T, G5IN>(in, V, yb, bB);
            hop_h<T, 0, +1, true>(acc, h, lk.at(0, 1, xb, s), us, (T)1);
        }
        project<T, 1, -1>(bA, h);
        load_site<T, G5IN>(in, V, zf, bA);
        hop_h<T, 1, -1, false>(acc, h, lk.at(1, 0, s, s), us, (T)1);
        project<T, 1, +1>(bB, h);
        load_site<T, G5IN>(in, V, zb, bB);
        hop_h<T, 1, +1, true>(acc, h, lk.at(1, 1, yb, s), us, (T)1);
        project<T, 2, -1>(bA, h);
        load_site<T, G5IN>(in, V, tf, bA);
        hop_h<T, 2, -1, false>(acc, h, lk.at(2, 0, s, s), us, (T)1);
        project<T, 2, +1>(bB, h);
        load_site<T, G5IN>(in, V, tb, bB);
        hop_h<T, 2, +1, true>(acc, h, lk.at(2, 1, zb, s), us, (T)1);
        project<T, 3, -1>(bA, h);
        hop_h<T, 3, -1, false>(acc, h, lk.at(3, 0, s, s), us, ff);
        project<T, 3, +1>(bB, h);
        hop_h<T, 3, +1, true>(acc, h, lk.at(3, 1, tb, s), us, fb);
        even_finish<T>(acc, a.scale, a.g5out);
    }
    }
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int k = 3 * sp + c;
            C<T> o = acc[sp][c];
            if (EPI != EPI_PLAIN) o = cadd(o, cscale(ld_stream<LK::staged>(v, k, V, s), sig0));
            if (EPI == EPI_SV2) o = csub(o, ld_stream<LK::staged>(wsub, k, V, s));
            if constexpr (LK::staged) {
                // streamed past L2: the output is not read again by this
                // sweep, and its lines would evict neighbour spinors
                C<T> &d = elem_at<true>(out, k, V, s);
                __builtin_nontemporal_store(o.x, &d.x);
                __builtin_nontemporal_store(o.y, &d.y);
            } else {
                elem_at<false>(out, k, V, s) = o;
            }
            if (EPI == EPI_MV) {
                const C<T> r = ld_stream<LK::staged>(rt, k, V, s);
                part[0] += (double)r.x * o.x + (double)r.y * o.y;
                part[1] += (double)r.x * o.y - (double)r.y * o.x;
            }
            // EPI_MVN: no r~ here, its dot comes from a sparse list
            if (epi_dots(EPI)) part[2] += (double)o.x * o.x + (double)o.y * o.y;
            if (EPI == EPI_MV_Y) {
                double2 &yr = elem_at<LK::staged>(y, k, V, s);
                double2 yv = ld_stream<LK::staged>(y, k, V, s);
                yv.x += (double)yc.x * o.x - (double)yc.y * o.y;
                yv.y += (double)yc.x * o.y + (double)yc.y * o.x;
                if constexpr (LK::staged) {
                    __builtin_nontemporal_store(yv.x, &yr.x);
                    __builtin_nontemporal_store(yv.y, &yr.y);
                } else {
                    yr = yv;
                }
            }
        }
    }
    }
}

// Operand pointers of right-hand side rhs.
template <typename T>
struct RhsOps {
    const C<T> *in;
    C<T> *out;
    const C<T> *v, *rt;
    double2 *y;
    C<T> yc;
    T sig0;
    const C<T> *w;
};
template <typename T, int EPI>
__device__ __forceinline__ RhsOps<T> rhs_ops(const DslashArgs<T> &a, int rhs) {
    const long nv = 12L * a.g.V;
    RhsOps<T> o;
    o.in = a.in + (size_t)rhs * (a.in_rs ? a.in_rs : nv);
    o.out = a.out + (size_t)rhs * (a.out_rs ? a.out_rs : nv);
    o.v = a.v ? a.v + (size_t)rhs * (a.v_rs ? a.v_rs : nv) : nullptr;
    o.rt = a.rt ? a.rt + (size_t)rhs * (a.rt_rs ? a.rt_rs : nv) : nullptr;
    o.y = a.y ? a.y + (size_t)rhs * (a.y_rs ? a.y_rs : nv) : nullptr;
    o.yc = mk<T>(0, 0);
    if (EPI == EPI_MV_Y) o.yc = to_c<T>(ld(a.ycoef, rhs));
    o.sig0 = a.sigma0_rhs ? (T)a.sigma0_rhs[rhs] : a.sigma0;
    o.w = a.w ? a.w + (size_t)rhs * (a.w_rs ? a.w_rs : nv) : nullptr;
    return o;
}

// Site-block stencil: one block per (256-site block, right-hand side), links
// read from global memory.  Partials: one per 64-site chunk (wavefront).
template <typename T, int EPI, bool G5IN>
__device__ __forceinline__ void dslash_site_block(const DslashArgs<T> &a, int sblk, int rhs) {
    if (!gate_open(a.gate, rhs)) return;
    const RhsOps<T> o = rhs_ops<T, EPI>(a, rhs);
    const GlobalLinks<T> lk{a.U, a.g.V};
    double part[3] = {0.0, 0.0, 0.0};
    dslash_sites<T, EPI, G5IN>(a, lk, o.in, o.out, o.v, o.rt, o.y, o.yc, o.sig0, o.w, sblk * BLOCK + threadIdx.x,
                              part);
    if (epi_dots(EPI))
        wave_reduce_store<3>(part, a.part + (size_t)rhs * PMAX * a.ps + sblk * (BLOCK / 64) + (threadIdx.x >> 6),
                             a.ps);
}

// Block p of the flattened grid (8 per blocks) to (site block, rhs): hardware
// block p runs on XCD p % 8, which owns the contiguous logical range
// [(p % 8) per, (p % 8 + 1) per); inside it the right-hand side varies
// fastest, so the sources of one site block run back to back on one XCD.
template <typename T, int EPI, bool G5IN>
__device__ __forceinline__ void dslash_body(const DslashArgs<T> &a, int p) {
    const int L = (p & 7) * a.per + (p >> 3);
    if (L >= a.nsb * a.nrhs) return;
    const int sblk = L / a.nrhs;
    dslash_site_block<T, EPI, G5IN>(a, sblk, L - sblk * a.nrhs);
}

// Chunked stencil for batches: one block of NW wavefronts per 64-site chunk.
// The block first stages the chunk's eight links per site (forward U_nu(x)
// and backward U_nu(x - nu)) in LDS, then its wavefronts take the right-hand
// sides in turn, one site per lane, reading the links from LDS: the links
// cross the memory fabric once per chunk instead of once per right-hand side
// (which is what bounded the site-block stencil on batches).  Chunks are
// dealt XCD-aware: XCD p % 8 owns a contiguous slab of chunks, walked with
// the time coordinate varying fastest so that the t -/+ 1 neighbour planes
// were read moments earlier by the same XCD.  Arithmetic, per site and per
// partial, is the site-block stencil's, bit for bit.
template <typename T, int EPI, bool G5IN, int NW>
__device__ __forceinline__ void dslash_chunk(const DslashArgs<T> &a, int p) {
    __shared__ C<T> Ls[8 * 9 * CHUNK];
    const int x8 = p & 7, i = p >> 3;
    const int s0 = x8 * a.per;
    int n = a.nch - s0;
    if (n > a.per) n = a.per;
    int c = i;
    if (a.tsc) {
        const int ntl = a.per_t / a.tsc;
        const int zc = i / ntl;
        c = (i - zc * ntl) * a.tsc + zc;
    }
    if (c >= n) return;
    const int chunk = s0 + c;
    const int V = a.g.V, Lx = a.g.Lx, Ly = a.g.Ly, Lz = a.g.Lz, Lt = a.g.Lt;
    const int base = chunk * CHUNK;
    for (int idx = threadIdx.x; idx < 8 * 9 * CHUNK; idx += 64 * NW) {
        const int hp = idx / (9 * CHUNK), e = (idx / CHUNK) % 9;
        const int s = base + idx % CHUNK;
        C<T> u = mk<T>(0, 0);
        if (s < V) {
            const int nu = hp >> 1;
            int sl = s;
            if (hp & 1) {
                const int x = s % Lx, q1 = s / Lx, yy = q1 % Ly, q2 = q1 / Ly, z = q2 % Lz, t = q2 / Lz;
                if (nu == 0) sl = (x == 0) ? s + (Lx - 1) : s - 1;
                else if (nu == 1) sl = (yy == 0) ? s + (Ly - 1) * Lx : s - Lx;
                else if (nu == 2) sl = (z == 0) ? s + (Lz - 1) * Lx * Ly : s - Lx * Ly;
                else sl = (t == 0) ? s + (Lt - 1) * Lx * Ly * Lz : s - Lx * Ly * Lz;
            }
            u = a.U[((size_t)nu * 9 + e) * V + sl];
        }
        Ls[idx] = u;
    }
    __syncthreads();
    const LdsLinks<T> lk{Ls, base};
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    for (int rhs = w; rhs < a.nrhs; rhs += NW) {
        if (!gate_open(a.gate, rhs)) continue;
        const RhsOps<T> o = rhs_ops<T, EPI>(a, rhs);
        double part[3] = {0.0, 0.0, 0.0};
        dslash_sites<T, EPI, G5IN>(a, lk, o.in, o.out, o.v, o.rt, o.y, o.yc, o.sig0, o.w, base + lane, part);
        if (epi_dots(EPI)) wave_reduce_store<3>(part, a.part + (size_t)rhs * PMAX * a.ps + chunk, a.ps);
    }
}

}  // namespace dev
}  // namespace msb
