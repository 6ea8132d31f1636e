// Internal definitions shared by the HIP sources of libmsb.
//
// Complex numbers are interleaved (re, im) pairs: double2 in FP64, float2 in
// FP32.  Spinors are stored [rhs][k = 3*spin + colour][site] so that a
// wavefront touching 64 consecutive sites issues one coalesced 64 x 16 B (or
// 64 x 8 B) access per component; links are [nu][a][b][site].
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

namespace msb {

constexpr int LMAX = 8;          // largest MR degree l
constexpr int NSMAX = 64;        // largest number of shifts per right-hand side
constexpr int BLOCK = 256;       // threads per block of every vector kernel
constexpr int NBMAX = 2048;      // largest number of blocks per RHS in a reduction
constexpr int GRAM_NBMAX = 512;  // blocks per RHS of the MR Gram matrix pass
constexpr int PMAX = 2 * (LMAX + 1) * (LMAX + 2) / 2;  // doubles per partial row
constexpr double BREAK_REL = 1e-14;
constexpr double CHOL_REL = 1e-14;
constexpr double ZETA_MIN = 1e-300;
// a shift freezes once its recursive residual estimate is at most
// FREEZE_FRAC tol: the rounding drift between the recursive and the true
// residual (about 1e-15 relative in FP64) then cannot lift the true residual
// above tol
constexpr double FREEZE_FRAC = 0.9;
// a shift whose |zeta psi| would exceed this has a residual estimate
// ||r_0|| / (|zeta psi| ||b||) below any tolerance (for ||r_0|| within 1e20 of
// ||b||) and 1 / (zeta psi) would underflow: it stops there as converged
constexpr double ZETA_MAX = 1e300;

enum Status { S_OK = 0, S_ERR_ARG = 1, S_ERR_HIP = 2, S_ERR_OOM = 3,
              S_NOT_CONVERGED = 4, S_BREAKDOWN = 5 };

template <typename T> struct cx;
template <> struct cx<double> { using t = double2; };
template <> struct cx<float> { using t = float2; };
template <typename T> using C = typename cx<T>::t;

template <typename T> __host__ __device__ inline C<T> mk(T re, T im) { C<T> z; z.x = re; z.y = im; return z; }

// complex helpers (templated on the complex type directly)
template <typename Z> __host__ __device__ inline Z cadd(Z a, Z b) { Z r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename Z> __host__ __device__ inline Z csub(Z a, Z b) { Z r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename Z> __host__ __device__ inline Z cmul(Z a, Z b) {
    Z r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
// conj(a) * b
template <typename Z> __host__ __device__ inline Z cmulc(Z a, Z b) {
    Z r; r.x = a.x * b.x + a.y * b.y; r.y = a.x * b.y - a.y * b.x; return r;
}
template <typename Z, typename R> __host__ __device__ inline Z cscale(Z a, R s) { Z r; r.x = a.x * s; r.y = a.y * s; return r; }
template <typename Z> __host__ __device__ inline Z ctimes_i(Z a) { Z r; r.x = -a.y; r.y = a.x; return r; }
template <typename Z> __host__ __device__ inline Z ctimes_mi(Z a) { Z r; r.x = a.y; r.y = -a.x; return r; }
template <typename Z> __host__ __device__ inline Z cneg(Z a) { Z r; r.x = -a.x; r.y = -a.y; return r; }
template <typename Z> __host__ __device__ inline Z cconj(Z a) { Z r; r.x = a.x; r.y = -a.y; return r; }
// a + s * b   (s complex)
template <typename Z> __host__ __device__ inline Z cfma(Z s, Z b, Z a) {
    Z r; r.x = a.x + s.x * b.x - s.y * b.y; r.y = a.y + s.x * b.y + s.y * b.x; return r;
}
__host__ __device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline double cabsd(double2 a) { return sqrt(a.x * a.x + a.y * a.y); }
// modulus without intermediate overflow or underflow (the shifts' zeta and
// psi range far beyond 1e+-154)
__host__ __device__ inline double cmod(double2 a) { return hypot(a.x, a.y); }
__host__ __device__ inline double2 cdiv(double2 a, double2 b) {
    // Smith's algorithm: scale by the larger component of b
    double2 r;
    if (fabs(b.x) >= fabs(b.y)) {
        double t = b.y / b.x, d = b.x + b.y * t;
        r.x = (a.x + a.y * t) / d;
        r.y = (a.y - a.x * t) / d;
    } else {
        double t = b.x / b.y, d = b.x * t + b.y;
        r.x = (a.x * t + a.y) / d;
        r.y = (a.y * t - a.x) / d;
    }
    return r;
}
__host__ __device__ inline double2 d2(double re, double im) { double2 z; z.x = re; z.y = im; return z; }
__host__ __device__ inline bool cfinite(double2 a) { return isfinite(a.x) && isfinite(a.y); }

template <typename T> __device__ inline C<T> to_c(double2 z) { return mk<T>((T)z.x, (T)z.y); }

// ---------------------------------------------------------------------------
// Deterministic block reduction (BLOCK = 256 threads = 4 wavefronts of 64).
// Values are reduced by a fixed shuffle tree inside each wavefront, then the
// four wavefront sums are added in order.  Thread k < NV writes value k to
// out[k * stride].
// ---------------------------------------------------------------------------
template <int NV>
__device__ inline void block_reduce_store(double (&v)[NV], double *out, int stride) {
    __shared__ double sh[NV][BLOCK / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();   // a block may call this back to back (persistent stages)
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        if (lane == 0) sh[k][wave] = x;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < NV; k += BLOCK) {
        double s = sh[k][0];
#pragma unroll
        for (int w = 1; w < BLOCK / 64; ++w) s += sh[k][w];
        out[(size_t)k * stride] = s;
    }
}

// Reduce NV doubles over the 64 lanes of a wavefront (fixed shuffle tree, so
// the same data always gives the same bits) and store them from lane 0 at
// out[k * stride].
template <int NV>
__device__ inline void wave_reduce_store(double (&v)[NV], double *out, long stride) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        if (lane == 0) out[(size_t)k * stride] = x;
    }
}

// Loads per row that the block sums below issue before their first add.  The
// partials they read usually come from another XCD's writes, so each load is
// a trip to memory, and one trip per add would serialise them.  A translation
// unit may lower it before including this header (the persistent kernel,
// whose register budget is the maximum over all its stages, sets 1); the
// sums are the same bits for any value.
#ifndef MSB_SUM_PREFETCH
#define MSB_SUM_PREFETCH 8
#endif

// Sum of p[0..n) by all BLOCK threads of one block, returned to every thread.
// Each thread adds p[t], p[t + BLOCK], ... in that order; a group of loads
// that runs past n adds +0.0 in their place, which leaves the sum's bits
// alone (the sum starts at +0.0 and round-to-nearest never makes it -0.0).
__device__ inline double block_sum(const double *p, int n) {
    __shared__ double sh[BLOCK / 64];
    __shared__ double result;
    constexpr int U = MSB_SUM_PREFETCH;
    double x = 0.0;
    for (int i = threadIdx.x; i < n; i += U * BLOCK) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = i + u * BLOCK < n ? p[i + u * BLOCK] : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) x += v[u];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    __syncthreads();
    if (lane == 0) sh[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = sh[0];
        for (int w = 1; w < BLOCK / 64; ++w) s += sh[w];
        result = s;
    }
    __syncthreads();
    return result;
}

// Up to NR sums at once: out[r] = the sum of p[rows[r] * stride + i] for
// i < n (r < cnt), returned to every thread.  Each row is added in exactly
// block_sum's order (per-thread strided partial sums, the same shuffle tree,
// the four wavefront sums in order), so the results are bitwise block_sum's;
// the rows share one pass over the block instead of one pass each.
template <int NR>
__device__ inline void block_sum_rows(const double *p, long stride, const int *rows, int cnt, int n,
                                      double (&out)[NR]) {
    __shared__ double sh[NR][BLOCK / 64];
    __shared__ double res[NR];
    constexpr int U = NR <= 4 ? MSB_SUM_PREFETCH : (MSB_SUM_PREFETCH + 1) / 2;   // loads per row in flight
    double x[NR];
    const double *pr[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        x[r] = 0.0;
        pr[r] = p + (size_t)rows[r < cnt ? r : 0] * stride;
    }
    for (int i = threadIdx.x; i < n; i += U * BLOCK) {
        double v[NR][U];
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int u = 0; u < U; ++u) v[r][u] = (r < cnt && i + u * BLOCK < n) ? pr[r][i + u * BLOCK] : 0.0;
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int u = 0; u < U; ++u) x[r] += v[r][u];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x[r] += __shfl_down(x[r], off, 64);
    }
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int r = 0; r < NR; ++r) sh[r][wave] = x[r];
    }
    __syncthreads();
    if (threadIdx.x < NR) {
        const int r = threadIdx.x;
        double s = sh[r][0];
#pragma unroll
        for (int w = 1; w < BLOCK / 64; ++w) s += sh[r][w];
        res[r] = s;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NR; ++r) out[r] = res[r];
}

// ---------------------------------------------------------------------------
// Device-resident solver state (one per right-hand side) and the per-step
// coefficient tables that the scalar kernels write and the vector kernels
// read.
// ---------------------------------------------------------------------------
struct SeedState {
    double2 rho0, alpha, omega, beta, rho1;
    double2 gam[LMAX];
    double bnorm, rtnorm, rnorm0, rnorm_j;
    double tol;
    int run;        // right-hand side still iterating
    int bicg_on;    // BiCG steps continue in this outer iteration
    int l_eff;      // BiCG steps completed in this outer iteration
    int l_mr;       // MR terms applied in this outer iteration
    int broken, exhausted, forced, partial;
    int m, n;       // outer iteration, global BiCG step
    int max_outer, max_steps;
    int status;
    int nact;       // active shifts
    int nshift;
    int mv, dots, axpys, reliable;
    int mixed;      // FP32 iteration: reliable updates on
    int rel;        // reliable update due at the end of this outer iteration
    double rmax;    // largest ||r_0|| since the last reliable update
    int act[NSMAX];
    // this outer iteration's BiCG steps (deferred shift updates):
    // flag 0 no step, 1 u-update and Mv only (gamma breakdown), 2 full step
    double2 step_beta[LMAX], step_alpha[LMAX];
    int step_flag[LMAX];
    // basis form (MSB_SEED_BASIS): this BiCG step's exhaustion test needs
    // ||r_0||, formed from the basis (set by the necessary-condition check)
    int exh_check;
    // basis form with a sparse r~: the first direction update of the next
    // outer iteration, u_0 = r_0 - beta u_0, made by the MR update with the
    // beta it computed (beta_spec); wu_ready: the next step 0 found the same
    // beta, so its own direction update is left out
    double2 beta_spec;
    double2 spec_rho1;   // <r~, r_0> after the MR step, from the list's entries
    int wu_ready;
};
// at most this many nonzero entries of r~ for the index-list inner products
constexpr int SPARSE_MAX = 16;

// Basis form of the seed (MSB_SEED_BASIS): the outer iteration's vectors as
// coefficients on its basis B_0 = r_0, B_1 = u_0 at the start of the
// iteration, B_{2+2j} = S u_j and B_{3+2j} = S r_j of BiCG step j:
//   r_i = sum_b r[i][b] B_b,  u_i = sum_b u[i][b] B_b  (i = 0..l).
constexpr int NBB = 2 * LMAX + 2;
struct SeedBasis {
    double2 r[LMAX + 1][NBB];
    double2 u[LMAX + 1][NBB];
    // replay of the double pass: r[0], u[0] hold r_0, u_0 after the outer
    // iteration's MR step, formed from the first nbu basis vectors (0: the
    // iteration leaves r_0 and u_0 as they are)
    int nbu;
    int pad_[3];
};

struct ShiftState {
    double2 zeta, zeta_prev, pi_prev, psi;
    double sp;      // sigma' = sigma_s - sigma_0
    double res;     // last collinear residual estimate
    int active, iters, force;
    int broken;     // stopped because zeta or q cancelled or is not finite
    int stopped;    // stopped inside an outer iteration (broken, or |zeta psi|
                    // past ZETA_MAX): iteration `iters` still applied part
};

struct StepCoef {   // one active shift, one BiCG step
    double2 kap, beta_s, alpha_s, a1, a2;
    double sp;
    int s, live;
};

struct MRCoef {     // one active shift, one MR step
    double2 kc[LMAX];   // kappa * c_k
    double2 inv_q;
    int s, live;
};

// Deferred single pass: one active shift's update over a whole outer
// iteration as coefficients on the iteration's basis
//   B = {r_0 at the start, u_0 at the start, S u_j and S r_j of step j = 0..l-1}
// (index 0, 1, 2 + 2j, 3 + 2j) plus the shift's own u^s_0 at the start (index
// 2l + 2):  u^s_0 <- sum_b cu[b] B_b + cu[2l+2] u^s_0,
//           x^s   <- x^s + sum_b cx[b] B_b + cx[2l+2] u^s_0.
constexpr int NDEF = 2 * LMAX + 3;
struct DeferCoef {
    double2 cu[NDEF], cx[NDEF];
    int s, live;
};

// Pass-1 record of the seed (read back by the host for the double-pass sweep)
struct TapeStep {
    double2 beta, alpha;
    int flag;       // 0: no step, 1: u-step only (gamma breakdown), 2: full step
    int pad;
};

// Pass-1 record of one outer iteration
struct TapeOuter {
    int l_eff;      // full BiCG steps
    int l_mr;       // MR terms applied (0: no MR)
    int partial;    // a u-step only (gamma breakdown) follows the full steps
    int exhausted;  // Krylov space exhausted: the iteration ended early
    int rel;        // a reliable update r_0 = b - S x followed the MR step
    int pad0, pad1, pad2;
};

// Pass-2 program entry (written by the host after the sweep)
struct ReplayStep {
    double2 beta, alpha, cu, cr;   // cu, cr: coefficients of the two Mv outputs
    int flag, pad0, pad1, pad2;    // flag: 0 none, 1 u-step only, 2 full step
};

struct ReplayOuter {
    double2 gam[LMAX];
    double2 crel;   // coefficient of the reliable-update Mv output S x
    int lm, rel, pad1, pad2;
};

struct Geom {
    int Lx, Ly, Lz, Lt, V;
};

}  // namespace msb

namespace msb {

// Launch gate: a kernel instance for right-hand side `rhs` does work only when
// (seed == nullptr || seed[rhs].run && (!need_bicg || seed[rhs].bicg_on)) and
// (flag == nullptr || flag[rhs * flag_stride] >= need, or == need with eq).
// The decision is
// uniform across a block (one block row per right-hand side).
struct Gate {
    const SeedState *seed = nullptr;
    int need_bicg = 0;
    const int *flag = nullptr;
    long flag_stride = 0;
    int need = 0;
    int eq = 0;                // flag must equal need (not merely reach it)
};

__device__ inline bool gate_open(const Gate &g, int rhs) {
    if (g.seed) {
        const SeedState &s = g.seed[rhs];
        if (!s.run) return false;
        if (g.need_bicg && !s.bicg_on) return false;
    }
    if (g.flag) {
        const int f = g.flag[(long)rhs * g.flag_stride];
        if (g.eq ? (f != g.need) : (f < g.need)) return false;
    }
    return true;
}

// Row length of the reduction-partial buffer: one entry per block of the
// widest reducing launch (the stencil uses one block per 256 sites).
// Row stride of the partial-sum buffers: the stencil writes one partial per
// 64-site chunk (one wavefront), the vector kernels at most NBMAX.
inline long part_stride(const Geom &g) {
    const long nch = ((long)g.V + 63) / 64;
    return nch > NBMAX ? nch : NBMAX;
}

inline int nblocks_for(long n) {
    long b = (n + BLOCK - 1) / BLOCK;
    if (b < 1) b = 1;
    return (int)(b > NBMAX ? NBMAX : b);
}

}  // namespace msb
