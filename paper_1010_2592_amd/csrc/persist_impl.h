// Persistent execution of a solve: one cooperative launch runs a table of
// stage operations (stencil, seed and shift vector updates, Gram partials,
// device scalar steps) in order, with a grid-wide barrier between consecutive
// operations.  The 12 right-hand sides of a batch share every stage, so the
// links each stencil stage loads are shared by all of them, and the host
// issues one launch for the whole iteration instead of about 9 l + 5 launches
// and a synchronisation per outer iteration.
//
// The table repeats (one outer iteration of the single-pass or double-pass
// first pass) until no right-hand side is still running, or runs once (the
// double-pass replay, whose every outer iteration is known in advance).
//
// Grid barrier: a three-level tree of monotone counters.  At the start of
// the launch every block reads the hardware ID of the XCD it runs on and
// takes a rank among the blocks of that XCD (a census behind one flat
// barrier), so the tree below follows where the blocks really run, whatever
// order the dispatcher dealt them in and however many XCDs the device has.
// Inside an XCD the blocks form groups of PERSIST_GROUP.  Every work-item
// first waits for its own stores to reach its XCD's L2; the last block of a
// group to arrive arrives at its XCD, and the last group of an XCD writes
// that L2 back (agent-scope release) and arrives at the global counter.  Release runs down the same tree, and every
// block ends with an agent-scope acquire (invalidating stale lines), so
// blocks on different XCDs see each other's results.  One L2 write-back per
// XCD instead of one per block is what makes this barrier about 7x cheaper
// than a flat one.  The launch is cooperative, so every block is resident and
// each wait ends; a wait that still exceeds its bound raises the abort flag,
// which every waiting block sees and leaves on, so no wave stays behind.
// one load per partial in flight in the block sums: this kernel's register
// budget is the maximum over all its stages (the sums are the same bits)
#define MSB_SUM_PREFETCH 1
#include "barrier_tree.h"
#include "blas_dev.h"
#include "scalar_dev.h"
#include "stencil_dev.h"

namespace msb {

namespace {

using namespace dev;

constexpr unsigned SPIN_LIMIT = 1u << 24;   // seconds of polling; a stage takes milliseconds

__device__ __forceinline__ bool spin_until(unsigned long long *p, unsigned long long v, int *abortf) {
    unsigned spins = 0;
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < v) {
        if (__hip_atomic_load(abortf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
        if (++spins > SPIN_LIMIT) {
            __hip_atomic_store(abortf, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return true;
}

// The XCD (accelerator complex die) this wave runs on: hardware register
// XCC_ID, bits 0..3.
__device__ __forceinline__ int xcc_id() {
    return (int)(__builtin_amdgcn_s_getreg(20 | (0 << 6) | ((4 - 1) << 11)) & 15u);
}

// A block's place in the barrier tree, from the census.
struct TreePos {
    int x, k, nx, nxcd;   // XCD, rank among its blocks, blocks on it, XCDs in use
};

// Census (thread 0 of every block): count the blocks on each XCD and give
// each block its rank there; every block waits until all are counted (the
// launch is cooperative, so all are resident).  False if the XCD ID is out
// of range or a wait exceeds its bound (abort flag raised).
__device__ __forceinline__ bool census(PersistCtl *ctl, TreePos *pos) {
    const int x = xcc_id();
    if (x < 0 || x >= 8) {
        __hip_atomic_store(&ctl->abort, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
    }
    pos->x = x;
    pos->k = (int)__hip_atomic_fetch_add(&ctl->xcount[x], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // the count above is visible before this arrival is (release), and every
    // count after the wait (acquire)
    __hip_atomic_fetch_add(&ctl->census, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if (!spin_until(&ctl->census, (unsigned long long)gridDim.x, &ctl->abort)) return false;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    pos->nx = (int)__hip_atomic_load(&ctl->xcount[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    pos->nxcd = 0;
    for (int i = 0; i < 8; ++i)
        pos->nxcd += __hip_atomic_load(&ctl->xcount[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > 0 ? 1 : 0;
    if (tree::group_of(0, pos->nx, PERSIST_GROUP).ng > PERSIST_MAX_GROUPS) {
        __hip_atomic_store(&ctl->abort, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
    }
    return true;
}

__device__ __forceinline__ bool grid_barrier(PersistCtl *ctl, unsigned long long number, const TreePos &pos) {
    __shared__ int ok_sh;
    // s_waitcnt vmcnt(0): this work-item's stores have reached the L2
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const int x = pos.x;
        const tree::Group tg = tree::group_of(pos.k, pos.nx, PERSIST_GROUP);
        const int g = tg.g, ng = tg.ng, gsize = tg.gsize;
        const int gi = x * PERSIST_MAX_GROUPS + g;
        const unsigned long long a =
            __hip_atomic_fetch_add(&ctl->gbar[gi], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
        if (a == number * (unsigned long long)gsize) {
            const unsigned long long ax =
                __hip_atomic_fetch_add(&ctl->xbar[x], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
            if (ax == number * (unsigned long long)ng) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // write this XCD's L2 back
                __hip_atomic_fetch_add(&ctl->bar, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = spin_until(&ctl->bar, number * (unsigned long long)pos.nxcd, &ctl->abort);
                __hip_atomic_store(&ctl->xrel[x], number, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                ok = spin_until(&ctl->xrel[x], number, &ctl->abort);
            }
            __hip_atomic_store(&ctl->grel[gi], number, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            ok = spin_until(&ctl->grel[gi], number, &ctl->abort);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");       // drop stale lines
        ok_sh = ok;
    }
    __syncthreads();
    return ok_sh != 0;
}

// virtual block vb of a vector op: element block vb % nblk of rhs vb / nblk
#define VLOOP_VEC(CALL)                                                       \
    for (int vb = blockIdx.x; vb < op.nvb; vb += gridDim.x) {                 \
        const int rhs = vb / op.nblk, bx = vb - rhs * op.nblk, gx = op.nblk;  \
        CALL;                                                                 \
        __syncthreads();                                                      \
    }
#define VLOOP(CALL)                                                           \
    for (int vb = blockIdx.x; vb < op.nvb; vb += gridDim.x) {                 \
        CALL;                                                                 \
        __syncthreads();                                                      \
    }

// The scalar stages run in one block per right-hand side and are latency
// bound; as separate functions their registers do not enter the allocation of
// the stencil and vector stages inlined into the kernel.
__device__ __noinline__ void call_sc_beta(const ScalarArgs *a, int rhs) { sc_beta_body(*a, rhs); }
__device__ __noinline__ void call_sc_alpha(const ScalarArgs *a, int rhs) { sc_alpha_body(*a, rhs); }
__device__ __noinline__ void call_sc_mr(const ScalarArgs *a, int rhs) { sc_mr_body(*a, rhs); }
__device__ __noinline__ void call_sc_rel(const ScalarArgs *a, int rhs) { sc_rel_body(*a, rhs); }
__device__ __noinline__ void call_sc_conv(const ScalarArgs *a, int rhs) { sc_conv_body(*a, rhs); }
// The site-block stencil in the form that keeps this kernel within the
// stencil's own register budget (three wavefronts per SIMD): the same
// arithmetic and per-wavefront partials as dslash_site_block and the chunked
// stencil, with the one-trip site loop written out in the block function.
template <typename T, int EPI, bool G5IN>
__device__ __forceinline__ void dslash_persist_body(const DslashArgs<T> &a, int p) {
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
        // the hop order of wilson_site_global (by the parity of z + t),
        // written out here: through that function the kernel's allocation
        // needs more than 256 VGPRs and spills
        const T ff = (t == Lt - 1) ? a.ef * a.bc : a.ef;
        const T fb = (t == 0) ? a.eb * a.bc : a.eb;
        if (order_parity(a.g, s)) {
            int sf, sb;
            sf = (z == Lz - 1) ? s - (Lz - 1) * sxy : s + sxy;
            sb = (z == 0) ? s + (Lz - 1) * sxy : s - sxy;
            hop<T, 2, -1, false, G5IN>(acc, in, U + (size_t)2 * 9 * V + s, V, V, sf, (T)1);
            hop<T, 2, +1, true, G5IN>(acc, in, U + (size_t)2 * 9 * V + sb, V, V, sb, (T)1);
            sf = (t == Lt - 1) ? s - (Lt - 1) * sxyz : s + sxyz;
            sb = (t == 0) ? s + (Lt - 1) * sxyz : s - sxyz;
            hop<T, 3, -1, false, G5IN>(acc, in, U + (size_t)3 * 9 * V + s, V, V, sf, ff);
            hop<T, 3, +1, true, G5IN>(acc, in, U + (size_t)3 * 9 * V + sb, V, V, sb, fb);
            sf = (x == Lx - 1) ? s - (Lx - 1) : s + 1;
            sb = (x == 0) ? s + (Lx - 1) : s - 1;
            hop<T, 0, -1, false, G5IN>(acc, in, U + (size_t)0 * 9 * V + s, V, V, sf, (T)1);
            hop<T, 0, +1, true, G5IN>(acc, in, U + (size_t)0 * 9 * V + sb, V, V, sb, (T)1);
            sf = (yy == Ly - 1) ? s - (Ly - 1) * Lx : s + Lx;
            sb = (yy == 0) ? s + (Ly - 1) * Lx : s - Lx;
            hop<T, 1, -1, false, G5IN>(acc, in, U + (size_t)1 * 9 * V + s, V, V, sf, (T)1);
            hop<T, 1, +1, true, G5IN>(acc, in, U + (size_t)1 * 9 * V + sb, V, V, sb, (T)1);
#pragma unroll
            for (int sp = 0; sp < 4; ++sp) {
                C<T> ps[3];
                load_spin<T, G5IN>(in, V, s, sp, ps);
                const T sg = ((a.g5out && sp >= 2) ? (T)-1 : (T)1) * a.scale;
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    acc[sp][c] = cscale(csub(cscale(ps[c], a.diag), cscale(acc[sp][c], (T)0.5)), sg);
            }
        } else {
            const T m2d = (T)-2 * a.diag;
#pragma unroll
            for (int sp = 0; sp < 4; ++sp) {
                C<T> ps[3];
                load_spin<T, G5IN>(in, V, s, sp, ps);
                diag_start_spin<T>(acc[sp], ps, m2d);
            }
            int sf, sb;
            sf = (x == Lx - 1) ? s - (Lx - 1) : s + 1;
            sb = (x == 0) ? s + (Lx - 1) : s - 1;
            hop<T, 0, -1, false, G5IN>(acc, in, U + (size_t)0 * 9 * V + s, V, V, sf, (T)1);
            hop<T, 0, +1, true, G5IN>(acc, in, U + (size_t)0 * 9 * V + sb, V, V, sb, (T)1);
            sf = (yy == Ly - 1) ? s - (Ly - 1) * Lx : s + Lx;
            sb = (yy == 0) ? s + (Ly - 1) * Lx : s - Lx;
            hop<T, 1, -1, false, G5IN>(acc, in, U + (size_t)1 * 9 * V + s, V, V, sf, (T)1);
            hop<T, 1, +1, true, G5IN>(acc, in, U + (size_t)1 * 9 * V + sb, V, V, sb, (T)1);
            sf = (z == Lz - 1) ? s - (Lz - 1) * sxy : s + sxy;
            sb = (z == 0) ? s + (Lz - 1) * sxy : s - sxy;
            hop<T, 2, -1, false, G5IN>(acc, in, U + (size_t)2 * 9 * V + s, V, V, sf, (T)1);
            hop<T, 2, +1, true, G5IN>(acc, in, U + (size_t)2 * 9 * V + sb, V, V, sb, (T)1);
            sf = (t == Lt - 1) ? s - (Lt - 1) * sxyz : s + sxyz;
            sb = (t == 0) ? s + (Lt - 1) * sxyz : s - sxyz;
            hop<T, 3, -1, false, G5IN>(acc, in, U + (size_t)3 * 9 * V + s, V, V, sf, ff);
            hop<T, 3, +1, true, G5IN>(acc, in, U + (size_t)3 * 9 * V + sb, V, V, sb, fb);
#pragma unroll
            for (int sp = 0; sp < 4; ++sp) {
                const T f = ((a.g5out && sp >= 2) ? (T)0.5 : (T)-0.5) * a.scale;
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[sp][c] = cscale(acc[sp][c], f);
            }
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
        wave_reduce_store<3>(part, a.part + (size_t)rhs * PMAX * a.ps + sblk * (BLOCK / 64) + (threadIdx.x >> 6),
                             a.ps);
}


template <typename T, int L, bool XH, int J>
__device__ __forceinline__ void exec_r_update_j(const POp &op, const VecArgs<T> &a) {
    if constexpr (J < L) {
        if (op.j == J) {
            if (op.shifts) VLOOP_VEC((r_update_body<T, J, true, XH>(a, bx, gx, rhs)))
            else VLOOP_VEC((r_update_body<T, J, false, XH>(a, bx, gx, rhs)))
            return;
        }
        exec_r_update_j<T, L, XH, J + 1>(op, a);
    }
}

template <typename T, int L, bool XH, int J>
__device__ __forceinline__ void exec_seed_u_j(const POp &op, const VecArgs<T> &a) {
    if constexpr (J < L) {
        if (op.j == J) {
            VLOOP_VEC((seed_u_body<T, J>(a, bx, gx, rhs)))
            return;
        }
        exec_seed_u_j<T, L, XH, J + 1>(op, a);
    }
}

// One instance per MR degree L keeps the kernel's register budget at that of
// its largest stage for this L (the Gram stage of L = 7, 8 alone needs more
// than 220 VGPRs).
template <typename T, int L>
__device__ __forceinline__ void exec_op(const POp &op) {
    // FP32 iterations keep FP64 seed solutions (reliable updates); FP64 ones do not
    constexpr bool XH = sizeof(T) != sizeof(double);
    switch (op.kind) {
    case OP_DS: {
        const DslashArgs<T> *a = reinterpret_cast<const DslashArgs<T> *>(op.blob);
        if (op.epi == EPI_PLAIN) VLOOP((dslash_persist_body<T, EPI_PLAIN, false>(*a, vb)))
        else if (op.epi == EPI_MV) VLOOP((dslash_persist_body<T, EPI_MV, false>(*a, vb)))
        else VLOOP((dslash_persist_body<T, EPI_MV_Y, false>(*a, vb)))
        break;
    }
    case OP_DS64: {
        if constexpr (XH) {
            const DslashArgs<double> *a = reinterpret_cast<const DslashArgs<double> *>(op.blob);
            if (op.epi == EPI_PLAIN) VLOOP((dslash_persist_body<double, EPI_PLAIN, false>(*a, vb)))
            else VLOOP((dslash_persist_body<double, EPI_SV, false>(*a, vb)))
        }
        break;
    }
    case OP_SEED_U: {
        exec_seed_u_j<T, L, XH, 0>(op, *reinterpret_cast<const VecArgs<T> *>(op.blob));
        break;
    }
    case OP_R_UPDATE:
        exec_r_update_j<T, L, XH, 0>(op, *reinterpret_cast<const VecArgs<T> *>(op.blob));
        break;
    case OP_GRAM: {
        const VecArgs<T> &a = *reinterpret_cast<const VecArgs<T> *>(op.blob);
        VLOOP_VEC((gram_body<T, L>(a, bx, gx, rhs)))
        break;
    }
    case OP_MR_UPDATE: {
        const VecArgs<T> &a = *reinterpret_cast<const VecArgs<T> *>(op.blob);
        if (op.shifts) VLOOP_VEC((mr_update_body<T, L, true, XH>(a, bx, gx, rhs)))
        else VLOOP_VEC((mr_update_body<T, L, false, XH>(a, bx, gx, rhs)))
        break;
    }
    case OP_REL_UPDATE: {
        if constexpr (XH) {
            const VecArgs<T> &a = *reinterpret_cast<const VecArgs<T> *>(op.blob);
            VLOOP_VEC((rel_update_body<T>(a, op.b, op.v, op.y, op.yc, bx, gx, rhs)))
        }
        break;
    }
    case OP_SC_BETA: {
        const ScalarArgs &a = *reinterpret_cast<const ScalarArgs *>(op.blob);
        VLOOP((call_sc_beta(&a, vb)))
        break;
    }
    case OP_SC_ALPHA: {
        const ScalarArgs &a = *reinterpret_cast<const ScalarArgs *>(op.blob);
        VLOOP((call_sc_alpha(&a, vb)))
        break;
    }
    case OP_SC_MR: {
        const ScalarArgs &a = *reinterpret_cast<const ScalarArgs *>(op.blob);
        VLOOP((call_sc_mr(&a, vb)))
        break;
    }
    case OP_SC_REL: {
        const ScalarArgs &a = *reinterpret_cast<const ScalarArgs *>(op.blob);
        VLOOP((call_sc_rel(&a, vb)))
        break;
    }
    case OP_SC_CONV: {
        const ScalarArgs &a = *reinterpret_cast<const ScalarArgs *>(op.blob);
        VLOOP((call_sc_conv(&a, vb)))
        break;
    }
    default:
        break;
    }
}

template <typename T, int L>
__global__ __launch_bounds__(BLOCK) void k_persistent(PersistArgs pa) {
    __shared__ TreePos pos_sh;
    __shared__ int census_ok;
    if (threadIdx.x == 0) census_ok = census(pa.ctl, &pos_sh) ? 1 : 0;
    __syncthreads();
    if (!census_ok) return;
    const TreePos pos = pos_sh;
    unsigned long long number = 0;
    const bool timer = pa.timing && blockIdx.x == 0 && threadIdx.x == 0;
    long long t0 = timer ? wall_clock64() : 0;
    for (int it = 0; it < pa.iters; ++it) {
        for (int k = 0; k < pa.nops; ++k) {
            const POp &op = pa.ops[k];
            exec_op<T, L>(op);
            if (!grid_barrier(pa.ctl, ++number, pos)) return;
            if (timer) {
                const long long t1 = wall_clock64();
                pa.ctl->ticks[op.cls] += (unsigned long long)(t1 - t0);
                pa.ctl->execs[op.cls] += 1;
                t0 = t1;
            }
        }
        if (pa.loop) {
            // SeedState::run changes only in the convergence step, which ends
            // the table, so every block reads the same values here
            int any = 0;
            for (int r = 0; r < pa.nrhs; ++r)
                any |= __hip_atomic_load(&pa.seed[r].run, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!any) break;
        }
    }
}

}  // namespace

// Entry points of one MR degree L (persist_l<L>.hip instantiates them).
template <typename T, int L>
int persistent_grid_l(int device) {
    int per_cu = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(k_persistent<T, L>), BLOCK,
                                                     0) != hipSuccess)
        return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
    long g = ((long)per_cu * ncu / 8) * 8;
    const long cap = 8L * PERSIST_GROUP * PERSIST_MAX_GROUPS;   // what the barrier tree holds
    if (g > cap) g = cap;
    return (int)g;
}

template <typename T, int L>
hipError_t launch_persistent_l(hipStream_t st, const PersistArgs &pa, int grid) {
    PersistArgs copy = pa;
    void *args[] = {&copy};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_persistent<T, L>), dim3(grid), dim3(BLOCK), args,
                                      0, st);
}

#define MSB_PERSIST_INSTANTIATE(L)                                                            \
    template int persistent_grid_l<double, L>(int);                                           \
    template int persistent_grid_l<float, L>(int);                                            \
    template hipError_t launch_persistent_l<double, L>(hipStream_t, const PersistArgs &, int); \
    template hipError_t launch_persistent_l<float, L>(hipStream_t, const PersistArgs &, int);

}  // namespace msb
