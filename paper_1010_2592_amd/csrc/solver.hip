// Host orchestration of multi-shift BiCGstab(l) on one GPU.
//
// Single-pass (pass = 1): the seed iteration and every shifted system advance
// together; the shift vectors u^s_0..u^s_l, x^s live in HBM and are updated by
// the fused r_update / mr_update kernels (Section 2: N_s (l+1) extra vectors,
// sum_s M_s l (0.5 l + 4.5) extra axpys).
//
// Double-pass (pass = 2, Section 2 option 1 after Eq. 2.2, Section 5): pass 1
// runs the seed and the shifts' scalar recurrences only and records the seed's
// scalars (beta_n, alpha_n, the MR coefficients) and each shift's M_s.  The
// single-pass program that would form y = sum_s w_s x^s is linear in its
// sources -- b and the 2 M l Mv outputs v_t -- with coefficients fixed by
// those scalars, so one backward sweep over the recorded program (scalar work
// on the host, O(N_s M l^2)) gives y = c_b b + sum_t c_t v_t.  Pass 2 replays
// the seed from b with the recorded scalars (no inner products) and adds
// c_t v_t in the epilogue of the stencil that produces v_t.  The sweep reaches
// the same y as the paper's closed-form coefficients (A_mj ... G_mj, x_BiCG)
// in a different bookkeeping; no shift vector is ever stored.
//
// Every inner-iteration decision is taken on the device (scalar kernels), so
// the host synchronises once per outer iteration to learn whether any
// right-hand side is still running.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "ctx.h"

namespace msb {

static thread_local std::string g_err;
const char *last_error_msg() { return g_err.c_str(); }

int set_error(int status, const std::string &msg) {
    g_err = msg;
    return status;
}

int hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return 0;
    return set_error(S_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(x)                                  \
    do {                                           \
        int rc_ = hip_check((x), #x);              \
        if (rc_) return rc_;                       \
    } while (0)
#define CHK(x)                                     \
    do {                                           \
        int rc_ = (x);                             \
        if (rc_) return rc_;                       \
    } while (0)

int ensure(Ctx *c, DevBuf &b, size_t bytes) {
    if (bytes < 256) bytes = 256;
    if (b.bytes >= bytes) return 0;
    if (c->arena) {
        // no-allocation call: a fresh region of the arena (a smaller region
        // this buffer held earlier in the call stays unused)
        Arena &a = *c->arena;
        const size_t off = (a.used + 255) & ~(size_t)255;
        if (off > a.cap || bytes > a.cap - off)
            return set_error(S_ERR_ARG, "workspace of more than " + std::to_string(a.cap) +
                                            " bytes needed: beyond the fixed scratch buffer of the "
                                            "no-allocation entry point");
        b.p = a.base + off;
        b.bytes = bytes;
        a.used = off + bytes;
        return 0;
    }
    if (b.p) {
        (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(S_ERR_OOM, "workspace allocation of " + std::to_string(bytes) + " bytes failed");
    }
    b.bytes = bytes;
    return 0;
}

static int ensure_host(Ctx *c, size_t bytes) {
    if (c->host_pinned_bytes >= bytes) return 0;
    if (c->arena) {
        // no-allocation call: pageable heap memory (the host reads it only
        // after synchronising the stream, as it does the pinned buffer)
        c->host_heap.resize(bytes);
        c->host_pinned = c->host_heap.data();
        c->host_pinned_bytes = bytes;
        return 0;
    }
    if (c->host_pinned) (void)hipHostFree(c->host_pinned);
    c->host_pinned = nullptr;
    c->host_pinned_bytes = 0;
    HIPCHK(hipHostMalloc(&c->host_pinned, bytes, hipHostMallocDefault));
    c->host_pinned_bytes = bytes;
    return 0;
}

// ---------------------------------------------------------------------------
// kernel timing hook
// ---------------------------------------------------------------------------
static hipEvent_t pool_get(Ctx *c) {
    if (c->ev_used < c->ev_pool.size()) return c->ev_pool[c->ev_used++];
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    c->ev_pool.push_back(e);
    c->ev_used++;
    return e;
}

Prof::Prof(Ctx *c_, int cls_, double bytes_) : c(c_), cls(cls_), bytes(bytes_) {
    c->bytes_acc += bytes;
    if (c->prof && cls >= 0 && cls < 32 && ((c->prof_mask >> cls) & 1u) && c->prof_seq++ % c->prof_stride == 0) {
        e0 = pool_get(c);
        if (cls == CL_STENCIL) {
            // every stencil-class scope holds one launch_dslash: its dispatch
            // records the pair itself
            e1 = e0 ? pool_get(c) : nullptr;
            if (e1) {
                stencil_timing_arm(e0, e1);
                armed = true;
            }
        } else if (e0) {
            (void)hipEventRecord(e0, c->stream);
        }
    }
}

Prof::~Prof() {
    if (armed) {
        if (stencil_timing_taken()) c->recs.push_back(Ctx::Rec{cls, bytes, e0, e1});
        return;
    }
    if (c->prof && e0) {
        hipEvent_t e1b = pool_get(c);
        if (e1b) {
            (void)hipEventRecord(e1b, c->stream);
            c->recs.push_back(Ctx::Rec{cls, bytes, e0, e1b});
        }
    }
}

int profile_enable(Ctx *c, bool on) {
    HIPCHK(c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize());
    c->prof = on;
    c->recs.clear();
    c->srecs.clear();
    c->ev_used = 0;
    return 0;
}

int profile_classes(Ctx *c, unsigned mask, int stride) {
    HIPCHK(c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize());
    c->prof_mask = mask;
    c->prof_stride = stride;
    c->prof_seq = 0;
    return 0;
}

int profile_read(Ctx *c, int ncls, long long *cnt, double *ms, double *bytes) {
    HIPCHK(c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize());
    for (int k = 0; k < ncls; ++k) {
        cnt[k] = 0;
        ms[k] = 0.0;
        bytes[k] = 0.0;
    }
    for (const Ctx::SRec &r : c->srecs) {
        if (r.cls >= ncls) continue;
        cnt[r.cls] += r.count;
        ms[r.cls] += r.ms;
        bytes[r.cls] += r.bytes;
    }
    for (const Ctx::Rec &r : c->recs) {
        if (r.cls >= ncls) continue;
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, r.e0, r.e1));
        cnt[r.cls] += 1;
        ms[r.cls] += t;
        bytes[r.cls] += r.bytes;
    }
    return 0;
}

template <typename T> static const C<T> *links(const Ctx *c);
template <> const C<double> *links<double>(const Ctx *c) { return c->U64; }
template <> const C<float> *links<float>(const Ctx *c) { return c->U32; }

template <typename T>
static DslashArgs<T> ds_args(const Ctx *c, bool neg_mu, bool g5out) {
    DslashArgs<T> a;
    a.U = links<T>(c);
    a.g = c->g;
    a.diag = (T)(4.0 + c->mass);
    const double mu = neg_mu ? -c->mu : c->mu;
    a.ef = (T)std::exp(mu);
    a.eb = (T)std::exp(-mu);
    a.bc = (T)c->bc_t;
    a.g5out = g5out ? 1 : 0;
    return a;
}

int ctx_create(Ctx *c, const int dims[4], double mass, double mu, int bc_t, const void *lk,
               hipStream_t st) {
    c->g.Lx = dims[0];
    c->g.Ly = dims[1];
    c->g.Lz = dims[2];
    c->g.Lt = dims[3];
    c->g.V = dims[0] * dims[1] * dims[2] * dims[3];
    c->mass = mass;
    c->mu = mu;
    c->bc_t = bc_t;
    c->stream = st;
    HIPCHK(hipGetDevice(&c->device));
    const size_t nl = 36ull * c->g.V;
    if (hipMalloc(&c->U64, nl * sizeof(double2)) != hipSuccess ||
        hipMalloc(&c->U32, nl * sizeof(float2)) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(S_ERR_OOM, "link allocation failed");
    }
    HIPCHK(hipMemcpyAsync(c->U64, lk, nl * sizeof(double2), hipMemcpyDeviceToDevice, st));
    launch_convert_in<float>(st, c->U32, c->U64, (long)nl, 0, 0, 1);
    HIPCHK(hipGetLastError());
    // the links' norm bound: sqrt of the largest Gershgorin bound of U^+ U,
    // widened by 1e-12 for the rounding of its sums
    const int nbl = link_gershgorin_blocks(c->g.V);
    double *gb = nullptr;
    if (hipMalloc(&gb, nbl * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(S_ERR_OOM, "link allocation failed");
    }
    launch_link_gershgorin(st, c->U64, c->g.V, gb);
    std::vector<double> hg(nbl);
    const hipError_t e1 = hipMemcpyAsync(hg.data(), gb, nbl * sizeof(double), hipMemcpyDeviceToHost, st);
    const hipError_t e2 = hipStreamSynchronize(st);
    (void)hipFree(gb);
    HIPCHK(e1);
    HIPCHK(e2);
    double gmax = 0.0;
    for (double v : hg) gmax = std::isfinite(v) ? std::max(gmax, v) : INFINITY;
    c->link_norm = std::sqrt(gmax * (1.0 + 1e-12));
    return 0;
}

void ctx_destroy(Ctx *c) {
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    DevBuf *bufs[] = {&c->ws_R, &c->ws_U, &c->ws_tmp, &c->ws_W, &c->ws_X, &c->ws_rt, &c->ws_b,
                      &c->ws_y, &c->ws_part, &c->ws_seed, &c->ws_shift, &c->ws_sc, &c->ws_mc,
                      &c->ws_tape, &c->ws_tape_gam, &c->ws_tape_outer, &c->ws_replay,
                      &c->ws_replay_outer, &c->ws_wts, &c->ws_sig0, &c->ws_cb, &c->ws_aux1,
                      &c->ws_aux2, &c->ws_aux3, &c->ws_aux4, &c->ws_bX, &c->ws_bZ, &c->ws_by,
                      &c->ws_beta, &c->ws_bA, &c->ws_bB, &c->ws_bdots, &c->ws_ops, &c->ws_pctl,
                      &c->ws_rX, &c->ws_rX2, &c->ws_ry, &c->ws_rB, &c->ws_rR, &c->ws_rt1, &c->ws_rt2,
                      &c->ws_rsig, &c->ws_rw, &c->ws_Bm, &c->ws_schist, &c->ws_dc, &c->ws_ones,
                      &c->ws_cg_r, &c->ws_cg_p, &c->ws_cg_w, &c->ws_cg_P, &c->ws_cg_seed, &c->ws_cg_shift,
                      &c->ws_cg_coef, &c->ws_cg_tape, &c->ws_cg_c, &c->ws_cg_n, &c->ws_eY, &c->ws_eW,
                      &c->ws_eZ, &c->ws_eP, &c->ws_eS, &c->ws_eG, &c->ws_sp, &c->ws_hs, &c->ws_hs64,
                      &c->ws_bw, &c->ws_sb};
    for (DevBuf *b : bufs)
        if (b->p) (void)hipFree(b->p);
    for (DevBuf &b : c->pstore)
        if (b.p) (void)hipFree(b.p);
    for (DevBuf &b : c->prel)
        if (b.p) (void)hipFree(b.p);
    if (c->U64) (void)hipFree(c->U64);
    if (c->U32) (void)hipFree(c->U32);
    if (c->host_pinned) (void)hipHostFree(c->host_pinned);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    c->ev_pool.clear();
}

// ---------------------------------------------------------------------------
// wilson_apply and the spectral-radius estimate
// ---------------------------------------------------------------------------
int apply_wilson(Ctx *c, const double2 *in, double2 *out, int nrhs, int flags) {
    const bool g5l = flags & 1, negmu = flags & 2, dag = flags & 4, mixed = flags & 8;
    // D^+ = gamma5 D(-mu) gamma5
    const bool g5in = dag, g5out = g5l != dag, nm = negmu != dag;
    const int V = c->g.V;
    const long n = 12L * V;
    if (!mixed) {
        DslashArgs<double> a = ds_args<double>(c, nm, g5out);
        a.in = in;
        a.out = out;
        launch_dslash<double>(c->stream, a, nrhs, EPI_PLAIN, g5in);
    } else {
        CHK(ensure(c, c->ws_aux1, (size_t)nrhs * n * sizeof(float2)));
        CHK(ensure(c, c->ws_aux2, (size_t)nrhs * n * sizeof(float2)));
        float2 *fi = (float2 *)c->ws_aux1.p, *fo = (float2 *)c->ws_aux2.p;
        launch_convert_in<float>(c->stream, fi, in, n, n, n, nrhs);
        DslashArgs<float> a = ds_args<float>(c, nm, g5out);
        a.in = fi;
        a.out = fo;
        launch_dslash<float>(c->stream, a, nrhs, EPI_PLAIN, g5in);
        launch_convert_out<float>(c->stream, out, fo, n, n, n, nrhs);
    }
    HIPCHK(hipGetLastError());
    return 0;
}

// sum of partial row `slot` of rhs 0 on the host (fixed order)
static double host_partial_sum(const double *row, int nblk) {
    double s = 0.0;
    for (int i = 0; i < nblk; ++i) s += row[i];
    return s;
}

int spectral_radius(Ctx *c, const double2 *start, int iters, double *rho) {
    const int V = c->g.V;
    const long n = 12L * V;
    const int nbv = nblocks_for(n);
    hipStream_t st = c->stream;
    CHK(ensure(c, c->ws_aux1, n * sizeof(double2)));
    CHK(ensure(c, c->ws_aux2, n * sizeof(double2)));
    CHK(ensure(c, c->ws_aux3, n * sizeof(double2)));
    const long ps = part_stride(c->g);
    CHK(ensure(c, c->ws_part, (size_t)PMAX * ps * sizeof(double)));
    CHK(ensure_host(c, 3 * ps * sizeof(double)));
    double2 *v = (double2 *)c->ws_aux1.p, *w = (double2 *)c->ws_aux2.p, *z = (double2 *)c->ws_aux3.p;
    double *part = (double *)c->ws_part.p;
    double *hp = (double *)c->host_pinned;
    auto norms = [&](const double2 *x, const double2 *y, double *re, double *yy) -> int {
        launch_dot_partials<double>(st, x, y, n, part, ps, 1, nbv, Gate{});
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(hp, part, 3 * ps * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        *re = host_partial_sum(hp, nbv);
        *yy = host_partial_sum(hp + 2 * ps, nbv);
        return 0;
    };
    double re, nn;
    CHK(norms(start, start, &re, &nn));
    if (!(nn > 0.0)) return set_error(S_ERR_ARG, "spectral_radius: zero start vector");
    launch_overlap_out(st, v, nullptr, start, V, 1, 0, 1.0 / std::sqrt(nn), nbv);
    double lam = 0.0;
    for (int it = 0; it < iters; ++it) {
        DslashArgs<double> a = ds_args<double>(c, false, false);
        a.in = v;
        a.out = w;
        launch_dslash<double>(st, a, 1, EPI_PLAIN, false);
        // D^+ w = gamma5 D(-mu) gamma5 w
        DslashArgs<double> b = ds_args<double>(c, true, true);
        b.in = w;
        b.out = z;
        launch_dslash<double>(st, b, 1, EPI_PLAIN, true);
        CHK(norms(v, z, &re, &nn));
        lam = re;
        if (!(nn > 0.0)) break;
        launch_overlap_out(st, v, nullptr, z, V, 1, 0, 1.0 / std::sqrt(nn), nbv);
    }
    HIPCHK(hipGetLastError());
    *rho = lam;
    return 0;
}

// ---------------------------------------------------------------------------
// double-pass coefficient sweep (host, FP64)
// ---------------------------------------------------------------------------
using cd = std::complex<double>;
static inline cd toc(double2 z) { return cd(z.x, z.y); }
static inline double2 fromc(cd z) { return d2(z.real(), z.imag()); }

struct SweepResult {
    cd cb;
    std::vector<ReplayStep> steps;     // [max_outer * l]
    std::vector<ReplayOuter> outer;    // [max_outer]
    int M = 0;
};

// One right-hand side.  tape: recorded full steps (and a trailing u-step on a
// gamma breakdown); outer: per-outer-iteration record; gam: MR coefficients;
// sp, w: relative shifts and weights; iters, stopped: per-shift M_s and
// whether the shift stopped inside outer iteration M_s (a guard of its
// recurrences), which then still took part in that iteration up to there.
static void sweep_rhs(int l, int M, const TapeStep *tape, const TapeOuter *outer,
                      const double2 *gam, int ns, const double *sp, const double *w,
                      const int *iters, const int *stopped, int max_outer, SweepResult *res) {
    struct Sh {
        cd as, bs, kap, kapn;
        bool live;
    };
    struct Mr {
        cd q, kap, c[LMAX];
        bool live;
    };
    std::vector<int> n0(M + 1, 0);
    for (int m = 0; m < M; ++m) n0[m + 1] = n0[m] + outer[m].l_eff;
    const int nfull = n0[M];
    std::vector<Sh> st((size_t)std::max(nfull, 1) * ns);
    std::vector<Mr> mr((size_t)std::max(M, 1) * ns);
    // forward: recompute the shifts' scalar recurrences
    std::vector<cd> zeta(ns, 1.0), zprev(ns, 1.0), piprev(ns, 0.0), psi(ns, 1.0);
    std::vector<char> alive(ns, 1);
    for (int m = 0; m < M; ++m) {
        std::vector<char> act(ns, 0);
        for (int s = 0; s < ns; ++s)
            act[s] = alive[s] && (m < iters[s] || (stopped[s] && m == iters[s]));
        for (int j = 0; j < outer[m].l_eff; ++j) {
            const int n = n0[m] + j;
            const cd alpha = toc(tape[n].alpha), beta = toc(tape[n].beta);
            for (int s = 0; s < ns; ++s) {
                Sh &h = st[(size_t)n * ns + s];
                h.live = false;
                if (!act[s]) continue;
                const cd z = zeta[s], zp = zprev[s];
                const cd pi_n = z - beta * piprev[s];
                const cd step = alpha * sp[s] * pi_n;
                const cd zn = z + step;
                // the guards of the device recurrences (broken or converged)
                if (!std::isfinite(zn.real()) || !std::isfinite(zn.imag()) || std::abs(zn) < ZETA_MIN ||
                    std::abs(zn) <= BREAK_REL * (std::abs(z) + std::abs(step)) ||
                    !(std::abs(zn) * std::abs(psi[s]) <= ZETA_MAX)) {
                    act[s] = alive[s] = 0;
                    continue;
                }
                h.as = alpha * z / zn;
                h.bs = beta * (zp / z) * (zp / z);
                h.kap = 1.0 / (z * psi[s]);
                h.kapn = 1.0 / (zn * psi[s]);
                h.live = true;
                zprev[s] = z;
                zeta[s] = zn;
                piprev[s] = pi_n;
            }
        }
        const int lm = outer[m].l_mr;
        for (int s = 0; s < ns; ++s) {
            Mr &q = mr[(size_t)m * ns + s];
            q.live = false;
            if (!act[s] || lm == 0) continue;
            cd qs = 1.0;
            double qterms = 1.0;
            for (int i = 1; i <= lm; ++i) {
                double p = 1.0;
                for (int k = 0; k < i; ++k) p *= -sp[s];
                const cd t = toc(gam[(size_t)m * LMAX + i - 1]) * p;
                qs -= t;
                qterms += std::abs(t);
            }
            if (!std::isfinite(qs.real()) || !std::isfinite(qs.imag()) || std::abs(qs) < ZETA_MIN ||
                std::abs(qs) <= BREAK_REL * qterms || !(std::abs(zeta[s]) * std::abs(psi[s]) * std::abs(qs) <= ZETA_MAX)) {
                act[s] = alive[s] = 0;
                continue;
            }
            q.q = qs;
            q.kap = 1.0 / (zeta[s] * psi[s]);
            for (int k = 0; k < LMAX; ++k) q.c[k] = 0.0;
            for (int k = 0; k < lm; ++k) {
                cd acc = 0.0;
                for (int i = k + 1; i <= lm; ++i) {
                    double p = 1.0;
                    for (int e = 0; e < i - 1 - k; ++e) p *= -sp[s];
                    acc += toc(gam[(size_t)m * LMAX + i - 1]) * p;
                }
                q.c[k] = acc / qs;
            }
            q.live = true;
            psi[s] *= qs;
        }
    }
    // backward: adjoint coefficients of every program variable
    std::vector<cd> lamR(l + 1, 0.0), lamU(l + 1, 0.0), lamW((size_t)ns * (l + 1), 0.0);
    cd cb_extra = 0.0;      // coefficient of b from reliable updates
    res->steps.assign((size_t)max_outer * l, ReplayStep{});
    res->outer.assign((size_t)max_outer, ReplayOuter{});
    for (int m = M - 1; m >= 0; --m) {
        const int lm = outer[m].l_mr;
        ReplayOuter &ro = res->outer[m];
        ro.lm = lm;
        ro.rel = outer[m].rel;
        ro.crel = d2(0, 0);
        for (int i = 0; i < LMAX; ++i) ro.gam[i] = (i < lm) ? gam[(size_t)m * LMAX + i] : d2(0, 0);
        if (outer[m].rel) {
            // reliable update r_0 <- b - v, v = S x (an Mv output): b and v are
            // sources; the old r_0 ends its history here
            ro.crel = fromc(-lamR[0]);
            cb_extra += lamR[0];
            lamR[0] = 0.0;
        }
        // MR, reversed: u_0 update, r_0 update, then the shifts
        for (int i = 1; i <= lm; ++i) lamU[i] += -toc(gam[(size_t)m * LMAX + i - 1]) * lamU[0];
        for (int i = 1; i <= lm; ++i) lamR[i] += -toc(gam[(size_t)m * LMAX + i - 1]) * lamR[0];
        for (int s = 0; s < ns; ++s) {
            const Mr &q = mr[(size_t)m * ns + s];
            if (!q.live) continue;
            cd *lw = &lamW[(size_t)s * (l + 1)];
            for (int i = 1; i <= lm; ++i) lw[i] += -toc(gam[(size_t)m * LMAX + i - 1]) * lw[0] / q.q;
            lw[0] = lw[0] / q.q;
            for (int k = 0; k < lm; ++k) lamR[k] += q.kap * q.c[k] * w[s];
        }
        const int le = outer[m].l_eff;
        if (outer[m].partial) {
            // trailing u-step (gamma breakdown): u_i <- r_i - beta u_i, u_{j+1} <- S u_j
            const int j = le;
            const TapeStep &t = tape[n0[m] + le];
            ReplayStep &rs = res->steps[(size_t)m * l + j];
            rs.flag = 1;
            rs.beta = t.beta;
            rs.cu = fromc(lamU[j + 1]);
            lamU[j + 1] = 0.0;
            const cd beta = toc(t.beta);
            for (int i = 0; i <= j; ++i) {
                lamR[i] += lamU[i];
                lamU[i] *= -beta;
            }
        }
        for (int j = le - 1; j >= 0; --j) {
            const int n = n0[m] + j;
            const cd alpha = toc(tape[n].alpha), beta = toc(tape[n].beta);
            ReplayStep &rs = res->steps[(size_t)m * l + j];
            rs.flag = 2;
            rs.beta = tape[n].beta;
            rs.alpha = tape[n].alpha;
            // r_{j+1} <- S r_j
            rs.cr = fromc(lamR[j + 1]);
            lamR[j + 1] = 0.0;
            // r_i <- r_i - alpha u_{i+1}
            for (int i = 0; i <= j; ++i) lamU[i + 1] += -alpha * lamR[i];
            // shifts (program order: u^s_i update, x^s update, u^s_{j+1})
            for (int s = 0; s < ns; ++s) {
                const Sh &h = st[(size_t)n * ns + s];
                if (!h.live) continue;
                cd *lw = &lamW[(size_t)s * (l + 1)];
                const cd a1 = (h.kap - h.kapn) / h.as;
                const cd a2 = h.kapn * alpha / h.as;
                lamR[j] += a1 * lw[j + 1];
                lamU[j + 1] += a2 * lw[j + 1];
                lw[j] += -sp[s] * lw[j + 1];
                lw[j + 1] = 0.0;
                lw[0] += h.as * w[s];
                for (int i = 0; i <= j; ++i) {
                    lamR[i] += h.kap * lw[i];
                    lw[i] *= -h.bs;
                }
            }
            // u_{j+1} <- S u_j
            rs.cu = fromc(lamU[j + 1]);
            lamU[j + 1] = 0.0;
            // u_i <- r_i - beta u_i
            for (int i = 0; i <= j; ++i) {
                lamR[i] += lamU[i];
                lamU[i] *= -beta;
            }
        }
    }
    res->cb = lamR[0] + cb_extra;
    res->M = M;
}

// ---------------------------------------------------------------------------
// Stage emitter: the solve's stage sequence is written once and either
// launched stage by stage (LAUNCH), recorded as an operation table for the
// persistent kernel (RECORD), or only priced for the byte model (COUNT).
// ---------------------------------------------------------------------------
template <typename T>
struct Emit {
    enum Mode { LAUNCH, RECORD, COUNT };
    Ctx *c;
    hipStream_t st;
    Mode mode;
    bool count_bytes;                  // RECORD: add each op's bytes to the call's model
    std::vector<POp> ops;
    double cls_bytes[CL_COUNT] = {};   // RECORD / COUNT: bytes per timing class
    Emit(Ctx *c_, Mode m, bool cb = false) : c(c_), st(c_->stream), mode(m), count_bytes(cb) {}

    bool launching(int cls, double bytes) {
        if (mode == LAUNCH) return true;
        if (mode == COUNT || count_bytes) {
            c->bytes_acc += bytes;
            cls_bytes[cls] += bytes;
        }
        return false;
    }
    template <typename A>
    void record(POp o, const A &a) {
        static_assert(sizeof(A) <= POP_BLOB, "operation arguments exceed the blob");
        std::memcpy(o.blob, &a, sizeof(A));
        ops.push_back(o);
    }
    static POp op(int kind, int cls, int nvb) {
        POp o;
        std::memset(&o, 0, sizeof(o));
        o.kind = kind;
        o.cls = cls;
        o.nvb = nvb;
        return o;
    }
    void ds(DslashArgs<T> a, int nrhs, int epi, int cls, double bytes) {
        if (launching(cls, bytes)) {
            Prof p(c, cls, bytes);
            launch_dslash<T>(st, a, nrhs, epi, false);
        } else if (mode == RECORD) {
            POp o = op(OP_DS, cls, (int)dslash_prepare(a, nrhs));
            o.epi = epi;
            record(o, a);
        }
    }
    void ds64(DslashArgs<double> a, int nrhs, int epi, int cls, double bytes) {
        if (launching(cls, bytes)) {
            Prof p(c, cls, bytes);
            launch_dslash<double>(st, a, nrhs, epi, false);
        } else if (mode == RECORD) {
            POp o = op(OP_DS64, cls, (int)dslash_prepare(a, nrhs));
            o.epi = epi;
            record(o, a);
        }
    }
    // mode and fused (see launch_seed_u / launch_r_update) exist for the
    // per-stage launches only; the persistent kernel runs the plain stages
    void seed_u(const VecArgs<T> &a, int j, int nrhs, int nblk, int cls, double bytes, int umode = 0) {
        if (launching(cls, bytes)) {
            Prof p(c, cls, bytes);
            launch_seed_u<T>(st, a, j, nrhs, nblk, umode);
        } else if (mode == RECORD) {
            POp o = op(OP_SEED_U, cls, nblk * nrhs);
            o.j = j;
            o.nblk = nblk;
            record(o, a);
        }
    }
    void r_update(const VecArgs<T> &a, int j, bool shifts, bool xh, int nrhs, int nblk, int cls, double bytes,
                  bool fused = false) {
        if (launching(cls, bytes)) {
            Prof p(c, cls, bytes);
            launch_r_update<T>(st, a, j, shifts, xh, nrhs, nblk, fused);
        } else if (mode == RECORD) {
            POp o = op(OP_R_UPDATE, cls, nblk * nrhs);
            o.j = j;
            o.shifts = shifts ? 1 : 0;
            o.nblk = nblk;
            record(o, a);
        }
    }
    void gram(const VecArgs<T> &a, int nrhs, int nblk, int cls, double bytes) {
        if (launching(cls, bytes)) {
            Prof p(c, cls, bytes);
            launch_gram<T>(st, a, nrhs, nblk);
        } else if (mode == RECORD) {
            POp o = op(OP_GRAM, cls, nblk * nrhs);
            o.nblk = nblk;
            record(o, a);
        }
    }
    void mr_update(const VecArgs<T> &a, bool shifts, bool xh, int nrhs, int nblk, int cls, double bytes) {
        if (launching(cls, bytes)) {
            Prof p(c, cls, bytes);
            launch_mr_update<T>(st, a, shifts, xh, nrhs, nblk);
        } else if (mode == RECORD) {
            POp o = op(OP_MR_UPDATE, cls, nblk * nrhs);
            o.shifts = shifts ? 1 : 0;
            o.nblk = nblk;
            record(o, a);
        }
    }
    // <r~, x> from the sparse list of r~ (per-stage launches only; the
    // solver turns the sparse form off for the persistent launch)
    void sparse_dot(const SparseDotArgs &a, int nrhs, double bytes) {
        if (launching(CL_SCALAR, bytes)) {
            Prof p(c, CL_SCALAR, bytes);
            launch_sparse_dot(st, a, nrhs);
        }
    }
    void rel_update(const VecArgs<T> &a, const double2 *bb, const double2 *v, double2 *yy, CoefRef yc, int nrhs,
                    int nblk, int cls, double bytes) {
        if (launching(cls, bytes)) {
            Prof p(c, cls, bytes);
            launch_rel_update<T>(st, a, bb, v, yy, yc, nrhs, nblk);
        } else if (mode == RECORD) {
            POp o = op(OP_REL_UPDATE, cls, nblk * nrhs);
            o.nblk = nblk;
            o.b = bb;
            o.v = v;
            o.y = yy;
            o.yc = yc;
            record(o, a);
        }
    }
    // deferred single pass (per-stage launches only)
    void snapshot(const VecArgs<T> &a, int nrhs, int nblk, int cls, double bytes) {
        if (launching(cls, bytes)) {
            Prof p(c, cls, bytes);
            launch_snapshot<T>(st, a, nrhs, nblk);
        }
    }
    void defer_update(const VecArgs<T> &a, int nrhs, int nblk, int cls, double bytes) {
        if (launching(cls, bytes)) {
            Prof p(c, cls, bytes);
            launch_defer_update<T>(st, a, nrhs, nblk);
        }
    }
    // basis form of the seed (FP64, per-stage launches only)
    void basis_axpy(const BasisArgs<double> &a, int nrhs, int nblk, int cls, double bytes) {
        if (launching(cls, bytes)) {
            Prof p(c, cls, bytes);
            launch_basis_axpy(st, a, nrhs, nblk);
        }
    }
    void basis_r0norm(const BasisArgs<double> &a, int nrhs, int nblk, int cls, double bytes) {
        if (launching(cls, bytes)) {
            Prof p(c, cls, bytes);
            launch_basis_r0norm(st, a, nrhs, nblk);
        }
    }
    void basis_gram(const BasisArgs<double> &a, int nrhs, int nblk, int cls, double bytes) {
        if (launching(cls, bytes)) {
            Prof p(c, cls, bytes);
            launch_basis_gram(st, a, nrhs, nblk);
        }
    }
    void basis_mr_update(const BasisArgs<double> &a, int nrhs, int nblk, int cls, double bytes) {
        if (launching(cls, bytes)) {
            Prof p(c, cls, bytes);
            launch_basis_mr_update(st, a, nrhs, nblk);
        }
    }
    void basis_spec(const BasisArgs<double> &a, int nrhs) {
        if (launching(CL_SCALAR, 0.0)) {
            Prof p(c, CL_SCALAR, 0);
            launch_basis_spec(st, a, nrhs);
        }
    }
    void basis_combine(const BasisArgs<double> &a, int nrhs, int nblk, int cls, double bytes) {
        if (launching(cls, bytes)) {
            Prof p(c, cls, bytes);
            launch_basis_combine(st, a, nrhs, nblk);
        }
    }
    void basis_replay(const BasisReplayArgs &a, int nrhs) {
        if (launching(CL_SCALAR, 0.0)) {
            Prof p(c, CL_SCALAR, 0);
            launch_sc_basis_replay(st, a, nrhs);
        }
    }
    void scalar(int kind, const ScalarArgs &a, int nrhs) {
        if (launching(CL_SCALAR, 0.0)) {
            Prof p(c, CL_SCALAR, 0);
            switch (kind) {
            case OP_SC_BASIS: launch_sc_basis(st, a, nrhs); break;
            case OP_SC_EXH: launch_sc_exh(st, a, nrhs); break;
            case OP_SC_BETA: launch_sc_beta(st, a, nrhs); break;
            case OP_SC_ALPHA: launch_sc_alpha(st, a, nrhs); break;
            case OP_SC_MR: launch_sc_mr(st, a, nrhs); break;
            case OP_SC_REL: launch_sc_rel(st, a, nrhs); break;
            case OP_SC_CONV: launch_sc_conv(st, a, nrhs); break;
            case OP_SC_DEFER: launch_sc_defer(st, a, nrhs); break;
            default: break;
            }
        } else if (mode == RECORD) {
            record(op(kind, CL_SCALAR, nrhs), a);
        }
    }
};

// Runs an operation table in one cooperative launch: the table `iters` times
// (loop: until no right-hand side runs), then waits for it.  With the timing
// hook on, the kernel's per-class wall-clock stage times become records of
// the hook, priced with cls_bytes.
template <typename T>
static int run_persistent(Ctx *c, const std::vector<POp> &ops, int iters, bool loop, int l, const SeedState *seed,
                          int nrhs, const double *cls_bytes) {
    if (ops.empty()) return 0;
    hipStream_t st = c->stream;
    const int key = (sizeof(T) == sizeof(double) ? 0 : 1) * 16 + l;
    int &grid = c->pgrid[key];
    if (grid == 0) grid = persistent_grid<T>(c->device, l);
    if (grid < 8) return set_error(S_ERR_HIP, "persistent launch: no co-resident grid for l = " + std::to_string(l));
    CHK(ensure(c, c->ws_ops, ops.size() * sizeof(POp)));
    CHK(ensure(c, c->ws_pctl, sizeof(PersistCtl)));
    HIPCHK(hipMemcpyAsync(c->ws_ops.p, ops.data(), ops.size() * sizeof(POp), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(c->ws_pctl.p, 0, sizeof(PersistCtl), st));
    PersistArgs pa;
    pa.ops = (const POp *)c->ws_ops.p;
    pa.nops = (int)ops.size();
    pa.iters = iters;
    pa.loop = loop ? 1 : 0;
    pa.seed = seed;
    pa.nrhs = nrhs;
    pa.timing = c->prof ? 1 : 0;
    pa.ctl = (PersistCtl *)c->ws_pctl.p;
    HIPCHK(launch_persistent<T>(st, pa, grid, l));
    PersistCtl host;
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(&host, c->ws_pctl.p, sizeof(PersistCtl), hipMemcpyDeviceToHost));
    if (host.abort == 2)
        return set_error(S_ERR_HIP, "persistent launch: the XCD census found an XCD ID outside 0..7 or more blocks "
                                    "on one XCD than the barrier tree holds");
    if (host.abort) return set_error(S_ERR_HIP, "persistent launch: a grid barrier wait exceeded its bound");
    if (c->prof) {
        int khz = 0;
        HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device));
        const unsigned long long *tk = host.ticks, *ex = host.execs;
        for (int k = 0; k < CL_COUNT && k < PERSIST_CLASSES; ++k) {
            if (!ex[k]) continue;
            c->srecs.push_back(Ctx::SRec{k, (long long)ex[k], khz > 0 ? (double)tk[k] / khz : 0.0,
                                         cls_bytes ? cls_bytes[k] : 0.0});
        }
    }
    return 0;
}

// ---------------------------------------------------------------------------
// the multi-shift solve
// ---------------------------------------------------------------------------
template <typename T>
static int solve_impl(Ctx *c, const SolveParams &P, const double2 *b, double2 *y,
                      double2 *xs_out, bool want_true, SolveReport *rep) {
    hipStream_t st = c->stream;
    const int V = c->g.V;
    const long n = 12L * V;
    const int nrhs = P.nrhs, ns = P.n_shift, l = P.l;
    const bool pass1 = P.pass == 1;
    const bool pass3 = P.pass == 3;          // pseudo-double pass: keep every Mv output
    const int nbd = (V + CHUNK - 1) / CHUNK;     // stencil partials: one per 64-site chunk
    const int nbv = nblocks_for(n);
    const long ps = part_stride(c->g);
    const size_t cs = sizeof(C<T>);
    const int max_outer = P.max_outer;
    const int max_steps = max_outer * l;
    c->bytes_acc = 0;
    std::vector<POp> persist_ops1;   // operation table of the persistent first pass
    // algorithmic HBM bytes of one launch (each operand read or written once)
    const double cB = (double)cs, nd = (double)n, Vd = (double)V;
    bool sparse_rt = false;   // r~ read from its sparse list (see below)
    auto ds_bytes = [&](int epi, int nr) {
        double per = 24 * cB;                                  // in + out
        if (epi == EPI_MV) per = 48 * cB;                      // + v + rt
        else if (epi == EPI_MVN) per = 36 * cB;               // EPI_MV without rt
        else if (epi == EPI_MV_Y) per = 36 * cB + 24 * 16.0;   // + v, y (FP64) read + write
        else if (epi == EPI_SV) per = 36 * cB;                 // + v
        return nr * per * Vd + 36 * cB * Vd;                   // links once per launch
    };

    // ---- workspace: every buffer of the call is sized here, before the
    // first launch (the pseudo-double pass's store grows by chunks during
    // the first pass, and the persistent launch sizes its operation table
    // when it starts)
    const bool mixed = sizeof(T) != sizeof(double);
    const bool deferred = pass1 && P.deferred;
    const int nb = 2 * l + 2;                  // deferred: basis vectors per outer iteration
    const int wslots = deferred ? 1 : l + 1;   // shift vectors kept per shift
    constexpr int SPMAX = SPARSE_MAX;          // sparse shadow residual: entries per rhs
    constexpr int NBL = 256;                   // blocks of its scan
    CHK(ensure(c, c->ws_R, (size_t)nrhs * (l + 1) * n * cs));
    CHK(ensure(c, c->ws_U, (size_t)nrhs * (l + 1) * n * cs));
    CHK(ensure(c, c->ws_tmp, (size_t)nrhs * n * cs));
    CHK(ensure(c, c->ws_part, (size_t)nrhs * PMAX * ps * sizeof(double)));
    CHK(ensure(c, c->ws_seed, (size_t)nrhs * sizeof(SeedState)));
    CHK(ensure(c, c->ws_shift, (size_t)nrhs * NSMAX * sizeof(ShiftState)));
    CHK(ensure(c, c->ws_sc, (size_t)nrhs * NSMAX * sizeof(StepCoef)));
    CHK(ensure(c, c->ws_mc, (size_t)nrhs * NSMAX * sizeof(MRCoef)));
    CHK(ensure(c, c->ws_sig0, (size_t)nrhs * sizeof(double)));
    CHK(ensure(c, c->ws_wts, (size_t)nrhs * ns * sizeof(double)));
    if (mixed) {
        // FP32 copy of r~; FP64 seed solution and the FP64 Mv of the
        // reliable updates
        CHK(ensure(c, c->ws_rt, (size_t)nrhs * n * cs));
        CHK(ensure(c, c->ws_aux1, (size_t)nrhs * n * sizeof(double2)));
        CHK(ensure(c, c->ws_aux2, (size_t)nrhs * n * sizeof(double2)));
        CHK(ensure(c, c->ws_aux3, (size_t)nrhs * n * sizeof(double2)));
    }
    if (deferred) {
        CHK(ensure(c, c->ws_Bm, (size_t)nrhs * nb * n * cs));
        CHK(ensure(c, c->ws_schist, (size_t)nrhs * LMAX * NSMAX * sizeof(StepCoef)));
        CHK(ensure(c, c->ws_dc, (size_t)nrhs * NSMAX * sizeof(DeferCoef)));
    }
    if (pass1) {
        CHK(ensure(c, c->ws_W, (size_t)nrhs * ns * wslots * n * cs));
        if (!xs_out) CHK(ensure(c, c->ws_X, (size_t)nrhs * ns * n * sizeof(double2)));
        if (want_true) {
            CHK(ensure(c, c->ws_aux1, (size_t)nrhs * n * sizeof(double2)));
            CHK(ensure(c, c->ws_aux2, (size_t)nrhs * n * sizeof(double2)));
            CHK(ensure(c, c->ws_aux3, (size_t)nrhs * n * sizeof(double2)));
        }
    } else {
        CHK(ensure(c, c->ws_tape, (size_t)nrhs * max_steps * sizeof(TapeStep)));
        CHK(ensure(c, c->ws_tape_gam, (size_t)nrhs * max_outer * LMAX * sizeof(double2)));
        CHK(ensure(c, c->ws_tape_outer, (size_t)nrhs * max_outer * sizeof(TapeOuter)));
        // the replay program written after the sweep (at most max_outer
        // outer iterations)
        CHK(ensure(c, c->ws_replay, (size_t)nrhs * max_outer * l * sizeof(ReplayStep)));
        CHK(ensure(c, c->ws_replay_outer, (size_t)nrhs * max_outer * sizeof(ReplayOuter)));
        CHK(ensure(c, c->ws_cb, (size_t)nrhs * sizeof(double2)));
        if (pass3 && mixed) CHK(ensure(c, c->ws_ones, (size_t)nrhs * sizeof(double2)));
        if (pass3) {
            // the seed's state (r_0, u_0; x in FP64 with mixed precision) at
            // the first outer iteration whose Mv outputs the store cannot hold
            CHK(ensure(c, c->ws_hs, (size_t)nrhs * 2 * n * cs));
            if (mixed) CHK(ensure(c, c->ws_hs64, (size_t)nrhs * n * sizeof(double2)));
        }
    }
    // basis form of the seed: the two vectors each BiCG step feeds its Mv
    // (u_j, r_j after their updates) and the basis coefficients
    const bool basis = P.seed_basis && !mixed && !P.persistent && (!pass1 || deferred);
    if (basis) {
        CHK(ensure(c, c->ws_bw, (size_t)2 * nrhs * n * cs));
        CHK(ensure(c, c->ws_sb, (size_t)nrhs * sizeof(SeedBasis)));
    }
    if (!P.persistent)
        CHK(ensure(c, c->ws_sp, (size_t)nrhs * (SPMAX * (sizeof(long) + sizeof(double2)) + (1 + NBL) * sizeof(int)) +
                                    256));
    CHK(ensure_host(c, std::max((size_t)nrhs * sizeof(SeedState), (size_t)ps * sizeof(double))));

    C<T> *R = (C<T> *)c->ws_R.p, *Uv = (C<T> *)c->ws_U.p, *tmp = (C<T> *)c->ws_tmp.p;
    double *part = (double *)c->ws_part.p;
    SeedState *seed = (SeedState *)c->ws_seed.p;
    ShiftState *sh = (ShiftState *)c->ws_shift.p;
    const C<T> *rt;
    if (!mixed) {
        rt = (const C<T> *)(P.shadow ? P.shadow : b);
    } else {
        launch_convert_in<T>(st, (C<T> *)c->ws_rt.p, P.shadow ? P.shadow : b, n, n, n, nrhs);
        rt = (const C<T> *)c->ws_rt.p;
    }
    C<T> *W = nullptr;
    double2 *X = nullptr;
    double2 *XH = nullptr, *t64 = nullptr, *v64 = nullptr;
    if (mixed) {
        XH = (double2 *)c->ws_aux1.p;
        t64 = (double2 *)c->ws_aux2.p;
        v64 = (double2 *)c->ws_aux3.p;
    }
    C<T> *Bm = deferred ? (C<T> *)c->ws_Bm.p : nullptr;
    if (pass1) {
        W = (C<T> *)c->ws_W.p;
        X = xs_out ? xs_out : (double2 *)c->ws_X.p;
    } else {
        HIPCHK(hipMemsetAsync(c->ws_tape.p, 0, (size_t)nrhs * max_steps * sizeof(TapeStep), st));
        HIPCHK(hipMemsetAsync(c->ws_tape_outer.p, 0, (size_t)nrhs * max_outer * sizeof(TapeOuter), st));
    }

    // ---- host-side initial state
    std::vector<SeedState> hs(nrhs);
    std::vector<ShiftState> hsh((size_t)nrhs * NSMAX);
    std::vector<double> sig0(nrhs);
    for (int r = 0; r < nrhs; ++r) {
        const double *sg = &P.shifts[(size_t)r * ns];
        sig0[r] = *std::min_element(sg, sg + ns);
        SeedState &S = hs[r];
        std::memset(&S, 0, sizeof(S));
        S.tol = P.tol_rhs.empty() ? P.tol : P.tol_rhs[r];
        S.nshift = ns;
        S.max_outer = max_outer;
        S.max_steps = max_steps;
        S.forced = P.force_iters ? 1 : 0;
        S.mixed = mixed ? 1 : 0;
        for (int s = 0; s < ns; ++s) {
            ShiftState &H = hsh[(size_t)r * NSMAX + s];
            std::memset(&H, 0, sizeof(H));
            H.zeta = d2(1, 0);
            H.zeta_prev = d2(1, 0);
            H.pi_prev = d2(0, 0);
            H.psi = d2(1, 0);
            H.sp = sg[s] - sig0[r];
            H.res = INFINITY;
            H.active = 1;
            H.force = P.force_iters ? P.force_iters[(size_t)r * ns + s] : 0;
        }
    }
    HIPCHK(hipMemcpyAsync(seed, hs.data(), nrhs * sizeof(SeedState), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(sh, hsh.data(), hsh.size() * sizeof(ShiftState), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(c->ws_sig0.p, sig0.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(c->ws_wts.p, P.weights.data(), (size_t)nrhs * ns * sizeof(double),
                          hipMemcpyHostToDevice, st));

    // ---- initial vectors: r_0 = b, everything else zero
    {
        Prof p(c, CL_OTHER, nrhs * nd * cB * (2.0 * (l + 1) + (pass1 ? ns * (double)wslots : 0.0)) +
                                (pass1 ? nrhs * nd * ns * 16.0 : 0.0) + (mixed ? nrhs * nd * 16.0 : 0.0) +
                                nrhs * nd * (16.0 + cB) + nrhs * nd * cB);
        if (basis) {
            // the basis form reads rows 1..l of R and U only where a step of
            // the current outer iteration wrote them: u_0 = 0 is all it needs
            launch_zero<T>(st, Uv, n, vs, nrhs);
        } else {
            launch_zero<T>(st, R, (long)nrhs * (l + 1) * n, 0, 1);
            launch_zero<T>(st, Uv, (long)nrhs * (l + 1) * n, 0, 1);
        }
        if (pass1) {
            launch_zero<T>(st, W, (long)nrhs * ns * wslots * n, 0, 1);
            launch_zero<double>(st, X, (long)nrhs * ns * n, 0, 1);
        }
        if (mixed) launch_zero<double>(st, XH, (long)nrhs * n, 0, 1);
        launch_convert_in<T>(st, R, b, n, (long)(l + 1) * n, n, nrhs);
        if (!P.shadow) {
            // r~ = b: <r~, r_0> and ||b||^2 in one pass
            launch_dot_partials<T>(st, rt, rt, n, part, ps, nrhs, nbv, Gate{});
        } else {
            // <r~, r_0> and ||b||^2 (rows 0..2), ||r~||^2 (row 5)
            const C<T> *r0 = (const C<T> *)b;
            if (sizeof(T) != sizeof(double)) {
                launch_convert_in<T>(st, tmp, b, n, n, n, nrhs);
                r0 = tmp;
            }
            launch_dot_partials<T>(st, rt, r0, n, part, ps, nrhs, nbv, Gate{});
            launch_dot_partials<T>(st, rt, rt, n, part + 3 * ps, ps, nrhs, nbv, Gate{});
        }
    }
    // A shadow residual with few nonzero entries (r~ = b for a point source
    // has one per right-hand side): the Mv epilogue and the MR update skip
    // their full read of r~ and <r~, .> is summed from an index list in a
    // one-wavefront kernel after them.  FP64 per-stage launches only.
    SparseDotArgs spa;
    if (!P.persistent) {
        long *spi = (long *)c->ws_sp.p;
        double2 *spv = (double2 *)(spi + (size_t)nrhs * SPMAX);
        int *spc = (int *)(spv + (size_t)nrhs * SPMAX);
        int *spw = spc + nrhs;
        // from the FP64 r~ (mixed precision: values rounded as in its FP32 copy)
        const int worst = sparse_list(st, P.shadow ? P.shadow : b, n, n, nrhs, SPMAX, spi, spv, spc, spw, NBL,
                                      mixed);
        if (worst < 0) return set_error(S_ERR_HIP, "scan of the shadow residual for nonzero entries failed");
        sparse_rt = worst <= SPMAX;
        spa.idx = spi;
        spa.val = spv;
        spa.cnt = spc;
        spa.spmax = SPMAX;
        spa.part = part;
        spa.ps = ps;
        spa.fp32 = mixed ? 1 : 0;
    }
    ScalarArgs sa;
    sa.seed = seed;
    sa.sh = sh;
    sa.sc = (StepCoef *)c->ws_sc.p;
    sa.mc = (MRCoef *)c->ws_mc.p;
    sa.tape = pass1 ? nullptr : (TapeStep *)c->ws_tape.p;
    sa.tape_gam = pass1 ? nullptr : (double2 *)c->ws_tape_gam.p;
    sa.tape_outer = pass1 ? nullptr : (TapeOuter *)c->ws_tape_outer.p;
    sa.part = part;
    sa.ps = ps;
    sa.l = l;
    sa.record = pass1 ? 0 : 1;            // the double and pseudo-double passes record the tape
    sa.nblk = nbv;
    sa.shadow = P.shadow ? 1 : 0;
    if (basis) {
        // ||S|| <= a ||D||^2 + max |sigma0| (a ||D|| + ... for A = a D), with
        // ||D|| <= |4 + m| + L (3 + exp|mu|), L the links' norm bound: the
        // hops along nu are P- A + P+ B with orthogonal spin projectors
        // P-+ = (1 -+ gamma_nu) / 2 and A, B a link times a shift, which act
        // on colour and site and so commute with them; hence
        // ||(P- A + P+ B) v||^2 = ||A P- v||^2 + ||B P+ v||^2
        //                       <= L^2 (||P- v||^2 + ||P+ v||^2) = L^2 ||v||^2,
        // with A, B scaled by exp(+-mu) in time (the free field reaches the
        // bound: |4 + m| + 4 at momentum pi in every direction, mu = 0)
        const double dn = std::fabs(4.0 + c->mass) + c->link_norm * (3.0 + std::exp(std::fabs(c->mu)));
        double s0 = 0.0;
        for (int r = 0; r < nrhs; ++r)
            s0 = std::max(s0, std::fabs(*std::min_element(&P.shifts[(size_t)r * ns], &P.shifts[(size_t)r * ns] + ns)));
        sa.basis = 1;
        sa.spec = sparse_rt ? 1 : 0;
        sa.norm_a = (P.op_wilson ? P.a_scale * dn : P.a_scale * dn * dn) + s0;
        sa.sb = (SeedBasis *)c->ws_sb.p;
    }
    if (deferred) {
        sa.sc_hist = (StepCoef *)c->ws_schist.p;
        sa.dc = (DeferCoef *)c->ws_dc.p;
    }
    {
        Prof p(c, CL_SCALAR, 0);
        launch_sc_init(st, sa, nrhs);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));

    // ---- argument blocks
    VecArgs<T> va;
    va.n = n;
    va.l = l;
    va.nshift = ns;
    va.R = R;
    va.U = Uv;
    va.W = W;
    va.X = X;
    va.XH = XH;
    va.rt = sparse_rt ? nullptr : rt;
    va.part = part;
    va.ps = ps;
    va.seed = seed;
    va.sc = sa.sc;
    va.mc = sa.mc;
    va.beta = CoefRef{(const char *)&seed[0].beta, (long)sizeof(SeedState)};
    va.alpha = CoefRef{(const char *)&seed[0].alpha, (long)sizeof(SeedState)};
    va.gam = CoefRef{(const char *)&seed[0].gam[0], (long)sizeof(SeedState)};
    if (deferred) {
        va.Bm = Bm;
        va.W0 = W;
        va.dc = (const DeferCoef *)c->ws_dc.p;
    }
    const bool shifts_step = pass1 && !deferred;   // shift vectors updated in every step
    Gate g_bicg;
    g_bicg.seed = seed;
    g_bicg.need_bicg = 1;
    Gate g_run;
    g_run.seed = seed;
    const long vs = (long)(l + 1) * n;   // rhs stride of R and U
    DslashArgs<T> d1 = ds_args<T>(c, P.neg_mu, true);
    d1.in_rs = vs;
    d1.out_rs = n;
    // A = a (g5 D)^2: two stencils per Mv (g5 D into tmp, then a g5 D tmp +
    // sigma0 v); A = a D (MSB_OP_WILSON): one stencil straight from the vector
    const bool opw = P.op_wilson;
    DslashArgs<T> d2 = d1;
    d2.scale = (T)P.a_scale;
    d2.sigma0_rhs = (const double *)c->ws_sig0.p;
    d2.in_rs = opw ? vs : n;
    if (opw) d2.g5out = 0;
    d2.out_rs = vs;
    d2.v_rs = vs;
    d2.rt = sparse_rt ? nullptr : rt;
    d2.rt_rs = n;
    d2.part = part;
    d2.ps = ps;

    // FP64 Mv of the reliable updates: v = a g5 D (g5 D x) + sigma0 x
    Gate g_rel;
    g_rel.seed = seed;
    g_rel.flag = &seed[0].rel;
    g_rel.flag_stride = (long)sizeof(SeedState) / (long)sizeof(int);
    g_rel.need = 1;
    DslashArgs<double> r1 = ds_args<double>(c, P.neg_mu, true);
    r1.in = XH;
    r1.out = t64;
    r1.gate = g_rel;
    DslashArgs<double> r2 = ds_args<double>(c, P.neg_mu, !opw);
    r2.in = opw ? XH : t64;
    r2.out = v64;
    r2.v = XH;
    r2.scale = P.a_scale;
    r2.sigma0_rhs = (const double *)c->ws_sig0.p;
    r2.gate = g_rel;
    const double ds64_plain = nrhs * 24 * 16.0 * Vd + 36 * 16.0 * Vd;
    const double ds64_sv = nrhs * 36 * 16.0 * Vd + 36 * 16.0 * Vd;
    auto reliable_update = [&](Emit<T> &e, const VecArgs<T> &vv, Gate g, double2 *yacc, CoefRef yc, int nr) {
        DslashArgs<double> q1 = r1, q2 = r2;
        q1.gate = g;
        q2.gate = g;
        if (!opw) e.ds64(q1, nrhs, EPI_PLAIN, CL_STENCIL, ds64_plain * nr / std::max(nrhs, 1));
        e.ds64(q2, nrhs, EPI_SV, CL_STENCIL, ds64_sv * nr / std::max(nrhs, 1));
        VecArgs<T> w = vv;
        w.gate = g;
        e.rel_update(w, b, v64, yacc, yc, nrhs, nbv, CL_SEED,
                     nr * nd * (32.0 + (sparse_rt ? 0.0 : cB) + cB + (yacc ? 32.0 : 0.0)));
        if (sparse_rt) {   // <r~, b - S x> from the list, as the update would have formed it
            SparseDotArgs a = spa;
            a.b = b;
            a.v = v64;
            a.x_rs = n;
            a.gate = g;
            e.sparse_dot(a, nrhs, nr * SPMAX * (8.0 + 16.0 + 32.0));
        }
    };

    // One outer iteration of the first pass: l BiCG steps, the MR step, the
    // reliable update (mixed) and the convergence step.  nr_run and nsh_act
    // (right-hand sides and shifts still iterating) only price the bytes.
    // pseudo-double pass: every Mv output of outer iteration m goes to slot
    // (m mod PSC) of storage chunk m / PSC, [rhs][PSC][2l][n]; with mixed
    // precision also the FP64 S x of its reliable update, [PSC][rhs][n]
    constexpr int PSC = 8;
    const long ps_rs = (long)PSC * 2 * l * n;
    // Storage chunk k for outer iterations k PSC .. k PSC + PSC - 1: false
    // when it would pass the context's store limit or cannot be allocated;
    // the solve then stores no further iteration (m_split) and regenerates
    // those after the sweep from the seed state saved where the store ended:
    // the pseudo-double pass where memory allows, the double pass beyond.
    const size_t chunk_bytes = (size_t)nrhs * ps_rs * cs + (mixed ? (size_t)nrhs * PSC * n * sizeof(double2) : 0);
    auto pstore_chunk = [&](int k) -> bool {
        if (c->store_limit && (size_t)(k + 1) * chunk_bytes > c->store_limit) return false;
        while ((int)c->pstore.size() <= k) c->pstore.push_back(DevBuf{});
        if (ensure(c, c->pstore[k], (size_t)nrhs * ps_rs * cs)) return false;
        if (mixed) {
            while ((int)c->prel.size() <= k) c->prel.push_back(DevBuf{});
            if (ensure(c, c->prel[k], (size_t)nrhs * PSC * n * sizeof(double2))) return false;
            launch_zero<double>(st, (double2 *)c->prel[k].p, (long)nrhs * PSC * n, 0, 1);
        }
        return true;
    };
    int m_split = max_outer;       // pass 3: the first outer iteration not stored
    if (pass3 && mixed) {
        CHK(ensure(c, c->ws_ones, (size_t)nrhs * sizeof(double2)));
        std::vector<double2> ones(nrhs, double2{1.0, 0.0});
        HIPCHK(hipMemcpyAsync(c->ws_ones.p, ones.data(), nrhs * sizeof(double2), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    }

    // <r~, x> for x = [rhs] rows at the seed-vector stride, into the partial
    // slots the preceding kernel left at zero
    auto sparse_dot_of = [&](Emit<T> &e, const void *x, const Gate &g, int nr_run, long x_rs) {
        SparseDotArgs a = spa;
        a.x = x;
        a.x_rs = x_rs;
        a.gate = g;
        e.sparse_dot(a, nrhs, nr_run * SPMAX * (8.0 + 16.0 + 16.0));
    };
    // pass 3 and the deferred single pass write each Mv output to their store
    // (or basis) slot only; the seed kernels read it from there until its
    // first update
    const int mv_epi = sparse_rt ? EPI_MVN : EPI_MV;
    const bool fuse_seed = !P.persistent;   // fused direction updates (per-stage launches)
    auto emit_outer = [&](Emit<T> &e, int nr_run, double nsh_act, int m) {
        VecArgs<T> v = va;
        ScalarArgs s = sa;
        DslashArgs<T> e1 = d1, e2 = d2;
        if (deferred) {
            // the iteration's basis starts with r_0 and u_0
            v.gate = g_run;
            e.snapshot(v, nrhs, nbv, CL_SHIFT, nr_run * 4.0 * nd * cB);
        }
        // Mv output t of this outer iteration (t = 2j: u_{j+1}, 2j + 1:
        // r_{j+1}): its slot in the pass-3 store, or in the deferred single
        // pass's basis (after B_0 = r_0, B_1 = u_0)
        const bool keep = pass3 && m < m_split;   // pass 3: this iteration's outputs are stored
        const bool stored = keep || deferred;
        const long store_rs = pass3 ? ps_rs : (long)nb * n;
        auto slot = [&](int t) {
            return pass3 ? (C<T> *)c->pstore[m / PSC].p + ((size_t)(m % PSC) * 2 * l + t) * n
                         : Bm + (size_t)(2 + t) * n;
        };
        auto from_store = [&](VecArgs<T> &x, int ri, int ui) {
            x.r_src_i = (stored && ri >= 1) ? ri : -1;
            x.u_src_i = (stored && ui >= 1) ? ui : -1;
            if (x.r_src_i >= 1) x.r_src = slot(2 * (ri - 1) + 1);
            if (x.u_src_i >= 1) x.u_src = slot(2 * (ui - 1));
            x.r_src_rs = x.u_src_rs = store_rs;
        };
        if constexpr (std::is_same<T, double>::value) {
            if (basis) {
                // basis form of the seed: each step updates only the two
                // vectors its Mv read (into the work vectors WU, WR); the
                // iteration's r_i and u_i are coefficients on its basis B
                // (B_0 = r_0, B_1 = u_0 at the start, the Mv outputs after:
                // the store slots of pass 3 or the deferred single pass's
                // basis slots, else rows 1..l of U and R), formed from it
                // for the Gram matrix and the MR update
                BasisArgs<double> ba;
                ba.n = n;
                ba.l = l;
                ba.sb = (const SeedBasis *)c->ws_sb.p;
                ba.seed = seed;
                ba.part = part;
                ba.ps = ps;
                ba.bv[0] = R;
                ba.brs[0] = vs;
                ba.bv[1] = Uv;
                ba.brs[1] = vs;
                for (int j = 0; j < l; ++j) {
                    ba.bv[2 + 2 * j] = stored ? slot(2 * j) : Uv + (size_t)(j + 1) * n;
                    ba.bv[3 + 2 * j] = stored ? slot(2 * j + 1) : R + (size_t)(j + 1) * n;
                    ba.brs[2 + 2 * j] = ba.brs[3 + 2 * j] = stored ? store_rs : vs;
                }
                double2 *WU = (double2 *)c->ws_bw.p, *WR = WU + (size_t)nrhs * n;
                Gate g_exh;
                g_exh.seed = seed;
                g_exh.need_bicg = 1;
                g_exh.flag = &seed[0].exh_check;
                g_exh.flag_stride = (long)sizeof(SeedState) / (long)sizeof(int);
                g_exh.need = 1;
                g_exh.eq = 1;
                for (int j = 0; j < l; ++j) {
                    s.j = j;
                    s.nblk2 = nbv;
                    if (j >= 1) {
                        // could this step's exhaustion test fire?  Then r_0
                        // after step j-1 (in B_0 .. B_2j) and its norm
                        e.scalar(OP_SC_EXH, s, nrhs);
                        BasisArgs<double> bn = ba;
                        bn.gate = g_exh;
                        bn.nbu = 2 * j + 1;
                        e.basis_r0norm(bn, nrhs, nbv, CL_SEED, 0.0);
                    }
                    s.nblk = (j == 0) ? nbv : nbd;
                    e.scalar(OP_SC_BETA, s, nrhs);
                    const int xi = (j == 0) ? 0 : 2 * j + 1;   // r_j before this step
                    const int yi = (j == 0) ? 1 : 2 * j;       // u_j before this step
                    // u_j = r_j - beta u_j (at j = 0 made by the previous MR
                    // update where its beta was this step's)
                    BasisArgs<double> bu = ba;
                    bu.gate = g_bicg;
                    if (j == 0 && sa.spec) {
                        bu.gate.flag = &seed[0].wu_ready;
                        bu.gate.flag_stride = (long)sizeof(SeedState) / (long)sizeof(int);
                        bu.gate.need = 0;
                        bu.gate.eq = 1;
                    }
                    bu.dst = WU;
                    bu.dst_rs = n;
                    bu.x = ba.bv[xi];
                    bu.x_rs = ba.brs[xi];
                    bu.y = ba.bv[yi];
                    bu.y_rs = ba.brs[yi];
                    bu.c = va.beta;
                    const bool made = j == 0 && sa.spec && m > 0;   // left out (unless the betas differ)
                    e.basis_axpy(bu, nrhs, nbv, CL_SEED, made ? 0.0 : nr_run * 3.0 * nd * cB);
                    // u_{j+1} = S u_j into B_{2+2j}
                    DslashArgs<T> f1 = d1, f2 = d2;
                    f1.in = WU;
                    f1.in_rs = n;
                    f1.out = tmp;
                    f1.gate = g_bicg;
                    if (!opw) e.ds(f1, nrhs, EPI_PLAIN, CL_STENCIL, ds_bytes(EPI_PLAIN, nr_run));
                    f2.in = opw ? WU : tmp;
                    f2.in_rs = n;
                    f2.out = (C<T> *)ba.bv[2 + 2 * j];
                    f2.out_rs = ba.brs[2 + 2 * j];
                    f2.v = WU;
                    f2.v_rs = n;
                    f2.gate = g_bicg;
                    e.ds(f2, nrhs, mv_epi, CL_STENCIL, ds_bytes(mv_epi, nr_run));
                    if (sparse_rt) sparse_dot_of(e, f2.out, f2.gate, nr_run, f2.out_rs);
                    s.nblk = nbd;
                    e.scalar(OP_SC_ALPHA, s, nrhs);
                    // r_j = r_j - alpha u_{j+1}, ||r_j||^2 into row 4
                    BasisArgs<double> br = ba;
                    br.gate = g_bicg;
                    br.dst = WR;
                    br.dst_rs = n;
                    br.x = ba.bv[xi];
                    br.x_rs = ba.brs[xi];
                    br.y = ba.bv[2 + 2 * j];
                    br.y_rs = ba.brs[2 + 2 * j];
                    br.c = va.alpha;
                    br.prow = 4;
                    e.basis_axpy(br, nrhs, nbv, CL_SEED, nr_run * 3.0 * nd * cB);
                    // r_{j+1} = S r_j into B_{3+2j}
                    f1.in = WR;
                    if (!opw) e.ds(f1, nrhs, EPI_PLAIN, CL_STENCIL, ds_bytes(EPI_PLAIN, nr_run));
                    f2.in = opw ? WR : tmp;
                    f2.out = (C<T> *)ba.bv[3 + 2 * j];
                    f2.out_rs = ba.brs[3 + 2 * j];
                    f2.v = WR;
                    e.ds(f2, nrhs, mv_epi, CL_STENCIL, ds_bytes(mv_epi, nr_run));
                    if (sparse_rt) sparse_dot_of(e, f2.out, f2.gate, nr_run, f2.out_rs);
                }
                // the MR step from the basis
                s.nblk = nbv;
                e.scalar(OP_SC_BASIS, s, nrhs);
                const int nbg = std::min(nbv, GRAM_NBMAX);
                BasisArgs<double> bg = ba;
                bg.gate = g_run;
                e.basis_gram(bg, nrhs, nbg, CL_SEED, nr_run * (2.0 * l + 1) * nd * cB);   // all but B_1
                s.nblk = nbg;
                e.scalar(OP_SC_MR, s, nrhs);
                s.nblk = nbv;
                BasisArgs<double> bm = ba;
                bm.gate = g_run;
                bm.R0 = R;
                bm.r0_rs = vs;
                bm.U0 = Uv;
                bm.u0_rs = vs;
                bm.rt = sparse_rt ? nullptr : rt;
                if (sa.spec) {
                    // with the sparse r~: <r~, r_0> and the next outer
                    // iteration's beta from the basis before the MR update
                    // overwrites r_0 and u_0, then the update also makes that
                    // iteration's first direction update
                    bm.seed_w = seed;
                    bm.sp_idx = spa.idx;
                    bm.sp_val = spa.val;
                    bm.sp_cnt = spa.cnt;
                    bm.sp_max = spa.spmax;
                    e.basis_spec(bm, nrhs);
                    bm.wu = WU;
                }
                // 2l + 2 basis vectors read, r_0 and u_0 written, and r~ read
                // (dense) or the next u_0 update written (sparse)
                e.basis_mr_update(bm, nrhs, nbv, CL_SEED, nr_run * (2.0 * l + 5) * nd * cB);
                if (sparse_rt && !sa.spec) sparse_dot_of(e, R, g_run, nr_run, vs);
                if (deferred) {
                    // every shift's update over the iteration from the basis
                    // (B_0, B_1 from the snapshot: the MR update has just
                    // overwritten r_0 and u_0)
                    e.scalar(OP_SC_DEFER, s, nrhs);
                    v.gate = g_run;
                    e.defer_update(v, nrhs, nbv, CL_SHIFT_MR, nr_run * nb * nd * cB + nsh_act * (2.0 * cB + 32.0) * nd);
                }
                e.scalar(OP_SC_CONV, s, nrhs);
                return;
            }
        }
        for (int j = 0; j < l; ++j) {
            s.j = j;
            s.nblk = (j == 0) ? nbv : nbd;
            s.nblk2 = nbv;
            e.scalar(OP_SC_BETA, s, nrhs);
            v.gate = g_bicg;
            from_store(v, j, j);     // r_j and u_j: this step's first update of both
            // fused form: only u_j before its Mv; u_0..u_{j-1} in the r-update
            const bool fu = fuse_seed && j >= 1;
            e.seed_u(v, j, nrhs, nbv, CL_SEED, nr_run * (fu ? 3.0 : 3.0 * (j + 1)) * nd * cB, fu ? 1 : 0);
            // u_{j+1} = S u_j = a g5 D (g5 D u_j) + sigma0 u_j, <rt, u_{j+1}>
            e1.in = Uv + (size_t)j * n;
            e1.out = tmp;
            e1.gate = g_bicg;
            if (!opw) e.ds(e1, nrhs, EPI_PLAIN, CL_STENCIL, ds_bytes(EPI_PLAIN, nr_run));
            e2.in = opw ? Uv + (size_t)j * n : tmp;
            e2.out = Uv + (size_t)(j + 1) * n;
            e2.v = Uv + (size_t)j * n;
            e2.gate = g_bicg;
            if (stored) {
                e2.out = slot(2 * j);
                e2.out_rs = store_rs;
            }
            e.ds(e2, nrhs, mv_epi, CL_STENCIL, ds_bytes(mv_epi, nr_run));
            if (sparse_rt) sparse_dot_of(e, e2.out, e2.gate, nr_run, stored ? store_rs : vs);
            s.nblk = nbd;
            e.scalar(OP_SC_ALPHA, s, nrhs);
            v.partials = 1;
            from_store(v, j, j + 1);     // r_j (first update) and u_{j+1} (read only)
            // seed: read r_i, u_{i+1}, write r_i; shift s (per-step form): read
            // u^s_0..j, x^s (FP64), write u^s_0..j+1, x^s
            e.r_update(v, j, shifts_step, mixed, nrhs, nbv, shifts_step ? CL_SHIFT : CL_SEED,
                       nr_run * ((fu ? 4.0 * j + 4 : 3.0 * (j + 1)) * cB + (mixed ? 32.0 : 0.0)) * nd +
                           (shifts_step ? nsh_act * ((2.0 * j + 3) * cB + 32.0) * nd : 0.0),
                       fu);
            if (fu) {
                // a step that ended after its u-Mv (alpha breakdown) still
                // owes u_0..u_{j-1} their update, which the partial MR step reads
                VecArgs<T> vc = v;
                vc.gate = g_run;
                vc.gate.flag = &seed[0].step_flag[j];
                vc.gate.flag_stride = (long)sizeof(SeedState) / (long)sizeof(int);
                vc.gate.need = 1;
                vc.gate.eq = 1;
                e.seed_u(vc, j, nrhs, nbv, CL_SEED, 0.0, 2);
            }
            // r_{j+1} = S r_j, <rt, r_{j+1}>
            e1.in = R + (size_t)j * n;
            if (!opw) e.ds(e1, nrhs, EPI_PLAIN, CL_STENCIL, ds_bytes(EPI_PLAIN, nr_run));
            else e2.in = R + (size_t)j * n;
            e2.out = R + (size_t)(j + 1) * n;
            e2.v = R + (size_t)j * n;
            if (stored) e2.out = slot(2 * j + 1);
            e.ds(e2, nrhs, mv_epi, CL_STENCIL, ds_bytes(mv_epi, nr_run));
            if (sparse_rt) sparse_dot_of(e, e2.out, e2.gate, nr_run, stored ? store_rs : vs);
        }
        v.gate = g_run;
        // the MR step reads r_L and u_L (L = the steps the iteration
        // completed, l unless a breakdown ended it early) from the store
        // where no step updated them since
        from_store(v, -1, -1);
        if (stored) {
            v.mr_dyn = 1;
            v.st_base = slot(0);
            v.st_rs = store_rs;
        }
        // the Gram matrix: (l+1)(l+2) partial sums per block, so fewer,
        // longer blocks than the other seed kernels (their reduction and
        // scattered partial stores would otherwise dominate the pass)
        const int nbg = std::min(nbv, GRAM_NBMAX);
        e.gram(v, nrhs, nbg, CL_SEED, nr_run * (l + 1.0) * nd * cB);
        s.nblk = nbg;
        e.scalar(OP_SC_MR, s, nrhs);
        s.nblk = nbv;   // the stages below read the MR update's nbv partials
        v.partials = 1;
        // seed: read r_0..r_l, u_0..u_l, rt, write r_0, u_0; shift s: read
        // u^s_0..u^s_l, x^s, write u^s_0, x^s
        e.mr_update(v, shifts_step, mixed, nrhs, nbv, shifts_step ? CL_SHIFT_MR : CL_SEED,
                    nr_run * ((2.0 * (l + 1) + (sparse_rt ? 2 : 3)) * cB + (mixed ? 32.0 : 0.0)) * nd +
                        (shifts_step ? nsh_act * ((l + 2.0) * cB + 32.0) * nd : 0.0));
        if (sparse_rt) sparse_dot_of(e, R, v.gate, nr_run, vs);
        v.mr_dyn = 0;
        if (deferred) {
            // every shift's update over the iteration, from the basis: read the
            // 2l+2 basis vectors once, each active shift's u^s_0 and x^s (FP64)
            // read and written
            e.scalar(OP_SC_DEFER, s, nrhs);
            v.gate = g_run;
            e.defer_update(v, nrhs, nbv, CL_SHIFT_MR, nr_run * nb * nd * cB + nsh_act * (2.0 * cB + 32.0) * nd);
        }
        if (mixed) {
            e.scalar(OP_SC_REL, s, nrhs);
            if (keep)   // keep S x of the update: slot += 1 * S x (the slot starts at zero)
                reliable_update(e, v, g_rel, (double2 *)c->prel[m / PSC].p + (size_t)(m % PSC) * nrhs * n,
                                CoefRef{(const char *)c->ws_ones.p, (long)sizeof(double2)}, nr_run);
            else
                reliable_update(e, v, g_rel, nullptr, CoefRef{}, nr_run);
        }
        e.scalar(OP_SC_CONV, s, nrhs);
    };

    CHK(ensure_host(c, (size_t)nrhs * sizeof(SeedState)));
    SeedState *hseed = (SeedState *)c->host_pinned;
    if (P.persistent) {
        // the whole first pass in one cooperative launch
        Emit<T> er(c, Emit<T>::RECORD);
        emit_outer(er, nrhs, (double)nrhs * ns, 0);
        std::vector<POp> ops = std::move(er.ops);
        persist_ops1.swap(ops);
        CHK(run_persistent<T>(c, persist_ops1, max_outer, true, l, seed, nrhs, nullptr));
    } else {
        int nr_run = nrhs;                       // right-hand sides still iterating
        double nsh_act = (double)nrhs * ns;      // active shifts over those
        Emit<T> el(c, Emit<T>::LAUNCH);
        for (int m = 0; m < max_outer; ++m) {
            if (pass3 && m < m_split && m % PSC == 0 && !pstore_chunk(m / PSC)) {
                (void)hipGetLastError();
                m_split = m;
                // the seed's state at the start of outer iteration m, for the replay
                HIPCHK(hipMemcpy2DAsync(c->ws_hs.p, n * cs, R, vs * cs, n * cs, nrhs, hipMemcpyDeviceToDevice, st));
                HIPCHK(hipMemcpy2DAsync((char *)c->ws_hs.p + (size_t)nrhs * n * cs, n * cs, Uv, vs * cs, n * cs, nrhs,
                                        hipMemcpyDeviceToDevice, st));
                if (mixed)
                    HIPCHK(hipMemcpyAsync(c->ws_hs64.p, XH, (size_t)nrhs * n * sizeof(double2),
                                          hipMemcpyDeviceToDevice, st));
            }
            emit_outer(el, nr_run, nsh_act, m);
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(hseed, seed, nrhs * sizeof(SeedState), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            nr_run = 0;
            nsh_act = 0;
            for (int r = 0; r < nrhs; ++r) {
                if (hseed[r].run) {
                    nr_run += 1;
                    nsh_act += hseed[r].nact;
                }
            }
            if (nr_run == 0) break;
        }
    }

    // ---- results of pass 1
    std::vector<SeedState> fs(nrhs);
    std::vector<ShiftState> fsh((size_t)nrhs * NSMAX);
    HIPCHK(hipMemcpy(fs.data(), seed, nrhs * sizeof(SeedState), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(fsh.data(), sh, fsh.size() * sizeof(ShiftState), hipMemcpyDeviceToHost));

    if (P.persistent) {
        // byte model of the persistent first pass, priced per outer iteration
        // with the right-hand sides and shifts that took part in it
        int Mrun = 0;
        for (int r = 0; r < nrhs; ++r) Mrun = std::max(Mrun, fs[r].m);
        Emit<T> ec(c, Emit<T>::COUNT);
        for (int m = 0; m < Mrun; ++m) {
            int nr = 0;
            double nsh = 0;
            for (int r = 0; r < nrhs; ++r) {
                if (fs[r].m <= m) continue;
                nr += 1;
                for (int s = 0; s < ns; ++s) nsh += (fsh[(size_t)r * NSMAX + s].iters > m) ? 1.0 : 0.0;
            }
            emit_outer(ec, nr, nsh, m);
        }
        if (c->prof) {
            // attach the bytes to the stage times the kernel reported
            for (Ctx::SRec &q : c->srecs)
                if (q.bytes == 0.0 && q.cls >= 0 && q.cls < CL_COUNT && q.pending) q.bytes = ec.cls_bytes[q.cls];
            for (Ctx::SRec &q : c->srecs) q.pending = false;
        }
    }

    rep->status = S_OK;
    rep->outer_max = 0;
    rep->steps_max = 0;
    rep->mv = 0;
    rep->dots = 0;
    rep->reliable = 0;
    rep->shift_iters.assign((size_t)nrhs * ns, 0);
    rep->shift_resid.assign((size_t)nrhs * ns, 0.0);
    rep->rhs_outer.assign(nrhs, 0);
    for (int r = 0; r < nrhs; ++r) {
        const SeedState &S = fs[r];
        int status = S.status;
        if (S.run) status = S_NOT_CONVERGED;   // max_outer reached without the device noticing
        if (status > rep->status) rep->status = status;
        rep->outer_max = std::max(rep->outer_max, S.m);
        rep->steps_max = std::max(rep->steps_max, S.n);
        rep->rhs_outer[r] = S.m;
        rep->mv += S.mv;
        rep->dots += S.dots;
        rep->reliable += S.reliable;
        for (int s = 0; s < ns; ++s) {
            const ShiftState &H = fsh[(size_t)r * NSMAX + s];
            rep->shift_iters[(size_t)r * ns + s] = H.iters;
            rep->shift_resid[(size_t)r * ns + s] = H.res;
        }
    }

    if (pass1) {
        Prof p(c, CL_OTHER, nrhs * nd * (ns * cB + 16.0));
        launch_ysum(st, y, X, (const double *)c->ws_wts.p, n, ns, nrhs, nbv);
        HIPCHK(hipGetLastError());
    } else {
        // ---- sweep on the host, then the replay
        std::vector<TapeStep> tp((size_t)nrhs * max_steps);
        std::vector<double2> tg((size_t)nrhs * max_outer * LMAX);
        std::vector<TapeOuter> to((size_t)nrhs * max_outer);
        HIPCHK(hipMemcpy(tp.data(), c->ws_tape.p, tp.size() * sizeof(TapeStep), hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(tg.data(), c->ws_tape_gam.p, tg.size() * sizeof(double2), hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(to.data(), c->ws_tape_outer.p, to.size() * sizeof(TapeOuter), hipMemcpyDeviceToHost));
        int Mmax = 0;
        for (int r = 0; r < nrhs; ++r) Mmax = std::max(Mmax, fs[r].m);
        const int Mcap = std::max(Mmax, 1);
        std::vector<ReplayStep> rsteps((size_t)nrhs * Mcap * l);
        std::vector<ReplayOuter> router((size_t)nrhs * Mcap);
        std::vector<double2> cb(nrhs);
        for (int r = 0; r < nrhs; ++r) {
            std::vector<double> spv(ns), wv(ns);
            std::vector<int> it(ns), br(ns);
            for (int s = 0; s < ns; ++s) {
                const ShiftState &H = fsh[(size_t)r * NSMAX + s];
                spv[s] = H.sp;
                wv[s] = P.weights[(size_t)r * ns + s];
                it[s] = H.iters;
                br[s] = H.stopped;
            }
            SweepResult sr;
            sweep_rhs(l, fs[r].m, &tp[(size_t)r * max_steps], &to[(size_t)r * max_outer],
                      &tg[(size_t)r * max_outer * LMAX], ns, spv.data(), wv.data(), it.data(),
                      br.data(), Mcap, &sr);
            cb[r] = fromc(sr.cb);
            std::copy(sr.steps.begin(), sr.steps.begin() + (size_t)Mcap * l, rsteps.begin() + (size_t)r * Mcap * l);
            std::copy(sr.outer.begin(), sr.outer.begin() + Mcap, router.begin() + (size_t)r * Mcap);
        }
        CHK(ensure(c, c->ws_replay, rsteps.size() * sizeof(ReplayStep)));
        CHK(ensure(c, c->ws_replay_outer, router.size() * sizeof(ReplayOuter)));
        CHK(ensure(c, c->ws_cb, nrhs * sizeof(double2)));
        ReplayStep *drs = (ReplayStep *)c->ws_replay.p;
        ReplayOuter *dro = (ReplayOuter *)c->ws_replay_outer.p;
        HIPCHK(hipMemcpyAsync(drs, rsteps.data(), rsteps.size() * sizeof(ReplayStep), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(dro, router.data(), router.size() * sizeof(ReplayOuter), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(c->ws_cb.p, cb.data(), nrhs * sizeof(double2), hipMemcpyHostToDevice, st));

        // outer iterations [0, m_rep) are summed from the store (pass 3), the
        // rest regenerated by the replay (pass 2: all of them)
        const int m_rep = pass3 ? std::min(m_split, Mmax) : 0;
        rep->stored_iters = pass3 ? m_rep : -1;
        if (pass3) {
            // pseudo-double pass: y = c_b b + sum_t c_t v_t over the stored Mv outputs
            Prof p(c, CL_OTHER, nrhs * nd * (32.0 + 16.0 + (double)m_rep * (2.0 * l * cB + (mixed ? 16.0 : 0.0))));
            launch_yinit(st, y, b, (const double2 *)c->ws_cb.p, n, nrhs, nbv);
            for (int m0 = 0; m0 < m_rep; m0 += PSC) {
                const int mc = std::min(PSC, m_rep - m0);
                launch_pstore_sum<T>(st, y, (const C<T> *)c->pstore[m0 / PSC].p, ps_rs,
                                     mixed ? (const double2 *)c->prel[m0 / PSC].p : nullptr, (long)nrhs * n, drs, dro,
                                     Mcap, l, m0, mc, n, nrhs, nbv);
            }
            HIPCHK(hipGetLastError());
        }
        // pass 2 always passes here: y = c_b b is set here even where no
        // right-hand side iterated (Mmax = 0); pass 3 set it above
        if (!pass3 || m_rep < Mmax) {
        // regenerate the Mv outputs of outer iterations m_rep.. and accumulate y
        if (m_rep == 0) {
            Prof p(c, CL_OTHER, nrhs * nd * (2.0 * (l + 1) * cB + 16.0 + cB + 32.0));
            if (basis) {
                launch_zero<T>(st, Uv, n, vs, nrhs);   // as at the start of the first pass
            } else {
                launch_zero<T>(st, R, (long)nrhs * (l + 1) * n, 0, 1);
                launch_zero<T>(st, Uv, (long)nrhs * (l + 1) * n, 0, 1);
            }
            launch_convert_in<T>(st, R, b, n, vs, n, nrhs);
            if (!pass3) launch_yinit(st, y, b, (const double2 *)c->ws_cb.p, n, nrhs, nbv);
            if (mixed) launch_zero<double>(st, XH, (long)nrhs * n, 0, 1);
        } else {
            // the seed's state saved at the start of outer iteration m_rep
            Prof p(c, CL_OTHER, nrhs * nd * (4.0 * cB + (mixed ? 32.0 : 0.0)));
            HIPCHK(hipMemcpy2DAsync(R, vs * cs, c->ws_hs.p, n * cs, n * cs, nrhs, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpy2DAsync(Uv, vs * cs, (const char *)c->ws_hs.p + (size_t)nrhs * n * cs, n * cs, n * cs,
                                    nrhs, hipMemcpyDeviceToDevice, st));
            if (mixed)
                HIPCHK(hipMemcpyAsync(XH, c->ws_hs64.p, (size_t)nrhs * n * sizeof(double2), hipMemcpyDeviceToDevice,
                                      st));
        }
        const long rstride = (long)Mcap * l * sizeof(ReplayStep);
        VecArgs<T> vb = va;
        vb.partials = 0;
        vb.seed = nullptr;
        DslashArgs<T> e1 = d1, e2 = d2;
        e2.rt = nullptr;
        e2.part = nullptr;
        e2.y = y;
        e2.y_rs = n;
        Emit<T> e(c, P.persistent ? Emit<T>::RECORD : Emit<T>::LAUNCH, true);
        for (int m = m_rep; m < Mmax; ++m) {
            int nr_m = 0;      // right-hand sides whose replay reaches outer iteration m
            for (int r = 0; r < nrhs; ++r) nr_m += (fs[r].m > m) ? 1 : 0;
            if constexpr (std::is_same<T, double>::value) {
                if (basis) {
                    // the replay in basis form: the first pass's two vector
                    // updates per step (recorded beta, alpha), its Mv outputs
                    // into rows 1..l of U and R, then r_0 and u_0 from the
                    // basis with the recorded MR coefficients
                    BasisArgs<double> ba;
                    ba.n = n;
                    ba.l = l;
                    ba.sb = (const SeedBasis *)c->ws_sb.p;
                    ba.bv[0] = R;
                    ba.bv[1] = Uv;
                    for (int t = 0; t < 2 * l + 2; ++t) ba.brs[t] = vs;
                    for (int j = 0; j < l; ++j) {
                        ba.bv[2 + 2 * j] = Uv + (size_t)(j + 1) * n;
                        ba.bv[3 + 2 * j] = R + (size_t)(j + 1) * n;
                    }
                    double2 *WU = (double2 *)c->ws_bw.p, *WR = WU + (size_t)nrhs * n;
                    for (int j = 0; j < l; ++j) {
                        const size_t idx = (size_t)m * l + j;
                        Gate gu;
                        gu.flag = &drs[idx].flag;
                        gu.flag_stride = rstride / (long)sizeof(int);
                        gu.need = 1;
                        Gate gr = gu;
                        gr.need = 2;
                        const int xi = (j == 0) ? 0 : 2 * j + 1, yi = (j == 0) ? 1 : 2 * j;
                        BasisArgs<double> bu = ba;
                        bu.gate = gu;
                        bu.dst = WU;
                        bu.dst_rs = n;
                        bu.x = ba.bv[xi];
                        bu.x_rs = vs;
                        bu.y = ba.bv[yi];
                        bu.y_rs = vs;
                        bu.c = CoefRef{(const char *)&drs[idx].beta, rstride};
                        e.basis_axpy(bu, nrhs, nbv, CL_SEED, nr_m * 3.0 * nd * cB);
                        DslashArgs<T> f1 = e1, f2 = e2;
                        f1.in = WU;
                        f1.in_rs = n;
                        f1.out = tmp;
                        f1.gate = gu;
                        if (!opw) e.ds(f1, nrhs, EPI_PLAIN, CL_STENCIL, ds_bytes(EPI_PLAIN, nr_m));
                        f2.in = opw ? WU : tmp;
                        f2.in_rs = n;
                        f2.out = (C<T> *)ba.bv[2 + 2 * j];
                        f2.v = WU;
                        f2.v_rs = n;
                        f2.ycoef = CoefRef{(const char *)&drs[idx].cu, rstride};
                        f2.gate = gu;
                        e.ds(f2, nrhs, EPI_MV_Y, CL_STENCIL, ds_bytes(EPI_MV_Y, nr_m));
                        BasisArgs<double> br = bu;
                        br.gate = gr;
                        br.dst = WR;
                        br.y = ba.bv[2 + 2 * j];
                        br.c = CoefRef{(const char *)&drs[idx].alpha, rstride};
                        e.basis_axpy(br, nrhs, nbv, CL_SEED, nr_m * 3.0 * nd * cB);
                        f1.in = WR;
                        f1.gate = gr;
                        if (!opw) e.ds(f1, nrhs, EPI_PLAIN, CL_STENCIL, ds_bytes(EPI_PLAIN, nr_m));
                        f2.in = opw ? WR : tmp;
                        f2.out = (C<T> *)ba.bv[3 + 2 * j];
                        f2.v = WR;
                        f2.ycoef = CoefRef{(const char *)&drs[idx].cr, rstride};
                        f2.gate = gr;
                        e.ds(f2, nrhs, EPI_MV_Y, CL_STENCIL, ds_bytes(EPI_MV_Y, nr_m));
                    }
                    BasisReplayArgs ra;
                    ra.rs = drs;
                    ra.ro = dro;
                    ra.Mcap = Mcap;
                    ra.l = l;
                    ra.m = m;
                    ra.sb = (SeedBasis *)c->ws_sb.p;
                    e.basis_replay(ra, nrhs);
                    BasisArgs<double> bm = ba;
                    bm.gate.flag = &((const SeedBasis *)c->ws_sb.p)[0].nbu;
                    bm.gate.flag_stride = (long)sizeof(SeedBasis) / (long)sizeof(int);
                    bm.gate.need = 1;
                    bm.R0 = R;
                    bm.r0_rs = vs;
                    bm.U0 = Uv;
                    bm.u0_rs = vs;
                    e.basis_combine(bm, nrhs, nbv, CL_SEED, nr_m * (2.0 * l + 4) * nd * cB);
                    HIPCHK(hipGetLastError());
                    continue;
                }
            }
            for (int j = 0; j < l; ++j) {
                const size_t idx = (size_t)m * l + j;
                Gate gu;
                gu.flag = &drs[idx].flag;
                gu.flag_stride = rstride / (long)sizeof(int);
                gu.need = 1;
                Gate gr = gu;
                gr.need = 2;
                vb.beta = CoefRef{(const char *)&drs[idx].beta, rstride};
                vb.alpha = CoefRef{(const char *)&drs[idx].alpha, rstride};
                vb.gate = gu;
                const bool fu = !P.persistent && j >= 1;
                e.seed_u(vb, j, nrhs, nbv, CL_SEED, nr_m * (fu ? 3.0 : 3.0 * (j + 1)) * nd * cB, fu ? 1 : 0);
                e1.in = Uv + (size_t)j * n;
                e1.out = tmp;
                e1.gate = gu;
                if (!opw) e.ds(e1, nrhs, EPI_PLAIN, CL_STENCIL, ds_bytes(EPI_PLAIN, nr_m));
                e2.in = opw ? Uv + (size_t)j * n : tmp;
                e2.out = Uv + (size_t)(j + 1) * n;
                e2.v = Uv + (size_t)j * n;
                e2.ycoef = CoefRef{(const char *)&drs[idx].cu, rstride};
                e2.gate = gu;
                e.ds(e2, nrhs, EPI_MV_Y, CL_STENCIL, ds_bytes(EPI_MV_Y, nr_m));
                vb.gate = gr;
                e.r_update(vb, j, false, mixed, nrhs, nbv, CL_SEED, nr_m * (fu ? 4.0 * j + 4 : 3.0 * (j + 1)) * nd * cB,
                           fu);
                if (fu) {
                    // the step ended after its u-Mv: complete u_0..u_{j-1}
                    VecArgs<T> vc = vb;
                    vc.gate = gu;
                    vc.gate.eq = 1;
                    e.seed_u(vc, j, nrhs, nbv, CL_SEED, 0.0, 2);
                }
                e1.in = R + (size_t)j * n;
                e1.gate = gr;
                if (!opw) e.ds(e1, nrhs, EPI_PLAIN, CL_STENCIL, ds_bytes(EPI_PLAIN, nr_m));
                else e2.in = R + (size_t)j * n;
                e2.out = R + (size_t)(j + 1) * n;
                e2.v = R + (size_t)j * n;
                e2.ycoef = CoefRef{(const char *)&drs[idx].cr, rstride};
                e2.gate = gr;
                e.ds(e2, nrhs, EPI_MV_Y, CL_STENCIL, ds_bytes(EPI_MV_Y, nr_m));
            }
            Gate gm;
            gm.flag = &dro[m].lm;
            gm.flag_stride = (long)Mcap * sizeof(ReplayOuter) / (long)sizeof(int);
            gm.need = 1;
            vb.gate = gm;
            vb.gam = CoefRef{(const char *)&dro[m].gam[0], (long)Mcap * (long)sizeof(ReplayOuter)};
            e.mr_update(vb, false, mixed, nrhs, nbv, CL_SEED, nr_m * (2.0 * (l + 1) + 2) * nd * cB);
            if (mixed) {
                Gate grl;
                grl.flag = &dro[m].rel;
                grl.flag_stride = (long)Mcap * sizeof(ReplayOuter) / (long)sizeof(int);
                grl.need = 1;
                vb.partials = 1;   // the reliable update writes partials (unused in pass 2)
                reliable_update(e, vb, grl, y,
                                CoefRef{(const char *)&dro[m].crel, (long)Mcap * (long)sizeof(ReplayOuter)}, nr_m);
                vb.partials = 0;
            }
            HIPCHK(hipGetLastError());
        }
        if (P.persistent) {
            CHK(run_persistent<T>(c, e.ops, 1, false, l, seed, nrhs, e.cls_bytes));
            for (Ctx::SRec &q : c->srecs) q.pending = false;
        }
        // the replayed Mv (pass 2: as many as the first pass)
        for (int r = 0; r < nrhs; ++r)
            for (int m = m_rep; m < fs[r].m; ++m)
                for (int j = 0; j < l; ++j) {
                    const int f = rsteps[((size_t)r * Mcap + m) * l + j].flag;
                    rep->mv += (f >= 1 ? 1 : 0) + (f >= 2 ? 1 : 0);
                }
        }
    }

    // ---- optional FP64 true residual of every shift (single-pass)
    if (pass1 && want_true) {
        rep->shift_true_resid.assign((size_t)nrhs * ns, 0.0);
        CHK(ensure(c, c->ws_aux1, (size_t)nrhs * n * sizeof(double2)));
        CHK(ensure(c, c->ws_aux2, (size_t)nrhs * n * sizeof(double2)));
        CHK(ensure(c, c->ws_aux3, (size_t)nrhs * n * sizeof(double2)));
        CHK(ensure_host(c, (size_t)std::max(nrhs * sizeof(SeedState), (size_t)ps * sizeof(double))));
        double2 *xd = (double2 *)c->ws_aux1.p, *t1 = (double2 *)c->ws_aux2.p, *t2 = (double2 *)c->ws_aux3.p;
        std::vector<double> rowbuf(ps);
        for (int s = 0; s < ns; ++s) {
            launch_convert_out<double>(st, xd, X + (size_t)s * n, n, n, (long)ns * n, nrhs);
            DslashArgs<double> a1 = ds_args<double>(c, P.neg_mu, true);
            a1.in = xd;
            a1.out = t1;
            if (!P.op_wilson) launch_dslash<double>(st, a1, nrhs, EPI_PLAIN, false);
            for (int r = 0; r < nrhs; ++r) {
                DslashArgs<double> a2 = ds_args<double>(c, P.neg_mu, !P.op_wilson);
                a2.in = (P.op_wilson ? xd : t1) + (size_t)r * n;
                a2.out = t2 + (size_t)r * n;
                a2.scale = P.a_scale;
                a2.sigma0 = P.shifts[(size_t)r * ns + s];
                a2.v = xd + (size_t)r * n;
                launch_dslash<double>(st, a2, 1, EPI_SV, false);
            }
            launch_diffnorm_partials<double>(st, b, t2, n, n, n, part, ps, nrhs, nbv);
            HIPCHK(hipGetLastError());
            for (int r = 0; r < nrhs; ++r) {
                HIPCHK(hipStreamSynchronize(st));
                HIPCHK(hipMemcpy(rowbuf.data(), part + (size_t)r * PMAX * ps, ps * sizeof(double),
                                 hipMemcpyDeviceToHost));
                const double d = std::sqrt(host_partial_sum(rowbuf.data(), nbv));
                rep->shift_true_resid[(size_t)r * ns + s] = d / fs[r].bnorm;
            }
        }
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    rep->bytes_model = c->bytes_acc;
    return 0;
}

// ---------------------------------------------------------------------------
// Refinement of a single-pass solve (MSB_REFINE).  The collinear residual
// estimate that freezes a shift is the iteration's recursive residual; in
// FP32 arithmetic the true residual b - (A + sigma_s) x_s stalls near
// eps_32 kappa(A + sigma_s) above it.  After the solve, every shift's true
// residual is computed in FP64; each (rhs, shift) above tol gets a correction
// solve (A + sigma_s) d = r_s, batched with one shift per batch member, to the
// relative tolerance that brings it below tol with a factor 2 to spare, and
// x_s += d in FP64.  At most three rounds; then y = sum_s w_s x_s again.
// ---------------------------------------------------------------------------
static int run_solve(Ctx *c, const SolveParams &P, const double2 *b, double2 *y, double2 *xs, SolveReport *rep) {
    if (P.mixed) return solve_impl<float>(c, P, b, y, xs, false, rep);
    return solve_impl<double>(c, P, b, y, xs, false, rep);
}

static int solve_refined(Ctx *c, const SolveParams &P, const double2 *b, double2 *y, double2 *x_shifts,
                         SolveReport *rep) {
    constexpr int KMAX = 48;        // correction solves per batch
    constexpr int ROUNDS = 3;
    const int V = c->g.V;
    const long n = 12L * V;
    const int nrhs = P.nrhs, ns = P.n_shift;
    const int nbv = nblocks_for(n);
    const long ps = part_stride(c->g);
    hipStream_t st = c->stream;
    double2 *X = x_shifts;
    if (!X) {
        CHK(ensure(c, c->ws_rX, (size_t)nrhs * ns * n * sizeof(double2)));
        X = (double2 *)c->ws_rX.p;
    }
    SolveParams P0 = P;
    P0.refine = false;
    CHK(run_solve(c, P0, b, y, X, rep));
    double bytes = rep->bytes_model;
    if (rep->status == S_ERR_ARG) return 0;

    CHK(ensure(c, c->ws_rt1, (size_t)nrhs * n * sizeof(double2)));
    CHK(ensure(c, c->ws_rt2, (size_t)nrhs * n * sizeof(double2)));
    CHK(ensure(c, c->ws_rR, (size_t)nrhs * n * sizeof(double2)));
    CHK(ensure(c, c->ws_rB, (size_t)KMAX * n * sizeof(double2)));
    CHK(ensure(c, c->ws_rX2, (size_t)KMAX * n * sizeof(double2)));
    CHK(ensure(c, c->ws_ry, (size_t)KMAX * n * sizeof(double2)));
    CHK(ensure(c, c->ws_rsig, (size_t)nrhs * ns * sizeof(double)));
    CHK(ensure(c, c->ws_rw, (size_t)nrhs * ns * sizeof(double)));
    double2 *t1 = (double2 *)c->ws_rt1.p, *t2 = (double2 *)c->ws_rt2.p, *R = (double2 *)c->ws_rR.p;
    double2 *RB = (double2 *)c->ws_rB.p, *DX = (double2 *)c->ws_rX2.p, *DY = (double2 *)c->ws_ry.p;
    // shifts by shift then rhs (the per-rhs sigma of one residual launch)
    std::vector<double> sig_sr((size_t)ns * nrhs);
    for (int r = 0; r < nrhs; ++r)
        for (int s = 0; s < ns; ++s) sig_sr[(size_t)s * nrhs + r] = P.shifts[(size_t)r * ns + s];
    double *sig_dev = (double *)c->ws_rsig.p;
    HIPCHK(hipMemcpyAsync(sig_dev, sig_sr.data(), sig_sr.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(c->ws_rw.p, P.weights.data(), (size_t)nrhs * ns * sizeof(double), hipMemcpyHostToDevice,
                          st));

    // ||b_r||
    std::vector<double> bnorm(nrhs);
    // ||.|| per rhs from partial slot `slot`: the nbv partials of every rhs in
    // one strided copy into pinned host memory (a stream-ordered DMA; the
    // synchronisation below then covers it)
    auto read_norms = [&](int nr, int slot, std::vector<double> &out) -> int {
        out.assign(nr, 0.0);
        CHK(ensure_host(c, (size_t)nr * nbv * sizeof(double)));
        double *rows = (double *)c->host_pinned;
        HIPCHK(hipMemcpy2DAsync(rows, nbv * sizeof(double), (double *)c->ws_part.p + (size_t)slot * ps,
                                (size_t)PMAX * ps * sizeof(double), nbv * sizeof(double), nr,
                                hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int r = 0; r < nr; ++r) out[r] = std::sqrt(host_partial_sum(&rows[(size_t)r * nbv], nbv));
        return 0;
    };
    CHK(ensure(c, c->ws_part, (size_t)std::max(nrhs, KMAX) * PMAX * ps * sizeof(double)));
    double *part = (double *)c->ws_part.p;
    launch_dot_partials<double>(st, b, b, n, part, ps, nrhs, nbv, Gate{});
    CHK(read_norms(nrhs, 2, bnorm));

    const double Vd = (double)V;
    // R = b - (a H^2 + sigma_s) x_s for every rhs of shift s; returns ||R_r||
    auto residuals = [&](int s, std::vector<double> &rn) -> int {
        DslashArgs<double> d1 = ds_args<double>(c, P.neg_mu, true);
        d1.in = X + (size_t)s * n;
        d1.in_rs = (long)ns * n;
        d1.out = t1;
        if (!P.op_wilson) launch_dslash<double>(st, d1, nrhs, EPI_PLAIN, false);
        DslashArgs<double> d2 = ds_args<double>(c, P.neg_mu, !P.op_wilson);
        d2.in = P.op_wilson ? X + (size_t)s * n : t1;
        if (P.op_wilson) d2.in_rs = (long)ns * n;
        d2.out = t2;
        d2.v = X + (size_t)s * n;
        d2.v_rs = (long)ns * n;
        d2.scale = P.a_scale;
        d2.sigma0_rhs = sig_dev + (size_t)s * nrhs;
        launch_dslash<double>(st, d2, nrhs, EPI_SV, false);
        launch_residual(st, R, b, n, t2, n, part, ps, nrhs, nbv);
        HIPCHK(hipGetLastError());
        bytes += nrhs * (24 + 36 + 48) * 16.0 * Vd + 2 * 36 * 16.0 * Vd;
        rep->mv += nrhs;
        return read_norms(nrhs, 0, rn);
    };

    struct Pair { int r, s; double rn; };
    std::vector<Pair> batch;
    auto flush = [&]() -> int {
        if (batch.empty()) return 0;
        const int K = (int)batch.size();
        SolveParams Q = P0;
        Q.nrhs = K;
        Q.n_shift = 1;
        Q.shifts.resize(K);
        Q.weights.assign(K, 1.0);
        Q.force_iters = nullptr;
        Q.shadow = nullptr;                // the corrections' own right-hand sides
        Q.persistent = false;
        // each correction to its own relative tolerance (factor 2 to spare)
        Q.tol_rhs.resize(K);
        for (int k = 0; k < K; ++k) {
            Q.shifts[k] = P.shifts[(size_t)batch[k].r * ns + batch[k].s];
            const double q = 0.5 * P.tol * bnorm[batch[k].r] / batch[k].rn;
            Q.tol_rhs[k] = std::min(0.5, std::max(q, P.tol));
        }
        SolveReport r2;
        CHK(run_solve(c, Q, RB, DY, DX, &r2));
        bytes += r2.bytes_model;
        rep->mv += r2.mv;
        rep->dots += r2.dots;
        rep->reliable += r2.reliable;
        for (int k = 0; k < K; ++k)
            launch_axpy_host(st, X + ((size_t)batch[k].r * ns + batch[k].s) * n, DX + (size_t)k * n, d2(1, 0), n,
                             nbv);
        HIPCHK(hipGetLastError());
        rep->refined += K;
        batch.clear();
        return 0;
    };

    rep->shift_true_resid.assign((size_t)nrhs * ns, 0.0);
    std::vector<double> rn;
    for (int round = 0; round <= ROUNDS; ++round) {
        int failing = 0;
        for (int s = 0; s < ns; ++s) {
            CHK(residuals(s, rn));
            for (int r = 0; r < nrhs; ++r) {
                // a zero right-hand side has x_s = 0 and a zero residual; any
                // other residual of it counts as failing
                const double rel = bnorm[r] > 0 ? rn[r] / bnorm[r] : (rn[r] > 0 ? INFINITY : 0.0);
                rep->shift_true_resid[(size_t)r * ns + s] = rel;
                if (!(rel <= FREEZE_FRAC * P.tol)) {
                    failing += 1;
                    if (round == ROUNDS || !std::isfinite(rel)) continue;   // last round: report only
                    HIPCHK(hipMemcpyAsync(RB + batch.size() * n, R + (size_t)r * n, n * sizeof(double2),
                                          hipMemcpyDeviceToDevice, st));
                    batch.push_back(Pair{r, s, rn[r]});
                    if ((int)batch.size() == KMAX) CHK(flush());
                }
            }
        }
        CHK(flush());
        if (failing == 0) break;
        if (round == ROUNDS && rep->status == S_OK) rep->status = S_NOT_CONVERGED;
    }
    launch_ysum(st, y, X, (const double *)c->ws_rw.p, n, ns, nrhs, nbv);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    rep->bytes_model = bytes;
    c->bytes_acc = bytes;
    return 0;
}

int solve_mshift(Ctx *c, const SolveParams &P, const double2 *b, double2 *y, double2 *x_shifts,
                 bool want_true_resid, SolveReport *rep) {
    if (P.refine && P.pass == 1) return solve_refined(c, P, b, y, x_shifts, rep);
    if (P.mixed) return solve_impl<float>(c, P, b, y, x_shifts, want_true_resid, rep);
    return solve_impl<double>(c, P, b, y, x_shifts, want_true_resid, rep);
}

// ---------------------------------------------------------------------------
// sign(H) b = sqrt(a) H f(A) b;  D_ov b = b + gamma5 sign(H) b
// ---------------------------------------------------------------------------
int sign_apply(Ctx *c, const SolveParams &P, const double2 *b, double2 *out, bool overlap,
               SolveReport *rep) {
    const int V = c->g.V;
    const long n = 12L * V;
    CHK(ensure(c, c->ws_y, (size_t)P.nrhs * n * sizeof(double2)));
    double2 *y = (double2 *)c->ws_y.p;
    CHK(solve_mshift(c, P, b, y, nullptr, false, rep));
    CHK(ensure(c, c->ws_aux4, (size_t)P.nrhs * n * sizeof(double2)));
    double2 *hy = (double2 *)c->ws_aux4.p;
    DslashArgs<double> a = ds_args<double>(c, P.neg_mu, true);   // H y = g5 D y
    a.in = y;
    a.out = hy;
    launch_dslash<double>(c->stream, a, P.nrhs, EPI_PLAIN, false);
    launch_overlap_out(c->stream, out, b, hy, V, P.nrhs, overlap ? 1 : 0, std::sqrt(P.a_scale),
                       nblocks_for(n));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    return 0;
}

// ---------------------------------------------------------------------------
// Backward of L = Re <eta, y>, y = f(A) b (mode 0) or y = sign(H) b (mode 1).
// With x_s = (A + sigma_s)^{-1} b and z_s = (A^+ + sigma_s)^{-1} eta (A^+ =
// A(-mu), a forward solve at -mu):
//   grad_b = sum_s w_s z_s, grad_w_s = Re <eta, x_s>,
//   grad_sigma_s = -w_s Re <z_s, x_s>,
//   links: pairs (gamma5 z_s, H x_s) and (gamma5 H(-mu) z_s = D(-mu) z_s, x_s)
//   with c = -a w_s through the link-force kernel; mode 1 adds the pair
//   (gamma5 eta, y) with c = sqrt(a) and uses eta' = sqrt(a) H(-mu) eta.
// ---------------------------------------------------------------------------
int sign_backward(Ctx *c, const SolveParams &P0, const double2 *b, const double2 *eta, int mode,
                  double2 *grad_b, double *grad_w, double *grad_sigma, double2 *grad_links, SolveReport *rep) {
    hipStream_t st = c->stream;
    const int V = c->g.V;
    const long n = 12L * V;
    const int nrhs = P0.nrhs, ns = P0.n_shift;
    const int nbv = nblocks_for(n);
    CHK(ensure(c, c->ws_bX, (size_t)nrhs * ns * n * sizeof(double2)));
    CHK(ensure(c, c->ws_bZ, (size_t)nrhs * ns * n * sizeof(double2)));
    CHK(ensure(c, c->ws_by, (size_t)nrhs * n * sizeof(double2)));
    CHK(ensure(c, c->ws_beta, (size_t)nrhs * n * sizeof(double2)));
    CHK(ensure(c, c->ws_bA, (size_t)nrhs * n * sizeof(double2)));
    CHK(ensure(c, c->ws_bB, (size_t)nrhs * n * sizeof(double2)));
    CHK(ensure(c, c->ws_bdots, (size_t)nrhs * ns * 2 * nbv * sizeof(double)));
    double2 *X = (double2 *)c->ws_bX.p, *Z = (double2 *)c->ws_bZ.p, *y = (double2 *)c->ws_by.p;
    double2 *eta2 = (double2 *)c->ws_beta.p, *tA = (double2 *)c->ws_bA.p, *tB = (double2 *)c->ws_bB.p;

    SolveParams P = P0;
    P.pass = 1;
    SolveReport rf, ra;
    CHK(solve_mshift(c, P, b, y, X, false, &rf));
    const double2 *etap = eta;
    const double sa = std::sqrt(P.a_scale);
    if (mode == 1) {
        DslashArgs<double> a1 = ds_args<double>(c, !P.neg_mu, true);    // sqrt(a) H^+ eta
        a1.in = eta;
        a1.out = eta2;
        a1.scale = sa;
        launch_dslash<double>(st, a1, nrhs, EPI_PLAIN, false);
        etap = eta2;
    }
    SolveParams Pa = P;
    Pa.neg_mu = !P.neg_mu;
    CHK(solve_mshift(c, Pa, etap, grad_b, Z, false, &ra));

    // grad_w, grad_sigma from per-(rhs, shift) inner products
    launch_shift_dots(st, etap, X, Z, n, ns, nrhs, nbv, (double *)c->ws_bdots.p);
    HIPCHK(hipGetLastError());
    std::vector<double> dots((size_t)nrhs * ns * 2 * nbv);
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(dots.data(), c->ws_bdots.p, dots.size() * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(hipStreamSynchronize(st));
    for (int s = 0; s < ns; ++s) {
        double gw = 0.0, gs = 0.0;
        for (int r = 0; r < nrhs; ++r) {
            const double *row = &dots[((size_t)r * ns + s) * 2 * nbv];
            gw += host_partial_sum(row, nbv);
            gs += host_partial_sum(row + nbv, nbv);
        }
        grad_w[s] = gw;
        grad_sigma[s] = -P.weights[s] * gs;
    }

    // link force, one launch per shift (two pairs, all right-hand sides)
    LinkForceArgs fa;
    fa.g = c->g;
    const double mu = P.neg_mu ? -c->mu : c->mu;
    fa.ef = std::exp(mu);
    fa.eb = std::exp(-mu);
    fa.bc = c->bc_t;
    fa.nrhs = nrhs;
    fa.G = grad_links;
    for (int s = 0; s < ns; ++s) {
        DslashArgs<double> hx = ds_args<double>(c, P.neg_mu, true);     // H x_s
        hx.in = X + (size_t)s * n;
        hx.in_rs = (long)ns * n;
        hx.out = tA;
        launch_dslash<double>(st, hx, nrhs, EPI_PLAIN, false);
        DslashArgs<double> dz = ds_args<double>(c, !P.neg_mu, false);   // D(-mu) z_s = g5 H(-mu) z_s
        dz.in = Z + (size_t)s * n;
        dz.in_rs = (long)ns * n;
        dz.out = tB;
        launch_dslash<double>(st, dz, nrhs, EPI_PLAIN, false);
        const double cf = -P.a_scale * P.weights[s];
        fa.npair = 2;
        fa.pairs[0] = LinkPair{Z + (size_t)s * n, tA, (long)ns * n, n, cf, 1};
        fa.pairs[1] = LinkPair{tB, X + (size_t)s * n, n, (long)ns * n, cf, 0};
        launch_link_force(st, fa);
    }
    if (mode == 1) {
        fa.npair = 1;
        fa.pairs[0] = LinkPair{eta, y, n, n, sa, 1};
        launch_link_force(st, fa);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    *rep = rf;
    rep->status = std::max(rf.status, ra.status);
    rep->mv = rf.mv + ra.mv;
    rep->dots = rf.dots + ra.dots;
    rep->reliable = rf.reliable + ra.reliable;
    rep->bytes_model = rf.bytes_model + ra.bytes_model;
    rep->outer_max = std::max(rf.outer_max, ra.outer_max);
    rep->steps_max = std::max(rf.steps_max, ra.steps_max);
    return 0;
}

}  // namespace msb
