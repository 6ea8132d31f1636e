#!/usr/bin/env python3
"""Benchmark of f(A) b = sum_s w_s (A + sigma_s)^{-1} b on one MI355X.

Workload: 16^3x32 lattice, SU(3) links exp(i 0.5 H) (seeded), Wilson mass -2,
mu = 0.05, antiperiodic in time; A = a (gamma5 D_w)^2 with a from the GPU
power iteration; Neuberger PFE with N_s = 30 poles; BiCGstab(l = 4); the 12
spin-colour point sources at the origin solved as one batch; tolerance 1e-8 on
every shift's relative residual.

One step = one f(A) b evaluation of the 12-source batch in the headline form
(--pass, --precision, --deferred, --seed-basis, --refine).  The default is the
fastest form that meets the tolerance on every shift: the pseudo-double pass
in FP64 (the seed's 2 M l Mv outputs kept in HBM, y summed from them with the
transposed sweep's coefficients; the same y as the single pass to rounding),
with the seed's BiCG steps in basis form (each step writes only the two
vectors its Mv reads; the others stay coefficients on the outer iteration's
basis until the MR step).  The
single pass (per-step or deferred shift updates), the double pass and the
mixed-precision forms (FP32 stencil and vectors, FP64 reductions,
accumulators and reliable updates; with per-shift refinement to reach the
tolerance) are in the comparison block with their errors.  ``value`` is f(A) b evaluations (one per
source) per second over the K timed steps.  Every kernel launch inside the timed steps is
bracketed by HIP events on its stream (the library's timing hook); the stencil
kernel's algorithmic bytes over its summed event time give roofline.achieved.
The other forms (single-pass / double-pass, FP64 / mixed, per-stage
launches / one persistent launch) run once each afterwards for the
comparison block.  The CPU oracle is timed on a bounded
sample (one outer iteration of one source) and extrapolated.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VARIANT_REPS = 3     # timed runs per comparison form (after one warm-up)
# timed steps: every 7th stencil launch carries timing events; 7 is coprime to
# the 4-launch pattern of a BiCG step (the two stencils of the u- and r-Mv)
# and to its 16 per outer iteration, so the sample covers every position
STENCIL_SAMPLE = 7
METRIC = "f(A)b time & HBM GB/s, 16^3x32, 1e-8 err; 2- vs 1-pass, mixed vs FP64"
WORKLOAD = "16x16x16x32"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def solver_flags(mixed, persistent, refine=False, deferred=False, basis=False):
    from paper_1010_2592_amd import msb
    return ((msb.MIXED if mixed else 0) | (msb.PERSISTENT if persistent else 0) | (msb.REFINE if refine else 0)
            | (msb.DEFERRED if deferred else 0) | (msb.SEED_BASIS if basis else 0))


def run_variant(ctx, b, a, sig, w, l, tol, max_outer, pass_, mixed, persistent=False, profile=False,
                refine=False, deferred=False, basis=False):
    import torch
    from paper_1010_2592_amd import msb
    flags = solver_flags(mixed, persistent, refine, deferred, basis)
    if profile:
        ctx.profile_enable(True)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    y, info, _ = ctx.mshift_bicgstabl(b, a, sig, w, l, tol, max_outer, pass_, flags=flags,
                                      allow=(msb.OK, msb.NOT_CONVERGED, msb.REDUCED_ACCURACY))
    e1.record()
    torch.cuda.synchronize()
    prof = ctx.profile_read() if profile else None
    if profile:
        ctx.profile_enable(False)
    return y, info, e0.elapsed_time(e1), prof


def workload_key(pass_, precision, refine, persistent, deferred=False, basis=False):
    return (f"{WORKLOAD} 12 rhs {precision} pass {pass_}" + (" deferred" if deferred else "")
            + (" seed basis" if basis else "") + (" refine" if refine else "")
            + (" persistent" if persistent else ""))


def measured_traffic(key):
    """HBM bytes per stencil launch from the committed rocprofv3 counter runs
    (profiles/dslash_traffic.json), or None when the stencil or solver sources
    changed since they were taken or the form differs from the one they were
    taken on."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "dslash_traffic.json")))
        from paper_1010_2592_amd.rocprof_summary import STENCIL_SOURCES, sources_hash
        if rec.get("sources") != STENCIL_SOURCES or sources_hash() != rec.get("sources_sha256_16"):
            return None
    except (OSError, ValueError, KeyError):
        return None
    if rec.get("workload") != key:
        return None
    return rec["traffic_bytes_per_launch"]


def mu0_block(wk, U, b, sig, w, l, with_cpu=True):
    """The same lattice, links and 12 sources at mu = 0, where A is Hermitian:
    multi-shift CG (single, double, pseudo-double pass) beside BiCGstab(l)
    (pseudo-double pass and deferred single pass), one run each after a
    warm-up, y compared with the CG single pass."""
    import numpy as np
    import torch
    from paper_1010_2592_amd import msb
    ctx = msb.Context(msb.Lattice(wk.dims, wk.mass, 0.0, wk.bc_t), U)
    rho = ctx.spectral_radius(torch.from_numpy(wk.power_start()[None]).to(U.device), 100)
    a0 = 1.0 / (1.01 * rho)
    allow = (msb.OK, msb.NOT_CONVERGED, msb.REDUCED_ACCURACY)
    forms = [("cg-1pass", "cg", 1, 0), ("cg-2pass", "cg", 2, 0), ("cg-3pass", "cg", 3, 0),
             (f"bicgstab{l}-3pass", "bi", 3, 0), (f"bicgstab{l}-1pass-deferred", "bi", 1, msb.DEFERRED)]
    out, ref = {}, None
    for name, kind, pass_, flags in forms:
        times, info, y = [], None, None
        for rep in range(2):
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            if kind == "cg":
                y, info, _ = ctx.mshift_cg(b, a0, sig, w, wk.tol, 20000, pass_, allow=allow)
            else:
                y, info, _ = ctx.mshift_bicgstabl(b, a0, sig, w, l, wk.tol, 4000, pass_, flags=flags, allow=allow)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        if ref is None:
            ref = y
        out[name] = {"ms": round(times[-1], 2), "iters": info.outer_iters, "mv": info.mv_count,
                     "status": info.status, "max_shift_resid": float(np.max(info.shift_resid)),
                     "rel_diff_vs_cg_1pass": float(torch.linalg.norm(y - ref) / torch.linalg.norm(ref))}
        log(f"[bench] mu=0 {name}: {out[name]}")
        del y
        torch.cuda.empty_cache()
    ctx.close()
    torch.cuda.empty_cache()
    res = {"workload": "the headline lattice, links and sources at mu = 0 (A Hermitian)", "forms": out}
    if with_cpu:
        # the CG oracle's pseudo-double pass: one point source, 8 iterations,
        # extrapolated to the GPU run's N and to 12 sources
        from oracle import cg as ocg
        from oracle import dirac as od
        import workloads as wl
        op = od.Dirac(U.cpu().numpy(), wk.dims, wk.mass, 0.0, wk.bc_t)
        b0 = wl.point_sources(wk.dims)[0]
        t0 = time.perf_counter()
        ocg.mshift_cg(lambda v: op.a_op(v, a0), b0, sig, w, wk.tol, 8, 3, force_iters=np.full(len(sig), 8))
        t8 = time.perf_counter() - t0
        N = out["cg-3pass"]["iters"]
        res["cpu_baseline"] = {"value": 1.0 / (t8 * N / 8), "unit": "f(A)b/s", "cores": 1, "kind": "oracle",
                               "sample": f"CG oracle pseudo-double pass, 1 point source, 8 forced iterations in "
                                         f"{t8:.1f} s; extrapolated to N = {N}; NumPy single-threaded",
                               "gpu_value": round(b.shape[0] / (out["cg-3pass"]["ms"] / 1e3), 2)}
        log(f"[bench] mu=0 CPU oracle sample: {res['cpu_baseline']}")
    return res


def deflation_block(wk, U, b, sig, w, l, with_cpu=True):
    """Low-mode deflation at mu = 0 on the headline lattice: the 12 eigenpairs
    of H = gamma5 D_w of smallest |lambda| (block of 24, Chebyshev degree up to
    200), then sign(H) b for the 12 point sources with and without those modes
    deflated (pseudo-double pass).  Reports the eigensolver's time, iterations,
    residuals and orthonormality, both sign applications, and the PFE error
    bound over the interval each one sees."""
    import numpy as np
    import torch

    import workloads as wl
    from paper_1010_2592_amd import msb
    dev = U.device
    ctx = msb.Context(msb.Lattice(wk.dims, wk.mass, 0.0, wk.bc_t), U)
    rho = ctx.spectral_radius(torch.from_numpy(wk.power_start()[None]).to(dev), 100)
    a0 = 1.0 / (1.01 * rho)
    nev, nblock, degree, tol_eig = 12, 24, 200, 1e-10
    start = torch.from_numpy(wl.gaussian_source(wk.dims, 6003, nblock)).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lam, vecs, res, iters = ctx.low_modes(nev, start, tol=tol_eig, degree=degree, max_iter=60,
                                          allow=(msb.OK, msb.NOT_CONVERGED, msb.REDUCED_ACCURACY))
    torch.cuda.synchronize()
    t_eig = (time.perf_counter() - t0) * 1e3
    del start
    vm = vecs.reshape(nev, -1)
    orth = float((vm.conj() @ vm.T - torch.eye(nev, dtype=vm.dtype, device=dev)).abs().max())
    eig = {"nev": nev, "block": nblock, "max_degree": degree, "tol": tol_eig, "ms": round(t_eig, 1),
           "iterations": iters, "abs_lambda": [float(x) for x in np.abs(lam)], "max_resid": float(np.max(res)),
           "orthonormality": orth}
    log(f"[bench] deflation low modes: {eig}")
    allow = (msb.OK, msb.NOT_CONVERGED, msb.REDUCED_ACCURACY)
    forms, outs = {}, {}
    for name in ("plain", "deflated"):
        times = []
        for rep in range(2):
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            if name == "plain":
                o, info = ctx.pfe_sign_apply(b, a0, sig, w, l, wk.tol, 4000, 3, allow=allow)
            else:
                o, info = ctx.pfe_sign_apply_deflated(b, a0, sig, w, l, wk.tol, 4000, lam, vecs, 3, allow=allow)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        outs[name] = o
        forms[name] = {"ms": round(times[-1], 2), "outer_iters": info.outer_iters, "status": info.status}
        log(f"[bench] deflation sign {name}: {forms[name]}")
    forms["rel_diff"] = float(torch.linalg.norm(outs["deflated"] - outs["plain"]) / torch.linalg.norm(outs["plain"]))
    # PFE error of sign over the interval each form sees: [a lambda_0^2, 1]
    # without deflation; the deflated source has no component below the
    # largest deflated |lambda| (a lower bound of the first kept one)

    def pfe_err(lo):
        x = np.logspace(np.log10(lo), 0.0, 20001)
        return float(np.max(np.abs(np.sqrt(x) * (w[None, :] / (x[:, None] + sig[None, :])).sum(axis=1) - 1.0)))
    absl = np.abs(lam)
    forms["pfe_error_bound_plain"] = pfe_err(a0 * absl.min() ** 2)
    forms["pfe_error_bound_deflated"] = pfe_err(a0 * absl.max() ** 2)
    log(f"[bench] deflation sign: rel diff {forms['rel_diff']:.2e}, PFE bounds "
        f"{forms['pfe_error_bound_plain']:.2e} -> {forms['pfe_error_bound_deflated']:.2e}")
    del outs, vecs, vm
    ctx.close()
    torch.cuda.empty_cache()
    res_out = {"workload": "the headline lattice, links and 12 point sources at mu = 0", "low_modes": eig,
               "sign": forms}
    if with_cpu:
        # the oracle's deflation (dense eigendecomposition for the low modes,
        # then the deflated sign of one source) on a 4^4 lattice beside the
        # library doing the same work there
        from oracle import deflation as odf
        from oracle import dirac as od
        dims = (4, 4, 4, 4)
        Us = wl.gauge_links(dims, wk.eps, wk.gauge_seed)
        op = od.Dirac(Us, dims, wk.mass, 0.0, wk.bc_t)
        b0 = wl.point_sources(dims)[:1]
        t0 = time.perf_counter()
        lam_o, vecs_o = odf.low_modes(op, nev)
        odf.sign_apply_deflated(op, a0, b0[0], lam_o, vecs_o, sig, w, l, wk.tol, 4000, 3)
        t_cpu = time.perf_counter() - t0
        cs = msb.Context(msb.Lattice(dims, wk.mass, 0.0, wk.bc_t), torch.from_numpy(Us).to(dev))
        st = torch.from_numpy(wl.gaussian_source(dims, 6003, nblock)).to(dev)
        bt = torch.from_numpy(b0).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lg, vg, _, _ = cs.low_modes(nev, st, tol=tol_eig, degree=degree, max_iter=60, allow=allow)
        cs.pfe_sign_apply_deflated(bt, a0, sig, w, l, wk.tol, 4000, lg, vg, 3, allow=allow)
        torch.cuda.synchronize()
        t_gpu = time.perf_counter() - t0
        cs.close()
        res_out["cpu_baseline"] = {"value": 1.0 / t_cpu, "unit": "deflated sign applications/s (4^4, 12 modes)",
                                   "cores": 1, "kind": "oracle",
                                   "sample": f"oracle on a 4^4 lattice: dense eigendecomposition for 12 low modes "
                                             f"plus the deflated sign of one point source in {t_cpu:.1f} s; "
                                             f"NumPy (dense eigensolver threaded by LAPACK)",
                                   "gpu_value": round(1.0 / t_gpu, 2)}
        log(f"[bench] deflation CPU oracle sample: {res_out['cpu_baseline']}")
    return res_out


def config4_block():
    """The 24^3x48 configuration (one Gaussian source, N_s = 58, tol 1e-8,
    mu = 0.05): every FP64 form for l = 2 and 6 (the seed in explicit and in
    basis form), each in a context of its own (one warm-up, then one timed
    solve), with the vectors each form holds."""
    import numpy as np
    import torch

    import workloads as wl
    from paper_1010_2592_amd import msb
    wk = wl.WORKLOADS["24x24x24x48"]
    dev = torch.device("cuda:0")
    log("[bench] cfg4: building 24x24x24x48 inputs")
    U = torch.from_numpy(wk.links()).to(dev)
    b = torch.from_numpy(wk.sources()).to(dev)
    vec_gb = 12 * wk.volume * 16 / 1e9
    sig, w = msb.neuberger_pfe(wk.n_shift)
    ctx = msb.Context(msb.Lattice(wk.dims, wk.mass, wk.mu, wk.bc_t), U)
    rho = ctx.spectral_radius(torch.from_numpy(wk.power_start()[None]).to(dev), 100)
    ctx.close()
    a = 1.0 / (1.01 * rho)
    out, ref = {}, {}
    for l in wk.ells:
        for name, pass_, flags in (("1pass", 1, 0), ("1pass-deferred", 1, msb.DEFERRED),
                                   ("1pass-deferred-basis", 1, msb.DEFERRED | msb.SEED_BASIS), ("2pass", 2, 0),
                                   ("2pass-basis", 2, msb.SEED_BASIS), ("3pass", 3, 0),
                                   ("3pass-basis", 3, msb.SEED_BASIS)):
            ctx = msb.Context(msb.Lattice(wk.dims, wk.mass, wk.mu, wk.bc_t), U)
            times = []
            for rep in range(2):
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                y, info, _ = ctx.mshift_bicgstabl(b, a, sig, w, l, wk.tol, 3000, pass_, flags=flags)
                e1.record()
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
            M = info.outer_iters
            # vectors beyond the seed's (the basis form adds its two work vectors)
            held = {"1pass": wk.n_shift * (l + 1), "1pass-deferred": wk.n_shift + 2 * l + 2,
                    "1pass-deferred-basis": wk.n_shift + 2 * l + 4, "2pass": 0, "2pass-basis": 2,
                    "3pass": 2 * M * l, "3pass-basis": 2 * M * l + 2}[name]
            key = f"l{l}-{name}"
            if l not in ref:
                ref[l] = y
            out[key] = {"ms": round(times[-1], 1), "outer_iters": M, "mv": info.mv_count, "status": info.status,
                        "max_shift_resid": float(np.max(info.shift_resid)),
                        "extra_vectors_GB": round(held * vec_gb, 1),
                        "rel_diff_vs_1pass": float(torch.linalg.vector_norm(y - ref[l]) /
                                                   torch.linalg.vector_norm(ref[l]))}
            log(f"[bench] cfg4 {key}: {out[key]}")
            del y
            ctx.close()
            torch.cuda.empty_cache()
    return {"workload": "24x24x24x48, 1 Gaussian source, N_s = 58, tol 1e-8, mu = 0.05, FP64", "forms": out}


def propagator_block(wk, U, b, l, with_cpu=True):
    """Multi-mass Wilson propagators of the 12 point sources on the headline
    lattice (mu = 0.05): D_w(m_s)^{-1} b for five masses from one Krylov space
    (A = D_w(m_0), sigma_s = m_s - m_0; a Gaussian shadow residual), single
    pass with the propagators returned; FP64 deferred and mixed + refinement.
    Reports ms per batch and the worst true residual over all 60 propagators."""
    import numpy as np
    import torch

    import workloads as wl
    from paper_1010_2592_amd import msb
    masses = np.array([0.1, 0.15, 0.25, 0.5, 1.0])
    m0 = float(masses.min())
    sig = masses - m0
    ctx = msb.Context(msb.Lattice(wk.dims, m0, wk.mu, wk.bc_t), U)
    shadow = torch.from_numpy(np.repeat(wl.gaussian_source(wk.dims, 5003), b.shape[0], axis=0)).to(U.device)
    out = {}
    for name, flags in (("fp64-deferred", msb.OP_WILSON | msb.DEFERRED),
                        ("mixed-refine", msb.OP_WILSON | msb.MIXED | msb.REFINE)):
        times = []
        for rep in range(2):
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            y, info, xs = ctx.mshift_bicgstabl(b, 1.0, sig, np.ones(len(sig)), l, wk.tol, 2000, 1, flags=flags,
                                               want_shifts=True, shadow=shadow,
                                               allow=(msb.OK, msb.NOT_CONVERGED, msb.REDUCED_ACCURACY))
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        worst = 0.0
        bn = torch.linalg.vector_norm(b.reshape(b.shape[0], -1), dim=1)
        for s in range(len(sig)):
            x = xs[:, s].contiguous()
            r = b - ctx.wilson_apply(x, 0) - sig[s] * x
            worst = max(worst, float((torch.linalg.vector_norm(r.reshape(b.shape[0], -1), dim=1) / bn).max()))
            del x, r
        out[name] = {"ms": round(times[-1], 2), "outer_iters": info.outer_iters, "mv": info.mv_count,
                     "status": info.status, "refined_shifts": info.refined_shifts,
                     "max_true_resid": worst, "propagators_per_s": round(b.shape[0] * len(sig) / (times[-1] / 1e3), 1)}
        log(f"[bench] propagators {name}: {out[name]}")
        del y, xs
        torch.cuda.empty_cache()
    ctx.close()
    torch.cuda.empty_cache()
    res = {"workload": f"12 point sources, masses {masses.tolist()}, mu = {wk.mu}, tol {wk.tol}", "forms": out}
    if with_cpu:
        # the oracle's multi-shift solve with A = D_w: one point source, one
        # forced outer iteration, extrapolated to the GPU run's M and 12 sources
        from oracle import dirac as od
        from oracle import krylov as ok
        op = od.Dirac(U.cpu().numpy(), wk.dims, m0, wk.mu, wk.bc_t)
        b0 = wl.point_sources(wk.dims)[0]
        t0 = time.perf_counter()
        ok.mshift_bicgstabl(op.dw, b0, sig, np.ones(len(sig)), l, wk.tol, 1, 1,
                            force_iters=np.ones(len(sig), dtype=int), shadow=wl.gaussian_source(wk.dims, 5003)[0])
        t1 = time.perf_counter() - t0
        M = out["fp64-deferred"]["outer_iters"]
        res["cpu_baseline"] = {"value": len(sig) / (t1 * M), "unit": "propagators/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"oracle single pass with A = D_w, 1 point source x {len(sig)} masses, "
                                         f"1 forced outer iteration in {t1:.1f} s; extrapolated to M = {M}; "
                                         f"NumPy single-threaded"}
        log(f"[bench] propagators CPU oracle sample: {res['cpu_baseline']}")
    return res


CPU_ITERS = 2     # forced outer iterations of the CPU oracle sample


def _cpu_worker(k, a, sig, w, l, K, barrier, out):
    """Child process: one point source, K forced outer iterations of the
    oracle's double pass, timed after every worker has built its inputs; sends
    back the timing and the oracle's y."""
    import numpy as np

    import workloads as wl
    from oracle import dirac as od
    from oracle import krylov as ok
    wk = wl.WORKLOADS[WORKLOAD]
    op = od.Dirac(wk.links(), wk.dims, wk.mass, wk.mu, wk.bc_t)
    b = wl.point_sources(wk.dims)[k]
    barrier.wait(timeout=600)
    t0 = time.time()
    y = ok.mshift_bicgstabl(lambda v: op.a_op(v, a), b, sig, w, l, wk.tol, K, 2,
                            force_iters=np.full(len(sig), K, dtype=int))[0]
    out.put((k, t0, time.time(), y))


def cpu_baseline_single(wk, a, sig, w, l, M_gpu, why, K=CPU_ITERS):
    """One source in this process (the fallback when worker processes cannot
    be started); returns (baseline, {source: oracle y})."""
    import numpy as np

    import workloads as wl
    from oracle import dirac as od
    from oracle import krylov as ok
    op = od.Dirac(wk.links(), wk.dims, wk.mass, wk.mu, wk.bc_t)
    b = wl.point_sources(wk.dims)[0]
    t0 = time.perf_counter()
    y = ok.mshift_bicgstabl(lambda v: op.a_op(v, a), b, sig, w, l, wk.tol, K, 2,
                            force_iters=np.full(len(sig), K, dtype=int))[0]
    t_iter = (time.perf_counter() - t0) / K
    return ({"value": 1.0 / (t_iter * M_gpu), "unit": "f(A)b/s", "cores": 1, "kind": "oracle",
             "sample": f"oracle double pass, 1 point source in this process, {K} forced outer iterations "
                       f"(l={l}: {4 * l} Mv each) at {t_iter:.1f} s per iteration; extrapolated x{M_gpu} outer "
                       f"iterations (the GPU run's M); NumPy single-threaded ({why})"}, {0: y})


def cpu_baseline(wk, a, sig, w, l, M_gpu, nproc=12, K=CPU_ITERS):
    """The oracle's double pass on the 12 point sources, one worker process
    per source (one thread each), each for K forced outer iterations (l BiCG
    steps per iteration, both passes); the wall time from the first start to
    the last end, per iteration, extrapolated linearly to the GPU's M.
    Returns (baseline, {source: oracle y after the K iterations})."""
    import multiprocessing as mp
    nsrc = 12
    nproc = max(1, min(nproc, nsrc, os.cpu_count() or 1))
    ctx = mp.get_context("spawn")
    barrier = ctx.Barrier(nproc)
    out = ctx.Queue()
    saved = {v: os.environ.get(v) for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for v in saved:
        os.environ[v] = "1"
    procs = []
    try:
        procs = [ctx.Process(target=_cpu_worker, args=(k, a, sig, w, l, K, barrier, out)) for k in range(nproc)]
        for p in procs:
            p.start()
        res = []
        t_start = time.time()
        while len(res) < nproc:
            try:
                res.append(out.get(timeout=5))
            except Exception:
                if any(p.exitcode not in (None, 0) for p in procs) or time.time() - t_start > 900:
                    raise RuntimeError("CPU oracle worker failed: exit codes "
                                       f"{[p.exitcode for p in procs]}")
        for p in procs:
            p.join(timeout=60)
    finally:
        for p in procs:        # only the workers started here
            if p.is_alive():
                p.terminate()
        for v, x in saved.items():
            if x is None:
                os.environ.pop(v, None)
            else:
                os.environ[v] = x
    t_all = max(e for _, _, e, _ in res) - min(s for _, s, _, _ in res)
    per = sorted(e - s for _, s, e, _ in res)
    t_fab = t_all / K * M_gpu
    return ({"value": nproc / t_fab, "unit": "f(A)b/s", "cores": nproc, "kind": "oracle",
             "sample": f"oracle double pass, {nproc} point sources in {nproc} worker processes "
                       f"(one thread each), {K} forced outer iterations each (l={l}: {4 * l} Mv per "
                       f"iteration): {t_all:.1f} s wall for all (per worker {per[0]:.1f}-{per[-1]:.1f} s); "
                       f"extrapolated x{M_gpu}/{K} outer iterations (the GPU run's M)"},
            {k: y for k, _, _, y in res})


def shift_true_residuals(ctx, b, a, sig, xs):
    """||b - (A + sigma_s) x_s|| / ||b|| per (rhs, shift) in FP64, with A
    applied by wilson_apply."""
    import numpy as np
    import torch
    from paper_1010_2592_amd import msb
    bn = torch.linalg.vector_norm(b.reshape(b.shape[0], -1), dim=1)
    tr = np.zeros((b.shape[0], len(sig)))
    for s in range(len(sig)):
        x = xs[:, s].contiguous()
        t = ctx.wilson_apply(ctx.wilson_apply(x, msb.G5_LEFT), msb.G5_LEFT)
        r = b - a * t - sig[s] * x
        tr[:, s] = (torch.linalg.vector_norm(r.reshape(b.shape[0], -1), dim=1) / bn).cpu().numpy()
        del x, t, r
    return tr


def mixed_floor_block(ctx, b, a, sig, w, l, tols=(1e-4, 1e-6, 1e-8)):
    """Where mixed precision without refinement pays: for each tolerance, the
    FP64 pseudo-double pass's time (the headline form: seed in basis form)
    beside the mixed deferred single pass's
    (one warm-up, median of VARIANT_REPS) and the mixed run's per-shift FP64
    true residuals (an untimed run of the same form that keeps the x_s).  The
    mixed run reaches tol only where its FP32 floor lies below it; the largest
    tol it misses and the floor itself are the break-even figures."""
    import numpy as np
    import torch
    from paper_1010_2592_amd import msb
    allow = (msb.OK, msb.NOT_CONVERGED, msb.REDUCED_ACCURACY)
    out = {}
    for tol in tols:
        row = {}
        for name, pass_, flags in (("fp64-3pass-basis", 3, msb.SEED_BASIS),
                                   ("mixed-deferred", 1, msb.MIXED | msb.DEFERRED)):
            ts = []
            for rep in range(VARIANT_REPS + 1):
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                y, info, _ = ctx.mshift_bicgstabl(b, a, sig, w, l, tol, 2000, pass_, flags=flags, allow=allow)
                e1.record()
                torch.cuda.synchronize()
                if rep:
                    ts.append(e0.elapsed_time(e1))
                del y
            row[name] = {"ms": round(float(np.median(ts)), 2), "outer_iters": info.outer_iters,
                         "status": info.status}
        _, info, xs = ctx.mshift_bicgstabl(b, a, sig, w, l, tol, 2000, 1, flags=msb.MIXED | msb.DEFERRED,
                                           want_shifts=True, allow=allow)
        tr = shift_true_residuals(ctx, b, a, sig, xs)
        del xs
        torch.cuda.empty_cache()
        row["mixed-deferred"].update({"max_true_resid": float(tr.max()),
                                      "median_true_resid": float(np.median(tr)),
                                      "worst_shift": int(np.unravel_index(np.argmax(tr), tr.shape)[1]),
                                      "seed_true_resid_max": float(tr[:, 0].max()),
                                      "meets_tol": bool(tr.max() <= tol)})
        out[f"{tol:.0e}"] = row
        log(f"[bench] mixed floor tol {tol:.0e}: {row}")
    return out


def true_residual_check(ctx, b, a, sig, w, l, tol, y_head):
    """Every shift's FP64 true residual ||b - (A + sigma_s) x_s|| / ||b|| for
    the 12-source batch, from the deferred single pass (which keeps the x_s and
    runs the same iteration as the headline pseudo-double pass), with A applied
    by wilson_apply; and the distance between that pass's y and the
    headline's."""
    import numpy as np
    import torch
    from paper_1010_2592_amd import msb
    y1, info, xs = ctx.mshift_bicgstabl(b, a, sig, w, l, tol, 2000, 1, flags=msb.DEFERRED, want_shifts=True,
                                        allow=(msb.OK, msb.NOT_CONVERGED))
    tr = shift_true_residuals(ctx, b, a, sig, xs)
    d = float(torch.linalg.vector_norm(y1 - y_head) / torch.linalg.vector_norm(y_head))
    out = {"max_true_resid": float(tr.max()), "max_shift_resid": float(np.max(info.shift_resid)),
           "freeze_threshold": 0.9 * tol, "pass1_vs_headline_y": d, "status": info.status}
    del y1, xs
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--pass", dest="pass_", type=int, default=3, choices=(1, 2, 3),
                    help="1 single pass, 2 double pass, 3 pseudo-double pass (Mv outputs stored)")
    ap.add_argument("--precision", default="fp64", choices=("fp64", "mixed"))
    ap.add_argument("--deferred", default="auto", choices=("auto", "on", "off"),
                    help="pass 1: shift vectors updated once per outer iteration; auto: on for pass 1")
    ap.add_argument("--seed-basis", default="auto", choices=("auto", "on", "off"),
                    help="passes 2, 3 and the deferred pass 1 (FP64, stages): the seed's lower vectors as "
                         "coefficients on the outer iteration's basis; auto: on where it applies")
    ap.add_argument("--refine", default="auto", choices=("auto", "on", "off"),
                    help="per-shift FP64 true residual + refinement (pass 1); auto: on for mixed pass 1")
    ap.add_argument("--launch", default="stages", choices=("stages", "persistent"),
                    help="one launch per stage, or the whole pass in one cooperative launch")
    ap.add_argument("--variants", default="all", choices=("all", "none"))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the true-residual check after the timed steps (profiler runs: its solves "
                         "would be counted with the headline's)")
    ap.add_argument("--max-outer", type=int, default=2000)
    ap.add_argument("--block", default=None, choices=("mu0", "propagators", "deflation", "cfg4"),
                    help="run only this extra block on the headline inputs and print its JSON "
                         "(for profiling it alone); the headline line is not printed")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy a 1 GiB tensor 3 times (reference kernel of known size "
                         "for the rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU: the 12 sources are independent "
                                   "and would shard one batch per GPU with no communication; run "
                                   "with --gpus 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as wl
    from paper_1010_2592_amd import msb

    wk = wl.WORKLOADS[WORKLOAD]
    l = wk.ells[0]
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        xc = torch.ones(1 << 26, dtype=torch.complex128, device=dev)   # 1 GiB
        for _ in range(3):
            yc = xc.clone()
        torch.cuda.synchronize()
        del xc, yc
        log("[bench] copy calibration: 3 x clone of 1 GiB")
    log(f"[bench] building inputs {WORKLOAD}")
    U = torch.from_numpy(wk.links()).to(dev)
    b = torch.from_numpy(wl.point_sources(wk.dims)).to(dev)
    ctx = msb.Context(msb.Lattice(wk.dims, wk.mass, wk.mu, wk.bc_t), U)
    rho = ctx.spectral_radius(torch.from_numpy(wk.power_start()[None]).to(dev), 100)
    a = 1.0 / (1.01 * rho)
    sig, w = msb.neuberger_pfe(wk.n_shift)
    if args.block:
        ctx.close()
        if args.block == "mu0":
            out = mu0_block(wk, U, b, sig, w, l, with_cpu=not args.no_cpu)
        elif args.block == "propagators":
            out = propagator_block(wk, U, b, l, with_cpu=not args.no_cpu)
        elif args.block == "cfg4":
            del U, b
            torch.cuda.empty_cache()
            out = config4_block()
        else:
            out = deflation_block(wk, U, b, sig, w, l, with_cpu=not args.no_cpu)
        print(json.dumps({"block": args.block, "workload": WORKLOAD, "result": out}), flush=True)
        return
    mixed = args.precision == "mixed"
    persistent = args.launch == "persistent"
    refine = args.pass_ == 1 and (args.refine == "on" or (args.refine == "auto" and mixed))
    deferred = args.pass_ == 1 and args.deferred != "off" and not persistent
    basis = (args.pass_ != 1 or deferred) and not mixed and not persistent and args.seed_basis != "off"
    log(f"[bench] spectral radius {rho:.6f}; headline pass={args.pass_} {args.precision} {args.launch}")

    for i in range(args.warmup):
        _, info, ms, _ = run_variant(ctx, b, a, sig, w, l, wk.tol, args.max_outer, args.pass_, mixed, persistent,
                                     refine=refine, deferred=deferred, basis=basis)
        log(f"[bench] warmup {i}: {ms:.1f} ms, M={info.outer_iters}, status {info.status}")

    # ---- timed steps (library timing hook on the stencil launches only, every
    # STENCIL_SAMPLE-th of them: the events take time on the stream, and the
    # roofline needs the stencil's average launch duration alone) ----
    ctx.profile_enable(True, classes=("stencil",), stride=STENCIL_SAMPLE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    infos = []
    y = None
    for k in range(args.steps):
        y, info, _ = ctx.mshift_bicgstabl(b, a, sig, w, l, wk.tol, args.max_outer, args.pass_,
                                          flags=solver_flags(mixed, persistent, refine, deferred, basis),
                                          allow=(msb.OK, msb.NOT_CONVERGED, msb.REDUCED_ACCURACY))
        infos.append(info)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps
    nrhs = b.shape[0]
    value = nrhs * args.steps / (ms_total / 1e3)
    info = infos[-1]
    st = prof["stencil"]
    achieved = st["bytes"] / (st["ms"] / 1e3) / 1e9 if st["ms"] > 0 else 0.0
    log(f"[bench] {args.steps} steps: {ms_step:.1f} ms/step (wall {wall:.2f} s), M={info.outer_iters}, "
        f"Mv={info.mv_count}, stencil {achieved:.0f} GB/s over {st['count']} sampled launches "
        f"(every {STENCIL_SAMPLE}th)")
    # every kernel class, from one more (untimed) step with all of them recorded
    ctx.profile_enable(True)
    ctx.mshift_bicgstabl(b, a, sig, w, l, wk.tol, args.max_outer, args.pass_,
                         flags=solver_flags(mixed, persistent, refine, deferred, basis),
                         allow=(msb.OK, msb.NOT_CONVERGED, msb.REDUCED_ACCURACY))
    prof_all = ctx.profile_read()
    ctx.profile_enable(False)
    for k, v in prof_all.items():
        if v["count"]:
            gbs = v["bytes"] / (v["ms"] / 1e3) / 1e9 if v["ms"] > 0 else 0
            log(f"[bench]   {k:16s} {v['count']:7d} launches {v['ms']:10.2f} ms {gbs:8.0f} GB/s")

    # ---- accuracy of the headline result (outside the timed region) ----
    if args.no_accuracy:
        accuracy = {"max_true_resid": None, "skipped": "--no-accuracy"}
    else:
        accuracy = true_residual_check(ctx, b, a, sig, w, l, wk.tol, y)
    accuracy["headline_shift_resid_max"] = float(np.max(info.shift_resid))
    log(f"[bench] accuracy: {accuracy}")
    # the headline form at CPU_ITERS forced outer iterations, for the oracle
    # comparison of the CPU leg
    yK = None
    if not args.no_cpu:
        yK = ctx.mshift_bicgstabl(b, a, sig, w, l, wk.tol, CPU_ITERS, args.pass_,
                                  flags=solver_flags(mixed, persistent, refine, deferred, basis),
                                  force_iters=np.full(len(sig), CPU_ITERS),
                                  allow=(msb.OK, msb.NOT_CONVERGED, msb.REDUCED_ACCURACY))[0].cpu().numpy()

    result = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "f(A)b/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if not mixed else "f32+f64",   # mixed: FP32 stencil/vectors, FP64 reductions/accumulators
        "data": "synthetic",
        "config": {"workload": f"{WORKLOAD} Wilson-Dirac mu=0.05 m=-2, 12 point sources, "
                               f"Neuberger N_s={wk.n_shift}, BiCGstab(l={l}), tol {wk.tol}",
                   "pass": args.pass_, "precision": args.precision, "deferred": deferred, "seed_basis": basis,
                   "refine": refine,
                   "launch": args.launch,
                   "rhs": nrhs,
                   "n_shift": wk.n_shift, "l": l, "outer_iters": info.outer_iters,
                   "mv_count": info.mv_count, "status": info.status,
                   "max_shift_resid": float(np.max(info.shift_resid)),
                   "max_true_resid": accuracy["max_true_resid"],
                   "refined_shifts": info.refined_shifts},
        "accuracy": accuracy,
        "hbm_GBps_whole_call": round(info.bytes_model / (ms_step / 1e3) / 1e9, 1),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(workload_key(args.pass_, args.precision, refine, persistent,
                                                              deferred, basis)),
                     "kernel": "dslash (Wilson stencil, all epilogues)",
                     "launches_sampled": st["count"], "sample_stride": STENCIL_SAMPLE,
                     "avg_launch_us": round(st["ms"] * 1e3 / max(st["count"], 1), 2),
                     "bytes_per_launch": round(st["bytes"] / max(st["count"], 1))},
        # per kernel class over one untimed step (every launch bracketed by events)
        "kernel_classes": {k: {"launches": v["count"], "ms": round(v["ms"], 3),
                               "GBps": round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1) if v["ms"] > 0 else None}
                           for k, v in prof_all.items() if v["count"]},
    }

    # ---- comparison forms, one run each ----
    if args.variants == "all":
        comps = {}
        ref = None
        # (pass, mixed, persistent, refine, deferred, seed basis)
        forms = [(1, False, False, False, False, False), (2, False, False, False, False, False),
                 (2, False, False, False, False, True), (1, True, False, False, False, False),
                 (2, True, False, False, False, False), (1, True, False, True, False, False),
                 (1, False, False, False, True, False), (1, False, False, False, True, True),
                 (1, True, False, False, True, False),
                 (1, True, False, True, True, False), (1, False, True, False, False, False),
                 (2, False, True, False, False, False), (1, True, True, False, False, False),
                 (1, True, True, True, False, False), (2, True, True, False, False, False),
                 (3, False, False, False, False, False), (3, False, False, False, False, True),
                 (3, True, False, False, False, False)]
        for (p, mx, pe, rf, df, sb) in forms:
            name = (f"{p}pass-{'mixed' if mx else 'fp64'}{'-refine' if rf else ''}{'-deferred' if df else ''}"
                    f"{'-basis' if sb else ''}-{'persistent' if pe else 'stages'}")
            try:
                # one warm-up, then the median of VARIANT_REPS runs (the
                # last of them with the kernel timing hook on)
                run_variant(ctx, b, a, sig, w, l, wk.tol, min(args.max_outer, 400), p, mx, pe, refine=rf,
                            deferred=df, basis=sb)
                times = []
                for rep in range(VARIANT_REPS):
                    yv, iv, msv, pv = run_variant(ctx, b, a, sig, w, l, wk.tol, min(args.max_outer, 400), p,
                                                  mx, pe, profile=rep == VARIANT_REPS - 1, refine=rf, deferred=df,
                                                  basis=sb)
                    times.append(msv)
                    if rep < VARIANT_REPS - 1:
                        del yv
                msv = float(np.median(times))
            except msb.MsbError as e:
                comps[name] = {"error": str(e)}
                continue
            if ref is None:
                ref = yv
            err = float(torch.linalg.norm(yv - ref) / torch.linalg.norm(ref))
            comps[name] = {"ms": round(msv, 2), "ms_runs": [round(t, 2) for t in times],
                           "outer_iters": iv.outer_iters, "mv": iv.mv_count,
                           "status": iv.status, "reliable_updates": iv.reliable_updates,
                           "GBps_model": round(iv.bytes_model / (msv / 1e3) / 1e9, 1),
                           "rel_diff_vs_1pass_fp64": err,
                           "max_shift_resid": float(np.max(iv.shift_resid)),
                           "max_true_resid": (float(np.max(iv.shift_true_resid))
                                              if iv.shift_true_resid is not None else None),
                           "refined_shifts": iv.refined_shifts,
                           "shift_update_GBps": (round(pv["shift_update"]["bytes"] / (pv["shift_update"]["ms"] / 1e3) / 1e9, 1)
                                                 if pv["shift_update"]["ms"] > 0 else None),
                           "stencil_GBps": (round(pv["stencil"]["bytes"] / (pv["stencil"]["ms"] / 1e3) / 1e9, 1)
                                            if pv["stencil"]["ms"] > 0 else None)}
            log(f"[bench] {name}: {comps[name]}")
            del yv
            torch.cuda.empty_cache()
        result["variants"] = comps
        result["mixed_floor"] = mixed_floor_block(ctx, b, a, sig, w, l)

    ctx.close()
    torch.cuda.empty_cache()
    if args.variants == "all":
        result["mu0"] = mu0_block(wk, U, b, sig, w, l, with_cpu=not args.no_cpu)
        result["propagators"] = propagator_block(wk, U, b, l, with_cpu=not args.no_cpu)
        result["deflation"] = deflation_block(wk, U, b, sig, w, l, with_cpu=not args.no_cpu)

    if not args.no_cpu:
        log("[bench] CPU oracle sample ...")
        try:
            base, ys = cpu_baseline(wk, a, sig, w, l, int(info.outer_iters))
        except Exception as e:   # worker processes unavailable: one source in this process
            log(f"[bench] CPU workers failed ({e}); timing one source in this process")
            base, ys = cpu_baseline_single(wk, a, sig, w, l, int(info.outer_iters),
                                           f"worker processes failed: {type(e).__name__}")
        result["cpu_baseline"] = base
        # the oracle's y after CPU_ITERS forced outer iterations against the
        # headline form's at the same forced iterations, source by source
        errs = {int(k): float(np.linalg.norm(yK[k] - yo) / np.linalg.norm(yo)) for k, yo in ys.items()}
        accuracy["oracle_forced_outer"] = CPU_ITERS
        accuracy["oracle_rel_err_max"] = max(errs.values())
        accuracy["oracle_rel_err_sources"] = len(errs)
        log(f"[bench] y vs oracle at {CPU_ITERS} forced outer iterations: max {max(errs.values()):.2e} "
            f"over {len(errs)} sources")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
