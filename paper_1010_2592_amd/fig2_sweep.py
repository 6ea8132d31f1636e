"""Run time against the number of shifts at a fixed Krylov dimension Ml, for
the single-, double- and pseudo-double-pass forms and l = 1, 2, 4, 8: the
measurement of the paper's Fig. 2 (Section 3), on one MI355X.

    python -m paper_1010_2592_amd.fig2_sweep [--dims 12 12 12 24] [--ml 256]
        [--ls 1 2 4 8] [--ns 2 4 8 16 32 64] [--reps 3] [--json OUT]

Every shift's freeze iteration is forced to M = Ml / l outer iterations, so
each solve runs exactly Ml BiCG steps whatever N_s (the figure's premise:
the work per shift is fixed and only the number of shifts varies).  Inputs:
seeded SU(3) links (eps 0.5), m = -2, mu = 0.05, antiperiodic in time, one
Gaussian source, Neuberger poles for each N_s, a = 1 / (1.01 rho) from the
library's power iteration.  Times: HIP events around each call on the
context's stream, median of --reps runs after one warm-up run.  Forms:
1-pass (the paper's per-step shift updates), 1-pass deferred, 2-pass,
3-pass (pseudo-double), and the last three with the seed's BiCG steps in
basis form (MSB_SEED_BASIS).  Output: one line per measurement as it finishes, a
markdown table at the end, and the raw numbers as JSON with --json.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


FORMS = (("1-pass", 1, "plain"), ("1-pass deferred", 1, "deferred"), ("2-pass", 2, "plain"),
         ("3-pass", 3, "plain"), ("1-pass deferred basis", 1, "deferred basis"), ("2-pass basis", 2, "basis"),
         ("3-pass basis", 3, "basis"))


def sweep(dims, ml, ls, ns_list, reps, log=print):
    """The measurement: one row per (l, N_s, form) with the median time of
    `reps` runs after a warm-up, the Mv count and the outer iterations."""
    import numpy as np
    import torch

    import workloads as wl
    from paper_1010_2592_amd import msb

    dims = tuple(dims)
    U = torch.as_tensor(wl.gauge_links(dims, 0.5, 1006)).cuda()
    b = torch.as_tensor(wl.gaussian_source(dims, 2006, 1)).cuda()
    ctx = msb.Context(msb.Lattice(dims, -2.0, 0.05, -1), U)
    rho = ctx.spectral_radius(torch.as_tensor(wl.start_vector(dims, 4006)[None]).cuda(), 100)
    a = 1.0 / (1.01 * rho)
    allow = (msb.OK, msb.NOT_CONVERGED, msb.BREAKDOWN)
    vec_mb = 12 * wl.volume(dims) * 16 / 1e6
    log(f"[fig2] {dims}, vector {vec_mb:.1f} MB (FP64), Ml = {ml}, rho = {rho:.6f}")
    rows = []
    for l in ls:
        M = max(ml // l, 1)
        for ns in ns_list:
            sig, w = msb.neuberger_pfe(ns)
            force = np.full(ns, M, dtype=np.int32)
            for name, pass_, kind in FORMS:
                flags = (msb.DEFERRED if kind.startswith("deferred") else 0) | \
                    (msb.SEED_BASIS if kind.endswith("basis") else 0)
                times = []
                for r in range(reps + 1):
                    torch.cuda.synchronize()
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record()
                    y, info, _ = ctx.mshift_bicgstabl(b, a, sig, w, l, 1e-8, M + 1, pass_, flags=flags,
                                                      force_iters=force, allow=allow)
                    e1.record()
                    torch.cuda.synchronize()
                    if r > 0:
                        times.append(e0.elapsed_time(e1))
                    del y
                ms = statistics.median(times)
                rows.append({"l": l, "M": M, "n_shift": ns, "form": name, "pass": pass_, "ms": ms,
                             "mv": info.mv_count, "outer": info.outer_iters, "status": info.status,
                             "shift_vectors_GB": (ns * (l + 1) * vec_mb / 1e3) if pass_ == 1 else 0.0})
                log(f"[fig2] l={l} M={M} N_s={ns:3d} {name:16s} {ms:9.2f} ms  Mv {info.mv_count}")
            torch.cuda.empty_cache()
    ctx.close()
    return rho, rows


def table(rows, ls, ns_list):
    """Markdown table: one row per (l, N_s), one column per form (ms)."""
    out = ["| l | N_s | " + " | ".join(f[0] for f in FORMS) + " |", "|---|---|" + "---|" * len(FORMS)]
    for l in ls:
        for ns in ns_list:
            ms = [next(r["ms"] for r in rows if r["l"] == l and r["n_shift"] == ns and r["form"] == f[0])
                  for f in FORMS]
            out.append(f"| {l} | {ns} | " + " | ".join(f"{m:.1f}" for m in ms) + " |")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--dims", type=int, nargs=4, default=[12, 12, 12, 24])
    ap.add_argument("--ml", type=int, default=256)
    ap.add_argument("--ls", type=int, nargs="+", default=[1, 2, 4, 8])
    ap.add_argument("--ns", type=int, nargs="+", default=[2, 4, 8, 16, 32, 64])
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--json", default=None)
    args = ap.parse_args()
    rho, rows = sweep(args.dims, args.ml, args.ls, args.ns, args.reps, log=lambda m: print(m, flush=True))
    print("\n" + table(rows, args.ls, args.ns))
    if args.json:
        with open(args.json, "w") as f:
            json.dump({"dims": list(args.dims), "ml": args.ml, "rho": rho, "rows": rows}, f, indent=1)


if __name__ == "__main__":
    main()
