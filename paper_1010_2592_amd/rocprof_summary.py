"""Summaries of rocprofv3 runs of bench.py for profiles/.

    python -m paper_1010_2592_amd.rocprof_summary trace --trace T.db --title ... --workload ... \
        --md profiles/X.md --cmd-trace "..." [--kernel-bytes NAME=BYTES ...]

writes the kernel table of one kernel-trace run (any bench.py command).  The
form below is the stencil's: trace, counters and the traffic record.

    python -m paper_1010_2592_amd.rocprof_summary --trace T.db --miss M.db --write W.db \
        --bench-json B.json --workload "16x16x16x32 12 rhs mixed pass 1 refine" \
        --md profiles/X.md --json profiles/dslash_traffic.json --cmd-trace "..." --cmd-fetch "..." --cmd-write "..."

Inputs are the rocpd databases rocprofv3 writes (-d DIR -o NAME gives
DIR/NAME_results.db) of three runs of the same bench command: a kernel trace
with --stats, a TCC_MISS_sum counter run (or FETCH_SIZE, --fetch) and a
WRITE_SIZE counter run (each counter in a run of its own).  Bytes read from
beyond L2 are 64 x TCC_MISS: the L2 counts its misses in 64-byte sectors
and the memory requests of a miss fetch exactly those sectors (128-byte
requests for two, 64-byte for one).  FETCH_SIZE's expression takes 128-byte
requests from TCC_BUBBLE, which reads zero on this part, and so counts them
as 64 bytes: a factor that a copy (all 128-byte requests) calibrates to 2
but that overstates a kernel issuing 64-byte requests too.  The counter runs
include bench.py --calibrate-copy: three copies of a 1 GiB tensor, which
check each reading (1048576 KiB read and written) and give its factor.

Outputs: a markdown summary (kernel table, stencil launch statistics, HBM
bytes per stencil launch against the algorithmic bytes) and the JSON record
bench.py reads for roofline.traffic, keyed by a hash of the stencil sources
so that it lapses when the stencil changes.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sqlite3

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# the stencil kernels, and the solver that chooses which of their epilogues
# run: a change to either lapses the measured traffic
STENCIL_SOURCES = ["paper_1010_2592_amd/csrc/stencil_dev.h", "paper_1010_2592_amd/csrc/dslash.hip",
                   "paper_1010_2592_amd/csrc/solver.hip"]
COPY_KIB = 1048576.0


def sources_hash(paths=STENCIL_SOURCES) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def is_stencil(name: str) -> bool:
    return "dslash" in name and "link_force" not in name


def short(name: str) -> str:
    return name.replace("msb::(anonymous namespace)::", "").replace("msb::", "")


def kernel_rows(db):
    cur = sqlite3.connect(db).cursor()
    return cur.execute("select name, count(*), avg(end - start), sum(end - start) from kernels "
                       "group by name order by sum(end - start) desc").fetchall()


def stencil_launches(db):
    """Stencil launches of the solves: those after the first solve begins
    (its sc_init kernel); the spectral-radius estimate runs before it."""
    cur = sqlite3.connect(db).cursor()
    rows = cur.execute("select name, start, end from kernels order by start").fetchall()
    t0 = min((s for n, s, e in rows if "sc_init" in n), default=0)
    return [(n, e - s) for n, s, e in rows if is_stencil(n) and s >= t0]


def counter_values(db, counter):
    cur = sqlite3.connect(db).cursor()
    return cur.execute("select kernel_name, dispatch_id, value from counters_collection where counter_name = ? "
                       "order by dispatch_id", (counter,)).fetchall()


def solve_dispatches(rows):
    """Counter rows of the solves: dispatches after the first solve begins
    (its sc_init kernel), as for the trace; the spectral-radius estimate's
    single-source stencils before it would dilute the per-launch average."""
    t0 = min((d for n, d, v in rows if "sc_init" in n), default=-1)
    return [(n, d, v) for n, d, v in rows if d > t0]


def scale(rows):
    """Counter units per byte from the 1 GiB copies (the three largest copy dispatches)."""
    copies = sorted((v for n, d, v in rows if "copyBuffer" in n), reverse=True)[:3]
    if not copies:
        return None
    return COPY_KIB / (sum(copies) / len(copies))


def trace_main(argv):
    """Kernel table of one --kernel-trace run, with the algorithmic bandwidth
    of the kernels given as NAME=BYTES (bytes per launch; NAME matches a
    substring of the kernel name)."""
    ap = argparse.ArgumentParser(prog="rocprof_summary trace")
    ap.add_argument("--trace", required=True)
    ap.add_argument("--title", required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--md", required=True)
    ap.add_argument("--cmd-trace", required=True)
    ap.add_argument("--kernel-bytes", action="append", default=[])
    ap.add_argument("--top", type=int, default=18)
    a = ap.parse_args(argv)
    rows = kernel_rows(a.trace)
    tot = sum(r[3] for r in rows)
    md = [f"# {a.title}\n", f"Workload: {a.workload}\n",
          "## Kernel trace\n\nCommand (from the repository root on the MI355X box):\n", f"    {a.cmd_trace}\n",
          "| kernel | calls | avg us | total ms | % |\n|---|---|---|---|---|"]
    for n, c, avg, s in rows[:a.top]:
        md.append(f"| `{short(n)[:90]}` | {c} | {avg / 1e3:.2f} | {s / 1e6:.2f} | {100 * s / tot:.1f} |")
    md.append("")
    if a.kernel_bytes:
        md.append("## Algorithmic bandwidth\n\n| kernel | bytes per launch | avg us | GB/s | of 8 TB/s |\n"
                  "|---|---|---|---|---|")
        for kb in a.kernel_bytes:
            name, b = kb.split("=")
            hit = [r for r in rows if name in r[0]]
            if not hit:
                continue
            n, c, avg, s = hit[0]
            gbs = float(b) / (avg / 1e9) / 1e9
            md.append(f"| `{name}` | {float(b) / 1e6:.1f} MB | {avg / 1e3:.1f} | {gbs:.0f} | {100 * gbs / 8000:.0f} % |")
        md.append("")
    os.makedirs(os.path.dirname(os.path.abspath(a.md)), exist_ok=True)
    with open(a.md, "w") as f:
        f.write("\n".join(md))
    print("\n".join(md))


def main():
    import sys
    if len(sys.argv) > 1 and sys.argv[1] == "trace":
        return trace_main(sys.argv[2:])
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", default=None, help="FETCH_SIZE run (older records)")
    ap.add_argument("--miss", default=None, help="TCC_MISS_sum run")
    ap.add_argument("--write", required=True)
    ap.add_argument("--bench-json", required=True, help="bench.py output line of the trace run")
    ap.add_argument("--workload", required=True)
    ap.add_argument("--md", required=True)
    ap.add_argument("--json", required=True)
    ap.add_argument("--cmd-trace", required=True)
    ap.add_argument("--cmd-fetch", required=True)
    ap.add_argument("--cmd-write", required=True)
    ap.add_argument("--top", type=int, default=18)
    a = ap.parse_args()

    bench = json.loads(open(a.bench_json).read().strip().splitlines()[-1])
    rows = kernel_rows(a.trace)
    tot = sum(r[3] for r in rows)
    st = stencil_launches(a.trace)
    st_avg_us = sum(d for _, d in st) / len(st) / 1e3
    if a.miss:
        # 64-byte sectors; the copy check gives its factor in KiB units
        fr = [(n, d, v * 64.0 / 1024.0) for n, d, v in counter_values(a.miss, "TCC_MISS_sum")]
        read_name = "64 B x TCC_MISS_sum"
    else:
        fr = counter_values(a.fetch, "FETCH_SIZE")
        read_name = "FETCH_SIZE"
    wr = counter_values(a.write, "WRITE_SIZE")
    fs, ws = scale(fr), scale(wr)
    f_st = [v for n, d, v in solve_dispatches(fr) if is_stencil(n)]
    w_st = [v for n, d, v in solve_dispatches(wr) if is_stencil(n)]
    fetch_b = sum(f_st) / len(f_st) * fs * 1024.0
    write_b = sum(w_st) / len(w_st) * ws * 1024.0
    traffic = fetch_b + write_b
    roof = bench["roofline"]
    alg = roof["bytes_per_launch"]

    md = []
    md.append(f"# Wilson stencil: {a.workload}\n")
    md.append("Workload: bench.py headline (16^3x32, mu = 0.05, m = -2, Neuberger N_s = 30, "
              "BiCGstab(l = 4), tol 1e-8, the 12 point sources in one batch); "
              f"form: {bench['config'].get('pass')}-pass, {bench['config'].get('precision')}, "
              f"seed basis {bench['config'].get('seed_basis', False)}, "
              f"refine {bench['config'].get('refine')}, {bench['config'].get('launch')} launches.\n")
    md.append("## Kernel trace\n\nCommand (from the repository root on the MI355X box):\n")
    md.append(f"    {a.cmd_trace}\n")
    md.append("| kernel | calls | avg us | total ms | % |\n|---|---|---|---|---|")
    for n, c, avg, s in rows[:a.top]:
        md.append(f"| `{short(n)[:90]}` | {c} | {avg / 1e3:.2f} | {s / 1e6:.2f} | {100 * s / tot:.1f} |")
    md.append("")
    md.append(f"Stencil launches of the solves (all `dslash` kernels, site-block and chunked, every "
              f"epilogue and precision, from the first solve on -- the spectral-radius estimate before "
              f"it is not part of a step; warm-up and timed steps): {len(st)} launches, average "
              f"{st_avg_us:.1f} us.  "
              f"bench.py's live HIP-event figure over its timed steps in the same run: "
              f"{roof['avg_launch_us']:.1f} us over {roof.get('launches_sampled', roof.get('launches'))} "
              f"launches (every {roof.get('sample_stride', 1)}th stencil launch of those steps) "
              f"({100 * abs(roof['avg_launch_us'] - st_avg_us) / st_avg_us:.1f} % apart).\n")
    md.append("## Traffic beyond L2 (rocprofv3 --pmc, one counter per run)\n\nCommands:\n")
    md.append(f"    {a.cmd_fetch}\n    {a.cmd_write}\n")
    md.append(f"Check (1 GiB copy, 1048576 KiB read and written): {read_name} x{fs:.3f}, "
              f"WRITE_SIZE x{ws:.3f}.\n")
    md.append("| per stencil launch | bytes |\n|---|---|")
    md.append(f"| read ({read_name}, scaled) | {fetch_b / 1e6:.1f} MB |")
    md.append(f"| WRITE_SIZE (scaled) | {write_b / 1e6:.1f} MB |")
    md.append(f"| traffic | {traffic / 1e6:.1f} MB |")
    md.append(f"| algorithmic (bench.py model) | {alg / 1e6:.1f} MB |")
    md.append(f"| traffic / algorithmic | {traffic / alg:.2f} |\n")
    md.append(f"Roofline of the timed steps: {roof['achieved']:.0f} GB/s algorithmic of {roof['peak']:.0f} "
              f"GB/s ({100 * roof['frac']:.1f} %); {len(f_st)} / {len(w_st)} stencil dispatches of the solves "
              f"counted (from the first solve's sc_init on, as in the trace table).\n")
    os.makedirs(os.path.dirname(os.path.abspath(a.md)), exist_ok=True)
    with open(a.md, "w") as f:
        f.write("\n".join(md))
    rec = {"kernel": "Wilson stencil (dslash_kernel and dslash_chunk_kernel, all epilogues and precisions)",
           "sources": STENCIL_SOURCES, "sources_sha256_16": sources_hash(),
           "workload": a.workload, "traffic_bytes_per_launch": round(traffic),
           "read_counter": read_name, "read_scale": fs, "write_scale": ws,
           "algorithmic_bytes_per_launch": alg,
           "summary": os.path.relpath(os.path.abspath(a.md), ROOT)}
    with open(a.json, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
