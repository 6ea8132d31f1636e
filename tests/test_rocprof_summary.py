"""The traffic record written from rocprofv3 databases: bytes read beyond
L2 are 64 B x TCC_MISS (checked against a 1 GiB copy in the same run, whose
reading must come to 1.000 of its bytes), bytes written are WRITE_SIZE, and
only the stencil dispatches of the solves count (from the first sc_init on:
the spectral-radius estimate's stencils before it are left out)."""
import json
import sqlite3
import sys

from paper_1010_2592_amd import rocprof_summary as rs

GiB_KiB = 1048576.0


def make_db(path, kernels=(), counters=()):
    con = sqlite3.connect(path)
    con.execute("create table kernels (name text, start integer, end integer)")
    con.execute("create table counters_collection (kernel_name text, dispatch_id integer, counter_name text, "
                "value real)")
    con.executemany("insert into kernels values (?, ?, ?)", kernels)
    con.executemany("insert into counters_collection values (?, ?, ?, ?)", counters)
    con.commit()
    con.close()


def dispatches(counter, copy_value, pre_value, chunk_values):
    """copy x3, two pre-solve single-source stencils, sc_init, the chunks"""
    rows, d = [], 0
    for _ in range(3):
        rows.append(("__amd_rocclr_copyBuffer", d, counter, copy_value))
        d += 1
    for _ in range(2):
        rows.append(("void dslash_kernel<double, 0, true>(DslashArgs<double>)", d, counter, pre_value))
        d += 1
    rows.append(("sc_init(ScalarArgs)", d, counter, 1.0))
    d += 1
    for v in chunk_values:
        rows.append(("void dslash_chunk_kernel<double, 0, false>(DslashArgs<double>)", d, counter, v))
        d += 1
    return rows


def test_traffic_from_l2_miss_sectors(tmp_path, monkeypatch):
    trace, miss, write = (str(tmp_path / n) for n in ("t.db", "m.db", "w.db"))
    make_db(trace, kernels=[("void dslash_kernel<double, 0, true>(DslashArgs<double>)", 0, 10),
                            ("sc_init(ScalarArgs)", 20, 21),
                            ("void dslash_chunk_kernel<double, 0, false>(DslashArgs<double>)", 30, 230),
                            ("void dslash_chunk_kernel<double, 0, false>(DslashArgs<double>)", 240, 440)])
    # a 1 GiB copy reads 2^24 sectors of 64 B; the chunks 1e7 and 9e6 sectors
    make_db(miss, counters=dispatches("TCC_MISS_sum", 16777216.0, 5.0e9, [1.0e7, 9.0e6]))
    make_db(write, counters=dispatches("WRITE_SIZE", GiB_KiB, 1.0e9, [2.5e5, 2.5e5]))
    bj = tmp_path / "b.json"
    bj.write_text(json.dumps({"config": {"pass": 3, "precision": "fp64", "refine": False, "launch": "stages"},
                              "roofline": {"bytes_per_launch": 5.0e8, "achieved": 2500.0, "peak": 8000.0,
                                           "frac": 0.3125, "avg_launch_us": 200.0, "launches_sampled": 2,
                                           "sample_stride": 1}}))
    md, js = tmp_path / "s.md", tmp_path / "s.json"
    monkeypatch.setattr(sys, "argv", ["rocprof_summary", "--trace", trace, "--miss", miss, "--write", write,
                                      "--bench-json", str(bj), "--workload", "w", "--md", str(md),
                                      "--json", str(js), "--cmd-trace", "t", "--cmd-fetch", "m",
                                      "--cmd-write", "w"])
    rs.main()
    rec = json.loads(js.read_text())
    assert rec["read_counter"] == "64 B x TCC_MISS_sum"
    assert abs(rec["read_scale"] - 1.0) < 1e-12 and abs(rec["write_scale"] - 1.0) < 1e-12
    read = 64.0 * (1.0e7 + 9.0e6) / 2
    written = 2.5e5 * 1024.0
    assert rec["traffic_bytes_per_launch"] == round(read + written)
    text = md.read_text()
    assert "2 / 2 stencil dispatches of the solves" in text
