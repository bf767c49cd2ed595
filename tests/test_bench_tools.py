"""Host-side checks of the profile tooling in bench.py that committed
summaries under profiles/ are produced with: the trace breakdown's kernel
totals, grid-size buckets and per-family concurrency (union of launch
intervals), on a synthetic rocprofv3-shaped database."""
import json
import os
import sqlite3
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _db(tmp_path, kernels, region=(0, 1_000_000)):
    path = str(tmp_path / "t.db")
    con = sqlite3.connect(path)
    cur = con.cursor()
    cur.execute("create table regions (extdata text, start int, end int)")
    cur.execute("create table kernels (name text, grid_x int, workgroup_x int, start int, end int)")
    cur.execute("insert into regions values (?, ?, ?)", (json.dumps({"message": "timed"}),) + region)
    for k in kernels:
        cur.execute("insert into kernels values (?, ?, ?, ?, ?)", k)
    con.commit()
    con.close()
    return path


def test_breakdown_totals_and_concurrency(tmp_path):
    import bench

    g = "void (anonymous namespace)::k_zgemm<0>(P)"
    f = "(anonymous namespace)::k_cgemm_bf16x3_filter(P)"
    path = _db(tmp_path, [
        (g, 256 * 100, 256, 0, 400_000),          # 100 work-groups, 0.4 ms
        (f, 256 * 300, 256, 100_000, 300_000),    # two filter launches overlapping each other
        (f, 256 * 300, 256, 200_000, 500_000),
        (g, 256 * 5000, 256, 600_000, 700_000),   # 5000 work-groups
        ("x", 256, 256, 2_000_000, 3_000_000),    # outside the range: ignored
    ])
    out = bench.rocprof_breakdown(path)
    assert "roctx range 'timed': 1.0 ms; 4 kernels inside it" in out
    # busy: union of [0, 0.5] and [0.6, 0.7] ms
    assert "busy (any kernel running) 0.6 ms" in out
    assert "k_zgemm<0>                       n=     2 total=     0.50 ms" in out
    assert "grid <256    n=     1" in out and "grid >=4096  n=     1" in out
    # one idle gap, 0.5 -> 0.6 ms, between the filter and the GEMM
    assert "idle gaps: 1, 0.1 ms in total" in out
    assert "k_cgemm_bf16x3_filter        -> k_zgemm<0>" in out
    # filter: summed 0.5 ms over a union of 0.4 ms -> concurrency 1.25
    assert ("family k_cgemm_bf16x3_filter: 2 launches, summed kernel time 0.5 ms, wall time with one "
            "or more running 0.4 ms (40.0% of the range), average concurrency 1.25") in out


def test_breakdown_without_range(tmp_path):
    import bench

    path = _db(tmp_path, [], region=(0, 1))
    con = sqlite3.connect(path)
    con.execute("delete from regions")
    con.commit()
    con.close()
    assert "no roctx range 'timed'" in bench.rocprof_breakdown(path)
