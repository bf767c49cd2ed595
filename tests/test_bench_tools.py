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


def test_committed_traffic_follows_the_source_hash(tmp_path):
    """The traffic figure is read only while the kernel source still has the
    SHA-256 recorded with the counters; any change to the source nulls it."""
    import hashlib

    import bench

    src_rel = bench.KERNEL_SOURCES["k_zgemm_family"]
    src = tmp_path / src_rel
    src.parent.mkdir(parents=True)
    src.write_bytes(b"kernel source v1\n")
    prof = tmp_path / "profiles"
    prof.mkdir()
    sha = hashlib.sha256(b"kernel source v1\n").hexdigest()
    (prof / "k_zgemm_family_n8192_nev820_seq12_hbm_counters.txt").write_text(
        "# comment: ignored\ntraffic_bytes_per_launch: 12345\n"
        f"source: {src_rel}\nsource_sha256: {sha}\n")
    assert bench.committed_traffic("k_zgemm_family", root=str(tmp_path)) == 12345.0
    src.write_bytes(b"kernel source v2\n")
    assert bench.committed_traffic("k_zgemm_family", root=str(tmp_path)) is None
    assert bench.committed_traffic("k_unknown", root=str(tmp_path)) is None


def test_committed_profiles_are_consistent():
    """Each committed counter summary either matches its source's current
    hash (and then gives a positive figure) or is reported as stale (None),
    never a figure for a source it was not taken on."""
    import hashlib

    import bench

    for kernel, src in bench.KERNEL_SOURCES.items():
        for name in os.listdir(os.path.join(ROOT, "profiles")):
            if not (name.startswith(kernel + "_") and name.endswith("_hbm_counters.txt")):
                continue
            workload = name[len(kernel) + 1:-len("_hbm_counters.txt")]
            vals = dict(line.split(":", 1) for line in open(os.path.join(ROOT, "profiles", name))
                        if ":" in line and not line.startswith("#"))
            sha = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()
            got = bench.committed_traffic(kernel, workload)
            if vals.get("source_sha256", "").strip() == sha:
                assert got is not None and got > 0, name
            else:
                assert got is None, name


def test_rocprof_summary_family_and_counters(tmp_path):
    """The summary's family average inside the 'timed' range (helpers add
    time, not launches), the per-dispatch counter average over the last L
    launches of the family, and the calibration factor from the 1 GiB copy."""
    import bench

    path = str(tmp_path / "c.db")
    con = sqlite3.connect(path)
    cur = con.cursor()
    cur.execute("create table regions (extdata text, start int, end int)")
    cur.execute("create table kernels (name text, start int, end int)")
    cur.execute("create table counters_collection (kernel_name text, counter_name text, value real, "
                "start int, grid_size int)")
    cur.execute("insert into regions values (?, ?, ?)", (json.dumps({"message": "timed"}), 1000, 10_000))
    # main kernel: one launch before the range, two inside; helper: one inside
    for s0, e0 in ((0, 500), (2000, 3000), (4000, 6000)):
        cur.execute("insert into kernels values (?, ?, ?)", ("k_main(P)", s0, e0))
    cur.execute("insert into kernels values (?, ?, ?)", ("k_help(P)", 3000, 3500))
    # counters: main launches 100, 200, 300 KiB, helper 50 KiB before the last
    for st, v in ((0, 100.0), (2000, 200.0), (4000, 300.0)):
        cur.execute("insert into counters_collection values (?, ?, ?, ?, ?)",
                    ("k_main(P)", "FETCH_SIZE", v, st, 1024))
    cur.execute("insert into counters_collection values (?, ?, ?, ?, ?)",
                ("k_help(P)", "FETCH_SIZE", 50.0, 3000, 1024))
    cur.execute("insert into counters_collection values (?, ?, ?, ?, ?)",
                ("__amd_rocclr_copyBuffer", "FETCH_SIZE", 524288.0, 0, 131072))
    con.commit()
    con.close()
    out = bench.rocprof_summary(path, "k_main|+k_help", pmc_last=2)
    assert "k_main: launches inside roctx range 'timed' 2, avg 0.0015 ms" in out
    # family: (1000 + 2000 + 500) ns over 2 launches
    assert "family inside 'timed': 2 launches, total 0.0 ms, avg per launch (helpers included) 0.0018 ms" in out
    # last 2 main dispatches (200, 300) plus the helper between them (50): 550 / 2
    assert "pmc FETCH_SIZE per dispatch over the last 2 (timed) dispatches (helpers included) 275.0 KiB" in out
    assert "factor to true bytes 2.0000" in out
