#!/usr/bin/env python3
"""Per-SCF-step eigensolve time of the seeded solver on one MI355X.

Workload: a 12-step synthetic SCF sequence of dense complex Hermitian pencils
(A_k, B) of order n = 8192, lowest nev = 820 eigenpairs, A_k = A_{k-1} +
eps_k H_k with eps_k = 5e-3 * 0.6^k (the stand-in for the paper's FLEUR
sequences, section 2; built on the GPU by paper_1007_4400_amd.synth).

A "step" is one whole solve of one SCF step: staging, Cholesky, reduction,
bounds, filtered subspace iteration seeded with the previous step's vectors,
back-transform and the FP64 residual check in the original basis.  The first
`--warmup` steps (step 0 is a cold start) are untimed; the next `--steps`
steps are timed between device synchronisations.  Every timed step must pass
max_i ||A x_i - lambda_i B x_i|| <= 1e-10 ||A||_2.

Also reported: the cold-start FP64 solve of the same steps (the comparator),
the filter GEMM's throughput against the MFMA roofline (HIP events around
each filter launch inside the timed region), and the CPU oracle timed on a
bounded sample.  Prints one JSON line.
"""
import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(n_target=8192, sizes=(2048, 4096)):
    """The oracle (plain FP64 CPU solver, all host threads) on one pencil of
    the same construction at each of `sizes`; the value is the largest
    sample scaled by (n_target / n)^3, the solver's dense O(n^3) cost, with
    the exponent measured between the two samples reported beside it."""
    from oracle import oracle
    from paper_1007_4400_amd import synth

    times = {}
    for n in sizes:
        wl = synth.scaled(synth.LARGE, n)
        p, _ = synth.make_pencil(wl, 0)
        t0 = time.perf_counter()
        oracle.solve(p.A, p.B, wl.nev)
        times[n] = time.perf_counter() - t0
        log(f"cpu baseline: oracle solve n={n} nev={wl.nev}: {times[n]:.1f} s")
    n1, n2 = sizes[0], sizes[-1]
    expo = math.log(times[n2] / times[n1]) / math.log(n2 / n1) if n2 != n1 else 3.0
    scale = (n_target / n2) ** 3
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": times[n2] * scale,
        "unit": "s/step",
        "cores": cores,
        "kind": "oracle",
        "sample": f"one oracle solve of a pencil of the same construction at n={n2}, "
                  f"nev={round(0.1 * n2)} ({times[n2]:.1f} s) scaled by (n/{n2})^3 = {scale:.0f} "
                  f"to n={n_target}; at n={n1} it took {times[n1]:.1f} s, a measured exponent of "
                  f"{expo:.2f} between the two (with that exponent: "
                  f"{times[n2] * (n_target / n2) ** expo:.0f} s)",
        "samples_s": {str(k): v for k, v in times.items()},
        "measured_exponent": expo,
    }


def _mark_push(name):
    try:
        import torch

        torch.cuda.nvtx.range_push(name)
    except Exception:
        pass


def _mark_pop():
    try:
        import torch

        torch.cuda.nvtx.range_pop()
    except Exception:
        pass


FILTER_KERNELS = {"fp64": "k_zgemm<1>", "fp32": "k_cgemm32_filter", "bf16x3": "k_cgemm_bf16x3_filter"}


KERNEL_SOURCES = {"k_cgemm_bf16x3_filter": "paper_1007_4400_amd/csrc/cgemm_bf16.hip",
                  "k_cgemm32_filter": "paper_1007_4400_amd/csrc/cgemm32.hip",
                  "k_zgemm<1>": "paper_1007_4400_amd/csrc/zgemm.hip",
                  "k_zgemm_family": "paper_1007_4400_amd/csrc/zgemm.hip",
                  "k_upd_scan": "paper_1007_4400_amd/csrc/update.hip",
                  "k_upd_apply": "paper_1007_4400_amd/csrc/update.hip"}


def committed_traffic(kernel, workload="n8192_nev820_seq12", root=None):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/<kernel>_<workload>_hbm_counters.txt under `root`, the
    repository by default), or None when there is none or the kernel's source
    has changed since the counters were taken (the summary records the
    source's SHA-256)."""
    import hashlib

    here = root or os.path.dirname(os.path.abspath(__file__))
    prof = os.path.join(here, "profiles", f"{kernel}_{workload}_hbm_counters.txt")
    src = KERNEL_SOURCES.get(kernel)
    if not src or not os.path.exists(prof):
        return None
    with open(os.path.join(here, src), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    vals = {}
    with open(prof) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != sha or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def _regions(cur):
    """{message: (start, end)} of the roctx ranges in a rocprofv3 database."""
    out = {}
    try:
        for extdata, st, en in cur.execute("select extdata, start, end from regions"):
            try:
                msg = json.loads(extdata or "{}").get("message")
            except ValueError:
                msg = None
            if msg:
                out[msg] = (st, en)
    except Exception:
        pass
    return out


def rocprof_summary(db_path, kernel_substr="k_cgemm_bf16x3_filter", region="timed", pmc_last=0):
    """Text summary of a rocprofv3 database: per-kernel totals from a
    --kernel-trace run, the filter kernel's launches inside the roctx range
    'timed' (the launches bench.py times with HIP events), and, for a --pmc
    run, the per-dispatch FETCH_SIZE / WRITE_SIZE of that kernel next to the
    calibration copy's (1 GiB read + 1 GiB written)."""
    import sqlite3

    con = sqlite3.connect(db_path)
    cur = con.cursor()
    lines = []
    rows = cur.execute("select name, count(*), sum(end-start), avg(end-start) from kernels "
                       "group by name order by sum(end-start) desc").fetchall()
    if rows:
        total = sum(r[2] for r in rows)
        lines += [f"kernels: {sum(r[1] for r in rows)} dispatches, {total / 1e6:.1f} ms total", "",
                  f"{'total ms':>10} {'calls':>7} {'avg ms':>9}  kernel"]
        for name, cnt, tot, avg in rows[:30]:
            lines.append(f"{tot / 1e6:10.2f} {cnt:7d} {avg / 1e6:9.4f}  {name[:110]}")
    reg = _regions(cur)
    lines.append("")
    # kernel_substr may list several kernels separated by '|' (a family whose
    # launches bench.py times together); the first ones are the launches, a
    # trailing '+name' is a helper kernel counted in the time but not the launches
    fam_total, fam_count = 0.0, 0
    for alt in kernel_substr.split("|"):
        helper = alt.startswith("+")
        name = alt.lstrip("+")
        sel = cur.execute("select start, end from kernels where name like ?",
                          ("%" + name + "%",)).fetchall()
        if not sel:
            continue
        d = [e - s for s, e in sel]
        lines.append(f"{name}: all launches {len(d)}, avg {sum(d) / len(d) / 1e6:.4f} ms")
        if region in reg:
            w0, w1 = reg[region]
            dw = [e - s for s, e in sel if s >= w0 and e <= w1]
            if dw:
                lines.append(f"{name}: launches inside roctx range '{region}' {len(dw)}, "
                             f"avg {sum(dw) / len(dw) / 1e6:.4f} ms, total {sum(dw) / 1e6:.1f} ms")
                fam_total += sum(dw)
                fam_count += 0 if helper else len(dw)
    if "|" in kernel_substr and fam_count:
        lines.append(f"family inside '{region}': {fam_count} launches, total {fam_total / 1e6:.1f} ms, "
                     f"avg per launch (helpers included) {fam_total / fam_count / 1e6:.4f} ms")
    # counters (pmc runs)
    try:
        pmc = cur.execute("select kernel_name, counter_name, avg(value), count(*) from counters_collection "
                          "group by kernel_name, counter_name").fetchall()
    except Exception:
        pmc = []
    names = [a.lstrip("+") for a in kernel_substr.split("|")]
    for kname, cname, val, cnt in pmc:
        if any(nm in kname for nm in names):
            lines.append(f"pmc {cname} avg per dispatch {val:.1f} KiB (x{cnt})  {kname[:80]}")
    if pmc and pmc_last > 0:
        # the last pmc_last dispatches of the kernel (or family; helper kernels
        # marked '+' add their bytes but are not counted as dispatches): the
        # launches of the timed steps (a --pmc run cannot carry the marker range)
        for cname in sorted({r[1] for r in pmc}):
            rows = []
            for alt in kernel_substr.split("|"):
                helper = alt.startswith("+")
                rows += [(st, v, helper) for st, v in cur.execute(
                    "select start, value from counters_collection where kernel_name like ? and "
                    "counter_name = ?", ("%" + alt.lstrip("+") + "%", cname)).fetchall()]
            rows.sort()
            main_idx = [i for i, r in enumerate(rows) if not r[2]]
            if len(main_idx) >= 1:
                first = main_idx[-pmc_last] if len(main_idx) >= pmc_last else main_idx[0]
                tail = rows[first:]
                nmain = sum(1 for r in tail if not r[2])
                lines.append(f"pmc {cname} per dispatch over the last {nmain} (timed) dispatches "
                             f"(helpers included) {sum(r[1] for r in tail) / max(nmain, 1):.1f} KiB")
    if pmc:
        # the calibration copy (1 GiB read, 1 GiB written) is the largest
        # device copy of the run
        cal = cur.execute("select counter_name, max(value), grid_size from counters_collection "
                          "where kernel_name like '%copyBuffer%' group by counter_name").fetchall()
        for cname, val, grid in cal:
            if val and val > 0:
                lines.append(f"calibration copy {cname} {val:.1f} KiB (grid {grid}); "
                             f"factor to true bytes {1048576.0 / val:.4f}")
    return "\n".join(lines)


def rocprof_breakdown(db_path, region="timed", families=("k_zgemm", "k_cgemm_bf16x3_filter")):
    """Kernel totals inside the roctx range `region` of a --kernel-trace
    database (every stream), the FP64 GEMM launches by work-groups per launch,
    and, for each kernel family, the wall time during which at least one of
    its kernels runs (the union of its launch intervals) next to its summed
    kernel time: with several streams their ratio is the family's average
    concurrency."""
    import sqlite3
    from collections import defaultdict

    cur = sqlite3.connect(db_path).cursor()
    reg = _regions(cur)
    if region not in reg:
        return f"no roctx range '{region}' in {db_path}"
    w0, w1 = reg[region]
    rows = cur.execute("select name, grid_x / workgroup_x, start, end from kernels "
                       "where start >= ? and end <= ? order by start", (w0, w1)).fetchall()

    def short(name):
        return name.split("::")[1].split("(")[0] if "::" in name else name[:40]

    def union(iv):
        tot, cs, ce = 0, None, None
        for s, e in sorted(iv):
            if ce is None or s > ce:
                if ce is not None:
                    tot += ce - cs
                cs, ce = s, e
            else:
                ce = max(ce, e)
        return tot + (ce - cs if ce is not None else 0)

    lines = [f"roctx range '{region}': {(w1 - w0) / 1e6:.1f} ms; {len(rows)} kernels inside it, "
             f"busy (any kernel running) {union([(s, e) for _, _, s, e in rows]) / 1e6:.1f} ms",
             "kernel totals inside it (all streams):"]
    agg = defaultdict(lambda: [0, 0])
    for name, _, s, e in rows:
        agg[short(name)][0] += 1
        agg[short(name)][1] += e - s
    for k, (n, t) in sorted(agg.items(), key=lambda x: -x[1][1])[:25]:
        lines.append(f"  {k:32s} n={n:6d} total={t / 1e6:9.2f} ms avg={t / n / 1e6:.4f} ms")
    lines.append("FP64 GEMM launches by work-groups per launch:")
    agg2 = defaultdict(lambda: [0, 0])
    for name, g, s, e in rows:
        if "k_zgemm" not in name:
            continue
        b = ("<64" if g < 64 else "<256" if g < 256 else "<1024" if g < 1024 else "<4096" if g < 4096
             else ">=4096")
        agg2[(short(name), b)][0] += 1
        agg2[(short(name), b)][1] += e - s
    for (k, b), (n, t) in sorted(agg2.items(), key=lambda x: -x[1][1]):
        lines.append(f"  {k:24s} grid {b:7s} n={n:6d} total={t / 1e6:8.2f} ms avg={t / n / 1e6:.4f} ms")
    # idle gaps (no kernel on any stream), the largest with the kernels around them
    gaps, last_end, last_name = [], None, None
    for name, _, st, en in rows:
        if last_end is not None and st > last_end:
            gaps.append((st - last_end, short(last_name), short(name)))
        if last_end is None or en > last_end:
            last_end, last_name = en, name
    if gaps:
        tot = sum(g[0] for g in gaps)
        lines.append(f"idle gaps: {len(gaps)}, {tot / 1e6:.1f} ms in total; the largest "
                     f"(after -> before):")
        by_pair = defaultdict(lambda: [0, 0])
        for d, a, b in gaps:
            by_pair[(a, b)][0] += 1
            by_pair[(a, b)][1] += d
        for (a, b), (k, d) in sorted(by_pair.items(), key=lambda x: -x[1][1])[:12]:
            lines.append(f"  {a:28s} -> {b:28s} n={k:5d} total={d / 1e6:7.2f} ms")
    for fam in families:
        iv = [(s, e) for name, _, s, e in rows if fam in name]
        if iv:
            u, t = union(iv), sum(e - s for s, e in iv)
            lines.append(f"family {fam}: {len(iv)} launches, summed kernel time {t / 1e6:.1f} ms, "
                         f"wall time with one or more running {u / 1e6:.1f} ms "
                         f"({u / (w1 - w0):.1%} of the range), average concurrency {t / max(u, 1):.2f}")
    return "\n".join(lines)


def run_batched(args):
    """32 independent k-point pencils of uneven size (n ~ U[1500, 3000],
    nev = round(0.1 n), per-problem spectrum shift), 8 SCF steps each; one
    gevp_solve_batched call per SCF step, seeded from the previous step.
    Timed: steps 1..7 (step 0 cold is the warm-up).  Also timed: the same
    steps solved one problem after another on one stream."""
    import torch

    from paper_1007_4400_amd import gevp, synth

    h = gevp.Handle(0)
    wls = synth.batched_workloads(count=32, seed=args.seed, steps=8)
    t0 = time.perf_counter()
    state = []
    for wl, sd in wls:
        A0, B, lam0, L, g = synth.make_pencil_torch(wl, sd)
        del L
        state.append({"wl": wl, "A": gevp.colmajor(A0), "B": gevp.colmajor(B.contiguous()), "g": g})
    torch.cuda.synchronize()
    log(f"generated 32 problems in {time.perf_counter() - t0:.1f}s")
    opts = gevp.make_opts(precision=args.precision, batch_streams=args.streams)
    X = [None] * len(wls)
    tuning = None
    per_step, single_step, worst = [], [], 0.0
    filt_ms = filt_flops = 0.0
    filt_launches = 0
    for k in range(8):
        if k > 0:
            for st in state:
                Hk = synth.unit_hermitian_torch(st["wl"].n, st["g"])
                st["A"] = gevp.colmajor((st["A"] + synth.eps(st["wl"], k) * Hk).contiguous())
                del Hk
        probs = [{"A": st["A"], "B": st["B"], "nev": st["wl"].nev, "X0": X[i],
                  "kx": h.block_size(st["wl"].n, st["wl"].nev, opts)} for i, st in enumerate(state)]
        if k == 1 and not args.no_autotune:
            # untimed: pick the launch configuration (streams, split-K mode) on
            # this step's problems; the timed steps use it
            tuning = h.autotune_batched(probs, tol=args.tol, opts=opts)
            log(f"autotuned: {tuning}")
        torch.cuda.synchronize()
        h.set_profiling(2 if k > 0 else 0)  # events around every filter launch of the timed steps
        if k == 1:
            _mark_push("timed")  # the batched solves of steps 1..7, for a profiler's trace
        ts = time.perf_counter()
        out = h.solve_batched(probs, tol=args.tol, opts=opts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - ts
        if k == 7:
            _mark_pop()
        h.set_profiling(0)
        if k > 0:
            for o in out:
                filt_ms += o[3]["filter_kernel_ms"]
                filt_flops += o[3]["filter_flops"]
                filt_launches += o[3]["filter_launches"]
        X = [o[1] for o in out]
        worst = max(worst, max(o[3]["max_resid"] for o in out))
        if k > 0:
            per_step.append(dt)
        log(f"batched step {k}: {dt * 1e3:.1f} ms, worst resid {worst:.2e}")
        if k == 7:  # the same step, one problem after another on one stream
            torch.cuda.synchronize()
            ts = time.perf_counter()
            for i, pr in enumerate(probs):
                h.solve(pr["A"], pr["B"], pr["nev"], X0=pr["X0"], tol=args.tol, kx=pr["kx"], opts=opts)
            torch.cuda.synchronize()
            single_step.append(time.perf_counter() - ts)
    value = sum(per_step) / len(per_step)
    kname = FILTER_KERNELS[args.precision]
    dtype = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16"}[args.precision]
    achieved = filt_flops / (filt_ms * 1e-3) / 1e12 if filt_ms > 0 else 0.0
    peak = PEAK_TFLOPS[dtype]
    out = {
        "metric": "batched k-point SCF step time (32 problems, n in [1500,3000], nev=0.1n)",
        "value": value, "unit": "s", "n_gpus": 1, "steps": len(per_step), "warmup": 1,
        "ms_per_step": value * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16x3": "bf16x3+f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"batched_32kpt_n1500-3000_steps8_{args.precision}",
                   "streams": tuning["streams"] if tuning else args.streams,
                   "split_mode": tuning["split_mode"] if tuning else 0,
                   "autotuned": tuning is not None, "sizes": [wl.n for wl, _ in wls]},
        "sequential_one_stream_s_per_step": single_step[0] if single_step else None,
        "max_resid_rel": worst,
        "roofline": {
            "bound": "mfma", "kernel": kname, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": None, "launches": filt_launches,
            "avg_launch_ms": filt_ms / max(filt_launches, 1),
            "algorithmic_flops_per_unit": "8 n^2 per filtered column-step (complex multiply-add = 8 flops)",
            "executed_per_algorithmic": 3.0 if dtype == "bf16" else 1.0,
            "note": "kernel time summed over the concurrent streams' launches",
        },
    }
    if not args.no_cpu_baseline:
        try:
            out["cpu_baseline"] = batched_cpu_baseline(wls)
        except Exception as e:
            out["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


def batched_cpu_baseline(wls):
    """Oracle solve of the batch's median-size problem (its step-0 pencil),
    scaled by sum_p (n_p / n_s)^3 to one SCF step of the whole batch."""
    from oracle import oracle
    from paper_1007_4400_amd import synth

    sizes = sorted(range(len(wls)), key=lambda i: wls[i][0].n)
    wl, sd = wls[sizes[len(sizes) // 2]]
    p, _ = synth.make_pencil(wl, sd)
    t0 = time.perf_counter()
    oracle.solve(p.A, p.B, wl.nev)
    t = time.perf_counter() - t0
    scale = sum((w.n / wl.n) ** 3 for w, _ in wls)
    return {"value": t * scale, "unit": "s/step",
            "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), "kind": "oracle",
            "sample": f"one oracle solve of the median problem (n={wl.n}, nev={wl.nev}, {t:.2f} s), "
                      f"scaled by sum (n_p/{wl.n})^3 = {scale:.1f} to the 32 problems"}


def _calibration_copy():
    """One 1 GiB device-to-device copy (1 GiB read, 1 GiB written): the
    reference dispatch that scales the HBM counters of a --pmc run."""
    import torch

    src = torch.empty(2 ** 27, dtype=torch.float64, device="cuda")
    src.fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    _mark_push("calibration_copy_1GiB")
    dst.copy_(src)
    torch.cuda.synchronize()
    _mark_pop()
    del src, dst


def _update_apply_bytes(mask_words, n, rechecked):
    """Bytes the apply kernel has to move for one update, from its mask: a
    tile with no update moves nothing; a tile updated everywhere reads A_new
    and writes A (32 bytes per lower entry); any other tile reads the scan's
    2-byte code per entry, A_new and A for every taken entry (16 + 16 bytes),
    and A and A_new for every entry whose code tied with the threshold's
    (`rechecked`, 32 bytes); every mask word of the n columns is written (4
    bytes)."""
    import numpy as np

    words = mask_words.shape[1]
    bits = np.unpackbits(np.ascontiguousarray(mask_words).view(np.uint8), axis=1,
                         bitorder="little")[:, :n].T  # [i, j]
    nt = (n + 63) // 64
    pad = nt * 64
    B = np.zeros((pad, pad), dtype=np.int32)
    B[:n, :n] = bits
    L = np.zeros((pad, pad), dtype=np.int32)
    L[:n, :n] = np.tril(np.ones((n, n), dtype=np.int32))
    u = B.reshape(nt, 64, nt, 64).sum(axis=(1, 3)).astype(np.int64)
    e = L.reshape(nt, 64, nt, 64).sum(axis=(1, 3)).astype(np.int64)
    low = np.tril(np.ones((nt, nt), dtype=bool))
    full = low & (u == e)
    part = low & (u > 0) & (u < e)
    return int(32 * e[full].sum() + 2 * e[part].sum() + 32 * u[part].sum() + 32 * rechecked +
               4 * n * words)


def run_update(args):
    """Thresholded partial matrix update (the paper's section 2, paragraph
    "Matrix generation"): a 12-step sequence of n = 8192 Hermitian
    Hamiltonians whose changes have the structure the paper describes (wide
    unchanged areas, a cross of frozen rows and columns, a share above
    threshold falling along the run; paper_1007_4400_amd.synth), all resident
    in HBM.  One step = one gevp_update_thresholded of the matrix in use
    towards the next generated matrix with p_t = 0.1 (delta, threshold,
    in-place update, entry mask, statistics).  Steps 1..warmup are untimed."""
    import numpy as np
    import torch

    from paper_1007_4400_amd import gevp, synth

    wl = synth.UPDATE_LARGE if args.n == 8192 else synth.update_scaled(synth.UPDATE_LARGE, args.n)
    nsteps = args.warmup + args.steps
    wl = synth.update_scaled(wl, wl.n, steps=nsteps) if nsteps != wl.steps else wl
    h = gevp.Handle(0)
    t0 = time.perf_counter()
    As = [gevp.colmajor(A) for A in synth.update_sequence_torch(wl, args.seed)]
    torch.cuda.synchronize()
    log(f"generated {len(As)} matrices n={wl.n} in {time.perf_counter() - t0:.1f}s")
    if args.calibration_copy:
        _calibration_copy()
    A_cur = As[0].clone()
    mask = gevp.empty_mask(wl.n, device="cuda")
    entries = wl.n * (wl.n + 1) // 2
    for k in range(1, args.warmup + 1):
        inf = h.update_thresholded(A_cur, As[k], wl.p_t, mask=mask)
        log(f"warmup step {k}: updated {inf['updated'] / entries:.3f}")
    h.set_profiling(2)
    infos, apply_bytes = [], []
    torch.cuda.synchronize()
    _mark_push("timed")
    t_start = time.perf_counter()
    for k in range(args.warmup + 1, nsteps + 1):
        infos.append(h.update_thresholded(A_cur, As[k], wl.p_t, mask=mask))
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    _mark_pop()
    h.set_profiling(0)
    # per-step apply traffic from the masks (recomputed untimed: replay the
    # timed steps on a copy with the same inputs; the results are identical)
    A_chk = As[0].clone()
    for k in range(1, args.warmup + 1):
        h.update_thresholded(A_chk, As[k], wl.p_t)
    for k in range(args.warmup + 1, nsteps + 1):
        inf = h.update_thresholded(A_chk, As[k], wl.p_t, mask=mask)
        assert inf["updated"] == infos[k - args.warmup - 1]["updated"]
        apply_bytes.append(_update_apply_bytes(mask.cpu().numpy(), wl.n, inf["rechecked"]))
    same = bool(torch.equal(torch.view_as_real(A_chk), torch.view_as_real(A_cur)))
    del A_chk
    for i, inf in enumerate(infos):
        log(f"step {args.warmup + 1 + i}: updated {inf['updated'] / entries:.3f} tiles "
            f"{inf['tiles_touched']}/{inf['tiles']} copied {inf['tiles_copied']} "
            f"scan {inf['scan_ms']:.3f} ms apply {inf['apply_ms']:.3f} ms")
    scan_ms = sum(i["scan_ms"] for i in infos)
    apply_ms = sum(i["apply_ms"] for i in infos)
    scan_bytes = 34.0 * entries  # both matrices' lower triangles read once, a 2-byte code written
    k_scan = {"kernel": "k_upd_scan", "avg_launch_ms": scan_ms / len(infos),
              "bytes_per_launch": scan_bytes,
              "achieved": scan_bytes * len(infos) / (scan_ms * 1e-3) / 1e9 if scan_ms > 0 else 0.0}
    k_apply = {"kernel": "k_upd_apply", "avg_launch_ms": apply_ms / len(infos),
               "bytes_per_launch": sum(apply_bytes) / len(apply_bytes),
               "achieved": sum(apply_bytes) / (apply_ms * 1e-3) / 1e9 if apply_ms > 0 else 0.0}
    dom = k_scan if scan_ms >= apply_ms else k_apply
    peak = 8000.0
    value = t_total / args.steps
    tag = f"n{wl.n}_pt{wl.p_t:g}_seq{nsteps}"
    out = {
        "metric": f"thresholded partial matrix update time per SCF step, N={wl.n}, p_t={wl.p_t:g}",
        "value": value, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": value * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"matrix_update_{tag}", "n": wl.n, "p_t": wl.p_t},
        "roofline": {
            "bound": "hbm", "kernel": dom["kernel"], "achieved": dom["achieved"], "peak": peak,
            "unit": "GB/s", "frac": dom["achieved"] / peak,
            "traffic": committed_traffic(dom["kernel"], tag),
            "traffic_unit": "bytes per launch (FETCH_SIZE x2.0 + WRITE_SIZE x1.0, calibrated)",
            "avg_launch_ms": dom["avg_launch_ms"], "bytes_per_launch": dom["bytes_per_launch"],
            "algorithmic_bytes_per_unit": ("scan: 34 per lower-triangle entry (A and A_new read, "
                                           "code written); apply: per tile, 0 / 32 per entry / 2 per "
                                           "entry + 32 per taken or re-checked entry, plus 4 per "
                                           "mask word"),
        },
        "kernels": {"scan": k_scan, "apply": k_apply},
        "updated_fraction": [i["updated"] / entries for i in infos],
        "tiles_touched": [i["tiles_touched"] for i in infos],
        "tiles_copied": [i["tiles_copied"] for i in infos],
        "rechecked": [i["rechecked"] for i in infos],
        "replay_identical": same,
    }
    if not args.no_cpu_baseline:
        try:
            from oracle import oracle

            a = As[args.warmup].cpu().numpy()
            b = As[args.warmup + 1].cpu().numpy()
            ts = time.perf_counter()
            oracle.threshold_update(a, b, wl.p_t)
            t = time.perf_counter() - ts
            out["cpu_baseline"] = {"value": t, "unit": "s/step", "cores": 1, "kind": "oracle",
                                   "sample": f"one oracle update of the sequence at n={wl.n} "
                                             "(numpy, single-threaded elementwise work)"}
        except Exception as e:
            out["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


def contour_cpu_baseline(n_sample=1024, n_target=8192):
    """Oracle's seeded contour-integral solve on step 1 of the same sequence
    at n_sample (seed: the oracle's step-0 eigenvectors), scaled by
    (n_target / n_sample)^3."""
    import numpy as np

    from oracle import oracle
    from paper_1007_4400_amd import synth

    wl = synth.scaled(synth.LARGE, n_sample, steps=2)
    (A0, B), (A1, _) = list(synth.sequence(wl, 0))
    nb = wl.nev + max(16, int(np.ceil(0.15 * wl.nev)))
    _, X0 = oracle.solve(A0, B, nb)
    t0 = time.perf_counter()
    oracle.contour_solve(A1, B, wl.nev, X0, nq=8)
    t = time.perf_counter() - t0
    scale = (n_target / n_sample) ** 3
    return {"value": t * scale, "unit": "s/step",
            "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), "kind": "oracle",
            "sample": f"oracle seeded contour solve (8 nodes, numpy/LAPACK) of step 1 at n={n_sample}, "
                      f"nev={wl.nev} ({t:.2f} s), scaled by (n/{n_sample})^3 = {scale:.0f} to n={n_target}"}


def _report_contour(args, wl, nsteps, kx, t_total, per_step, infos, cold_mean, parity):
    """JSON line of the contour-filter variant: per-step time, and the filter
    stage's FP64 matrix-core throughput (shifted factorisations and solves)
    timed with HIP events (stage timer) against the FP64 peak."""
    n = wl.n
    timed = [i for i in infos if i["ms"]["filter"] > 0]  # the solves that carried the stage timers
    stage_ms = sum(i["ms"]["filter"] for i in timed)
    flops = sum(i["contour_points"] * (8.0 / 3.0) * n ** 3 +
                8.0 * n * n * i["contour_points"] * i["contour_columns"] for i in timed)
    achieved = flops / (stage_ms * 1e-3) / 1e12 if stage_ms > 0 else 0.0
    f64 = args.precision == "fp64"
    peak = PEAK_TFLOPS["f64" if f64 else "f32"]
    value = t_total / args.steps
    out = {
        "metric": "per-SCF-step eigensolve time N=8192 nev=820, contour-integral filter, resid<=1e-10",
        "value": value, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": value * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if f64 else "f32+f64", "data": "synthetic",
        "config": {"workload": f"scf_sequence_n{wl.n}_nev{wl.nev}_steps{nsteps}_seeded_contour_"
                               f"{'fp64' if f64 else 'fp32'}",
                   "n": wl.n, "nev": wl.nev, "block": kx, "tol": args.tol, "filter": "contour",
                   "factorisation": "fp64" if f64 else "fp32 (residual correction)",
                   "nodes": infos[0]["contour_points"] if infos else None},
        "roofline": {
            "bound": "mfma",
            "kernel": ("contour filter stage (k_getrf_block<zd>, k_zgemm<0>)" if f64 else
                       "contour filter stage (k_getrf_block<zf>, k_cgemm32_filter)"),
            "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": None,
            "stage_ms_per_step": stage_ms / max(len(timed), 1),
            "algorithmic_flops_per_unit": "8 n^3 / 3 per shifted factorisation, 8 n^2 per node and filtered column",
        },
        "contour": [{"a": i["contour_a"], "b": i["contour_b"], "applications": i["contour_applications"],
                     "columns": i["contour_columns"], "outer": i["outer_iters"]} for i in infos],
        "cold_fp64_s_per_step": cold_mean,
        "speedup_vs_cold_fp64": cold_mean / value if value > 0 else None,
        "per_step_s": per_step,
        "parity": parity,
    }
    if not args.no_cpu_baseline:
        try:
            out["cpu_baseline"] = contour_cpu_baseline(1024, wl.n)
        except Exception as e:
            out["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


GEMM_FAMILY = "k_zgemm<0>, k_zgemm_nc, k_zgemm_cn, k_zgemm_cc, k_zgemm_sk (+ k_zgemm_splitk_reduce)"


def _roofline_gemm(infos):
    infos = [i for i in infos if i["gemm_launches"] > 0]  # the solves that carried the events
    ms = sum(i["gemm_kernel_ms"] for i in infos)
    fl = sum(i["gemm_flops"] for i in infos)
    la = sum(i["gemm_launches"] for i in infos)
    achieved = fl / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    peak = PEAK_TFLOPS["f64"]
    return {
        "bound": "mfma", "kernel": "FP64 complex GEMM family: " + GEMM_FAMILY,
        "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
        "traffic": committed_traffic("k_zgemm_family"),
        "traffic_unit": "bytes per launch (FETCH_SIZE x2.0 + WRITE_SIZE x1.0, calibrated; "
                        "k_zgemm_splitk_reduce dispatches included)",
        "launches": la, "avg_launch_ms": ms / max(la, 1), "flops_per_launch": fl / max(la, 1),
        "kernel_ms_per_step": ms / max(len(infos), 1),
        "algorithmic_flops_per_unit": "8 flops per complex multiply-add: 8 m n k for a dense product, "
                                      "half where only one triangle of the output or of op(A) is involved",
        # the kernels form a complex product from three real products (Gauss),
        # so they execute 6 of the 8 algorithmic flops of a complex multiply-add
        "executed_per_algorithmic": 0.75,
        "executed_frac": achieved * 0.75 / peak,
    }


def _roofline_filter(infos, precision):
    infos = [i for i in infos if i["filter_launches"] > 0]  # the solves that carried the events
    ms = sum(i["filter_kernel_ms"] for i in infos)
    fl = sum(i["filter_flops"] for i in infos)
    la = sum(i["filter_launches"] for i in infos)
    dtype = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16"}[precision]
    kname = FILTER_KERNELS[precision]
    achieved = fl / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    peak = PEAK_TFLOPS[dtype]
    ex = 3.0 if dtype == "bf16" else 1.0
    return {
        "bound": "mfma", "kernel": kname, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
        "frac": achieved / peak if peak else None,
        "traffic": committed_traffic(kname),
        "traffic_unit": "bytes per launch (FETCH_SIZE x2.0 + WRITE_SIZE x1.0, calibrated)",
        "launches": la, "avg_launch_ms": ms / max(la, 1), "flops_per_launch": fl / max(la, 1),
        "kernel_ms_per_step": ms / max(len(infos), 1),
        "algorithmic_flops_per_unit": "8 n^2 per filtered column-step (complex multiply-add = 8 flops)",
        "timed_span": "operand split + product + split-K reduction of each filter product",
        # a split-BF16 product executes 3 BF16 MFMA products per real product
        "executed_per_algorithmic": ex,
        "executed_frac": achieved * ex / peak if peak else None,
    }


def run_medium(args):
    """Plain FP64, seeded against cold: the 20-step sequence at n = 2048,
    nev = 205 (clustered lowest eigenvalues with gaps >= 1e-4, cond(B) ~ 1e2,
    eps_k = 1e-2 0.5^k).  Every step is solved cold and, from step 1 on,
    seeded with the previous seeded step's vectors; both timed between
    device synchronisations.  Per step: seeded and cold times, outer
    iterations, the largest eigenvalue difference between the two, the
    library residual; the oracle (host) checks steps 0 and 19."""
    import numpy as np
    import torch

    from paper_1007_4400_amd import gevp, synth

    wl = synth.MEDIUM
    h = gevp.Handle(0)
    A0, B, lam0, L, g = synth.make_pencil_torch(wl, args.seed)
    del L
    B = gevp.colmajor(B.contiguous())
    As = [gevp.colmajor(A0)]
    for k in range(1, wl.steps):
        Hk = synth.unit_hermitian_torch(wl.n, g)
        As.append(gevp.colmajor((As[-1] + synth.eps(wl, k) * Hk).contiguous()))
    opts = gevp.make_opts(precision="fp64")
    kx = h.block_size(wl.n, wl.nev, opts)

    def timed(A, X0, prof=0):
        h.set_profiling(prof)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        lam, X, _, info = h.solve(A, B, wl.nev, X0=X0, tol=args.tol, kx=kx, opts=opts)
        torch.cuda.synchronize()
        h.set_profiling(0)
        if info["max_resid"] > args.tol:
            raise RuntimeError(f"residual {info['max_resid']:.3e} above tol")
        return time.perf_counter() - ts, lam, X, info

    for _ in range(2):  # warm-up: code objects, workspace, graphs
        timed(As[0], None)
    steps = []
    X = None
    infos = []
    lam_seed = {}
    for k in range(wl.steps):
        tc, lam_c, Xc, ic = timed(As[k], None)
        row = {"step": k, "cold_s": tc, "cold_outer": ic["outer_iters"], "resid_cold": ic["max_resid"]}
        if k == 0:
            X = Xc
            lam_seed[k] = lam_c
        else:
            ts, lam_s, X, is_ = timed(As[k], X, prof=4)
            infos.append(is_)
            lam_seed[k] = lam_s
            d = (lam_s[: wl.nev] - lam_c[: wl.nev]).abs() / lam_c[: wl.nev].abs().clamp(min=1.0)
            row.update({"seeded_s": ts, "seeded_outer": is_["outer_iters"],
                        "col_degrees": is_["col_degrees"], "resid_seeded": is_["max_resid"],
                        "seeded_vs_cold_lambda_err_max": float(d.max())})
        steps.append(row)
        log(f"step {k}: cold {row['cold_s'] * 1e3:.1f} ms" +
            (f", seeded {row['seeded_s'] * 1e3:.1f} ms outer {row['seeded_outer']}"
             f" dlambda {row['seeded_vs_cold_lambda_err_max']:.1e}" if k else ""))
    parity = {}
    try:  # the oracle on the host at the first and the last step
        from oracle import oracle

        Bn = B.cpu().numpy()
        for k in (0, wl.steps - 1):
            An = As[k].cpu().numpy()
            lo, _ = oracle.solve(An, Bn, wl.nev)
            ls = lam_seed[k][: wl.nev].cpu().numpy()
            parity[f"step{k}_lambda_err_vs_oracle_max"] = float(
                (abs(ls - lo) / np.maximum(abs(lo), 1.0)).max())
    except Exception as e:  # reported, never silently skipped
        parity["oracle_error"] = repr(e)
    seeded = [r["seeded_s"] for r in steps[1:]]
    cold = [r["cold_s"] for r in steps[1:]]
    value = sum(seeded) / len(seeded)
    rg = _roofline_gemm(infos)
    rg["traffic"] = None
    rg.pop("traffic_unit", None)
    out = {
        "metric": "seeded plain-FP64 per-SCF-step eigensolve time N=2048 nev=205, 20 steps, resid<=1e-10",
        "value": value, "unit": "s", "n_gpus": 1, "steps": len(seeded), "warmup": 2,
        "ms_per_step": value * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "fp64_sequence_n2048_nev205_steps20_seeded_vs_cold", "n": wl.n,
                   "nev": wl.nev, "block": kx, "tol": args.tol},
        "cold_fp64_s_per_step": sum(cold) / len(cold),
        "speedup_seeded_vs_cold": sum(cold) / sum(seeded),
        "per_step": steps,
        "parity": parity,
        "roofline": rg,
    }
    print(json.dumps(out), flush=True)


def run_sequence(args):
    """The headline workload.  A 12-step SCF sequence (step 0 the constructed
    pencil, A_k = A_{k-1} + eps_k H_k).  Step 0 is solved cold once (its time
    is reported); its eigenvectors seed step 1.  The timed region is
    `--steps` seeded solves cycling through steps 1..11 of the sequence, each
    repeat starting again from step 0's vectors, bracketed by device
    synchronisations; `--warmup` untimed seeded solves along the same cycle
    come first.  Then the cold-start FP64 comparator solves every step once."""
    import torch

    from paper_1007_4400_amd import gevp, synth

    wl = synth.LARGE if (args.n, args.nev) == (8192, 820) else synth.scaled(synth.LARGE, args.n, nev=args.nev)
    K = wl.steps
    h = gevp.Handle(0)
    t0 = time.perf_counter()
    A0, B, lam0, L, g = synth.make_pencil_torch(wl, args.seed, qr_on_host=args.host_qr)
    del L
    B = gevp.colmajor(B.contiguous())
    As = [gevp.colmajor(A0)]
    for k in range(1, K):
        Hk = synth.unit_hermitian_torch(wl.n, g)
        As.append(gevp.colmajor((As[-1] + synth.eps(wl, k) * Hk).contiguous()))
        del Hk
    exact0 = torch.sort(lam0).values[: wl.nev]
    torch.cuda.synchronize()
    log(f"generated {K} steps n={wl.n} in {time.perf_counter() - t0:.1f}s")
    if args.calibration_copy:
        _calibration_copy()

    contour = args.filter == "contour"
    opts = gevp.make_opts(precision=args.precision, filter=args.filter)
    opts64 = gevp.make_opts(precision="fp64")
    kx = h.block_size(wl.n, wl.nev, opts)
    parity = {}

    def solve(A, X0, o):
        lam, Xo, res, info = h.solve(A, B, wl.nev, X0=X0, tol=args.tol, kx=kx, opts=o, want_resid=False)
        if info["max_resid"] > args.tol:
            raise RuntimeError(f"residual {info['max_resid']:.3e} above tol")
        return lam, Xo, info

    # step 0, cold, in the form under test: its vectors seed every repeat
    torch.cuda.synchronize()
    ts = time.perf_counter()
    lam, X_step0, info0 = solve(As[0], None, opts)
    t_cold0_mixed = time.perf_counter() - ts
    err0 = ((lam[: wl.nev] - exact0).abs() / exact0.abs().clamp(min=1.0))
    parity["step0_lambda_err_max"] = float(err0.max())
    parity["step0_lambda_err_mean"] = float(err0.mean())
    log(f"cold step 0 ({args.precision}): {t_cold0_mixed * 1e3:.1f} ms outer {info0['outer_iters']} "
        f"lambda err vs constructed {parity['step0_lambda_err_max']:.2e}")

    def cycle_step(j):
        return 1 + (j % (K - 1))

    X = X_step0
    for j in range(args.warmup):
        k = cycle_step(j)
        if k == 1:
            X = X_step0
        lam, X, info = solve(As[k], X, opts)
        log(f"warmup step {k}: outer {info['outer_iters']} resid {info['max_resid']:.2e}")

    # timed region: seeded solves along the cycle; gevp_solve returns after
    # its work has completed, so each step's host time is its device time.
    # The first cycle (K - 1 solves) records HIP events around every filter
    # product and FP64 GEMM launch (the rooflines); the later cycles run
    # without them, so the repeats show what the instrumentation costs.
    prof_flags = 3 if contour else 6  # events: filter products and FP64 GEMMs (contour: stages)
    h.set_profiling(prof_flags)
    per_step, infos, lam_first, seed_of = [], [], {}, {}
    torch.cuda.synchronize()
    _mark_push("timed")
    t_start = time.perf_counter()
    for j in range(args.steps):
        k = cycle_step(j)
        if k == 1:
            X = X_step0
        if k not in seed_of:
            seed_of[k] = X
        if j == K - 1:
            h.set_profiling(0)
        ts = time.perf_counter()
        lam, X, info = solve(As[k], X, opts)
        per_step.append((k, time.perf_counter() - ts))
        infos.append(info)
        if k not in lam_first:
            lam_first[k] = lam[: wl.nev].clone()
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    _mark_pop()
    h.set_profiling(0)
    for (k, t), info in zip(per_step, infos):
        log(f"step {k}: {t * 1e3:.1f} ms outer {info['outer_iters']} coldeg {info['col_degrees']} "
            f"resid {info['max_resid']:.2e}")
    parity["max_resid_rel"] = max(i["max_resid"] for i in infos)
    last_k = per_step[-1][0]

    # per-step medians over the repeats
    by_step = {}
    for k, t in per_step:
        by_step.setdefault(k, []).append(t)
    med = {k: statistics.median(v) for k, v in sorted(by_step.items())}
    repeats = [sum(t for (k, t) in per_step[r * (K - 1):(r + 1) * (K - 1)]) / (K - 1)
               for r in range(len(per_step) // (K - 1))]

    # cold-start FP64 comparator on the same steps (and step 0), each once,
    # compared eigenvalue by eigenvalue with the seeded mixed solves
    cold = {}
    dlam = {}
    steps_cold = [] if args.cold_steps == 0 else \
        [0] + sorted(med)[: args.cold_steps if args.cold_steps > 0 else None]
    for k in steps_cold:
        torch.cuda.synchronize()
        ts = time.perf_counter()
        lam_c, _, info = solve(As[k], None, opts64)
        cold[k] = time.perf_counter() - ts
        if k in lam_first:
            d = (lam_first[k] - lam_c[: wl.nev]).abs() / lam_c[: wl.nev].abs().clamp(min=1.0)
            dlam[k] = float(d.max())
        log(f"cold fp64 step {k}: {cold[k] * 1e3:.1f} ms outer {info['outer_iters']}"
            + (f" max|dlambda| vs seeded {dlam[k]:.2e}" if k in dlam else ""))
    both = [k for k in med if k in cold]
    sum_cold = sum(cold[k] for k in both)
    sum_seed = sum(med[k] for k in both)

    parity["seeded_vs_cold_fp64_lambda_err_max"] = max(dlam.values()) if dlam else None
    parity["seeded_vs_cold_fp64_lambda_err_per_step"] = {str(k): v for k, v in sorted(dlam.items())}

    # sampled independent check of returned pairs at the last timed step by the
    # oracle's O(n^2) residual on the host, scaled by a host lower bound of ||A||_2
    try:
        from oracle import oracle

        An = As[last_k].cpu().numpy()
        Bn = B.cpu().numpy()
        lam_h = lam.cpu().numpy()
        Xh = X.cpu().numpy()
        nA = oracle.norm2_lower(An, iters=20)
        parity["host_normA_lower"] = nA
        for i in (0, wl.nev - 1):
            r, q = oracle.pair_residual(An, Bn, lam_h[i], Xh[:, i])
            parity[f"oracle_pair_resid_{i}"] = r / nA
            parity[f"oracle_xBx_{i}"] = q
        del An, Bn
    except Exception as e:  # the check is reported, never silently skipped
        parity["oracle_pair_check_error"] = repr(e)

    # the forms side by side (untimed): one seeded solve of the middle step
    forms = {}
    mid = 6 if 6 in seed_of else sorted(seed_of)[len(seed_of) // 2]
    if not contour and not args.no_side_reports:
        for form in ("fp64", "fp32", "bf16x3"):
            o = gevp.make_opts(precision=form)
            kxf = h.block_size(wl.n, wl.nev, o)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            lf, _, _, inf_f = h.solve(As[mid], B, wl.nev, X0=seed_of[mid][:, :kxf], tol=args.tol, kx=kxf, opts=o)
            forms[form] = {"s": time.perf_counter() - ts, "outer": inf_f["outer_iters"],
                           "col_degrees": inf_f["col_degrees"], "max_resid": inf_f["max_resid"]}
        forms["step"] = mid

    # seed monitor (untimed): principal-angle RMS sine and deviation angles of
    # the last step's result against its seed, and what the monitor adds
    monitor = {}
    try:
        if contour or args.no_side_reports:
            raise StopIteration  # the seed monitor side report belongs to the Chebyshev run
        X0m = seed_of[last_k]
        om = gevp.make_opts(precision=args.precision, seed_monitor=True)
        t_on, t_off = [], []
        for _ in range(2):
            for o_, acc in ((om, t_on), (opts, t_off)):
                torch.cuda.synchronize()
                ts = time.perf_counter()
                _, _, _, inf_m = h.solve(As[last_k], B, wl.nev, X0=X0m, tol=args.tol, kx=kx, opts=o_)
                torch.cuda.synchronize()
                acc.append(time.perf_counter() - ts)
                if o_ is om:
                    monitor = {k_: inf_m[k_] for k_ in ("seed_sin_rms", "seed_dev_mean", "seed_dev_max",
                                                         "seed_reindexed")}
        monitor["added_ms"] = (min(t_on) - min(t_off)) * 1e3
        monitor["step"] = last_k
    except StopIteration:
        monitor = {}
    except Exception as e:  # reported, never silently skipped
        monitor = {"error": repr(e)}

    value = t_total / args.steps
    cold_mean = sum(cold[k] for k in both) / len(both) if both else None
    if contour:
        return _report_contour(args, wl, K, kx, t_total, [t for _, t in per_step], infos, cold_mean,
                               parity)
    rf = _roofline_filter(infos, args.precision)
    rg = _roofline_gemm(infos)
    # the dominant kernel of the timed step by summed event time
    primary, secondary = (rg, rf) if rg["kernel_ms_per_step"] >= rf["kernel_ms_per_step"] else (rf, rg)
    out = {
        "metric": "per-SCF-step eigensolve time N=8192 nev=820, mixed vs FP64, resid<=1e-10",
        "value": value,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": value * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16x3": "bf16x3+f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"scf_sequence_n{wl.n}_nev{wl.nev}_steps{K}_seeded_{args.precision}",
                   "timed_steps": f"seeded steps 1..{K - 1} of the {K}-step sequence, cycled "
                                  f"({args.steps} solves; every repeat restarts from step 0's vectors)",
                   "n": wl.n, "nev": wl.nev, "block": kx, "tol": args.tol,
                   "precision": args.precision},
        "roofline": primary,
        "roofline_secondary": secondary,
        "median_s_per_step": sum(med.values()) / len(med),
        "per_step_median_s": {str(k): v for k, v in med.items()},
        "repeat_mean_s_per_step": repeats,
        "instrumented_solves": f"the first {min(K - 1, args.steps)} of {args.steps} timed solves carry HIP "
                               f"events around every filter product and FP64 GEMM launch (the rooflines); "
                               f"repeat_mean_s_per_step[0] is that cycle",
        "cold_step0_s": {"fp64": cold.get(0), args.precision: t_cold0_mixed},
        "cold_fp64_s_per_step": cold_mean,
        "cold_fp64_per_step_s": {str(k): v for k, v in sorted(cold.items())},
        "speedup_vs_cold_fp64": sum_cold / sum_seed if sum_seed > 0 else None,
        "speedup_vs_cold_fp64_steps": (f"sum over steps {both[0]}..{both[-1]} of cold FP64 / median seeded"
                                       if both else None),
        "speedup_incl_step0": ((sum_cold + cold[0]) / (sum_seed + t_cold0_mixed)
                               if sum_seed > 0 and 0 in cold else None),
        "forms_seeded_one_step": forms,
        "parity": parity,
        "seed_monitor": monitor,
    }
    if not args.no_cpu_baseline:
        try:
            out["cpu_baseline"] = cpu_baseline(wl.n)
        except Exception as e:
            out["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 33 = three repeats of seeded steps 1..11 for the "
                         "sequence, 11 for the update workload)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default 2; update: 1)")
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--nev", type=int, default=820)
    ap.add_argument("--precision", default="bf16x3", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--filter", default="chebyshev", choices=["chebyshev", "contour"],
                    help="contour: seeded steps use the contour-integral (Sakurai-Sugiura) filter; "
                         "FP64 factorisations with --precision fp64, else FP32 ones in the "
                         "residual-correction form (cold steps keep the Chebyshev filter)")
    ap.add_argument("--cold-steps", type=int, default=-1,
                    help="cold FP64 comparator on the first N timed steps (-1: all of them)")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-side-reports", action="store_true",
                    help="skip the untimed forms and seed-monitor solves (counter runs: the "
                         "timed launches are then the last ones of the run)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workload", default="sequence", choices=["sequence", "batched", "update", "medium"],
                    help="sequence: the n=8192 SCF sequence (headline); batched: 32 uneven "
                         "k-point problems, n in [1500, 3000], 8 SCF steps; update: thresholded "
                         "partial matrix update, n=8192, p_t=0.1, 12 steps; medium: plain FP64 "
                         "seeded vs cold over the 20-step sequence at n=2048, nev=205")
    ap.add_argument("--streams", type=int, default=8, help="concurrent streams (batched)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched: keep --streams and split-K by the cost model instead of autotuning")
    ap.add_argument("--rocprof-summary", metavar="DB", help="summarise a rocprofv3 database and exit")
    ap.add_argument("--summary-kernel", default=None, help="kernel name for --rocprof-summary")
    ap.add_argument("--rocprof-breakdown", metavar="DB",
                    help="kernel totals and family concurrency inside the 'timed' range of a "
                         "rocprofv3 kernel-trace database, and exit")
    ap.add_argument("--host-qr", action="store_true",
                    help="factor the generator's Gaussian matrix on the host (for counter runs)")
    ap.add_argument("--pmc-last", type=int, default=0,
                    help="with --rocprof-summary: average counters over the kernel's last N dispatches")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="run one 1 GiB device-to-device copy first (HBM counter calibration)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 11 if args.workload == "update" else 33
    if args.warmup is None:
        args.warmup = 1 if args.workload == "update" else 2
    if args.rocprof_summary:
        print(rocprof_summary(args.rocprof_summary, args.summary_kernel or FILTER_KERNELS[args.precision],
                              pmc_last=args.pmc_last))
        return
    if args.rocprof_breakdown:
        print(rocprof_breakdown(args.rocprof_breakdown))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; --gpus above 1 is not supported "
                          "(k-point sharding across GPUs is a design note only)"}))
        sys.exit(2)
    if args.workload == "batched":
        return run_batched(args)
    if args.workload == "update":
        return run_update(args)
    if args.workload == "medium":
        return run_medium(args)

    return run_sequence(args)


if __name__ == "__main__":
    main()
