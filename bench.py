#!/usr/bin/env python3
"""Benchmark: VGC BFS + reachability on one MI355X.

Workload (the headline configuration): a directed 5-NN graph of 10^7 seeded
uniform points in [0,1)^2 (50,000,000 arcs, int32 CSR, Z-order vertex
layout) and 16 seeded random sources. One step is the whole job for that
batch of sources, inputs resident in HBM:
  * 16 BFS queries (one per source) in one batched persistent VGC launch
    (pasgal_batch_run, hipGraph-captured), and
  * reachability from the 16 sources in one VGC launch with 16-bit masks
    (pasgal_reach_ex, k = 16).
By default (--schedule concurrent) the two launches run at the same time on
two streams, each sized to a share of every compute unit (pasgal_opts
device_share: 75% and 768-thread workgroups for the BFS batch, 25% and
256-thread workgroups for reach): both are latency-bound, and each loses
little when given part of the wavefronts. --schedule sequential runs them
one after the other on the whole device (1024-thread workgroups).
value = traversed edges per second (GTEPS): per query, the arcs whose tail the
source reaches (BFS and reach alike), summed over the 32 queries, over the
wall time of the timed steps.

The JSON line also carries
  roofline      dominant kernel: the multi-query persistent VGC BFS kernel.
                achieved = algorithmic bytes of one launch (16 B per reached
                vertex + 8 B per arc of a reached vertex, per query) / the
                launch's duration (HIP events recorded around the kernel on
                its own stream, averaged over the timed steps; under the
                concurrent schedule the reach launch runs beside it); peak
                8 TB/s; traffic from committed rocprofv3 counter runs when
                they were taken on the same kernel source and setting, else
                null. detail.job_* gives both launches' algorithmic bytes over
                the step time.
  cpu_baseline  the CPU oracle (sequential queue BFS / DFS reach, one host
                thread) on a bounded sample of the same queries.
  extras        single-source calls: plain (one launch per BFS level) vs VGC
                per tau, the same job run sequentially on the whole device,
                and the latency floor: eccentricity x the time of one
                dependent access (pasgal_probe_latency) beside the measured
                single-source time.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--tau T] [--window W]
                [--schedule concurrent|sequential] [--layout morton|draw]
                [--no-extras] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_COUNTERS = os.path.join(ROOT, "profiles", "vgc_bfs_batched16_knn10m_counters.txt")


def log(msg):
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "kern.h", "devutil.h"):
        with open(os.path.join(ROOT, "paper_2404_17101_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _counter_means(path):
    import collections
    import csv

    agg = collections.defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in agg.items()}


SUITE_TRACES = {
    "grid": ("Kernel trace: grid suite, first setting only (16 BFS queries in one batched launch on the 8192x8192 "
             "grid, tau 1024, window 32; one warm-up and three timed launches)",
             "vgc_kernel<0, true, false, false> is the multi-query BFS kernel (kind 0 = BFS, multi-query, no "
             "arc-range prefetch, no test-first read); each launch covers all 16 queries. The suite's roofline "
             "fraction is 16 x (16 n + 8 m) bytes over that kernel's average time."),
    "scc": ("Kernel trace: SCC suite (road4096, knn 10M/5, RMAT-20; VGC, tau 1, no trim, no split; 3 runs each)",
            "vgc_kernel<1, false, true, false> is the reach kernel (arc-range prefetch on, the SCC default) running "
            "the forward and backward searches of a "
            "batch together on the packed 2n-vertex graph; pack_kernel<false/true> count and scatter the arcs that "
            "stay inside one subproblem; union_kernel / piece_label_kernel are the weak-connectivity split; "
            "trim_kernel, select_kernel, refine_kernel and min_member_kernel are the per-batch steps."),
    "sssp": ("Kernel trace: SSSP suite (knn 10M/5, road4096, RMAT-22; weights uniform in [1, 1000]; VGC and tau 1)",
             "vgc_kernel<2, false, true, false> is the SSSP kernel (kind 2 = weighted distances) with arc-range "
             "prefetch, the default at tau above 1, and vgc_kernel<2, false, false, false> the same without it "
             "(tau 1: RMAT-22 and the tau1 rows); sum_u32_kernel is the "
             "mean-weight reduction behind the default bucket width."),
    "bfs_do": ("Kernel trace: direction-optimizing BFS suite (RMAT-24 and knn 10M/5, 4 sources each, and one "
               "16-source run per graph)",
               "bottom_up_kernel, collect_kernel and degsum_kernel belong to the direction-optimizing BFS; "
               "plain_level_kernel<0> runs its top-down levels and the plain BFS; ms_* kernels are the multi-source "
               "run (one bit per source; on the k-NN graph its many bottom-up levels dominate the suite's time); "
               "vgc_kernel<0, false, true, false> is the VGC BFS (arc-range prefetch on, the single-source default)."),
}


def summarize_suite_trace(suite, d):
    """profiles/<suite>_trace.md from the kernel-stats CSV of a traced suite run."""
    import csv

    title, note = SUITE_TRACES[suite]
    rows = list(csv.DictReader(open(os.path.join(d, f"prof_{suite}", "run_kernel_stats.csv"))))
    lines = [f"# {title}", "", "Command (GPU host, `TMPDIR=/tmp`, run from `/tmp`):", "", "```",
             f"rocprofv3 --kernel-trace --stats --output-format csv -d <out>/prof_{suite} -o run -- \\",
             f"    python3 <repo>/bench.py --suite {suite}" + (" --grid-default-only" if suite == "grid" else ""),
             "```", "",
             f"Summarised by `python bench.py --summarize-suite-trace {suite} <out>`. Times include every "
             f"configuration the suite runs; rocprofv3 may end with a segmentation fault in its own exit handler "
             f"after the program's last line, the CSV files were complete.", "",
             "| kernel | calls | avg (ms) | min (ms) | max (ms) | total (ms) | share |", "|---|---|---|---|---|---|---|"]
    for r in rows[:14]:
        name = r["Name"].replace("|", "/")
        if len(name) > 80:
            name = name[:77] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | "
                     f"{float(r['MinNs']) / 1e6:.3f} | {float(r['MaxNs']) / 1e6:.3f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.1f} | {float(r['Percentage']):.1f}% |")
    lines += ["", note]
    with open(os.path.join(ROOT, "profiles", f"{suite}_trace.md"), "w") as f:
        f.write("\n".join(lines) + "\n")


def summarize_scc_traces(d):
    """profiles/scc_trace.md from one traced run of the default pasgal_scc call
    per graph (DIR/prof_scc_<graph>/run_kernel_stats.csv)."""
    import csv

    lines = ["# Kernel traces: the default `pasgal_scc` call, one graph per run", "",
             "Command per graph (GPU host, `TMPDIR=/tmp`, run from `/tmp`):", "", "```",
             "rocprofv3 --kernel-trace --stats --output-format csv -d <out>/prof_scc_<graph> -o run -- \\",
             "    python3 <repo>/bench.py --suite scc --scc-graphs <graph> --scc-default-only", "```", "",
             "Summarised by `python bench.py --summarize-scc-traces <out>`. Each run makes three default calls "
             "(tau by mean degree, one trimming pass, weak-connectivity split) after one transpose; the shares "
             "below are of the GPU time of that run.", ""]
    for graph in ("road4096", "knn10m", "rmat20"):
        path = os.path.join(d, f"prof_scc_{graph}", "run_kernel_stats.csv")
        if not os.path.exists(path):
            continue
        rows = list(csv.DictReader(open(path)))
        lines += [f"## {graph}", "", "| kernel | calls | avg (ms) | total (ms) | share |", "|---|---|---|---|---|"]
        for r in rows[:12]:
            name = r["Name"].replace("|", "/")
            if len(name) > 80:
                name = name[:77] + "..."
            lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | "
                         f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.1f}% |")
        lines.append("")
    lines.append("`vgc_kernel<1, false, ...>` is the reach kernel running the forward and backward searches of a "
                 "batch on the packed 2n-vertex graph; `pack_kernel` builds that graph; `select_kernel` draws the "
                 "pivots; `union_kernel`/`piece_label_kernel` are the weak-connectivity split; `transpose` kernels "
                 "(`hist_kernel`, `scatter_kernel`, scans) run once per run.")
    with open(os.path.join(ROOT, "profiles", "scc_trace.md"), "w") as f:
        f.write("\n".join(lines) + "\n")


TRACE_STEPS, TRACE_WARMUP = 5, 1  # the kernel-trace run of the headline job


def summarize_profiles(d, args, out_dir=None):
    """Turn the rocprofv3 CSVs of the trace, counter and copy-calibration runs
    into the committed summaries under profiles/ (or out_dir)."""
    import csv

    kb = "void pg::vgc_kernel<0, true, false, false>(pg::VgcArgs)"
    kr = "void pg::vgc_kernel<1, false, true, true>(pg::VgcArgs)"
    cp = "__amd_rocclr_copyBuffer"
    rows = list(csv.DictReader(open(os.path.join(d, "prof_trace", "run_kernel_stats.csv"))))
    # the timed steps' dispatches of the two traversal kernels (the trace run
    # makes TRACE_WARMUP warm-up steps, then TRACE_STEPS timed ones; the
    # first launch of a kernel also pays its first touch of the buffers)
    disp = {}
    for r in csv.DictReader(open(os.path.join(d, "prof_trace", "run_kernel_trace.csv"))):
        disp.setdefault(r["Kernel_Name"], []).append((int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    timed = {k: [(e - b) / 1e6 for b, e in sorted(v)[TRACE_WARMUP:TRACE_WARMUP + TRACE_STEPS]]
             for k, v in disp.items()}
    F = _counter_means(os.path.join(d, "prof_fetch", "run_counter_collection.csv"))
    W = _counter_means(os.path.join(d, "prof_write", "run_counter_collection.csv"))
    CF = _counter_means(os.path.join(d, "prof_cfetch", "run_counter_collection.csv"))
    CW = _counter_means(os.path.join(d, "prof_cwrite", "run_counter_collection.csv"))
    f_scale = (1 << 30) / (CF[cp] * 1024)
    w_scale = (1 << 30) / (CW[cp] * 1024)
    traffic_b = F[kb] * 1024 * f_scale + W[kb] * 1024 * w_scale
    traffic_r = F[kr] * 1024 * f_scale + W[kr] * 1024 * w_scale
    avg = {k: sum(v) / len(v) for k, v in timed.items() if v}
    conc = args.schedule == "concurrent"
    wg = args.wg if args.wg > 0 else (max(64, (1024 * args.bfs_share + 3200) // 6400 * 64) if conc else 1024)
    sched = (f"the two launches run concurrently on two streams, the batch on {args.bfs_share}% of every CU "
             f"({wg}-thread workgroups) and reach on the rest ({1024 - wg}-thread workgroups, tau "
             f"{args.reach_tau if args.reach_tau > 0 else 256})" if conc else
             f"the two launches run one after the other ({wg}-thread workgroups)")
    out = {"kernel": kb, "kernel_hash": kernel_source_hash(), "layout": args.layout, "tau": args.tau,
           "window": args.window, "wg_size": wg, "schedule": args.schedule, "bfs_share": args.bfs_share if conc else 100, "fetch_kib_per_dispatch": round(F[kb], 1), "write_kib_per_dispatch": round(W[kb], 1),
           "copy_calibration": {"fetch_kib_per_1GiB_copy": round(CF[cp], 1), "write_kib_per_1GiB_copy": round(CW[cp], 1),
                                "fetch_scale": round(f_scale, 5), "write_scale": round(w_scale, 5)},
           "hbm_bytes_per_launch": int(traffic_b), "kernel_avg_ms": round(avg.get(kb, 0.0), 4),
           "reach16_kernel": kr, "reach16_fetch_kib": round(F[kr], 1), "reach16_write_kib": round(W[kr], 1),
           "reach16_hbm_bytes_per_launch": int(traffic_r), "reach16_avg_ms": round(avg.get(kr, 0.0), 4)}
    prof = out_dir or os.path.join(ROOT, "profiles")
    with open(os.path.join(prof, "vgc_bfs_batched16_knn10m_counters.txt"), "w") as f:
        f.write(json.dumps(out, indent=1) + "\n")
    lines = ["# Kernel trace: batched 16-source BFS + 16-source reach on the 10M-point 5-NN graph", "",
             "Command (GPU host, `TMPDIR=/tmp`, run from `/tmp`):", "", "```",
             "rocprofv3 --kernel-trace --stats --output-format csv -d <out>/prof_trace -o run -- \\",
             f"    python3 <repo>/bench.py --steps {TRACE_STEPS} --warmup {TRACE_WARMUP} --no-extras --no-cpu", "```", "",
             f"Summarised by `python bench.py --summarize-profiles <out>`. Workload: directed 5-NN graph of 10^7 "
             f"uniform points ({args.layout} layout), 16 sources; each step is one batched VGC BFS launch (16 "
             f"queries, tau {args.tau}, window {args.window}) and one 16-source VGC reach launch; {sched}; "
             f"{TRACE_WARMUP} warm-up + {TRACE_STEPS} timed steps. rocprofv3 may end with a segmentation fault in its own exit "
             f"handler after the program's last line; the CSV files were complete.", "",
             "Timed steps only (from `run_kernel_trace.csv`; the warm-up launch also pays the first touch of the "
             "buffers):", "", "| kernel | timed dispatches | avg (ms) | min (ms) | max (ms) |", "|---|---|---|---|---|"]
    for k in (kb, kr):
        v = timed.get(k, [])
        if v:
            lines.append(f"| `{k}` | {len(v)} | {sum(v) / len(v):.3f} | {min(v):.3f} | {max(v):.3f} |")
    lines += ["", "Every dispatch of the run (`run_kernel_stats.csv`, warm-up included):", "",
              "| kernel | calls | avg (ms) | min (ms) | max (ms) | share |", "|---|---|---|---|---|---|"]
    for r in rows[:8]:
        name = r["Name"].replace("|", "/")
        if len(name) > 70:
            name = name[:67] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | "
                     f"{float(r['MinNs']) / 1e6:.3f} | {float(r['MaxNs']) / 1e6:.3f} | {float(r['Percentage']):.1f}% |")
    lines += ["", "`vgc_kernel<0, true, false, false>` is the multi-query BFS kernel (kind 0 = BFS, multi-query, no "
                  "arc-range prefetch, no test-first read); `vgc_kernel<1, false, true, true>` is the single-query "
                  "reach kernel with arc-range prefetch and test-first reads (the defaults for 16 sources on this "
                  "graph) and source implications, run with a 16-bit mask. "
                  "`__amd_rocclr_copyBuffer` dispatches are the graph upload before the timed steps."]
    with open(os.path.join(prof, "vgc_bfs_batched16_knn10m_trace.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    lines = ["# HBM traffic counters: batched 16-source BFS kernel and 16-source reach kernel", "",
             "Commands (GPU host, `TMPDIR=/tmp`, run from `/tmp`; one counter per pass):", "", "```",
             "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out>/prof_fetch -o run -- \\",
             "    python3 <repo>/bench.py --steps 1 --warmup 1 --no-extras --no-cpu",
             "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <out>/prof_write -o run -- \\",
             "    python3 <repo>/bench.py --steps 1 --warmup 1 --no-extras --no-cpu",
             "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out>/prof_cfetch -o run -- python3 <repo>/bench.py --calibrate-copy",
             "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <out>/prof_cwrite -o run -- python3 <repo>/bench.py --calibrate-copy",
             "```", "", "Per dispatch (KiB as reported), averaged over the dispatches of each kernel:", "",
             "| kernel | FETCH_SIZE | WRITE_SIZE | HBM bytes (calibrated) |", "|---|---|---|---|",
             f"| `vgc_kernel<0, true, false, false>` (BFS, 16 queries) | {F[kb]:,.1f} | {W[kb]:,.1f} | {traffic_b / 1e9:.2f} GB |",
             f"| `vgc_kernel<1, false, true, true>` (reach, k = 16) | {F[kr]:,.1f} | {W[kr]:,.1f} | {traffic_r / 1e9:.2f} GB |",
             f"| `{cp}`, 1 GiB copy (calibration) | {CF[cp]:,.1f} | {CW[cp]:,.1f} | 2.15 GB |", "",
             f"Calibration: a plain 1 GiB copy reads and writes 1 GiB; the counters report {CF[cp] / 1048576:.3f} GiB and "
             f"{CW[cp] / 1048576:.3f} GiB, so FETCH_SIZE is scaled by {f_scale:.3f} and WRITE_SIZE by {w_scale:.3f}.",
             "", "Under counter collection the profiler runs dispatches one at a time, so these bytes are each "
                 "kernel's own even where the bench overlaps the two launches.",
             "", "`vgc_bfs_batched16_knn10m_counters.txt` holds these figures with the hash of the kernel source they "
                 "were taken on; bench.py reports `traffic` only while that hash matches the current source."]
    with open(os.path.join(prof, "vgc_bfs_batched16_knn10m_counters.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print(json.dumps(out, indent=1))


SQ_COUNTERS = ("SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR "
               "SQ_ACTIVE_INST_ANY SQ_WAIT_INST_ANY")
TCC_COUNTERS = "TCC_HIT_sum TCC_MISS_sum TCC_EA0_RDREQ_sum TCC_EA0_ATOMIC_sum"


def summarize_pmc(d, out_dir=None):
    """profiles/vgc_bfs_batched16_knn10m_sq.md from the two instruction and L2
    counter passes (DIR/pmc_sq, DIR/pmc_tcc), per dispatch of each of the two
    headline kernels."""
    import collections
    import csv

    kb = "void pg::vgc_kernel<0, true, false, false>(pg::VgcArgs)"
    kr = "void pg::vgc_kernel<1, false, true, true>(pg::VgcArgs)"
    agg = collections.defaultdict(list)
    for sub in ("pmc_sq", "pmc_tcc"):
        with open(os.path.join(d, sub, "run_counter_collection.csv")) as f:
            for r in csv.DictReader(f):
                agg[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
    mean = {k: sum(v) / len(v) for k, v in agg.items()}
    names = SQ_COUNTERS.split() + TCC_COUNTERS.split()
    lines = ["# Instruction and L2 counters: batched 16-source BFS kernel and 16-source reach kernel "
             "(10M-point 5-NN graph)", "",
             "Commands (GPU host, `TMPDIR=/tmp`, run from `/tmp`; one pass per counter block):", "", "```",
             f"rocprofv3 --pmc {SQ_COUNTERS} \\",
             "    --output-format csv -d <out>/pmc_sq -o run -- python3 <repo>/bench.py --steps 1 --warmup 1 --no-extras --no-cpu",
             f"rocprofv3 --pmc {TCC_COUNTERS} \\",
             "    --output-format csv -d <out>/pmc_tcc -o run -- python3 <repo>/bench.py --steps 1 --warmup 1 --no-extras --no-cpu",
             "```", "",
             "Summarised by `python bench.py --summarize-pmc <out>`. Per dispatch, averaged over the dispatches of "
             "each kernel (the profiler serialises dispatches under counter collection).", "",
             "| counter | `vgc_kernel<0, true, false, false>` (BFS, 16 queries) | "
             "`vgc_kernel<1, false, true, true>` (reach, k = 16) |", "|---|---|---|"]
    for c in names:
        b, r = mean.get((kb, c)), mean.get((kr, c))
        fmt = lambda x: "n/a" if x is None else f"{x:,.0f}"
        lines.append(f"| {c} | {fmt(b)} | {fmt(r)} |")
    with open(os.path.join(out_dir or os.path.join(ROOT, "profiles"), "vgc_bfs_batched16_knn10m_sq.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tau", type=int, default=1024)
    ap.add_argument("--reach-tau", type=int, default=0,
                    help="tau of the reach launch (default 256 under the concurrent schedule, where it measured "
                         "best on half the device, else --tau)")
    ap.add_argument("--window", type=int, default=0,
                    help="BFS distance window (default 32, measured best under both schedules)")
    ap.add_argument("--wg", type=int, default=0,
                    help="BFS workgroup size (default: the BFS share of 1024 threads in whole wavefronts when "
                         "concurrent, 1024 sequential)")
    ap.add_argument("--bfs-share", type=int, default=75,
                    help="concurrent schedule: percent of every compute unit the batched BFS launch takes (the "
                         "reach launch takes the rest; workgroup sizes follow the shares). 75/25 measured best: "
                         "79.1 GTEPS against 74.4 at 50/50; the shares between (odd wavefront counts) measured worse")
    ap.add_argument("--schedule", choices=["concurrent", "sequential"], default="concurrent")
    ap.add_argument("--bpc", type=int, default=1)
    ap.add_argument("--filter-slots", type=int, default=0,
                    help="LDS filter entries per wavefront of the BFS launch (0: the library default)")
    ap.add_argument("--prefetch", choices=["auto", "on", "off"], default="auto",
                    help="arc ranges carried in the local queue (auto: each entry point's default)")
    ap.add_argument("--points", type=int, default=10_000_000)
    ap.add_argument("--sources", type=int, default=16)
    ap.add_argument("--layout", default="morton", choices=["morton", "draw"])
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy 3 times (counter calibration for rocprofv3 runs)")
    ap.add_argument("--suite", choices=["c1", "c3", "c4", "c5", "scc", "sssp", "bfs_do", "grid"], default=None,
                    help="run one of the other configurations instead of the headline job (one JSON line)")
    ap.add_argument("--rates", default="5,10,20,40,100,300,1000,3000,10000", help="c5: Poisson arrival rates (q/s)")
    ap.add_argument("--server-tau", type=int, default=0, help="c5: the server's local-search budget (0: its default)")
    ap.add_argument("--slice-rounds", type=int, default=0, help="c5: rounds per server launch (0: the server default)")
    ap.add_argument("--server-fixed-slices", action="store_true",
                    help="c5: every server launch runs at most --slice-rounds rounds (no long launch for a lone request)")
    ap.add_argument("--server-no-do", action="store_true",
                    help="c5: RMAT BFS requests in the batched launches instead of the direction-optimizing BFS")
    ap.add_argument("--scc-graphs", default="", help="scc: comma list of graphs to run (road4096, knn10m, rmat20)")
    ap.add_argument("--scc-default-only", action="store_true", help="scc: only the library's default call")
    ap.add_argument("--grid-default-only", action="store_true",
                    help="grid: only the first setting (tau 1024, window 32), e.g. for a kernel trace")
    ap.add_argument("--summarize-suite-trace", nargs=2, metavar=("SUITE", "DIR"), default=None,
                    help="write profiles/SUITE_trace.md from DIR/prof_SUITE/run_kernel_stats.csv")
    ap.add_argument("--summarize-pmc", metavar="DIR", default=None,
                    help="write profiles/vgc_bfs_batched16_knn10m_sq.md from DIR/pmc_sq and DIR/pmc_tcc")
    ap.add_argument("--summarize-scc-traces", metavar="DIR", default=None,
                    help="write profiles/scc_trace.md from DIR/prof_scc_<graph>/run_kernel_stats.csv")
    ap.add_argument("--summarize-profiles", metavar="DIR", default=None,
                    help="write profiles/ summaries from rocprofv3 CSV output under DIR (prof_trace, prof_fetch, "
                         "prof_write, prof_cfetch, prof_cwrite)")
    args = ap.parse_args()
    if args.window <= 0:
        args.window = 32

    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles, args)
        return
    if args.summarize_suite_trace:
        summarize_suite_trace(*args.summarize_suite_trace)
        return
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc)
        return
    if args.summarize_scc_traces:
        summarize_scc_traces(args.summarize_scc_traces)
        return

    if args.suite:
        import bench_suites

        bench_suites.run(args.suite, args)
        return

    if args.calibrate_copy:
        import torch

        nbytes = 1 << 30
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read_per_dispatch": nbytes,
                          "bytes_written_per_dispatch": nbytes, "dispatches": 3}), flush=True)
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): every configuration fits one "
              f"MI355X, and the multi-GPU partitioning exists as design only.", file=sys.stderr)
        sys.exit(2)

    import torch

    import graphgen as gg
    import paper_2404_17101_amd as pg

    pg.load()  # raises if the HIP library is missing: there is no fallback path
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    t0 = time.time()
    g = gg.knn(args.points, 5, 2, layout=args.layout)
    srcs = [int(s) for s in gg.sources(g, args.sources, 1002)]
    log(f"generated knn n={g.n} m={g.m} in {time.time() - t0:.1f}s ({gg.threads()} threads)")
    d = pg.DeviceGraph.from_graph(g)
    n, nq = g.n, len(srcs)
    stream = torch.cuda.current_stream()
    conc = args.schedule == "concurrent"
    if args.wg <= 0:
        args.wg = max(64, (1024 * args.bfs_share + 3200) // 6400 * 64) if conc else 1024
    # the reach launch takes the rest of every CU, in as many workgroups per CU
    rwg = max(64, (1024 - args.wg * args.bpc) // args.bpc // 64 * 64) if conc else args.wg
    vgc = dict(tau=args.tau, window=args.window, wg_size=args.wg, blocks_per_cu=args.bpc, stream=stream,
               filter_slots=args.filter_slots,
               device_share=args.bfs_share if conc else 0,
               prefetch={"auto": None, "on": True, "off": False}[args.prefetch])
    rstream = torch.cuda.Stream() if conc else stream  # the reach launch's stream
    if args.reach_tau <= 0:
        args.reach_tau = 256 if conc else args.tau
    rvgc = dict(vgc, stream=rstream, asynchronous=conc, tau=args.reach_tau, wg_size=rwg,
                device_share=100 - args.bfs_share if conc else 0)
    srcs_dev = pg.device_sources(srcs, "cuda", rstream)  # pasgal_reach takes a device array

    # outputs: 16 distance arrays (one batched launch) and one 16-bit mask word per vertex
    dist16 = torch.empty(n * nq, dtype=torch.int32, device="cuda")
    mask = torch.empty((n, 1), dtype=torch.int64, device="cuda")
    vb = np.array([0, n], dtype=np.int32)
    batch = pg.Batch(d, vb, np.zeros(nq, np.int32), np.array(srcs, np.int32), np.arange(nq, dtype=np.int64) * n,
                     dist16, **vgc)
    torch.cuda.synchronize()

    def step(rec=None):
        if conc:
            # reach enqueued on its own stream first, then the batch on the
            # caller's stream; pasgal_batch_run returns when the batch is done,
            # pasgal_wait when the reach launch is (and reports its status)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(rstream)
            pg.reach(d, srcs_dev, label_out=mask, **rvgc)
            e1.record(rstream)
            bst = batch.run()
            pg.wait(rstream)
            rst = {"events": (e0, e1)}
        else:
            bst = batch.run()
            _, rst = pg.reach(d, srcs_dev, label_out=mask, stats=True, **rvgc)
        if rec is not None:
            rec.append((bst, rst))

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()

    # work per query from the results (reached vertices, arcs out of them)
    deg = np.diff(g.offsets).astype(np.int64)
    dd = dist16.view(nq, n).cpu().numpy()
    mk = mask.cpu().numpy().view(np.uint64)[:, 0]
    bfs_nr, bfs_mr, rch_mr = [], [], []
    for i in range(nq):
        r = dd[i] >= 0
        bfs_nr.append(int(r.sum()))
        bfs_mr.append(int(deg[r].sum()))
        rr = ((mk >> np.uint64(i)) & np.uint64(1)).astype(bool)
        rch_mr.append(int(deg[rr].sum()))
    edges_per_step = sum(bfs_mr) + sum(rch_mr)

    rec = []
    torch.cuda.synchronize()
    ta = time.perf_counter()
    for _ in range(args.steps):
        step(rec)
    torch.cuda.synchronize()
    wall = time.perf_counter() - ta
    gteps = edges_per_step * args.steps / wall / 1e9
    # the timed steps must reproduce the warm-up results (distances and masks
    # are unique), which also shows that every asynchronous launch completed
    if not (np.array_equal(dist16.view(nq, n).cpu().numpy(), dd) and
            np.array_equal(mask.cpu().numpy().view(np.uint64)[:, 0], mk)):
        raise RuntimeError("timed steps did not reproduce the warm-up results")
    for _, r in rec:
        if "events" in r:
            r["kernel_ms"] = r["events"][0].elapsed_time(r["events"][1])
            r["rounds"] = float("nan")

    # roofline of the batched BFS kernel
    alg_bytes = float(sum(16 * a + 8 * b for a, b in zip(bfs_nr, bfs_mr)))
    # the reach launch moves one 64-bit mask word per vertex for all 16
    # sources: 20 B per vertex any source reaches and 12 B per arc out of one
    # (the TEPS credit above still counts every source)
    rch_union = mk != 0
    rch_nu, rch_mu = int(rch_union.sum()), int(deg[rch_union].sum())
    rch_alg = float(20 * rch_nu + 12 * rch_mu)
    kms = float(np.mean([b["kernel_ms"] for b, _ in rec]))
    achieved = alg_bytes / (kms * 1e-3) / 1e9
    traffic, note, traffic_frac = None, None, None
    if os.path.exists(PROFILE_COUNTERS):
        with open(PROFILE_COUNTERS) as f:
            pc = json.load(f)
        if (pc.get("kernel_hash") == kernel_source_hash() and pc.get("layout") == args.layout
                and pc.get("tau") == args.tau and pc.get("window") == args.window
                and pc.get("wg_size", 1024) == args.wg and pc.get("schedule", "sequential") == args.schedule
                and pc.get("bfs_share", 100) == (args.bfs_share if conc else 100)):
            traffic = pc.get("hbm_bytes_per_launch")
            traffic_frac = traffic / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS
        else:
            note = "committed counter profile was taken on a different kernel source or setting"
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                "traffic_frac": None if traffic_frac is None else round(traffic_frac, 5),
                "kernel": "vgc_kernel<BFS, multi-query>", "kernel_ms_avg": round(kms, 4),
                "alg_bytes_per_launch": int(alg_bytes)}
    if conc:
        # the reach launch runs beside this one: both launches' algorithmic
        # bytes over the step time
        roofline["concurrent_with"] = "16-source reach launch on a second stream"
        roofline["pair_achieved"] = round((alg_bytes + rch_alg) / (wall / args.steps) / 1e9, 2)
        roofline["pair_frac"] = round(roofline["pair_achieved"] / HBM_PEAK_GBS, 5)
    if note:
        roofline["note"] = note
    rkms = float(np.mean([r["kernel_ms"] for _, r in rec]))
    detail = {
        "schedule": args.schedule,
        "job_alg_bytes_per_step": int(alg_bytes + rch_alg),
        "job_achieved_gbs": round((alg_bytes + rch_alg) / (wall / args.steps) / 1e9, 2),
        "job_frac": round((alg_bytes + rch_alg) / (wall / args.steps) / 1e9 / HBM_PEAK_GBS, 5),
        "bfs_batched_ms": float(np.mean([b["device_ms"] for b, _ in rec])),
        "bfs_kernel_ms": kms,
        "bfs_rounds": float(np.mean([b["rounds"] for b, _ in rec])),
        "bfs_expansions_per_reached": float(np.mean([b["expansions"] for b, _ in rec]) / sum(bfs_nr)),
        "reach16_kernel_ms" if not conc else "reach16_stream_ms": rkms,
        "reach16_rounds": float(np.mean([r["rounds"] for _, r in rec])) if not conc else None,
        "reach16_alg_bytes_per_launch": int(rch_alg),
        "reach16_roofline_frac": round(rch_alg / (rkms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
        "reach16_union_vertices": rch_nu,
        "reach16_union_arcs": rch_mu,
        "arc_passes_per_s": round(float(np.mean([b["arcs_scanned"] for b, _ in rec])) / (kms * 1e-3), 1),
        "reached_vertices_avg": float(np.mean(bfs_nr)),
        "reached_arcs_avg": float(np.mean(bfs_mr)),
        "queries_per_s": round(2 * nq * args.steps / wall, 2),
    }

    # expansions of the reach launch (an untimed call with counters): how
    # often a vertex is expanded again because new source bits reached it
    _, rstat = pg.reach(d, srcs_dev, label_out=mask, stats=True, **dict(rvgc, asynchronous=False))
    detail["reach16_expansions"] = rstat["expansions"]
    detail["reach16_expansions_per_reached"] = round(rstat["expansions"] / max(1, rch_nu), 3)
    detail["reach16_rounds_untimed"] = rstat["rounds"]
    detail["reach16_arcs_scanned"] = rstat["arcs_scanned"]

    cpu = None
    if not args.no_cpu:
        import oracle

        edges, calls, used = 0, 0, 0.0
        for i, s in enumerate(srcs):
            if used > args.cpu_seconds:
                break
            a = time.perf_counter()
            oracle.bfs(g, s)
            oracle.reach(g, [s])
            used += time.perf_counter() - a
            edges += bfs_mr[i] + rch_mr[i]
            calls += 2
        cpu = {"value": round(edges / used / 1e9, 5), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": f"{calls} of the {2 * nq} queries (BFS and reach from the first {calls // 2} sources) "
                         f"in {used:.1f} s on one host thread",
               "host": f"1 of {os.cpu_count()} cores ({_cpu_model()})"}

    extras = {}
    if not args.no_extras:
        dist = torch.empty(n, dtype=torch.int32, device="cuda")
        m1 = torch.empty((n, 1), dtype=torch.int64, device="cuda")
        sub = srcs[:4]
        e_sub = sum(bfs_mr[:4])
        for label, kw in [("plain", dict(mode="plain")), ("tau1", dict(tau=1, window=0)),
                          ("tau64", dict(tau=64, window=0)), ("tau256", dict(tau=256, window=0)),
                          ("tau1024", dict(tau=1024, window=0)), ("tau4096", dict(tau=4096, window=0)),
                          ("tau1024_window32", dict(tau=1024, window=32))]:
            torch.cuda.synchronize()
            a = time.perf_counter()
            rounds, infl = [], []
            for i, s in enumerate(sub):
                _, st = pg.bfs(d, s, dist_out=dist, stats=True, stream=stream, **kw)
                rounds.append(st["rounds"])
                infl.append(st["expansions"] / bfs_nr[i])
            torch.cuda.synchronize()
            el = time.perf_counter() - a
            extras[f"bfs_single_{label}"] = {"gteps": round(e_sub / el / 1e9, 3),
                                             "ms_per_query": round(el / len(sub) * 1e3, 3),
                                             "rounds": float(np.mean(rounds)),
                                             "expansions_per_reached": round(float(np.mean(infl)), 3)}
        for label, kw in [("plain", dict(mode="plain")), ("tau256", dict(tau=256)), ("tau1024", dict(tau=1024)),
                          ("tau4096", dict(tau=4096))]:
            torch.cuda.synchronize()
            a = time.perf_counter()
            for s in sub:
                pg.reach(d, [s], label_out=m1, stream=stream, **kw)
            torch.cuda.synchronize()
            el = time.perf_counter() - a
            extras[f"reach_single_{label}"] = {"gteps": round(sum(rch_mr[:4]) / el / 1e9, 3),
                                               "ms_per_query": round(el / len(sub) * 1e3, 3)}
        if conc:
            # the same job with the two launches one after the other, each on the whole device
            full = dict(tau=args.tau, window=32, wg_size=1024, blocks_per_cu=1, stream=stream)
            sb = pg.Batch(d, vb, np.zeros(nq, np.int32), np.array(srcs, np.int32),
                          np.arange(nq, dtype=np.int64) * n, dist16, **full)
            for rep_ in range(2):
                torch.cuda.synchronize()
                a = time.perf_counter()
                for _ in range(3):
                    sb.run()
                    pg.reach(d, srcs_dev, label_out=mask, **full)
                torch.cuda.synchronize()
                el = (time.perf_counter() - a) / 3
            sb.close()
            extras["job_sequential_full_device"] = {"gteps": round(edges_per_step / el / 1e9, 3),
                                                    "ms_per_step": round(el * 1e3, 3)}
        # latency floor: a BFS from a source of eccentricity e makes e dependent
        # accesses one after the other; this design's level is three (offsets,
        # targets, the returning atomic)
        hop = {k: pg.probe_latency(1 << 30, 20000, k, stream=stream) for k in ("load", "coherent", "atomic")}
        hop_l2 = pg.probe_latency(1 << 20, 20000, "load", stream=stream)
        eccs = []
        for s in sub:
            _, st = pg.bfs(d, s, dist_out=dist, stats=True, stream=stream, mode="plain")
            eccs.append(st["rounds"] - 1)
        ecc = float(np.mean(eccs))
        floor_ms = ecc * hop["load"] * 1e-6
        chain_ms = ecc * (2 * hop["load"] + hop["atomic"]) * 1e-6
        meas = extras["bfs_single_tau1024_window32"]["ms_per_query"]
        extras["latency_floor"] = {
            "t_hop_ns_1GiB": {k: round(v, 1) for k, v in hop.items()}, "t_hop_ns_1MiB_load": round(hop_l2, 1),
            "ecc_mean_of_4_sources": ecc, "ecc_max_of_4_sources": float(max(eccs)),
            "single_bfs_floor_ms": round(floor_ms, 3), "single_bfs_chain_floor_ms": round(chain_ms, 3),
            "single_bfs_measured_ms": meas, "measured_over_floor": round(meas / floor_ms, 2),
            "measured_over_chain_floor": round(meas / chain_ms, 2),
            "job_floor_ms": round(float(max(eccs)) * hop["load"] * 1e-6, 3),
            "note": "floor = eccentricity x one dependent load (1 GiB random cycle); chain floor = eccentricity x "
                    "(2 loads + 1 atomic), the dependent accesses of one level in this design; the job's 16 "
                    "queries run at once, so its floor is the largest eccentricity (of the 4 sampled) x one load"}
        plain_ms = extras["bfs_single_plain"]["ms_per_query"] + extras["reach_single_plain"]["ms_per_query"]
        extras["job_plain_sequential_estimate"] = {
            "gteps": round(edges_per_step / (plain_ms * nq * 1e-3) / 1e9, 3),
            "note": "16 x (plain BFS + plain reach) per-query launches, from the 4-source means above"}

    out = {
        "metric": "GTEPS (16-source BFS + reachability job, VGC; directed 5-NN of 1e7 uniform points)",
        "value": round(gteps, 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"knn5 n={n} m={g.m} points uniform in [0,1)^2 (seed 2, {args.layout} layout), "
                               f"{nq} sources (seed 1002); step = 16 BFS in one batched launch + "
                               f"16-source reach in one launch"
                               + (f", run concurrently on two streams, the batch on {args.bfs_share}% of every CU "
                                  f"and reach on the rest" if conc else
                                  ", one after the other"),
                   "schedule": args.schedule,
                   "tau": args.tau, "reach_tau": args.reach_tau, "window": args.window, "wg_size": args.wg,
                   "reach_wg_size": rwg, "bfs_device_share": args.bfs_share if conc else 100,
                   "blocks_per_cu": args.bpc},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": detail,
        "extras": extras,
    }
    batch.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
