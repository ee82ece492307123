"""Host checks of bench.py's profile summaries: the per-launch HBM traffic
figure (FETCH_SIZE and WRITE_SIZE scaled by what the same counters read for
a 1 GiB copy), the trace average over the timed dispatches only, and the
instruction-counter table. Synthetic rocprofv3 CSVs, no GPU."""
import csv
import json
import os
import types

import bench

BFS = "void pg::vgc_kernel<0, true, false, false>(pg::VgcArgs)"
REACH = "void pg::vgc_kernel<1, false, true, true>(pg::VgcArgs)"
COPY = "__amd_rocclr_copyBuffer"


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(header)
        w.writerows(rows)


def _counters(path, entries):
    _write(path, ["Kernel_Name", "Counter_Name", "Counter_Value"], entries)


def _make_run(d):
    # trace: one warm-up dispatch per kernel, then the timed ones, then one
    # more that the summary must leave out (it takes exactly the timed steps)
    start = 1_000_000
    rows = []
    for name, durs in ((BFS, [30.0] + [10.0, 11.0, 12.0, 13.0, 14.0][:bench.TRACE_STEPS] + [99.0]),
                       (REACH, [20.0] + [5.0] * bench.TRACE_STEPS + [77.0])):
        t = start
        for ms in durs:
            rows.append([name, t, t + int(ms * 1e6)])
            t += int(ms * 1e6) + 1000
        start += 10_000_000_000
    _write(os.path.join(d, "prof_trace", "run_kernel_trace.csv"),
           ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    _write(os.path.join(d, "prof_trace", "run_kernel_stats.csv"),
           ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"],
           [[BFS, 7, 1.89e8, 2.7e7, 70.0, 1.0e7, 9.9e7, 0.0], [REACH, 7, 1.2e8, 1.7e7, 30.0, 5.0e6, 7.7e7, 0.0]])
    # counters in KiB per dispatch; the summary averages the dispatches of a kernel
    _counters(os.path.join(d, "prof_fetch", "run_counter_collection.csv"),
              [[BFS, "FETCH_SIZE", 1000.0], [BFS, "FETCH_SIZE", 3000.0], [REACH, "FETCH_SIZE", 600.0],
               [COPY, "FETCH_SIZE", 3.0]])
    _counters(os.path.join(d, "prof_write", "run_counter_collection.csv"),
              [[BFS, "WRITE_SIZE", 4000.0], [REACH, "WRITE_SIZE", 100.0], [REACH, "WRITE_SIZE", 300.0]])
    # a 1 GiB copy reads 0.5 GiB and writes 1 GiB by these counters
    _counters(os.path.join(d, "prof_cfetch", "run_counter_collection.csv"), [[COPY, "FETCH_SIZE", 524288.0]])
    _counters(os.path.join(d, "prof_cwrite", "run_counter_collection.csv"), [[COPY, "WRITE_SIZE", 1048576.0]])


def _args(**kw):
    a = dict(layout="morton", tau=1024, window=32, wg=0, bfs_share=75, schedule="concurrent", reach_tau=0)
    a.update(kw)
    return types.SimpleNamespace(**a)


def test_traffic_is_scaled_by_the_copy_calibration(tmp_path):
    d, out = str(tmp_path / "run"), str(tmp_path / "out")
    os.makedirs(out)
    _make_run(d)
    bench.summarize_profiles(d, _args(), out_dir=out)
    pc = json.load(open(os.path.join(out, "vgc_bfs_batched16_knn10m_counters.txt")))
    cal = pc["copy_calibration"]
    assert abs(cal["fetch_scale"] - 2.0) < 1e-9 and abs(cal["write_scale"] - 1.0) < 1e-9
    # BFS: mean fetch 2000 KiB x 2 + write 4000 KiB x 1
    assert pc["hbm_bytes_per_launch"] == 2000 * 1024 * 2 + 4000 * 1024
    # reach: fetch 600 KiB x 2 + mean write 200 KiB x 1
    assert pc["reach16_hbm_bytes_per_launch"] == 600 * 1024 * 2 + 200 * 1024
    # the timed steps only: neither the warm-up launch nor the one after them
    timed = [10.0, 11.0, 12.0, 13.0, 14.0][:bench.TRACE_STEPS]
    assert abs(pc["kernel_avg_ms"] - sum(timed) / len(timed)) < 1e-6
    assert abs(pc["reach16_avg_ms"] - 5.0) < 1e-6
    # the setting the bench compares before it reports traffic
    assert pc["kernel_hash"] == bench.kernel_source_hash()
    assert (pc["window"], pc["wg_size"], pc["bfs_share"], pc["schedule"]) == (32, 768, 75, "concurrent")
    md = open(os.path.join(out, "vgc_bfs_batched16_knn10m_counters.md")).read()
    assert "scaled by 2.000" in md and "by 1.000" in md
    trace = open(os.path.join(out, "vgc_bfs_batched16_knn10m_trace.md")).read()
    assert f"| `{BFS}` | {len(timed)} | {sum(timed) / len(timed):.3f} | 10.000 |" in trace


def test_sequential_setting_is_recorded_as_whole_device(tmp_path):
    d, out = str(tmp_path / "run"), str(tmp_path / "out")
    os.makedirs(out)
    _make_run(d)
    bench.summarize_profiles(d, _args(schedule="sequential"), out_dir=out)
    pc = json.load(open(os.path.join(out, "vgc_bfs_batched16_knn10m_counters.txt")))
    assert (pc["wg_size"], pc["bfs_share"], pc["schedule"]) == (1024, 100, "sequential")


def test_instruction_counter_table(tmp_path):
    d, out = str(tmp_path / "run"), str(tmp_path / "out")
    os.makedirs(out)
    sq = [[BFS, c, 10.0 * (i + 1)] for i, c in enumerate(bench.SQ_COUNTERS.split())]
    sq += [[BFS, "SQ_WAVES", 30.0]]  # two dispatches: mean 20
    sq += [[REACH, "SQ_INSTS_VALU", 7.0]]
    _counters(os.path.join(d, "pmc_sq", "run_counter_collection.csv"), sq)
    _counters(os.path.join(d, "pmc_tcc", "run_counter_collection.csv"),
              [[BFS, "TCC_HIT_sum", 1234567.0], [REACH, "TCC_MISS_sum", 5.0]])
    bench.summarize_pmc(d, out_dir=out)
    md = open(os.path.join(out, "vgc_bfs_batched16_knn10m_sq.md")).read()
    assert "| SQ_WAVES | 20 | n/a |" in md
    assert "| SQ_INSTS_VALU | 20 | 7 |" in md
    assert "| TCC_HIT_sum | 1,234,567 | n/a |" in md
    assert "| TCC_MISS_sum | n/a | 5 |" in md
