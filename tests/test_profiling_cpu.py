"""Host logic of the rocprofv3 summariser (synthetic profiler output, no GPU)."""
import csv
import json
import os

import pytest

from paper_2312_10318_amd import profiling

SWEEP = "void trt::(anonymous namespace)::sweep_pair_kernel<1, false>(trt::InstDesc, int, int)"
COPY = "copyBuffer"


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def _fake_run(root, sweep_ns, copy_ns, fetch_kib, write_kib, copy_fetch, copy_write):
    t = os.path.join(root, "T", "host")
    rows, clock = [], 0
    for dt in sweep_ns:
        rows.append((SWEEP, clock, clock + dt))
        clock += dt + 10
    for dt in copy_ns:
        rows.append((COPY, clock, clock + dt))
        clock += dt + 10
    _write(os.path.join(t, "run_kernel_trace.csv"),
           ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    _write(os.path.join(t, "run_kernel_stats.csv"), ["Name", "Calls", "AverageNs", "MinNs", "MaxNs"],
           [(SWEEP, len(sweep_ns), sum(sweep_ns) / len(sweep_ns),
             min(sweep_ns), max(sweep_ns))])
    for sub, counter, sv, cv in (("F", "FETCH_SIZE", fetch_kib, copy_fetch),
                                 ("W", "WRITE_SIZE", write_kib, copy_write)):
        rows = [(SWEEP, counter, v) for v in sv] + [(COPY, counter, v) for v in cv]
        _write(os.path.join(root, sub, "host", "run_counter_collection.csv"),
               ["Kernel_Name", "Counter_Name", "Counter_Value"], rows)
    log = os.path.join(root, "run.log")
    with open(log, "w") as fh:
        fh.write("noise\n" + json.dumps({"profile": "done", "source_hash": "abc123"}) + "\n")
    return [os.path.join(root, d) for d in "TFW"], log


@pytest.mark.parametrize("workload,link", [("tg", 0), ("creeping", 2)])
def test_summary_scales_counters_by_the_copy_kernel(tmp_path, workload, link):
    n = 64
    nodes = n * n
    alg = (72 + link) * nodes
    # the copy reads 1 GiB and the fetch counter shows half of it: scale 2;
    # the write counter shows all of it: scale 1
    copy_fetch, copy_write = [(1 << 30) / 2048.0] * 3, [(1 << 30) / 1024.0] * 3
    # sweeps: two warm-up dispatches (skipped), then 1000 ns each moving
    # 1.5x the algorithmic reads and exactly the algorithmic writes
    sweep_ns = [5000, 4000] + [1000] * 4
    rd, wr = alg / 2 * 1.5, alg / 2
    fetch = [999.0, 999.0] + [rd / 2 / 1024.0] * 4
    write = [999.0, 999.0] + [wr / 1024.0] * 4
    (t, f, w), log = _fake_run(str(tmp_path), sweep_ns, [2000] * 3, fetch, write, copy_fetch,
                               copy_write)
    out = os.path.join(str(tmp_path), "summary")
    rec = profiling.summarize(t, f, w, "f32", n, 4, 2, out, run_log=log, workload=workload)
    assert rec["dispatches"] == 4 and rec["avg_duration_us"] == 1.0
    assert rec["algorithmic_bytes_per_launch"] == alg
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    assert rec["hbm_read_bytes_per_launch"] == int(rd)
    assert rec["hbm_write_bytes_per_launch"] == int(wr)
    assert rec["traffic_over_algorithmic"] == 1.25
    assert rec["achieved_GBps_algorithmic"] == round(alg / 1e-6 / 1e9, 1)
    assert rec["source_hash"] == "abc123"
    assert rec["kernel"] == "sweep_pair_kernel<1, false>"
    assert rec["workload"] == ("taylor_green_64x64" if workload == "tg" else "creeping_cylinder_64x64")
    md = open(out + ".md").read()
    assert ("--workload creeping" in md) == (workload == "creeping")
    assert json.load(open(out + "_hbm_counters.json")) == rec


def test_source_hash_ignores_comments_but_not_code():
    from paper_2312_10318_amd.profiling import code_of
    a = "int x;  // one\n// two\n\nint y;\n"
    b = "int x;\n/* three\n   four */\nint y;   \n"
    assert code_of(a) == code_of(b) == "int x;\nint y;"
    assert code_of("int x;\nint z;\n") != code_of(a)
