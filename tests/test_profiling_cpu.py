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


def _fake_run(root, sweep_ns, copy_ns, fetch_kib, write_kib, copy_fetch, copy_write,
              sweep=SWEEP, tail=(), upload=None):
    """Profiler output of `sweep` dispatches (then `tail`: (name, ns, fetch,
    write) dispatches of another sweep kernel) and copies; `upload`: (ns,
    fetch, write) of a small copy dispatched before the sweeps."""
    t = os.path.join(root, "T", "host")
    rows, clock = [], 0
    first = [] if upload is None else [(COPY, upload[0])]
    for k, (name, dt) in enumerate(first + [(sweep, dt) for dt in sweep_ns] +
                                   [(x[0], x[1]) for x in tail] + [(COPY, dt) for dt in copy_ns]):
        rows.append((name, clock, clock + dt, k + 1))
        clock += dt + 10
    _write(os.path.join(t, "run_kernel_trace.csv"),
           ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Dispatch_Id"], rows)
    _write(os.path.join(t, "run_kernel_stats.csv"), ["Name", "Calls", "AverageNs", "MinNs", "MaxNs"],
           [(sweep, len(sweep_ns), sum(sweep_ns) / len(sweep_ns),
             min(sweep_ns), max(sweep_ns))])
    for sub, counter, sv, cv, k in (("F", "FETCH_SIZE", fetch_kib, copy_fetch, 2),
                                    ("W", "WRITE_SIZE", write_kib, copy_write, 3)):
        pre = [] if upload is None else [(COPY, upload[k - 1])]
        vals = (pre + [(sweep, v) for v in sv] + [(x[0], x[k]) for x in tail] +
                [(COPY, v) for v in cv])
        rows = [(name, counter, v, j + 1) for j, (name, v) in enumerate(vals)]
        _write(os.path.join(root, sub, "host", "run_counter_collection.csv"),
               ["Kernel_Name", "Counter_Name", "Counter_Value", "Dispatch_Id"], rows)
    log = os.path.join(root, "run.log")
    with open(log, "w") as fh:
        fh.write("noise\n" + json.dumps({"profile": "done", "source_hash": "abc123"}) + "\n")
    return [os.path.join(root, d) for d in "TFW"], log


@pytest.mark.parametrize("upload", [None, (300, 0.5, 0.03125)])
@pytest.mark.parametrize("workload,link", [("tg", 0), ("creeping", 2)])
def test_summary_scales_counters_by_the_copy_kernel(tmp_path, workload, link, upload):
    """The counters are scaled by the run's three closing 1 GiB copies; a
    small copy earlier in the run (an upload) does not enter the scale."""
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
                               copy_write, upload=upload)
    out = os.path.join(str(tmp_path), "summary")
    rec = profiling.summarize(t, f, w, "f32", n, 4, 2, out, run_log=log, workload=workload)
    assert rec["copy_avg_duration_us"] == 2.0
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


def test_two_step_launches_count_two_updates_and_a_trailing_one_step_sweep_is_ignored(tmp_path):
    """A run of two-step launches (sweep_tb2_kernel) that ends on a one-step
    sweep: the summary covers the two-step kernel only, and its algorithmic
    bytes per launch are two lattice updates' (a measured traffic of half of
    them is then a traffic ratio of 0.5)."""
    n = 64
    tb2 = "void trt::(anonymous namespace)::sweep_tb2_kernel<1, 2>(trt::InstDesc, int, int)"
    alg = 2 * 72 * n * n
    copy_fetch, copy_write = [(1 << 30) / 1024.0] * 3, [(1 << 30) / 1024.0] * 3
    fetch = [1.0, 1.0] + [alg / 4 / 1024.0] * 4
    write = [1.0, 1.0] + [alg / 4 / 1024.0] * 4
    tail = [(SWEEP, 777, 5e6, 5e6)]
    (t, f, w), log = _fake_run(str(tmp_path), [3000, 3000] + [2000] * 4, [2000] * 3, fetch,
                               write, copy_fetch, copy_write, sweep=tb2, tail=tail)
    # an SQ pass over the same dispatches
    sq = os.path.join(str(tmp_path), "S", "host")
    vals = {"SQ_WAVES": 4480, "SQ_INSTS_VALU": 8.0e7, "SQ_ACTIVE_INST_VALU": 8.1e7,
            "SQ_WAVE_CYCLES": 3.0e8, "SQ_WAIT_INST_ANY": 1.2e8, "GRBM_GUI_ACTIVE": 4.0e6}
    rows = [(tb2, c, v) for _ in range(6) for c, v in vals.items()]
    rows += [(SWEEP, "SQ_INSTS_VALU", 1.0)]
    _write(os.path.join(sq, "run_counter_collection.csv"),
           ["Kernel_Name", "Counter_Name", "Counter_Value"], rows)
    out = os.path.join(str(tmp_path), "summary")
    rec = profiling.summarize(t, f, w, "f32", n, 4, 2, out, run_log=log,
                              sq_dir=os.path.join(str(tmp_path), "S"))
    assert rec["kernel"] == "sweep_tb2_kernel<1, 2>" and rec["updates_per_launch"] == 2
    assert rec["dispatches"] == 4 and rec["avg_duration_us"] == 2.0
    assert rec["algorithmic_bytes_per_launch"] == alg
    assert rec["traffic_over_algorithmic"] == 0.5
    # 8e7 VALU instructions x 4 cycles over 1024 SIMDs x 5e5 cycles per XCD
    assert rec["valu_busy_frac"] == round(8.0e7 * 4 / (1024 * 4.0e6 / 8), 4)
    assert rec["wave_wait_frac"] == 0.4
    assert "SQ_INSTS_VALU" in open(out + ".md").read()

