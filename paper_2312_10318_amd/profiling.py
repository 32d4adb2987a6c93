"""Turn rocprofv3 output for the benchmark workload into the short summaries
kept under profiles/.

Three profiler runs of `python3 bench.py --profile ...` (sweeps of the
benchmark lattice followed by a plain 1 GiB device copy):

  rocprofv3 --kernel-trace --stats -f csv -d <T> -o run -- python3 bench.py --profile ...
  rocprofv3 --pmc FETCH_SIZE --kernel-trace -f csv -d <F> -o run -- python3 bench.py --profile ...
  rocprofv3 --pmc WRITE_SIZE --kernel-trace -f csv -d <W> -o run -- python3 bench.py --profile ...

FETCH_SIZE and WRITE_SIZE are reported in KiB per dispatch.  Each is scaled
by the ratio of the copy kernel's known bytes (1 GiB read, 1 GiB written) to
what the same counter reads for that copy, so the sweep's HBM traffic is in
bytes of the same kind as the algorithmic figure.

  python -m paper_2312_10318_amd.profiling <T> <F> <W> --storage f32 --n 4096 \
      --steps 10 --warmup 2 --out profiles/sweep_tg4096_f32 --run-log <stdout of a run>
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SWEEP_SOURCES = ["paper_2312_10318_amd/csrc/sweep.hip", "paper_2312_10318_amd/csrc/lattice.hpp",
                 "paper_2312_10318_amd/csrc/kernels.hpp", "paper_2312_10318_amd/csrc/probe.hip"]
COPY_BYTES = 1 << 30
BYTES_PER_LU = {"f64": 144, "f32": 72, "f16": 36}


def code_of(text: str) -> str:
    """C++ source without its comments, trailing blanks and blank lines
    (the sweep sources hold no string literal with a comment marker)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


def sweep_source_hash() -> str:
    """Hash of the sweep's code (comments and blank lines excluded, so a
    comment edit keeps profiles valid)."""
    h = hashlib.sha256()
    for p in SWEEP_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as fh:
            h.update(code_of(fh.read()).encode())
    return h.hexdigest()[:16]


def _csv(d, suffix):
    fs = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not fs:
        raise FileNotFoundError("no *%s under %s" % (suffix, d))
    with open(fs[0]) as fh:
        return list(csv.DictReader(fh))


def _is_sweep(name):
    return ("sweep_single_kernel" in name or "sweep_pair_kernel" in name or
            "sweep_tb2_kernel" in name or "sweep_tb2_batch_kernel" in name or
            "sweep_tb3_kernel" in name or "sweep_tb3_batch_kernel" in name or
            "sweep_batch_kernel" in name or
            "pattern_probe_kernel" in name)


def updates_per_launch(kernel_name) -> int:
    """Time steps one launch of a sweep kernel advances the lattice by."""
    name = kernel_name or ""
    return 3 if "sweep_tb3" in name else 2 if "sweep_tb2" in name else 1


def _is_copy(name):
    return "copyBuffer" in name


# `bench.py --profile` ends with this many plain copies of COPY_BYTES; only
# those (the last copy dispatches) scale the counters -- a run may also
# copy small buffers on the way (uploads)
COPIES = 3


def _last_copies(copies):
    """Values of the run's closing copies from (dispatch id, value) pairs."""
    return [v for _, v in sorted(copies)[-COPIES:]]


def kernel_durations(trace_dir):
    """Durations (ns) of the run's sweep kernel -- the sweep kernel with the
    most dispatches (a run of two-step launches may end on a one-step
    sweep) -- and of the copy kernel, and the sweep kernel's name."""
    rows = _csv(trace_dir, "kernel_trace.csv")
    by_name, copy = {}, []
    for r in rows:
        dt = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        if _is_sweep(r["Kernel_Name"]):
            by_name.setdefault(r["Kernel_Name"], []).append(dt)
        elif _is_copy(r["Kernel_Name"]):
            copy.append((int(r["Dispatch_Id"]), dt))
    copy = _last_copies(copy)
    if not by_name:
        return [], copy, None
    name = max(by_name, key=lambda k: len(by_name[k]))
    return by_name[name], copy, name


def counter_values(pmc_dir, counter, kernel=None):
    """Values of `counter` per dispatch of the sweep kernel `kernel` (any
    sweep kernel when None) and of the copy kernel."""
    rows = _csv(pmc_dir, "counter_collection.csv")
    sweep, copy = [], []
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        v = float(r["Counter_Value"])
        if _is_sweep(r["Kernel_Name"]) and (kernel is None or r["Kernel_Name"] == kernel):
            sweep.append(v)
        elif _is_copy(r["Kernel_Name"]):
            copy.append((int(r["Dispatch_Id"]), v))
    return sweep, _last_copies(copy)


def _run_record(log_path):
    """The record `bench.py --profile` printed at run time."""
    with open(log_path) as fh:
        for line in fh:
            line = line.strip()
            if line.startswith("{") and '"profile"' in line:
                return json.loads(line)
    raise ValueError("no profile record in " + log_path)


def _run_hash(log_path):
    """The sweep source hash that `bench.py --profile` printed at run time."""
    return _run_record(log_path).get("source_hash")


# Workloads of `bench.py --profile`: (title, name, link code bytes per node).
WORKLOADS = {
    "tg": ("Taylor-Green %dx%d", "taylor_green_%dx%d", 0),
    "creeping": ("creeping flow past a square cylinder (Sec. III.D), %dx%d, obstacle, "
                 "inflow wall and pressure outlet", "creeping_cylinder_%dx%d", 2),
    "channel": ("force-driven channel (Sec. III.C), %dx%d, walls on the first and last rows "
                "(whole-row walls: no link codes read)", "channel_%dx%d", 0),
    "batch": ("the 256-member batch (Taylor-Green and double-shear-layer members, sides "
              "64 to 1024, %d nodes in all, the library's default batch shape)", "batch256", 0),
    "stream": ("access-pattern probe (the sweep's loads, stores, launch shape and barriers "
               "without its arithmetic) on the Taylor-Green lattice %dx%d",
               "pattern_probe_%dx%d", 0),
}


SQ_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_WAVE_CYCLES",
               "SQ_WAIT_INST_ANY", "GRBM_GUI_ACTIVE")
SIMDS = 1024  # 256 CUs x 4 SIMDs
XCDS = 8


def sq_summary(sq_dir, kernel, skip_first=2):
    """Instruction-issue figures of the sweep kernel from one rocprofv3 pass
    over SQ_COUNTERS: VALU instructions per launch and the fraction of the
    SIMDs' issue cycles they fill (a wave64 VALU instruction occupies its
    16-lane SIMD for 4 cycles; GRBM_GUI_ACTIVE counts the busy cycles of
    each XCD, summed over the eight)."""
    vals = {}
    for c in SQ_COUNTERS:
        v, _ = counter_values(sq_dir, c, kernel)
        v = v[skip_first:]
        if v:
            vals[c] = sum(v) / len(v)
    out = {"sq_" + k.lower(): round(v, 1) for k, v in vals.items()}
    if "SQ_INSTS_VALU" in vals and "GRBM_GUI_ACTIVE" in vals:
        cycles = vals["GRBM_GUI_ACTIVE"] / XCDS
        out["valu_busy_frac"] = round(vals["SQ_INSTS_VALU"] * 4 / (SIMDS * cycles), 4)
    if "SQ_WAIT_INST_ANY" in vals and "SQ_WAVE_CYCLES" in vals:
        out["wave_wait_frac"] = round(vals["SQ_WAIT_INST_ANY"] / vals["SQ_WAVE_CYCLES"], 4)
    return out


def summarize(trace_dir, fetch_dir, write_dir, storage, n, steps, warmup, out_prefix,
              skip_first=2, run_log=None, workload="tg", nodes=None, tuning=None,
              sq_dir=None):
    sweep_ns, copy_ns, kname = kernel_durations(trace_dir)
    fs, fc = counter_values(fetch_dir, "FETCH_SIZE", kname)
    ws, wc = counter_values(write_dir, "WRITE_SIZE", kname)
    # the first dispatches include cold-cache and launch warm-up effects
    sweep_ns, fs, ws = sweep_ns[skip_first:], fs[skip_first:], ws[skip_first:]
    avg = lambda v: sum(v) / len(v)
    fetch_scale = COPY_BYTES / (avg(fc) * 1024.0)
    write_scale = COPY_BYTES / (avg(wc) * 1024.0)
    fetch_b = avg(fs) * 1024.0 * fetch_scale
    write_b = avg(ws) * 1024.0 * write_scale
    title, wname, link_bytes = WORKLOADS[workload]
    if workload == "batch":
        if not nodes:
            raise ValueError("the batch workload needs its node count")
        label, wlabel = title % nodes, wname
    else:
        nodes = n * n
        label, wlabel = title % (n, n), wname % (n, n)
    # 9 populations read and written (+ the link code read, with a link map)
    # per lattice update; a two-step launch counts two updates per node
    ups = updates_per_launch(kname)
    alg = (BYTES_PER_LU[storage] + link_bytes) * nodes * ups
    dur = avg(sweep_ns) * 1e-9
    rec = {
        "kernel": (re.search(r"(sweep_(single|pair|tb2_batch|tb2|tb3_batch|tb3|batch)|pattern_probe)_kernel(<[^>]*>)?",
                             kname or "") or re.search(r".*", "sweep")).group(0),
        "workload": wlabel, "storage": storage, "nodes": nodes, "updates_per_launch": ups,
        "source_hash": _run_hash(run_log) if run_log else sweep_source_hash(),
        "dispatches": len(sweep_ns), "avg_duration_us": round(dur * 1e6, 3),
        "algorithmic_bytes_per_launch": alg,
        "achieved_GBps_algorithmic": round(alg / dur / 1e9, 1),
        "fetch_counter_KiB": round(avg(fs), 1), "write_counter_KiB": round(avg(ws), 1),
        "copy_fetch_counter_KiB": round(avg(fc), 1), "copy_write_counter_KiB": round(avg(wc), 1),
        "fetch_scale": round(fetch_scale, 4), "write_scale": round(write_scale, 4),
        "hbm_read_bytes_per_launch": int(fetch_b), "hbm_write_bytes_per_launch": int(write_b),
        "hbm_bytes_per_launch": int(fetch_b + write_b),
        "traffic_over_algorithmic": round((fetch_b + write_b) / alg, 4),
        "hbm_GBps_measured": round((fetch_b + write_b) / dur / 1e9, 1),
        "copy_avg_duration_us": round(avg(copy_ns) * 1e-3, 3) if copy_ns else None,
    }
    if sq_dir:
        rec.update(sq_summary(sq_dir, kname, skip_first))
    if workload in ("tg", "stream", "channel"):
        cmd = ("python3 bench.py --profile%s --storage %s --n %d --steps %d --warmup %d"
               % ("" if workload == "tg" else " --workload " + workload, storage, n, steps,
                  warmup))
    else:
        cmd = ("python3 bench.py --profile --workload %s --storage %s --steps %d --warmup %d"
               % (workload, storage, steps, warmup))
    if tuning:
        cmd += " --tuning " + tuning
        rec["launch_shape"] = tuning
    if run_log and _run_record(run_log).get("launch"):
        # (rows, wavefronts per workgroup, XCD remap, columns per lane, longest
        # graph, time steps per launch, prefetch rows) in effect
        rec["launch_in_effect"] = _run_record(run_log)["launch"]
    with open(out_prefix + "_hbm_counters.json", "w") as fh:
        json.dump(rec, fh, indent=1)
    with open(out_prefix + ".md", "w") as fh:
        fh.write("# Fused sweep, %s, %s storage\n\n" % (label, storage))
        fh.write("Commands (run from the repository root, one profiler run each):\n\n")
        if workload == "tg" and not tuning:
            fh.write("    python3 bench.py --tune-only --storage %s --n %d   # the autotuner's "
                     "launch shape, cached for the runs below\n" % (storage, n))
        fh.write("    rocprofv3 --kernel-trace --stats -f csv -d <T> -o run -- %s\n" % cmd)
        fh.write("    rocprofv3 --pmc FETCH_SIZE --kernel-trace -f csv -d <F> -o run -- %s\n" % cmd)
        fh.write("    rocprofv3 --pmc WRITE_SIZE --kernel-trace -f csv -d <W> -o run -- %s\n" % cmd)
        if sq_dir:
            fh.write("    rocprofv3 --pmc %s --kernel-trace -f csv -d <S> -o run -- %s\n"
                     % (" ".join(SQ_COUNTERS), cmd))
        fh.write("    python -m paper_2312_10318_amd.profiling <T> <F> <W> --workload %s "
                 "--storage %s --n %d --steps %d --warmup %d%s%s%s --out %s\n\n"
                 % (workload, storage, n, steps, warmup,
                    " --nodes %d" % nodes if workload == "batch" else "",
                    " --tuning %s" % tuning if tuning else "",
                    " --sq <S>" if sq_dir else "",
                    os.path.relpath(out_prefix, ROOT)))
        fh.write("| quantity | value |\n|---|---|\n")
        for k, v in rec.items():
            fh.write("| %s | %s |\n" % (k, v))
        fh.write("\nAlgorithmic bytes per launch: bytes per lattice update (9 populations "
                 "read and written) x nodes x time steps per launch.\n")
        fh.write("\nCounters are KiB per dispatch; the scale factors are 1 GiB divided by "
                 "what the same counter reads for a plain 1 GiB device copy.\n")
        if sq_dir:
            fh.write("\nvalu_busy_frac: VALU instructions x 4 cycles / (1024 SIMDs x busy "
                     "cycles per XCD); wave_wait_frac: SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES "
                     "(the share of the wavefronts' lifetime spent waiting to issue).\n")
        stats = _csv(trace_dir, "kernel_stats.csv")
        fh.write("\n`--kernel-trace --stats` summary (durations in ns):\n\n")
        fh.write("| kernel | calls | average | min | max |\n|---|---|---|---|---|\n")
        for r in stats:
            nm = r["Name"]
            m = re.search(r"(\w+_kernel(<[^>]*>)?|copyBuffer)", nm)
            fh.write("| %s | %s | %.0f | %s | %s |\n" % (m.group(1) if m else nm[:40],
                     r["Calls"], float(r["AverageNs"]), r["MinNs"], r["MaxNs"]))
    return rec


def bench_trace_summary(trace_dir, bench_json, out_prefix, cmd):
    """The rocprofv3 kernel trace of a bench.py run next to the average
    launch duration that run measured live with HIP events (its JSON line):
    the traced average of the roofline's kernel must agree with it."""
    with open(bench_json) as fh:
        rec = json.loads([l for l in fh if l.strip().startswith("{")][-1])
    live = rec["roofline"]["avg_duration_us"]
    want = rec["roofline"]["kernel"].split("<")[0]
    stats = _csv(trace_dir, "kernel_stats.csv")
    traced = [r for r in stats if want in r["Name"]]
    if not traced:
        raise ValueError("no %s in the trace" % want)
    t = traced[0]
    out = {"kernel": want, "workload": rec["config"]["workload"], "dtype": rec["dtype"],
           "source_hash": rec["roofline"]["source_hash"], "dispatches": int(t["Calls"]),
           "traced_avg_duration_us": round(float(t["AverageNs"]) * 1e-3, 3),
           "live_avg_duration_us": live,
           "traced_over_live": round(float(t["AverageNs"]) * 1e-3 / live, 4),
           "value": rec["value"], "unit": rec["unit"], "frac": rec["roofline"]["frac"]}
    with open(out_prefix + ".json", "w") as fh:
        json.dump(out, fh, indent=1)
    with open(out_prefix + ".md", "w") as fh:
        fh.write("# Kernel trace of the benchmark command, %s\n\n" % out["workload"])
        fh.write("Command (run from the repository root):\n\n")
        fh.write("    rocprofv3 --kernel-trace --stats -f csv -d <T> -o run -- %s\n" % cmd)
        fh.write("    python -m paper_2312_10318_amd.profiling --bench-trace <T> <stdout of the "
                 "run> --cmd '%s' --out %s\n\n" % (cmd, os.path.relpath(out_prefix, ROOT)))
        fh.write("| quantity | value |\n|---|---|\n")
        for k, v in out.items():
            fh.write("| %s | %s |\n" % (k, v))
        fh.write("\nlive_avg_duration_us: the run's own HIP-event time per launch on the "
                 "sweep's stream (bench.py's roofline.avg_duration_us).\n")
        fh.write("\n`--kernel-trace --stats` summary (durations in ns):\n\n")
        fh.write("| kernel | calls | average | min | max |\n|---|---|---|---|---|\n")
        for r in stats:
            nm = r["Name"]
            m = re.search(r"(\w+_kernel(<[^>]*>)?|copyBuffer)", nm)
            fh.write("| %s | %s | %.0f | %s | %s |\n" % (m.group(1) if m else nm[:40],
                     r["Calls"], float(r["AverageNs"]), r["MinNs"], r["MaxNs"]))
    return out


def main():
    if len(os.sys.argv) > 1 and os.sys.argv[1] == "--bench-trace":
        bp = argparse.ArgumentParser()
        bp.add_argument("--bench-trace", nargs=2, metavar=("TRACE_DIR", "BENCH_STDOUT"))
        bp.add_argument("--cmd", required=True, help="the traced bench.py command")
        bp.add_argument("--out", required=True)
        b = bp.parse_args()
        out = os.path.join(ROOT, b.out) if not os.path.isabs(b.out) else b.out
        print(json.dumps(bench_trace_summary(*b.bench_trace, out, b.cmd), indent=1))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("trace_dir")
    ap.add_argument("fetch_dir")
    ap.add_argument("write_dir")
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--workload", default="tg", choices=sorted(WORKLOADS))
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--out", required=True)
    ap.add_argument("--run-log", default=None,
                    help="stdout of the profiled bench.py run (carries the source hash the "
                         "profiled kernel was built from)")
    ap.add_argument("--tuning", default=None,
                    help="the --tuning argument of the profiled bench.py run, if any")
    ap.add_argument("--sq", default=None,
                    help="output directory of a rocprofv3 pass over the SQ_COUNTERS")
    ap.add_argument("--nodes", type=int, default=None,
                    help="lattice updates per launch of the batch workload (printed by the "
                         "profiled run)")
    a = ap.parse_args()
    rec = summarize(a.trace_dir, a.fetch_dir, a.write_dir, a.storage, a.n, a.steps, a.warmup,
                    os.path.join(ROOT, a.out) if not os.path.isabs(a.out) else a.out,
                    run_log=a.run_log, workload=a.workload, nodes=a.nodes, tuning=a.tuning,
                    sq_dir=a.sq)
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
