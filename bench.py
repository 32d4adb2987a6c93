"""Throughput benchmark of the fused D2Q9 TRT-RLB sweep on one MI355X.

Workload (one "step" = one time step of the whole lattice): Taylor-Green
vortex 4096 x 4096, periodic, u0 = 0.01, tau_s = 0.6, Lambda_s = 1/4
(tau_s2 = 3), populations stored as f - w in FP32, FP32 arithmetic.  The
lattices are resident in HBM before timing starts; K steps are timed with HIP
events on the stream the sweeps are launched on.

The JSON line reports MLUPS (lattice updates per second / 1e6), the roofline
of the sweep kernel (algorithmic bytes per lattice update x updates per
launch / average launch time, against the 8 TB/s HBM peak), and the FP64 CPU
oracle timed on a bounded sample of the same workload on the host cores.
By the library default the FP32 benchmark lattice runs three time steps per
launch and FP16 two, so a launch counts that many lattice updates per node;
it moves each population through HBM about once, and the measured traffic
(rocprofv3 counters) is a fraction of the algorithmic bytes.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--storage f32]
                      [--no-extra] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_LU = {"f64": 144, "f32": 72, "f16": 36}  # 9 reads + 9 writes per node
COUNTERS_FILE = os.path.join(ROOT, "profiles", "sweep_tg%d_%s_hbm_counters.json")


def sweep_source_hash() -> str:
    from paper_2312_10318_amd.profiling import sweep_source_hash as h
    return h()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_steps(lat, steps, warmup):
    """Average time per step (ms) over `steps` steps after `warmup` steps."""
    import torch
    # the step graphs the warm-up and the timed steps replay are captured
    # first (for the timed steps from either lattice the warm-up may end on),
    # so the warm-up runs right before the timed region and no host-side
    # capture falls between them or in it
    lat.prepare(warmup)
    for n in (steps - 1, steps, steps + 1):
        lat.prepare(max(n, 0))
    lat.step(warmup)
    torch.cuda.synchronize()
    with torch.cuda.stream(lat.stream):
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record(lat.stream)
        lat.step(steps)
        end.record(lat.stream)
    end.synchronize()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps


def time_probe(lat, launches, warmup=3):
    """Average time per launch (ms) of the access-pattern probe on the
    lattice's stream (the probe scrambles the lattice)."""
    import torch
    lat.pattern_probe(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(lat.stream)
    lat.pattern_probe(launches)
    end.record(lat.stream)
    end.synchronize()
    return start.elapsed_time(end) / launches


def tg_lattice(n, storage, tau1=0.6, lam=0.25, tuning=None):
    from paper_2312_10318_amd import inputs, params
    from paper_2312_10318_amd.lattice import Lattice
    tau2 = params.tau2_from_magic(tau1, lam)
    rho, ux, uy = inputs.taylor_green(n, 0.01, seed=0)
    lat = Lattice(n, n, tau1, tau2, storage=storage)
    if tuning:
        lat.set_tuning(*tuning)
    lat.init_equilibrium(rho, ux, uy)
    return lat


def headline_shape(lat, n, storage):
    """The launch shape a Taylor-Green benchmark lattice runs in: the
    autotuner's pick among the shapes of the lattice's default pass (its
    time steps per launch), timed on a scratch lattice and cached per box
    like every tuner result.  Returns (shape, record)."""
    from paper_2312_10318_amd import autotune
    rows, waves, remap, cols, _, sps, prefetch = lat.tuning()
    default = (rows, waves, remap, cols if sps == 1 else 2, 0, sps, prefetch)
    key = autotune.key(n, n, storage, False) + "|steps%d" % sps
    cache = autotune.load_cache()
    if key in cache:
        c = cache[key]
        return tuple(c["best"]), c
    shapes = [sh for sh in autotune.candidates(n, n, False, storage) if sh[5] == sps]
    if default not in shapes:
        shapes.append(default)
    res = autotune.tune(n, n, storage, shapes=shapes)
    table = {tuple(sh): ms for sh, ms in res["table"]}
    rec = {"best": res["best"], "ms": res["ms"], "default": list(default),
           "default_ms": table[default], "candidates": len(shapes), "when": res["when"]}
    cache[key] = rec
    autotune.save_cache(cache)
    return tuple(res["best"]), rec


def rel_errors(u, v, ur, vr):
    """(relative max, relative L2) velocity error against reference fields;
    the L2 norm sums both components (the error measure of Sec. III)."""
    import numpy as np
    scale = max(np.max(np.abs(ur)), np.max(np.abs(vr)))
    emax = max(np.max(np.abs(u - ur)), np.max(np.abs(v - vr))) / scale
    el2 = np.sqrt((np.sum((u - ur) ** 2) + np.sum((v - vr) ** 2)) /
                  (np.sum(ur ** 2) + np.sum(vr ** 2)))
    return float("%.3e" % emax), float("%.3e" % el2)


def velocity(lat):
    """(ux, uy) of a lattice as numpy FP64 arrays."""
    _, u, v = lat.macros()
    return u.cpu().numpy(), v.cpu().numpy()


def fp64_alone(nx, ny, tau1, tau2, steps, fields, g=(0.0, 0.0), mask=None, inflow=None):
    """Velocity of the same problem run alone in FP64 storage on the GPU (the
    path the parity tests hold to the FP64 oracle within 1e-12), the
    reference of the batched and served errors."""
    from paper_2312_10318_amd.lattice import Lattice
    lat = Lattice(nx, ny, tau1, tau2, g=g, mask=mask, storage="f64", inflow=inflow)
    lat.init_equilibrium(*fields).step(steps)
    out = velocity(lat)
    lat.close()
    return out


def accuracy_vs_oracle(n, ref):
    """Errors of the benchmark lattice in every storage against the oracle
    state of the CPU-baseline sample (same seeded lattice, same steps)."""
    steps, ur, vr = ref
    out = {"reference": "FP64 CPU oracle, the cpu_baseline sample", "steps": steps}
    for storage in ("f32", "f16", "f64"):
        lat = tg_lattice(n, storage)
        lat.step(steps)
        u, v = velocity(lat)
        lat.close()
        emax, el2 = rel_errors(u, v, ur, vr)
        out[storage] = {"err_max": emax, "err_L2": el2}
        log("accuracy %s after %d steps vs oracle: rel max %.3e, rel L2 %.3e"
            % (storage, steps, emax, el2))
    return out


def cpu_baseline(n=4096, budget_s=12.0):
    """The FP64 oracle on the host cores, on a bounded sample: the same
    4096^2 Taylor-Green lattice, as many whole steps as fit in ~budget_s.
    Returns the record and the sample's final state (steps, ux, uy), which
    the GPU runs are compared with."""
    import numpy as np  # noqa: F401
    import oracle
    from paper_2312_10318_amd import inputs, params
    tau1 = 0.6
    tau2 = params.tau2_from_magic(tau1, 0.25)
    rho, ux, uy = inputs.taylor_green(n, 0.01, seed=0)
    f = oracle.init_equilibrium(rho, ux, uy)
    t0 = time.perf_counter()
    f = oracle.step(f, tau1, tau2)
    t1 = time.perf_counter() - t0
    extra = max(0, int(budget_s / max(t1, 1e-9)) - 1)
    t0 = time.perf_counter()
    if extra:
        f = oracle.run(f, extra, tau1, tau2)
    t2 = time.perf_counter() - t0
    steps = 1 + extra
    total = t1 + t2
    cores = oracle.num_threads()
    # one thread, on a smaller sample (1024^2, one step: ~0.2-0.5 s)
    m = 1024
    r1, u1, v1 = inputs.taylor_green(m, 0.01, seed=0)
    f1 = oracle.init_equilibrium(r1, u1, v1)
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.step(f1, tau1, tau2)
        single = m * m / (time.perf_counter() - t0) / 1e6
    finally:
        oracle.set_num_threads(cores)
    _, ur, vr = oracle.macros(f)
    return ({"value": round(n * n * steps / total / 1e6, 3), "unit": "MLUPS",
             "cores": cores, "kind": "oracle",
             "sample": "Taylor-Green %dx%d FP64, %d whole steps (%.1f s)" % (n, n, steps, total),
             "single_thread_MLUPS": round(single, 3),
             "single_thread_sample": "Taylor-Green %dx%d FP64, one step" % (m, m),
             "configs": cpu_configs(cores),
             "cpu_model": cpu_model()}, (steps, ur, vr))


def cpu_configs(cores):
    """The oracle on the two small configurations, all host cores and one
    thread: Taylor-Green 64^2 x 1000 steps (u0 = 0.01, tau_s = 0.6,
    Lambda_s = 1/4) and the double shear layer 1024^2 (U0 = 0.04, kappa = 80,
    delta = 0.05, Re = 1e4, 1/tau_s2 = 1.6) x 100 steps (x 5 on one
    thread).  A few seconds on 16 cores."""
    import oracle
    from paper_2312_10318_amd import inputs, params
    out = {}

    def timed(label, f, steps, tau1, tau2, nodes, threads):
        oracle.set_num_threads(threads)
        try:
            t0 = time.perf_counter()
            oracle.run(f, steps, tau1, tau2)
            sec = time.perf_counter() - t0
        finally:
            oracle.set_num_threads(cores)
        out[label] = {"MLUPS": round(nodes * steps / sec / 1e6, 3), "threads": threads,
                      "steps": steps, "seconds": round(sec, 3)}

    tau1 = 0.6
    tau2 = params.tau2_from_magic(tau1, 0.25)
    f = oracle.init_equilibrium(*inputs.taylor_green(64, 0.01, seed=0))
    timed("taylor_green_64x64_x1000", f, 1000, tau1, tau2, 64 * 64, cores)
    timed("taylor_green_64x64_x1000_1thread", f, 1000, tau1, tau2, 64 * 64, 1)
    n, u0 = 1024, 0.04
    tau1 = 0.5 + 3.0 * u0 * n / 1e4
    f = oracle.init_equilibrium(*inputs.double_shear_layer(n, u0))
    timed("double_shear_layer_1024x1024_x100", f, 100, tau1, 1 / 1.6, n * n, cores)
    timed("double_shear_layer_1024x1024_x5_1thread", f, 5, tau1, 1 / 1.6, n * n, 1)
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def profile_record(n, storage):
    """The committed rocprofv3 summary of this workload, if it was taken on
    the current sweep source; else None."""
    try:
        with open(COUNTERS_FILE % (n, storage)) as fh:
            c = json.load(fh)
    except (OSError, ValueError):
        return None
    if c.get("source_hash") != sweep_source_hash() or c.get("nodes") != n * n or \
            c.get("storage") != storage:
        return None
    return c


def traffic_from_counters(n, storage):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current sweep source; else None."""
    c = profile_record(n, storage)
    return None if c is None else c.get("hbm_bytes_per_launch")


def run_batch(count=256, steps=5000, storage="f32", seed=0):
    """The batched workload: `count` independent periodic lattices (sides
    log-uniform in [64, 1024], half Taylor-Green and half double shear layer,
    Re log-uniform in [1e2, 1e7], tau_s2 uniform in [0.5, 2]) advanced by one
    batched launch per step (graph-captured pairs), in the launch shape the
    autotuner picks on scratch copies of the members (before the timed
    region)."""
    import torch
    from paper_2312_10318_amd import autotune, inputs
    from paper_2312_10318_amd.lattice import Batch, Lattice
    members = inputs.batch_workload(count, seed=seed)
    lats = []
    for k, m in enumerate(members):
        rho, ux, uy = inputs.member_fields(m, seed=k)
        lats.append(Lattice(m.n, m.n, m.tau1, m.tau2, storage=storage).init_equilibrium(rho, ux, uy))
    tuned = autotune.tune_batch(lats)
    table = {tuple(s): ms for s, ms in tuned["table"]}
    b = Batch(lats)
    b.set_tuning(*tuned["best"])
    b.step(20)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(b.stream)
    b.step(steps)
    end.record(b.stream)
    end.synchronize()
    sec = start.elapsed_time(end) * 1e-3
    diag = b.diagnostics()
    nodes = sum(m.n * m.n for m in members)
    bad = [k for k in range(count) if diag[k, 4] > 0]
    # accuracy at the end of the timed run: sampled members (smallest and
    # largest, odd and even widths, both flow kinds, none diverged) against
    # the same member run alone in FP64
    ok = [k for k in range(count) if k not in bad]
    sizes = {k: members[k].n for k in ok}
    pick = [min(ok, key=sizes.get), max(ok, key=sizes.get)]
    pick += [k for k in ok if members[k].n % 2 == 1][:1] + [k for k in ok if members[k].n % 2 == 0][:1]
    pick += [k for k in ok if members[k].kind == "dsl"][:1] + [k for k in ok if members[k].kind == "tg"][:1]
    acc = []
    for k in sorted(set(pick)):
        m = members[k]
        ur, vr = fp64_alone(m.n, m.n, m.tau1, m.tau2, 20 + steps, inputs.member_fields(m, seed=k))
        u, v = velocity(lats[k])
        emax, el2 = rel_errors(u, v, ur, vr)
        acc.append({"member": k, "kind": m.kind, "n": m.n, "Re": float("%.3g" % m.re),
                    "err_max": emax, "err_L2": el2})
    b.close()
    for l in lats:
        l.close()
    return {"instances": count, "steps": steps, "storage": storage, "nodes": nodes,
            "seconds": round(sec, 4), "solves_per_s": round(count / sec, 3),
            "aggregate_MLUPS": round(nodes * steps / sec / 1e6, 1),
            "launch_shape": list(tuned["best"]),
            "tuned_ms_per_step": round(tuned["ms"], 4),
            "default_ms_per_step": round(table.get((0, 4, 0, 0, -1, 1), float("nan")), 4),
            "accuracy": {"reference": "each sampled member run alone in FP64 storage on the GPU",
                         "steps": 20 + steps, "members": acc,
                         "err_max": max(a["err_max"] for a in acc),
                         "err_L2": max(a["err_L2"] for a in acc)},
            "diverged_instances": len(bad),
            "diverged": ["%s n=%d Re=%.3g 1/tau2=%.3f" % (members[k].kind, members[k].n,
                                                         members[k].re, 1 / members[k].tau2)
                         for k in bad[:40]]}


def run_serving(storage, rate=200.0, duration=2.0, budget_gb=64.0, seed=0):
    """Poisson solve stream through the continuous-batching server."""
    from paper_2312_10318_amd import inputs, serving
    reqs = serving.serving_workload(rate=rate, duration=duration, seed=seed)
    # the smallest request of each kind keeps its final fields (checked below)
    sample = {kind: min((r for r in reqs if r.kind == kind), key=lambda r: r.nx * r.ny).rid
              for kind in ("cylinder", "poiseuille", "taylor_green")}
    ex = serving.GpuExecutor(storage)
    sched = serving.Scheduler(ex, budget_bytes=int(budget_gb * (1 << 30)), quantum=100,
                              keep_fields=set(sample.values()))
    t0 = time.perf_counter()
    res = sched.run(reqs)
    wall = time.perf_counter() - t0
    ex.shutdown()
    out = serving.summarize(res, wall)
    by = {r.rid: r for r in res}
    acc = []
    for kind, rid in sample.items():
        q = next(r for r in reqs if r.rid == rid)
        fields = q.fields() if q.fields else inputs.rest_state(q.ny, q.nx)
        ur, vr = fp64_alone(q.nx, q.ny, q.tau1, q.tau2, q.steps, fields, g=q.g, mask=q.mask,
                            inflow=q.inflow)
        _, u, v = by[rid].fields
        emax, el2 = rel_errors(u, v, ur, vr)
        acc.append({"request": rid, "kind": kind, "nx": q.nx, "ny": q.ny, "steps": q.steps,
                    "err_max": emax, "err_L2": el2})
    out["accuracy"] = {"reference": "each sampled request run alone in FP64 storage on the GPU",
                       "requests": acc, "err_max": max(a["err_max"] for a in acc),
                       "err_L2": max(a["err_L2"] for a in acc)}
    out.update({"storage": storage, "offered_rate_per_s": rate, "arrival_window_s": duration,
                "peak_active": sched.peak_active, "peak_bytes": sched.peak_used,
                "quanta": sched.quanta})
    return out


def run_extra(steps):
    """Companion measurements: the same lattice in FP16 and FP64 storage,
    a force-driven channel of the same size (FP32, whole-row walls), the
    batched workload (FP32 and FP16), the serving stream (FP16 and FP32), the
    double-shear-layer stability study, the Taylor-Green convergence study
    and the Poiseuille slip study."""
    out = {}
    for storage in ("f16", "f64"):
        lat = tg_lattice(4096, storage)
        shape = headline_shape(lat, 4096, storage)[0]
        lat.set_tuning(*shape)
        ms = time_steps(lat, steps, 20)
        lat.close()
        mlups = 4096 * 4096 / (ms * 1e-3) / 1e6
        out["tg4096_" + storage] = {
            "MLUPS": round(mlups, 1), "ms_per_step": round(ms, 5), "launch_shape": list(shape),
            "hbm_frac": round(mlups * 1e6 * BYTES_PER_LU[storage] / (HBM_PEAK_GBS * 1e9), 4)}
        log("extra %s: %.1f MLUPS" % (storage, mlups))
    out["channel4096_f32"] = run_channel(steps)
    log("extra channel: %s" % out["channel4096_f32"])
    out["batch256_f32"] = run_batch()
    log("extra batch: %s" % out["batch256_f32"])
    # the same batch in FP16 storage (set against single-instance FP64 above)
    out["batch256_f16"] = run_batch(storage="f16")
    log("extra batch f16: %s" % out["batch256_f16"])
    for storage in ("f16", "f32"):
        out["serving_" + storage] = run_serving(storage)
        log("extra serving %s: %s" % (storage, out["serving_" + storage]))
    out["dsl1024_error_curve"] = run_dsl_curve()
    out["dsl_critical_mach_f64"] = run_stability()
    log("extra stability study: %s" % out["dsl_critical_mach_f64"])
    out["tg_convergence_f64"] = run_convergence()
    log("extra convergence study: %s" % out["tg_convergence_f64"])
    out["poiseuille_slip_f64"] = run_poiseuille()
    log("extra Poiseuille slip study: %s" % out["poiseuille_slip_f64"])
    return out


def run_channel(steps, n=4096):
    """The force-driven channel (whole-row walls) at the benchmark's size in
    FP32, the library's default launch shape; its error against the same
    channel run alone in FP64 storage after the same steps."""
    lat = channel_lattice(n, "f32")
    ms = time_steps(lat, steps, 20)
    shape = list(lat.tuning())
    total = lat.state()[1]
    u, v = velocity(lat)
    lat.close()
    tau1, tau2, g, mask, fields = channel_problem(n)
    ur, vr = fp64_alone(n, n, tau1, tau2, total, fields, g=(g, 0.0), mask=mask)
    emax, el2 = rel_errors(u, v, ur, vr)
    mlups = n * n / (ms * 1e-3) / 1e6
    return {"MLUPS": round(mlups, 1), "ms_per_step": round(ms, 5), "launch_shape": shape,
            "hbm_frac": round(mlups * 1e6 * BYTES_PER_LU["f32"] / (HBM_PEAK_GBS * 1e9), 4),
            "steps": total, "err_max": emax, "err_L2": el2,
            "reference": "the same channel run alone in FP64 storage on the GPU"}


def run_dsl_curve(n=1024, u0=0.04, checkpoints=(1000, 2000, 5000, 10000, 20000)):
    """The double shear layer at its benchmark size (Sec. III.A set-up:
    1024^2, U0 = 0.04, kappa = 80, delta = 0.05, 1/tau_s2 = 1.6) to 20000
    steps at Re = 1e4 and 1e7: FP32 and FP16 (f - w) storage against the FP64
    run of the same set-up on the GPU (which the parity tests hold to the
    FP64 oracle within 1.3e-13 over the first 1000 steps), error against step."""
    from paper_2312_10318_amd import inputs, params
    from paper_2312_10318_amd.lattice import Lattice
    out = {}
    rho, ux, uy = inputs.double_shear_layer(n, u0)
    for re in (1e4, 1e7):
        tau1 = params.tau_from_re(u0, n, re)
        lats = {st: Lattice(n, n, tau1, 1 / 1.6, storage=st).init_equilibrium(rho, ux, uy)
                for st in ("f64", "f32", "f16")}
        curve = {"f32": [], "f16": []}
        done = 0
        for c in checkpoints:
            for lat in lats.values():
                lat.step(c - done)
            done = c
            ur, vr = velocity(lats["f64"])
            for st in ("f32", "f16"):
                if lats[st].diagnostics()["n_diverged"] > 0:
                    curve[st].append({"step": c, "diverged": True})
                    continue
                u, v = velocity(lats[st])
                emax, el2 = rel_errors(u, v, ur, vr)
                curve[st].append({"step": c, "err_max": emax, "err_L2": el2})
        for lat in lats.values():
            lat.close()
        out["Re=%g" % re] = {"tau1": tau1, **curve}
        log("extra DSL %d^2 Re=%g error curve: %s" % (n, re, curve))
    out["reference"] = "FP64 storage on the GPU, same set-up"
    return out


def run_stability():
    """The double-shear-layer critical-Mach study of Sec. III.A (128^2, six
    Reynolds numbers x twenty 1/tau_s2 values + RLB, bisection to dMa = 0.01,
    stable up to t/t_c = 2) as batched rounds on the GPU, FP64."""
    from paper_2312_10318_amd import stability
    res = stability.critical_mach([5e3, 1e4, 5e4, 1e5, 1e6, 1e7],
                                  [round(0.1 * k, 1) for k in range(1, 21)], storage="f64")
    return {"cases": len(res["cases"]), "rounds": res["rounds"], "seconds": res["seconds"],
            "per_re": {"%g" % k: v for k, v in stability.summary(res).items()}}


def run_poiseuille():
    """Poiseuille slip against Lambda_s, the set-up of Sec. III.C (4 x 32,
    u_c = 0.1, Re = 1): steady relative L2 error per Lambda_s and for RLB."""
    from paper_2312_10318_amd import poiseuille
    res = poiseuille.sweep()
    return {"l2": {("RLB" if r["model"] == "RLB" else "%.5g" % r["lambda"]): float("%.4e" % r["l2"])
                   for r in res},
            "seconds": res[-1]["seconds"]}


def run_convergence():
    """Taylor-Green grid convergence of Sec. III.B (N = 32 ... 512, FP64):
    L2 error at t_d and the orders, TRT-RLB and RLB."""
    from paper_2312_10318_amd import convergence
    out = {}
    for rlb in (False, True):
        r = convergence.run(convergence.PAPER_NS, "f64", rlb=rlb)
        out[r["model"]] = {"l2": [float("%.4e" % e) for e in r["l2"]],
                           "order": [round(o, 3) for o in r["order"]], "seconds": r["seconds"]}
    out["n"] = list(convergence.PAPER_NS)
    return out


def creeping_lattice(storage, tuning=None):
    """The creeping-flow geometry of Sec. III.D (Table 1, Re = 1e-3): 1050^2,
    a 21 x 21 square cylinder, inflow wall and pressure outlet -- the sweep
    with the link map."""
    from paper_2312_10318_amd import creeping
    from paper_2312_10318_amd.lattice import Lattice
    c = creeping.Case(1e-3)
    mask = creeping.cylinder_mask(c.n, c.D)
    lat = Lattice(c.n, c.n, c.tau1, c.tau2, mask=mask, storage=storage,
                  inflow=(c.u0, 1.0, 1.0))
    if tuning:
        lat.set_tuning(*tuning)
    lat.init_equilibrium(*creeping.initial_fields(c, mask))
    return lat


def channel_lattice(n, storage, tuning=None):
    """A force-driven channel (the set-up of Sec. III.C) of n x n nodes:
    walls on the first and last rows, g for a centre-line velocity of 0.01,
    Lambda = 3/16, started from its steady parabola -- the multi-step passes
    over whole-row walls."""
    from paper_2312_10318_amd.lattice import Lattice
    tau1, tau2, g, mask, fields = channel_problem(n)
    lat = Lattice(n, n, tau1, tau2, g=(g, 0.0), mask=mask, storage=storage)
    if tuning:
        lat.set_tuning(*tuning)
    lat.init_equilibrium(*fields)
    return lat


def channel_problem(n, uc=0.01):
    """(tau1, tau2, g, mask, (rho, ux, uy)) of the n x n force-driven
    channel: fluid rows 1 ... n - 2 between half-way walls, the steady
    parabola of centre-line velocity uc as the initial velocity."""
    import numpy as np
    from paper_2312_10318_amd import inputs, params
    tau1 = 0.8
    tau2 = params.tau2_from_magic(tau1, 3 / 16)
    g = 8 * params.nu_from_tau(tau1) * uc / (n - 2) ** 2
    mask = inputs.channel_mask(n, n - 2)
    rho, _, uy = inputs.rest_state(n, n)
    y = (np.arange(n, dtype=np.float64) - (n - 1) / 2) / ((n - 2) / 2)
    ux = np.where(mask != 0, 0.0, (uc * (1.0 - y * y))[:, None] * np.ones((1, n)))
    return tau1, tau2, g, mask, (rho, ux, uy)


def profile_run(n, storage, steps, warmup, tuning, workload="tg"):
    """Kernels for rocprofv3: `steps` sweeps of the benchmark lattice (or of
    the creeping-flow lattice), then a plain copy of 1 GiB (known bytes) to
    scale the HBM counters."""
    import torch
    nodes = None
    launch = None
    if workload == "batch":
        # the benchmark's 256-member batch in the library's default batch shape
        from paper_2312_10318_amd import inputs
        from paper_2312_10318_amd.lattice import Batch, Lattice
        members = inputs.batch_workload(256, seed=0)
        lats = []
        for k, m in enumerate(members):
            rho, ux, uy = inputs.member_fields(m, seed=k)
            lats.append(Lattice(m.n, m.n, m.tau1, m.tau2, storage=storage)
                        .init_equilibrium(rho, ux, uy))
        b = Batch(lats)
        if tuning:
            b.set_tuning(*tuning)
        b.step(warmup + steps)
        torch.cuda.synchronize()
        b.close()
        for l in lats:
            l.close()
        nodes = sum(m.n * m.n for m in members)
    else:
        if workload == "creeping":
            lat = creeping_lattice(storage, tuning)
            n = lat.nx
        elif workload == "channel":
            lat = channel_lattice(n, storage, tuning)
        else:
            lat = tg_lattice(n, storage, tuning=tuning)
            if tuning is None and workload == "tg":
                # the shape the benchmark runs in (bench.py --tune-only beforehand
                # puts it in the tuner's cache, so no tuning runs under the profiler)
                lat.set_tuning(*headline_shape(lat, n, storage)[0])
        if workload != "stream":   # the probe keeps the one-step sweep's tiling
            launch = list(lat.tuning())
        if workload == "stream":
            # the sweep's access pattern without its arithmetic
            lat.pattern_probe(warmup + steps)
        else:
            lat.step(warmup + steps)
        torch.cuda.synchronize()
        lat.close()
    src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"profile": "done", "sweeps": warmup + steps, "copy_bytes": 1 << 30,
                      "copies": 3, "storage": storage, "n": n, "workload": workload,
                      "nodes": nodes if nodes is not None else n * n,
                      "launch": launch, "source_hash": sweep_source_hash()}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "f64"])
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tune-only", action="store_true",
                    help="run (or read from the tuner's cache) the launch-shape choice of "
                         "the --storage/--n benchmark lattice, print it and exit (so that "
                         "later profiled runs read it from the cache)")
    ap.add_argument("--no-tune", action="store_true",
                    help="time the library's default launch shape instead of the "
                         "autotuner's pick")
    ap.add_argument("--tuning", default="",
                    help="rows_per_wave,waves_per_block,xcd_remap[,cols_per_lane"
                         "[,graph_steps[,steps_per_sweep[,prefetch_rows]]]]")
    ap.add_argument("--profile", action="store_true",
                    help="profiler driver: run warmup + steps sweeps untimed, then a plain "
                         "1 GiB device copy (the counter calibration kernel), and exit")
    ap.add_argument("--workload", default="tg",
                    choices=["tg", "creeping", "channel", "batch", "stream"],
                    help="lattice of --profile: the Taylor-Green benchmark (--n), the "
                         "creeping-flow cylinder of Table 1 (1050^2, link map), a "
                         "force-driven channel (--n, whole-row walls), the "
                         "256-member batch, or the access-pattern probe on the benchmark "
                         "lattice (the sweep's loads and stores without its arithmetic)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: the TRT-RLB sweep is built and measured on a "
              "single MI355X; multi-GPU slab decomposition is a design note, not a run.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)

    n, storage = args.n, args.storage
    tuning = tuple(int(v) for v in args.tuning.split(",")) if args.tuning else None
    if args.tune_only:
        lat = tg_lattice(n, storage)
        shape, rec = headline_shape(lat, n, storage)
        lat.close()
        print(json.dumps({"tune": {"n": n, "storage": storage, "shape": list(shape),
                                   "ms": rec.get("ms")}}), flush=True)
        return
    if args.profile:
        profile_run(n, storage, args.steps, args.warmup, tuning, args.workload)
        return
    log("bench: TG %dx%d %s, warmup %d, steps %d" % (n, n, storage, args.warmup, args.steps))
    lat = tg_lattice(n, storage, tuning=tuning)
    tuned = None
    if tuning is None and not args.no_tune:
        shape, tuned = headline_shape(lat, n, storage)
        lat.set_tuning(*shape)
        log("bench: launch shape %s chosen by the autotuner (%.4f ms per step; the default "
            "shape %s: %.4f)" % (shape, tuned["ms"], tuned["default"], tuned["default_ms"]))
    ms = time_steps(lat, args.steps, args.warmup)
    stable = lat.check()
    rows, waves, remap, cols, graph_steps, steps_per_sweep, prefetch = lat.tuning()
    probe_ms = None
    if cols == 2 and n % 128 == 0:
        # the same launch shape moving the same bytes without the arithmetic
        # (scrambles the lattice, which is not used afterwards)
        probe_ms = time_probe(lat, max(10, args.steps))
    lat.close()
    lups = n * n / (ms * 1e-3)
    mlups = lups / 1e6
    # one launch advances the lattice by steps_per_sweep steps: its
    # algorithmic bytes are those of that many lattice updates, and its
    # duration that many steps' time
    # (with a step count that is not a multiple of steps_per_sweep the timed
    # region ends on a launch of fewer steps, counted as that fraction of a
    # launch)
    bytes_step = BYTES_PER_LU[storage] * n * n
    bytes_launch = bytes_step * steps_per_sweep
    launch_ms = ms * steps_per_sweep
    achieved = bytes_launch / (launch_ms * 1e-3) / 1e9
    traffic = traffic_from_counters(n, storage)
    log("bench: %.4f ms/step, %.1f MLUPS, %.1f GB/s algorithmic (%.1f%% of peak)" %
        (ms, mlups, achieved, 100 * achieved / HBM_PEAK_GBS))

    rec = {
        "metric": "D2Q9 TRT-RLB MLUPS (% HBM roofline)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": storage,
        "data": "synthetic",
        "config": {"workload": "taylor_green_%dx%d" % (n, n), "storage": storage + "_shifted"
                   if storage != "f64" else "f64", "tau_s": 0.6, "tau_s2": 3.0, "u0": 0.01,
                   "nodes": n * n, "launch": {"rows_per_wave": rows, "waves_per_block": waves,
                                              "xcd_remap": remap, "cols_per_lane": cols,
                                              "graph_steps": graph_steps,
                                              "steps_per_sweep": steps_per_sweep,
                                              "prefetch_rows": prefetch},
                   "launch_chosen_by": ("autotuner" if tuned else
                                        "--tuning" if tuning else "library default"),
                   "autotune": ({"candidates": tuned.get("candidates"),
                                 "tuned_ms_per_step": round(tuned["ms"], 5),
                                 "default_shape": tuned.get("default"),
                                 "default_ms_per_step": round(tuned["default_ms"], 5)}
                                if tuned and "default_ms" in tuned else None),
                   "stable": bool(stable)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "bytes_per_lu": BYTES_PER_LU[storage],
                     "updates_per_launch": steps_per_sweep,
                     "kernel": ("sweep_tb3_kernel<%s>" if steps_per_sweep == 3 else
                                "sweep_tb2_kernel<%s>" if steps_per_sweep == 2 else
                                "sweep_pair_kernel<%s>" if cols == 2 else
                                "sweep_single_kernel<%s,nomask>") % storage,
                     "source_hash": sweep_source_hash(),
                     # live average duration per launch (HIP events on the
                     # sweep's stream) next to the traced one of the committed
                     # rocprofv3 summary (traced dispatches run slightly slower)
                     "avg_duration_us": round(launch_ms * 1e3, 2),
                     "profiled_avg_duration_us":
                         (profile_record(n, storage) or {}).get("avg_duration_us")},
    }
    prof = profile_record(n, storage) or {}
    if traffic:
        # what HBM actually carries per launch (rocprofv3 counters) over the
        # live launch time: with two steps per launch well below the
        # B_LU x updates figure above, which can then exceed the peak
        tg = traffic / (launch_ms * 1e-3) / 1e9
        rec["roofline"]["traffic_GBps"] = round(tg, 1)
        rec["roofline"]["traffic_frac"] = round(tg / HBM_PEAK_GBS, 4)
    if "valu_busy_frac" in prof:
        rec["roofline"]["valu_busy_frac"] = prof["valu_busy_frac"]
    if probe_ms is not None:
        # the probe moves one step's bytes per launch
        probe_gbs = bytes_step / (probe_ms * 1e-3) / 1e9
        rec["roofline"]["access_pattern"] = {
            "kernel": "pattern_probe_kernel<%s>" % storage,
            "avg_duration_us": round(probe_ms * 1e3, 2),
            "achieved": round(probe_gbs, 1), "frac": round(probe_gbs / HBM_PEAK_GBS, 4),
            "sweep_over_pattern": round(achieved / probe_gbs, 4)}
        log("bench: access-pattern probe %.4f ms/launch, %.1f GB/s (%.1f%% of peak); the sweep "
            "reaches %.1f%% of it" % (probe_ms, probe_gbs, 100 * probe_gbs / HBM_PEAK_GBS,
                                      100 * achieved / probe_gbs))
    if not args.no_extra:
        rec["extra"] = run_extra(max(200, args.steps // 4))
    if not args.no_cpu:
        log("bench: timing the CPU oracle on a bounded sample")
        rec["cpu_baseline"], ref = cpu_baseline(n)
        # every storage of the benchmark lattice against that oracle state
        acc = accuracy_vs_oracle(n, ref)
        rec["accuracy"] = {"reference": acc["reference"], "steps": acc["steps"],
                           **acc[storage]}
        for st in ("f16", "f64"):
            key = "tg4096_" + st
            if n == 4096 and key in rec.get("extra", {}):
                rec["extra"][key]["accuracy"] = {"reference": acc["reference"],
                                                 "steps": acc["steps"], **acc[st]}
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
