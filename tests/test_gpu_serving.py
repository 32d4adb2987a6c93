"""The solve server on the GPU: every request's result is bit-for-bit the
result of running it alone, whatever shared its launches."""
import numpy as np
import pytest

import oracle
from gpu_util import TOL, rel_errors, say
from paper_2312_10318_amd import inputs, params
from paper_2312_10318_amd.serving import Request, Scheduler, summarize

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_10318_amd import lattice
    return lattice


def _requests():
    rng = np.random.default_rng(3)
    reqs, t = [], 0.0
    mask = inputs.cylinder_channel_mask(160, 80, 12)
    obstacle = inputs.square_obstacle_mask(160, 80, 12)
    for k in range(14):
        t += float(rng.exponential(0.004))
        kind = ("cylinder", "poiseuille", "taylor_green")[k % 3]
        if kind == "cylinder" and k % 2:
            # the paper's set-up: inflow wall, pressure outlet, periodic in y
            tau1 = float(np.exp(rng.uniform(np.log(0.6), np.log(300.0))))
            tau2 = params.tau2_from_magic(tau1, 3 / 16)
            u = 1e-3
            r = Request(k, kind, 160, 80, tau1, tau2, 150 + 37 * k, (0.0, 0.0), obstacle,
                        (lambda device=None, u=u: (np.ones((80, 160)),
                                                   np.where(obstacle != 0, 0.0, u),
                                                   np.zeros((80, 160)))), t,
                        inflow=(u, 1.0, 1.0))
        elif kind == "cylinder":
            tau1 = float(np.exp(rng.uniform(np.log(0.6), np.log(300.0))))
            tau2 = params.tau2_from_magic(tau1, 3 / 16)
            g = 8 * params.nu_from_tau(tau1) * 1e-3 / 78.0 ** 2
            r = Request(k, kind, 160, 80, tau1, tau2, 150 + 37 * k, (g, 0.0), mask, None, t)
        elif kind == "poiseuille":
            n = int(rng.integers(40, 130))
            tau1 = float(rng.uniform(0.55, 1.5))
            tau2 = params.tau2_from_magic(tau1, 3 / 16)
            g = 8 * params.nu_from_tau(tau1) * 0.01 / (n - 2) ** 2
            r = Request(k, kind, n, n, tau1, tau2, 100 + 29 * k, (g, 0.0),
                        inputs.channel_mask(n, n - 2), None, t)
        else:
            n = int(rng.integers(64, 200))
            # served: fields built on the device; alone: numpy (the same bits)
            r = Request(k, kind, n, n, 0.6, 3.0, 120 + 31 * k, (0.0, 0.0), None,
                        (lambda device=None, n=n, s=k:
                         inputs.taylor_green(n, 0.01, seed=s, device=device)), t)
        reqs.append(r)
    return reqs


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_served_results_equal_results_alone(L, storage):
    from paper_2312_10318_amd.serving import GpuExecutor
    reqs = _requests()
    ex = GpuExecutor(storage)
    sched = Scheduler(ex, budget_bytes=2 << 30, quantum=40, keep_fields=True)
    res = sched.run(reqs)
    ex.shutdown()
    st = summarize(res, wall=max(r.finished for r in res))
    say("case: serving %s, %d requests, peak active %d, quanta %d: %s" %
        (storage, len(res), sched.peak_active, sched.quanta, st))
    assert len(res) == len(reqs) and sched.peak_active >= 3
    by = {r.rid: r for r in res}
    for q in reqs:
        lat = L.Lattice(q.nx, q.ny, q.tau1, q.tau2, g=q.g, mask=q.mask, storage=storage,
                        inflow=q.inflow)
        rho, ux, uy = q.fields() if q.fields else inputs.rest_state(q.ny, q.nx)
        lat.init_equilibrium(rho, ux, uy).step(q.steps)
        alone = [t.cpu().numpy() for t in lat.macros()]
        lat.close()
        got = by[q.rid].fields
        for a, b in zip(alone, got):
            assert np.array_equal(a, b), "request %d (%s) differs alone vs served" % (q.rid, q.kind)
        assert not by[q.rid].diverged
    if storage != "f32":
        return
    # the first served request of each kind against the FP64 oracle run of
    # the same problem (FP32 storage tolerance, relative max and L2)
    for kind in ("cylinder", "poiseuille", "taylor_green"):
        q = next(r for r in reqs if r.kind == kind)
        rho, ux, uy = q.fields() if q.fields else inputs.rest_state(q.ny, q.nx)
        f = oracle.run(oracle.init_equilibrium(rho, ux, uy, q.mask), q.steps, q.tau1, q.tau2,
                       q.g[0], q.g[1], q.mask)
        _, ur, vr = oracle.macros(f, q.g[0], q.g[1], q.mask)
        _, u, v = by[q.rid].fields
        emax, el2 = rel_errors(u, v, ur, vr)
        say("  served %s %dx%d, %d steps, vs oracle: rel max %.3e L2 %.3e"
            % (kind, q.nx, q.ny, q.steps, emax, el2))
        assert emax <= TOL["f32"] and el2 <= TOL["f32"]


def test_converged_requests_equal_results_alone(L):
    """Poiseuille channels served with a convergence tolerance end at a check
    point; the same request run alone with the same check points converges
    at the same step, with the same fields bit for bit."""
    import torch
    from paper_2312_10318_amd.serving import GpuExecutor
    reqs = []
    for k, n in enumerate((18, 26, 34)):
        tau1 = 0.8 + 0.2 * k
        tau2 = params.tau2_from_magic(tau1, 3 / 16)
        g = 8 * params.nu_from_tau(tau1) * 0.01 / (n - 2) ** 2
        r = Request(k, "poiseuille", 16, n, tau1, tau2, 60_000, (g, 0.0),
                    inputs.channel_mask(16, n - 2), None, 0.001 * k)
        r.tol, r.check = 1e-8, 250
        reqs.append(r)
    ex = GpuExecutor("f64")
    sched = Scheduler(ex, budget_bytes=1 << 30, quantum=100, keep_fields=True)
    res = {r.rid: r for r in sched.run(reqs)}
    ex.shutdown()
    for q in reqs:
        r = res[q.rid]
        say("case: served Poiseuille n=%d: converged=%s after %d steps (change %.2e)" %
            (q.ny, r.converged, r.steps, r.change))
        assert r.converged and r.steps % q.check == 0 and r.steps < q.steps
        lat = L.Lattice(q.nx, q.ny, q.tau1, q.tau2, g=q.g, mask=q.mask, storage="f64",
                        inflow=q.inflow)
        lat.init_equilibrium(*inputs.rest_state(q.ny, q.nx))
        prev = tuple(torch.zeros((q.ny, q.nx), dtype=torch.float64, device=lat.device)
                     for _ in range(2))
        lat.velocity_change(prev)
        steps = 0
        while True:
            lat.step(q.check)
            steps += q.check
            _, s2, n2, _ = lat.velocity_change(prev)
            if np.sqrt(s2 / n2) < q.tol:
                break
        assert steps == r.steps
        alone = [t.cpu().numpy() for t in lat.macros()]
        lat.close()
        for a, b in zip(alone, r.fields):
            assert np.array_equal(a, b)


def test_device_taylor_green_fields_equal_host_fields(L):
    """The serving workload builds Taylor-Green fields on the GPU; they are
    the host generator's values bit for bit."""
    import torch
    for n, kw in ((64, {}), (2048, {"seed": 7}), (129, {"nu": 0.02, "t": 50.0, "seed": 3})):
        host = inputs.taylor_green(n, 0.01, **kw)
        dev = inputs.taylor_green(n, 0.01, device="cuda", **kw)
        for h, d in zip(host, dev):
            assert d.is_cuda and d.dtype == torch.float64 and d.is_contiguous()
            assert np.array_equal(h, d.cpu().numpy())


@pytest.mark.parametrize("storage", ["f16", "f32"])
def test_full_serving_stream_sampled_requests_equal_results_alone(L, storage):
    """The benchmark's serving run as it is timed (Poisson arrivals at
    200 solves/s for 2 s, FP16 and FP32 storage, 64 GiB budget, quanta of 100 steps):
    a sample of requests of every kind, the largest Taylor-Green one
    included, gives bit for bit the result it gives alone."""
    from paper_2312_10318_amd import serving
    from paper_2312_10318_amd.serving import GpuExecutor
    reqs = serving.serving_workload(rate=200.0, duration=2.0, seed=0)
    pick = set()
    for kind in ("cylinder", "poiseuille", "taylor_green"):
        ks = [q for q in reqs if q.kind == kind]
        pick.update(q.rid for q in (ks[0], ks[len(ks) // 2], max(ks, key=lambda q: q.nx * q.ny)))
    ex = GpuExecutor(storage)
    sched = Scheduler(ex, budget_bytes=64 << 30, quantum=100, keep_fields=pick)
    res = sched.run(reqs)
    ex.shutdown()
    say("case: full serving stream %s, %d requests, peak active %d, %d sampled" %
        (storage, len(res), sched.peak_active, len(pick)))
    assert len(res) == len(reqs) and sched.peak_active >= 10
    by = {r.rid: r for r in res}
    for q in reqs:
        if q.rid not in pick:
            continue
        lat = L.Lattice(q.nx, q.ny, q.tau1, q.tau2, g=q.g, mask=q.mask, storage=storage,
                        inflow=q.inflow)
        rho, ux, uy = q.fields() if q.fields else inputs.rest_state(q.ny, q.nx)
        lat.init_equilibrium(rho, ux, uy).step(q.steps)
        alone = [t.cpu().numpy() for t in lat.macros()]
        lat.close()
        say("  request %d %s %dx%d, %d steps" % (q.rid, q.kind, q.nx, q.ny, q.steps))
        for a, b in zip(alone, by[q.rid].fields):
            assert np.array_equal(a, b), "request %d (%s) differs alone vs served" % (q.rid, q.kind)
        assert not by[q.rid].diverged
