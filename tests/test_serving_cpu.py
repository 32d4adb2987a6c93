"""Scheduler logic of the solve server, on the CPU with a test-double
executor that models only footprints and step counts (no device)."""
import math

import numpy as np
import pytest

from paper_2312_10318_amd.serving import Request, Scheduler, serving_workload, summarize


class FakeExecutor:
    """Records every step given to every handle; 100 bytes per node."""

    def __init__(self):
        self.stepped = {}
        self.log = []

    def footprint(self, req):
        return req.nx * req.ny * 100

    def start(self, req):
        h = {"rid": req.rid, "steps": 0}
        self.log.append(("start", req.rid))
        return h

    def step(self, handles, n):
        assert n >= 1
        self.log.append(("step", tuple(h["rid"] for h in handles), n))
        for h in handles:
            h["steps"] += n

    def change(self, h):
        """Scripted convergence: the change halves at every check."""
        h["checks"] = h.get("checks", 0) + 1
        self.log.append(("check", h["rid"], h["steps"]))
        return 0.5 ** h["checks"]

    def finish(self, h, keep_fields=False):
        self.stepped[h["rid"]] = h["steps"]
        self.log.append(("finish", h["rid"]))
        return {"n_diverged": 0.0}, (("fields", h["rid"]) if keep_fields else None)

    def close(self, h):
        pass


class Clock:
    """Deterministic clock: each call advances 1 ms."""

    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-3
        return self.t


def _req(rid, n, steps, arrival=0.0):
    return Request(rid, "taylor_green", n, n, 0.6, 3.0, steps, arrival=arrival)


def test_every_request_gets_exactly_its_steps():
    ex = FakeExecutor()
    s = Scheduler(ex, budget_bytes=10**9, quantum=64, clock=Clock())
    reqs = [_req(k, 32 + k, steps) for k, steps in enumerate([1, 63, 64, 65, 200, 7, 1000])]
    res = s.run(reqs)
    assert sorted(r.rid for r in res) == list(range(7))
    assert ex.stepped == {k: r.steps for k, r in enumerate(reqs)}
    # quanta never exceed the smallest remaining budget among the active set
    for entry in ex.log:
        if entry[0] == "step":
            assert entry[2] <= 64


def test_admission_respects_the_memory_budget_in_fifo_order():
    ex = FakeExecutor()
    budget = 3 * 64 * 64 * 100
    s = Scheduler(ex, budget_bytes=budget, quantum=10, clock=Clock())
    reqs = [_req(k, 64, 30) for k in range(7)]
    s.run(reqs)
    assert s.peak_used <= budget
    assert s.peak_active == 3
    starts = [e[1] for e in ex.log if e[0] == "start"]
    assert starts == list(range(7))


def test_slot_limit_and_oversized_request():
    ex = FakeExecutor()
    s = Scheduler(ex, budget_bytes=10**9, max_slots=2, quantum=5, clock=Clock())
    s.run([_req(k, 16, 12) for k in range(5)])
    assert s.peak_active == 2
    s2 = Scheduler(FakeExecutor(), budget_bytes=1000, clock=Clock())
    with pytest.raises(ValueError):
        s2.submit(_req(0, 64, 10))


def test_late_arrivals_join_running_work():
    """Continuous batching: a request arriving while a long one runs is
    admitted and stepped together with it, and can finish first."""
    ex = FakeExecutor()
    clock = Clock()
    s = Scheduler(ex, budget_bytes=10**9, quantum=10, clock=clock)
    long_job = _req(0, 64, 500, arrival=0.0)
    short_job = _req(1, 32, 20, arrival=0.02)
    res = s.run([long_job, short_job])
    by = {r.rid: r for r in res}
    assert by[1].finished < by[0].finished
    assert by[1].admitted < by[0].finished
    shared = [e for e in ex.log if e[0] == "step" and set(e[1]) == {0, 1}]
    assert shared, "the two requests never shared a launch"
    st = summarize(res, wall=1.0)
    assert st["solves"] == 2 and st["p99_latency_s"] >= st["p50_latency_s"]


def test_serving_workload_mix_and_parameters():
    reqs = serving_workload(rate=200.0, duration=1.0, seed=0)
    assert 150 <= len(reqs) <= 250
    kinds = {r.kind for r in reqs}
    assert kinds == {"cylinder", "poiseuille", "taylor_green"}
    times = [r.arrival for r in reqs]
    assert times == sorted(times) and 0 < times[0] and times[-1] <= 1.0
    for r in reqs:
        assert r.tau1 > 0.5 and r.tau2 >= 0.5
        if r.kind == "cylinder":
            assert (r.nx, r.ny) == (400, 200) and r.mask is not None
            assert r.mask[100, 200] == 1 and r.mask[100, 0] == 0
            # the paper's set-up: no walls and no body force; inflow u_c =
            # c_s Ma through the left wall, outlet at rho = 1
            assert r.mask.sum() == 400 and not r.mask[0].any() and r.g == (0.0, 0.0)
            u = r.inflow[0]
            assert r.inflow[1:] == (1.0, 1.0) and u == r.meta["u_in"]
            assert abs(u - math.sqrt(1 / 3) * math.sqrt(0.1 * r.meta["re"])) < 1e-15
            rho, ux, uy = r.fields()
            assert np.all(rho == 1) and np.all(ux[r.mask == 0] == u) and np.all(ux[r.mask != 0] == 0)
            # T = Ma^2 / Re = 0.1 and Lambda_s = 3/16 (Sec. III.D set-up)
            assert abs((r.tau1 - 0.5) * (r.tau2 - 0.5) - 3 / 16) < 1e-9
        else:
            assert 64 <= r.nx <= 2048 and r.nx == r.ny


def test_requests_with_a_tolerance_end_at_their_first_converged_check():
    ex = FakeExecutor()
    s = Scheduler(ex, budget_bytes=10**9, quantum=64, clock=Clock())
    reqs = [_req(0, 32, 10_000), _req(1, 40, 10_000), _req(2, 48, 500), _req(3, 56, 777)]
    reqs[0].tol, reqs[0].check = 0.1, 100      # 0.5**4 < 0.1: converges at the 4th check
    reqs[1].tol, reqs[1].check = 0.01, 37      # 0.5**7 < 0.01: 7th check
    reqs[2].tol, reqs[2].check = 1e-9, 50      # never: ends on its budget, not converged
    res = {r.rid: r for r in s.run(reqs)}
    assert res[0].converged and res[0].steps == 400 and ex.stepped[0] == 400
    assert res[1].converged and res[1].steps == 7 * 37 and ex.stepped[1] == 7 * 37
    assert res[2].converged is False and res[2].steps == 500
    assert res[3].converged is None and res[3].steps == 777
    # every check happened exactly on the request's own check grid
    for e in ex.log:
        if e[0] == "check":
            rid, at = e[1], e[2]
            assert at % reqs[rid].check == 0
    st = summarize(list(res.values()), wall=1.0)
    assert st["converged"] == 2 and st["with_tolerance"] == 3


def test_fields_are_kept_for_all_none_or_the_listed_requests():
    for keep, want in ((True, set(range(6))), (False, set()), ({1, 4}, {1, 4})):
        s = Scheduler(FakeExecutor(), budget_bytes=10**9, quantum=16, keep_fields=keep,
                      clock=Clock())
        res = s.run([_req(k, 32, 20 + k) for k in range(6)])
        assert {r.rid for r in res if r.fields is not None} == want
        assert all(r.fields == ("fields", r.rid) for r in res if r.fields is not None)
