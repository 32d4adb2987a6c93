"""Continuous-batching solve server for parameter-sweep TRT-RLB requests.

Requests (a lattice, its relaxation times, force, optional obstacle mask,
initial fields and a step budget, optionally a convergence tolerance)
arrive over time.  The scheduler admits a
request as soon as a slot is free and its device footprint fits the memory
budget, keeps every admitted lattice resident on the device, and advances
all active lattices together in quanta of steps: one batched launch per step
covers every active lattice (lattices with and without obstacles go in two
launches).  A request that arrives while others run joins at the next
quantum boundary; a finished request leaves at the quantum boundary where
its budget is used up, its slot and memory are reused at once.  Latency is
measured from arrival to the result being on the host.

A request with a tolerance ends early once it has converged: at check
points every `check` steps of its own clock, the relative L2 change of its
velocity field since the previous check point (computed on the device) is
compared with the tolerance (the steady-state test of Sec. III).

The scheduler talks to an executor; ``GpuExecutor`` runs the HIP library.
Quanta never cross a request's budget or its next check point, so each
result is exactly the result of running that request alone (the sweep's
arithmetic per node does not depend on which other lattices share the
launch).
"""
from __future__ import annotations

import collections
import dataclasses
import heapq
import math
import time
from typing import Callable, Optional

import numpy as np

from . import inputs, params


@dataclasses.dataclass
class Request:
    rid: int
    kind: str                 # "cylinder", "poiseuille" or "taylor_green"
    nx: int
    ny: int
    tau1: float
    tau2: float
    steps: int
    g: tuple = (0.0, 0.0)
    mask: Optional[np.ndarray] = None
    # (rho, ux, uy), float64 [ny, nx]: fields(device=None) may return numpy
    # arrays, or tensors on the device the GPU executor passes
    fields: Optional[Callable[..., tuple]] = None
    arrival: float = 0.0      # seconds since the start of the run
    meta: dict = dataclasses.field(default_factory=dict)
    tol: Optional[float] = None   # end when the velocity change per check is below tol
    check: int = 1000             # steps between convergence checks (with tol)
    inflow: Optional[tuple] = None  # (u_in, rho_in, rho_out): open x boundaries


@dataclasses.dataclass
class Result:
    rid: int
    kind: str
    arrival: float
    admitted: float
    finished: float
    steps: int                      # steps taken
    diverged: bool
    diagnostics: dict
    nodes: int = 0
    fields: Optional[tuple] = None  # (rho, ux, uy) numpy, when kept
    converged: Optional[bool] = None  # requests with a tolerance only
    change: Optional[float] = None    # last relative L2 velocity change

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Scheduler:
    """Admission by memory budget and slot count; FIFO order; quanta of at
    most `quantum` steps that never cross a request's step budget or its
    next convergence check point."""

    def __init__(self, executor, budget_bytes: int, max_slots: int = 4096,
                 quantum: int = 100, keep_fields=False, clock=time.perf_counter):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_slots = max_slots
        self.quantum = quantum
        # True / False, or the ids of the requests whose final fields are kept
        self.keep_fields = keep_fields
        self.clock = clock
        self.queue = collections.deque()
        # rid -> [request, handle, remaining, admitted_at, footprint, to_check, change]
        self.active = {}
        self.used = 0
        self.results = []
        self.draining = []        # results on their way to the host (asynchronous executors)
        self.t0 = None
        self.peak_used = 0
        self.peak_active = 0
        self.quanta = 0

    def now(self) -> float:
        return self.clock() - self.t0

    def submit(self, req: Request):
        fp = self.ex.footprint(req)
        if fp > self.budget:
            raise ValueError("request %d needs %d bytes, more than the whole budget" %
                             (req.rid, fp))
        self.queue.append((req, fp))

    def _admit(self):
        while self.queue and len(self.active) < self.max_slots:
            req, fp = self.queue[0]
            if self.used + fp > self.budget:
                break  # FIFO: the head waits for memory, later requests wait behind it
            self.queue.popleft()
            handle = self.ex.start(req)
            self.used += fp
            to_check = req.check if req.tol is not None else None
            self.active[req.rid] = [req, handle, req.steps, self.now(), fp, to_check, None]
        self.peak_used = max(self.peak_used, self.used)
        self.peak_active = max(self.peak_active, len(self.active))

    def _retire(self, rid, converged=None):
        req, handle, remaining, admitted, fp, _, change = self.active.pop(rid)
        if req.tol is not None and converged is None:
            converged = False
        info = (req, admitted, req.steps - remaining, converged, change)
        keep = (self.keep_fields if isinstance(self.keep_fields, bool)
                else rid in self.keep_fields)
        if hasattr(self.ex, "finish_async"):
            # the result is copied to the host behind the work already queued;
            # the slot and the memory are free at once (the device reuses the
            # lattice's memory only after the copy, in stream order)
            ticket = self.ex.finish_async(handle, keep_fields=keep)
            self.ex.close(handle)
            self.used -= fp
            self.draining.append((info, ticket))
            return
        diag, fields = self.ex.finish(handle, keep_fields=keep)
        self.ex.close(handle)
        self.used -= fp
        self._record(info, diag, fields)

    def _record(self, info, diag, fields):
        req, admitted, steps, converged, change = info
        diverged = bool(diag.get("n_diverged", 0) > 0)
        self.results.append(Result(req.rid, req.kind, req.arrival, admitted, self.now(), steps,
                                   diverged, diag, req.nx * req.ny, fields, converged, change))

    def _collect(self, wait: bool = False):
        """Record the results that have reached the host."""
        pending = []
        for info, ticket in self.draining:
            if wait or self.ex.ready(ticket):
                diag, fields = self.ex.result(ticket)
                self._record(info, diag, fields)
            else:
                pending.append((info, ticket))
        self.draining = pending

    def step_quantum(self):
        """Advance every active request by one quantum (host-synchronous)."""
        if not self.active:
            return
        q = self.quantum
        for a in self.active.values():
            q = min(q, a[2] if a[5] is None else min(a[2], a[5]))
        self.ex.step([a[1] for a in self.active.values()], q)
        self.quanta += 1
        done = []
        for rid, a in self.active.items():
            a[2] -= q
            converged = None
            if a[5] is not None:
                a[5] -= q
                if a[5] == 0:
                    a[6] = self.ex.change(a[1])
                    a[5] = a[0].check
                    if a[6] < a[0].tol:
                        converged = True
            if converged or a[2] <= 0:
                done.append((rid, converged))
        for rid, converged in done:
            self._retire(rid, converged)

    def run(self, arrivals, idle_sleep: float = 2e-4):
        """Serve a list of requests whose `arrival` times are seconds from
        now; returns the results in completion order."""
        pending = [(r.arrival, r.rid, r) for r in arrivals]
        heapq.heapify(pending)
        self.t0 = self.clock()
        while pending or self.queue or self.active or self.draining:
            t = self.now()
            while pending and pending[0][0] <= t:
                _, _, r = heapq.heappop(pending)
                self.submit(r)
            self._admit()
            if self.active:
                self.step_quantum()
                self._collect()
            elif self.draining:
                self._collect(wait=not pending)
            elif pending:
                wait = pending[0][0] - self.now()
                if wait > 0:
                    time.sleep(min(wait, idle_sleep * 50))
            elif self.queue:
                raise RuntimeError("queued request cannot be admitted (budget or slots)")
        return self.results


def summarize(results, wall: float) -> dict:
    lat = np.array([r.latency for r in results]) if results else np.zeros(1)
    lups = sum(r.nodes * r.steps for r in results)
    with_tol = [r for r in results if r.converged is not None]
    out = {"solves": len(results), "wall_s": round(wall, 3),
           "solves_per_s": round(len(results) / wall, 2) if wall > 0 else None,
           "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
           "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
           "mean_latency_s": round(float(np.mean(lat)), 4),
           "diverged": int(sum(r.diverged for r in results))}
    if lups:
        out["aggregate_MLUPS"] = round(lups / wall / 1e6, 1)
    if with_tol:
        out["converged"] = int(sum(bool(r.converged) for r in with_tol))
        out["with_tolerance"] = len(with_tol)
    return out


class GpuExecutor:
    """Runs requests on the GPU through the library (Lattice / Batch).

    Active lattices without obstacles and with obstacles form two batches
    (two launches per step), kept across quanta and updated in place when
    their membership changes.  Quanta are enqueued without waiting for the
    device: at most `run_ahead` quanta are in flight, so the host admits and
    prepares requests while the GPU steps.  Finished lattices hand their
    buffers back at once; their handles are destroyed in groups (a destroy
    waits for the device)."""

    def __init__(self, storage: str = "f32", stream=None, run_ahead: int = 2,
                 destroy_every: int = 128):
        self.storage = storage
        self.stream = stream
        self.run_ahead = run_ahead
        self.destroy_every = destroy_every
        self._batches = [None, None]   # open, walled
        self._members = [[], []]
        self._events = collections.deque()
        self._graveyard = []

    def footprint(self, req: Request) -> int:
        from .lattice import footprint_bytes
        return footprint_bytes(req.nx, req.ny, self.storage,
                               req.mask is not None or req.inflow is not None)

    def start(self, req: Request):
        from .lattice import Lattice
        lat = Lattice(req.nx, req.ny, req.tau1, req.tau2, g=req.g, mask=req.mask,
                      storage=self.storage, stream=self.stream, inflow=req.inflow)
        if req.fields:
            rho, ux, uy = req.fields(device=lat.device)
        else:
            rho, ux, uy = inputs.rest_state(req.ny, req.nx, device=lat.device)
        lat.init_equilibrium(rho, ux, uy, sync=False)
        lat._prev_u = None
        if req.tol is not None:
            import torch
            z = torch.zeros((req.ny, req.nx), dtype=torch.float64, device=lat.device)
            lat._prev_u = (z, z.clone())
            lat.velocity_change(lat._prev_u)   # the initial velocity
        return lat

    def change(self, lat) -> float:
        """Relative L2 change of the velocity since the previous check."""
        _, s2, n2, _ = lat.velocity_change(lat._prev_u)
        return math.sqrt(s2 / n2) if n2 > 0 else math.inf

    def step(self, handles, nsteps: int):
        import torch

        from .lattice import Batch
        # lattices with a link map (masks, open boundaries) batch apart
        linked = [h.mask is not None or h.inflow is not None for h in handles]
        groups = ([h for h, k in zip(handles, linked) if not k],
                  [h for h, k in zip(handles, linked) if k])
        for g in (0, 1):
            members = groups[g]
            if [id(l) for l in members] != [id(l) for l in self._members[g]]:
                if not members:
                    if self._batches[g] is not None:
                        self._batches[g].close()
                        self._batches[g] = None
                elif self._batches[g] is None:
                    self._batches[g] = Batch(members)
                else:
                    self._batches[g].update(members)
                self._members[g] = list(members)
        self._flush_graveyard()
        for g in (0, 1):
            if self._batches[g] is not None:
                self._batches[g].step(nsteps)
        ev = torch.cuda.Event()
        ev.record(handles[0].stream)
        self._events.append(ev)
        while len(self._events) > self.run_ahead:
            self._events.popleft().synchronize()

    def finish(self, lat, keep_fields: bool = False):
        diag = lat.diagnostics()
        fields = tuple(t.cpu().numpy() for t in lat.macros()) if keep_fields else None
        return diag, fields

    def finish_async(self, lat, keep_fields: bool = False):
        """Enqueue the result's extraction (diagnostics, optionally the fields)
        and its copy to pinned host memory; returns a ticket for ready() /
        result()."""
        import torch

        from . import capi
        from .lattice import DIAG_NAMES
        dev = torch.empty(capi.TRT_NDIAG, dtype=torch.float64, device=lat.device)
        capi.trt_diagnostics(lat.handle, dev.data_ptr())
        host = [torch.empty(capi.TRT_NDIAG, dtype=torch.float64, pin_memory=True)]
        srcs = [dev]
        if keep_fields:
            out = torch.empty((3, lat.ny, lat.nx), dtype=torch.float64, device=lat.device)
            n = lat.nx * lat.ny * 8
            capi.trt_macros(lat.handle, out.data_ptr(), out.data_ptr() + n, out.data_ptr() + 2 * n)
            for f in out:
                host.append(torch.empty(f.shape, dtype=f.dtype, pin_memory=True))
                srcs.append(f)
        with torch.cuda.stream(lat.stream):
            for h, d in zip(host, srcs):
                h.copy_(d, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(lat.stream)
        return (ev, host, srcs, DIAG_NAMES, keep_fields)

    def ready(self, ticket) -> bool:
        return ticket[0].query()

    def result(self, ticket):
        ev, host, _, names, keep = ticket
        ev.synchronize()
        diag = {k: float(v) for k, v in zip(names, host[0].numpy())}
        fields = tuple(h.numpy() for h in host[1:]) if keep else None
        return diag, fields

    def close(self, lat):
        lat.release()
        self._graveyard.append(lat)

    def _flush_graveyard(self, force: bool = False):
        # only lattices that no batch lists any more
        if not self._graveyard or (len(self._graveyard) < self.destroy_every and not force):
            return
        live = {id(l) for m in self._members for l in m}
        keep = []
        for lat in self._graveyard:
            if id(lat) in live:
                keep.append(lat)
            else:
                lat.close()
        self._graveyard = keep

    def shutdown(self):
        for g in (0, 1):
            if self._batches[g] is not None:
                self._batches[g].close()
                self._batches[g] = None
            self._members[g] = []
        self._events.clear()
        self._flush_graveyard(force=True)


MAX_G_TAU1 = 0.05


def _inflow_fields(mask: np.ndarray, u: float):
    """rho = 1 and the inflow velocity (u, 0) at every fluid node."""
    ny, nx = mask.shape
    return np.ones((ny, nx)), np.where(mask != 0, 0.0, u), np.zeros((ny, nx))


def serving_workload(rate: float = 200.0, duration: float = 2.0, seed: int = 0,
                     side_lo: int = 64, side_hi: int = 2048, steps=None):
    """Poisson stream of solves: one third creeping flow past a centred
    square cylinder (side 20) in a 400 x 200 domain with the set-up of
    Sec. III.D -- uniform inflow through a moving wall on the left, a
    pressure outlet on the right, periodic top and bottom; Re log-uniform in
    [1e-7, 1], T = Ma^2/Re = 0.1, Lambda_s = 3/16, starting from the inflow
    velocity at every fluid node -- one third force-driven Poiseuille
    channels and one third Taylor-Green vortices with sides log-uniform in
    [side_lo, side_hi].  Channel body forces are capped at g tau1 <=
    MAX_G_TAU1 (stability of very viscous forced runs)."""
    steps = steps or {"cylinder": 2000, "poiseuille": 1000, "taylor_green": 1000}
    rng = np.random.default_rng(seed)
    t, rid, out = 0.0, 0, []
    cyl_mask = inputs.square_obstacle_mask(400, 200, 20)
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        kind = ("cylinder", "poiseuille", "taylor_green")[rid % 3]
        if kind == "cylinder":
            re = math.exp(rng.uniform(math.log(1e-7), math.log(1.0)))
            ma = params.mach_from_T(0.1, re)
            u = params.u_from_mach(ma)
            tau1 = params.tau_from_re(u, 20.0, re)
            tau2 = params.tau2_from_magic(tau1, 3 / 16)
            req = Request(rid, kind, 400, 200, tau1, tau2, steps[kind], (0.0, 0.0), cyl_mask,
                          (lambda device=None, u=u: _inflow_fields(cyl_mask, u)), t,
                          {"re": re, "u_in": u}, inflow=(u, 1.0, 1.0))
        else:
            n = int(round(math.exp(rng.uniform(math.log(side_lo), math.log(side_hi)))))
            if kind == "poiseuille":
                tau1 = float(rng.uniform(0.51, 2.0))
                tau2 = params.tau2_from_magic(tau1, 3 / 16)
                nu = params.nu_from_tau(tau1)
                g = min(8 * nu * 0.01 / max(1, n - 2) ** 2, MAX_G_TAU1 / tau1)
                req = Request(rid, kind, n, n, tau1, tau2, steps[kind], (g, 0.0),
                              inputs.channel_mask(n, n - 2), None, t, {})
            else:
                tau1 = 0.6
                tau2 = params.tau2_from_magic(tau1, 0.25)
                seed_k = rid
                req = Request(rid, kind, n, n, tau1, tau2, steps[kind], (0.0, 0.0), None,
                              (lambda device=None, n=n, s=seed_k:
                               inputs.taylor_green(n, 0.01, seed=s, device=device)), t, {})
        req.meta["nodes"] = req.nx * req.ny
        out.append(req)
        rid += 1
    return out
