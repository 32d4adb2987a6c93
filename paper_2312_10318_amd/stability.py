"""Critical Mach number of the double shear layer (Sec. III.A, Fig. 1) as a
batched search on the GPU.

The study: on an N x N periodic lattice (N = 128) the double shear layer
(kappa = 80, delta = 0.05, rho = 1) is run at Reynolds number Re and Mach
number Ma for t = 2 t_c, t_c = L / (c_s Ma); in lattice units the flow speed
is U0 = c_s Ma, tau_s1 follows from Re = U0 N / nu, and t_c = N / (c_s Ma)
steps.  The critical Mach number Ma_c is the largest Ma on the grid
dMa = 0.01 for which the run does not diverge, for each Re and each rate
1/tau_s2 (the RLB model is the case tau_s2 = tau_s1).

Search.  Stability is taken to be monotone in Ma (stable below Ma_c,
divergent above), so Ma_c is found by bisection on the grid: every round
runs the midpoint of every unresolved case, all cases of the round in one
batch on the GPU (one launch per step for all members).  A member leaves the
batch when it diverges (checked every `quantum` steps with the on-device
diagnostics) or when its own budget of steps is used up; the batch is
rebuilt only when its membership changes.  Divergence is the library's
criterion: a non-finite density or velocity, rho <= 0 or |u| >= 1 at any
fluid node.
"""
from __future__ import annotations

import dataclasses
import json
import math
import time
from typing import Optional

from . import inputs, params

C_S = math.sqrt(params.CS2)


@dataclasses.dataclass(frozen=True)
class Case:
    re: float
    inv_tau2: Optional[float]  # None: the RLB case tau_s2 = tau_s1

    @property
    def label(self) -> str:
        return "Re=%g %s" % (self.re, "RLB" if self.inv_tau2 is None
                             else "1/tau2=%g" % self.inv_tau2)


def run_parameters(n: int, re: float, ma: float, inv_tau2: Optional[float],
                   periods: float = 2.0):
    """(U0, tau_s1, tau_s2, steps) of one double-shear-layer run."""
    u0 = C_S * ma
    tau1 = params.tau_from_re(u0, n, re)
    tau2 = tau1 if inv_tau2 is None else 1.0 / inv_tau2
    steps = int(math.ceil(periods * n / u0))
    return u0, tau1, tau2, steps


def classify(runs, n: int = 128, storage: str = "f64", quantum: int = 256, periods: float = 2.0,
             log=None):
    """Run every (re, ma, inv_tau2) of `runs` on the GPU for t = periods * t_c
    and return one flag per run: True if it never diverged."""
    from .lattice import Batch, Lattice

    lats, remaining = [], []
    for re, ma, inv_tau2 in runs:
        u0, tau1, tau2, steps = run_parameters(n, re, ma, inv_tau2, periods)
        lat = Lattice(n, n, tau1, tau2, storage=storage)
        lat.init_equilibrium(*inputs.double_shear_layer(n, u0))
        lats.append(lat)
        remaining.append(steps)
    result = [None] * len(runs)
    alive = list(range(len(runs)))
    batch, members = None, None
    try:
        while alive:
            if members != alive:
                if batch is not None:
                    batch.close()
                members = list(alive)
                batch = Batch([lats[i] for i in members])
            q = min(quantum, min(remaining[i] for i in members))
            batch.step(q)
            diag = batch.diagnostics()
            for row, i in zip(diag, members):
                remaining[i] -= q
                if row[4] > 0:
                    result[i] = False
                elif remaining[i] == 0:
                    result[i] = True
            alive = [i for i in members if result[i] is None]
    finally:
        if batch is not None:
            batch.close()
        for lat in lats:
            lat.close()
    if log:
        log("classified %d runs" % len(runs))
    return result


def critical_mach(res, inv_tau2s, rlb: bool = True, n: int = 128, dma: float = 0.01,
                  ma_max: float = 1.0, storage: str = "f64", periods: float = 2.0, log=None):
    """Ma_c for every Re in `res` and every 1/tau_s2 in `inv_tau2s` (and the RLB
    case per Re when `rlb`).  Returns {"cases": [...], "rounds": k, "seconds": s}
    with one record per case: re, inv_tau2 (None for RLB), ma_c and the
    bracketing stable / divergent grid points."""
    cases = [Case(float(re), float(it)) for re in res for it in inv_tau2s]
    if rlb:
        cases += [Case(float(re), None) for re in res]
    kmax = int(round(ma_max / dma))
    lo = {c: 0 for c in cases}          # largest grid index known stable (0: none)
    hi = {c: kmax + 1 for c in cases}   # smallest grid index known divergent
    t0 = time.perf_counter()
    rounds = 0
    while True:
        open_cases = [c for c in cases if hi[c] - lo[c] > 1]
        if not open_cases:
            break
        mids = {c: (lo[c] + hi[c]) // 2 for c in open_cases}
        flags = classify([(c.re, mids[c] * dma, c.inv_tau2) for c in open_cases], n=n,
                         storage=storage, periods=periods)
        for c, ok in zip(open_cases, flags):
            if ok:
                lo[c] = mids[c]
            else:
                hi[c] = mids[c]
        rounds += 1
        if log:
            log("round %d: %d cases open" % (rounds, len(open_cases)))
    out = [{"re": c.re, "inv_tau2": c.inv_tau2, "ma_c": round(lo[c] * dma, 6),
            "stable_at": round(lo[c] * dma, 6) if lo[c] > 0 else None,
            "diverged_at": round(hi[c] * dma, 6) if hi[c] <= kmax else None} for c in cases]
    return {"n": n, "storage": storage, "dma": dma, "periods": periods, "rounds": rounds,
            "seconds": round(time.perf_counter() - t0, 3), "cases": out}


def divergence_steps(runs, n: int = 128, storage: str = "f64", quantum: int = 16,
                     periods: float = 4.0):
    """For every (re, ma, inv_tau2) of `runs`: the first check (every
    `quantum` steps) at which the run has diverged, in units of t_c, or None
    if it has not within `periods` t_c.  Shows how close to the horizon of
    the study a run near Ma_c diverges."""
    from .lattice import Batch, Lattice

    lats, tcs, remaining = [], [], []
    for re, ma, inv_tau2 in runs:
        u0, tau1, tau2, steps = run_parameters(n, re, ma, inv_tau2, periods)
        lat = Lattice(n, n, tau1, tau2, storage=storage)
        lat.init_equilibrium(*inputs.double_shear_layer(n, u0))
        lats.append(lat)
        tcs.append(n / u0)
        remaining.append(steps)
    out = [None] * len(runs)
    done = [False] * len(runs)
    taken = 0
    batch = Batch(lats)
    members = list(range(len(runs)))
    try:
        while members:
            q = min(quantum, min(remaining[i] - taken for i in members))
            batch.step(q)
            taken += q
            diag = batch.diagnostics()
            for row, i in zip(diag, members):
                if row[4] > 0:
                    out[i], done[i] = taken / tcs[i], True
                elif taken >= remaining[i]:
                    done[i] = True
            alive = [i for i in members if not done[i]]
            if alive != members:
                batch.close()
                batch = Batch([lats[i] for i in alive]) if alive else None
                members = alive
    finally:
        if batch is not None:
            batch.close()
        for lat in lats:
            lat.close()
    return out


def summary(result) -> dict:
    """Per Re: the TRT-RLB maximum of Ma_c over 1/tau_s2 (and where), and RLB."""
    by_re = {}
    for r in result["cases"]:
        d = by_re.setdefault(r["re"], {"trt_rlb_max": 0.0, "at_inv_tau2": None, "rlb": None})
        if r["inv_tau2"] is None:
            d["rlb"] = r["ma_c"]
        elif r["ma_c"] > d["trt_rlb_max"]:
            d["trt_rlb_max"], d["at_inv_tau2"] = r["ma_c"], r["inv_tau2"]
    return by_re


def main():
    import argparse
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--re", type=float, nargs="+", default=[5e3, 1e4, 5e4, 1e5, 1e6, 1e7])
    ap.add_argument("--inv-tau2", type=float, nargs="+",
                    default=[round(0.1 * k, 1) for k in range(1, 21)])
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--storage", default="f64", choices=["f64", "f32", "f16"])
    ap.add_argument("--no-rlb", action="store_true")
    ap.add_argument("--out", default=None)
    ap.add_argument("--divergence", type=float, nargs="+", default=None, metavar="MA",
                    help="instead of the search: when each Mach number diverges (in t_c, "
                         "up to 4 t_c) at every --re and --inv-tau2 (and RLB)")
    a = ap.parse_args()
    import sys
    if a.divergence:
        rates = list(a.inv_tau2) + ([] if a.no_rlb else [None])
        runs = [(re, ma, r) for re in a.re for r in rates for ma in a.divergence]
        times = divergence_steps(runs, n=a.n, storage=a.storage)
        for (re, ma, r), t in zip(runs, times):
            print(json.dumps({"re": re, "inv_tau2": r, "ma": ma,
                              "diverged_at_tc": None if t is None else round(t, 3)}),
                  flush=True)
        return
    res = critical_mach(a.re, a.inv_tau2, rlb=not a.no_rlb, n=a.n, storage=a.storage,
                        log=lambda m: print(m, file=sys.stderr, flush=True))
    res["summary"] = {str(k): v for k, v in summary(res).items()}
    text = json.dumps(res, indent=1)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text)
    print(json.dumps(res["summary"]), flush=True)


if __name__ == "__main__":
    main()
