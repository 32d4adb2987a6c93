"""Grid convergence of the decaying Taylor-Green vortex (Sec. III.B) on the GPU.

Set-up (Sec. III.B): the unit square, periodic, u0 = 0.01, rho0 = 1,
nu = 0.01 and diffusive scaling dx^2 / dt = 0.01 pi^2 with dx = 1/N, so in
lattice units nu = 1/pi^2 (tau_s1 = 1/2 + 3/pi^2), the velocity scale is
u0 dt/dx = 1/(pi^2 N) and the decay time t_d = 1/(8 nu pi^2) is N^2/8 steps;
Lambda_s = 1/4.  The error is the relative L2 norm of the velocity against
the analytic field (the error measure of Sec. III, both components summed)
at t = t_d, computed on the device.  The RLB model is the case
tau_s2 = tau_s1.

All grid sizes of a call run as one batch (one launch per step); a member
leaves the batch when it reaches its t_d.
"""
from __future__ import annotations

import math
import time

from . import inputs, params

PAPER_NS = (32, 64, 128, 256, 512)


def case(n: int, rlb: bool = False, lam: float = 0.25):
    """(tau_s1, tau_s2, u0 in lattice units, steps to t_d) for grid n."""
    nu = 1.0 / math.pi ** 2
    tau1 = params.tau_from_nu(nu)
    tau2 = tau1 if rlb else params.tau2_from_magic(tau1, lam)
    return tau1, tau2, 1.0 / (math.pi ** 2 * n), n * n // 8


def run(ns=PAPER_NS, storage: str = "f64", rlb: bool = False, lam: float = 0.25):
    """L2 error at t_d for every grid size in `ns`; returns {"n": [...],
    "l2": [...], "order": [log2(e_N / e_2N) between consecutive sizes],
    "seconds": s}."""
    from .lattice import Batch, Lattice

    t0 = time.perf_counter()
    lats, remaining, cases = [], [], []
    for n in ns:
        tau1, tau2, u0, steps = case(n, rlb, lam)
        lat = Lattice(n, n, tau1, tau2, storage=storage)
        lat.init_equilibrium(*inputs.taylor_green(n, u0, seed=None))
        lats.append(lat)
        remaining.append(steps)
        cases.append((tau1, u0, steps))
    l2 = [None] * len(ns)
    alive = list(range(len(ns)))
    batch, members = None, None
    try:
        while alive:
            if members != alive:
                if batch is not None:
                    batch.close()
                members = list(alive)
                batch = Batch([lats[i] for i in members])
            q = min(remaining[i] for i in members)
            batch.step(q)
            for i in members:
                remaining[i] -= q
                if remaining[i] == 0:
                    n = ns[i]
                    tau1, u0, steps = cases[i]
                    _, ua, va = inputs.taylor_green(n, u0, nu=params.nu_from_tau(tau1),
                                                    t=float(steps), seed=None,
                                                    device=lats[i].device)
                    l2[i] = lats[i].velocity_error(ua, va)[0]
            alive = [i for i in members if remaining[i] > 0]
    finally:
        if batch is not None:
            batch.close()
        for lat in lats:
            lat.close()
    order = [math.log2(l2[k] / l2[k + 1]) for k in range(len(ns) - 1)]
    return {"n": list(ns), "l2": l2, "order": order, "storage": storage,
            "model": "RLB" if rlb else "TRT-RLB",
            "seconds": round(time.perf_counter() - t0, 3)}


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="Taylor-Green grid convergence (Sec. III.B)")
    ap.add_argument("--n", type=int, nargs="+", default=list(PAPER_NS))
    ap.add_argument("--storage", default="f64", choices=["f64", "f32", "f16"])
    ap.add_argument("--rlb", action="store_true", help="the RLB model (tau_s2 = tau_s1)")
    a = ap.parse_args()
    print(json.dumps(run(a.n, a.storage, a.rlb)), flush=True)


if __name__ == "__main__":
    main()
