"""Creeping flow past a square cylinder (Sec. III.D, Table 1) on the GPU.

Set-up (Sec. III.D): a square domain of side L = 50 D lattice nodes with a
square cylinder of side D = 21 nodes at its centre; uniform inflow u_c from
the left through a half-way bounce-back wall moving with (u_c, 0), a
pressure outlet (rho = rho_0 = 1, Zou and He) on the right, periodic top and
bottom, half-way bounce-back on the cylinder; Lambda_s = 3/16.  The
incompressibility parameter T = Ma^2 / Re = 0.1 fixes Ma = sqrt(T Re),
u_c = c_s Ma and tau_s1 = 1/2 + 3 u_c D / Re.  The RLB model is the case
tau_s2 = tau_s1.

Readings (the paper is silent on them): the flow starts from rest density
and the uniform inflow velocity at every fluid node; the cylinder occupies
nodes [(n - D) // 2, (n - D) // 2 + D) in x and y; a run has converged when
the relative L2 change of the velocity field over one check interval
(1000 steps) falls below 1e-9 (the paper's termination criterion L_2 <
1e-9, Eq. for L_2 in Sec. III applied to successive fields); a run has
diverged when the library's divergence count is non-zero.

Drag (Sec. III.D): F_x from momentum exchange with the cylinder during the
last collision, C_d = 2 F_x / (rho_0 u_c^2 D), C_d,mu = C_d Re.

All cases of a call run as one batch (one launch per step); a member leaves
the batch when it converges or diverges.
"""
from __future__ import annotations

import dataclasses
import math
import sys
import time

import numpy as np

from . import params

C_S = math.sqrt(params.CS2)


@dataclasses.dataclass(frozen=True)
class Case:
    re: float
    rlb: bool = False          # tau_s2 = tau_s1 (the RLB model)
    T: float = 0.1             # Ma^2 / Re
    D: int = 21
    ratio: int = 50            # L / D
    lam: float = 3.0 / 16.0

    @property
    def n(self) -> int:
        return self.ratio * self.D

    @property
    def ma(self) -> float:
        return math.sqrt(self.T * self.re)

    @property
    def u0(self) -> float:
        return C_S * self.ma

    @property
    def tau1(self) -> float:
        return params.tau_from_re(self.u0, self.D, self.re)

    @property
    def tau2(self) -> float:
        return self.tau1 if self.rlb else params.tau2_from_magic(self.tau1, self.lam)

    @property
    def label(self) -> str:
        return "Re=%g %s" % (self.re, "RLB" if self.rlb else "TRT-RLB")


def cylinder_mask(n: int, D: int) -> np.ndarray:
    m = np.zeros((n, n), np.uint8)
    s = (n - D) // 2
    m[s:s + D, s:s + D] = 1
    return m


def initial_fields(case: Case, mask: np.ndarray):
    n = case.n
    ux = np.where(mask != 0, 0.0, case.u0)
    return np.ones((n, n)), ux, np.zeros((n, n))


def drag(case: Case, fx: float) -> dict:
    cd = 2.0 * fx / (1.0 * case.u0 ** 2 * case.D)
    return {"Fx": fx, "Cd": cd, "Cd_mu": cd * case.re}


def solve(cases, storage: str = "f64", check: int = 1000, tol: float = 1e-9,
          max_steps: int = 3_000_000, log=None):
    """Run every case to convergence (or divergence, or max_steps) in one
    batch; returns one record per case."""
    import torch

    from .lattice import Batch, Lattice

    lats, prev, res = [], [], []
    t0 = time.perf_counter()
    for c in cases:
        mask = cylinder_mask(c.n, c.D)
        lat = Lattice(c.n, c.n, c.tau1, c.tau2, mask=mask, storage=storage,
                      inflow=(c.u0, 1.0, 1.0))
        lat.init_equilibrium(*initial_fields(c, mask))
        lats.append(lat)
        z = torch.zeros((c.n, c.n), dtype=torch.float64, device=lat.device)
        prev.append((z, z.clone()))
        lat.velocity_change(prev[-1])  # prev <- the initial velocity
        res.append({"re": c.re, "model": "RLB" if c.rlb else "TRT-RLB", "n": c.n, "D": c.D,
                    "Ma": c.ma, "u0": c.u0, "tau1": c.tau1, "tau2": c.tau2, "steps": 0,
                    "status": None, "l2_change": None})
    alive = list(range(len(cases)))
    batch, members = None, None
    try:
        while alive:
            if members != alive:
                if batch is not None:
                    batch.close()
                members = list(alive)
                batch = Batch([lats[i] for i in members])
            batch.step(check)
            diag = batch.diagnostics()
            for row, i in zip(diag, members):
                r = res[i]
                r["steps"] += check
                if row[4] > 0:
                    r["status"] = "diverged"
                    continue
                mx, s2, n2, _ = lats[i].velocity_change(prev[i])
                r["l2_change"] = math.sqrt(s2 / n2) if n2 > 0 else float("inf")
                r["max_change"] = mx / cases[i].u0
                if r["l2_change"] < tol:
                    r["status"] = "converged"
                elif r["steps"] >= max_steps:
                    r["status"] = "max_steps"
                if r["status"] is not None:
                    r.update(drag(cases[i], lats[i].wall_force()[0]))
                    r["seconds"] = round(time.perf_counter() - t0, 2)
                    if log:
                        log("%s: %s after %d steps, Cd_mu = %.4f" %
                            (cases[i].label, r["status"], r["steps"], r["Cd_mu"]))
            for i in members:
                if res[i]["status"] == "diverged" and "seconds" not in res[i]:
                    res[i]["seconds"] = round(time.perf_counter() - t0, 2)
                    if log:
                        log("%s: diverged after %d steps" % (cases[i].label, res[i]["steps"]))
            alive = [i for i in members if res[i]["status"] is None]
    finally:
        if batch is not None:
            batch.close()
        for lat in lats:
            lat.close()
    return res


TABLE1_RE = (1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7)


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="Creeping flow past a square cylinder (Table 1)")
    ap.add_argument("--re", type=float, nargs="+", default=list(TABLE1_RE))
    ap.add_argument("--rlb", type=float, nargs="*", default=[1e-1, 1e-2, 1e-3],
                    help="Reynolds numbers also run with the RLB model (tau_s2 = tau_s1)")
    ap.add_argument("--D", type=int, default=21)
    ap.add_argument("--ratio", type=int, default=50)
    ap.add_argument("--storage", default="f64", choices=["f64", "f32", "f16"])
    ap.add_argument("--tol", type=float, default=1e-9)
    ap.add_argument("--check", type=int, default=1000)
    ap.add_argument("--max-steps", type=int, default=3_000_000)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    cases = [Case(re, False, D=a.D, ratio=a.ratio) for re in a.re]
    cases += [Case(re, True, D=a.D, ratio=a.ratio) for re in a.rlb]
    res = solve(cases, storage=a.storage, check=a.check, tol=a.tol, max_steps=a.max_steps,
                log=lambda m: print(m, file=sys.stderr, flush=True))
    text = json.dumps(res, indent=1)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text)
    for r in res:
        print(json.dumps({k: r.get(k) for k in ("re", "model", "status", "steps", "Cd_mu",
                                                "tau1", "seconds")}), flush=True)


if __name__ == "__main__":
    main()
