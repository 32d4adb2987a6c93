"""Force-driven Poiseuille flow: numerical slip against the magic parameter
(Sec. III.C) on the GPU.

Set-up (Sec. III.C): channel width L = 1 resolved by N_y = 32 fluid rows
between half-way bounce-back walls (solid rows j = 0 and N + 1), N_x = 4
columns, periodic in x; u_c = 0.1, rho_0 = 1, Re = u_c L / nu = 1, so in
lattice units nu = 3.2 (tau_s1 = 10.1) and the body force is
g = 8 nu u_c / N^2 (centre-line velocity u_c of the parabola
u(y) = 4 u_c y (N - y) / N^2, walls at y = 0 and N).  The flow starts from
rest and runs until the relative L2 change of the velocity over 1000 steps
falls below `tol`; the error is the relative L2 norm of the velocity against
the parabola (the error measure of Sec. III), computed on the device.

Sec. II.D predicts a uniform slip u_s = (16 tau1 tau2 - 8 tau1 - 8 tau2 + 1)
g / (4 (2 tau1 - 1)), zero at Lambda_s = 3/16; for such a profile the
relative L2 error is |u_s| sqrt(N / sum_y u(y)^2).  The RLB model is the
case tau_s2 = tau_s1.
"""
from __future__ import annotations

import math
import time

from . import inputs, params

N_Y, N_X, U_C, RE = 32, 4, 0.1, 1.0
PAPER_LAMBDAS = (1 / 16, 1 / 12, 1 / 8, 5 / 32, 3 / 16, 7 / 32, 1 / 4, 3 / 8, 1 / 2)


def setup(n: int = N_Y, uc: float = U_C, re: float = RE):
    """(tau_s1, g) of the channel."""
    nu = uc * n / re
    return params.tau_from_nu(nu), 8.0 * nu * uc / n ** 2


def parabola(n: int = N_Y, nx: int = N_X, uc: float = U_C):
    """Analytic u_x on the lattice rows (0 on the solid rows), float64 [n+2, nx]."""
    import numpy as np
    y = np.arange(n + 2, dtype=np.float64) - 0.5
    u = 4.0 * uc * y * (n - y) / n ** 2
    u[0] = u[-1] = 0.0
    return np.repeat(u[:, None], nx, axis=1)


def predicted_l2(tau1: float, tau2: float, g: float, n: int = N_Y, uc: float = U_C) -> float:
    """Relative L2 error of a parabola shifted by the closed-form slip."""
    us = (16 * tau1 * tau2 - 8 * tau1 - 8 * tau2 + 1) / (4 * (2 * tau1 - 1)) * g
    y = [j + 0.5 for j in range(n)]
    s2 = sum((4.0 * uc * v * (n - v) / n ** 2) ** 2 for v in y)
    return abs(us) * math.sqrt(n / s2)


def sweep(lams=PAPER_LAMBDAS, rlb: bool = True, storage: str = "f64", tol: float = 1e-14,
          check: int = 1000, max_steps: int = 2_000_000):
    """Steady L2 error for every Lambda_s in `lams` (and the RLB model when
    `rlb`), all channels in one batch.  Returns a list of records."""
    import torch

    from .lattice import Batch, Lattice

    t0 = time.perf_counter()
    tau1, g = setup()
    labels = [("TRT-RLB", lam, params.tau2_from_magic(tau1, lam)) for lam in lams]
    if rlb:
        labels.append(("RLB", None, tau1))
    mask = inputs.channel_mask(N_X, N_Y)
    ua = parabola()
    lats, prev, res = [], [], []
    for model, lam, tau2 in labels:
        lat = Lattice(N_X, N_Y + 2, tau1, tau2, g=(g, 0.0), mask=mask, storage=storage)
        lat.init_equilibrium(*inputs.rest_state(N_Y + 2, N_X))
        lats.append(lat)
        z = torch.zeros((N_Y + 2, N_X), dtype=torch.float64, device=lat.device)
        prev.append((z, z.clone()))
        lat.velocity_change(prev[-1])
        res.append({"model": model, "lambda": lam, "tau1": tau1, "tau2": tau2, "g": g,
                    "steps": 0, "status": None})
    alive = list(range(len(labels)))
    batch, members = None, None
    try:
        while alive:
            if members != alive:
                if batch is not None:
                    batch.close()
                members = list(alive)
                batch = Batch([lats[i] for i in members])
            batch.step(check)
            for i in members:
                r = res[i]
                r["steps"] += check
                _, s2, n2, _ = lats[i].velocity_change(prev[i])
                change = math.sqrt(s2 / n2) if n2 > 0 else math.inf
                if change < tol or r["steps"] >= max_steps:
                    r["status"] = "converged" if change < tol else "max_steps"
                    r["l2"], r["max_abs"] = lats[i].velocity_error(ua, 0.0 * ua)
                    r["predicted_l2"] = predicted_l2(tau1, r["tau2"], g)
            alive = [i for i in members if res[i]["status"] is None]
    finally:
        if batch is not None:
            batch.close()
        for lat in lats:
            lat.close()
    for r in res:
        r["seconds"] = round(time.perf_counter() - t0, 3)
    return res


def main():
    import json
    for r in sweep():
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
