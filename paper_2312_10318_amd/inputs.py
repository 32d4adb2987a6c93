"""Seeded synthetic workloads: initial fields, masks and parameter draws.

Every input of the tests and of the benchmark comes from here, for the GPU
path and for the CPU oracle alike.  This module holds no collision, streaming
or equilibrium arithmetic: it only evaluates the paper's initial and boundary
conditions (Sec. III) on the lattice and draws random parameters.

Coordinates: node (i, j) sits at x = i, y = j in lattice units; a periodic
domain of side N has x / L = i / N.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import params


def taylor_green(n: int, u0: float = 0.01, rho0: float = 1.0, *, nu: float = 0.0,
                 t: float = 0.0, seed: int | None = 0, phase=None, device=None):
    """Decaying Taylor-Green vortex on an n x n periodic lattice (Sec. III.B).

    u_x = -u0 cos(2 pi x) sin(2 pi y) e^{-t/t_d},
    u_y =  u0 cos(2 pi y) sin(2 pi x) e^{-t/t_d},
    rho = rho0 - rho0 u0^2 / (4 c_s^2) [cos 4 pi x + cos 4 pi y] e^{-2 t/t_d},
    with x = (i + phi_x) / n, y = (j + phi_y) / n and t_d = 1 / (8 nu pi^2)
    in units of the domain side (nu here is the lattice viscosity, so
    t_d = n^2 / (8 nu pi^2) steps).  The phase (phi_x, phi_y) is drawn from
    ``seed`` in [0, n)^2 unless given; seed=None means no phase.
    Returns (rho, ux, uy), float64 [n, n], indexed [y, x]: numpy arrays, or
    torch tensors on `device` when one is given (the per-axis factors are
    formed on the host and the n x n products and sums on the device, in the
    same order, so the values are the same bits).
    """
    if phase is None:
        phase = (0.0, 0.0) if seed is None else tuple(np.random.default_rng(seed).uniform(0, n, 2))
    px, py = phase
    i = np.arange(n, dtype=np.float64)
    x = ((i + px) / n)[None, :]
    y = ((i + py) / n)[:, None]
    if t > 0.0:
        td = n * n / (8.0 * nu * math.pi ** 2)
        decay = math.exp(-t / td)
    else:
        decay = 1.0
    coef = rho0 * u0 ** 2 / (4.0 * params.CS2)
    if device is not None:
        import torch

        def dev(a):
            # pinned and asynchronous on the current stream: a pageable copy
            # would wait for the work already queued there
            h = torch.from_numpy(np.ascontiguousarray(a))
            if torch.device(device).type == "cuda":
                h = h.pin_memory()
            return h.to(device, non_blocking=True)
        ax, sy = dev(-u0 * np.cos(2 * np.pi * x)), dev(np.sin(2 * np.pi * y))
        ay, sx = dev(u0 * np.cos(2 * np.pi * y)), dev(np.sin(2 * np.pi * x))
        cx4, cy4 = dev(np.cos(4 * np.pi * x)), dev(np.cos(4 * np.pi * y))
        ux = (ax * sy * decay).contiguous()
        uy = (ay * sx * decay).contiguous()
        rho = (rho0 - coef * (cx4 + cy4) * decay ** 2).contiguous()
        return rho, ux, uy
    ux = -u0 * np.cos(2 * np.pi * x) * np.sin(2 * np.pi * y) * decay
    uy = u0 * np.cos(2 * np.pi * y) * np.sin(2 * np.pi * x) * decay
    rho = rho0 - coef * (np.cos(4 * np.pi * x) + np.cos(4 * np.pi * y)) * decay ** 2
    return (np.ascontiguousarray(rho), np.ascontiguousarray(np.broadcast_to(ux, (n, n))),
            np.ascontiguousarray(np.broadcast_to(uy, (n, n))))


def double_shear_layer(n: int, u0: float = 0.04, kappa: float = 80.0, delta: float = 0.05,
                       rho0: float = 1.0):
    """Double shear layer on an n x n periodic lattice (Sec. III.A).

    u_x = u0 tanh[kappa (y/L - 1/4)] for y/L <= 1/2, u0 tanh[kappa (3/4 - y/L)]
    otherwise; u_y = u0 delta sin[2 pi (x/L + 1/4)]; rho = rho0; y/L = j / n.
    Returns (rho, ux, uy), float64 [n, n].
    """
    s = np.arange(n, dtype=np.float64) / n
    yl = s[:, None]
    ux = np.where(yl <= 0.5, u0 * np.tanh(kappa * (yl - 0.25)), u0 * np.tanh(kappa * (0.75 - yl)))
    uy = u0 * delta * np.sin(2 * np.pi * (s[None, :] + 0.25))
    rho = np.full((n, n), rho0)
    return (rho, np.ascontiguousarray(np.broadcast_to(ux, (n, n))),
            np.ascontiguousarray(np.broadcast_to(uy, (n, n))))


def channel_mask(nx: int, n_fluid: int) -> np.ndarray:
    """Channel of n_fluid fluid rows between two solid rows (Sec. II.D set-up).

    Rows j = 0 and j = n_fluid + 1 are solid; fluid row j sits at distance
    j - 1/2 from the lower half-way wall.  Shape [n_fluid + 2, nx], 1 = solid.
    """
    m = np.zeros((n_fluid + 2, nx), dtype=np.uint8)
    m[0, :] = 1
    m[-1, :] = 1
    return m


def square_obstacle_mask(nx: int = 400, ny: int = 200, side: int = 20) -> np.ndarray:
    """A centred square obstacle of `side` nodes (nodes [(n - side) // 2,
    (n - side) // 2 + side) in x and y), nothing else solid."""
    m = np.zeros((ny, nx), dtype=np.uint8)
    x0 = (nx - side) // 2
    y0 = (ny - side) // 2
    m[y0:y0 + side, x0:x0 + side] = 1
    return m


def cylinder_channel_mask(nx: int = 400, ny: int = 200, side: int = 20) -> np.ndarray:
    """Channel with solid top/bottom rows and a centred square obstacle.

    A force-driven stand-in for the square-cylinder problem of Sec. III.D
    (used by tests of walled batches).
    """
    m = np.zeros((ny, nx), dtype=np.uint8)
    m[0, :] = 1
    m[-1, :] = 1
    x0 = (nx - side) // 2
    y0 = (ny - side) // 2
    m[y0:y0 + side, x0:x0 + side] = 1
    return m


def rest_state(ny: int, nx: int, rho0: float = 1.0, device=None):
    """Uniform fluid at rest (numpy arrays, or torch tensors on `device`)."""
    if device is not None:
        import torch
        return (torch.full((ny, nx), rho0, dtype=torch.float64, device=device),
                torch.zeros((ny, nx), dtype=torch.float64, device=device),
                torch.zeros((ny, nx), dtype=torch.float64, device=device))
    return np.full((ny, nx), rho0), np.zeros((ny, nx)), np.zeros((ny, nx))


def random_populations(rng: np.random.Generator, shape, rho0: float = 1.0, amp: float = 0.05):
    """Random positive populations near rest equilibrium weights.

    Used only to exercise identities on arbitrary (non-equilibrium) states:
    f_i = w_i rho0 (1 + amp * U[-1, 1]).  The D2Q9 weights are the lattice's
    data (Sec. II.B), not collision arithmetic.
    """
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    shape = tuple(shape)
    pert = rng.uniform(-1.0, 1.0, size=(9,) + shape)
    return w.reshape((9,) + (1,) * len(shape)) * rho0 * (1.0 + amp * pert)


@dataclasses.dataclass
class BatchMember:
    """One instance of the batched workload."""
    kind: str            # "tg" or "dsl"
    n: int               # side length (nx = ny = n)
    re: float
    tau1: float
    tau2: float
    u0: float


def batch_workload(count: int = 256, seed: int = 0, side_lo: int = 64, side_hi: int = 1024,
                   re_lo: float = 1e2, re_hi: float = 1e7):
    """Batched configuration: sides log-uniform in [side_lo, side_hi], half
    Taylor-Green (u0 = 0.01) and half double shear layer (U0 = 0.04), Re
    log-uniform in [re_lo, re_hi], tau_s1 from Re, tau_s2 uniform in [0.5, 2]
    (drawn in (0.5, 2] so that 1 / tau_s2 stays finite and below 2)."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(round(math.exp(rng.uniform(math.log(side_lo), math.log(side_hi)))))
        re = math.exp(rng.uniform(math.log(re_lo), math.log(re_hi)))
        tau2 = float(rng.uniform(0.5, 2.0))
        tau2 = max(tau2, 0.5 + 1e-3)
        kind = "tg" if k % 2 == 0 else "dsl"
        u0 = 0.01 if kind == "tg" else 0.04
        tau1 = params.tau_from_re(u0, n, re)
        out.append(BatchMember(kind, n, re, tau1, tau2, u0))
    return out


def member_fields(m: BatchMember, seed: int = 0):
    """Initial (rho, ux, uy) of one batch member."""
    if m.kind == "tg":
        return taylor_green(m.n, m.u0, seed=seed)
    return double_shear_layer(m.n, m.u0)
