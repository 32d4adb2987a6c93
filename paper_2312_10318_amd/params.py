"""Parameter relations of the TRT-RLB model in lattice units (dx = dt = c = 1).

Host-side helpers only; none of the collision arithmetic lives here.
"""
from __future__ import annotations

import math

CS2 = 1.0 / 3.0  # c_s^2 = c^2 / 3 (Sec. II.B)


def nu_from_tau(tau1: float) -> float:
    """Kinematic viscosity nu = c_s^2 (tau_s1 - 1/2) dt (Sec. II.C, viscosity relation)."""
    return CS2 * (tau1 - 0.5)


def tau_from_nu(nu: float) -> float:
    """Inverse of :func:`nu_from_tau`."""
    return nu / CS2 + 0.5


def magic(tau1: float, tau2: float) -> float:
    """Magic parameter Lambda_s = (tau_s1 - 1/2)(tau_s2 - 1/2) (Sec. II.D)."""
    return (tau1 - 0.5) * (tau2 - 0.5)


def tau2_from_magic(tau1: float, lam: float) -> float:
    """tau_s2 that gives the magic parameter ``lam`` at tau_s1 (Sec. II.D).

    lam = 3/16 removes the half-way bounce-back slip; lam = 1/4 is the
    Taylor-Green setting of Sec. III.B.
    """
    if tau1 <= 0.5:
        raise ValueError("tau_s1 must exceed 1/2")
    return 0.5 + lam / (tau1 - 0.5)


def tau_from_re(u: float, length: float, re: float) -> float:
    """tau_s1 for Reynolds number Re = u L / nu at lattice velocity u."""
    return tau_from_nu(u * length / re)


def mach_from_T(T: float, re: float) -> float:
    """Mach number from the incompressibility parameter T = Ma^2 / Re (Sec. III.D)."""
    return math.sqrt(T * re)


def u_from_mach(ma: float) -> float:
    """Lattice velocity u = Ma c_s."""
    return ma * math.sqrt(CS2)
