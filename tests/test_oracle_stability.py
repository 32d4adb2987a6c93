"""The oracle against the paper's printed double-shear-layer stability limit.

Sec. III.A reports that at Re = 5e3 the TRT-RLB model stays stable up to
t/t_c = 2 for Mach numbers up to Ma_c = 0.62 on a dMa = 0.01 grid, at its
best 1/tau_s2 (the optimum is near 1.6).  The oracle, run on the paper's
set-up (N = 128, kappa = 80, delta = 0.05), must be stable at Ma = 0.62 and
diverge at Ma = 0.63 for 1/tau_s2 = 1.6.  The run parameters (U0 = c_s Ma,
tau_s1 from Re = U0 N / nu, 2 t_c = 2 N / U0 steps) come from the host
helper that the GPU study uses; the arithmetic is the oracle's.
"""
import os

import numpy as np
import pytest

from paper_2312_10318_amd import inputs, stability

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "dsl_critical_mach.txt")


def golden():
    out = {}
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, lo, hi, v = line.split()
            out[name] = (float(lo), float(hi), float(v))
    return out


def diverged(orc, re, inv_tau2, ma, n=128):
    u0, tau1, tau2, steps = stability.run_parameters(n, re, ma, inv_tau2)
    f = orc.run(orc.init_equilibrium(*inputs.double_shear_layer(n, u0)), steps, tau1, tau2)
    rho, ux, uy = orc.macros(f)
    bad = ~np.isfinite(rho) | ~np.isfinite(ux) | ~np.isfinite(uy) | (rho <= 0)
    bad |= np.hypot(np.nan_to_num(ux), np.nan_to_num(uy)) >= 1.0
    return bool(bad.any())


def test_run_parameters_follow_the_setup():
    u0, tau1, tau2, steps = stability.run_parameters(128, 5e3, 0.62, 1.6)
    assert u0 == pytest.approx(0.62 / np.sqrt(3))
    assert tau1 == pytest.approx(0.5 + 3 * u0 * 128 / 5e3)
    assert tau2 == pytest.approx(1 / 1.6)
    assert steps == int(np.ceil(2 * 128 / u0))
    # RLB: tau_s2 = tau_s1
    assert stability.run_parameters(128, 5e3, 0.3, None)[2] == stability.run_parameters(
        128, 5e3, 0.3, None)[1]


def test_oracle_reproduces_printed_critical_mach(orc):
    re, _, ma_c = golden()["trt_rlb_max"]
    assert not diverged(orc, re, 1.6, ma_c)
    assert diverged(orc, re, 1.6, round(ma_c + 0.01, 2))
