"""Grid convergence of the decaying Taylor-Green vortex (Sec. III.B) on the GPU.

* Parity: at N = 32 and 64 the GPU's relative L2 error at t_d (FP64) equals
  the error of the oracle run on the same set-up to 1e-8 of its value.
* The paper's sweep N = 32 ... 512 (its grid-convergence figure for
  Sec. III.B): second-order spatial convergence of TRT-RLB, each halving of
  dx dividing the error by 2^(2 +- 0.2); the RLB case (tau_s2 = tau_s1) is
  also second order, with a larger error at every grid, as the paper
  finds.
"""
import math

import numpy as np
import pytest

import oracle
from gpu_util import say
from paper_2312_10318_amd import convergence, inputs, params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_10318_amd import lattice
    return lattice


def _oracle_l2(n):
    tau1, tau2, u0, steps = convergence.case(n)
    rho, ux, uy = inputs.taylor_green(n, u0, seed=None)
    f = oracle.run(oracle.init_equilibrium(rho, ux, uy), steps, tau1, tau2)
    _, un, vn = oracle.macros(f)
    _, ua, va = inputs.taylor_green(n, u0, nu=params.nu_from_tau(tau1), t=float(steps), seed=None)
    return math.sqrt((np.sum((un - ua) ** 2) + np.sum((vn - va) ** 2)) /
                     (np.sum(ua ** 2) + np.sum(va ** 2)))


def test_error_at_decay_time_equals_the_oracles(L):
    res = convergence.run((32, 64), "f64")
    for n, got in zip(res["n"], res["l2"]):
        want = _oracle_l2(n)
        say("case: TG N=%d FP64 L2 at t_d: GPU %.12e oracle %.12e" % (n, got, want))
        assert abs(got - want) <= 1e-8 * want


def test_second_order_convergence_paper_sweep(L):
    """TRT-RLB and RLB are second order over the paper's grids, and TRT-RLB
    has the lower error at every grid (the paper's finding)."""
    out = {}
    for rlb in (False, True):
        res = convergence.run(convergence.PAPER_NS, "f64", rlb=rlb)
        say("case: TG convergence %s FP64 N=%s L2=%s orders=%s (%.2f s)" % (
            res["model"], res["n"], ["%.3e" % e for e in res["l2"]],
            ["%.3f" % o for o in res["order"]], res["seconds"]))
        assert all(1.8 < o < 2.2 for o in res["order"])
        out[res["model"]] = res["l2"]
    assert out["TRT-RLB"][-1] < 1e-4
    assert all(a < b for a, b in zip(out["TRT-RLB"], out["RLB"]))
