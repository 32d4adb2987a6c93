"""FP16 (f - w) storage against the FP16-rounded oracle (tests/f16_harness.py)
and against the unrounded oracle.

What the format itself allows.  The harness rounds the oracle's stored
values to IEEE half after every step, so it carries exactly the format's
quantisation and nothing else.  Its own error against the unrounded oracle
is the format's limit: on the Taylor-Green set-up of Sec. III.B (64^2,
u0 = 0.01, 1000 steps) 0.95e-3 to 1.36e-3 in the relative max norm and
0.50e-3 to 0.63e-3 in the relative L2 norm over six phase seeds; on a
force-driven walled channel and the open-boundary cylinder it exceeds 1e-3
in both norms.  A 1000-step max norm within 1e-3 is therefore out of reach
of FP16 storage whatever the kernel does.

Why the GPU is not held to the harness step for step.  The GPU computes in
FP32 and the harness in FP64; about one stored value in 10^4 falls on the
other side of an FP16 rounding boundary.  After one step the two agree
population by population (checked below: every value within one FP16 step,
>= 99.9% identical), but a single flipped value changes later rounding
decisions of its neighbours, and within ~10 steps the GPU run and the
harness are two different realisations of the same quantisation noise.

So the checks are:
* one step, population by population, against the harness;
* the paper's error measure (relative L2, Sec. III) against the unrounded
  oracle within 1e-3 where the format meets it (Taylor-Green 1000 steps,
  uniform inflow), and one step within 1e-3 in both norms;
* multi-step error statistics: the GPU's error against the unrounded oracle
  must match the harness's (same format, exact arithmetic) -- the mean over
  six seeds within 1.25 times the harness's mean, a single realisation
  within 1.5 times.  A kernel error comparable to the format's error
  (~5e-4) would double the GPU's figure.
"""
import numpy as np
import pytest

import f16_harness as H
import oracle
from gpu_util import rel_errors, say
from paper_2312_10318_amd import creeping, inputs, params

pytestmark = pytest.mark.gpu

SEEDS = range(6)


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_10318_amd import lattice
    return lattice


def _np(t):
    return t.detach().cpu().numpy()


def _population_agreement(lat, fh, mask=None):
    """(fraction of stored populations equal to the harness's, largest
    difference in FP16 steps of the larger of the two values)."""
    g = _np(lat.get_populations())
    fluid = np.ones(fh.shape[1:], bool) if mask is None else (np.asarray(mask) == 0)
    a, b = (g - H.W)[:, fluid], (fh - H.W)[:, fluid]
    ulp = np.spacing(np.maximum(np.abs(a), np.abs(b)).astype(np.float16)).astype(np.float64)
    return float(np.mean(a == b)), float(np.max(np.abs(a - b) / ulp))


def test_taylor_green_64_f16_ensemble(L):
    n, tau1, steps = 64, 0.6, 1000
    tau2 = params.tau2_from_magic(tau1, 0.25)
    fields = [inputs.taylor_green(n, 0.01, seed=s) for s in SEEDS]
    lats = [L.Lattice(n, n, tau1, tau2, storage="f16").init_equilibrium(*fl) for fl in fields]
    batch = L.Batch(lats)
    batch.step(1)
    f0s = [oracle.init_equilibrium(*fl) for fl in fields]
    for s, lat, f0 in zip(SEEDS, lats, f0s):
        h1, _ = H.run(f0, 1, tau1, tau2)
        same, ulps = _population_agreement(lat, h1)
        _, gu, gv = (_np(t) for t in lat.macros())
        _, ou, ov = oracle.macros(oracle.step(f0, tau1, tau2))
        e1 = rel_errors(gu, gv, ou, ov)
        say("TG64 seed %d step 1: %.5f of populations equal to the FP16 harness, largest "
            "difference %.1f FP16 steps; vs oracle rel max %.3e L2 %.3e" % ((s, same, ulps) + e1))
        assert same >= 0.999 and ulps <= 1.0
        assert max(e1) <= 1e-3
    batch.step(steps - 1)
    e_gpu, e_har = [], []
    for s, lat, f0 in zip(SEEDS, lats, f0s):
        fh, _ = H.run(f0, steps, tau1, tau2)
        _, ou, ov = oracle.macros(oracle.run(f0, steps, tau1, tau2))
        _, gu, gv = (_np(t) for t in lat.macros())
        _, hu, hv = oracle.macros(fh)
        e_gpu.append(rel_errors(gu, gv, ou, ov))
        e_har.append(rel_errors(hu, hv, ou, ov))
        say("TG64 seed %d step %d vs oracle: GPU rel max %.3e L2 %.3e | FP16 harness rel max "
            "%.3e L2 %.3e" % ((s, steps) + e_gpu[-1] + e_har[-1]))
        assert e_gpu[-1][1] <= 1e-3
    batch.close()
    for lat in lats:
        lat.close()
    g, h = np.mean(e_gpu, axis=0), np.mean(e_har, axis=0)
    say("TG64 %d steps, mean over %d seeds: GPU rel max %.3e L2 %.3e | harness rel max %.3e "
        "L2 %.3e" % (steps, len(SEEDS), g[0], g[1], h[0], h[1]))
    assert g[0] <= 1.25 * h[0] and g[1] <= 1.25 * h[1]


def _single(name, gpu, har, orc_):
    e_go = rel_errors(gpu[0], gpu[1], orc_[0], orc_[1])
    e_ho = rel_errors(har[0], har[1], orc_[0], orc_[1])
    say("%s vs oracle: GPU rel max %.3e L2 %.3e | FP16 harness rel max %.3e L2 %.3e"
        % ((name,) + e_go + e_ho))
    assert e_go[0] <= 1.5 * e_ho[0] and e_go[1] <= 1.5 * e_ho[1]


def test_walled_channel_f16(L):
    """Force-driven channel between half-way bounce-back walls (Sec. III.C
    set-up) from rest, 1000 steps."""
    nx, nf, steps, tau1 = 32, 30, 1000, 0.8
    tau2 = params.tau2_from_magic(tau1, 3 / 16)
    g = 8 * params.nu_from_tau(tau1) * 0.01 / nf ** 2
    mask = inputs.channel_mask(nx, nf)
    rho, ux, uy = inputs.rest_state(nf + 2, nx)
    f0 = oracle.init_equilibrium(rho, ux, uy, mask)
    lat = L.Lattice(nx, nf + 2, tau1, tau2, g=(g, 0.0), mask=mask, storage="f16")
    lat.init_equilibrium(rho, ux, uy).step(1)
    h1, _ = H.run(f0, 1, tau1, tau2, g, 0.0, mask)
    same, ulps = _population_agreement(lat, h1, mask)
    say("channel step 1: %.5f of populations equal to the FP16 harness, largest difference "
        "%.1f FP16 steps" % (same, ulps))
    assert same >= 0.999 and ulps <= 1.0
    lat.step(steps - 1)
    fh, _ = H.run(f0, steps, tau1, tau2, g, 0.0, mask)
    fo = oracle.run(f0, steps, tau1, tau2, g, 0.0, mask)
    _, gu, gv = (_np(t) for t in lat.macros())
    lat.close()
    _single("channel 32x30 %d steps" % steps, (gu, gv), oracle.macros(fh, g, 0.0, mask)[1:],
            oracle.macros(fo, g, 0.0, mask)[1:])


def test_open_cylinder_f16(L):
    """The small creeping-flow cylinder (Sec. III.D set-up: inflow wall,
    pressure outlet, D = 5, L = 6 D, Re = 0.1), 500 steps."""
    c = creeping.Case(0.1, D=5, ratio=6)
    steps = 500
    mask = creeping.cylinder_mask(c.n, c.D)
    fields = creeping.initial_fields(c, mask)
    f0 = oracle.init_equilibrium(*fields, mask)
    lat = L.Lattice(c.n, c.n, c.tau1, c.tau2, mask=mask, storage="f16", inflow=(c.u0, 1.0, 1.0))
    lat.init_equilibrium(*fields).step(1)
    _, gu, gv = (_np(t) for t in lat.macros())
    _, ou, ov = oracle.macros(oracle.step_open(f0, c.tau1, c.tau2, c.u0, mask=mask), mask=mask)
    e1 = rel_errors(gu, gv, ou, ov)
    say("open cylinder step 1 vs oracle: rel max %.3e L2 %.3e" % e1)
    assert max(e1) <= 1e-3
    lat.step(steps - 1)
    fh = H.run_open(f0, steps, c.tau1, c.tau2, c.u0, mask=mask)
    fo = oracle.run_open(f0, steps, c.tau1, c.tau2, u_in=c.u0, mask=mask)
    _, gu, gv = (_np(t) for t in lat.macros())
    lat.close()
    _single("open cylinder 30x30 %d steps" % steps, (gu, gv), oracle.macros(fh, mask=mask)[1:],
            oracle.macros(fo, mask=mask)[1:])
