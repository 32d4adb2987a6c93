"""An FP16-storage reference built from the oracle (test harness only).

FP16 (f - w) storage keeps, after every step, each population minus its
weight rounded to nearest even in IEEE half.  This harness does the same to
the FP64 oracle: after each oracle step the stored values are replaced by
their FP16 roundings, so it carries the format's quantisation and nothing
else.  A GPU FP16 run then differs from it only through the GPU's FP32
arithmetic (which moves a value across an FP16 rounding boundary now and
then), while it differs from the unrounded oracle by the whole quantisation
error -- so comparing with this harness can expose a kernel error far below
the format's own error.

Which values are rounded: the lattice stores the post-collision populations
of every fluid node.  For periodic and walled lattices every pre-collision
value of the next step is a copy of one stored value (streaming or half-way
bounce-back), so rounding the oracle's pre-collision state after each step is
the same as rounding the stored values.  With the open x boundaries the
inflow wall adds its correction to a stored value and the outlet rule
computes three populations from stored ones, so there the harness rounds the
oracle's post-collision state (oracle.collide) before streaming it
(oracle.stream_open).  The initial state is the oracle's f(x, 0) rounded the
same way (for the open ends this differs from the GPU's stored initial state
by at most one FP16 step in the three boundary populations of each row).
"""
import numpy as np

import oracle

W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)[:, None, None]


def to_f16_storage(f, mask=None):
    """The populations FP16 (f - w) storage holds for f (solid nodes: 0)."""
    g = (np.asarray(f, dtype=np.float64) - W).astype(np.float16).astype(np.float64) + W
    if mask is not None:
        g[:, np.asarray(mask) != 0] = 0.0
    return g


def run(f0, nsteps, tau1, tau2, gx=0.0, gy=0.0, mask=None, checkpoints=()):
    """nsteps FP16-rounded oracle steps (periodic, walls, obstacles); returns
    the final state and {step: state} at the requested checkpoints."""
    f = to_f16_storage(f0, mask)
    saved = {}
    for s in range(1, nsteps + 1):
        f = to_f16_storage(oracle.step(f, tau1, tau2, gx, gy, mask), mask)
        if s in checkpoints:
            saved[s] = f.copy()
    return f, saved


def run_open(f0, nsteps, tau1, tau2, u_in, rho_w=1.0, rho_out=1.0, gx=0.0, gy=0.0, mask=None):
    """nsteps FP16-rounded oracle steps with the open x boundaries."""
    f = to_f16_storage(f0, mask)
    for _ in range(nsteps):
        fs = oracle.collide(f, tau1, tau2, gx, gy, mask, True, u_in, rho_w)
        f = oracle.stream_open(to_f16_storage(fs, mask), u_in, rho_w, rho_out, mask)
    return f
