"""Lattices whose solid nodes fill whole rows (walls parallel to x, the
channels of Sec. III.C) take two time steps per launch (FP32 and FP16) and
three (FP32).  Next to a
wall row the first step's loads read the node's own slots of the bounced
populations, and the later steps bounce them in registers from the node's
own post-collision values (half-way bounce-back, Sec. II.D); Phi is 0 on a
wall row and wall rows keep zeros.  Every node's arithmetic is that of the
one-step sweep over the link map, so the results are its bits: channels,
adjacent wall rows, a single fluid row between walls, a wall whose
neighbour lies across the periodic seam, an all-solid and an all-fluid
mask, heights of one to three rows, odd widths, lattices narrower than
one window, every launch shape,
both march directions and the deep two-step pipeline; alone and in a
batch; and a channel against the oracle.  A mask whose solid nodes do not
fill whole rows keeps one step per launch, as does FP64 storage."""
import numpy as np
import pytest

import oracle
from gpu_util import TOL, rel_errors, say
from paper_2312_10318_amd import inputs, params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_10318_amd import lattice
    return lattice


def _np(t):
    return t.detach().cpu().numpy()


def _case(seed, nx, ny, walls):
    rng = np.random.default_rng(seed)
    f = inputs.random_populations(rng, (ny, nx), amp=0.05)
    mask = np.zeros((ny, nx), np.uint8)
    mask[list(walls)] = 1
    f[:, mask.astype(bool)] = 0.0
    g = tuple(rng.uniform(-1e-4, 1e-4, 2))
    return f, mask, g, float(rng.uniform(0.52, 2.0)), float(rng.uniform(0.5, 3.0))


WALLS = [(128, 37, (0, 36)),              # a channel
         (97, 33, (0, 1, 20)),            # odd width, two adjacent wall rows
         (200, 12, (5, 7)),               # one fluid row between two walls
         (130, 9, (8,)),                  # the wall's upper neighbour is row 0
         (256, 5, (2,)),
         (1000, 41, (0, 13, 14, 40)),
         (241, 20, (3, 19)),
         (3, 6, (0, 3)),                  # narrower than one window
         (121, 7, tuple(range(7))),       # every row solid
         (250, 9, ()),                    # a mask without a solid node
         (200, 2, (1,)),                  # heights of one to three rows
         (130, 1, ()),
         (97, 3, (0, 2))]
TILINGS = [(0, 0, -1), (1, 1, 0), (3, 2, 1), (8, 4, 1)]


def _equal_runs(L, nx, ny, walls, tiling, ksteps, seed, storage="f32"):
    f, mask, g, tau1, tau2 = _case(seed, nx, ny, walls)
    one = L.Lattice(nx, ny, tau1, tau2, g=g, storage=storage, mask=mask).set_populations(f)
    one.set_tuning(steps_per_sweep=1)
    assert one.tuning()[5] == 1
    many = L.Lattice(nx, ny, tau1, tau2, g=g, storage=storage, mask=mask).set_populations(f)
    many.set_tuning(*tiling, 2, 8, ksteps)
    assert many.tuning()[5] == ksteps and many.tuning()[1] <= 4
    for k in (1, 2, 5, 4, 11, 3, 6, 13):   # 45 steps: every remainder, graphs
        one.step(k)
        many.step(k)
    assert one.state()[1] == many.state()[1] == 45
    a, b = _np(one.get_populations()), _np(many.get_populations())
    say("  differs at %d of %d entries" % (int(np.sum(a != b)), a.size))
    assert np.array_equal(a, b)
    one.close()
    many.close()


@pytest.mark.parametrize("nx,ny,walls", WALLS)
@pytest.mark.parametrize("tiling", TILINGS)
@pytest.mark.parametrize("storage,ksteps", [("f32", 2), ("f32", 3), ("f16", 2)])
def test_wall_rows_multi_step_launches_equal_one_step_sweeps(L, nx, ny, walls, tiling, storage,
                                                            ksteps):
    say("case: wall rows %s in %dx%d %s, %d steps per launch, tiling=%s"
        % (walls, nx, ny, storage, ksteps, tiling))
    _equal_runs(L, nx, ny, walls, tiling, ksteps, nx + 3 * ny + len(walls), storage)


@pytest.mark.parametrize("storage,ksteps,tiling", [("f32", 2, (1, 4, 1)), ("f32", 3, (1, 4, 1)),
                                                   ("f32", 3, (2, 1, 1)), ("f16", 2, (1, 4, 1))])
def test_wall_rows_deep_pipeline_and_down_march(L, storage, ksteps, tiling):
    """At least 4096 wavefronts: the two-step pass loads two rows ahead in
    FP32 (and marches odd row blocks down), as the three-step pass does."""
    nx, ny, walls = 1000, 520, (0, 100, 101, 257, 519)
    assert -(-nx // 120) * ny >= 4096
    say("case: wall rows deep %dx%d %s, %d steps per launch, tiling=%s"
        % (nx, ny, storage, ksteps, tiling))
    _equal_runs(L, nx, ny, walls, tiling, ksteps, 7, storage)


def test_wall_rows_eligibility(L):
    """Whole solid rows allow FP32 launches of two and three steps and FP16
    launches of two (and the defaults take them); a solid node outside a
    whole row, a wall along y, FP64 storage and open x boundaries keep one
    step."""
    ny, nx = 40, 256
    rows = np.zeros((ny, nx), np.uint8)
    rows[[0, ny - 1]] = 1
    for want in (2, 3):
        lat = L.Lattice(nx, ny, 0.7, 1.0, storage="f32", mask=rows)
        lat.set_tuning(steps_per_sweep=want)
        assert lat.tuning()[5] == want
        lat.close()
    for storage in ("f32", "f16"):
        lat = L.Lattice(nx, ny, 0.7, 1.0, storage=storage, mask=rows)
        assert lat.tuning()[5] == 2                 # the default below 2048^2
        lat.set_tuning(steps_per_sweep=3)
        assert lat.tuning()[5] == (3 if storage == "f32" else 2)
        lat.close()
    part = rows.copy()
    part[0, 5] = 0
    cols = np.zeros((ny, nx), np.uint8)
    cols[:, 0] = 1
    for mask, storage in ((part, "f32"), (cols, "f32"), (part, "f16"), (rows, "f64")):
        lat = L.Lattice(nx, ny, 0.7, 1.0, storage=storage, mask=mask)
        lat.set_tuning(steps_per_sweep=3)
        assert lat.tuning()[5] == 1, storage
        lat.close()
    lat = L.Lattice(nx, ny, 0.7, 1.0, storage="f32", mask=rows, inflow=(0.01, 1.0, 1.0))
    lat.set_tuning(steps_per_sweep=3)
    assert lat.tuning()[5] == 1
    lat.close()


@pytest.mark.parametrize("storage,ksteps", [("f32", 2), ("f32", 3), ("f16", 2)])
def test_wall_row_members_in_a_batch(L, storage, ksteps):
    """A batch of channels (odd and even widths), a mask that is not whole
    rows and an open lattice advances every member to the bits of a one-step
    batch; the channels take the multi-step launches."""
    specs = [(130, 37, (0, 36)), (97, 20, (0, 1, 19)), (64, 64, None), (200, 12, (5, 7)),
             (66, 9, "part")]
    runs = {}
    for sps in (1, ksteps):
        lats = []
        for k, (nx, ny, walls) in enumerate(specs):
            if walls is None:
                f, _, g, tau1, tau2 = _case(50 + k, nx, ny, ())
                mask = None
            elif walls == "part":
                f, mask, g, tau1, tau2 = _case(50 + k, nx, ny, ())
                mask[0, :40] = 1
                f[:, mask.astype(bool)] = 0.0
            else:
                f, mask, g, tau1, tau2 = _case(50 + k, nx, ny, walls)
            lats.append(L.Lattice(nx, ny, tau1, tau2, g=g, storage=storage,
                                  mask=mask).set_populations(f))
        b = L.Batch(lats)
        b.set_tuning(steps_per_sweep=sps, graph_steps=8)
        assert b.tuning()[7] == sps
        for k in (1, 2, 5, 4, 11, 3, 8):
            b.step(k)
        b.update(lats[1:])
        b.step(7)
        b.update(lats)
        b.step(6)
        runs[sps] = [(_np(m.get_populations()), m.state()[1]) for m in lats]
        b.close()
        for m in lats:
            m.close()
    for j, ((a, ta), (c, tc)) in enumerate(zip(runs[1], runs[ksteps])):
        say("case: batch member %d %s, %d steps per launch: time %d/%d, differs at %d entries"
            % (j, storage, ksteps, ta, tc, int(np.sum(a != c))))
        assert ta == tc and np.array_equal(a, c), j


def test_wall_rows_three_steps_against_the_oracle(L):
    """A force-driven channel (32 x 24 fluid rows between walls, Sec. III.C
    set-up, g for u_c = 0.01) from a perturbed parabola, FP32 with three
    steps per launch, 300 steps: within the FP32 tolerance of the FP64
    oracle."""
    nx, n = 32, 24
    tau1 = 0.8
    tau2 = params.tau2_from_magic(tau1, 3 / 16)
    g = 8 * params.nu_from_tau(tau1) * 0.01 / n ** 2
    mask = inputs.channel_mask(nx, n)
    rho, _, uy = inputs.rest_state(n + 2, nx)
    # a parabola a little off the steady profile, plus a small cross flow
    y = np.arange(n + 2)[:, None] - (n + 1) / 2
    ux = np.clip(0.012 * (1.0 - (y / (n / 2)) ** 2), 0.0, None) * np.ones((1, nx))
    uy = 1e-3 * np.sin(2 * np.pi * np.arange(nx) / nx)[None, :] * np.ones((n + 2, 1))
    ux = np.where(mask != 0, 0.0, ux)
    uy = np.where(mask != 0, 0.0, uy)
    f0 = oracle.init_equilibrium(rho, ux, uy, mask)
    lat = L.Lattice(nx, n + 2, tau1, tau2, g=(g, 0.0), mask=mask, storage="f32")
    lat.set_tuning(steps_per_sweep=3)
    assert lat.tuning()[5] == 3
    lat.set_populations(f0).step(300)
    _, u, v = (_np(t) for t in lat.macros())
    _, ur, vr = oracle.macros(oracle.run(f0, 300, tau1, tau2, g, 0.0, mask), g, 0.0, mask)
    emax, el2 = rel_errors(u, v, ur, vr)
    say("case: channel 32x%d FP32 three steps per launch, 300 steps: rel max %.3e L2 %.3e"
        % (n, emax, el2))
    assert emax <= TOL["f32"] and el2 <= TOL["f32"]
    lat.close()
