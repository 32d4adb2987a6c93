"""Two time steps per launch (trt_tuning.steps_per_sweep = 2) give the bits
of the one-step sweep, FP32 and FP16: every node's arithmetic is the same
and the first step's results are exactly what the one-step sweep stores and
loads back (FP16: rounded to the stored words in registers).  Ragged and tiny heights (row blocks that wrap past the lattice), one
and several strips, widths that are not multiples of the stored window
(windows that wrap, a last window only partly inside the lattice, lattices
narrower than one window), odd widths (pairs across the wrap and on odd
columns), every row and workgroup shape, odd step counts;
and the same run against the oracle within the FP32 tolerance."""
import numpy as np
import pytest

import oracle
from gpu_util import TOL, rel_errors, say, stored_state
from paper_2312_10318_amd import inputs

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


def _state(seed, nx, ny):
    rng = np.random.default_rng(seed)
    f = inputs.random_populations(rng, (ny, nx), amp=0.05)
    g = tuple(rng.uniform(-1e-4, 1e-4, 2))
    return f, g, float(rng.uniform(0.52, 2.0)), float(rng.uniform(0.5, 3.0))


@pytest.mark.parametrize("nx,ny", [(128, 37), (256, 9), (384, 130), (128, 3), (256, 5),
                                   (512, 64), (200, 37), (250, 9), (130, 66), (6, 5), (2, 4),
                                   (1000, 41), (362, 1), (201, 37), (97, 33), (241, 20),
                                   (121, 7), (127, 9), (129, 4), (1, 5), (3, 6), (5, 3),
                                   (999, 12)])
@pytest.mark.parametrize("tiling", [(0, 0, -1), (1, 1, 0), (3, 2, 1), (8, 4, 1), (64, 4, 0)])
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_two_steps_per_launch_equal_one_step_sweeps(L, nx, ny, tiling, storage):
    f, g, tau1, tau2 = _state(nx + 7 * ny, nx, ny)
    say("case: two steps per launch %dx%d %s tiling=%s" % (nx, ny, storage, tiling))
    one = L.Lattice(nx, ny, tau1, tau2, g=g, storage=storage).set_populations(f)
    one.set_tuning(steps_per_sweep=1)
    assert one.tuning()[5] == 1
    two = L.Lattice(nx, ny, tau1, tau2, g=g, storage=storage).set_populations(f)
    two.set_tuning(*tiling, 2, 8, 2)
    assert two.tuning()[5] == 2 and two.tuning()[1] <= 4   # at most four wavefronts
    for k in (1, 2, 5, 4, 11, 3):   # 26 steps: singles, two-step launches, graphs
        one.step(k)
        two.step(k)
    assert one.state()[1] == two.state()[1] == 26
    a, b = _np(one.get_populations()), _np(two.get_populations())
    say("  differs at %d of %d entries" % (int(np.sum(a != b)), a.size))
    assert np.array_equal(a, b)
    one.close()
    two.close()


@pytest.mark.parametrize("nx,ny", [(128, 37), (256, 9), (384, 130), (128, 3), (232, 5),
                                   (512, 64), (200, 37), (250, 9), (130, 66), (6, 5), (2, 4),
                                   (1000, 41), (362, 1), (201, 37), (97, 33), (241, 20),
                                   (117, 7), (115, 9), (116, 4), (1, 5), (3, 6), (5, 3),
                                   (999, 12), (4096, 73)])
@pytest.mark.parametrize("tiling", [(0, 0, -1), (1, 1, 0), (3, 2, 1), (8, 4, 1), (64, 4, 0)])
def test_three_steps_per_launch_equal_one_step_sweeps(L, nx, ny, tiling):
    """FP32 three steps per launch (116 stored columns of a 128-column
    window, odd row blocks marching down): the bits of one-step sweeps."""
    f, g, tau1, tau2 = _state(nx + 5 * ny, nx, ny)
    say("case: three steps per launch %dx%d tiling=%s" % (nx, ny, tiling))
    one = L.Lattice(nx, ny, tau1, tau2, g=g, storage="f32").set_populations(f)
    one.set_tuning(steps_per_sweep=1)
    three = L.Lattice(nx, ny, tau1, tau2, g=g, storage="f32").set_populations(f)
    three.set_tuning(*tiling, 2, 8, 3)
    assert three.tuning()[5] == 3 and three.tuning()[6] == 1 and three.tuning()[1] <= 4
    for k in (1, 2, 5, 4, 11, 3, 6, 13):   # 45 steps: every remainder, graphs
        one.step(k)
        three.step(k)
    assert one.state()[1] == three.state()[1] == 45
    a, b = _np(one.get_populations()), _np(three.get_populations())
    say("  differs at %d of %d entries" % (int(np.sum(a != b)), a.size))
    assert np.array_equal(a, b)
    one.close()
    three.close()


def test_three_steps_per_launch_apply_to_fp32_alone(L):
    """FP16 lattices asked for three steps per launch take two, FP64 ones
    and masked ones whose solid nodes do not fill whole rows one (FP32 wall
    rows take three); a batch of FP32 members takes three by default (two
    when asked), an FP16 batch two."""
    for storage, want in (("f32", 3), ("f16", 2), ("f64", 1)):
        lat = L.Lattice(256, 64, 0.7, 1.0, storage=storage)
        lat.set_tuning(steps_per_sweep=3)
        assert lat.tuning()[5] == want, storage
        lat.close()
    mask = np.zeros((64, 256), np.uint8)
    mask[0] = mask[-1] = 1
    for m, want in ((mask, 3), (np.roll(mask, 1, axis=1) * (np.arange(256) > 3), 1)):
        lat = L.Lattice(256, 64, 0.7, 1.0, storage="f32", mask=m)
        lat.set_tuning(steps_per_sweep=3)
        assert lat.tuning()[5] == want
        lat.close()
    for storage, want in (("f32", 3), ("f16", 2)):
        lats = [L.Lattice(n, n, 0.7, 1.0, storage=storage) for n in (64, 130)]
        b = L.Batch(lats)
        assert b.tuning()[7] == want
        b.set_tuning(steps_per_sweep=2)
        assert b.tuning()[7] == 2
        b.set_tuning(steps_per_sweep=3)
        assert b.tuning()[7] == want and b.tuning()[8] == 1
        b.close()
        for l in lats:
            l.close()


# Launches of at least 4096 wavefronts load two rows ahead, and in FP32 their
# odd row blocks march down the block instead of up: an even and an odd
# number of row blocks, a last block shorter than the rest, an odd width.
@pytest.mark.parametrize("nx,ny,tiling", [((1000, 520, (1, 4, 1))), ((4096, 391, (3, 4, 1))),
                                          ((2047, 1001, (4, 4, 0))), ((2048, 1030, (4, 2, 1)))])
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_deep_two_step_launches_equal_one_step_sweeps(L, nx, ny, tiling, storage):
    f, g, tau1, tau2 = _state(nx + 3 * ny, nx, ny)
    windows = -(-nx // 120)
    assert windows * -(-ny // tiling[0]) >= 4096   # the deep pipeline
    say("case: deep two-step launches %dx%d %s tiling=%s" % (nx, ny, storage, tiling))
    one = L.Lattice(nx, ny, tau1, tau2, g=g, storage=storage).set_populations(f)
    one.set_tuning(steps_per_sweep=1)
    two = L.Lattice(nx, ny, tau1, tau2, g=g, storage=storage).set_populations(f)
    two.set_tuning(*tiling, 2, 8, 2)
    assert two.tuning()[:2] == tiling[:2] and two.tuning()[5] == 2
    for k in (1, 2, 5, 4, 11, 3):
        one.step(k)
        two.step(k)
    a, b = _np(one.get_populations()), _np(two.get_populations())
    say("  differs at %d of %d entries" % (int(np.sum(a != b)), a.size))
    assert np.array_equal(a, b)
    one.close()
    two.close()


def test_two_steps_per_launch_against_the_oracle(L):
    nx, ny, steps = 256, 70, 40
    f, g, tau1, tau2 = _state(3, nx, ny)
    lat = L.Lattice(nx, ny, tau1, tau2, g=g, storage="f32").set_populations(f)
    lat.set_tuning(steps_per_sweep=2)
    lat.step(steps)
    _, u, v = (_np(t) for t in lat.macros())
    lat.close()
    fo = oracle.run(stored_state(f, "f32"), steps, tau1, tau2, g[0], g[1])
    _, ur, vr = oracle.macros(fo, g[0], g[1])
    emax, el2 = rel_errors(u, v, ur, vr)
    say("case: two steps per launch %dx%d, %d steps vs oracle: rel max %.3e L2 %.3e"
        % (nx, ny, steps, emax, el2))
    assert emax <= TOL["f32"] and el2 <= TOL["f32"]


def test_three_steps_per_launch_against_the_oracle(L):
    nx, ny, steps = 256, 70, 42
    f, g, tau1, tau2 = _state(4, nx, ny)
    lat = L.Lattice(nx, ny, tau1, tau2, g=g, storage="f32").set_populations(f)
    lat.set_tuning(steps_per_sweep=3)
    assert lat.tuning()[5] == 3
    lat.step(steps)
    _, u, v = (_np(t) for t in lat.macros())
    lat.close()
    fo = oracle.run(stored_state(f, "f32"), steps, tau1, tau2, g[0], g[1])
    _, ur, vr = oracle.macros(fo, g[0], g[1])
    emax, el2 = rel_errors(u, v, ur, vr)
    say("case: three steps per launch %dx%d, %d steps vs oracle: rel max %.3e L2 %.3e"
        % (nx, ny, steps, emax, el2))
    assert emax <= TOL["f32"] and el2 <= TOL["f32"]


def test_two_steps_per_launch_fp16_one_launch_against_the_oracle(L):
    """FP16: one two-step launch from a state held in FP16 against two oracle
    steps from the same state, within the FP16 tolerance (the first step's
    results are rounded to FP16 in registers, as a store would)."""
    nx, ny = 256, 70
    f, g, tau1, tau2 = _state(5, nx, ny)
    lat = L.Lattice(nx, ny, tau1, tau2, g=g, storage="f16").set_populations(f)
    assert lat.tuning()[5] == 2
    lat.step(2)
    _, u, v = (_np(t) for t in lat.macros())
    lat.close()
    fo = oracle.run(stored_state(f, "f16"), 2, tau1, tau2, g[0], g[1])
    _, ur, vr = oracle.macros(fo, g[0], g[1])
    emax, el2 = rel_errors(u, v, ur, vr)
    say("case: FP16 two steps per launch %dx%d vs oracle: rel max %.3e L2 %.3e"
        % (nx, ny, emax, el2))
    assert emax <= TOL["f16"] and el2 <= TOL["f16"]


def test_two_steps_per_launch_applies_only_where_eligible(L):
    """FP64 storage and masks keep one step per launch (and say so) -- but
    for wall rows, which take two; every width takes two."""
    cases = [dict(nx=256, ny=8, storage="f64"), dict(nx=201, ny=8, storage="f64")]
    for c in cases:
        lat = L.Lattice(c["nx"], c["ny"], 0.7, 1.0, storage=c["storage"])
        lat.set_tuning(steps_per_sweep=2)
        assert lat.tuning()[5] == 1, c
        lat.close()
    for nx in (201, 1, 3):
        for storage in ("f32", "f16"):
            lat = L.Lattice(nx, 8, 0.7, 1.0, storage=storage)
            assert lat.tuning()[5] == 2, (nx, storage)
            lat.close()
    mask = np.zeros((8, 256), np.uint8)
    mask[0] = 1
    part = mask.copy()
    part[0, 200:] = 0
    for m, storage, want in ((mask, "f32", 2), (mask, "f16", 2), (part, "f32", 1),
                             (part, "f16", 1)):
        lat = L.Lattice(256, 8, 0.7, 1.0, storage=storage, mask=m)
        lat.set_tuning(steps_per_sweep=2)
        assert lat.tuning()[5] == want, storage
        lat.close()


def test_steps_per_launch_default_and_reported_shape(L):
    """Unless asked otherwise, FP32 lattices of at least 2048^2 nodes take
    three steps per launch and other eligible ones two.  The reported rows,
    wavefronts and prefetch rows are those of the pass in effect: two steps
    -- 120-column windows, the longest rows of 32 down to 8 that give 6144
    wavefronts (else 2048), four-wavefront workgroups from 4096 wavefronts
    on, loads two rows ahead in FP32 from 4096 wavefronts on; three steps --
    116-column windows, the rows that make four-wavefront workgroups fill
    the machine in the fewest whole rounds with 8 to 192 rows (XCD
    round-robin), else rows of 48 down to 16 for 3072 wavefronts (four per
    workgroup, XCD round-robin; else rows down to 8 for 1536, one per
    workgroup, XCD bands), loads one row ahead; an
    explicit request is kept (at most four wavefronts, no more than the
    windows need)."""
    cases = [((4096, 4096), (), "f32", (74, 4, 1, 3)), ((4096, 4096), (), "f16", (16, 4, 1, 2)),
             ((8192, 8192), (), "f32", (147, 4, 1, 3)), ((2048, 2048), (), "f32", (21, 4, 1, 3)),
             ((3000, 3000), (), "f32", (42, 4, 1, 3)),
             ((1024, 1024), (), "f32", (8, 1, 1, 2)), ((256, 8), (), "f32", (8, 1, 1, 2)),
             ((4096, 64), (5, 16), "f32", (5, 4, 1, 2)), ((240, 64), (16, 4), "f32", (16, 2, 1, 2)),
             ((4096, 4096), (0, 0, 1, 0, 0, 2), "f32", (16, 4, 2, 2)),
             ((4096, 4096), (0, 0, 1, 0, 0, 2, 1), "f32", (16, 4, 1, 2)),
             ((4096, 4096), (0, 0, 1, 0, 0, 0, 2), "f16", (16, 4, 2, 2)),
             ((1024, 1024), (0, 0, 1, 0, 0, 3), "f32", (8, 1, 1, 3)),
             ((4096, 4096), (32, 2, 1, 0, 0, 3, 2), "f32", (32, 2, 1, 3))]
    for (nx, ny), asked, storage, want in cases:
        lat = L.Lattice(nx, ny, 0.7, 1.0, storage=storage)
        lat.set_tuning(*asked)
        got = lat.tuning()
        say("case: %dx%d %s asked %s -> rows %d waves %d prefetch %d steps %d"
            % (nx, ny, storage, asked, got[0], got[1], got[6], got[5]))
        assert (got[0], got[1], got[6], got[5]) == want
        if not asked and want[3] == 3:
            assert got[2] == (0 if want[1] == 4 else 1)   # XCD order of the three-step pass
        rows, waves = (tuple(asked) + (0, 0))[:2]
        lat.set_tuning(rows, waves, -1, 0, 0, 1)
        assert lat.tuning()[5] == 1 and lat.tuning()[6] == 0
        lat.close()



@pytest.mark.parametrize("storage,ksteps", [("f32", 2), ("f16", 2), ("f32", 3)])
def test_batch_two_step_members_equal_one_step_batches(L, storage, ksteps):
    """A batch whose members mix k-step members (even and odd widths) with a
    one-step one (a mask) advances every member to the bits a one-step
    batch gives, over odd and even splits, graph ladders and a membership
    change; the batch reports k steps per launch only while a member takes
    them."""
    specs = [(64, 64), (200, 37), (97, 33), (128, 130), (131, 40), (250, 9), (66, 3)]
    mask = np.zeros((37, 200), np.uint8)
    mask[0, :150] = 1   # not a whole row: one step per launch
    runs = {}
    for sps in (1, ksteps):
        lats = []
        for k, (nx, ny) in enumerate(specs):
            f, g, tau1, tau2 = _state(100 + k, nx, ny)
            mk = mask if k == 1 else None
            if mk is not None:
                f = f.copy()
                f[:, mk.astype(bool)] = 0.0
            lats.append(L.Lattice(nx, ny, tau1, tau2, g=g, storage=storage,
                                  mask=mk).set_populations(f))
        b = L.Batch(lats)
        b.set_tuning(steps_per_sweep=sps, graph_steps=8)
        assert b.tuning()[7] == sps
        for k in (1, 2, 5, 4, 11, 3, 8):
            b.step(k)
        b.update(lats[2:])
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
    # only one-step members: the batch takes one step per launch
    wall = np.zeros((8, 64), np.uint8)
    wall[0, :40] = 1
    lats = [L.Lattice(64, 8, 0.7, 1.0, storage=storage, mask=wall),
            L.Lattice(64, 8, 0.9, 1.0, storage=storage, mask=wall)]
    b = L.Batch(lats)
    assert b.tuning()[7] == 1
    b.close()
    for m in lats:
        m.close()
