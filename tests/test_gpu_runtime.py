"""GPU runtime behaviour: state round trips, step-graph splitting,
diagnostics, checkpoint/resume, divergence detection and batching."""
import numpy as np
import pytest

import oracle
from gpu_util import rel_errors, say
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


def test_set_get_populations_roundtrip_fp64(L):
    rng = np.random.default_rng(1)
    nx, ny = 70, 9
    mask = np.zeros((ny, nx), np.uint8)
    mask[0] = mask[-1] = 1
    mask[4, 10:13] = 1
    f = inputs.random_populations(rng, (ny, nx))
    f[:, mask.astype(bool)] = 0.0
    lat = L.Lattice(nx, ny, 0.7, 1.1, mask=mask, storage="f64").set_populations(f)
    got = _np(lat.get_populations())
    assert np.array_equal(got, f)
    lat.close()


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_set_get_populations_rounding(L, storage):
    rng = np.random.default_rng(2)
    f = inputs.random_populations(rng, (8, 33))
    lat = L.Lattice(33, 8, 0.7, 1.1, storage=storage).set_populations(f)
    got = _np(lat.get_populations())
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)[:, None, None]
    dt = np.float32 if storage == "f32" else np.float16
    want = (f - w).astype(dt).astype(np.float64) + w
    assert np.array_equal(got, want)
    lat.close()


def test_step_splitting_is_bitwise_identical(L):
    """trt_step(n) replays a captured pair of sweeps plus at most one plain
    launch; any split of the same number of steps gives the same bits."""
    n = 96
    rho, ux, uy = inputs.taylor_green(n, 0.02, seed=3)
    a = L.Lattice(n, n, 0.57, 1.9, storage="f32").init_equilibrium(rho, ux, uy)
    b = L.Lattice(n, n, 0.57, 1.9, storage="f32").init_equilibrium(rho, ux, uy)
    a.step(37)
    for k in (1, 2, 5, 1, 9, 4, 15):
        b.step(k)
    assert a.state()[1] == b.state()[1] == 37
    assert np.array_equal(_np(a.get_populations()), _np(b.get_populations()))
    a.close()
    b.close()


def test_diagnostics_match_the_oracle_and_are_reproducible(L):
    """FP64 diagnostics (mass, momentum, max |u|, min rho) equal the same
    sums over the oracle's fields of the same run, and repeat bit for bit."""
    n = 80
    rho, ux, uy = inputs.double_shear_layer(n, 0.04)
    g = (2e-5, -1e-5)
    tau1, tau2 = 0.55, 1.3
    lat = L.Lattice(n, n, tau1, tau2, g=g, storage="f64").init_equilibrium(rho, ux, uy).step(50)
    d1 = lat.diagnostics()
    d2 = lat.diagnostics()
    assert d1 == d2
    f = oracle.run(oracle.init_equilibrium(rho, ux, uy), 50, tau1, tau2, g[0], g[1])
    r, u, v = oracle.macros(f, g[0], g[1])
    say("case: diagnostics DSL 80^2 50 steps: GPU mass %.17g mom (%.6e, %.6e) | oracle mass "
        "%.17g mom (%.6e, %.6e)" % (d1["mass"], d1["mom_x"], d1["mom_y"], r.sum(),
                                    (r * u).sum(), (r * v).sum()))
    assert d1["n_fluid"] == n * n and d1["n_diverged"] == 0 and d1["time"] == 50
    assert abs(d1["mass"] - r.sum()) < 1e-11
    assert abs(d1["mom_x"] - (r * u).sum()) < 1e-12
    assert abs(d1["mom_y"] - (r * v).sum()) < 1e-12
    assert d1["max_speed"] == pytest.approx(np.max(np.hypot(u, v)), rel=1e-12)
    assert d1["min_rho"] == pytest.approx(np.min(r), rel=1e-14)
    # momentum grows by sum(rho) g per step (the collision adds F dt)
    lat.step(1)
    d3 = lat.diagnostics()
    assert d3["mom_x"] - d1["mom_x"] == pytest.approx(d1["mass"] * g[0], rel=1e-9)
    lat.close()


def test_checkpoint_resume_bitwise(L):
    n = 64
    rho, ux, uy = inputs.taylor_green(n, 0.01, seed=4)
    a = L.Lattice(n, n, 0.6, 3.0, storage="f16").init_equilibrium(rho, ux, uy).step(11)
    raw, cur, t = a.raw_state()
    a.step(13)
    ref = _np(a.get_populations())
    # restoring the raw bytes into the lattice a fresh handle reads
    # reproduces the run bit for bit
    b = L.Lattice(n, n, 0.6, 3.0, storage="f16")
    cur_b, _ = b.state()
    (b.fb if cur_b else b.fa).copy_(raw)
    b.step(13)
    assert np.array_equal(_np(b.get_populations()), ref)
    a.close()
    b.close()


def test_divergence_is_detected_from_a_forced_nan(L):
    """Divergence (non-finite, rho <= 0 or |u| >= 1) is forced from the host
    by writing a NaN population; the kernels run normally."""
    rng = np.random.default_rng(6)
    f = inputs.random_populations(rng, (16, 16))
    lat = L.Lattice(16, 16, 0.8, 1.0, storage="f32").set_populations(f)
    assert lat.check()
    f[3, 5, 7] = np.nan
    lat.set_populations(f)
    assert not lat.check()
    d = lat.diagnostics()
    assert d["n_diverged"] >= 1
    lat.step(3)
    assert lat.diagnostics()["n_diverged"] > 1
    lat.close()


def test_batch_matches_instances_alone_bitwise(L):
    """Instances of uneven size and parameters in one batch give exactly the
    bits they give alone (same launch shape)."""
    specs = [(64, 64, 0.6, 3.0), (200, 130, 0.51, 0.7), (97, 33, 1.7, 1.2), (128, 256, 0.55, 1.6),
             (131, 40, 0.8, 1.1), (385, 9, 0.7, 0.9)]
    alone, members = [], []
    for k, (nx, ny, t1, t2) in enumerate(specs):
        rng = np.random.default_rng(10 + k)
        f = inputs.random_populations(rng, (ny, nx), amp=0.05)
        a = L.Lattice(nx, ny, t1, t2, g=(1e-6 * k, 0.0), storage="f32").set_populations(f)
        m = L.Lattice(nx, ny, t1, t2, g=(1e-6 * k, 0.0), storage="f32").set_populations(f)
        a.step(3)
        m.step(3)  # members may start at odd parity
        alone.append(a)
        members.append(m)
    members[1].step(1)
    alone[1].step(1)
    batch = L.Batch(members)
    batch.step(25)
    for a in alone:
        a.step(25)
    for a, m in zip(alone, members):
        # same time step and bits; which of its two lattices holds the state
        # may differ (alone, FP32 lattices take two steps per launch)
        assert a.state()[1] == m.state()[1]
        assert np.array_equal(_np(a.get_populations()), _np(m.get_populations()))
    assert [m.tuning()[3] for m in members] == [1, 2, 1, 2, 2, 1]  # odd 131: two columns
    dg = batch.diagnostics()
    assert dg.shape == (6, 8) and np.all(dg[:, 4] == 0)
    batch.close()
    for x in alone + members:
        x.close()


def test_batch_update_changes_members_without_changing_results(L):
    """Members join and leave a batch in place (trt_batch_update): every
    lattice gets exactly the bits it gets alone, stepped the same number of
    times; a member that left may step alone again; a lattice already in
    another batch is refused."""
    from paper_2312_10318_amd import capi
    specs = [(64, 40, 0.6, 3.0), (130, 70, 0.7, 1.1), (97, 33, 1.7, 1.2), (256, 64, 0.55, 1.6)]
    mask = inputs.channel_mask(130, 68)
    alone, members = [], []
    for k, (nx, ny, t1, t2) in enumerate(specs):
        rng = np.random.default_rng(40 + k)
        f = inputs.random_populations(rng, (ny, nx), amp=0.05)
        mk = mask if nx == 130 else None
        if mk is not None:
            f[:, mk.astype(bool)] = 0.0
        alone.append(L.Lattice(nx, ny, t1, t2, mask=mk, storage="f32").set_populations(f))
        members.append(L.Lattice(nx, ny, t1, t2, mask=mk, storage="f32").set_populations(f))
    batch = L.Batch(members[:2])
    batch.step(7)                         # 0, 1: 7 steps
    batch.update(members[1:3])            # 1 stays, 0 leaves, 2 joins
    batch.step(5)                         # 1: 12, 2: 5
    members[0].step(4)                    # 0 alone again: 11
    batch.update([members[3], members[1]])
    batch.step(3)                         # 3: 3, 1: 15
    other = L.Batch([members[2]])
    with pytest.raises(capi.TrtError) as e:
        batch.update([members[2]])
    assert e.value.status == capi.TRT_ESTATE
    other.close()
    for a, n in zip(alone, (11, 15, 5, 3)):
        a.step(n)
    batch.close()
    for a, m in zip(alone, members):
        assert a.state()[1] == m.state()[1]
        assert np.array_equal(_np(a.get_populations()), _np(m.get_populations()))
    for x in alone + members:
        x.close()


def test_batch_member_cannot_step_alone(L):
    from paper_2312_10318_amd import capi
    a = L.Lattice(32, 32, 0.6, 1.0, storage="f32").init_equilibrium(*inputs.rest_state(32, 32))
    b = L.Batch([a])
    with pytest.raises(capi.TrtError) as e:
        a.step(1)
    assert e.value.status == capi.TRT_ESTATE
    b.close()
    a.step(1)
    a.close()


def test_batch_vs_oracle_mixed_workload(L):
    """A small version of the batched workload (Taylor-Green and double shear
    layer members of different sizes and relaxation times), FP32, against
    the oracle member by member."""
    members = inputs.batch_workload(6, seed=1, side_lo=32, side_hi=96, re_hi=1e4)
    lats, refs = [], []
    for k, m in enumerate(members):
        rho, ux, uy = inputs.member_fields(m, seed=k)
        lats.append(L.Lattice(m.n, m.n, m.tau1, m.tau2, storage="f32").init_equilibrium(rho, ux, uy))
        refs.append(oracle.run(oracle.init_equilibrium(rho, ux, uy), 200, m.tau1, m.tau2))
    b = L.Batch(lats)
    b.step(200)
    for lat, ref, m in zip(lats, refs, members):
        _, u, v = (_np(t) for t in lat.macros())
        _, ur, vr = oracle.macros(ref)
        emax, el2 = rel_errors(u, v, ur, vr)
        say("case: batch member %s n=%d tau1=%.4f tau2=%.3f: rel max %.3e L2 %.3e" %
            (m.kind, m.n, m.tau1, m.tau2, emax, el2))
        assert emax <= 1e-5
    b.close()


def test_full_batch_workload_sampled_members_vs_oracle(L):
    """The benchmark's batch as it is timed (256 members from the same
    generator and seeds, FP32, one launch per step, automatic launch shape):
    after 3 batched steps, sampled members (smallest, largest, odd and even
    widths, both flow kinds) match the oracle run of that member alone, and
    every member conserves its mass."""
    members = inputs.batch_workload(256, seed=0)
    lats = []
    for k, m in enumerate(members):
        rho, ux, uy = inputs.member_fields(m, seed=k)
        lats.append(L.Lattice(m.n, m.n, m.tau1, m.tau2, storage="f32").init_equilibrium(rho, ux, uy))
    b = L.Batch(lats)
    d0 = b.diagnostics()
    b.step(3)
    d1 = b.diagnostics()
    drift = np.abs(d1[:, 0] - d0[:, 0]) / d0[:, 0]
    say("case: full batch, %d members, %d nodes: max relative mass drift %.2e" %
        (len(members), sum(m.n * m.n for m in members), float(drift.max())))
    assert np.all(d1[:, 4] == 0) and np.all(d1[:, 7] == 3)
    assert float(drift.max()) <= 1e-8
    sizes = [m.n for m in members]
    pick = {int(np.argmin(sizes)), int(np.argmax(sizes))}
    pick.update([k for k, m in enumerate(members) if m.n % 2 == 1][:2])
    pick.update([k for k, m in enumerate(members) if m.n % 2 == 0 and m.n >= 128][:2])
    pick.update([k for k, m in enumerate(members) if m.n % 128 == 1][:1])
    pick.update([k for k, m in enumerate(members) if m.kind == "dsl"][:1])
    for k in sorted(pick):
        m = members[k]
        rho, ux, uy = inputs.member_fields(m, seed=k)
        ref = oracle.run(oracle.init_equilibrium(rho, ux, uy), 3, m.tau1, m.tau2)
        _, u, v = (_np(t) for t in lats[k].macros())
        _, ur, vr = oracle.macros(ref)
        emax, el2 = rel_errors(u, v, ur, vr)
        say("  member %d %s n=%d cols=%d tau1=%.4f tau2=%.3f: rel max %.3e L2 %.3e" %
            (k, m.kind, m.n, lats[k].tuning()[3], m.tau1, m.tau2, emax, el2))
        assert emax <= 1e-5
    b.close()
    for x in lats:
        x.close()


def test_batch_autotune_leaves_members_untouched_and_results_unchanged(L):
    """The batch tuner times every candidate shape on scratch copies of the
    members: the members' state is untouched, the best shape is one of the
    candidates, and a batch in that shape gives the bits of the default
    shape."""
    from paper_2312_10318_amd import autotune
    members = inputs.batch_workload(6, seed=2, side_lo=40, side_hi=300, re_hi=1e4)

    def make():
        out = []
        for k, m in enumerate(members):
            rho, ux, uy = inputs.member_fields(m, seed=k)
            out.append(L.Lattice(m.n, m.n, m.tau1, m.tau2, storage="f32")
                       .init_equilibrium(rho, ux, uy))
        return out
    a, b = make(), make()
    before = [_np(x.get_populations()) for x in a]
    res = autotune.tune_batch(a, steps=10)
    say("case: batch tuner, %d members: best %s %.4f ms" % (len(a), res["best"], res["ms"]))
    assert tuple(res["best"]) in autotune.batch_candidates()
    assert len(res["table"]) == len(autotune.batch_candidates())
    for x, f in zip(a, before):
        assert x.state()[1] == 0          # no member was stepped
        assert np.array_equal(_np(x.get_populations()), f)
    ba, bb = L.Batch(a), L.Batch(b)
    ba.set_tuning(*res["best"])
    ba.step(15)
    bb.step(15)
    for x, y in zip(a, b):
        assert np.array_equal(_np(x.get_populations()), _np(y.get_populations()))
    ba.close()
    bb.close()
    for x in a + b:
        x.close()


@pytest.mark.parametrize("sps", [1, 2, 3])
def test_longer_step_graphs_are_bitwise_identical(L, sps):
    """Every graph ladder (longest graph 2, 8, 32 sweeps or the default)
    gives the same bits for any split of the steps, including splits that
    start on the odd lattice, with one, two or three time steps per
    launch."""
    n = 96
    rho, ux, uy = inputs.taylor_green(n, 0.02, seed=5)
    runs = {}
    for g, splits in [(2, (37, 40)), (0, (77,)), (8, (1, 36, 17, 23)), (32, (77,)),
                      (32, (3, 33, 41))]:
        lat = L.Lattice(n, n, 0.57, 1.9, storage="f32").init_equilibrium(rho, ux, uy)
        lat.set_tuning(graph_steps=g, steps_per_sweep=sps)
        assert g == 0 or lat.tuning()[4] == g
        assert lat.tuning()[5] == sps
        for k in splits:
            lat.step(k)
        assert lat.state()[1] == 77
        runs[(g, splits)] = _np(lat.get_populations())
        lat.close()
    ref = runs[(2, (37, 40))]
    for key, f in runs.items():
        assert np.array_equal(f, ref), key


@pytest.mark.parametrize("sps", [1, 2, 3])
def test_prepared_step_graphs_change_nothing(L, sps):
    """trt_prepare_steps captures graphs only: state and time stay, and the
    prepared steps give the bits of unprepared ones (from either lattice)."""
    n = 96
    rho, ux, uy = inputs.taylor_green(n, 0.02, seed=6)
    out = []
    for prep in (False, True):
        lat = L.Lattice(n, n, 0.57, 1.9, storage="f32").init_equilibrium(rho, ux, uy)
        lat.set_tuning(graph_steps=8, steps_per_sweep=sps)
        for k in (29, 1, 40):
            if prep:
                before = _np(lat.get_populations()), lat.state()
                lat.prepare(k)
                assert lat.state() == before[1]
                assert np.array_equal(_np(lat.get_populations()), before[0])
            lat.step(k)
        assert lat.state()[1] == 70
        out.append(_np(lat.get_populations()))
        lat.close()
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("shape", [(0, 4, 0, 0, 16384, 2, 8), (0, 2, 1, 0, 32768, 1, 16),
                                   (16, 4, 0, 0, 0, 2, 2)])
def test_batch_tilings_orders_and_graphs_are_bitwise_identical(L, shape):
    """A batch cut into work items by a batch-wide row cap, in costliest-first
    order, or with longer captured graphs, gives every member the bits of
    the default shape."""
    members = inputs.batch_workload(7, seed=4, side_lo=40, side_hi=400, re_hi=1e4)

    def make():
        out = []
        for k, m in enumerate(members):
            rho, ux, uy = inputs.member_fields(m, seed=k)
            out.append(L.Lattice(m.n, m.n, m.tau1, m.tau2, storage="f32")
                       .init_equilibrium(rho, ux, uy))
        return out
    a, b = make(), make()
    ba, bb = L.Batch(a), L.Batch(b)
    ba.set_tuning(*shape)
    for k in (1, 22, 8):
        ba.step(k)
    bb.step(31)
    for x, y in zip(a, b):
        assert x.state()[1] == y.state()[1] == 31
        assert np.array_equal(_np(x.get_populations()), _np(y.get_populations()))
    ba.close()
    bb.close()
    for x in a + b:
        x.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_pattern_probe_moves_the_pull_rows(L, storage):
    """The access-pattern probe reads, for every lattice row y, population
    row i of source row y - e_iy and writes it to row y of the other
    lattice (the pull's row pattern), leaving every other word unchanged
    except where the edge lanes fold in the elements they read beyond the
    strip (population 1, strip columns 0 and 126)."""
    import torch
    nx, ny = 256, 11
    rng = np.random.default_rng(9)
    lat = L.Lattice(nx, ny, 0.7, 1.1, storage=storage)
    lat.set_tuning(4, 2, 1, 2)
    lat.set_populations(inputs.random_populations(rng, (ny, nx)))
    cur, _ = lat.state()
    src = (lat.fb if cur else lat.fa).clone()
    lat.pattern_probe(1)
    torch.cuda.synchronize()
    assert lat.state()[0] == 1 - cur
    dst = lat.fa if cur else lat.fb
    view = lambda t: t.cpu().numpy().view({"f64": np.uint64, "f32": np.uint32,
                                           "f16": np.uint16}[storage]).reshape(ny, 9, -1)
    a, b = view(src), view(dst)
    ey = [0, 0, 1, 0, -1, 1, 1, -1, -1]
    for i in range(9):
        want = np.roll(a[:, i, :nx], ey[i], axis=0)
        got = b[:, i, :nx]
        if i == 1:
            keep = np.ones(nx, bool)
            keep[0::128] = keep[126::128] = False
            assert np.array_equal(got[:, keep], want[:, keep])
        else:
            assert np.array_equal(got, want), i
    lat.close()


def test_library_loaded_before_torch_uses_its_runtime():
    """A process that loads the library (a footprint query) before it first
    uses PyTorch still steps a lattice: the library binds to the HIP runtime
    PyTorch ships, not to a second one that would find no GPU."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2312_10318_amd import lattice\n"
            "assert lattice.footprint_bytes(64, 64, 'f32', has_mask=True) > 0\n"
            "import numpy as np\n"
            "m = np.zeros((16, 64), np.uint8); m[0] = 1\n"
            "lat = lattice.Lattice(64, 16, 0.7, 1.0, storage='f32', mask=m)\n"
            "lat.step(5)\n"
            "print('steps', lat.state()[1], flush=True)\n"
            "lat.close()\n" % root)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=90)
    say("case: library before torch: rc %d, %s" % (r.returncode, r.stdout.strip()))
    assert r.returncode == 0, r.stderr[-2000:]
    assert "steps 5" in r.stdout
