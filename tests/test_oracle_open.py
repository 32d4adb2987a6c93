"""Pins of the oracle's open boundaries (inflow wall, pressure outlet) and
momentum exchange with solid nodes (the creeping-flow case of Sec. III.D).

* A uniform flow u = (u0, 0), rho = 1 with an inflow wall moving at u0 and an
  outlet held at rho = 1 is an exact steady solution of the scheme: the
  equilibrium is a collision fixed point, the moving-wall return reproduces
  the incoming equilibrium populations exactly (their difference to the
  outgoing ones is 2 w_i rho e_i.u / c_s^2 when u_y = 0), Zou and He's rule
  returns equilibrium values for an equilibrium input, and Phi is uniform.
* Zou and He's rule imposes the outlet density and zero transverse momentum
  on any state.
* At the steady state of a force-driven channel the momentum handed to the
  walls per step equals the momentum the body force adds (sum of rho g).
* The open ends do not see each other: one step moves information by one
  node, so with open x boundaries the first column cannot depend on the last
  columns, nor the last column on the first ones (no periodic leakage
  through streaming or through the Phi gradient).
"""
import numpy as np
import pytest

from paper_2312_10318_amd import inputs, params


def _uniform(nx, ny, u0):
    return (np.ones((ny, nx)), np.full((ny, nx), u0), np.zeros((ny, nx)))


@pytest.mark.parametrize("u0,tau1", [(0.03, 0.8), (0.05, 0.55), (1e-3, 37.0)])
def test_uniform_inflow_is_a_fixed_point(orc, u0, tau1):
    nx, ny = 12, 5
    tau2 = params.tau2_from_magic(tau1, 3 / 16)
    f0 = orc.init_equilibrium(*_uniform(nx, ny, u0))
    f = orc.run_open(f0, 5, tau1, tau2, u_in=u0, rho_w=1.0, rho_out=1.0)
    assert np.max(np.abs(f - f0)) < 4e-16


def test_uniform_inflow_with_an_obstacle_is_not_a_fixed_point(orc):
    """Control for the test above: the same run with an obstacle changes
    the state (the fixed point is not an artefact of a no-op step)."""
    nx, ny, u0 = 12, 7, 0.03
    mask = np.zeros((ny, nx), np.uint8)
    mask[3, 6] = 1
    f0 = orc.init_equilibrium(*_uniform(nx, ny, u0), mask=mask)
    f = orc.run_open(f0, 3, 0.8, 1.0, u_in=u0, mask=mask)
    assert np.max(np.abs(f - f0)) > 1e-4


@pytest.mark.parametrize("rho_out", [1.0, 0.97])
def test_outlet_density_and_transverse_momentum(orc, rho_out):
    rng = np.random.default_rng(3)
    nx, ny = 9, 6
    f = inputs.random_populations(rng, (ny, nx), amp=0.1)
    out = orc.step_open(f, 0.7, 1.3, u_in=0.02, rho_w=1.0, rho_out=rho_out)
    col = out[:, :, -1]
    ey = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
    assert np.max(np.abs(col.sum(axis=0) - rho_out)) < 1e-15
    assert np.max(np.abs(np.tensordot(ey, col, axes=1))) < 1e-16


@pytest.mark.parametrize("g", [1e-5, 4e-5])
def test_wall_force_balances_body_force_at_steady_state(orc, g):
    nx, n_fluid, tau1 = 4, 8, 0.8
    tau2 = params.tau2_from_magic(tau1, 3 / 16)
    mask = inputs.channel_mask(nx, n_fluid)
    f = orc.init_equilibrium(*inputs.rest_state(n_fluid + 2, nx), mask=mask)
    f = orc.run(f, 6000, tau1, tau2, g, 0.0, mask)
    rho, _, _ = orc.macros(f, g, 0.0, mask)
    fx, fy = orc.wall_force(f, tau1, tau2, g, 0.0, mask)
    added = g * rho[mask == 0].sum()
    assert fx == pytest.approx(added, rel=1e-10)
    # top and bottom walls push with equal and opposite pressure forces of O(1)
    assert abs(fy) < 1e-13


def test_open_ends_do_not_see_each_other(orc):
    rng = np.random.default_rng(5)
    nx, ny = 10, 6
    a = inputs.random_populations(rng, (ny, nx), amp=0.1)
    b = a.copy()
    b[:, :, -2:] = inputs.random_populations(rng, (ny, 2), amp=0.1)
    c = a.copy()
    c[:, :, :2] = inputs.random_populations(rng, (ny, 2), amp=0.1)
    kw = dict(u_in=0.04, rho_w=1.0, rho_out=1.0)
    sa, sb, sc = (orc.step_open(f, 0.7, 1.2, **kw) for f in (a, b, c))
    assert np.array_equal(sa[:, :, 0], sb[:, :, 0])
    assert np.array_equal(sa[:, :, -1], sc[:, :, -1])
    # control: the columns next to the changed ones do change
    assert not np.array_equal(sa[:, :, -3], sb[:, :, -3])


def test_collide_then_stream_open_is_step_open(orc):
    """The two halves the oracle exposes compose to its open step exactly."""
    rng = np.random.default_rng(11)
    nx, ny = 14, 9
    mask = np.zeros((ny, nx), np.uint8)
    mask[3:5, 6:8] = 1
    f = inputs.random_populations(rng, (ny, nx))
    f[:, mask.astype(bool)] = 0.0
    tau1, tau2, u = 0.7, 1.3, 0.02
    want = orc.step_open(f, tau1, tau2, u, 1.01, 0.99, 1e-5, -2e-6, mask)
    fs = orc.collide(f, tau1, tau2, 1e-5, -2e-6, mask, True, u, 1.01)
    assert np.array_equal(orc.stream_open(fs, u, 1.01, 0.99, mask), want)
    assert np.all(fs[:, mask.astype(bool)] == 0.0)


def test_periodic_collide_streams_into_step(orc):
    """Without solids, rolling each post-collision plane by e_i gives the
    periodic step exactly."""
    rng = np.random.default_rng(12)
    f = inputs.random_populations(rng, (7, 10))
    tau1, tau2, gx, gy = 0.65, 2.0, 3e-6, 1e-6
    fs = orc.collide(f, tau1, tau2, gx, gy)
    want = orc.step(f, tau1, tau2, gx, gy)
    ex = [0, 1, 0, -1, 0, 1, -1, -1, 1]
    ey = [0, 0, 1, 0, -1, 1, 1, -1, -1]
    got = np.stack([np.roll(fs[i], (ey[i], ex[i]), axis=(0, 1)) for i in range(9)])
    assert np.array_equal(got, want)
