"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake in a copy of the oracle's C source (on the CPU,
in a temporary directory), builds it, and runs the pin tests against it: at
least one pin must fail.  This is what makes the oracle trustworthy as the
reference for the GPU path.
"""
import os

import pytest

import oracle
import test_oracle_flows as flows
import test_oracle_identities as ident
import test_oracle_open as opn

MUTATIONS = {
    "G dropped": (
        "G[i] = -WGT[i] * s / (6.0 * CS2 * CS2 * CS2) * (1.0 - 1.0 / (2.0 * tau1));",
        "G[i] = 0.0 * s * tau1;"),
    "gradient sign reversed": (
        "0.5 * (phix[(long)y * nx + wrap(x + 1, nx)] - phix[(long)y * nx + wrap(x - 1, nx)])",
        "0.5 * (phix[(long)y * nx + wrap(x - 1, nx)] - phix[(long)y * nx + wrap(x + 1, nx)])"),
    "G with 2 c_s^4 but c_s^2 = 1/2": (
        "G[i] = -WGT[i] * s / (6.0 * CS2 * CS2 * CS2)",
        "G[i] = -WGT[i] * s / (6.0 * CS2 * CS2 * 0.5)"),
    "third order relaxed with tau1": (
        "(1.0 - 1.0 / tau2) * WGT[i] * r3",
        "(1.0 - 1.0 / tau1) * WGT[i] * r3 + 0.0 * tau2"),
    "third-order equilibrium term dropped": (
        "(1.0 + s1 / CS2 + s2 / (2.0 * CS2 * CS2) + s3 / (6.0 * CS2 * CS2 * CS2))",
        "(1.0 + s1 / CS2 + s2 / (2.0 * CS2 * CS2) + 0.0 * s3)"),
    "no He velocity shift": (
        "*ux_out = (j[0] + 0.5 * F[0]) / rho;",
        "*ux_out = (j[0] + 0.0 * F[0]) / rho;"),
    "force factor (1 - 1/(2 tau1)) replaced by 1": (
        "(1.0 - 1.0 / (2.0 * tau1)) * Fi[i];",
        "Fi[i];"),
    "bounce-back into the same direction": (
        "fout[(long)opp[i] * n + k] = fs[i];",
        "fout[(long)i * n + k] = fs[i];"),
    "Hermite third-order tensor sign": (
        "return (double)E[i][a] * (double)E[i][b] * (double)E[i][c] -\n           CS2 * (",
        "return (double)E[i][a] * (double)E[i][b] * (double)E[i][c] +\n           CS2 * ("),
    "streaming with x and y swapped for diagonals": (
        "const int xd = wrap(x + E[i][0], nx), yd = wrap(y + E[i][1], ny);",
        "const int xd = wrap(x + E[i][i >= 5 ? 1 : 0], nx), yd = wrap(y + E[i][i >= 5 ? 0 : 1], ny);"),
    "diagonal weight 1/36 -> 1/18 for one direction": (
        "1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};",
        "1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 18.0};"),
    "inflow wall correction with the wrong sign": (
        "fout[(long)back * n + k] = v - 2.0 * WGT[i] * rho_w * (E[i][0] * u_in) / CS2;",
        "fout[(long)back * n + k] = v + 2.0 * WGT[i] * rho_w * (E[i][0] * u_in) / CS2;"),
    "inflow wall correction without 1/c_s^2": (
        "fout[(long)back * n + k] = v - 2.0 * WGT[i] * rho_w * (E[i][0] * u_in) / CS2;",
        "fout[(long)back * n + k] = v - 2.0 * WGT[i] * rho_w * (E[i][0] * u_in);"),
    "outlet rule diagonal coefficient": (
        "fout[7 * n + k] = f[5] + 0.5 * (f[2] - f[4]) - 1.0 / 6.0 * rho_out * ux;",
        "fout[7 * n + k] = f[5] + 0.5 * (f[2] - f[4]) - 1.0 / 3.0 * rho_out * ux;"),
    "outlet rule axis coefficient": (
        "fout[3 * n + k] = f[1] - 2.0 / 3.0 * rho_out * ux;",
        "fout[3 * n + k] = f[1] - 1.0 / 3.0 * rho_out * ux;"),
    "outlet ghost Phi taken as 0": (
        "if (open_x && x == nx - 1) right = px[k];",
        "if (open_x && x == nx - 1) right = 0.0;"),
    "inlet ghost Phi taken periodic": (
        "if (open_x && x == 0) left = rho_w * u_in * u_in * u_in;",
        "if (open_x && x == 0) left = left + 0.0 * rho_w;"),
    "wall force without the returned population": (
        "fx += E[i][0] * (fstar[(long)i * n + k] + returned);",
        "fx += E[i][0] * (fstar[(long)i * n + k] + 0.0 * returned);"),
    "second-order projection coefficient 1/c_s^4": (
        "(1.0 - 1.0 / tau1) * WGT[i] * r2 / (2.0 * CS2 * CS2)",
        "(1.0 - 1.0 / tau1) * WGT[i] * r2 / (CS2 * CS2)"),
}


def _battery(o):
    """Run the pins against oracle instance ``o``; return the names that failed."""
    failed = []
    checks = [
        ("eq moments", lambda: ident.test_equilibrium_moments(o, 0)),
        ("source moments", lambda: ident.test_source_moments(o, 0)),
        ("He shift", lambda: ident.test_moments_with_he_shift(o, 0)),
        ("conservation", lambda: ident.test_collision_conserves_mass_and_adds_force(o, 0)),
        ("change of basis", lambda: ident.test_collision_equals_hermite_change_of_basis(o, 0)),
        ("poiseuille", lambda: flows.test_poiseuille_profile_plus_slip(o, 4, 8, 0.6, 1 / 12)),
        ("mass", lambda: flows.test_mass_is_conserved_exactly_with_walls(o)),
        ("momentum", lambda: flows.test_periodic_momentum_grows_by_the_force(o)),
        ("rotation", lambda: flows.test_rotation_symmetry(o)),
        ("sound", lambda: flows.test_sound_attenuation_is_galilean_invariant(o)),
        ("uniform inflow", lambda: opn.test_uniform_inflow_is_a_fixed_point(o, 0.03, 0.8)),
        ("outlet moments", lambda: opn.test_outlet_density_and_transverse_momentum(o, 0.97)),
        ("wall force", lambda: opn.test_wall_force_balances_body_force_at_steady_state(o, 4e-5)),
        ("open ends", lambda: opn.test_open_ends_do_not_see_each_other(o)),
    ]
    for name, fn in checks:
        try:
            fn()
        except (AssertionError, MemoryError, FloatingPointError, ValueError):
            failed.append(name)
    return failed


def test_unmutated_oracle_passes_the_battery(orc):
    assert _battery(oracle.Oracle()) == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTATIONS[name]
    src = oracle.source_text()
    assert src.count(old) == 1, "mutation target not found: " + name
    lib = oracle.build_variant(src.replace(old, new), os.path.join(str(tmp_path), "mut.so"))
    failed = _battery(oracle.Oracle(lib))
    assert failed, "no pin caught: " + name
