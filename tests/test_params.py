"""Host-side parameter relations pinned to the values the paper prints."""
import math
import os

import pytest

from paper_2312_10318_amd import params

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_creeping_flow.txt")


def _rows():
    with open(GOLDEN) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                yield line.split()


@pytest.mark.parametrize("row", list(_rows()))
def test_table1_relaxation_times(row):
    """Sec. III.D, Table 1: with T = 0.1 and D = 21, Ma = sqrt(T Re),
    u = Ma c_s, nu = u D / Re and tau_s1 = 3 nu + 1/2 reproduce the printed
    Ma, Kn (= Ma / Re) and tau_s1 columns."""
    re, ma_p, kn_p, tau_p = float(row[0]), float(row[1]), float(row[2]), int(row[3])
    ma = params.mach_from_T(0.1, re)
    assert float("%.3g" % ma) == pytest.approx(ma_p, rel=1e-12)
    assert float("%.3g" % (ma / re)) == pytest.approx(kn_p, rel=1e-12)
    tau1 = params.tau_from_re(params.u_from_mach(ma), 21.0, re)
    assert round(tau1) == tau_p


def test_magic_parameter_roundtrip_and_zero_slip_value():
    """Sec. II.D: the slip factor 16 tau1 tau2 - 8 tau1 - 8 tau2 + 1 equals
    16 Lambda_s - 3, so it vanishes at Lambda_s = 3/16."""
    for tau1 in (0.51, 0.6, 1.0, 3.7, 100.0):
        tau2 = params.tau2_from_magic(tau1, 3 / 16)
        assert params.magic(tau1, tau2) == pytest.approx(3 / 16, rel=1e-14)
        assert abs(16 * tau1 * tau2 - 8 * tau1 - 8 * tau2 + 1) < 1e-12 * tau1 * tau2


def test_viscosity_relation():
    """Sec. II.C: mu = rho c_s^2 (tau_s1 - 1/2) dt, c_s^2 = 1/3."""
    assert params.nu_from_tau(0.6) == pytest.approx(0.1 / 3, rel=1e-15)
    assert params.tau_from_nu(params.nu_from_tau(1.7)) == pytest.approx(1.7, rel=1e-15)
    with pytest.raises(ValueError):
        params.tau2_from_magic(0.5, 0.25)
    assert math.isclose(params.u_from_mach(1.0), 1 / math.sqrt(3))
