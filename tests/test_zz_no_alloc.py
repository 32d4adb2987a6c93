"""trt_diagnostics_noalloc (reduction partials in a static device array, no
allocation) against trt_diagnostics on the same state: bitwise equal, on two
calls in a row, the second with a smaller lattice; each also against the
oracle's mass and momentum sums."""
import ctypes

import numpy as np
import pytest

import oracle
from gpu_util import say
from paper_2312_10318_amd import capi, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_10318_amd import lattice
    return lattice


def _noalloc(lat):
    import torch
    cur, t = lat.state()
    lattice = lat.fb if cur else lat.fa
    out = torch.full((capi.TRT_NDIAG,), float("nan"), dtype=torch.float64, device=lat.device)
    capi.trt_diagnostics_noalloc(lat.prob, lattice.data_ptr(), t, out.data_ptr(),
                                 lat.stream.cuda_stream)
    lat.stream.synchronize()
    return out.cpu().numpy()


def _case_obstacle_open_f64(L):
    nx, ny, steps = 230, 130, 41
    mask = np.zeros((ny, nx), np.uint8)
    mask[50:71, 60:81] = 1
    rho = np.ones((ny, nx))
    ux = np.full((ny, nx), 0.02)
    uy = np.zeros((ny, nx))
    ux[mask.astype(bool)] = 0.0
    lat = L.Lattice(nx, ny, 0.8, 1.3, mask=mask, storage="f64", inflow=(0.02, 1.0, 1.0))
    lat.init_equilibrium(rho, ux, uy).step(steps)
    f = oracle.run_open(oracle.init_equilibrium(rho, ux, uy, mask), steps, 0.8, 1.3, 0.02, 1.0,
                        1.0, mask=mask)
    r, u, v = oracle.macros(f, mask=mask)
    return lat, (r.sum(), (r * u).sum(), (r * v).sum(), int((mask == 0).sum())), (1e-13, 1e-12)


def _case_channel_f32(L):
    nx, nf, steps = 70, 22, 29
    mask = inputs.channel_mask(nx, nf)
    rho, ux, uy = inputs.rest_state(nf + 2, nx)
    g = 2e-5
    lat = L.Lattice(nx, nf + 2, 0.9, 1.2, g=(g, 0.0), mask=mask, storage="f32")
    lat.init_equilibrium(rho, ux, uy).step(steps)
    f = oracle.run(oracle.init_equilibrium(rho, ux, uy, mask), steps, 0.9, 1.2, g, 0.0, mask)
    r, u, v = oracle.macros(f, g, 0.0, mask)
    return lat, (r.sum(), (r * u).sum(), (r * v).sum(), int((mask == 0).sum())), (1e-10, 1e-5)


def test_noalloc_diagnostics_equal_the_allocating_call(L):
    for make in (_case_obstacle_open_f64, _case_channel_f32):
        lat, (mass, mx, my, nfluid), (tol_mass, tol) = make(L)
        say("noalloc diagnostics: %dx%d %s" % (lat.nx, lat.ny, lat.storage))
        want = lat.diagnostics()
        got = _noalloc(lat)
        ref = np.array([want[k] for k in lattice_names()])
        assert np.array_equal(got, ref), (got, ref)
        # and the sums themselves against the oracle's fields
        assert got[5] == nfluid and got[4] == 0
        say("  mass %.17g (oracle %.17g), momentum (%.6e, %.6e) (oracle %.6e, %.6e)"
            % (got[0], mass, got[1], got[2], mx, my))
        assert abs(got[0] - mass) <= tol_mass * mass
        scale = max(abs(mx), abs(my), 1e-300)
        assert abs(got[1] - mx) <= tol * scale and abs(got[2] - my) <= tol * scale
        lat.close()


def lattice_names():
    from paper_2312_10318_amd.lattice import DIAG_NAMES
    return DIAG_NAMES


def test_noalloc_rejects_invalid_arguments_without_touching_the_device(L):
    p = capi.trt_problem(16, 16, 0.6, 1.0, 0.0, 0.0, None, 1)
    lib = capi.load()
    assert lib.trt_diagnostics_noalloc(ctypes.byref(p), None, 0, None, None) == capi.TRT_EINVAL
