"""The C ABI library loads without a GPU, exports every symbol its header
declares, and validates arguments before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2312_10318_amd import capi, lattice

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "trtlbm.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(trt_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(capi.LIB_PATH):
        from paper_2312_10318_amd import build
        build.build()
    return capi.load()


def test_every_declared_symbol_is_exported(lib):
    declared = _declared()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(capi.EXPORTED) == declared


def test_pitch_and_sizes(lib):
    assert capi.trt_pitch(4096, capi.TRT_F32_SHIFTED) == 4096
    assert capi.trt_pitch(400, capi.TRT_F32_SHIFTED) == 448
    assert capi.trt_pitch(400, capi.TRT_F64) == 416
    assert capi.trt_pitch(400, capi.TRT_F16_SHIFTED) == 512
    assert capi.trt_pitch(0, capi.TRT_F64) == -1
    assert capi.trt_pitch(5, 7) == -1
    assert capi.trt_row_stride(64, capi.TRT_F64) == 9 * 64
    assert capi.trt_row_stride(400, capi.TRT_F16_SHIFTED) == 9 * 512
    assert capi.trt_row_stride(0, capi.TRT_F64) == -1
    p = lattice.problem(4096, 4096, 0.6, 3.0, storage="f32")
    assert capi.trt_lattice_bytes(p) == 9 * 4096 * 4096 * 4
    assert capi.trt_footprint_bytes(p) >= 2 * 9 * 4096 * 4096 * 4
    assert lattice.footprint_bytes(400, 200, "f16", has_mask=True) >= 2 * 9 * 512 * 200 * 2 + 80000


@pytest.mark.parametrize("kw,msg", [
    (dict(nx=0), "nx and ny"),
    (dict(ny=50000), "nx and ny"),
    (dict(tau_s=0.5), "tau_s"),
    (dict(tau_s=float("nan")), "tau_s"),
    (dict(tau_s2=0.49), "tau_s2"),
    (dict(gx=float("inf")), "g must be finite"),
    (dict(storage=9), "storage"),
])
def test_create_rejects_invalid_problems(lib, kw, msg):
    args = dict(nx=16, ny=16, tau_s=0.6, tau_s2=1.0, gx=0.0, gy=0.0, storage=1)
    args.update(kw)
    p = capi.trt_problem(args["nx"], args["ny"], args["tau_s"], args["tau_s2"], args["gx"],
                         args["gy"], None, args["storage"])
    with pytest.raises(capi.TrtError) as e:
        capi.trt_create(p, 4096, 8192, 0)
    assert e.value.status == capi.TRT_EINVAL
    assert msg in str(e.value)
    assert capi.trt_lattice_bytes(p) == 0


def test_create_rejects_bad_buffers(lib):
    p = capi.trt_problem(16, 16, 0.6, 1.0, 0.0, 0.0, None, 1)
    for a, b, msg in [(0, 1 << 20, "required"), (256 + 4, 1 << 20, "aligned"),
                      (1 << 20, (1 << 20) + 256, "overlap")]:
        with pytest.raises(capi.TrtError) as e:
            capi.trt_create(p, a, b, 0)
        assert e.value.status == capi.TRT_EINVAL and msg in str(e.value)


def test_null_handles_are_rejected(lib):
    for fn, args in [(lib.trt_step, (None, 1)), (lib.trt_macros, (None, None, None, None)),
                     (lib.trt_diagnostics, (None, None)), (lib.trt_batch_step, (None, 1)),
                     (lib.trt_check, (None,)), (lib.trt_prepare_steps, (None, 6))]:
        assert fn(*args) == capi.TRT_EINVAL
    out = ctypes.c_void_p()
    assert lib.trt_batch_create(0, None, ctypes.byref(out)) == capi.TRT_EINVAL
    lib.trt_destroy(None)
    lib.trt_batch_destroy(None)
    assert "batch" in capi.trt_last_error()
    assert "gfx950" in capi.trt_version()


@pytest.mark.parametrize("xb,nx,u_in,rho_in,rho_out,msg", [
    (2, 16, 0.0, 1.0, 1.0, "x_boundary"),
    (1, 1, 0.01, 1.0, 1.0, "nx >= 2"),
    (1, 16, float("nan"), 1.0, 1.0, "u_in"),
    (1, 16, 0.01, 0.0, 1.0, "rho_in"),
    (1, 16, 0.01, 1.0, -1.0, "rho_out"),
])
def test_create_rejects_invalid_open_boundaries(lib, xb, nx, u_in, rho_in, rho_out, msg):
    p = capi.trt_problem(nx, 16, 0.6, 1.0, 0.0, 0.0, None, 1, xb, u_in, rho_in, rho_out)
    with pytest.raises(capi.TrtError) as e:
        capi.trt_create(p, 4096, 8192, 0)
    assert e.value.status == capi.TRT_EINVAL and msg in str(e.value)


def test_open_boundary_problem_is_valid(lib):
    p = capi.trt_problem(16, 16, 0.6, 1.0, 0.0, 0.0, None, 1, capi.TRT_X_INFLOW_OUTFLOW, 0.01,
                         1.0, 1.0)
    assert capi.trt_lattice_bytes(p) == 9 * 16 * capi.trt_pitch(16, 1) * 4


def test_diagnostics_noalloc_validates_before_any_device_call(lib):
    p = capi.trt_problem(16, 16, 0.6, 1.0, 0.0, 0.0, None, 1)
    bad = capi.trt_problem(0, 16, 0.6, 1.0, 0.0, 0.0, None, 1)
    for prob, lat, t, out, msg in [(bad, 4096, 0, 8192, "nx and ny"),
                                   (p, 0, 0, 8192, "required"),
                                   (p, 4096, 0, 0, "required"),
                                   (p, 4096 + 8, 0, 8192, "aligned"),
                                   (p, 4096, -1, 8192, "time")]:
        with pytest.raises(capi.TrtError) as e:
            capi.trt_diagnostics_noalloc(prob, lat, t, out, 0)
        assert e.value.status == capi.TRT_EINVAL and msg in str(e.value)


@pytest.mark.parametrize("nx,ny,masked,xb,ok", [
    (46340, 46340, True, 0, False),    # link map 2 * 46340 * 46464 B > 4 GiB
    (46340, 46340, False, 1, False),   # open x boundaries need the link map too
    (46337, 46219, True, 0, False),
    (46336, 46340, True, 0, True),     # 2 * 46340 * 46336 B < 4 GiB
    (46340, 46218, True, 0, True),     # 2 * 46218 * 46464 B < 4 GiB
    (46340, 46219, True, 0, False),
    (46340, 46340, False, 0, True),    # no link map: only the side limit applies
])
def test_link_map_limit_at_the_largest_sides(lib, nx, ny, masked, xb, ok):
    p = capi.trt_problem(nx, ny, 0.6, 1.0, 0.0, 0.0, 4096 if masked else None, 1, xb, 0.01,
                         1.0, 1.0)
    if ok:
        assert capi.trt_lattice_bytes(p) == ny * 9 * capi.trt_pitch(nx, 1) * 4
        return
    assert capi.trt_lattice_bytes(p) == 0 and capi.trt_footprint_bytes(p) == 0
    with pytest.raises(capi.TrtError) as e:
        capi.trt_create(p, 4096, 1 << 40, 0)
    assert e.value.status == capi.TRT_EINVAL and "link map" in str(e.value)


@pytest.mark.parametrize("field,value,ok", [("graph_steps", 6, False), ("graph_steps", 2048, False),
                                            ("graph_steps", 1, False), ("graph_steps", 256, True),
                                            ("batch_items", -2, False), ("batch_order", 3, False),
                                            ("batch_items", 4096, True),
                                            ("prefetch_rows", 3, False),
                                            ("prefetch_rows", -1, False),
                                            ("prefetch_rows", 2, True)])
def test_tuning_fields_are_validated(lib, field, value, ok):
    """Launch-shape fields are checked before anything else (a NULL batch
    handle is reported only after a valid shape)."""
    t = capi.trt_tuning()
    setattr(t, field, value)
    st = lib.trt_batch_set_tuning(None, ctypes.byref(t))
    assert st == capi.TRT_EINVAL
    msg = capi.trt_last_error()
    assert ("batch handle" in msg) == ok, msg
