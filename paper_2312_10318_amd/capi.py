"""Thin ctypes binding of include/trtlbm.h (argument marshalling only).

Every function here has the name of the C entry point it calls and passes
raw pointers and sizes through; all computation happens in the HIP library
``libtrtlbm.so`` built in-tree by ``paper_2312_10318_amd.build``.  Loading
fails loudly when the library is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# TRTLBM_LIB selects another build of the same library (e.g. an instrumented
# or differently compiled copy); the default is the in-tree build.
LIB_PATH = os.environ.get("TRTLBM_LIB") or os.path.join(HERE, "libtrtlbm.so")

TRT_OK, TRT_EINVAL, TRT_ENOMEM, TRT_EDEVICE, TRT_EUNSTABLE, TRT_ESTATE = range(6)
TRT_F64, TRT_F32_SHIFTED, TRT_F16_SHIFTED = 0, 1, 2
TRT_X_PERIODIC, TRT_X_INFLOW_OUTFLOW = 0, 1
TRT_NDIAG = 8

STATUS_NAMES = {0: "TRT_OK", 1: "TRT_EINVAL", 2: "TRT_ENOMEM", 3: "TRT_EDEVICE",
                4: "TRT_EUNSTABLE", 5: "TRT_ESTATE"}

# Symbols declared in include/trtlbm.h (checked against the header by the tests).
EXPORTED = [
    "trt_pitch", "trt_row_stride", "trt_lattice_bytes", "trt_footprint_bytes", "trt_create",
    "trt_set_tuning", "trt_get_tuning", "trt_init_equilibrium", "trt_set_populations",
    "trt_get_populations", "trt_step", "trt_prepare_steps", "trt_pattern_probe", "trt_macros", "trt_diagnostics",
    "trt_diagnostics_noalloc", "trt_row_mean_ux",
    "trt_wall_force", "trt_velocity_change", "trt_velocity_error",
    "trt_check", "trt_state", "trt_destroy", "trt_batch_create", "trt_batch_update",
    "trt_batch_step",
    "trt_batch_diagnostics", "trt_batch_set_tuning", "trt_batch_get_tuning", "trt_batch_destroy",
    "trt_last_error",
    "trt_version",
]


class trt_problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("tau_s", ctypes.c_double),
                ("tau_s2", ctypes.c_double), ("gx", ctypes.c_double), ("gy", ctypes.c_double),
                ("mask", ctypes.c_void_p), ("storage", ctypes.c_int32),
                ("x_boundary", ctypes.c_int32), ("u_in", ctypes.c_double),
                ("rho_in", ctypes.c_double), ("rho_out", ctypes.c_double)]


class trt_tuning(ctypes.Structure):
    _fields_ = [("rows_per_wave", ctypes.c_int32), ("waves_per_block", ctypes.c_int32),
                ("xcd_remap", ctypes.c_int32), ("cols_per_lane", ctypes.c_int32),
                ("batch_items", ctypes.c_int32), ("batch_order", ctypes.c_int32),
                ("graph_steps", ctypes.c_int32), ("steps_per_sweep", ctypes.c_int32),
                ("prefetch_rows", ctypes.c_int32)]


class TrtError(RuntimeError):
    def __init__(self, status, where, msg):
        self.status = status
        super().__init__("%s: %s (%s)" % (where, msg, STATUS_NAMES.get(status, status)))


_lib = None


def load():
    """Load libtrtlbm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libtrtlbm.so is not built (run __graft_entry__.build() or "
                          "python -m paper_2312_10318_amd.build); the TRT-RLB path has no "
                          "fallback")
    # PyTorch ships its own HIP runtime under the same soname: it is loaded
    # first, so that the library binds to it (a second HIP runtime in the
    # process would find no GPU once the first has opened it)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    PP = ctypes.POINTER(ctypes.c_void_p)
    prob = ctypes.POINTER(trt_problem)
    tun = ctypes.POINTER(trt_tuning)
    sig = {
        "trt_pitch": (I32, [I32, I32]),
        "trt_row_stride": (I64, [I32, I32]),
        "trt_lattice_bytes": (ctypes.c_size_t, [prob]),
        "trt_footprint_bytes": (ctypes.c_size_t, [prob]),
        "trt_create": (ctypes.c_int, [prob, P, P, P, PP]),
        "trt_set_tuning": (ctypes.c_int, [P, tun]),
        "trt_get_tuning": (ctypes.c_int, [P, tun]),
        "trt_init_equilibrium": (ctypes.c_int, [P, P, P, P]),
        "trt_set_populations": (ctypes.c_int, [P, P]),
        "trt_get_populations": (ctypes.c_int, [P, P]),
        "trt_step": (ctypes.c_int, [P, I64]),
        "trt_prepare_steps": (ctypes.c_int, [P, I64]),
        "trt_pattern_probe": (ctypes.c_int, [P, I64]),
        "trt_macros": (ctypes.c_int, [P, P, P, P]),
        "trt_diagnostics": (ctypes.c_int, [P, P]),
        "trt_diagnostics_noalloc": (ctypes.c_int, [prob, P, I64, P, P]),
        "trt_row_mean_ux": (ctypes.c_int, [P, P]),
        "trt_wall_force": (ctypes.c_int, [P, P]),
        "trt_velocity_change": (ctypes.c_int, [P, P, P, P]),
        "trt_velocity_error": (ctypes.c_int, [P, P, P, P]),
        "trt_check": (ctypes.c_int, [P]),
        "trt_state": (ctypes.c_int, [P, ctypes.POINTER(I32), ctypes.POINTER(I64)]),
        "trt_destroy": (None, [P]),
        "trt_batch_create": (ctypes.c_int, [I32, PP, PP]),
        "trt_batch_update": (ctypes.c_int, [P, I32, PP]),
        "trt_batch_step": (ctypes.c_int, [P, I64]),
        "trt_batch_diagnostics": (ctypes.c_int, [P, P]),
        "trt_batch_set_tuning": (ctypes.c_int, [P, tun]),
        "trt_batch_get_tuning": (ctypes.c_int, [P, tun]),
        "trt_batch_destroy": (None, [P]),
        "trt_last_error": (ctypes.c_char_p, []),
        "trt_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(st, where):
    if st != TRT_OK:
        raise TrtError(st, where, load().trt_last_error().decode())
    return st


def _prob(nx, ny, tau_s, tau_s2, gx, gy, mask_ptr, storage, x_boundary=TRT_X_PERIODIC,
          u_in=0.0, rho_in=1.0, rho_out=1.0):
    return trt_problem(nx, ny, tau_s, tau_s2, gx, gy, mask_ptr, storage, x_boundary, u_in,
                       rho_in, rho_out)


def trt_pitch(nx: int, storage: int) -> int:
    return load().trt_pitch(nx, storage)


def trt_row_stride(nx: int, storage: int) -> int:
    return load().trt_row_stride(nx, storage)


def trt_lattice_bytes(p: trt_problem) -> int:
    return load().trt_lattice_bytes(ctypes.byref(p))


def trt_footprint_bytes(p: trt_problem) -> int:
    return load().trt_footprint_bytes(ctypes.byref(p))


def trt_create(p: trt_problem, f_a: int, f_b: int, stream: int) -> int:
    out = ctypes.c_void_p()
    _check(load().trt_create(ctypes.byref(p), f_a, f_b, stream, ctypes.byref(out)), "trt_create")
    return out.value


def trt_set_tuning(sim: int, rows_per_wave: int = 0, waves_per_block: int = 0,
                   xcd_remap: int = -1, cols_per_lane: int = 0, graph_steps: int = 0,
                   steps_per_sweep: int = 0, prefetch_rows: int = 0) -> None:
    t = trt_tuning(rows_per_wave, waves_per_block, xcd_remap, cols_per_lane, 0, 0, graph_steps,
                   steps_per_sweep, prefetch_rows)
    _check(load().trt_set_tuning(sim, ctypes.byref(t)), "trt_set_tuning")


def trt_get_tuning(sim: int) -> tuple:
    t = trt_tuning()
    _check(load().trt_get_tuning(sim, ctypes.byref(t)), "trt_get_tuning")
    return (t.rows_per_wave, t.waves_per_block, t.xcd_remap, t.cols_per_lane, t.graph_steps,
            t.steps_per_sweep, t.prefetch_rows)


def trt_init_equilibrium(sim: int, rho: int, ux: int, uy: int) -> None:
    _check(load().trt_init_equilibrium(sim, rho, ux, uy), "trt_init_equilibrium")


def trt_set_populations(sim: int, f: int) -> None:
    _check(load().trt_set_populations(sim, f), "trt_set_populations")


def trt_get_populations(sim: int, f: int) -> None:
    _check(load().trt_get_populations(sim, f), "trt_get_populations")


def trt_step(sim: int, nsteps: int) -> None:
    _check(load().trt_step(sim, nsteps), "trt_step")


def trt_prepare_steps(sim: int, nsteps: int) -> None:
    _check(load().trt_prepare_steps(sim, nsteps), "trt_prepare_steps")


def trt_pattern_probe(sim: int, nsweeps: int) -> None:
    _check(load().trt_pattern_probe(sim, nsweeps), "trt_pattern_probe")


def trt_macros(sim: int, rho: int, ux: int, uy: int) -> None:
    _check(load().trt_macros(sim, rho, ux, uy), "trt_macros")


def trt_diagnostics(sim: int, out: int) -> None:
    _check(load().trt_diagnostics(sim, out), "trt_diagnostics")


def trt_diagnostics_noalloc(p: trt_problem, lattice: int, time: int, out: int,
                            stream: int) -> None:
    _check(load().trt_diagnostics_noalloc(ctypes.byref(p), lattice, time, out, stream),
           "trt_diagnostics_noalloc")


def trt_wall_force(sim: int, out: int) -> None:
    _check(load().trt_wall_force(sim, out), "trt_wall_force")


def trt_velocity_change(sim: int, prev_ux: int, prev_uy: int, out: int) -> None:
    _check(load().trt_velocity_change(sim, prev_ux, prev_uy, out), "trt_velocity_change")


def trt_velocity_error(sim: int, ref_ux: int, ref_uy: int, out: int) -> None:
    _check(load().trt_velocity_error(sim, ref_ux, ref_uy, out), "trt_velocity_error")


def trt_row_mean_ux(sim: int, out: int) -> None:
    _check(load().trt_row_mean_ux(sim, out), "trt_row_mean_ux")


def trt_check(sim: int) -> int:
    """Returns TRT_OK or TRT_EUNSTABLE; raises on any other status."""
    st = load().trt_check(sim)
    if st not in (TRT_OK, TRT_EUNSTABLE):
        _check(st, "trt_check")
    return st


def trt_state(sim: int) -> tuple:
    cur, t = ctypes.c_int32(), ctypes.c_int64()
    _check(load().trt_state(sim, ctypes.byref(cur), ctypes.byref(t)), "trt_state")
    return cur.value, t.value


def trt_destroy(sim: int) -> None:
    load().trt_destroy(sim)


def trt_batch_create(sims) -> int:
    arr = (ctypes.c_void_p * len(sims))(*sims)
    out = ctypes.c_void_p()
    _check(load().trt_batch_create(len(sims), arr, ctypes.byref(out)), "trt_batch_create")
    return out.value


def trt_batch_update(batch: int, sims) -> None:
    arr = (ctypes.c_void_p * len(sims))(*sims)
    _check(load().trt_batch_update(batch, len(sims), arr), "trt_batch_update")


def trt_batch_step(batch: int, nsteps: int) -> None:
    _check(load().trt_batch_step(batch, nsteps), "trt_batch_step")


def trt_batch_diagnostics(batch: int, out: int) -> None:
    _check(load().trt_batch_diagnostics(batch, out), "trt_batch_diagnostics")


def trt_batch_set_tuning(batch: int, rows_per_wave: int = 0, waves_per_block: int = 0,
                         xcd_remap: int = -1, cols_per_lane: int = 0, batch_items: int = 0,
                         batch_order: int = 0, graph_steps: int = 0,
                         steps_per_sweep: int = 0, prefetch_rows: int = 0) -> None:
    t = trt_tuning(rows_per_wave, waves_per_block, xcd_remap, cols_per_lane, batch_items,
                   batch_order, graph_steps, steps_per_sweep, prefetch_rows)
    _check(load().trt_batch_set_tuning(batch, ctypes.byref(t)), "trt_batch_set_tuning")


def trt_batch_get_tuning(batch: int) -> tuple:
    """(rows, waves per workgroup, XCD remap, columns per lane, batch_items,
    batch_order, longest captured graph, time steps per launch, rows the
    two-step loads run ahead)."""
    t = trt_tuning()
    _check(load().trt_batch_get_tuning(batch, ctypes.byref(t)), "trt_batch_get_tuning")
    return (t.rows_per_wave, t.waves_per_block, t.xcd_remap, t.cols_per_lane, t.batch_items,
            t.batch_order, t.graph_steps, t.steps_per_sweep, t.prefetch_rows)


def trt_batch_destroy(batch: int) -> None:
    load().trt_batch_destroy(batch)


def trt_last_error() -> str:
    return load().trt_last_error().decode()


def trt_version() -> str:
    return load().trt_version().decode()
