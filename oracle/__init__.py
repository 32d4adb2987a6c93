"""FP64 CPU oracle for the D2Q9 TRT-RLB step (arXiv:2312.10318).

TEST INFRASTRUCTURE ONLY: this package is the checker that the GPU path is
compared against.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import it.  It shares no code with the GPU library and
never imports it.

The arithmetic lives in ``trt_oracle.c`` (plain C, FP64, no fused
multiply-add, OpenMP over nodes); this module builds it with gcc and wraps it
with ctypes.  Arrays are numpy float64 / uint8, populations ``[9, ny, nx]``
holding the pre-collision distribution f(x, t).

Parity status per function (how each is pinned, in tests/test_oracle_*.py):
  feq, source_G, source_F   moment identities of Sec. II.C (Eqs. 16-17)
  collide_node              conservation, Hermite change-of-basis (MRT form),
                            BGK identity at tau2 = tau1, fixed point
  collide, stream_open       the two halves of a step: their composition equals
                            step / step_open bit for bit
  step / run                Poiseuille closed form + slip law (Sec. II.D),
                            Taylor-Green decay and second-order convergence
                            (Sec. III.B), lattice symmetry, exact mass
  gradient reading R1       (central difference, 0 at solids) is parity
                            unpinned; the printed results it can touch move
                            by <= 1.1e-7 under the other natural reading.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "trt_oracle.c")
_LIB = os.path.join(_HERE, "libtrt_oracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-std=c99", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/libtrt_oracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_ARGTYPES = None


def _bind(lib):
    d, i, L = ctypes.c_double, ctypes.c_int, ctypes.c_long
    P = ctypes.c_void_p
    lib.orc_feq.argtypes = [d, d, d, P]
    lib.orc_moments.argtypes = [P, d, d, P, P, P]
    lib.orc_source_G.argtypes = [d, d, d, P]
    lib.orc_source_F.argtypes = [d, d, d, d, P]
    lib.orc_collide_node.argtypes = [P, d, d, d, d, d, d, P]
    lib.orc_macros.argtypes = [i, i, P, P, d, d, P, P, P]
    lib.orc_init_equilibrium.argtypes = [i, i, P, P, P, P, P]
    lib.orc_step.argtypes = [i, i, P, P, P, d, d, d, d]
    lib.orc_step.restype = i
    lib.orc_run.argtypes = [i, i, P, P, L, d, d, d, d]
    lib.orc_run.restype = i
    lib.orc_step_open.argtypes = [i, i, P, P, P, d, d, d, d, d, d, d]
    lib.orc_step_open.restype = i
    lib.orc_run_open.argtypes = [i, i, P, P, L, d, d, d, d, d, d, d]
    lib.orc_run_open.restype = i
    lib.orc_collide.argtypes = [i, i, P, P, P, d, d, d, d, i, d, d]
    lib.orc_collide.restype = i
    lib.orc_stream_open.argtypes = [i, i, P, P, P, d, d, d]
    lib.orc_stream_open.restype = None
    lib.orc_wall_force.argtypes = [i, i, P, P, d, d, d, d, i, d, d, P]
    lib.orc_wall_force.restype = i
    lib.orc_num_threads.restype = i
    lib.orc_set_num_threads.argtypes = [i]
    lib.orc_set_num_threads.restype = None
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _mask(mask, ny, nx):
    if mask is None:
        return None
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    if m.shape != (ny, nx):
        raise ValueError("mask must be [ny, nx]")
    return m


class Oracle:
    """The oracle's entry points bound to one compiled library.

    The default instance (module-level functions below) loads
    oracle/libtrt_oracle.so; the mutation tests bind deliberately broken
    builds of the same source to check that the pins catch them.
    """

    def __init__(self, lib_path: str | None = None):
        if lib_path is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            lib_path = _LIB
        self.lib = _bind(ctypes.CDLL(lib_path))

    def feq(self, rho: float, ux: float, uy: float) -> np.ndarray:
        """Third-order Hermite equilibrium of one node (Sec. II.B, Eq. 5)."""
        out = np.empty(9)
        self.lib.orc_feq(rho, ux, uy, _p(out))
        return out

    def moments(self, f) -> tuple:
        """(rho, ux, uy) of one node without force (Eqs. 12-13)."""
        return self.moments_forced(f, 0.0, 0.0)

    def moments_forced(self, f, gx: float, gy: float) -> tuple:
        """(rho, ux, uy) of one node with He's shift u = (j + F/2)/rho, F = rho g."""
        f = _f64(f)
        r, ux, uy = (np.empty(1) for _ in range(3))
        self.lib.orc_moments(_p(f), gx, gy, _p(r), _p(ux), _p(uy))
        return float(r[0]), float(ux[0]), float(uy[0])

    def source_G(self, tau1: float, dphix: float, dphiy: float) -> np.ndarray:
        """Cubic-error compensation G_i (Sec. II.B, Eq. 8)."""
        out = np.empty(9)
        self.lib.orc_source_G(tau1, dphix, dphiy, _p(out))
        return out

    def source_F(self, Fx: float, Fy: float, ux: float, uy: float) -> np.ndarray:
        """Forcing term F_i (Sec. II.B, Eq. 11)."""
        out = np.empty(9)
        self.lib.orc_source_F(Fx, Fy, ux, uy, _p(out))
        return out

    def collide_node(self, f, gx: float, gy: float, dphix: float, dphiy: float, tau1: float,
                     tau2: float) -> np.ndarray:
        """Post-collision populations of one node (Sec. II.B, Eq. 2)."""
        f = _f64(f)
        out = np.empty(9)
        self.lib.orc_collide_node(_p(f), gx, gy, dphix, dphiy, tau1, tau2, _p(out))
        return out

    def init_equilibrium(self, rho, ux, uy, mask=None) -> np.ndarray:
        """f(x, 0) = f^eq(rho, u) at fluid nodes, 0 at solid nodes; [9, ny, nx]."""
        rho, ux, uy = _f64(rho), _f64(ux), _f64(uy)
        ny, nx = rho.shape
        m = _mask(mask, ny, nx)
        f = np.empty((9, ny, nx))
        self.lib.orc_init_equilibrium(nx, ny, _p(m), _p(rho), _p(ux), _p(uy), _p(f))
        return f

    def macros(self, f, gx: float = 0.0, gy: float = 0.0, mask=None) -> tuple:
        """(rho, ux, uy) fields [ny, nx] of a population array; solid -> 0."""
        f = _f64(f)
        _, ny, nx = f.shape
        m = _mask(mask, ny, nx)
        rho, ux, uy = (np.empty((ny, nx)) for _ in range(3))
        self.lib.orc_macros(nx, ny, _p(m), _p(f), gx, gy, _p(rho), _p(ux), _p(uy))
        return rho, ux, uy

    def step(self, f, tau1: float, tau2: float, gx: float = 0.0, gy: float = 0.0,
             mask=None) -> np.ndarray:
        """One time step; returns a new [9, ny, nx] array."""
        f = _f64(f)
        _, ny, nx = f.shape
        m = _mask(mask, ny, nx)
        out = np.empty_like(f)
        if self.lib.orc_step(nx, ny, _p(m), _p(f), _p(out), tau1, tau2, gx, gy) != 0:
            raise MemoryError("oracle step: allocation failed")
        return out

    def run(self, f, nsteps: int, tau1: float, tau2: float, gx: float = 0.0, gy: float = 0.0,
            mask=None) -> np.ndarray:
        """nsteps time steps; returns a new [9, ny, nx] array."""
        f = np.array(f, dtype=np.float64, order="C", copy=True)
        _, ny, nx = f.shape
        m = _mask(mask, ny, nx)
        if self.lib.orc_run(nx, ny, _p(m), _p(f), int(nsteps), tau1, tau2, gx, gy) != 0:
            raise MemoryError("oracle run: allocation failed")
        return f


    def step_open(self, f, tau1: float, tau2: float, u_in: float, rho_w: float = 1.0,
                  rho_out: float = 1.0, gx: float = 0.0, gy: float = 0.0,
                  mask=None) -> np.ndarray:
        """One step with the inflow wall at x = -1/2 and the pressure outlet at
        x = nx - 1 (periodic in y); returns a new [9, ny, nx] array."""
        f = _f64(f)
        _, ny, nx = f.shape
        m = _mask(mask, ny, nx)
        out = np.empty_like(f)
        if self.lib.orc_step_open(nx, ny, _p(m), _p(f), _p(out), tau1, tau2, gx, gy, u_in,
                                  rho_w, rho_out) != 0:
            raise MemoryError("oracle step: allocation failed")
        return out

    def run_open(self, f, nsteps: int, tau1: float, tau2: float, u_in: float,
                 rho_w: float = 1.0, rho_out: float = 1.0, gx: float = 0.0, gy: float = 0.0,
                 mask=None) -> np.ndarray:
        """nsteps steps of :meth:`step_open`; returns a new array."""
        f = np.array(f, dtype=np.float64, order="C", copy=True)
        _, ny, nx = f.shape
        m = _mask(mask, ny, nx)
        if self.lib.orc_run_open(nx, ny, _p(m), _p(f), int(nsteps), tau1, tau2, gx, gy, u_in,
                                 rho_w, rho_out) != 0:
            raise MemoryError("oracle run: allocation failed")
        return f

    def collide(self, f, tau1: float, tau2: float, gx: float = 0.0, gy: float = 0.0,
                mask=None, open_x: bool = False, u_in: float = 0.0,
                rho_w: float = 1.0) -> np.ndarray:
        """Post-collision populations f*(x, t) of every fluid node (0 at solid
        nodes), the first half of :meth:`step` / :meth:`step_open`; open_x
        takes the open ends' Phi as :meth:`step_open` does."""
        f = _f64(f)
        _, ny, nx = f.shape
        m = _mask(mask, ny, nx)
        out = np.empty_like(f)
        if self.lib.orc_collide(nx, ny, _p(m), _p(f), _p(out), tau1, tau2, gx, gy, int(open_x),
                                u_in, rho_w) != 0:
            raise MemoryError("oracle collide: allocation failed")
        return out

    def stream_open(self, fstar, u_in: float, rho_w: float = 1.0, rho_out: float = 1.0,
                    mask=None) -> np.ndarray:
        """Streaming of post-collision populations with the inflow wall and
        the pressure outlet, the second half of :meth:`step_open`."""
        fstar = _f64(fstar)
        _, ny, nx = fstar.shape
        m = _mask(mask, ny, nx)
        out = np.empty_like(fstar)
        self.lib.orc_stream_open(nx, ny, _p(m), _p(fstar), _p(out), u_in, rho_w, rho_out)
        return out

    def wall_force(self, f, tau1: float, tau2: float, gx: float = 0.0, gy: float = 0.0,
                   mask=None, open_x: bool = False, u_in: float = 0.0,
                   rho_w: float = 1.0) -> tuple:
        """(F_x, F_y) handed to the solid nodes by the collision of state f."""
        f = _f64(f)
        _, ny, nx = f.shape
        m = _mask(mask, ny, nx)
        out = np.zeros(2)
        if self.lib.orc_wall_force(nx, ny, _p(m), _p(f), tau1, tau2, gx, gy, int(open_x), u_in,
                                   rho_w, _p(out)) != 0:
            raise MemoryError("oracle wall force: allocation failed")
        return float(out[0]), float(out[1])


_default = None


def _inst() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def feq(*a, **k):
    return _inst().feq(*a, **k)


def moments(*a, **k):
    return _inst().moments(*a, **k)


def moments_forced(*a, **k):
    return _inst().moments_forced(*a, **k)


def source_G(*a, **k):
    return _inst().source_G(*a, **k)


def source_F(*a, **k):
    return _inst().source_F(*a, **k)


def collide_node(*a, **k):
    return _inst().collide_node(*a, **k)


def init_equilibrium(*a, **k):
    return _inst().init_equilibrium(*a, **k)


def macros(*a, **k):
    return _inst().macros(*a, **k)


def step(*a, **k):
    return _inst().step(*a, **k)


def run(*a, **k):
    return _inst().run(*a, **k)


def step_open(*a, **k):
    return _inst().step_open(*a, **k)


def run_open(*a, **k):
    return _inst().run_open(*a, **k)


def wall_force(*a, **k):
    return _inst().wall_force(*a, **k)


def collide(*a, **k):
    return _inst().collide(*a, **k)


def stream_open(*a, **k):
    return _inst().stream_open(*a, **k)


def num_threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(_inst().lib.orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads for the oracle's OpenMP loops (for timing; results do not
    depend on it)."""
    _inst().lib.orc_set_num_threads(int(n))


def build_variant(source_text: str, out_path: str) -> str:
    """Compile an edited copy of the oracle source (used only by the tests
    that plant mistakes in the oracle to show the pins catch them)."""
    src = out_path + ".c"
    with open(src, "w") as fh:
        fh.write(source_text)
    subprocess.run(["gcc", *CFLAGS, src, "-o", out_path, "-lm"], check=True)
    return out_path


def source_text() -> str:
    with open(_SRC) as fh:
        return fh.read()
