"""Python front end of the TRT-RLB library: device memory and streams come
from PyTorch (ROCm); every step of the method runs in libtrtlbm.so."""
from __future__ import annotations

import numpy as np

from . import capi

STORAGES = {"f64": capi.TRT_F64, "f32": capi.TRT_F32_SHIFTED, "f16": capi.TRT_F16_SHIFTED}
STORAGE_BYTES = {"f64": 8, "f32": 4, "f16": 2}
DIAG_NAMES = ("mass", "mom_x", "mom_y", "max_speed", "n_diverged", "n_fluid", "min_rho", "time")


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the TRT-RLB library needs a ROCm GPU (torch.cuda is unavailable)")
    return torch


_UPLOAD = {}


def _upload_stream(device):
    """A side stream per device (default priority) for uploads that must be
    complete before a library call."""
    torch = _torch()
    key = str(device)
    if key not in _UPLOAD:
        _UPLOAD[key] = torch.cuda.Stream(device)
    return _UPLOAD[key]


def problem(nx, ny, tau_s, tau_s2, g=(0.0, 0.0), storage="f32", mask_ptr=None, inflow=None):
    """The C problem struct (no device memory touched).  inflow = (u_in,
    rho_in, rho_out) selects the open x boundaries (inflow wall, outlet)."""
    xb, u_in, rho_in, rho_out = capi.TRT_X_PERIODIC, 0.0, 1.0, 1.0
    if inflow is not None:
        xb = capi.TRT_X_INFLOW_OUTFLOW
        u_in, rho_in, rho_out = (float(v) for v in inflow)
    return capi.trt_problem(int(nx), int(ny), float(tau_s), float(tau_s2), float(g[0]),
                            float(g[1]), mask_ptr, STORAGES[storage], xb, u_in, rho_in, rho_out)


def footprint_bytes(nx, ny, storage="f32", has_mask=False) -> int:
    """Device bytes a simulation needs (two lattices, mask, scratch)."""
    p = problem(nx, ny, 0.6, 0.6, storage=storage, mask_ptr=1 if has_mask else None)
    return capi.trt_footprint_bytes(p)


class Lattice:
    """One D2Q9 TRT-RLB simulation on the GPU.

    nx, ny      lattice size (periodic in x and y; walls are mask rows)
    tau_s       tau_s1 > 1/2 (viscosity nu = (tau_s - 1/2) / 3)
    tau_s2      free third-order relaxation time >= 1/2
    g           body acceleration (F = rho g)
    mask        optional [ny, nx] array, nonzero = solid (half-way bounce-back)
    storage     "f64", "f32" (f - w) or "f16" (f - w)
    stream      torch.cuda.Stream to enqueue on (default: the current stream)
    inflow      optional (u_in, rho_in, rho_out): open x boundaries, an inflow
                wall at x = -1/2 moving with (u_in, 0) and a pressure outlet
                at x = nx - 1 (the creeping-flow set-up of Sec. III.D)
    """

    def __init__(self, nx, ny, tau_s, tau_s2, g=(0.0, 0.0), mask=None, storage="f32",
                 stream=None, device="cuda", inflow=None):
        torch = _torch()
        self.nx, self.ny = int(nx), int(ny)
        self.tau_s, self.tau_s2 = float(tau_s), float(tau_s2)
        self.g = (float(g[0]), float(g[1]))
        self.storage = storage
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.mask = None
        if mask is not None:
            m = np.ascontiguousarray(np.asarray(mask) != 0, dtype=np.uint8)
            if m.shape != (self.ny, self.nx):
                raise ValueError("mask must have shape [ny, nx]")
            # trt_create reads the mask (on a stream of its own), so its copy
            # must be complete by then: it goes up on a side stream, which is
            # waited for alone (not the work queued on the lattice's stream)
            up = _upload_stream(self.device)
            with torch.cuda.stream(up):
                self.mask = torch.from_numpy(m).pin_memory().to(self.device, non_blocking=True)
            up.synchronize()
            self.mask.record_stream(self.stream)
        self.inflow = None if inflow is None else tuple(float(v) for v in inflow)
        prob = problem(self.nx, self.ny, self.tau_s, self.tau_s2, self.g, storage,
                       self.mask.data_ptr() if self.mask is not None else None, self.inflow)
        self.prob = prob  # the C problem struct (its mask pointer stays valid with self.mask)
        nbytes = capi.trt_lattice_bytes(prob)
        if nbytes == 0:
            capi.trt_create(prob, 0, 0, 0)  # raises with the validation message
        self.lattice_bytes = nbytes
        # allocated on the lattice's stream, where every sweep runs: the
        # caching allocator then reuses this memory only in that stream's
        # order once it is released
        with torch.cuda.stream(self.stream):
            self.fa = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.fb = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self._diag = torch.empty(capi.TRT_NDIAG, dtype=torch.float64, device=self.device)
        self.handle = capi.trt_create(prob, self.fa.data_ptr(), self.fb.data_ptr(),
                                      self.stream.cuda_stream)

    # ---------------------------------------------------------------- helpers
    def _dev64(self, a, shape):
        """A device FP64 copy of `a` (numpy arrays go through pinned memory
        and an asynchronous copy on the lattice's stream; a tensor made on
        the current stream is ordered before the lattice stream's use)."""
        torch = _torch()
        if torch.is_tensor(a):
            t = a.to(device=self.device, dtype=torch.float64).contiguous()
            cur = torch.cuda.current_stream(self.device)
            if cur != self.stream:
                self.stream.wait_stream(cur)
                t.record_stream(self.stream)
        else:
            h = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
            if tuple(h.shape) != tuple(shape):
                raise ValueError("expected shape %s, got %s" % (shape, tuple(h.shape)))
            with torch.cuda.stream(self.stream):
                t = h.pin_memory().to(self.device, non_blocking=True)
        if tuple(t.shape) != tuple(shape):
            raise ValueError("expected shape %s, got %s" % (shape, tuple(t.shape)))
        return t

    def _sync(self):
        self.stream.synchronize()

    # ------------------------------------------------------------------- API
    def set_tuning(self, rows_per_wave=0, waves_per_block=0, xcd_remap=-1, cols_per_lane=0,
                   graph_steps=0, steps_per_sweep=0, prefetch_rows=0):
        capi.trt_set_tuning(self.handle, rows_per_wave, waves_per_block, xcd_remap, cols_per_lane,
                            graph_steps, steps_per_sweep, prefetch_rows)

    def tuning(self):
        """(rows per wavefront, wavefronts per workgroup, XCD remap, columns per
        lane, longest captured graph, time steps per launch, rows the two-step
        loads run ahead: 0 for one step per launch) in effect."""
        return capi.trt_get_tuning(self.handle)

    def init_equilibrium(self, rho, ux, uy, sync=True):
        """f(x, 0) = f^eq(rho, u).  With sync=False the call returns once the
        work is enqueued (the inputs are copied asynchronously)."""
        shape = (self.ny, self.nx)
        r, u, v = self._dev64(rho, shape), self._dev64(ux, shape), self._dev64(uy, shape)
        capi.trt_init_equilibrium(self.handle, r.data_ptr(), u.data_ptr(), v.data_ptr())
        if sync:
            self._sync()
        return self

    def set_populations(self, f):
        t = self._dev64(f, (9, self.ny, self.nx))
        capi.trt_set_populations(self.handle, t.data_ptr())
        self._sync()
        return self

    def get_populations(self):
        torch = _torch()
        out = torch.empty((9, self.ny, self.nx), dtype=torch.float64, device=self.device)
        capi.trt_get_populations(self.handle, out.data_ptr())
        self._sync()
        return out

    def step(self, nsteps=1):
        capi.trt_step(self.handle, int(nsteps))
        return self

    def prepare(self, nsteps):
        """Capture the step graphs that step(nsteps) would replay from the
        current state, launching nothing."""
        capi.trt_prepare_steps(self.handle, int(nsteps))
        return self

    def pattern_probe(self, nsweeps=1):
        """Launches of the access-pattern probe (scrambles the state)."""
        capi.trt_pattern_probe(self.handle, int(nsweeps))
        return self

    def macros(self):
        """(rho, ux, uy) as float64 device tensors [ny, nx]."""
        torch = _torch()
        out = torch.empty((3, self.ny, self.nx), dtype=torch.float64, device=self.device)
        n = self.nx * self.ny * 8
        base = out.data_ptr()
        capi.trt_macros(self.handle, base, base + n, base + 2 * n)
        self._sync()
        return out[0], out[1], out[2]

    def diagnostics(self) -> dict:
        capi.trt_diagnostics(self.handle, self._diag.data_ptr())
        self._sync()
        vals = self._diag.cpu().numpy()
        return dict(zip(DIAG_NAMES, (float(v) for v in vals)))

    def row_mean_ux(self):
        torch = _torch()
        out = torch.empty(self.ny, dtype=torch.float64, device=self.device)
        capi.trt_row_mean_ux(self.handle, out.data_ptr())
        self._sync()
        return out

    def check(self) -> bool:
        """True while no fluid node has diverged (synchronous)."""
        return capi.trt_check(self.handle) == capi.TRT_OK

    def wall_force(self):
        """(F_x, F_y) handed to the solid nodes by the last collision
        (momentum exchange, synchronous)."""
        torch = _torch()
        out = torch.empty(2, dtype=torch.float64, device=self.device)
        capi.trt_wall_force(self.handle, out.data_ptr())
        self._sync()
        v = out.cpu().numpy()
        return float(v[0]), float(v[1])

    def velocity_change(self, prev):
        """Compare the velocity with prev = (ux, uy) device FP64 tensors (then
        overwritten with the current velocity); returns (max |du|, sum |du|^2,
        sum |u|^2, sum |u_prev|^2) (synchronous)."""
        torch = _torch()
        out = torch.empty(4, dtype=torch.float64, device=self.device)
        capi.trt_velocity_change(self.handle, prev[0].data_ptr(), prev[1].data_ptr(),
                                 out.data_ptr())
        self._sync()
        return tuple(float(v) for v in out.cpu().numpy())

    def velocity_error(self, ux_ref, uy_ref):
        """Relative L2 error of the velocity against reference fields (the
        error measure of Sec. III), computed on the device; also returns
        the max-norm difference.  (rel_l2, max |u - u_ref|)."""
        torch = _torch()
        shape = (self.ny, self.nx)
        a, b = self._dev64(ux_ref, shape), self._dev64(uy_ref, shape)
        out = torch.empty(4, dtype=torch.float64, device=self.device)
        capi.trt_velocity_error(self.handle, a.data_ptr(), b.data_ptr(), out.data_ptr())
        self._sync()
        v = out.cpu().numpy()
        return (float(np.sqrt(v[1] / v[3])) if v[3] > 0 else float("inf"), float(v[0]))

    def state(self):
        """(index of the lattice holding the state, steps taken)."""
        return capi.trt_state(self.handle)

    def raw_state(self):
        """The storage bytes of the current lattice (exact checkpoint)."""
        cur, t = self.state()
        return (self.fb if cur else self.fa).clone(), cur, t

    def release(self):
        """Give the lattice buffers back now (the simulation must not be used
        again except for close(); the handle's own small scratch stays until
        close, whose device-wide frees a caller may want to defer)."""
        self.fa = self.fb = None

    def close(self):
        if getattr(self, "handle", None):
            capi.trt_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent lattices advanced together, one launch per step."""

    def __init__(self, lattices):
        if not lattices:
            raise ValueError("empty batch")
        self.lattices = list(lattices)
        self.stream = self.lattices[0].stream
        self.handle = capi.trt_batch_create([l.handle for l in self.lattices])
        torch = _torch()
        self._diag = torch.empty((len(self.lattices), capi.TRT_NDIAG), dtype=torch.float64,
                                 device=self.lattices[0].device)

    def set_tuning(self, rows_per_wave=0, waves_per_block=0, xcd_remap=-1, cols_per_lane=0,
                   batch_items=0, batch_order=0, graph_steps=0, steps_per_sweep=0,
                   prefetch_rows=0):
        capi.trt_batch_set_tuning(self.handle, rows_per_wave, waves_per_block, xcd_remap,
                                  cols_per_lane, batch_items, batch_order, graph_steps,
                                  steps_per_sweep, prefetch_rows)

    def tuning(self):
        """(rows, wavefronts per workgroup, XCD remap, columns per lane,
        batch_items, batch_order, longest captured graph, time steps per
        launch: 2 if some member takes two-step launches, rows the two-step
        loads run ahead)."""
        return capi.trt_batch_get_tuning(self.handle)

    def update(self, lattices):
        """Replace the members (no device-wide wait)."""
        lattices = list(lattices)
        if not lattices:
            raise ValueError("empty batch")
        capi.trt_batch_update(self.handle, [l.handle for l in lattices])
        self.lattices = lattices
        if self._diag.shape[0] < len(lattices):
            torch = _torch()
            self._diag = torch.empty((len(lattices), capi.TRT_NDIAG), dtype=torch.float64,
                                     device=self.lattices[0].device)
        return self

    def step(self, nsteps=1):
        capi.trt_batch_step(self.handle, int(nsteps))
        return self

    def diagnostics(self):
        """[n, TRT_NDIAG] numpy array (synchronous)."""
        capi.trt_batch_diagnostics(self.handle, self._diag.data_ptr())
        self.stream.synchronize()
        return self._diag[:len(self.lattices)].cpu().numpy()

    def close(self):
        if getattr(self, "handle", None):
            capi.trt_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
