// kernels.hpp -- host-side launchers of the device kernels (internal to the
// library; the public interface is include/trtlbm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.hpp"

namespace trt {

struct Launch {
    int rows_per_wave;
    int waves_per_block;
    int xcd_remap;
};

// Tiling of one instance for a launch shape.
inline void tile(InstDesc &d, const Launch &l) {
    d.rows = l.rows_per_wave;
    d.strips = (d.nx + kStripWidth - 1) / kStripWidth;
    d.rowblocks = (d.ny + d.rows - 1) / d.rows;
}

// One fused sweep of one instance; src selects the lattice read (0/1).
hipError_t launch_sweep(const InstDesc &d, int storage, bool mask, int src, const Launch &l,
                        hipStream_t stream);

// Whether a lattice of this instance fits one buffer resource (<= 4 GiB),
// which selects the buffer-instruction variant of the sweep.
bool buffer_addressable(const InstDesc &d, int storage);

// One fused sweep of every instance of a batch.  descs: device InstDesc[n];
// items: device int4[nitems] of (instance, strip, rowblock, 0); the lattice
// read by instance k is buf[descs[k].cur ^ flip].  `buf` may be true only if
// every instance is buffer_addressable.
hipError_t launch_sweep_batch(const InstDesc *descs, const int4 *items, int nitems, int storage,
                              bool mask, bool buf, int flip, const Launch &l,
                              hipStream_t stream);

// Pre-collision state <-> device FP64 [9][ny][nx]; f^eq initialisation.
hipError_t launch_set_populations(const InstDesc &d, int storage, int src, const double *f,
                                  hipStream_t stream);
hipError_t launch_get_populations(const InstDesc &d, int storage, int src, double *f,
                                  hipStream_t stream);
hipError_t launch_init_equilibrium(const InstDesc &d, int storage, int src, const double *rho,
                                   const double *ux, const double *uy, hipStream_t stream);
hipError_t launch_macros(const InstDesc &d, int storage, int src, double *rho, double *ux,
                         double *uy, hipStream_t stream);

// Diagnostics: partials must hold diag_partial_count() * TRT_NDIAG doubles.
int diag_partial_count();
hipError_t launch_diagnostics(const InstDesc &d, int storage, int src, double *partials,
                              double *out, double time, hipStream_t stream);
hipError_t launch_row_mean_ux(const InstDesc &d, int storage, int src, double *out,
                              hipStream_t stream);

}  // namespace trt
