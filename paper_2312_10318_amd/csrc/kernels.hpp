// kernels.hpp -- host-side launchers of the device kernels (internal to the
// library; the public interface is include/trtlbm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.hpp"

namespace trt {

struct Launch {
    int rows_per_wave;    // 0: chosen per lattice by auto_rows()
    int waves_per_block;  // 0: chosen per storage and column mode
    int xcd_remap;
    int cols_per_lane;    // 0: two-column strips wherever they apply; 1 or 2
    // batches only (see trt_tuning): the minimum number of work items that
    // sets one batch-wide row cap (-1: each member's own rows), and the
    // work-list order (1: member by member, 2: costliest items first)
    int batch_items;
    int batch_order;
    int graph_steps;  // sweeps per captured graph (even)
    int steps_per_sweep;  // 2 or 3: time steps per launch where tb2_eligible / tb3_eligible
    int prefetch_rows;    // two-step pass: loads 1 or 2 rows ahead (0: automatic)
    int remap_asked;      // xcd_remap was set by the caller (else the pass's default)
};

// Wavefronts per workgroup of a single-lattice sweep.  The one-column
// kernels take at most 4 (256 threads), the two-column kernels 16 (FP64:
// 8, for its register budget).  The two-column workgroups are synchronised
// per row, and wider ones keep more adjacent strips in step: measured best
// on 4096^2 are 8 (FP32) and 16 (FP16); FP64 gains nothing beyond 4.  A
// workgroup never has more wavefronts than the lattice has strips (rounded
// up to a power of two).  When the choice is automatic it is also halved
// until at most one in eight wavefronts of a row block's workgroups has no
// strip: those only meet barriers, and on narrow lattices they cost more
// than wide workgroups gain (1050^2, 9 strips: 8 wavefronts 27.3 GLUPS FP32,
// 2 wavefronts 42.9).
inline int single_waves_per_block(const InstDesc &d, int storage, const Launch &l) {
    if (d.cols != 2) return l.waves_per_block > 0 ? (l.waves_per_block < 4 ? l.waves_per_block : 4) : 4;
    const int cap = storage == ST_F64 ? 8 : 16;
    // FP16 with a link map: 8 (4096^2, obstacle: 55.5% of peak against 53.0
    // with 16)
    const int fp16 = d.links != nullptr ? 8 : 16;
    int w = l.waves_per_block > 0 ? l.waves_per_block
                                  : (storage == ST_F16 ? fp16 : (storage == ST_F32 ? 8 : 4));
    if (w > cap) w = cap;
    while (w > 1 && w / 2 >= d.strips) w /= 2;
    if (l.waves_per_block <= 0) {
        auto slots = [&](int v) { return (d.strips + v - 1) / v * v; };
        while (w > 1 && 8 * (slots(w) - d.strips) > slots(w)) w /= 2;
    }
    return w;
}

// Wavefronts per workgroup of a batched sweep (at most 4; default 4).
inline int batch_waves_per_block(const Launch &l) {
    return l.waves_per_block > 0 ? (l.waves_per_block < 4 ? l.waves_per_block : 4) : 4;
}

// Whether an instance can use two-column strips: nx not 1 mod 128 (the
// last strip holds at least two columns, so no lane is both edges), a
// lattice within one buffer resource, and, with obstacles or open
// boundaries, its link map.
bool pair_eligible(const InstDesc &d, int storage);

// Rows per wavefront when the launch shape leaves it open.  Long strips
// re-read fewer halo rows, but a lattice must still give the 1024 SIMDs
// enough wavefronts, and narrower storage needs more of them to keep enough
// bytes in flight.  Measured optima on 4096^2: with 64-column strips FP32
// 128 rows (~2048 wavefronts), FP64 64 rows (~4096), FP16 16-32 rows
// (~8192); with two-column strips in synchronised workgroups FP32 64 rows
// (~2048), FP64 128 (~1024: one 4-wavefront workgroup per CU), FP16 32
// (~4096).  The rows are the largest power of two in [4, 128] that leaves
// at least that many wavefronts.  Lattices with a link map (walls,
// obstacles, open boundaries) aim for twice as many: the rows that cross an
// obstacle cost more, and more, shorter workgroups per CU let the hardware
// balance them (4096^2, centred 84^2 obstacle, two-column strips: FP64
// 66.6 -> 70.3%, FP32 60.4 -> 62.8%, FP16 50.9 -> 55.5% of peak; channel
// walls change by +1.4 / -0.9 / +0.2 points).
inline int auto_rows(int nx, int ny, int storage, int cols, bool linked) {
    const int width = kStripWidth * cols;
    const int strips = (nx + width - 1) / width;
    const long long open = cols == 2 ? (storage == ST_F16 ? 4096 : (storage == ST_F32 ? 2048 : 1024))
                                     : (storage == ST_F64 ? 4096 : (storage == ST_F32 ? 2048 : 8192));
    const long long target = linked ? 2 * open : open;
    const long long per = (long long)strips * ny / target;
    int r = 4;
    while (r < 128 && (long long)(2 * r) <= per) r *= 2;
    return r;
}

// Tiling of one instance for a launch shape.
inline void tile(InstDesc &d, const Launch &l, int storage) {
    const bool can = pair_eligible(d, storage);
    d.cols = (l.cols_per_lane == 1 || !can) ? 1 : (l.cols_per_lane == 2 || d.nx >= 2 * kStripWidth ? 2 : 1);
    d.rows = l.rows_per_wave > 0 ? l.rows_per_wave
                                 : auto_rows(d.nx, d.ny, storage, d.cols, d.links != nullptr);
    d.strips = (d.nx + kStripWidth * d.cols - 1) / (kStripWidth * d.cols);
    d.rowblocks = (d.ny + d.rows - 1) / d.rows;
}

// One fused sweep of one instance; src selects the lattice read (0/1).
hipError_t launch_sweep(const InstDesc &d, int storage, bool mask, int src, const Launch &l,
                        hipStream_t stream);

// Whether a lattice of this instance fits one buffer resource (<= 4 GiB),
// which selects the buffer-instruction variant of the sweep.
bool buffer_addressable(const InstDesc &d, int storage);

// One fused sweep of every instance of a batch.  descs: device InstDesc[n];
// items: device int4[nitems] of (instance, strip, rowblock, class); the
// lattice read by instance k is buf[descs[k].cur ^ flip] for class 0 and
// buf[descs[k].cur ^ flip1] for class 1.  `buf` may be true only if
// every instance is buffer_addressable; instances with descs[k].cols == 2
// (tiled so only where pair_eligible) are swept with two-column strips.
hipError_t launch_sweep_batch(const InstDesc *descs, const int4 *items, int nitems, int storage,
                              bool mask, bool buf, int flip, int flip1, const Launch &l,
                              hipStream_t stream);
// Two time steps of the batch members named by items (device int4 of
// (index into descs, window, row block, -); descs: device InstDesc[ndescs]
// tiled by tb2_desc): each reads lattice cur ^ flip.  Items naming no
// descriptor are skipped.  deep: loads two rows ahead
// (tb2_batch_prefetch_rows).
hipError_t launch_sweep_tb2_batch(const InstDesc *descs, int ndescs, const int4 *items,
                                  int nitems, int storage, int flip, bool deep, const Launch &l,
                                  hipStream_t stream);

// Two time steps per launch (FP32 or FP16 storage, open periodic lattices):
// reads lattice src, writes the other one, two steps later.
// Gives the bits of two one-step sweeps.  A wavefront computes a
// 128-column window and stores its middle kTb2Valid columns.
constexpr int kTb2Valid = 120;
bool tb2_eligible(const InstDesc &d, int storage);
// The tiling of the two-step pass: windows of 120 stored columns and,
// unless the launch shape sets them, rows per wavefront for at least 6144
// wavefronts (else 2048).
InstDesc tb2_desc(const InstDesc &d, const Launch &l);
// Wavefronts per workgroup of the two-step pass (at most four).
int tb2_waves_per_block(const InstDesc &d, int storage, const Launch &l);
// Rows ahead of their use that the two-step pass issues its loads: 1 or 2.
int tb2_prefetch_rows(const InstDesc &d, int storage, const Launch &l);
// The same for the batched two-step pass over `items` work items.
int tb2_batch_prefetch_rows(int items, int storage, const Launch &l);
hipError_t launch_sweep_tb2(const InstDesc &d, int storage, int src, const Launch &l,
                            hipStream_t stream);

// Three time steps per launch (FP32 storage, open periodic lattices, as
// for two): reads lattice src, writes the other one, three steps later,
// with the bits of three one-step sweeps.  A wavefront computes a
// 128-column window and stores its middle kTb3Valid columns.
constexpr int kTb3Valid = 116;
bool tb3_eligible(const InstDesc &d, int storage);
InstDesc tb3_desc(const InstDesc &d, const Launch &l);
int tb3_waves_per_block(const InstDesc &d, const Launch &l);
int tb3_prefetch_rows(const InstDesc &d, const Launch &l);
// XCD remap of the three-step pass: as asked, else off from kTb3ManyWaves
// wavefronts on and on below.
int tb3_xcd_remap(const InstDesc &d, const Launch &l);
hipError_t launch_sweep_tb3(const InstDesc &d, int storage, int src, const Launch &l,
                            hipStream_t stream);
// Three time steps of the batch members named by items, as
// launch_sweep_tb2_batch (descs tiled by tb3_desc; FP32 only).
hipError_t launch_sweep_tb3_batch(const InstDesc *descs, int ndescs, const int4 *items,
                                  int nitems, int storage, int flip, const Launch &l,
                                  hipStream_t stream);

// The access-pattern probe (a measurement aid): one launch moves the lattice
// `src` to the other one with the two-column sweep's loads, stores, launch
// shape and barriers and none of its arithmetic.  Only for two-column
// tilings of open periodic lattices whose width is a multiple of 128 and
// that fit one buffer resource (else hipErrorInvalidValue).
hipError_t launch_pattern_probe(const InstDesc &d, int storage, int src, const Launch &l,
                                hipStream_t stream);

// Link map of an instance with a mask or open x boundaries: d.links (device,
// ny * d.lpitch 16-bit codes) receives, per node, bit 0 = solid and bit i
// (1..8) = the pull source x - e_i is solid or beyond the inflow wall; then
// d.rowsum receives the link summary (see InstDesc).
hipError_t launch_link_map(const InstDesc &d, hipStream_t stream);

// *mixed (device int) = 0 when every row of the dense [ny][nx] mask is all
// solid or all fluid, else 1.
hipError_t launch_mask_rows(const uint8_t *mask, int nx, int ny, int *mixed, hipStream_t stream);

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

// Momentum handed to solid nodes by the last collision (the post-collision
// lattice `src`): out[2] = (F_x, F_y).  partials as for the diagnostics.
hipError_t launch_wall_force(const InstDesc &d, int storage, int src, double *partials,
                             double *out, hipStream_t stream);

// He-shifted velocity against reference fields ref_ux, ref_uy (dense FP64
// [ny][nx]) over the fluid nodes: out[0] = max over nodes and components of
// |u - u_ref|, out[1] = sum |u - u_ref|^2, out[2] = sum |u|^2, out[3] =
// sum |u_ref|^2; with `update` the reference fields are then replaced by u.
hipError_t launch_velocity_compare(const InstDesc &d, int storage, int src, double *ref_ux,
                                   double *ref_uy, bool update, double *partials, double *out,
                                   hipStream_t stream);

}  // namespace trt
