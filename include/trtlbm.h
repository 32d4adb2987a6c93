/*
 * trtlbm.h -- C ABI of the MI355X (gfx950) D2Q9 TRT-RLB lattice Boltzmann
 * library.
 *
 * The library advances the two-relaxation-time regularized lattice Boltzmann
 * (TRT-RLB) model of Yu, Qin, Chen, Shu and Yuan, "Two-relaxation-time
 * regularized lattice Boltzmann model for Navier-Stokes equations"
 * (arXiv:2312.10318) on the GPU.  One time step is the evolution equation of
 * Sec. II.B (Eq. 2): density and He-shifted velocity (Eqs. 12-13), the
 * third-order Hermite equilibrium (Eq. 5), the regularized projections of the
 * non-equilibrium part (Eq. 6), relaxation of orders 1-2 at tau_s and of
 * order 3 at the free rate tau_s2, the cubic-error compensation G_i
 * (Eqs. 8-10) and the forcing term F_i (Eq. 11); then streaming with periodic
 * wrap and half-way bounce-back at solid nodes (Sec. II.D).  Lattice units
 * throughout: dx = dt = c = 1, c_s^2 = 1/3.
 *
 * Conventions shared by every call:
 *  - All calls return a trt_status; no C++ exception crosses the ABI.  On an
 *    error, trt_last_error() (thread-local, never NULL) holds a message.
 *  - Work is enqueued asynchronously on the HIP stream given at creation
 *    (a hipStream_t passed as void*; NULL is the legacy default stream).
 *    Results in device memory are ready once that stream reaches them.
 *  - The caller owns and frees every lattice-sized buffer (population
 *    lattices, mask, field arrays).  The library owns small scratch memory
 *    (reduction partials, batch tables), HIP graphs and, for a simulation
 *    with a mask or open x boundaries, a link map of two bytes per node
 *    (derived from the mask at creation: per node, whether it is solid and
 *    which of its pull sources are solid) with a summary of four bytes per
 *    row and 64 columns, all freed by the matching destroy call and counted
 *    by trt_footprint_bytes.
 *  - Population lattices are device buffers of trt_lattice_bytes() bytes,
 *    256-byte aligned, laid out row-interleaved as [y][i][x]: the nine
 *    population rows of lattice row y follow one another, each
 *    trt_pitch(nx, storage) elements long, so f_i of node (x, y) is element
 *    y * trt_row_stride(nx, storage) + i * trt_pitch(nx, storage) + x.
 *    (A row's pull reads then touch three consecutive lattice rows and its
 *    writes one, which the memory system serves faster than nine separate
 *    population planes.)  Storage TRT_F64 holds f_i;
 *    TRT_F32_SHIFTED / TRT_F16_SHIFTED hold f_i - w_i (the population minus
 *    its rest-state weight) rounded to nearest even.  The stored values are
 *    post-collision populations of the previous step (pull streaming); use
 *    trt_get_populations / trt_set_populations to read or write the
 *    pre-collision state f(x, t) in a storage-independent form.
 *  - Field arrays exchanged with the caller (rho, ux, uy, f) are dense FP64
 *    device arrays [ny][nx] (populations: [9][ny][nx]), x fastest.
 *  - The mask, when present, is a device uint8 array [ny][nx]; nonzero marks
 *    a solid node.  Solid nodes are never collided; their rho, u and f read
 *    back as 0 and they contribute nothing to diagnostics.  A mask whose
 *    solid nodes fill whole rows (walls parallel to x, as the channels of
 *    Sec. III.C) lets FP32 and FP16 simulations take several steps per
 *    launch.
 */
#ifndef TRTLBM_H
#define TRTLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TRT_OK = 0,
    TRT_EINVAL = 1,    /* invalid argument; nothing was enqueued */
    TRT_ENOMEM = 2,    /* library scratch allocation failed */
    TRT_EDEVICE = 3,   /* a HIP call failed; message in trt_last_error() */
    TRT_EUNSTABLE = 4, /* divergence detected (non-finite, rho <= 0 or |u| >= 1) */
    TRT_ESTATE = 5     /* call not valid in the object's current state */
} trt_status;

typedef enum {
    TRT_F64 = 0,         /* FP64 storage, FP64 arithmetic */
    TRT_F32_SHIFTED = 1, /* FP32 storage of f - w, FP32 arithmetic */
    TRT_F16_SHIFTED = 2  /* IEEE half storage of f - w, FP32 arithmetic */
} trt_storage;

typedef enum {
    TRT_X_PERIODIC = 0,       /* periodic in x (and always in y) */
    TRT_X_INFLOW_OUTFLOW = 1  /* inflow wall at x = -1/2, pressure outlet at x = nx - 1 */
} trt_x_boundary;

/* One simulation: the problem statement of the paper (Sec. II.B-II.D), and
 * optionally the open x boundaries of the creeping flow of Sec. III.D:
 *  - inflow: a half-way bounce-back wall at x = -1/2 moving with (u_in, 0);
 *    a population leaving column 0 through it returns with the moving-wall
 *    correction -2 w_i rho_in (e_i . u_wall) / c_s^2 (Ladd's rule);
 *  - outflow: column nx - 1 held at density rho_out with zero transverse
 *    velocity; its three populations entering from outside follow Zou and
 *    He's pressure rule; populations leaving through x = nx are lost;
 *  - the gradient of Phi = rho u^3 sees rho_in u_in^3 beyond the inflow
 *    wall and the last column's value beyond the outlet.
 * Neither rule includes the body force.  Open-boundary lattices run the
 * sweep with the link map (one or two columns per lane). */
typedef struct {
    int32_t nx, ny;        /* lattice size, 1..46340 each; periodic in y (and x unless open) */
    double tau_s;          /* tau_s1 > 1/2: viscosity nu = (tau_s - 1/2)/3 (Sec. II.C) */
    double tau_s2;         /* tau_s2 >= 1/2: free third-order rate (Sec. II.B) */
    double gx, gy;         /* body acceleration g; the force is F = rho g (Sec. II.D) */
    const uint8_t *mask;   /* device [ny][nx], nonzero = solid (half-way bounce-back); NULL = none */
    int32_t storage;       /* trt_storage */
    int32_t x_boundary;    /* trt_x_boundary (0: periodic) */
    double u_in;           /* inflow wall velocity (x), lattice units; open x only */
    double rho_in;         /* density in the inflow wall's correction (> 0); open x only */
    double rho_out;        /* outlet density (> 0); open x only */
} trt_problem;

/* Launch shape of the fused sweep.  Zero fields take the built-in default
 * (rows per wavefront chosen from the lattice size, wavefronts per
 * workgroup chosen per storage, XCD remap on, two columns per lane where
 * that applies).  trt_get_tuning reports the rows, wavefronts per workgroup,
 * columns per lane, time steps per launch and prefetch rows in effect
 * (prefetch_rows 0 when the simulation takes one step per launch).
 * Two columns per lane (a wavefront sweeps 128-column strips with one
 * paired access per population) applies to lattices of at most 4 GiB whose
 * width is not 1 mod 128, with or without a mask or open boundaries;
 * elsewhere the sweep uses one column per lane whatever is asked.  The two
 * shapes compute the same arithmetic per node. */
typedef struct {
    int32_t rows_per_wave;   /* rows one wavefront marches through, 1..4096 (0: automatic) */
    int32_t waves_per_block; /* wavefronts per workgroup: 1, 2, 4, 8 or 16 (0: automatic); the
                                one-column and batched sweeps and the two-step pass use at
                                most 4, the two-column sweep at most 16 (FP64: 8) */
    int32_t xcd_remap;       /* 1: give each XCD a contiguous band of rows; 0: off; -1: default
                                (on for one simulation -- except three-step launches in
                                their automatic rows from about 1500^2 nodes on, or of at
                                least 3072 wavefronts, which run off -- and off for a
                                batch) */
    int32_t cols_per_lane;   /* 1 or 2 columns per lane (0: 2 where it applies and nx >= 128) */
    /* Batches only (ignored for one simulation; rows_per_wave > 0 overrides
     * both): how members are cut into work items of one wavefront each. */
    int32_t batch_items;     /* 0: default; -1: every member keeps the rows it would have
                                alone; n > 0: one batch-wide cap on the rows, the longest
                                (a power of two in 4..256) that still leaves at least n work
                                items -- members no taller than the cap sweep their whole
                                height as one item per strip, taller ones in equal blocks */
    int32_t batch_order;     /* 0: default; 1: member by member; 2: costliest items (rows x
                                columns) first, so short items fill in at the end */
    int32_t graph_steps;     /* longest captured HIP graph, in sweeps: a power of two in
                                2..1024 (0: default, 64).  trt_step / trt_batch_step replay
                                whole graphs of this length, then one graph per binary digit
                                of the rest (graphs of 2, 4, ... sweeps, captured at first
                                use): the GPU idles ~8 us at each graph boundary and ~0.2 us
                                between the sweeps inside one graph. */
    int32_t steps_per_sweep; /* time steps per launch: 1, 2 or 3 (0: automatic -- three for
                                FP32 simulations of at least 2048^2 nodes that allow it, else
                                two where allowed; in a batch three for FP32 members, two for
                                FP16).  k steps per launch move each
                                population through HBM once per k steps and give the bits of
                                k one-step sweeps.  Two apply to FP32 and FP16 simulations,
                                alone or in a batch, without a mask or open boundaries, or
                                with a mask whose solid nodes fill whole rows (x periodic);
                                three to such FP32 simulations, alone or in an FP32 batch;
                                elsewhere sweeps take fewer steps.  With
                                two or three steps per launch, rows_per_wave and
                                waves_per_block shape that pass (cols_per_lane the one-step
                                sweeps of leftover steps). */
    int32_t prefetch_rows;   /* two-step pass: how many rows ahead of their use its loads
                                are issued, 1 or 2 (0: automatic -- 2 for FP32 launches of
                                at least 4096 wavefronts, else 1; the three-step pass always
                                loads one row ahead).  Two rows ahead keeps
                                more loads in flight per wavefront but needs more
                                registers, so fewer wavefronts fit on a SIMD.  No effect on
                                results. */
} trt_tuning;

typedef struct trt_sim trt_sim;
typedef struct trt_batch trt_batch;

/* Number of FP64 values written by trt_diagnostics, and their order:
 *   [0] sum of rho over fluid nodes (mass)
 *   [1] sum of rho u_x, [2] sum of rho u_y (He-shifted velocity, Eq. 13)
 *   [3] max |u| over fluid nodes with finite values
 *   [4] number of divergent fluid nodes (non-finite rho or u, rho <= 0, or
 *       |u| >= 1 = c)
 *   [5] number of fluid nodes
 *   [6] min rho over fluid nodes with finite values
 *   [7] time steps taken since creation or the last trt_set_populations */
#define TRT_NDIAG 8

/* Elements of one population row: nx rounded up so each population row is
 * a multiple of 256 B (the nine population rows of a lattice row follow one
 * another; see trt_row_stride).  Returns -1 for an invalid size or storage. */
int32_t trt_pitch(int32_t nx, int32_t storage);

/* Elements between lattice rows y and y+1 of a population lattice (nine
 * population rows: 9 * trt_pitch).  -1 if invalid. */
int64_t trt_row_stride(int32_t nx, int32_t storage);

/* Bytes of one population lattice (ny * trt_row_stride elements).  0 if the
 * problem is invalid. */
size_t trt_lattice_bytes(const trt_problem *p);

/* Device bytes one simulation needs: two lattices, the mask, and the
 * library's scratch.  Used for admission by memory budget.  0 if invalid. */
size_t trt_footprint_bytes(const trt_problem *p);

/* Create a simulation over two caller-owned lattices f_a and f_b (ping-pong:
 * each step reads one and writes the other; they must not overlap).  The
 * state starts undefined: call trt_init_equilibrium or trt_set_populations
 * next.  The problem (including the mask pointer) is copied; the mask memory
 * must stay valid while the simulation exists, and its contents must not
 * change (the sweep reads the link map derived from it on the stream at
 * creation).  The mask must hold its contents when trt_create is called:
 * with periodic x it is also read at once, on a stream of the library's own
 * (created at the first such call per device, kept until the process
 * ends), and waited for there, to find whether its solid nodes fill whole
 * rows -- so creation does not wait for the work queued on hip_stream.
 * EINVAL on a NULL or
 * misaligned pointer, a size out of range, tau_s <= 1/2, tau_s2 < 1/2 or a
 * non-finite parameter.  With a mask or open x boundaries the link map
 * (2 * ny * (nx rounded up to 128) bytes) must stay below 4 GiB, which
 * excludes nx > 46336 together with ny > 46218. */
trt_status trt_create(const trt_problem *p, void *f_a, void *f_b, void *hip_stream,
                      trt_sim **out);

/* Replace the sweep's launch shape (re-captures the step graph). */
trt_status trt_set_tuning(trt_sim *s, const trt_tuning *t);
trt_status trt_get_tuning(const trt_sim *s, trt_tuning *t);

/* f(x, 0) = f^eq(rho, u), the third-order Hermite equilibrium of Eq. 5, at
 * every fluid node (no non-equilibrium part).  rho, ux, uy: device FP64
 * [ny][nx]; ux, uy are the velocities that enter f^eq.  Resets time to 0. */
trt_status trt_init_equilibrium(trt_sim *s, const double *rho, const double *ux,
                                const double *uy);

/* Set the pre-collision state f(x, t) from a device FP64 array [9][ny][nx]
 * (unshifted populations; entries at solid nodes are ignored).  Resets
 * time to 0. */
trt_status trt_set_populations(trt_sim *s, const double *f);

/* Read the pre-collision state f(x, t) into a device FP64 array
 * [9][ny][nx] (unshifted; 0 at solid nodes). */
trt_status trt_get_populations(trt_sim *s, double *f);

/* Advance nsteps >= 0 time steps (Eq. 2 followed by streaming), enqueued on
 * the stream as replays of captured HIP graphs (see trt_tuning.graph_steps)
 * plus at most three plain launches; two or three time steps per launch
 * where trt_tuning.steps_per_sweep allows it.  Any split of the steps, and
 * any number of steps per launch, gives the same bits. */
trt_status trt_step(trt_sim *s, int64_t nsteps);

/* Capture the step graphs that trt_step(s, nsteps) would replay from the
 * current state, without launching anything (the state and time are
 * unchanged), so that a later trt_step(s, nsteps) spends no host time on
 * capture.  Graphs stay captured until the launch shape changes. */
trt_status trt_prepare_steps(trt_sim *s, int64_t nsteps);

/* A measurement aid, not a step of the method: nsweeps launches that move
 * the lattice holding the state to the other one (alternating) with the
 * access pattern of the simulation's sweep -- its launch shape, the pull's
 * nine population-row loads per lattice row (rows y, y - 1, y + 1 by
 * population), the strip edges' extra loads, nine stores per row, one
 * barrier per row -- and none of its arithmetic.  Its time per launch is the
 * bandwidth ceiling of the sweep's access pattern on the same lattice.  The
 * populations are scrambled: set the state again before stepping.  EINVAL
 * unless the lattice is open and periodic, nx is a multiple of 128, it fits
 * 4 GiB and the sweep runs two columns per lane. */
trt_status trt_pattern_probe(trt_sim *s, int64_t nsweeps);

/* rho and He-shifted u (Eq. 13) at time t into device FP64 [ny][nx];
 * 0 at solid nodes.  Any of the three pointers may be NULL. */
trt_status trt_macros(trt_sim *s, double *rho, double *ux, double *uy);

/* FP64 diagnostics (see TRT_NDIAG) into device memory out[TRT_NDIAG],
 * reduced in a fixed order (bitwise reproducible). */
trt_status trt_diagnostics(trt_sim *s, double *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * diagnostics of trt_diagnostics for a population lattice the caller holds,
 * with no simulation object and no allocation of any kind.
 *  - p: the problem the lattice belongs to (validated as by trt_create; its
 *    mask, if any, is read on the device).
 *  - lattice: the lattice holding the current state (the one trt_state
 *    names), 256-byte aligned, trt_lattice_bytes(p) bytes, storage p->storage.
 *  - time: copied to out[7].
 *  - out: device FP64 out[TRT_NDIAG], bitwise equal to trt_diagnostics on
 *    the same state (same kernels, same fixed reduction order).
 *  - hip_stream: the stream to enqueue on (NULL: the legacy default stream).
 * Scratch: the reduction partials live in one static device array of 512 x
 * TRT_NDIAG doubles (32 KiB) per GPU, held until the process ends; every
 * lattice trt_create accepts needs exactly that many, and any other size or
 * argument trt_create would refuse is rejected with TRT_EINVAL before any HIP
 * call.  The first call on a device looks the array's address up there (a
 * HIP call that must not run under stream capture: make one call on each
 * device before capturing).  All calls on one GPU share the array: calls
 * whose work overlaps on that GPU (different streams, no ordering between
 * them) race and may return wrong sums; calls ordered on one stream do not. */
trt_status trt_diagnostics_noalloc(const trt_problem *p, const void *lattice, int64_t time,
                                   double *out, void *hip_stream);

/* Mean of u_x over the fluid nodes of each row, FP64, into device
 * out[ny] (0 for a row without fluid) -- the slip measurement of Sec. III.C. */
trt_status trt_row_mean_ux(trt_sim *s, double *out);

/* Momentum handed to the solid nodes by the last collision (the drag of
 * Sec. III.D, momentum exchange): every link from a fluid node x_f to a
 * solid node x_f + e_i carries e_i [f*_i(x_f) + f*_opp(i)(x_s)] = 2 e_i
 * f*_i(x_f) under half-way bounce-back.  Links through open x ends are not
 * wall links.  Device FP64 out[2] = (F_x, F_y), fixed-order reduction.
 * ESTATE before the first step after the state was set.  Uses library
 * scratch: calls on one simulation are ordered by its stream. */
trt_status trt_wall_force(trt_sim *s, double *out);

/* Steady-state test (Sec. III, convergence criterion): compares the current
 * He-shifted velocity with prev_ux, prev_uy (device FP64 [ny][nx], caller
 * owned) over the fluid nodes and then overwrites them with the current
 * velocity.  Device FP64 out[4] = (max over nodes and components of
 * |u - u_prev|, sum |u - u_prev|^2, sum |u|^2, sum |u_prev|^2); the
 * criterion of Sec. III is out[0] / u_c, a relative L2 change is
 * sqrt(out[1] / out[2]).  Uses library scratch. */
trt_status trt_velocity_change(trt_sim *s, double *prev_ux, double *prev_uy, double *out);

/* Error against a reference velocity field (the relative L2 error of
 * Sec. III): the same four sums as trt_velocity_change with ref_ux, ref_uy
 * (device FP64 [ny][nx], not modified) in place of the previous field; the
 * relative L2 error is sqrt(out[1] / out[3]).  Uses library scratch. */
trt_status trt_velocity_error(trt_sim *s, const double *ref_ux, const double *ref_uy,
                              double *out);

/* Synchronous check: runs trt_diagnostics into library scratch, waits for
 * the stream, and returns TRT_EUNSTABLE if any fluid node diverged. */
trt_status trt_check(trt_sim *s);

/* Which caller lattice holds the current state (0 = f_a, 1 = f_b), and the
 * steps taken. */
trt_status trt_state(const trt_sim *s, int32_t *current, int64_t *time);

void trt_destroy(trt_sim *s);

/* ---- batching: many independent simulations advanced by one launch per
 * step.  All members must share one storage type and stream; each keeps its
 * own lattices, parameters and time.  The member objects must outlive the
 * batch and must not be stepped on their own while it exists. ---- */

/* Build the tile work list over n >= 1 simulations. */
trt_status trt_batch_create(int32_t n, trt_sim *const *sims, trt_batch **out);

/* Replace the members by n >= 1 simulations (same rules as create; members
 * may stay).  Members that leave may be stepped on their own or destroyed
 * afterwards.  The call does not wait for the launches already enqueued:
 * the new tables are copied on the batch's stream behind them, from one of
 * a ring of pinned staging buffers, and the call waits at most for the copy
 * that last used that buffer (several updates earlier).  Serving uses this
 * at every change of the active set. */
trt_status trt_batch_update(trt_batch *b, int32_t n, trt_sim *const *sims);

/* Advance every member nsteps steps (replays of captured graphs of batched
 * launches as for trt_step, plus at most a few plain launches).  With
 * the default steps_per_sweep, members that allow it (FP32 or FP16 without
 * a mask or open boundaries, or with walls that fill whole rows) advance
 * three (FP32) or two (FP16) steps per launch and the others by one-step
 * sweeps in the same graphs; every member gets the bits it gets alone. */
trt_status trt_batch_step(trt_batch *b, int64_t nsteps);

/* Diagnostics of every member into device out[n][TRT_NDIAG]. */
trt_status trt_batch_diagnostics(trt_batch *b, double *out);

/* Launch shape used for the whole batch. */
trt_status trt_batch_set_tuning(trt_batch *b, const trt_tuning *t);

/* The batch's launch shape as set (0 where automatic); steps_per_sweep
 * reports 2 only if some member takes two-step launches, prefetch_rows the
 * two-step launches' rows ahead in effect (0 without such members).  EINVAL
 * for a NULL handle or out. */
trt_status trt_batch_get_tuning(const trt_batch *b, trt_tuning *t);

void trt_batch_destroy(trt_batch *b);

/* Thread-local description of the last error; never NULL. */
const char *trt_last_error(void);

/* Library version string. */
const char *trt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TRTLBM_H */
