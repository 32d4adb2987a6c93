// api.hip -- the C ABI of include/trtlbm.h: argument validation, the
// simulation and batch objects, step-graph capture and error reporting.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/trtlbm.h"
#include "kernels.hpp"

using trt::InstDesc;
using trt::Launch;

namespace {

thread_local std::string g_err = "no error";

// Record the message of a failing call.  No C++ exception may leave the C
// ABI: a message that cannot be stored (out of host memory) is dropped.
trt_status fail(trt_status st, const char *msg) noexcept {
    try {
        g_err = msg;
    } catch (...) {
    }
    return st;
}

trt_status fail_hip(hipError_t e, const char *what) noexcept {
    try {
        g_err = std::string(what) + ": " + hipGetErrorString(e);
    } catch (...) {
    }
    return TRT_EDEVICE;
}

// Run an entry point's body that uses host containers; an allocation
// failure becomes TRT_ENOMEM instead of an exception crossing the C ABI.
template <class F>
trt_status guarded(F &&body) noexcept {
    try {
        return body();
    } catch (const std::bad_alloc &) {
        return fail(TRT_ENOMEM, "out of host memory");
    } catch (...) {
        return fail(TRT_EDEVICE, "unexpected host error");
    }
}

#define TRT_HIP(expr)                                    \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return fail_hip(e_, #expr); \
    } while (0)

// Default launch shape: rows per wave chosen per lattice (auto_rows), four
// wavefronts per workgroup, XCD-contiguous workgroup order.
// Sweeps per captured graph: graphs of 2, 4, ..., graph_steps sweeps are
// captured as needed (graph level k holds 2^(k+1) sweeps), and trt_step
// replays whole graphs of graph_steps sweeps, then one graph per binary digit
// of the rest.  Between sweeps inside one graph the GPU idles ~0.2 us, at a
// graph boundary ~8 us (kernel trace of 126 double-shear-layer lattices of
// 128^2, FP64, 62 us per batched sweep: 4.1 us per step with two-sweep graphs,
// 0.25 with 128); 4096^2 FP32 214.0 -> 210.9 us per step.
// Several time steps per launch wherever the lattice allows it (FP32 or
// FP16 storage, open periodic; sim_k): two steps per launch took FP32
// 4096^2 from 210 to 127 us per step, 2048^2 59.6 -> 35.7, 1024^2 19.6 ->
// 12.6, FP16 4096^2 118 -> 85, 2048^2 36.0 -> 26.4; three (FP32 from 2048^2
// on) take 4096^2 to 96, 8192^2 to 346 (two steps: 122, 454); bit for bit
// the same results.
constexpr int kMaxGraphLevels = 10;  // up to 1024 sweeps per graph
constexpr int kDefaultGraphSteps = 64;
constexpr Launch kDefaultLaunch = {0, 0, 1, 0, 0, 0, kDefaultGraphSteps, 0, 0};
// Batches: no XCD remap by default.  A batch's work list runs member by
// member, and spreading each member's items over all XCDs (the hardware's
// round-robin) measured 3% faster than giving XCDs contiguous ranges of the
// list (256 members of 64^2 ... 1024^2, FP32: 67.7 against 65.8 GLUPS).
constexpr Launch kBatchDefaultLaunch = {0, 0, 0, 0, -1, 1, kDefaultGraphSteps, 0, 0};
constexpr int kMaxSide = 46340;

int elem_size(int storage) {
    switch (storage) {
        case TRT_F64: return 8;
        case TRT_F32_SHIFTED: return 4;
        case TRT_F16_SHIFTED: return 2;
        default: return 0;
    }
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

trt_status check_problem(const trt_problem *p) {
    if (!p) return fail(TRT_EINVAL, "problem is NULL");
    if (elem_size(p->storage) == 0) return fail(TRT_EINVAL, "unknown storage type");
    if (p->nx < 1 || p->ny < 1 || p->nx > kMaxSide || p->ny > kMaxSide)
        return fail(TRT_EINVAL, "nx and ny must lie in [1, 46340]");
    if (!isfinite(p->tau_s) || !(p->tau_s > 0.5))
        return fail(TRT_EINVAL, "tau_s must be finite and > 1/2");
    if (!isfinite(p->tau_s2) || !(p->tau_s2 >= 0.5))
        return fail(TRT_EINVAL, "tau_s2 must be finite and >= 1/2");
    if (!isfinite(p->gx) || !isfinite(p->gy)) return fail(TRT_EINVAL, "g must be finite");
    if (p->x_boundary != TRT_X_PERIODIC && p->x_boundary != TRT_X_INFLOW_OUTFLOW)
        return fail(TRT_EINVAL, "x_boundary must be TRT_X_PERIODIC or TRT_X_INFLOW_OUTFLOW");
    // The link map of a lattice with a mask or open x boundaries (two bytes
    // per node, rows of nx rounded up to 128 codes) is read through one
    // buffer resource, whose byte range and offsets are 32-bit: it must stay
    // below 4 GiB (this excludes only nx > 46336 with ny > 46218).
    if ((p->mask != nullptr || p->x_boundary == TRT_X_INFLOW_OUTFLOW) &&
        2 * (uint64_t)p->ny * (((uint64_t)p->nx + 127) / 128 * 128) >= (1ull << 32))
        return fail(TRT_EINVAL,
                    "with a mask or open x boundaries, 2 * ny * (nx rounded up to 128) must be "
                    "below 2^32 (the link map's 4 GiB limit)");
    if (p->x_boundary == TRT_X_INFLOW_OUTFLOW) {
        if (p->nx < 2) return fail(TRT_EINVAL, "open x boundaries need nx >= 2");
        if (!isfinite(p->u_in) || !isfinite(p->rho_in) || !isfinite(p->rho_out) ||
            !(p->rho_in > 0.0) || !(p->rho_out > 0.0))
            return fail(TRT_EINVAL, "u_in must be finite and rho_in, rho_out finite and > 0");
    }
    return TRT_OK;
}

trt_status check_launch(const trt_tuning *t, Launch &l, const Launch &defaults) {
    l = defaults;
    if (!t) return TRT_OK;
    if (t->rows_per_wave != 0) {
        if (t->rows_per_wave < 1 || t->rows_per_wave > 4096)
            return fail(TRT_EINVAL, "rows_per_wave must be 0 (automatic) or lie in [1, 4096]");
        l.rows_per_wave = t->rows_per_wave;
    }
    if (t->waves_per_block != 0) {
        const int w = t->waves_per_block;
        if (w != 1 && w != 2 && w != 4 && w != 8 && w != 16)
            return fail(TRT_EINVAL, "waves_per_block must be 0 (automatic), 1, 2, 4, 8 or 16");
        l.waves_per_block = t->waves_per_block;
    }
    if (t->xcd_remap != -1) {
        if (t->xcd_remap != 0 && t->xcd_remap != 1)
            return fail(TRT_EINVAL, "xcd_remap must be -1, 0 or 1");
        l.xcd_remap = t->xcd_remap;
        l.remap_asked = 1;
    }
    if (t->cols_per_lane != 0) {
        if (t->cols_per_lane != 1 && t->cols_per_lane != 2)
            return fail(TRT_EINVAL, "cols_per_lane must be 0 (automatic), 1 or 2");
        l.cols_per_lane = t->cols_per_lane;
    }
    if (t->batch_items != 0) {
        if (t->batch_items < -1 || t->batch_items > (1 << 24))
            return fail(TRT_EINVAL, "batch_items must be 0 (default), -1 or lie in [1, 2^24]");
        l.batch_items = t->batch_items;
    }
    if (t->batch_order != 0) {
        if (t->batch_order != 1 && t->batch_order != 2)
            return fail(TRT_EINVAL, "batch_order must be 0 (default), 1 or 2");
        l.batch_order = t->batch_order;
    }
    if (t->graph_steps != 0) {
        const int g = t->graph_steps;
        if (g < 2 || g > (2 << (kMaxGraphLevels - 1)) || (g & (g - 1)) != 0)
            return fail(TRT_EINVAL,
                        "graph_steps must be 0 (default) or a power of two in [2, 1024]");
        l.graph_steps = g;
    }
    if (t->steps_per_sweep != 0) {
        if (t->steps_per_sweep < 1 || t->steps_per_sweep > 3)
            return fail(TRT_EINVAL, "steps_per_sweep must be 0 (default), 1, 2 or 3");
        l.steps_per_sweep = t->steps_per_sweep;
    }
    if (t->prefetch_rows != 0) {
        if (t->prefetch_rows != 1 && t->prefetch_rows != 2)
            return fail(TRT_EINVAL, "prefetch_rows must be 0 (automatic), 1 or 2");
        l.prefetch_rows = t->prefetch_rows;
    }
    return TRT_OK;
}

}  // namespace

struct trt_sim {
    trt_problem prob;
    hipStream_t stream;
    InstDesc desc;  // desc.cur stays 0: the lattice read is passed per launch
    Launch launch;
    int cur;        // lattice holding the current state
    int64_t time;
    double *scratch;  // diagnostics partials + one TRT_NDIAG result
    uint16_t *links;  // link map (mask or open x boundaries), else null
    hipStream_t cap_stream;
    // captured graphs: level k holds 2^(k+1) sweeps, starting and ending on
    // lattice 0 (null until first used)
    hipGraphExec_t graphs[kMaxGraphLevels];
    bool in_batch;
};

struct trt_batch {
    std::vector<trt_sim *> sims;
    int storage;
    bool mask;
    bool buf;  // every member fits one buffer resource
    hipStream_t stream;
    Launch launch;
    InstDesc *d_descs;  // device tables, grown by doubling and reused
    int4 *d_items;
    size_t cap_descs, cap_items;
    // Pinned staging of the tables: a ring of slots, each reused only once
    // the copy that last read it has run (its event), so a membership
    // change waits for a copy several changes old, not for the work queued
    // on the stream ahead of the latest one.
    struct Staging {
        InstDesc *descs;
        int4 *items;
        size_t cap_descs, cap_items;
        hipEvent_t done;
        bool pending;
    };
    static constexpr int kStagingSlots = 4;
    Staging stage[kStagingSlots];
    int next_stage;
    // Outgrown tables and staging buffers, freed with the batch: freeing
    // them at once would wait for the launches queued on the stream.
    std::vector<void *> retired_dev, retired_host;
    int nitems;  // one-step items: members of class 0, then of class 1
    int parity;  // steps taken by the batch, mod 2 (with two-step launches:
                 // the lattice parity of the class-0 members)
    // Two time steps per launch for the members that allow it (class 1,
    // two[k] = 1): their descriptors tiled for the two-step pass follow the
    // n one-step ones, their two-step items follow the one-step items.
    std::vector<char> two;
    int nitems0;  // one-step items of class-0 members (a prefix of the list)
    int nitems2;  // two-step items
    int ndescs2;  // two-step descriptors (class-1 members)
    bool deep2;   // two-step launches load two rows ahead
    int k2;       // time steps per class-1 launch: 2, or 3 (FP32, steps_per_sweep 3)
    int parity2;  // class-1 launches and one-step sweeps of class 1, mod 2
    hipStream_t cap_stream;
    hipGraphExec_t graphs[kMaxGraphLevels];  // level k: 2^(k+1) batched sweeps
                                             // (two-step mode: 2^(k+1) units)
};

namespace {

void release_graph(hipGraphExec_t &g) {
    if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
}

void release_graphs(hipGraphExec_t (&gs)[kMaxGraphLevels]) {
    for (hipGraphExec_t &g : gs) release_graph(g);
}

// Graph level of a power-of-two sweep count >= 2.
int graph_level(int64_t sweeps) {
    int k = 0;
    while (((int64_t)2 << k) < sweeps) ++k;
    return k;
}

// Replay an even number of sweeps through the graph ladder: whole graphs of
// the top level, then one graph per remaining binary digit.  `ensure(k)`
// captures level k if needed.
// With run = false the graphs are only captured (nothing is launched).
template <class Ensure>
trt_status replay_ladder(int64_t nsteps, int64_t graph_steps, hipGraphExec_t (&gs)[kMaxGraphLevels],
                         hipStream_t stream, Ensure ensure, bool run = true) {
    const int top = graph_level(graph_steps);
    const int64_t big = (int64_t)2 << top;
    if (nsteps >= big) {
        trt_status st = ensure(top);
        if (st != TRT_OK) return st;
        if (run)
            for (int64_t k = 0; k < nsteps / big; ++k) TRT_HIP(hipGraphLaunch(gs[top], stream));
        nsteps %= big;
    }
    for (int k = top - 1; k >= 0; --k) {
        if (nsteps & ((int64_t)2 << k)) {
            trt_status st = ensure(k);
            if (st != TRT_OK) return st;
            if (run) TRT_HIP(hipGraphLaunch(gs[k], stream));
        }
    }
    return TRT_OK;
}

// Capture `body` (which enqueues work on the given stream) into an
// executable graph.
template <class F> trt_status capture(hipStream_t cap, hipGraphExec_t &out, F body) {
    hipGraph_t g = nullptr;
    TRT_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = body(cap);
    hipError_t e2 = hipStreamEndCapture(cap, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail_hip(e, "kernel launch during capture");
    }
    if (e2 != hipSuccess) return fail_hip(e2, "hipStreamEndCapture");
    hipError_t e3 = hipGraphInstantiate(&out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) {
        out = nullptr;
        return fail_hip(e3, "hipGraphInstantiate");
    }
    // move the graph's launch resources to the device now rather than at
    // its first replay
    TRT_HIP(hipGraphUpload(out, cap));
    TRT_HIP(hipStreamSynchronize(cap));
    return TRT_OK;
}

// Time steps per launch of a simulation: three, two or one, as asked (0:
// automatic) and as the lattice allows.  Automatic: three for FP32 lattices
// of at least 2048^2 nodes, else two.  Measured (us per step, each pass at
// its default shape, FP32): 8192^2 two steps 453.5, three 345.5; 6144^2
// 284.8 / 211.5; 4096^2 122.3 / 96.2; 3000^2 74.5 / 62.3; 2048^2 35.5 /
// 29.0; below, three steps gain nothing (1536^2 21.0 / 20.9, 1024^2 12.6 /
// 12.8, 512^2 8.6 / 9.2): the extra fill rows and window columns cost more
// than the HBM traffic saved on lattices that largely stay in the
// memory-side cache.
constexpr int64_t kTb3MinNodes = 2048LL * 2048LL;
int sim_k(const trt_sim *s) {
    const int want = s->launch.steps_per_sweep;
    const int st = s->prob.storage;
    if (trt::tb3_eligible(s->desc, st) &&
        (want == 3 || (want == 0 && (int64_t)s->desc.nx * s->desc.ny >= kTb3MinNodes)))
        return 3;
    if (want != 1 && trt::tb2_eligible(s->desc, st)) return 2;
    return 1;
}

// One launch of k time steps (k as sim_k or lower) reading lattice src.
hipError_t sim_launch(const trt_sim *s, int k, int src, hipStream_t stream) {
    const int st = s->prob.storage;
    if (k == 3) return trt::launch_sweep_tb3(s->desc, st, src, s->launch, stream);
    if (k == 2) return trt::launch_sweep_tb2(s->desc, st, src, s->launch, stream);
    return trt::launch_sweep(s->desc, st, s->prob.mask != nullptr, src, s->launch, stream);
}

// Capture `sweeps` (even) launches of a simulation, starting from lattice 0,
// into `out` (each launch sim_k steps).
trt_status sim_capture(trt_sim *s, hipGraphExec_t &out, int64_t sweeps) {
    release_graph(out);
    if (!s->cap_stream) {
        hipError_t e = hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            s->cap_stream = nullptr;
            return fail_hip(e, "hipStreamCreateWithFlags");
        }
    }
    const int ks = sim_k(s);
    return capture(s->cap_stream, out, [&](hipStream_t cs) {
        for (int64_t k = 0; k < sweeps; ++k) {
            hipError_t e = sim_launch(s, ks, (int)(k & 1), cs);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    });
}

trt_status check_sim(const trt_sim *s) {
    if (!s) return fail(TRT_EINVAL, "simulation handle is NULL");
    return TRT_OK;
}

}  // namespace

extern "C" {

int32_t trt_pitch(int32_t nx, int32_t storage) {
    const int es = elem_size(storage);
    if (es == 0 || nx < 1 || nx > kMaxSide) return -1;
    const int per = 256 / es;
    return (nx + per - 1) / per * per;
}

int64_t trt_row_stride(int32_t nx, int32_t storage) {
    const int32_t p = trt_pitch(nx, storage);
    if (p < 0) return -1;
    return (int64_t)9 * p;
}

size_t trt_lattice_bytes(const trt_problem *p) {
    if (check_problem(p) != TRT_OK) return 0;
    return (size_t)p->ny * (size_t)trt_row_stride(p->nx, p->storage) *
           (size_t)elem_size(p->storage);
}

namespace {
// elements of a link-map row: nx rounded up to 256 bytes
int64_t link_pitch(int32_t nx) { return ((int64_t)nx + 127) / 128 * 128; }
// entries of a link-summary row: two per 128-column strip
int32_t summary_count(int32_t nx) { return 2 * ((nx + 127) / 128); }
bool needs_links(const trt_problem *p) {
    return p->mask != nullptr || p->x_boundary == TRT_X_INFLOW_OUTFLOW;
}
// one allocation: the link map, then (256-byte aligned) the link summary
size_t link_map_bytes(int32_t nx) { return 2 * (size_t)link_pitch(nx); }  // per row
size_t summary_offset(int32_t nx, int32_t ny) {
    return (link_map_bytes(nx) * (size_t)ny + 255) / 256 * 256;
}
size_t link_alloc_bytes(int32_t nx, int32_t ny) {
    return summary_offset(nx, ny) + 4 * (size_t)summary_count(nx) * (size_t)ny;
}
}  // namespace

namespace {
// The library's own stream on the current device (non-blocking, default
// priority, kept until the process ends): the mask check of trt_create runs
// and waits there, so creating a simulation does not wait for the work
// queued on the caller's stream.
hipError_t own_stream(hipStream_t &out) {
    static std::mutex mu;
    static hipStream_t streams[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(mu);
    if (!streams[dev]) {
        e = hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking);
        if (e != hipSuccess) {
            streams[dev] = nullptr;
            return e;
        }
    }
    out = streams[dev];
    return hipSuccess;
}

// rows = 1 when every row of the problem's mask is all solid or all fluid
// (walls parallel to x): the mask is read on the library's own stream, with
// `scratch` (at least one int) for the device flag.
hipError_t mask_in_rows(const trt_problem *p, void *scratch, int32_t &rows) {
    rows = 0;
    hipStream_t st = nullptr;
    hipError_t e = own_stream(st);
    if (e != hipSuccess) return e;
    int *flag = static_cast<int *>(scratch);
    int mixed = 1;
    e = trt::launch_mask_rows(p->mask, p->nx, p->ny, flag, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&mixed, flag, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess && mixed == 0) rows = 1;
    return e;
}

// The descriptor of a problem over the lattices f_a, f_b (no link map yet;
// tiled for the default launch shape by the caller).
void fill_desc(InstDesc &d, const trt_problem *p, void *f_a, void *f_b) {
    d.buf[0] = f_a;
    d.buf[1] = f_b;
    d.mask = p->mask;
    d.nx = p->nx;
    d.ny = p->ny;
    d.plane = trt_pitch(p->nx, p->storage);
    d.pitch = (int32_t)trt_row_stride(p->nx, p->storage);
    d.cur = 0;
    d.cols = 1;
    d.omega1 = 1.0 - 1.0 / p->tau_s;
    d.omega2 = 1.0 - 1.0 / p->tau_s2;
    d.phi = 1.0 - 1.0 / (2.0 * p->tau_s);
    d.gx = p->gx;
    d.gy = p->gy;
    d.xbc = p->x_boundary == TRT_X_INFLOW_OUTFLOW ? 1 : 0;
    d.pad2_ = 0;
    d.u_in = d.xbc ? p->u_in : 0.0;
    d.rho_in = d.xbc ? p->rho_in : 1.0;
    d.rho_out = d.xbc ? p->rho_out : 1.0;
    d.links = nullptr;
    d.lpitch = link_pitch(p->nx);
    d.rowsum = nullptr;
    d.nsum = summary_count(p->nx);
    d.rowwalls = 0;
}
}  // namespace

size_t trt_footprint_bytes(const trt_problem *p) {
    const size_t lat = trt_lattice_bytes(p);
    if (lat == 0) return 0;
    const size_t mask = p->mask ? (size_t)p->nx * p->ny : 0;
    const size_t links = needs_links(p) ? link_alloc_bytes(p->nx, p->ny) : 0;
    const size_t scratch = (size_t)(trt::diag_partial_count() + 1) * TRT_NDIAG * sizeof(double);
    return 2 * lat + mask + links + scratch;
}

trt_status trt_create(const trt_problem *p, void *f_a, void *f_b, void *hip_stream,
                      trt_sim **out) {
    if (!out) return fail(TRT_EINVAL, "out is NULL");
    *out = nullptr;
    trt_status st = check_problem(p);
    if (st != TRT_OK) return st;
    if (!f_a || !f_b) return fail(TRT_EINVAL, "both lattices f_a and f_b are required");
    if (!aligned(f_a, 256) || !aligned(f_b, 256))
        return fail(TRT_EINVAL, "lattices must be 256-byte aligned");
    const size_t bytes = trt_lattice_bytes(p);
    const char *a = (const char *)f_a, *b = (const char *)f_b;
    if (a < b + bytes && b < a + bytes) return fail(TRT_EINVAL, "lattices overlap");

    trt_sim *s = new (std::nothrow) trt_sim();
    if (!s) return fail(TRT_ENOMEM, "out of host memory");
    s->prob = *p;
    s->stream = (hipStream_t)hip_stream;
    s->launch = kDefaultLaunch;
    s->cur = 0;
    s->time = 0;
    InstDesc &d = s->desc;
    fill_desc(d, p, f_a, f_b);

    hipError_t e = hipMalloc((void **)&s->scratch, (size_t)(trt::diag_partial_count() + 1) *
                                                      TRT_NDIAG * sizeof(double));
    if (e != hipSuccess) {
        delete s;
        return fail_hip(e, "hipMalloc(scratch)");
    }
    if (needs_links(p)) {
        e = hipMalloc((void **)&s->links, link_alloc_bytes(p->nx, p->ny));
        if (e == hipSuccess) {
            d.links = s->links;
            d.rowsum = reinterpret_cast<const uint32_t *>(
                reinterpret_cast<const char *>(s->links) + summary_offset(p->nx, p->ny));
            e = trt::launch_link_map(d, s->stream);
        }
        if (e != hipSuccess) {
            if (s->links) (void)hipFree(s->links);
            (void)hipFree(s->scratch);
            delete s;
            return fail_hip(e, "link map");
        }
    }
    if (p->mask != nullptr && d.xbc == 0) {
        e = mask_in_rows(p, s->scratch, d.rowwalls);
        if (e != hipSuccess) {
            (void)hipFree(s->links);
            (void)hipFree(s->scratch);
            delete s;
            return fail_hip(e, "mask check");
        }
    }
    trt::tile(d, s->launch, p->storage);
    // the capture stream is created at the first capture (batch members never
    // capture their own step)
    *out = s;
    return TRT_OK;
}

trt_status trt_set_tuning(trt_sim *s, const trt_tuning *t) {
    Launch l;
    trt_status st = check_launch(t, l, kDefaultLaunch);
    if (st != TRT_OK) return st;
    if (check_sim(s) != TRT_OK) return TRT_EINVAL;
    if (s->in_batch) return fail(TRT_ESTATE, "simulation is a batch member");
    s->launch = l;
    trt::tile(s->desc, l, s->prob.storage);
    release_graphs(s->graphs);
    return TRT_OK;
}

trt_status trt_get_tuning(const trt_sim *s, trt_tuning *t) {
    if (check_sim(s) != TRT_OK) return TRT_EINVAL;
    if (!t) return fail(TRT_EINVAL, "out is NULL");
    const int ks = sim_k(s);
    t->rows_per_wave = ks == 3   ? trt::tb3_desc(s->desc, s->launch).rows
                       : ks == 2 ? trt::tb2_desc(s->desc, s->launch).rows
                                 : s->desc.rows;
    t->waves_per_block =
        ks == 3   ? trt::tb3_waves_per_block(s->desc, s->launch)
        : ks == 2 ? trt::tb2_waves_per_block(s->desc, s->prob.storage, s->launch)
                  : trt::single_waves_per_block(s->desc, s->prob.storage, s->launch);
    t->xcd_remap = ks == 3 ? trt::tb3_xcd_remap(s->desc, s->launch) : s->launch.xcd_remap;
    t->cols_per_lane = s->desc.cols;
    t->batch_items = 0;
    t->batch_order = 0;
    t->graph_steps = s->launch.graph_steps;
    t->steps_per_sweep = ks;
    t->prefetch_rows = ks == 3   ? trt::tb3_prefetch_rows(s->desc, s->launch)
                       : ks == 2 ? trt::tb2_prefetch_rows(s->desc, s->prob.storage, s->launch)
                                 : 0;
    return TRT_OK;
}

trt_status trt_init_equilibrium(trt_sim *s, const double *rho, const double *ux,
                                const double *uy) {
    if (check_sim(s) != TRT_OK) return TRT_EINVAL;
    if (!rho || !ux || !uy) return fail(TRT_EINVAL, "rho, ux and uy are required");
    if (s->in_batch) return fail(TRT_ESTATE, "simulation is a batch member");
    TRT_HIP(trt::launch_init_equilibrium(s->desc, s->prob.storage, s->cur, rho, ux, uy, s->stream));
    s->time = 0;
    return TRT_OK;
}

trt_status trt_set_populations(trt_sim *s, const double *f) {
    if (check_sim(s) != TRT_OK) return TRT_EINVAL;
    if (!f) return fail(TRT_EINVAL, "f is NULL");
    if (s->in_batch) return fail(TRT_ESTATE, "simulation is a batch member");
    TRT_HIP(trt::launch_set_populations(s->desc, s->prob.storage, s->cur, f, s->stream));
    s->time = 0;
    return TRT_OK;
}

trt_status trt_get_populations(trt_sim *s, double *f) {
    if (check_sim(s) != TRT_OK) return TRT_EINVAL;
    if (!f) return fail(TRT_EINVAL, "f is NULL");
    TRT_HIP(trt::launch_get_populations(s->desc, s->prob.storage, s->cur, f, s->stream));
    return TRT_OK;
}

trt_status trt_step(trt_sim *s, int64_t nsteps) {
    if (check_sim(s) != TRT_OK) return TRT_EINVAL;
    if (nsteps < 0) return fail(TRT_EINVAL, "nsteps must be >= 0");
    if (s->in_batch) return fail(TRT_ESTATE, "simulation is a batch member");
    if (nsteps == 0) return TRT_OK;
    const int st = s->prob.storage;
    const bool m = s->prob.mask != nullptr;
    if (s->cur == 1) {
        TRT_HIP(trt::launch_sweep(s->desc, st, m, 1, s->launch, s->stream));
        s->cur = 0;
        ++s->time;
        --nsteps;
    }
    // every graph holds an even number of launches, so each replay starts and
    // ends on lattice 0
    const int ks = sim_k(s);
    if (ks > 1) {
        // ks steps per launch: graphs of 2, 4, ... launches (2 ks, 4 ks, ...
        // steps), then at most one ks-step launch, and the rest (fewer than
        // ks steps) as one two-step launch and one-step sweeps
        if (nsteps >= 2 * ks) {
            const int64_t launches = nsteps / (2 * ks) * 2;
            trt_status rs = replay_ladder(
                launches, std::max<int64_t>(2, s->launch.graph_steps / 2), s->graphs, s->stream,
                [&](int k) -> trt_status {
                    if (s->graphs[k]) return TRT_OK;
                    return sim_capture(s, s->graphs[k], (int64_t)2 << k);
                });
            if (rs != TRT_OK) return rs;
            s->time += ks * launches;
            nsteps -= ks * launches;
        }
        // fewer than 2 ks steps are left: ks, then 2 (when ks is 3), then 1
        for (int k : {ks, 2, 1}) {
            if (k > ks || nsteps < k) continue;
            TRT_HIP(sim_launch(s, k, s->cur, s->stream));
            s->cur ^= 1;
            s->time += k;
            nsteps -= k;
        }
        return TRT_OK;
    }
    if (nsteps >= 2) {
        const int64_t even = nsteps / 2 * 2;
        trt_status rs = replay_ladder(even, s->launch.graph_steps, s->graphs, s->stream,
                                      [&](int k) -> trt_status {
                                          if (s->graphs[k]) return TRT_OK;
                                          return sim_capture(s, s->graphs[k], (int64_t)2 << k);
                                      });
        if (rs != TRT_OK) return rs;
        s->time += even;
    }
    if (nsteps % 2) {
        TRT_HIP(trt::launch_sweep(s->desc, st, m, 0, s->launch, s->stream));
        s->cur = 1;
        ++s->time;
    }
    return TRT_OK;
}

trt_status trt_prepare_steps(trt_sim *s, int64_t nsteps) {
    if (check_sim(s) != TRT_OK) return TRT_EINVAL;
    if (nsteps < 0) return fail(TRT_EINVAL, "nsteps must be >= 0");
    if (s->in_batch) return fail(TRT_ESTATE, "simulation is a batch member");
    // the launches trt_step would replay as graphs (see there)
    int64_t n = nsteps;
    if (s->cur == 1 && n > 0) --n;
    const int ks = sim_k(s);
    const int64_t launches = ks > 1 ? n / (2 * ks) * 2 : n / 2 * 2;
    if (launches == 0) return TRT_OK;
    const int64_t longest =
        ks > 1 ? std::max<int64_t>(2, s->launch.graph_steps / 2) : s->launch.graph_steps;
    return replay_ladder(
        launches, longest, s->graphs, s->stream,
        [&](int k) -> trt_status {
            if (s->graphs[k]) return TRT_OK;
            return sim_capture(s, s->graphs[k], (int64_t)2 << k);
        },
        false);
}

trt_status trt_pattern_probe(trt_sim *s, int64_t nsweeps) {
    if (check_sim(s) != TRT_OK) return TRT_EINVAL;
    if (nsweeps < 0) return fail(TRT_EINVAL, "nsweeps must be >= 0");
    if (s->in_batch) return fail(TRT_ESTATE, "simulation is a batch member");
    const InstDesc &d = s->desc;
    if (d.cols != 2 || d.nx % 128 != 0 || d.links != nullptr ||
        !trt::buffer_addressable(d, s->prob.storage))
        return fail(TRT_EINVAL, "the pattern probe needs an open periodic lattice of at most "
                                "4 GiB, nx a multiple of 128, swept with two columns per lane");
    for (int64_t k = 0; k < nsweeps; ++k) {
        TRT_HIP(trt::launch_pattern_probe(d, s->prob.storage, s->cur, s->launch, s->stream));
        s->cur ^= 1;
    }
    return TRT_OK;
}

trt_status trt_macros(trt_sim *s, double *rho, double *ux, double *uy) {
    if (check_sim(s) != TRT_OK) return TRT_EINVAL;
    if (!rho && !ux && !uy) return TRT_OK;
    TRT_HIP(trt::launch_macros(s->desc, s->prob.storage, s->cur, rho, ux, uy, s->stream));
    return TRT_OK;
}

trt_status trt_diagnostics(trt_sim *s, double *out) {
    if (check_sim(s) != TRT_OK) return TRT_EINVAL;
    if (!out) return fail(TRT_EINVAL, "out is NULL");
    TRT_HIP(trt::launch_diagnostics(s->desc, s->prob.storage, s->cur, s->scratch, out,
                                    (double)s->time, s->stream));
    return TRT_OK;
}

}  // extern "C"

// ------------------------------------------- diagnostics without allocation
//
// trt_diagnostics_noalloc keeps its reduction partials in one file-scope
// device array.  Host code never passes the array's name to a kernel (on the
// host it names a stand-in, not device memory): the first call on a device
// resolves the array's address there with hipGetSymbolAddress, and every
// later call on that device uses the resolved pointer.
namespace {
constexpr size_t kNoAllocDoubles = 512 * TRT_NDIAG;  // 32 KiB per GPU
__device__ __align__(256) double noalloc_scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
double *g_noalloc_ptr[kMaxDevices];  // device address of noalloc_scratch, per device

// The array's address on device `dev` (made current for the lookup).
trt_status noalloc_scratch_on(int dev, double **ptr) {
    if (dev < 0 || dev >= kMaxDevices) return fail(TRT_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        int prev = -1;
        TRT_HIP(hipGetDevice(&prev));
        if (prev != dev) TRT_HIP(hipSetDevice(dev));
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
        if (prev != dev) {
            hipError_t e2 = hipSetDevice(prev);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(noalloc_scratch)");
        if (!p) return fail(TRT_EDEVICE, "hipGetSymbolAddress returned NULL");
        g_noalloc_ptr[dev] = static_cast<double *>(p);
    }
    *ptr = g_noalloc_ptr[dev];
    return TRT_OK;
}
}  // namespace

extern "C" {

trt_status trt_diagnostics_noalloc(const trt_problem *p, const void *lattice, int64_t time,
                                   double *out, void *hip_stream) {
    trt_status st = check_problem(p);
    if (st != TRT_OK) return st;
    if (!lattice || !out) return fail(TRT_EINVAL, "lattice and out are required");
    if (!aligned(lattice, 256)) return fail(TRT_EINVAL, "the lattice must be 256-byte aligned");
    if (time < 0) return fail(TRT_EINVAL, "time must be >= 0");
    const size_t need = (size_t)trt::diag_partial_count() * TRT_NDIAG;
    if (need > kNoAllocDoubles)
        return fail(TRT_EINVAL, "diagnostics need more partials than the static scratch holds");
    const hipStream_t stream = (hipStream_t)hip_stream;
    int dev = -1;
    if (stream) {
        hipDevice_t sd;
        TRT_HIP(hipStreamGetDevice(stream, &sd));
        dev = (int)sd;
    } else {
        TRT_HIP(hipGetDevice(&dev));
    }
    double *partials = nullptr;
    st = noalloc_scratch_on(dev, &partials);
    if (st != TRT_OK) return st;
    InstDesc d;
    fill_desc(d, p, const_cast<void *>(lattice), const_cast<void *>(lattice));
    // every partial is written before it is read: nothing needs clearing
    TRT_HIP(trt::launch_diagnostics(d, p->storage, 0, partials, out, (double)time, stream));
    return TRT_OK;
}

trt_status trt_wall_force(trt_sim *s, double *out) {
    if (check_sim(s) != TRT_OK) return TRT_EINVAL;
    if (!out) return fail(TRT_EINVAL, "out is NULL");
    if (s->time == 0) return fail(TRT_ESTATE, "no step taken since the state was set");
    TRT_HIP(trt::launch_wall_force(s->desc, s->prob.storage, s->cur, s->scratch, out, s->stream));
    return TRT_OK;
}

trt_status trt_velocity_change(trt_sim *s, double *prev_ux, double *prev_uy, double *out) {
    if (check_sim(s) != TRT_OK) return TRT_EINVAL;
    if (!prev_ux || !prev_uy || !out) return fail(TRT_EINVAL, "prev_ux, prev_uy and out are required");
    TRT_HIP(trt::launch_velocity_compare(s->desc, s->prob.storage, s->cur, prev_ux, prev_uy, true,
                                         s->scratch, out, s->stream));
    return TRT_OK;
}

trt_status trt_velocity_error(trt_sim *s, const double *ref_ux, const double *ref_uy,
                              double *out) {
    if (check_sim(s) != TRT_OK) return TRT_EINVAL;
    if (!ref_ux || !ref_uy || !out) return fail(TRT_EINVAL, "ref_ux, ref_uy and out are required");
    TRT_HIP(trt::launch_velocity_compare(s->desc, s->prob.storage, s->cur,
                                         const_cast<double *>(ref_ux),
                                         const_cast<double *>(ref_uy), false, s->scratch, out,
                                         s->stream));
    return TRT_OK;
}

trt_status trt_row_mean_ux(trt_sim *s, double *out) {
    if (check_sim(s) != TRT_OK) return TRT_EINVAL;
    if (!out) return fail(TRT_EINVAL, "out is NULL");
    TRT_HIP(trt::launch_row_mean_ux(s->desc, s->prob.storage, s->cur, out, s->stream));
    return TRT_OK;
}

trt_status trt_check(trt_sim *s) {
    if (check_sim(s) != TRT_OK) return TRT_EINVAL;
    double *res = s->scratch + (size_t)trt::diag_partial_count() * TRT_NDIAG;
    trt_status st = trt_diagnostics(s, res);
    if (st != TRT_OK) return st;
    double h[TRT_NDIAG];
    TRT_HIP(hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, s->stream));
    TRT_HIP(hipStreamSynchronize(s->stream));
    if (h[4] > 0.0) {
        char buf[128];
        snprintf(buf, sizeof buf, "%.0f of %.0f fluid nodes diverged at step %lld", h[4], h[5],
                 (long long)s->time);
        return fail(TRT_EUNSTABLE, buf);
    }
    return TRT_OK;
}

trt_status trt_state(const trt_sim *s, int32_t *current, int64_t *time) {
    if (check_sim(s) != TRT_OK) return TRT_EINVAL;
    if (current) *current = s->cur;
    if (time) *time = s->time;
    return TRT_OK;
}

void trt_destroy(trt_sim *s) {
    if (!s) return;
    release_graphs(s->graphs);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    if (s->scratch) (void)hipFree(s->scratch);
    if (s->links) (void)hipFree(s->links);
    delete s;
}

// ---------------------------------------------------------------- batches

// Grow a device or pinned host buffer to at least `need` elements (contents
// are not kept).
extern "C++" {
// Table capacity for `need` entries: at least 4096, growing fourfold, so a
// batch whose membership keeps changing reallocates rarely.
static size_t table_capacity(size_t cap, size_t need) {
    size_t c = cap ? cap : 4096;
    while (c < need) c *= 4;
    return c;
}
template <class E>
static hipError_t grow_device(E *&p, size_t &cap, size_t need, std::vector<void *> &retired) {
    if (need <= cap && p) return hipSuccess;
    const size_t c = table_capacity(cap, need);
    if (p) retired.push_back(p);
    p = nullptr;
    cap = 0;
    hipError_t e = hipMalloc((void **)&p, c * sizeof(E));
    if (e == hipSuccess) cap = c;
    return e;
}
template <class E>
static hipError_t grow_pinned(E *&p, size_t &cap, size_t need, std::vector<void *> &retired) {
    if (need <= cap && p) return hipSuccess;
    const size_t c = table_capacity(cap, need);
    if (p) retired.push_back(p);
    p = nullptr;
    cap = 0;
    hipError_t e = hipHostMalloc((void **)&p, c * sizeof(E), hipHostMallocDefault);
    if (e == hipSuccess) cap = c;
    return e;
}
}  // extern "C++"

// (Re)build the work list and descriptor tables of the current members.  The
// tables are copied from pinned staging buffers on the batch's stream, so no
// device-wide wait is needed: launches already enqueued read the old tables
// first (stream order).  Only a staging slot waits, for the copy that last
// read it (several rebuilds ago).
// Rows per wavefront of every member under the batch's launch shape (see
// trt_tuning.batch_items) and the work list in the batch's order.  The
// tiling changes no result: every node's arithmetic is the same whatever
// rows or order a sweep uses.
static void batch_tile(trt_batch *b, std::vector<InstDesc> &descs, std::vector<int4> &items) {
    const size_t n = b->sims.size();
    descs.resize(n);
    for (size_t k = 0; k < n; ++k) {
        InstDesc &d = descs[k];
        d = b->sims[k]->desc;
        d.cur = b->sims[k]->cur;
        trt::tile(d, b->launch, b->sims[k]->prob.storage);
    }
    if (b->launch.rows_per_wave <= 0 && b->launch.batch_items > 0) {
        // the longest power-of-two cap that leaves at least batch_items items
        auto count = [&](int cap) {
            size_t c = 0;
            for (size_t k = 0; k < n; ++k)
                c += (size_t)descs[k].strips * (size_t)((descs[k].ny + cap - 1) / cap);
            return c;
        };
        int cap = 256;
        while (cap > 4 && count(cap) < (size_t)b->launch.batch_items) cap /= 2;
        for (size_t k = 0; k < n; ++k) {
            InstDesc &d = descs[k];
            const int blocks = (d.ny + cap - 1) / cap;
            d.rows = (d.ny + blocks - 1) / blocks;  // equal blocks of at most cap rows
            d.rowblocks = (d.ny + d.rows - 1) / d.rows;
        }
    }
    // class 1: members that take multi-step launches: three steps per launch
    // in FP32 (unless two are asked for), two in FP16.  The 256-member
    // benchmark batch (sides 64 to 1024), FP32: 155.4 GLUPS with three steps
    // per launch against 118.0 with two -- its members are small, but
    // together they far exceed the memory-side cache.
    const int sps = b->launch.steps_per_sweep;
    b->k2 = ((sps == 0 || sps == 3) && b->storage == trt::ST_F32) ? 3 : 2;
    b->two.assign(n, 0);
    if (b->launch.steps_per_sweep != 1)
        for (size_t k = 0; k < n; ++k)
            b->two[k] = (b->k2 == 3 ? trt::tb3_eligible(descs[k], b->sims[k]->prob.storage)
                                    : trt::tb2_eligible(descs[k], b->sims[k]->prob.storage))
                            ? 1
                            : 0;
    const int valid2 = b->k2 == 3 ? trt::kTb3Valid : trt::kTb2Valid;
    const auto cost = [&](const int4 &it) {
        // two-step items (it.w == 2) index the two-step descriptors, which
        // follow the n one-step ones
        const InstDesc &d = descs[it.w == 2 ? n + (size_t)it.x : (size_t)it.x];
        const int rows = std::min(d.rows, d.ny - it.z * d.rows);
        return (int64_t)rows * (it.w == 2 ? valid2 : trt::kStripWidth * d.cols);
    };
    const auto order = [&](size_t from) {
        // costliest first: rows in the block x columns per strip (stable, so
        // equal items keep member, row block and strip order)
        if (b->launch.batch_order == 2)
            std::stable_sort(items.begin() + (std::ptrdiff_t)from, items.end(),
                             [&](const int4 &a, const int4 &c) { return cost(a) > cost(c); });
    };
    items.clear();
    for (int cls = 0; cls < 2; ++cls) {
        const size_t from = items.size();
        for (size_t k = 0; k < n; ++k)
            if (b->two[k] == cls)
                for (int r = 0; r < descs[k].rowblocks; ++r)
                    for (int c = 0; c < descs[k].strips; ++c)
                        items.push_back(make_int4((int)k, c, r, cls));
        order(from);
        if (cls == 0) b->nitems0 = (int)items.size();
    }
    b->nitems = (int)items.size();
    // the multi-step tables: descriptors tiled for the pass (rows shared by
    // the batch unless set -- a batch of small members needs many short
    // items to balance.  Two steps: the longest of 32, 24, 16, 12, 8 rows
    // that gives 32768 items (256 members of 64^2 ... 1024^2, 4-wavefront
    // workgroups: FP32 (loads two rows ahead) 112.5 / 116.5 / 118.1 GLUPS at
    // 24 / 16 / 12 rows, FP16 (one row ahead) 163.5 / 169.9 / 173.3).  Three
    // steps (ten rows of fill per block): the longest of 32, 24, 20, 16, 12,
    // 8 that gives 24576 items (FP32 152.7 / 154.5 / 155.4 / 153.8 / 147.2
    // GLUPS at 32 / 24 / 20 / 16 / 12 rows).  Else 8.), then their items
    std::vector<size_t> mem;
    for (size_t k = 0; k < n; ++k)
        if (b->two[k]) mem.push_back(k);
    b->nitems2 = 0;
    b->ndescs2 = (int)mem.size();
    b->deep2 = false;
    if (mem.empty()) return;
    Launch l2 = b->launch;
    if (l2.rows_per_wave <= 0) {
        static const int kRows2[] = {32, 24, 16, 12, 8};
        static const int kRows3[] = {32, 24, 20, 16, 12, 8};
        const int *rows = b->k2 == 3 ? kRows3 : kRows2;
        const int nrows = b->k2 == 3 ? 6 : 5;
        const long long target = b->k2 == 3 ? 24576 : 32768;
        l2.rows_per_wave = 8;
        for (int i = 0; i < nrows; ++i) {
            const int r = rows[i];
            long long c = 0;
            for (size_t k : mem)
                c += (long long)((descs[k].nx + valid2 - 1) / valid2) *
                     ((descs[k].ny + r - 1) / r);
            if (c >= target) {
                l2.rows_per_wave = r;
                break;
            }
        }
    }
    const size_t from = items.size();
    for (size_t j = 0; j < mem.size(); ++j) {
        InstDesc d2 = b->k2 == 3 ? trt::tb3_desc(descs[mem[j]], l2)
                                 : trt::tb2_desc(descs[mem[j]], l2);
        descs.push_back(d2);
        // the two-step kernel's descriptor table starts after the n
        // one-step ones: its items name j (entry n + j of the whole table)
        for (int r = 0; r < d2.rowblocks; ++r)
            for (int c = 0; c < d2.strips; ++c)
                items.push_back(make_int4((int)j, c, r, 2));
    }
    order(from);
    b->nitems2 = (int)(items.size() - from);
    b->deep2 = b->k2 == 2 &&
               trt::tb2_batch_prefetch_rows(b->nitems2, b->storage, b->launch) == 2;
}

static trt_status batch_build(trt_batch *b) {
    std::vector<InstDesc> descs;
    std::vector<int4> list;
    batch_tile(b, descs, list);
    const size_t n = descs.size();
    const size_t nitems = list.size();
    if (nitems > (size_t)INT32_MAX) return fail(TRT_EINVAL, "batch work list too long");
    trt_batch::Staging &sg = b->stage[b->next_stage];
    b->next_stage = (b->next_stage + 1) % trt_batch::kStagingSlots;
    if (sg.pending) {
        TRT_HIP(hipEventSynchronize(sg.done));
        sg.pending = false;
    }
    TRT_HIP(grow_pinned(sg.descs, sg.cap_descs, n, b->retired_host));
    TRT_HIP(grow_pinned(sg.items, sg.cap_items, nitems, b->retired_host));
    TRT_HIP(grow_device(b->d_descs, b->cap_descs, n, b->retired_dev));
    TRT_HIP(grow_device(b->d_items, b->cap_items, nitems, b->retired_dev));
    for (size_t k = 0; k < n; ++k) sg.descs[k] = descs[k];
    for (size_t j = 0; j < nitems; ++j) sg.items[j] = list[j];
    TRT_HIP(hipMemcpyAsync(b->d_descs, sg.descs, n * sizeof(InstDesc), hipMemcpyHostToDevice,
                           b->stream));
    TRT_HIP(hipMemcpyAsync(b->d_items, sg.items, nitems * sizeof(int4), hipMemcpyHostToDevice,
                           b->stream));
    TRT_HIP(hipEventRecord(sg.done, b->stream));
    sg.pending = true;
    b->parity = 0;
    b->parity2 = 0;
    release_graphs(b->graphs);
    return TRT_OK;
}

// Membership checks shared by create and update: n >= 1 distinct members of
// one storage type and stream, none in another batch.
static trt_status check_members(int32_t n, trt_sim *const *sims, const trt_batch *self) {
    if (n < 1 || !sims) return fail(TRT_EINVAL, "a batch needs n >= 1 simulations");
    for (int k = 0; k < n; ++k) {
        if (!sims[k]) return fail(TRT_EINVAL, "NULL batch member");
        bool mine = false;
        if (self)
            for (trt_sim *m : self->sims) mine = mine || m == sims[k];
        if (sims[k]->in_batch && !mine) return fail(TRT_ESTATE, "simulation already in a batch");
        if (sims[k]->prob.storage != sims[0]->prob.storage)
            return fail(TRT_EINVAL, "batch members must share one storage type");
        if (sims[k]->stream != sims[0]->stream)
            return fail(TRT_EINVAL, "batch members must share one stream");
        if (self && sims[k]->stream != self->stream)
            return fail(TRT_EINVAL, "batch members must use the batch's stream");
        for (int j = 0; j < k; ++j)
            if (sims[j] == sims[k]) return fail(TRT_EINVAL, "duplicate batch member");
    }
    return TRT_OK;
}

static void batch_set_members(trt_batch *b, int32_t n, trt_sim *const *sims) {
    std::vector<trt_sim *> next(sims, sims + n);  // may throw: nothing changed yet
    for (trt_sim *m : b->sims) m->in_batch = false;
    b->sims.swap(next);
    b->storage = sims[0]->prob.storage;
    b->mask = false;
    b->buf = true;
    for (int k = 0; k < n; ++k) {
        b->mask = b->mask || sims[k]->prob.mask != nullptr || sims[k]->prob.x_boundary != 0;
        b->buf = b->buf && trt::buffer_addressable(sims[k]->desc, sims[k]->prob.storage);
        sims[k]->in_batch = true;
    }
}

trt_status trt_batch_create(int32_t n, trt_sim *const *sims, trt_batch **out) {
    if (!out) return fail(TRT_EINVAL, "out is NULL");
    *out = nullptr;
    trt_status st = check_members(n, sims, nullptr);
    if (st != TRT_OK) return st;
    trt_batch *b = new (std::nothrow) trt_batch();
    if (!b) return fail(TRT_ENOMEM, "out of host memory");
    st = guarded([&]() -> trt_status {
        b->stream = sims[0]->stream;
        b->launch = kBatchDefaultLaunch;
        hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
        for (auto &sg : b->stage)
            if (e == hipSuccess) e = hipEventCreateWithFlags(&sg.done, hipEventDisableTiming);
        if (e != hipSuccess) return fail_hip(e, "batch stream/event");
        batch_set_members(b, n, sims);
        return batch_build(b);
    });
    if (st != TRT_OK) {
        trt_batch_destroy(b);
        return st;
    }
    *out = b;
    return TRT_OK;
}

trt_status trt_batch_update(trt_batch *b, int32_t n, trt_sim *const *sims) {
    return guarded([&]() -> trt_status {
        if (!b) return fail(TRT_EINVAL, "batch handle is NULL");
        trt_status st = check_members(n, sims, b);
        if (st != TRT_OK) return st;
        batch_set_members(b, n, sims);
        return batch_build(b);
    });
}

trt_status trt_batch_set_tuning(trt_batch *b, const trt_tuning *t) {
    Launch l;
    trt_status st = check_launch(t, l, kBatchDefaultLaunch);
    if (st != TRT_OK) return st;
    if (!b) return fail(TRT_EINVAL, "batch handle is NULL");
    // members' cur already reflects every step taken; rebuilding restarts
    // the batch parity from there
    b->launch = l;
    return guarded([&] { return batch_build(b); });
}

// Host state of the members after `steps` time steps in which class-0
// members' lattices flipped `flips0` times and class-1 members' `flips1`.
trt_status trt_batch_get_tuning(const trt_batch *b, trt_tuning *t) {
    if (!b) return fail(TRT_EINVAL, "batch handle is NULL");
    if (!t) return fail(TRT_EINVAL, "out is NULL");
    t->rows_per_wave = b->launch.rows_per_wave;
    t->waves_per_block = trt::batch_waves_per_block(b->launch);
    t->xcd_remap = b->launch.xcd_remap;
    t->cols_per_lane = b->launch.cols_per_lane;
    t->batch_items = b->launch.batch_items;
    t->batch_order = b->launch.batch_order;
    t->graph_steps = b->launch.graph_steps;
    t->steps_per_sweep = b->nitems2 > 0 ? b->k2 : 1;
    t->prefetch_rows = b->nitems2 > 0 ? (b->deep2 ? 2 : 1) : 0;
    return TRT_OK;
}

static void batch_sync_members(trt_batch *b, int64_t steps, int64_t flips0, int64_t flips1) {
    for (size_t k = 0; k < b->sims.size(); ++k) {
        trt_sim *s = b->sims[k];
        s->time += steps;
        if (((b->two.empty() || !b->two[k]) ? flips0 : flips1) & 1) s->cur ^= 1;
    }
}

// Launches of the two-step mode.  single: one step of every member (class 0
// at parity f0, class 1 at f1).  unit: two steps -- one two-step launch of
// the class-1 members (parity f1) and two one-step sweeps of the class-0
// members (parity f0, then f0 ^ 1).
static hipError_t batch_single(const trt_batch *b, int f0, int f1, hipStream_t s) {
    return trt::launch_sweep_batch(b->d_descs, b->d_items, b->nitems, b->storage, b->mask, b->buf,
                                   f0, f1, b->launch, s);
}
// One unit of k2 steps: one k2-step launch of class 1 and k2 one-step
// sweeps of class 0 (parities f0 and f1 at its start).
static hipError_t batch_unit(const trt_batch *b, int f0, int f1, hipStream_t s) {
    const size_t n = b->sims.size();
    hipError_t e =
        b->k2 == 3
            ? trt::launch_sweep_tb3_batch(b->d_descs + n, b->ndescs2, b->d_items + b->nitems,
                                          b->nitems2, b->storage, f1, b->launch, s)
            : trt::launch_sweep_tb2_batch(b->d_descs + n, b->ndescs2, b->d_items + b->nitems,
                                          b->nitems2, b->storage, f1, b->deep2, b->launch, s);
    for (int h = 0; h < b->k2 && e == hipSuccess && b->nitems0 > 0; ++h)
        e = trt::launch_sweep_batch(b->d_descs, b->d_items, b->nitems0, b->storage, b->mask,
                                    b->buf, f0 ^ (h & 1), f0 ^ (h & 1), b->launch, s);
    return e;
}

// Capture `sweeps` (even) batched sweeps, starting from parity 0, into `out`;
// in multi-step mode `sweeps` units (2 k2 steps per pair) from parities 0, 0
// (unit u starts class 0 on parity u k2 mod 2).
static trt_status batch_capture(trt_batch *b, hipGraphExec_t &out, int64_t sweeps) {
    release_graph(out);
    return capture(b->cap_stream, out, [&](hipStream_t cs) {
        for (int64_t k = 0; k < sweeps; ++k) {
            hipError_t e = b->nitems2 > 0
                               ? batch_unit(b, (int)((k * b->k2) & 1), (int)(k & 1), cs)
                               : trt::launch_sweep_batch(b->d_descs, b->d_items, b->nitems,
                                                         b->storage, b->mask, b->buf, (int)(k & 1),
                                                         (int)(k & 1), b->launch, cs);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    });
}

// Multi-step mode: class-1 members advance k2 steps per k2-step launch,
// class-0 members by one-step sweeps, each class with its own lattice
// parity (parity, parity2); graphs start and end at parities 0, 0.
static trt_status batch_step_two(trt_batch *b, int64_t n) {
    const int k2 = b->k2;
    auto single = [&]() -> trt_status {
        TRT_HIP(batch_single(b, b->parity, b->parity2, b->stream));
        b->parity ^= 1;
        b->parity2 ^= 1;
        batch_sync_members(b, 1, 1, 1);
        return TRT_OK;
    };
    auto unit = [&]() -> trt_status {
        TRT_HIP(batch_unit(b, b->parity, b->parity2, b->stream));
        b->parity ^= k2 & 1;
        b->parity2 ^= 1;
        batch_sync_members(b, k2, k2, 1);
        return TRT_OK;
    };
    // back to parities 0, 0: a single step flips both classes, a unit class
    // 1 and, for odd k2, class 0 (at most two launches)
    while (n > 0 && (b->parity || b->parity2)) {
        const bool unit_returns = (b->parity ^ (k2 & 1)) == 0 && (b->parity2 ^ 1) == 0;
        const bool one = n < k2 || !unit_returns;
        trt_status st = one ? single() : unit();
        if (st != TRT_OK) return st;
        n -= one ? 1 : k2;
    }
    if (n >= 2 * k2) {
        // graphs of 2, 4, ... units (2 k2, 4 k2, ... steps), each from and
        // back to parities 0, 0
        const int64_t units = n / (2 * k2) * 2;
        trt_status rs = replay_ladder(
            units, std::max<int64_t>(2, b->launch.graph_steps / 2), b->graphs, b->stream,
            [&](int k) -> trt_status {
                if (b->graphs[k]) return TRT_OK;
                return batch_capture(b, b->graphs[k], (int64_t)2 << k);
            });
        if (rs != TRT_OK) return rs;
        batch_sync_members(b, k2 * units, k2 * units, units);
        n -= k2 * units;
    }
    if (n >= k2) {
        trt_status st = unit();
        if (st != TRT_OK) return st;
        n -= k2;
    }
    while (n > 0) {
        trt_status st = single();
        if (st != TRT_OK) return st;
        --n;
    }
    return TRT_OK;
}

trt_status trt_batch_step(trt_batch *b, int64_t nsteps) {
    if (!b) return fail(TRT_EINVAL, "batch handle is NULL");
    if (nsteps < 0) return fail(TRT_EINVAL, "nsteps must be >= 0");
    int64_t n = nsteps;
    if (n == 0) return TRT_OK;
    if (b->nitems2 > 0) return batch_step_two(b, n);
    if (b->parity == 1) {
        TRT_HIP(trt::launch_sweep_batch(b->d_descs, b->d_items, b->nitems, b->storage, b->mask,
                                        b->buf, 1, 1, b->launch, b->stream));
        b->parity = 0;
        batch_sync_members(b, 1, 1, 1);
        --n;
    }
    if (n >= 2) {
        const int64_t even = n / 2 * 2;
        trt_status rs = replay_ladder(even, b->launch.graph_steps, b->graphs, b->stream,
                                      [&](int k) -> trt_status {
                                          if (b->graphs[k]) return TRT_OK;
                                          return batch_capture(b, b->graphs[k], (int64_t)2 << k);
                                      });
        if (rs != TRT_OK) return rs;
        batch_sync_members(b, even, even, even);
    }
    if (n % 2) {
        TRT_HIP(trt::launch_sweep_batch(b->d_descs, b->d_items, b->nitems, b->storage, b->mask,
                                        b->buf, 0, 0, b->launch, b->stream));
        b->parity = 1;
        batch_sync_members(b, 1, 1, 1);
    }
    return TRT_OK;
}

trt_status trt_batch_diagnostics(trt_batch *b, double *out) {
    if (!b) return fail(TRT_EINVAL, "batch handle is NULL");
    if (!out) return fail(TRT_EINVAL, "out is NULL");
    for (size_t k = 0; k < b->sims.size(); ++k) {
        trt_status st = trt_diagnostics(b->sims[k], out + k * TRT_NDIAG);
        if (st != TRT_OK) return st;
    }
    return TRT_OK;
}

void trt_batch_destroy(trt_batch *b) {
    if (!b) return;
    for (trt_sim *s : b->sims) s->in_batch = false;
    release_graphs(b->graphs);
    for (auto &sg : b->stage) {
        if (sg.pending) (void)hipEventSynchronize(sg.done);
        if (sg.done) (void)hipEventDestroy(sg.done);
        if (sg.descs) (void)hipHostFree(sg.descs);
        if (sg.items) (void)hipHostFree(sg.items);
    }
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->d_descs) (void)hipFree(b->d_descs);
    if (b->d_items) (void)hipFree(b->d_items);
    for (void *p : b->retired_dev) (void)hipFree(p);
    for (void *p : b->retired_host) (void)hipHostFree(p);
    delete b;
}

const char *trt_last_error(void) { return g_err.c_str(); }

const char *trt_version(void) { return "trtlbm 0.1 (gfx950)"; }

}  // extern "C"
