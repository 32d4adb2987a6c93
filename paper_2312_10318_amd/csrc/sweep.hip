// sweep.hip -- the fused D2Q9 TRT-RLB stream-and-collide sweep for gfx950.
//
// One launch performs one time step of the evolution equation (Yu et al.,
// arXiv:2312.10318, Sec. II.B, Eq. 2) on every node: pull-gather with
// periodic wrap and half-way bounce-back (Sec. II.D), moments with the He
// shift (Eqs. 12-13), the compensation term's gradient of Phi = rho u^3
// (Eqs. 8-10) from the neighbours' moments at the same time level, the
// regularized TRT collision, and one store per population.
//
// Work decomposition.  A wavefront owns a strip of 62 columns and marches
// down `rows` consecutive rows.  Lane l holds column 62*strip + l - 1: lanes
// 1..62 produce output, lanes 0 and 63 compute the moments of the two
// neighbouring columns so that d_x Phi_x of the edge columns can be formed.
// The x-neighbours' Phi_x come from the adjacent lanes (cross-lane shuffle);
// the y-neighbours' Phi_y come from a three-row register window (the row
// below is kept from the previous iteration, the row above is gathered one
// row ahead).  Each population is read once per node from HBM and written
// once; the edge lanes and the first/last row of a strip re-read data that
// neighbouring strips also read (served by L2).  No LDS, no barriers: waves
// are independent.
//
// The gradient d_gamma Phi is the central difference of rho u_x^3 (rho u_y^3)
// between the two neighbours in x (y) at time t; a solid neighbour
// contributes Phi = 0.
#include "kernels.hpp"

namespace trt {

namespace {

// Remap the hardware workgroup index so that each of the 8 XCDs (dispatched
// round-robin) receives one contiguous range of logical workgroups; with
// strips varying fastest, an XCD then sweeps a contiguous band of rows and
// the halo rows shared by neighbouring wavefronts stay in its own L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    constexpr int kXcd = 8;
    const int per = (nb + kXcd - 1) / kXcd;
    const int tall = (nb % kXcd == 0) ? kXcd : nb % kXcd;
    const int xcd = b % kXcd, local = b / kXcd;
    return xcd < tall ? xcd * per + local : tall * per + (xcd - tall) * (per - 1) + local;
}

template <class C, bool SHIFTED> struct RowState {
    C f[9];
    Moments<C, SHIFTED> m;
    C phix, phiy;
    bool solid;
};

template <class T, class C, bool SHIFTED, bool MASK>
__device__ __forceinline__ void load_row(RowState<C, SHIFTED> &r, const T *src, int64_t plane,
                                         int pitch, const uint8_t *mask, int nx, int ny, int y,
                                         int xm, int xc, int xp, C gx, C gy) {
    r.solid = gather<T, C, MASK>(src, plane, pitch, mask, nx, ny, y, xm, xc, xp, r.f);
    r.m.compute(r.f, gx, gy);
    const C px = r.m.rho * r.m.ux * r.m.ux * r.m.ux;
    const C py = r.m.rho * r.m.uy * r.m.uy * r.m.uy;
    r.phix = r.solid ? C(0) : px;
    r.phiy = r.solid ? C(0) : py;
}

template <int ST, bool MASK>
__device__ __forceinline__ void sweep_strip(const InstDesc &d, int strip, int rb, int srcsel) {
    using T = typename Store<ST>::T;
    using C = typename Store<ST>::C;
    constexpr bool SH = Store<ST>::shifted;

    const int lane = threadIdx.x & 63;
    const int nx = d.nx, ny = d.ny, pitch = d.pitch;
    const int64_t plane = d.plane;
    // select without indexing so that a descriptor held in registers is
    // never spilled to scratch
    const T *__restrict__ src = static_cast<const T *>(srcsel ? d.buf[1] : d.buf[0]);
    T *__restrict__ dst = static_cast<T *>(srcsel ? d.buf[0] : d.buf[1]);
    const uint8_t *mask = MASK ? d.mask : nullptr;

    const int c = strip * kStripWidth + lane - 1;
    int xc = c % nx;
    if (xc < 0) xc += nx;
    const int xm = (xc == 0) ? nx - 1 : xc - 1;
    const int xp = (xc == nx - 1) ? 0 : xc + 1;
    const bool writer = lane >= 1 && lane <= kStripWidth && c < nx;

    const C gx = (C)d.gx, gy = (C)d.gy;
    const C w1 = (C)d.omega1, w2 = (C)d.omega2, ph = (C)d.phi;

    const int y0 = rb * d.rows;
    const int y1 = min(y0 + d.rows, ny);

    // register window: Phi_y of row y-1, full state of rows y and y+1
    C phiy_below;
    {
        RowState<C, SH> t;
        load_row<T, C, SH, MASK>(t, src, plane, pitch, mask, nx, ny, (y0 + ny - 1) % ny, xm, xc,
                                 xp, gx, gy);
        phiy_below = t.phiy;
    }
    RowState<C, SH> cur, nxt;
    load_row<T, C, SH, MASK>(cur, src, plane, pitch, mask, nx, ny, y0, xm, xc, xp, gx, gy);
    load_row<T, C, SH, MASK>(nxt, src, plane, pitch, mask, nx, ny, (y0 + 1) % ny, xm, xc, xp, gx,
                             gy);

    for (int y = y0; y < y1; ++y) {
        const bool more = y + 1 < y1;
        RowState<C, SH> ahead;
        if (more)
            load_row<T, C, SH, MASK>(ahead, src, plane, pitch, mask, nx, ny, (y + 2) % ny, xm, xc,
                                     xp, gx, gy);

        const C phix_l = __shfl_up(cur.phix, 1);
        const C phix_r = __shfl_down(cur.phix, 1);
        const C dphix = C(0.5) * (phix_r - phix_l);
        const C dphiy = C(0.5) * (nxt.phiy - phiy_below);
        if (writer && !cur.solid) {
            collide<C, SH>(cur.f, cur.m, dphix, dphiy, w1, w2, ph, gx, gy);
            T *o = dst + (int64_t)y * pitch + xc;
#pragma unroll
            for (int i = 0; i < 9; ++i) o[i * plane] = from_c<T, C>(cur.f[i]);
        }
        phiy_below = cur.phiy;
        cur = nxt;
        if (more) nxt = ahead;
    }
}

template <int ST, bool MASK>
__global__ __launch_bounds__(256) void sweep_single_kernel(InstDesc d, int srcsel, int remap) {
    int b = blockIdx.x;
    if (remap) b = xcd_remap(b, gridDim.x);
    const int wpb = blockDim.x >> 6;
    const int wave = b * wpb + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= d.strips * d.rowblocks) return;
    const int rb = wave / d.strips;
    const int strip = wave - rb * d.strips;
    sweep_strip<ST, MASK>(d, strip, rb, srcsel);
}

template <int ST, bool MASK>
__global__ __launch_bounds__(256) void sweep_batch_kernel(const InstDesc *__restrict__ descs,
                                                           const int4 *__restrict__ items,
                                                           int nitems, int flip, int remap) {
    int b = blockIdx.x;
    if (remap) b = xcd_remap(b, gridDim.x);
    const int wpb = blockDim.x >> 6;
    const int wave = b * wpb + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= nitems) return;
    const int4 it = items[wave];
    const InstDesc d = descs[it.x];
    sweep_strip<ST, MASK>(d, it.y, it.z, d.cur ^ flip);
}

template <int ST, bool MASK>
hipError_t launch_single_t(const InstDesc &d, int src, const Launch &l, hipStream_t s) {
    const int waves = d.strips * d.rowblocks;
    const int wpb = l.waves_per_block;
    const int blocks = (waves + wpb - 1) / wpb;
    sweep_single_kernel<ST, MASK><<<blocks, 64 * wpb, 0, s>>>(d, src, l.xcd_remap);
    return hipGetLastError();
}

template <int ST, bool MASK>
hipError_t launch_batch_t(const InstDesc *descs, const int4 *items, int nitems, int flip,
                          const Launch &l, hipStream_t s) {
    const int wpb = l.waves_per_block;
    const int blocks = (nitems + wpb - 1) / wpb;
    sweep_batch_kernel<ST, MASK><<<blocks, 64 * wpb, 0, s>>>(descs, items, nitems, flip,
                                                            l.xcd_remap);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sweep(const InstDesc &d, int storage, bool mask, int src, const Launch &l,
                        hipStream_t stream) {
    switch (storage * 2 + (mask ? 1 : 0)) {
        case 0: return launch_single_t<ST_F64, false>(d, src, l, stream);
        case 1: return launch_single_t<ST_F64, true>(d, src, l, stream);
        case 2: return launch_single_t<ST_F32, false>(d, src, l, stream);
        case 3: return launch_single_t<ST_F32, true>(d, src, l, stream);
        case 4: return launch_single_t<ST_F16, false>(d, src, l, stream);
        case 5: return launch_single_t<ST_F16, true>(d, src, l, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep_batch(const InstDesc *descs, const int4 *items, int nitems, int storage,
                              bool mask, int flip, const Launch &l, hipStream_t stream) {
    switch (storage * 2 + (mask ? 1 : 0)) {
        case 0: return launch_batch_t<ST_F64, false>(descs, items, nitems, flip, l, stream);
        case 1: return launch_batch_t<ST_F64, true>(descs, items, nitems, flip, l, stream);
        case 2: return launch_batch_t<ST_F32, false>(descs, items, nitems, flip, l, stream);
        case 3: return launch_batch_t<ST_F32, true>(descs, items, nitems, flip, l, stream);
        case 4: return launch_batch_t<ST_F16, false>(descs, items, nitems, flip, l, stream);
        case 5: return launch_batch_t<ST_F16, true>(descs, items, nitems, flip, l, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace trt
