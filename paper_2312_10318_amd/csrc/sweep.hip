// sweep.hip -- the fused D2Q9 TRT-RLB stream-and-collide sweep for gfx950.
//
// One launch performs one time step of the evolution equation (Yu et al.,
// arXiv:2312.10318, Sec. II.B, Eq. 2) on every node: pull-gather with
// periodic wrap and half-way bounce-back (Sec. II.D), moments with the He
// shift (Eqs. 12-13), the compensation term's gradient of Phi = rho u^3
// (Eqs. 8-10) from the neighbours' moments at the same time level, the
// regularized TRT collision, and one store per population.
//
// Work decomposition.  A wavefront owns an aligned strip of 64 columns and
// marches down `rows` consecutive rows, lane l holding column 64*strip + l,
// so every load and store of a population row is one aligned, fully used
// segment.  The x-neighbours' Phi_x come from the adjacent lanes (cross-lane
// shuffle); at the strip edges, lanes 0 and 63 also gather the two halo
// columns 64*strip - 1 and 64*strip + 64 (a predicated gather with two
// active lanes) to form their Phi_x;
// the y-neighbours' Phi_y come from a register window (Phi_y of the row
// below is kept from the previous iteration; the row above is gathered
// while the current row's collision coefficients are formed, and becomes
// the current row of the next iteration).  Each population is read once per node from HBM and written
// once; the edge lanes and the first/last row of a strip re-read data that
// neighbouring strips also read (served by L2).  No LDS, no barriers: waves
// are independent.
//
// The gradient d_gamma Phi is the central difference of rho u_x^3 (rho u_y^3)
// between the two neighbours in x (y) at time t; a solid neighbour
// contributes Phi = 0.
#include <type_traits>

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

// Per-lane geometry of one strip column.
struct Column {
    int xm, xc, xp;        // wrapped columns x-1, x, x+1
    uint32_t om, oc, op;   // their byte offsets within a row
};

__device__ __forceinline__ Column column_of(int c, int nx, uint32_t elem) {
    Column col;
    col.xc = c % nx;
    if (col.xc < 0) col.xc += nx;
    col.xm = (col.xc == 0) ? nx - 1 : col.xc - 1;
    col.xp = (col.xc == nx - 1) ? 0 : col.xc + 1;
    col.om = (uint32_t)col.xm * elem;
    col.oc = (uint32_t)col.xc * elem;
    col.op = (uint32_t)col.xp * elem;
    return col;
}

// Raw (storage-precision) populations of one node, gathered but not yet
// widened, so that a prefetched row costs as few registers as possible.
template <class T> struct Raw {
    T v[9];
    bool solid;
};

template <class T, bool MASK, class Acc>
__device__ __forceinline__ void gather_raw(Raw<T> &r, const Acc &in, const T *src, int64_t plane,
                                           int pitch, const uint8_t *mask, int nx, int ny, int y,
                                           const Column &col) {
    const int ym = (y == 0) ? ny - 1 : y - 1;
    const int yp = (y == ny - 1) ? 0 : y + 1;
    r.solid = false;
    if (MASK && mask != nullptr) {
        r.solid = gather_masked_raw<T>(src, plane, pitch, mask, nx, ym, y, yp, col.xm, col.xc,
                                       col.xp, r.v);
        return;
    }
    const int64_t e0 = (int64_t)y * pitch, em = (int64_t)ym * pitch, ep = (int64_t)yp * pitch;
    r.v[0] = in.ld(e0, col.oc);
    r.v[1] = in.ld(plane + e0, col.om);
    r.v[2] = in.ld(2 * plane + em, col.oc);
    r.v[3] = in.ld(3 * plane + e0, col.op);
    r.v[4] = in.ld(4 * plane + ep, col.oc);
    r.v[5] = in.ld(5 * plane + em, col.om);
    r.v[6] = in.ld(6 * plane + em, col.op);
    r.v[7] = in.ld(7 * plane + ep, col.op);
    r.v[8] = in.ld(8 * plane + ep, col.om);
}

template <class C, bool SHIFTED> struct RowState {
    C f[9];
    Moments<C, SHIFTED> m;
    C phix, phiy;
    bool solid;
};

template <class T, class C, bool SHIFTED>
__device__ __forceinline__ void widen(RowState<C, SHIFTED> &r, const Raw<T> &raw, C gx, C gy) {
#pragma unroll
    for (int i = 0; i < 9; ++i) r.f[i] = to_c(raw.v[i]);
    r.solid = raw.solid;
    r.m.compute(r.f, gx, gy);
    const C px = r.m.rho * r.m.ux * r.m.ux * r.m.ux;
    const C py = r.m.rho * r.m.uy * r.m.uy * r.m.uy;
    r.phix = r.solid ? C(0) : px;
    r.phiy = r.solid ? C(0) : py;
}

// Phi_x of a halo node from its raw populations (0 at a solid node).
template <class T, class C, bool SHIFTED>
__device__ __forceinline__ C halo_phix(const Raw<T> &raw, C gx, C gy) {
    C f[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = to_c(raw.v[i]);
    Moments<C, SHIFTED> m;
    m.compute(f, gx, gy);
    return raw.solid ? C(0) : m.rho * m.ux * m.ux * m.ux;
}

static_assert(kStripWidth == 64, "one strip column per lane of a 64-wide wavefront");

template <int ST, bool MASK, bool BUF>
__device__ __forceinline__ void sweep_strip(const InstDesc &d, int strip, int rb, int srcsel) {
    using T = typename Store<ST>::T;
    using C = typename Store<ST>::C;
    using Acc = typename std::conditional<BUF, BufAccess<T>, PtrAccess<T>>::type;
    constexpr bool SH = Store<ST>::shifted;

    const int lane = threadIdx.x & 63;
    const int nx = d.nx, ny = d.ny, pitch = d.pitch;
    const int64_t plane = d.plane;
    // select without indexing so that a descriptor held in registers is
    // never spilled to scratch
    const T *__restrict__ src = static_cast<const T *>(srcsel ? d.buf[1] : d.buf[0]);
    T *__restrict__ dst = static_cast<T *>(srcsel ? d.buf[0] : d.buf[1]);
    const uint8_t *mask = MASK ? d.mask : nullptr;
    const uint64_t bytes = 9ull * (uint64_t)plane * sizeof(T);
    const Acc in(src, bytes), out(dst, bytes);

    const int x0 = strip * kStripWidth;
    const Column col = column_of(x0 + lane, nx, sizeof(T));
    // halo columns x0 - 1 (lane 0) and x0 + 64 (lane 63)
    const bool edge = lane == 0 || lane == kStripWidth - 1;
    const Column hcol = column_of(lane == 0 ? x0 - 1 : x0 + kStripWidth, nx, sizeof(T));
    const bool writer = x0 + lane < nx;

    const C gx = (C)d.gx, gy = (C)d.gy;
    const C w1 = (C)d.omega1, w2 = (C)d.omega2, ph = (C)d.phi;

    const int y0 = rb * d.rows;
    const int y1 = min(y0 + d.rows, ny);

    // Register window.  Row y: widened state `cur` and its halo Phi_x; row
    // y+1: raw populations (and halo raw populations), gathered while row y's
    // collision is formed.  Phi_y of row y-1 is kept as a scalar.
    C phiy_below;
    {
        Raw<T> t;
        RowState<C, SH> w;
        gather_raw<T, MASK>(t, in, src, plane, pitch, mask, nx, ny, (y0 + ny - 1) % ny, col);
        widen<T, C, SH>(w, t, gx, gy);
        phiy_below = w.phiy;
    }
    RowState<C, SH> cur;
    C hphix = C(0);
    {
        Raw<T> t;
        gather_raw<T, MASK>(t, in, src, plane, pitch, mask, nx, ny, y0, col);
        widen<T, C, SH>(cur, t, gx, gy);
        if (edge) {
            Raw<T> h;
            gather_raw<T, MASK>(h, in, src, plane, pitch, mask, nx, ny, y0, hcol);
            hphix = halo_phix<T, C, SH>(h, gx, gy);
        }
    }

    for (int y = y0; y < y1; ++y) {
        // row y+1: its Phi_y is needed now, its state in the next iteration
        const int yn = (y + 1 == ny) ? 0 : y + 1;
        Raw<T> nraw, nhalo;
        gather_raw<T, MASK>(nraw, in, src, plane, pitch, mask, nx, ny, yn, col);
        if (edge) gather_raw<T, MASK>(nhalo, in, src, plane, pitch, mask, nx, ny, yn, hcol);

        // row y: everything of the collision except the y-gradient of Phi
        const C up = __shfl_up(cur.phix, 1), dn = __shfl_down(cur.phix, 1);
        const C phix_l = (lane == 0) ? hphix : up;
        const C phix_r = (lane == kStripWidth - 1) ? hphix : dn;
        const C dphix = C(0.5) * (phix_r - phix_l);
        Coeffs<C> cf = collide_coeffs<C, SH>(cur.f, cur.m, dphix, w1, w2, ph, gx, gy);
        // pin the coefficients here, ahead of the wait for row y+1's loads
        // (otherwise they are sunk into the masked store block below)
        asm volatile("" : "+v"(cf.base), "+v"(cf.bx), "+v"(cf.by), "+v"(cf.bxx), "+v"(cf.byy),
                     "+v"(cf.bxy), "+v"(cf.bxxy), "+v"(cf.bxyy));

        RowState<C, SH> nxt;
        widen<T, C, SH>(nxt, nraw, gx, gy);
        const C nhphix = edge ? halo_phix<T, C, SH>(nhalo, gx, gy) : C(0);

        const C dphiy = C(0.5) * (nxt.phiy - phiy_below);
        C fo[9];
        reconstruct<C>(fo, cf.base, cf.bx, cf.by, cf.bxx, cf.byy - ph * dphiy, cf.bxy, cf.bxxy,
                       cf.bxyy);
        if (writer && !cur.solid) {
            const int64_t e0 = (int64_t)y * pitch;
#pragma unroll
            for (int i = 0; i < 9; ++i) out.st(i * plane + e0, col.oc, from_c<T, C>(fo[i]));
        }
        phiy_below = cur.phiy;
        cur = nxt;
        hphix = nhphix;
    }
}

template <int ST, bool MASK, bool BUF>
__global__ __launch_bounds__(256) void sweep_single_kernel(InstDesc d, int srcsel, int remap) {
    int b = blockIdx.x;
    if (remap) b = xcd_remap(b, gridDim.x);
    const int wpb = blockDim.x >> 6;
    const int wave = b * wpb + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= d.strips * d.rowblocks) return;
    const int rb = wave / d.strips;
    const int strip = wave - rb * d.strips;
    sweep_strip<ST, MASK, BUF>(d, strip, rb, srcsel);
}

template <int ST, bool MASK, bool BUF>
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
    sweep_strip<ST, MASK, BUF>(d, it.y, it.z, d.cur ^ flip);
}

template <int ST, bool MASK, bool BUF>
hipError_t launch_single_t(const InstDesc &d, int src, const Launch &l, hipStream_t s) {
    const int waves = d.strips * d.rowblocks;
    const int wpb = l.waves_per_block;
    const int blocks = (waves + wpb - 1) / wpb;
    sweep_single_kernel<ST, MASK, BUF><<<blocks, 64 * wpb, 0, s>>>(d, src, l.xcd_remap);
    return hipGetLastError();
}

template <int ST, bool MASK, bool BUF>
hipError_t launch_batch_t(const InstDesc *descs, const int4 *items, int nitems, int flip,
                          const Launch &l, hipStream_t s) {
    const int wpb = l.waves_per_block;
    const int blocks = (nitems + wpb - 1) / wpb;
    sweep_batch_kernel<ST, MASK, BUF><<<blocks, 64 * wpb, 0, s>>>(descs, items, nitems, flip,
                                                                 l.xcd_remap);
    return hipGetLastError();
}

template <int ST, bool MASK>
hipError_t launch_single_b(const InstDesc &d, int src, const Launch &l, bool buf, hipStream_t s) {
    return buf ? launch_single_t<ST, MASK, true>(d, src, l, s)
               : launch_single_t<ST, MASK, false>(d, src, l, s);
}

template <int ST, bool MASK>
hipError_t launch_batch_b(const InstDesc *descs, const int4 *items, int nitems, int flip,
                          const Launch &l, bool buf, hipStream_t s) {
    return buf ? launch_batch_t<ST, MASK, true>(descs, items, nitems, flip, l, s)
               : launch_batch_t<ST, MASK, false>(descs, items, nitems, flip, l, s);
}

}  // namespace

bool buffer_addressable(const InstDesc &d, int storage) {
    const uint64_t es = storage == ST_F64 ? 8 : (storage == ST_F32 ? 4 : 2);
    return 9ull * (uint64_t)d.plane * es <= 0xffffffffull;
}

hipError_t launch_sweep(const InstDesc &d, int storage, bool mask, int src, const Launch &l,
                        hipStream_t stream) {
    const bool buf = buffer_addressable(d, storage);
    switch (storage * 2 + (mask ? 1 : 0)) {
        case 0: return launch_single_b<ST_F64, false>(d, src, l, buf, stream);
        case 1: return launch_single_b<ST_F64, true>(d, src, l, buf, stream);
        case 2: return launch_single_b<ST_F32, false>(d, src, l, buf, stream);
        case 3: return launch_single_b<ST_F32, true>(d, src, l, buf, stream);
        case 4: return launch_single_b<ST_F16, false>(d, src, l, buf, stream);
        case 5: return launch_single_b<ST_F16, true>(d, src, l, buf, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep_batch(const InstDesc *descs, const int4 *items, int nitems, int storage,
                              bool mask, bool buf, int flip, const Launch &l,
                              hipStream_t stream) {
    switch (storage * 2 + (mask ? 1 : 0)) {
        case 0: return launch_batch_b<ST_F64, false>(descs, items, nitems, flip, l, buf, stream);
        case 1: return launch_batch_b<ST_F64, true>(descs, items, nitems, flip, l, buf, stream);
        case 2: return launch_batch_b<ST_F32, false>(descs, items, nitems, flip, l, buf, stream);
        case 3: return launch_batch_b<ST_F32, true>(descs, items, nitems, flip, l, buf, stream);
        case 4: return launch_batch_b<ST_F16, false>(descs, items, nitems, flip, l, buf, stream);
        case 5: return launch_batch_b<ST_F16, true>(descs, items, nitems, flip, l, buf, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace trt
