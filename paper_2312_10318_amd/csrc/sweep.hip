// sweep.hip -- the fused D2Q9 TRT-RLB stream-and-collide sweep for gfx950.
//
// One launch performs one time step of the evolution equation (Yu et al.,
// arXiv:2312.10318, Sec. II.B, Eq. 2) on every node: pull-gather with
// periodic wrap and half-way bounce-back (Sec. II.D), moments with the He
// shift (Eqs. 12-13), the compensation term's gradient of Phi = rho u^3
// (Eqs. 8-10) from the neighbours' moments at the same time level, the
// regularized TRT collision, and one store per population.
//
// Work decomposition (one column per lane; the two-column variant below
// keeps the same structure with 128-column strips).  A wavefront owns an
// aligned strip of 64 columns and marches down `rows` consecutive rows, lane
// l holding column 64*strip + l, so every load and store of a population row
// is one aligned, fully used segment.  The x-neighbours' Phi_x come from the
// adjacent lanes (DPP whole-wave shifts); at the strip edges, lanes 0 and 63
// also gather the two halo columns 64*strip - 1 and 64*strip + 64 (a
// predicated gather with two active lanes) to form their Phi_x; the
// y-neighbours' Phi_y come from a register window (Phi_y of the row below is
// kept from the previous iteration; the row above is gathered while the
// current row's collision coefficients are formed, and becomes the current
// row of the next iteration).  Each population is read once per node from
// HBM and written once; the edge lanes and the first/last row of a strip
// re-read data that neighbouring strips also read (served by L2).  No LDS.
// One-column wavefronts are independent; single-lattice two-column launches
// keep the adjacent strips of a workgroup in step with one barrier per row.
//
// The gradient d_gamma Phi is the central difference of rho u_x^3 (rho u_y^3)
// between the two neighbours in x (y) at time t; a solid neighbour
// contributes Phi = 0.
#include <type_traits>

#include "kernels.hpp"

namespace trt {


namespace {


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
// With a link map, lk holds the node's link code (bit 0: solid; bit i: f_i
// bounces back) and own[i] the node's own slot opp(i) wherever some lane of
// the wavefront needs it.
template <class T> struct Raw {
    T v[9];
    T own[9];
    bool solid;
    uint32_t lk;
};

// Pull-gather of node (col, y) (periodic wrap).  With a link map the node's
// link code lk is already known (it is read one row ahead), so the own-slot
// loads of the bounce-back directions are issued here, together with the
// pulls; link_fix selects later, where the loads are waited for anyway.
template <class T, class Acc>
__device__ __forceinline__ void gather_raw(Raw<T> &r, const Acc &in, int64_t plane, int pitch,
                                           int ny, int y, const Column &col, bool linked,
                                           uint32_t lk, uint32_t own) {
    const int ym = (y == 0) ? ny - 1 : y - 1;
    const int yp = (y == ny - 1) ? 0 : y + 1;
    r.solid = false;
    r.lk = lk;
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
    if (linked && (own & 0xfffeu) != 0u) {
#pragma unroll
        for (int i = 1; i < 9; ++i)
            if ((own >> i) & 1u) r.own[i] = in.ld(kOppDir[i] * plane + e0, col.oc);
    }
}

// Apply a gathered node's link code: bounce-back sources and solidity (only
// rows that touch a wall or an obstacle do any work).
template <class T>
__device__ __forceinline__ void link_fix(Raw<T> &r) {
    if (__builtin_amdgcn_ballot_w64(r.lk != 0) == 0) return;
#pragma unroll
    for (int i = 1; i < 9; ++i)
        if (__builtin_amdgcn_ballot_w64((r.lk >> i) & 1u) != 0)
            r.v[i] = ((r.lk >> i) & 1u) ? r.own[i] : r.v[i];
    r.solid = (r.lk & 1u) != 0;
}

// One row's state per lane: moments (raw ones included) and Phi.
template <class C, bool SHIFTED> struct RowState {
    Moments<C, SHIFTED> m;
    C phix, phiy;
    bool solid;
};

// Boundary data of open x boundaries, in the arithmetic precision.
template <class C> struct OpenX {
    bool on;
    int nx;
    C u_in, rho_in, rho_out, phi_wall;
};

template <class T, class C, bool SHIFTED>
__device__ __forceinline__ void widen(RowState<C, SHIFTED> &r, const Raw<T> &raw, C gx, C gy,
                                      const OpenX<C> &ox, int xc) {
    C f[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = to_c(raw.v[i]);
    if (ox.on) open_x_fix<C, SHIFTED>(f, xc, ox.nx, ox.u_in, ox.rho_in, ox.rho_out);
    r.solid = raw.solid;
    r.m.compute(f, gx, gy);
    const C px = r.m.rho * r.m.ux * r.m.ux * r.m.ux;
    const C py = r.m.rho * r.m.uy * r.m.uy * r.m.uy;
    r.phix = r.solid ? C(0) : px;
    r.phiy = r.solid ? C(0) : py;
}

// Phi_x of a halo node from its raw populations (0 at a solid node): only
// rho and j_x are needed.  The partial sums are taken in exactly the order of
// Moments::compute, so a halo lane reproduces bit for bit the Phi_x that the
// lane owning that column computes: results do not depend on where strips
// begin and end.
template <class T, class C, bool SHIFTED>
__device__ __forceinline__ C halo_phix(const Raw<T> &raw, C gx, const OpenX<C> &ox, int xc) {
    C f[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = to_c(raw.v[i]);
    if (ox.on) open_x_fix<C, SHIFTED>(f, xc, ox.nx, ox.u_in, ox.rho_in, ox.rho_out);
    const C s56 = f[5] + f[6], s78 = f[7] + f[8];
    const C d56 = f[5] - f[6], d78 = f[7] - f[8];
    const C diag = s56 + s78;
    const C qxyy = d56 - d78;
    const C a13 = f[1] + f[3], a24 = f[2] + f[4];
    const C jx = (f[1] - f[3]) + qxyy;
    const C base = (f[0] + a13) + (a24 + diag);
    const C rho = SHIFTED ? C(1) + base : base;
    const C ux = jx * recip(rho) + C(0.5) * gx;
    return raw.solid ? C(0) : rho * ux * ux * ux;
}

static_assert(kStripWidth == 64, "one strip column per lane of a 64-wide wavefront");

// DPP whole-wavefront shifts: lane i receives lane i-1 (shr) or lane i+1
// (shl); the lane with no source keeps `old`.
__device__ __forceinline__ float dpp_shr(float old, float src) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                                  __builtin_bit_cast(int, src),
                                                                  0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float dpp_shl(float old, float src) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                                  __builtin_bit_cast(int, src),
                                                                  0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ uint32_t dpp_shr(uint32_t old, uint32_t src) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ uint32_t dpp_shl(uint32_t old, uint32_t src) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, 0x130, 0xf, 0xf, false);
}
__device__ __forceinline__ double dpp_shr(double old, double src) {
    const uint64_t o = __builtin_bit_cast(uint64_t, old), v = __builtin_bit_cast(uint64_t, src);
    const uint32_t lo = __builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)v, 0x138, 0xf,
                                                    0xf, false);
    const uint32_t hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(v >> 32),
                                                    0x138, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double dpp_shl(double old, double src) {
    const uint64_t o = __builtin_bit_cast(uint64_t, old), v = __builtin_bit_cast(uint64_t, src);
    const uint32_t lo = __builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)v, 0x130, 0xf,
                                                    0xf, false);
    const uint32_t hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(v >> 32),
                                                    0x130, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Store the FP16 population held in the low half of a register.
template <class Acc>
__device__ __forceinline__ void store_half(const Acc &out, int64_t e, uint32_t oc, uint32_t r) {
    out.st(e, oc, __builtin_bit_cast(_Float16, (unsigned short)(r & 0xffffu)));
}

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
    const uint64_t bytes = (uint64_t)ny * (uint64_t)pitch * sizeof(T);
    const Acc in(src, bytes), out(dst, bytes);
    // obstacles and open boundaries: the link map (general kernels only)
    const bool linked = MASK && d.links != nullptr;
    const LinkAccess la(d.links, (uint64_t)ny * (uint64_t)d.lpitch);
    const int64_t lp = d.lpitch;

    const int x0 = strip * kStripWidth;
    const Column col = column_of(x0 + lane, nx, sizeof(T));
    // halo columns x0 - 1 (lane 0) and x0 + 64 (lane 63)
    const bool edge = lane == 0 || lane == kStripWidth - 1;
    const Column hcol = column_of(lane == 0 ? x0 - 1 : x0 + kStripWidth, nx, sizeof(T));
    const bool writer = x0 + lane < nx;

    const C gx = (C)d.gx, gy = (C)d.gy;
    const C w1 = (C)d.omega1, w2 = (C)d.omega2, ph = (C)d.phi;
    // open x boundaries: only in the general (MASK) kernels
    OpenX<C> ox;
    ox.on = MASK && d.xbc != 0;
    ox.nx = nx;
    ox.u_in = (C)d.u_in;
    ox.rho_in = (C)d.rho_in;
    ox.rho_out = (C)d.rho_out;
    ox.phi_wall = ox.rho_in * ox.u_in * ox.u_in * ox.u_in;

    const int y0 = rb * d.rows;
    const int y1 = min(y0 + d.rows, ny);

    // Register window.  Row y: widened state `cur` and its halo Phi_x; row
    // y+1: raw populations (and halo raw populations), gathered while row y's
    // collision is formed.  Phi_y of row y-1 is kept as a scalar.
    // link codes (0 without a link map): rows y0 - 1 and y0 now, row y0 + 1
    // one row ahead, and so on (for the halo column of the edge lanes too)
    // the strip's link summary of a row (scalar; 0: no link step), and a
    // node's code, read only in rows whose summary is not 0
    const RowSum rsum(d.rowsum, d.nsum);
    const auto summary = [&](int row) -> uint32_t { return linked ? rsum.one(row, strip) : 0u; };
    const auto code = [&](int row, const Column &c, uint32_t rs) -> uint32_t {
        return (linked && rs != 0u) ? la.ld1((uint32_t)((int64_t)row * lp), (uint32_t)c.xc) : 0u;
    };
    const int ym0 = (y0 + ny - 1) % ny, yp0 = (y0 + 1) % ny;
    C phiy_below;
    {
        Raw<T> t;
        RowState<C, SH> w;
        const uint32_t rs = summary(ym0);
        gather_raw<T>(t, in, plane, pitch, ny, ym0, col, linked, code(ym0, col, rs), rs);
        if (linked) link_fix(t);
        widen<T, C, SH>(w, t, gx, gy, ox, col.xc);
        phiy_below = w.phiy;
    }
    RowState<C, SH> cur;
    C hphix = C(0);
    {
        Raw<T> t;
        const uint32_t rs = summary(y0);
        gather_raw<T>(t, in, plane, pitch, ny, y0, col, linked, code(y0, col, rs), rs);
        if (linked) link_fix(t);
        widen<T, C, SH>(cur, t, gx, gy, ox, col.xc);
        if (edge) {
            Raw<T> h;
            gather_raw<T>(h, in, plane, pitch, ny, y0, hcol, linked, code(y0, hcol, rs), rs);
            if (linked) link_fix(h);
            hphix = halo_phix<T, C, SH>(h, gx, ox, hcol.xc);
        }
    }
    // link summaries are read one row ahead of the gather they gate; codes
    // with the row's populations (needed only where those are)
    uint32_t rs_next = summary(yp0);

    for (int y = y0; y < y1; ++y) {
        // row y+1: its Phi_y is needed now, its state in the next iteration
        const int yn = (y + 1 == ny) ? 0 : y + 1;
        Raw<T> nraw, nhalo;
        gather_raw<T>(nraw, in, plane, pitch, ny, yn, col, linked, code(yn, col, rs_next), rs_next);
        if (edge)
            gather_raw<T>(nhalo, in, plane, pitch, ny, yn, hcol, linked, code(yn, hcol, rs_next),
                          rs_next);
        rs_next = summary((yn + 1 == ny) ? 0 : yn + 1);

        // row y: everything of the collision except the y-gradient of Phi
        // x-neighbours' Phi_x from the adjacent lanes (lanes 0 and 63: the
        // halo column's, through the shift's `old` operand)
        C phix_l = dpp_shr(hphix, cur.phix);
        C phix_r = dpp_shl(hphix, cur.phix);
        if (ox.on) {
            // Phi beyond the inflow wall is the wall's; beyond the outlet, the last column's
            if (col.xc == 0) phix_l = ox.phi_wall;
            if (col.xc == nx - 1) phix_r = cur.phix;
        }
        const C dphix = C(0.5) * (phix_r - phix_l);
        Coeffs<C> cf = collide_coeffs<C, SH>(cur.m, dphix, w1, w2, ph, gx, gy);
        // pin the coefficients here, ahead of the wait for row y+1's loads
        // (otherwise they are sunk into the masked store block below)
        asm volatile("" : "+v"(cf.base), "+v"(cf.bx), "+v"(cf.by), "+v"(cf.bxx), "+v"(cf.byy),
                     "+v"(cf.bxy), "+v"(cf.bxxy), "+v"(cf.bxyy));

        RowState<C, SH> nxt;
        if (linked) link_fix(nraw);
        widen<T, C, SH>(nxt, nraw, gx, gy, ox, col.xc);
        C nhphix = C(0);
        if (edge) {
            if (linked) link_fix(nhalo);
            nhphix = halo_phix<T, C, SH>(nhalo, gx, ox, hcol.xc);
        }

        const C dphiy = C(0.5) * (nxt.phiy - phiy_below);
        if constexpr (ST == ST_F16) {
            // the same single FP16 rounding per population as the two-column sweep
            HalfPairs p;
            reconstruct_pairs(p, cf.base, cf.bx, cf.by, cf.bxx, cf.byy - ph * dphiy, cf.bxy,
                              cf.bxxy, cf.bxyy);
            if (writer && !cur.solid) {
                const int64_t e0 = (int64_t)y * pitch;
                store_half(out, e0, col.oc, half_out<0, false>(p));
                store_half(out, plane + e0, col.oc, half_out<1, false>(p));
                store_half(out, 2 * plane + e0, col.oc, half_out<2, false>(p));
                store_half(out, 3 * plane + e0, col.oc, half_out<3, false>(p));
                store_half(out, 4 * plane + e0, col.oc, half_out<4, false>(p));
                store_half(out, 5 * plane + e0, col.oc, half_out<5, false>(p));
                store_half(out, 6 * plane + e0, col.oc, half_out<6, false>(p));
                store_half(out, 7 * plane + e0, col.oc, half_out<7, false>(p));
                store_half(out, 8 * plane + e0, col.oc, half_out<8, false>(p));
            }
        } else {
            C fo[9];
            reconstruct<C>(fo, cf.base, cf.bx, cf.by, cf.bxx, cf.byy - ph * dphiy, cf.bxy,
                           cf.bxxy, cf.bxyy);
            if (writer && !cur.solid) {
                const int64_t e0 = (int64_t)y * pitch;
#pragma unroll
                for (int i = 0; i < 9; ++i) out.st(i * plane + e0, col.oc, from_c<T, C>(fo[i]));
            }
        }
        phiy_below = cur.phiy;
        cur = nxt;
        hphix = nhphix;
    }
}

// ---------------------------------------------------------------------------
// Two columns per lane.  A wavefront owns an aligned strip of 128 columns,
// lane l holding the adjacent pair (2l, 2l + 1) and moving both with one
// access per population (4 bytes for FP16, 8 for FP32, 16 for FP64), which
// halves the memory instructions per node and the share of halo work.  The
// x-streamed populations take the missing neighbour element from the
// adjacent lane with a DPP whole-wave shift; the strip's two edge lanes
// supply the elements beyond the strip (and the two halo columns' Phi_x)
// through DPP's "old" operand.  With an odd width the lane holding the last
// column (its node A; node B falls in the row padding and is never read as
// data) also takes column 0's elements and Phi_x as a right edge.  Used for
// every lattice that fits one buffer resource, except widths whose last strip
// holds a single column (nx = 1 mod 128, where lane 0 would be both edges);
// obstacles and open boundaries go through the link map.

constexpr int kStripWidth2 = 128;

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// One pair of adjacent storage elements as loaded/stored by one access.
template <class T> struct PairIO;
template <> struct PairIO<_Float16> {
    typedef uint32_t W;
    __device__ static __forceinline__ W ld(const BufAccess<_Float16> &a, int64_t e, uint32_t v) {
        return __builtin_amdgcn_raw_buffer_load_b32(a.r, v, (uint32_t)(e * 2), 0);
    }
    __device__ static __forceinline__ void split(W w, float &x, float &y) {
        x = (float)__builtin_bit_cast(_Float16, (unsigned short)(w & 0xffffu));
        y = (float)__builtin_bit_cast(_Float16, (unsigned short)(w >> 16));
    }
    __device__ static __forceinline__ void st(const BufAccess<_Float16> &a, int64_t e, uint32_t v,
                                              float x, float y) {
        // a half-precision pair: each conversion writes its own half of the
        // register, with no separate shift and merge
        typedef _Float16 h2 __attribute__((ext_vector_type(2)));
        h2 h;
        h.x = (_Float16)x;
        h.y = (_Float16)y;
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, h), a.r, v,
                                              (uint32_t)(e * 2), TRT_STORE_CPOL);
    }
};
template <> struct PairIO<float> {
    typedef u32x2 W;
    __device__ static __forceinline__ W ld(const BufAccess<float> &a, int64_t e, uint32_t v) {
        return __builtin_amdgcn_raw_buffer_load_b64(a.r, v, (uint32_t)(e * 4), 0);
    }
    __device__ static __forceinline__ void split(W w, float &x, float &y) {
        // elements go through plain scalars: this compiler lowers
        // __builtin_bit_cast of a vector element (w.y) to a read of element 0
        const uint32_t lo = w.x, hi = w.y;
        x = __builtin_bit_cast(float, lo);
        y = __builtin_bit_cast(float, hi);
    }
    __device__ static __forceinline__ void st(const BufAccess<float> &a, int64_t e, uint32_t v,
                                              float x, float y) {
        W w;
        w.x = __builtin_bit_cast(uint32_t, x);
        w.y = __builtin_bit_cast(uint32_t, y);
        __builtin_amdgcn_raw_buffer_store_b64(w, a.r, v, (uint32_t)(e * 4), TRT_STORE_CPOL);
    }
};
template <> struct PairIO<double> {
    typedef u32x4 W;
    __device__ static __forceinline__ W ld(const BufAccess<double> &a, int64_t e, uint32_t v) {
        return __builtin_amdgcn_raw_buffer_load_b128(a.r, v, (uint32_t)(e * 8), 0);
    }
    __device__ static __forceinline__ void split(W w, double &x, double &y) {
        x = __builtin_bit_cast(double, ((uint64_t)w.y << 32) | w.x);
        y = __builtin_bit_cast(double, ((uint64_t)w.w << 32) | w.z);
    }
    __device__ static __forceinline__ void st(const BufAccess<double> &a, int64_t e, uint32_t v,
                                              double x, double y) {
        const uint64_t bx = __builtin_bit_cast(uint64_t, x), by = __builtin_bit_cast(uint64_t, y);
        W w;
        w.x = (uint32_t)bx;
        w.y = (uint32_t)(bx >> 32);
        w.z = (uint32_t)by;
        w.w = (uint32_t)(by >> 32);
        __builtin_amdgcn_raw_buffer_store_b128(w, a.r, v, (uint32_t)(e * 8), TRT_STORE_CPOL);
    }
};

// Raw populations of one row of a lane's pair, plus the lane's edge elements
// (lanes 0 and 63 only), its halo node (for the halo Phi_x) and, with a link
// map, the pair's link codes (node A in the low half, node B in the high one).
template <class T> struct PairRow {
    typename PairIO<T>::W w[9];
    typename PairIO<T>::W own[9];  // own slots opp(i) of bounce-back directions
    T edge[3];
    Raw<T> halo;
    uint32_t lk;
    uint32_t rs;  // the row's link summary for this strip (wave-uniform)
};

// Where a lane's pair lives and how to reach its own slots.
template <class T> struct PairCtx {
    const BufAccess<T> &in;
    int64_t plane;
    int pitch, ny;
    uint32_t opair;        // byte offset of the pair's first column
    uint32_t ca;           // the pair's first column
    bool edge;
    const uint32_t *ve;    // edge elements: plane and column per edge lane
    const Column &hcol;    // the edge lane's halo column
    const LinkAccess &la;  // link map (used when `linked`)
    bool linked;
    int64_t lpitch;
    uint32_t edge_shift;   // 16 where an edge element feeds a node A (FP16 words)
    bool tail;             // holds an odd width's last column as its node A
};

// The link codes of row y: the pair's (ld2) and the edge lane's halo node.
template <class T>
__device__ __forceinline__ void pair_codes(const PairCtx<T> &c, int y, uint32_t rs, uint32_t &lk,
                                           uint32_t &hlk) {
    lk = hlk = 0u;
    if (c.linked && rs != 0u) {
        const uint32_t ro = (uint32_t)((int64_t)y * c.lpitch);
        lk = c.la.ld2(ro, c.ca);
        if (c.edge) hlk = c.la.ld1(ro, (uint32_t)c.hcol.xc);
    }
}

// Gather one row of a lane's pair.  The link codes lk (pair) and hlk (halo
// node) of the row are already known (read one row ahead), so the own-slot
// loads of bounce-back directions are issued together with the pulls.
template <class T, bool HALO>
__device__ __forceinline__ void gather_pair_row(PairRow<T> &r, const PairCtx<T> &c, int y,
                                                uint32_t rs) {
    // the row's link codes are loaded with its populations, straight into the
    // row (rows whose summary is 0 load none): they are needed only where the
    // populations are, so they add no earlier wait
    uint32_t lk, hlk;
    pair_codes(c, y, rs, lk, hlk);
    const int ym = (y == 0) ? c.ny - 1 : y - 1;
    const int yp = (y == c.ny - 1) ? 0 : y + 1;
    const int64_t e0 = (int64_t)y * c.pitch, em = (int64_t)ym * c.pitch,
                  ep = (int64_t)yp * c.pitch;
    const int64_t plane = c.plane;
    r.lk = lk;
    r.rs = rs;
    r.w[0] = PairIO<T>::ld(c.in, e0, c.opair);
    r.w[1] = PairIO<T>::ld(c.in, plane + e0, c.opair);
    r.w[2] = PairIO<T>::ld(c.in, 2 * plane + em, c.opair);
    r.w[3] = PairIO<T>::ld(c.in, 3 * plane + e0, c.opair);
    r.w[4] = PairIO<T>::ld(c.in, 4 * plane + ep, c.opair);
    r.w[5] = PairIO<T>::ld(c.in, 5 * plane + em, c.opair);
    r.w[6] = PairIO<T>::ld(c.in, 6 * plane + em, c.opair);
    r.w[7] = PairIO<T>::ld(c.in, 7 * plane + ep, c.opair);
    r.w[8] = PairIO<T>::ld(c.in, 8 * plane + ep, c.opair);
    if (c.linked && (rs & 0xfffeu) != 0u) {
#pragma unroll
        for (int i = 1; i < 9; ++i)
            if ((rs >> i) & 1u) r.own[i] = PairIO<T>::ld(c.in, kOppDir[i] * plane + e0, c.opair);
    }
    r.edge[0] = r.edge[1] = r.edge[2] = T(0);
    if (c.edge) {
        // lane 0: planes 1, 5, 8 at column x0 - 1; lane 63: planes 3, 6, 7 at
        // column x0 + 128 (ve[] carries the plane and column per lane)
        r.edge[0] = c.in.ld(e0, c.ve[0]);
        r.edge[1] = c.in.ld(em, c.ve[1]);
        r.edge[2] = c.in.ld(ep, c.ve[2]);
        if (HALO) gather_raw<T>(r.halo, c.in, plane, c.pitch, c.ny, y, c.hcol, c.linked, hlk, rs);
    }
}

// Widen a pair row into the two nodes' populations, streaming in x through
// the lane neighbours, apply the link bits (half-way bounce-back from the
// nodes' own slots, solid nodes) and the open x boundaries, and form both
// nodes' moments and Phi.
// HALVES (FP16 storage without a link map or open boundaries): the words are
// shifted across lanes whole and the moments summed from their FP16 halves.
// WALLS (passes of several steps over whole-row walls, row flags in r.rs as
// set by tb2_gather): populations bounced at a solid row below or above
// were loaded from the node's own slots and take no shift in x.
template <class T, class C, bool SHIFTED, bool HALVES = false, bool WALLS = false>
__device__ __forceinline__ void widen_pair(RowState<C, SHIFTED> &a, RowState<C, SHIFTED> &b,
                                           const PairRow<T> &r, const PairCtx<T> &c, C gx, C gy,
                                           const OpenX<C> &ox) {
    if constexpr (HALVES) {
        static_assert(sizeof(T) == 2 && sizeof(C) == 4, "FP16 storage only");
        // edge elements as words: lane 0 (and an odd width's last lane)
        // feeds node A's high half (a previous lane's node B, or column 0),
        // lane 63 node B's low half (a next lane's node A); pinned here as
        // the FP16 path pins its conversions
        T e0 = r.edge[0], e1 = r.edge[1], e2 = r.edge[2];
        asm volatile("" : "+v"(e0), "+v"(e1), "+v"(e2));
        const uint32_t sh = c.edge_shift;
        const uint32_t h0 = (uint32_t)__builtin_bit_cast(unsigned short, e0) << sh;
        const uint32_t h1 = (uint32_t)__builtin_bit_cast(unsigned short, e1) << sh;
        const uint32_t h2 = (uint32_t)__builtin_bit_cast(unsigned short, e2) << sh;
        // e_x = +1 (planes 1, 5, 8): node A pulls the previous lane's node B;
        // e_x = -1 (planes 3, 6, 7): node B pulls the next lane's node A
        const uint32_t w1 = dpp_shr(h0, r.w[1]), w5 = dpp_shr(h1, r.w[5]), w8 = dpp_shr(h2, r.w[8]);
        const uint32_t w3 = dpp_shl(h0, r.w[3]), w6 = dpp_shl(h1, r.w[6]), w7 = dpp_shl(h2, r.w[7]);
        if constexpr (WALLS) {
            // as below, but where a wall row below (5, 6) or above (7, 8)
            // bounces a population, each node takes its own half of the
            // own-slot word its load brought, moved to the half its sums read
            uint32_t a5 = w5, a6 = c.tail ? h1 : r.w[6], a7 = c.tail ? h2 : r.w[7], a8 = w8;
            uint32_t b5 = r.w[5], b6 = w6, b7 = w7, b8 = r.w[8];
            if (r.rs & 2u) {
                a5 = r.w[5] << 16;
                a6 = r.w[6] << 16;
                b5 = r.w[5] >> 16;
                b6 = r.w[6] >> 16;
            }
            if (r.rs & 4u) {
                a7 = r.w[7] << 16;
                a8 = r.w[8] << 16;
                b7 = r.w[7] >> 16;
                b8 = r.w[8] >> 16;
            }
            {
                const uint32_t o3 = c.tail ? h0 : r.w[3];
                const float a13 = hsum<true, false>(w1, o3);
                a.m.finish(hsum<true, false>(a5, a6), hsum<true, true>(a5, a6),
                           hsum<true, false>(a7, a8), hsum<true, true>(a7, a8), a13,
                           hsum<true, true>(w1, o3), hsum<false, false>(r.w[2], r.w[4]),
                           hsum<false, true>(r.w[2], r.w[4]), hadd<false>(r.w[0], a13), gx, gy);
            }
            {
                const float a13 = hsum<false, false>(r.w[1], w3);
                b.m.finish(hsum<false, false>(b5, b6), hsum<false, true>(b5, b6),
                           hsum<false, false>(b7, b8), hsum<false, true>(b7, b8), a13,
                           hsum<false, true>(r.w[1], w3), hsum<true, false>(r.w[2], r.w[4]),
                           hsum<true, true>(r.w[2], r.w[4]), hadd<true>(r.w[0], a13), gx, gy);
            }
            a.solid = b.solid = (r.rs & 1u) != 0;
            const float pxa = a.m.rho * a.m.ux * a.m.ux * a.m.ux;
            const float pya = a.m.rho * a.m.uy * a.m.uy * a.m.uy;
            const float pxb = b.m.rho * b.m.ux * b.m.ux * b.m.ux;
            const float pyb = b.m.rho * b.m.uy * b.m.uy * b.m.uy;
            a.phix = a.solid ? 0.0f : pxa;
            a.phiy = a.solid ? 0.0f : pya;
            b.phix = b.solid ? 0.0f : pxb;
            b.phiy = b.solid ? 0.0f : pyb;
            return;
        }
        // node A: f0 f2 f4 in the low halves of its own words; f1 f5 f8 in
        // the high halves of the shifted ones; f3 f6 f7 in the high halves of
        // its own (node B's column), or of the edge words for an odd width's
        // last column
        {
            const uint32_t o3 = c.tail ? h0 : r.w[3], o6 = c.tail ? h1 : r.w[6],
                           o7 = c.tail ? h2 : r.w[7];
            const float a13 = hsum<true, false>(w1, o3);
            a.m.finish(hsum<true, false>(w5, o6), hsum<true, true>(w5, o6),
                       hsum<true, false>(o7, w8), hsum<true, true>(o7, w8), a13,
                       hsum<true, true>(w1, o3), hsum<false, false>(r.w[2], r.w[4]),
                       hsum<false, true>(r.w[2], r.w[4]), hadd<false>(r.w[0], a13), gx, gy);
        }
        // node B: f0 f2 f4 in the high halves of its own words; f1 f5 f8 in
        // the low halves of its own (node A's column); f3 f6 f7 in the low
        // halves of the shifted ones
        {
            const float a13 = hsum<false, false>(r.w[1], w3);
            b.m.finish(hsum<false, false>(r.w[5], w6), hsum<false, true>(r.w[5], w6),
                       hsum<false, false>(w7, r.w[8]), hsum<false, true>(w7, r.w[8]), a13,
                       hsum<false, true>(r.w[1], w3), hsum<true, false>(r.w[2], r.w[4]),
                       hsum<true, true>(r.w[2], r.w[4]), hadd<true>(r.w[0], a13), gx, gy);
        }
        a.solid = b.solid = false;
        a.phix = a.m.rho * a.m.ux * a.m.ux * a.m.ux;
        a.phiy = a.m.rho * a.m.uy * a.m.uy * a.m.uy;
        b.phix = b.m.rho * b.m.ux * b.m.ux * b.m.ux;
        b.phiy = b.m.rho * b.m.uy * b.m.uy * b.m.uy;
        return;
    }
    C pa[9], pb[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) PairIO<T>::split(r.w[i], pa[i], pb[i]);
    // the edge elements are converted here, once the row is needed: left to
    // itself the compiler moves an FP16 conversion into the edge lanes' load
    // branch, and its wait for the element (memory operations complete in
    // issue order) then waits for the whole row before the previous row's
    // coefficients are formed
    T e0 = r.edge[0], e1 = r.edge[1], e2 = r.edge[2];
    asm volatile("" : "+v"(e0), "+v"(e1), "+v"(e2));
    const C h0 = to_c(e0), h1 = to_c(e1), h2 = to_c(e2);
    C fa[9], fb[9];
    fa[0] = pa[0]; fb[0] = pb[0];
    fa[2] = pa[2]; fb[2] = pb[2];
    fa[4] = pa[4]; fb[4] = pb[4];
    // e_x = +1: node A pulls from the previous lane's B (lane 0: edge element)
    fa[1] = dpp_shr(h0, pb[1]); fb[1] = pa[1];
    fa[5] = dpp_shr(h1, pb[5]); fb[5] = pa[5];
    fa[8] = dpp_shr(h2, pb[8]); fb[8] = pa[8];
    // e_x = -1: node B pulls from the next lane's A (lane 63: edge element);
    // node A from its own B, or, at an odd width's last column, from the
    // edge elements of column 0
    fa[3] = c.tail ? h0 : pb[3]; fb[3] = dpp_shl(h0, pa[3]);
    fa[6] = c.tail ? h1 : pb[6]; fb[6] = dpp_shl(h1, pa[6]);
    fa[7] = c.tail ? h2 : pb[7]; fb[7] = dpp_shl(h2, pa[7]);
    a.solid = b.solid = false;
    if constexpr (WALLS) {
        if (r.rs & 2u) {
            fa[5] = pa[5]; fb[5] = pb[5];
            fa[6] = pa[6]; fb[6] = pb[6];
        }
        if (r.rs & 4u) {
            fa[7] = pa[7]; fb[7] = pb[7];
            fa[8] = pa[8]; fb[8] = pb[8];
        }
        a.solid = b.solid = (r.rs & 1u) != 0;
    }
    if (c.linked && r.rs != 0u) {
        // only rows that touch a wall or an obstacle pay for the link codes
        const uint32_t la_ = r.lk & 0xffffu, lb_ = r.lk >> 16;
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            if ((r.rs >> i) & 1u) {
                // used here, after the row's wait: left free, the compiler
                // merges this select into the load's branch (same condition)
                // and waits for the row there
                typename PairIO<T>::W o = r.own[i];
                asm volatile("" : "+v"(o));
                C oa, ob;
                PairIO<T>::split(o, oa, ob);
                fa[i] = ((la_ >> i) & 1u) ? oa : fa[i];
                fb[i] = ((lb_ >> i) & 1u) ? ob : fb[i];
            }
        }
        a.solid = (la_ & 1u) != 0;
        b.solid = (lb_ & 1u) != 0;
    }
    if (ox.on) {
        open_x_fix<C, SHIFTED>(fa, (int)c.ca, ox.nx, ox.u_in, ox.rho_in, ox.rho_out);
        open_x_fix<C, SHIFTED>(fb, (int)c.ca + 1, ox.nx, ox.u_in, ox.rho_in, ox.rho_out);
    }
    a.m.compute(fa, gx, gy);
    b.m.compute(fb, gx, gy);
    const C pxa = a.m.rho * a.m.ux * a.m.ux * a.m.ux;
    const C pya = a.m.rho * a.m.uy * a.m.uy * a.m.uy;
    const C pxb = b.m.rho * b.m.ux * b.m.ux * b.m.ux;
    const C pyb = b.m.rho * b.m.uy * b.m.uy * b.m.uy;
    a.phix = a.solid ? C(0) : pxa;
    a.phiy = a.solid ? C(0) : pya;
    b.phix = b.solid ? C(0) : pxb;
    b.phiy = b.solid ? C(0) : pyb;
}

// Halo Phi_x of an edge lane (the link bits and open boundaries applied as
// for the node's own lane).
template <class T, class C, bool SHIFTED, bool HALVES>
__device__ __forceinline__ C pair_halo_phix(Raw<T> &h, const PairCtx<T> &c, C gx,
                                            const OpenX<C> &ox) {
    if constexpr (HALVES) {
        // halo_phix's operations, summed from the FP16 values directly
        const _Float16 *v = h.v;
        const float s56 = hsum<false, false>(v[5], v[6]), s78 = hsum<false, false>(v[7], v[8]);
        const float d56 = hsum<false, true>(v[5], v[6]), d78 = hsum<false, true>(v[7], v[8]);
        const float diag = s56 + s78;
        const float qxyy = d56 - d78;
        const float a13 = hsum<false, false>(v[1], v[3]), a24 = hsum<false, false>(v[2], v[4]);
        const float jx = hsum<false, true>(v[1], v[3]) + qxyy;
        const float base = hadd<false>(v[0], a13) + (a24 + diag);
        const float rho = 1.0f + base;
        const float ux = jx * recip(rho) + 0.5f * gx;
        return rho * ux * ux * ux;
    } else {
        if (c.linked) link_fix(h);
        return halo_phix<T, C, SHIFTED>(h, gx, ox, c.hcol.xc);
    }
}

// LINKED: the lattice may have obstacles or open x boundaries (link map);
// without it the link code is compiled out.
template <int ST, bool SYNC, bool LINKED>
__device__ __forceinline__ void sweep_strip2(const InstDesc &d, int strip, int rb, int srcsel) {
    using T = typename Store<ST>::T;
    using C = typename Store<ST>::C;
    constexpr bool SH = Store<ST>::shifted;
    // FP16 without a link map: moments straight from the stored halves
    constexpr bool HALVES = ST == ST_F16 && !LINKED;

    const int lane = threadIdx.x & 63;
    const int nx = d.nx, ny = d.ny, pitch = d.pitch;
    const int64_t plane = d.plane;
    const T *__restrict__ src = static_cast<const T *>(srcsel ? d.buf[1] : d.buf[0]);
    T *__restrict__ dst = static_cast<T *>(srcsel ? d.buf[0] : d.buf[1]);
    const uint64_t bytes = (uint64_t)ny * (uint64_t)pitch * sizeof(T);
    const BufAccess<T> in(src, bytes), out(dst, bytes);
    const LinkAccess lacc(d.links, (uint64_t)ny * (uint64_t)d.lpitch);
    const bool linked = LINKED && d.links != nullptr;

    const int x0 = strip * kStripWidth2;
    const int c2 = x0 + 2 * lane;
    // lanes past the last column hold a wrapped, even column (with an even
    // width exactly the columns that follow the seam, so the lane shifts
    // also carry the periodic wrap)
    const int ca = c2 < nx ? c2 : (c2 % nx) & ~1;
    const bool writer = c2 < nx;
    // odd width: the lane holding the last column nx - 1 (as its node A;
    // its node B lies in the row padding) takes that column's x + 1
    // neighbour, column 0, as a right edge lane does
    const bool tail = (nx & 1) && c2 == nx - 1;
    const bool edge = lane == 0 || lane == 63 || tail;
    const Column hcol = column_of(lane == 0 ? x0 - 1 : (tail ? nx : x0 + kStripWidth2), nx, sizeof(T));
    const int pe0 = lane == 0 ? 1 : 3, pe1 = lane == 0 ? 5 : 6, pe2 = lane == 0 ? 8 : 7;
    const uint32_t ve[3] = {(uint32_t)(pe0 * plane * (int64_t)sizeof(T)) + hcol.oc,
                            (uint32_t)(pe1 * plane * (int64_t)sizeof(T)) + hcol.oc,
                            (uint32_t)(pe2 * plane * (int64_t)sizeof(T)) + hcol.oc};
    const PairCtx<T> cx{in, plane, pitch, ny, (uint32_t)ca * (uint32_t)sizeof(T), (uint32_t)ca,
                        edge, ve, hcol, lacc, linked, d.lpitch,
                        (lane == 0 || tail) ? 16u : 0u, tail};

    const C gx = (C)d.gx, gy = (C)d.gy;
    const C w1 = (C)d.omega1, w2 = (C)d.omega2, ph = (C)d.phi;
    OpenX<C> ox;
    ox.on = LINKED && d.xbc != 0;
    ox.nx = nx;
    ox.u_in = (C)d.u_in;
    ox.rho_in = (C)d.rho_in;
    ox.rho_out = (C)d.rho_out;
    ox.phi_wall = ox.rho_in * ox.u_in * ox.u_in * ox.u_in;
    const int y0 = rb * d.rows;
    const int y1 = min(y0 + d.rows, ny);

    // the strip's link summary of a row (scalar; 0: no link step)
    const RowSum rsum(d.rowsum, d.nsum);
    const auto summary = [&](int row) -> uint32_t { return linked ? rsum.two(row, strip) : 0u; };

    C phiy_below_a, phiy_below_b;
    {
        PairRow<T> t;
        RowState<C, SH> a, b;
        const int ym0 = (y0 + ny - 1) % ny;
        gather_pair_row<T, false>(t, cx, ym0, summary(ym0));
        widen_pair<T, C, SH, HALVES>(a, b, t, cx, gx, gy, ox);
        phiy_below_a = a.phiy;
        phiy_below_b = b.phiy;
    }
    RowState<C, SH> ca_, cb_;
    C hphix = C(0);
    {
        PairRow<T> t;
        gather_pair_row<T, true>(t, cx, y0, summary(y0));
        widen_pair<T, C, SH, HALVES>(ca_, cb_, t, cx, gx, gy, ox);
        if (edge) hphix = pair_halo_phix<T, C, SH, HALVES>(t.halo, cx, gx, ox);
    }
    // link summaries are read one row ahead of the gather they gate
    uint32_t rs_next = summary((y0 + 1) % ny);

    for (int y = y0; y < y1; ++y) {
        const int yn = (y + 1 == ny) ? 0 : y + 1;
        PairRow<T> nr;
        gather_pair_row<T, true>(nr, cx, yn, rs_next);
        rs_next = summary((yn + 1 == ny) ? 0 : yn + 1);

        // row y: both nodes' coefficients except the y-gradient of Phi
        C left = dpp_shr(hphix, cb_.phix);   // x - 1 of node A
        C right = dpp_shl(hphix, ca_.phix);  // x + 1 of node B
        C right_a = tail ? hphix : cb_.phix;  // x + 1 of node A
        if (ox.on) {
            // Phi beyond the inflow wall is the wall's; beyond the outlet, the last column's
            if (ca == 0) left = ox.phi_wall;
            if (ca + 1 == nx - 1) right = cb_.phix;
            if (ca == nx - 1) right_a = ca_.phix;
        }
        const C dpx_a = C(0.5) * (right_a - left);
        const C dpx_b = C(0.5) * (right - ca_.phix);
        Coeffs<C> fa = collide_coeffs<C, SH>(ca_.m, dpx_a, w1, w2, ph, gx, gy);
        Coeffs<C> fb = collide_coeffs<C, SH>(cb_.m, dpx_b, w1, w2, ph, gx, gy);
        asm volatile("" : "+v"(fa.base), "+v"(fa.bx), "+v"(fa.by), "+v"(fa.bxx), "+v"(fa.byy),
                     "+v"(fa.bxy), "+v"(fa.bxxy), "+v"(fa.bxyy));
        asm volatile("" : "+v"(fb.base), "+v"(fb.bx), "+v"(fb.by), "+v"(fb.bxx), "+v"(fb.byy),
                     "+v"(fb.bxy), "+v"(fb.bxxy), "+v"(fb.bxyy));

        RowState<C, SH> na, nb;
        widen_pair<T, C, SH, HALVES>(na, nb, nr, cx, gx, gy, ox);
        C nhphix = C(0);
        if (edge) nhphix = pair_halo_phix<T, C, SH, HALVES>(nr.halo, cx, gx, ox);

        // the same operations per node as the one-column sweep
        const C dphiy_a = C(0.5) * (na.phiy - phiy_below_a);
        const C dphiy_b = C(0.5) * (nb.phiy - phiy_below_b);
        if constexpr (ST == ST_F16) {
            // each store word: node A's population in the low half, node B's
            // in the high one, each rounded once
            HalfPairs pa, pb;
            reconstruct_pairs(pa, fa.base, fa.bx, fa.by, fa.bxx, fa.byy - ph * dphiy_a, fa.bxy,
                              fa.bxxy, fa.bxyy);
            reconstruct_pairs(pb, fb.base, fb.bx, fb.by, fb.bxx, fb.byy - ph * dphiy_b, fb.bxy,
                              fb.bxxy, fb.bxyy);
            uint32_t wd[9];
            wd[0] = half_out<0, true>(pb, half_out<0, false>(pa));
            wd[1] = half_out<1, true>(pb, half_out<1, false>(pa));
            wd[2] = half_out<2, true>(pb, half_out<2, false>(pa));
            wd[3] = half_out<3, true>(pb, half_out<3, false>(pa));
            wd[4] = half_out<4, true>(pb, half_out<4, false>(pa));
            wd[5] = half_out<5, true>(pb, half_out<5, false>(pa));
            wd[6] = half_out<6, true>(pb, half_out<6, false>(pa));
            wd[7] = half_out<7, true>(pb, half_out<7, false>(pa));
            wd[8] = half_out<8, true>(pb, half_out<8, false>(pa));
            if (LINKED && __builtin_amdgcn_ballot_w64(ca_.solid || cb_.solid) != 0) {
                // solid nodes keep zeros (their slots are never read)
                const uint32_t keep = (ca_.solid ? 0u : 0x0000ffffu) | (cb_.solid ? 0u : 0xffff0000u);
#pragma unroll
                for (int i = 0; i < 9; ++i) wd[i] &= keep;
            }
            if (writer) {
                const int64_t e0 = (int64_t)y * pitch;
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    __builtin_amdgcn_raw_buffer_store_b32(wd[i], out.r, cx.opair,
                                                          (uint32_t)((i * plane + e0) * 2),
                                                          TRT_STORE_CPOL);
            }
        } else {
            C oa[9], ob[9];
            reconstruct<C>(oa, fa.base, fa.bx, fa.by, fa.bxx, fa.byy - ph * dphiy_a, fa.bxy,
                           fa.bxxy, fa.bxyy);
            reconstruct<C>(ob, fb.base, fb.bx, fb.by, fb.bxx, fb.byy - ph * dphiy_b, fb.bxy,
                           fb.bxxy, fb.bxyy);
            if (LINKED && __builtin_amdgcn_ballot_w64(ca_.solid || cb_.solid) != 0) {
                // solid nodes keep zeros (their slots are never read)
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    oa[i] = ca_.solid ? C(0) : oa[i];
                    ob[i] = cb_.solid ? C(0) : ob[i];
                }
            }
            if (writer) {
                const int64_t e0 = (int64_t)y * pitch;
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    PairIO<T>::st(out, i * plane + e0, cx.opair, oa[i], ob[i]);
            }
        }
        phiy_below_a = ca_.phiy;
        phiy_below_b = cb_.phiy;
        ca_ = na;
        cb_ = nb;
        hphix = nhphix;
        // keep the workgroup's wavefronts (adjacent strips) on the same row, so
        // that their accesses to each population row stay contiguous in time
        if (SYNC) __builtin_amdgcn_s_barrier();
    }
}

// ---------------------------------------------------------------------------
// Two time steps per pass (FP32 or FP16 storage, open periodic lattices).
//
// One launch advances the lattice by two time steps and moves each
// population through HBM once.  A wavefront owns a 128-column window (lane
// l: the column pair s + 2l, s + 2l + 1, wrapped) and marches it through a
// row block as a pipeline; in pipeline row y it
//   (a) issues the loads of a later row of the stored state (the pull of the
//       first step, as in the one-step sweep),
//   (b) forms the moments, Phi and collision coefficients of row y + 3
//       (first step) from a row loaded earlier,
//   (c) collides row y + 2 (first step): its post-collision populations stay
//       in registers,
//   (d) pulls row y + 1 of the second step from the first step's results of
//       rows y, y + 1 and y + 2 (populations 2, 5, 6 from the row below,
//       0, 1, 3 from the row itself, 4, 7, 8 from the row above; neighbours
//       in x through DPP lane shifts) and forms its moments, Phi and
//       coefficients,
//   (e) collides row y (second step) and stores it.
// Each stage's stencil reaches one column further than the last (the first
// step's pull, its Phi gradient, the second step's pull, its Phi gradient),
// so a window edge spoils one column per stage; the wavefront stores only
// the window's middle 120 columns [s + 4, s + 124), and windows overlap by
// eight columns.  Every lane runs the same code: no halo loads and no edge
// lane work (odd widths: see Tb2Lane) (a first design ran the first step on the two columns beyond a
// 128-column strip in its edge lanes, and the other 62 lanes' issue slots
// paid for it: 153 against 127 us per step on 4096^2).  A row block of R
// rows runs R + 6 pipeline rows and reads R + 6 rows of each population.
// Every node's arithmetic is the one-step sweep's, operation for operation,
// and the first step's results are exactly what that sweep would store and
// load back (FP16: rounded to the stored words in registers), so two steps
// per pass reproduce its bits.

// The first step's post-collision populations of one node between the
// iteration that makes them and the two iterations that pull them.  UP (the
// march goes up, rows y, y + 1, ...): lo holds row y's populations 2, 5, 6
// (they stream up), mid row y + 1's 0, 1, 3 and 2, 5, 6; down the march the
// roles of 2, 5, 6 and 4, 7, 8 swap.
template <class C> struct MidWindow {
    C lo[3];   // two rows behind the fresh row: the populations streaming forward
    C mid[6];  // one row behind: populations 0, 1, 3 and those streaming forward
};

// WALLS, solid_mid: the row leaving the middle is a solid row, so the new
// middle row's pull bounces the populations it would take from it; lo then
// keeps the new middle row's own populations that come back (4, 7, 8 up the
// march, 2, 5, 6 down it) in the slots of those they replace.
template <class C, bool UP = true, bool WALLS = false>
__device__ __forceinline__ void mid_shift(MidWindow<C> &w, const C f[9], bool solid_mid = false) {
    w.lo[0] = w.mid[3];
    w.lo[1] = w.mid[4];
    w.lo[2] = w.mid[5];
    if constexpr (WALLS) {
        w.lo[0] = solid_mid ? f[UP ? 4 : 2] : w.lo[0];
        w.lo[1] = solid_mid ? f[UP ? 7 : 5] : w.lo[1];
        w.lo[2] = solid_mid ? f[UP ? 8 : 6] : w.lo[2];
    }
    w.mid[0] = f[0];
    w.mid[1] = f[1];
    w.mid[2] = f[3];
    w.mid[3] = f[UP ? 2 : 4];
    w.mid[4] = f[UP ? 5 : 7];
    w.mid[5] = f[UP ? 6 : 8];
}

// Pre-collision populations (second step) of a node in the row between its
// window's rows and the freshly collided row, from its own window and fresh
// row (s, sf) and those of its left (x - 1: l, lf) and right (x + 1: r, rf)
// neighbours: 0, 1, 3 from the middle row, the populations streaming
// forward from the row behind, the others from the fresh row ahead.
// WALLS: behind (ahead) the row behind (ahead) is solid, and the populations
// it would give come back from the node's own slots (half-way bounce-back):
// those of the row ahead from the node's window (mid[3..5]), those of the
// row behind from lo (kept there by mid_shift), with no shift in x.
template <class C, bool UP = true, bool WALLS = false>
__device__ __forceinline__ void mid_pull(C f[9], const MidWindow<C> &s, const C sf[9],
                                         const MidWindow<C> &l, const C lf[9],
                                         const MidWindow<C> &r, const C rf[9],
                                         bool behind = false, bool ahead = false) {
    f[0] = s.mid[0];
    f[1] = l.mid[1];
    f[3] = r.mid[2];
    if (UP) {
        f[2] = s.lo[0];
        f[5] = l.lo[1];
        f[6] = r.lo[2];
        f[4] = sf[4];
        f[7] = rf[7];
        f[8] = lf[8];
    } else {
        f[4] = s.lo[0];
        f[7] = r.lo[1];
        f[8] = l.lo[2];
        f[2] = sf[2];
        f[5] = lf[5];
        f[6] = rf[6];
    }
    if constexpr (WALLS) {
        if (UP) {
            f[5] = behind ? s.lo[1] : f[5];
            f[6] = behind ? s.lo[2] : f[6];
            f[4] = ahead ? s.mid[3] : f[4];
            f[7] = ahead ? s.mid[4] : f[7];
            f[8] = ahead ? s.mid[5] : f[8];
        } else {
            f[7] = behind ? s.lo[1] : f[7];
            f[8] = behind ? s.lo[2] : f[8];
            f[2] = ahead ? s.mid[3] : f[2];
            f[5] = ahead ? s.mid[4] : f[5];
            f[6] = ahead ? s.mid[5] : f[6];
        }
    }
}

// Moments, Phi_x and Phi_y of one node from its populations, as widen()
// (Phi 0 at a solid node).
template <class C, bool SHIFTED>
__device__ __forceinline__ void node_state(RowState<C, SHIFTED> &st, const C f[9], C gx, C gy,
                                           bool solid = false) {
    st.solid = solid;
    st.m.compute(f, gx, gy);
    const C px = st.m.rho * st.m.ux * st.m.ux * st.m.ux;
    const C py = st.m.rho * st.m.uy * st.m.uy * st.m.uy;
    st.phix = solid ? C(0) : px;
    st.phiy = solid ? C(0) : py;
}

// A lane's pair in a window: the columns ca (node A) and cb (node B, the
// next column, wrapped).  With an odd width a pair can start on an odd
// column or straddle the wrap (nx - 1, 0); such a lane ("split") loads its
// two elements one by one into the word a paired load would give.  Its
// paired load, issued by every lane, goes to the aligned pair below ca (or
// to (nx - 1, padding): an odd width always leaves row padding, which
// nothing reads as data), and its store too, which only a stored lane
// issues (a stored pair starts on an even column inside the lattice, so it
// is split only at (nx - 1, padding)).
struct Tb2Lane {
    bool split;
    uint32_t oa, ob;  // byte offsets of columns ca and cb within a row
};

template <class T> struct Tb2Word;
template <> struct Tb2Word<float> {
    __device__ static __forceinline__ u32x2 get(const BufAccess<float> &in, int64_t e,
                                                const Tb2Lane &ln) {
        u32x2 w;
        w.x = __builtin_bit_cast(uint32_t, in.ld(e, ln.oa));
        w.y = __builtin_bit_cast(uint32_t, in.ld(e, ln.ob));
        return w;
    }
};
template <> struct Tb2Word<_Float16> {
    __device__ static __forceinline__ uint32_t get(const BufAccess<_Float16> &in, int64_t e,
                                                   const Tb2Lane &ln) {
        const uint32_t lo = __builtin_bit_cast(unsigned short, in.ld(e, ln.oa));
        const uint32_t hi = __builtin_bit_cast(unsigned short, in.ld(e, ln.ob));
        return lo | (hi << 16);
    }
};

// Walls that fill whole rows (InstDesc::rowwalls): every node of a row has
// the same link code, so the first link-summary entry of row y holds its
// state -- bit 0: the row is solid, bit 2: its pull source for direction 2,
// row y - 1 (wrapped), is; bit 4: row y + 1 is (one scalar load).
struct RowWalls {
    RowSum sum;
    __device__ __forceinline__ explicit RowWalls(const InstDesc &d) : sum(d.rowsum, d.nsum) {}
    // the pull flags of row y (0 <= y < ny): bit 0 the row is solid, bit 1
    // the row below it, bit 2 the row above it
    __device__ __forceinline__ uint32_t flags(int y) const { return of_entry(sum.one(y, 0)); }
    // the same from the row's summary entry
    __device__ static __forceinline__ uint32_t of_entry(uint32_t e) {
        return (e & 1u) | (((e >> 2) & 1u) << 1) | (((e >> 4) & 1u) << 2);
    }
};

// The wall flags (RowWalls::flags) of the rows a pass loads, which follow
// one another in the march's order: the flags of the next row to load are
// kept, and those of the row after it are read one load ahead, so the
// scalar load's wait falls a pipeline row after its issue.
template <bool UP, bool WALLS> struct LoadWalls {
    int row = 0;        // the row after the next one to load
    uint32_t next = 0;  // the next row to load's summary entry, as loaded
    // first: the first row to load (any integer)
    __device__ __forceinline__ LoadWalls(const InstDesc &d, int first) {
        if constexpr (WALLS) {
            int r = first < 0 ? first + d.ny : (first >= d.ny ? first - d.ny : first);
            if (r < 0 || r >= d.ny) r = ((first % d.ny) + d.ny) % d.ny;
            next = RowWalls(d).sum.one(r, 0);
            row = step(r, d.ny);
        }
    }
    // row + dir, wrapped
    __device__ static __forceinline__ int step(int r, int ny) {
        r += UP ? 1 : -1;
        return r == ny ? 0 : (r < 0 ? ny - 1 : r);
    }
    // the flags of the next row to load; then moves on by one row
    __device__ __forceinline__ uint32_t take(const InstDesc &d) {
        if constexpr (!WALLS) {
            return 0u;
        } else {
            const uint32_t f = RowWalls::of_entry(next);
            next = RowWalls(d).sum.one(row, 0);
            row = step(row, d.ny);
            return f;
        }
    }
};

// One row of a lane's pair for the pull (as gather_pair_row), split lanes
// element by element.  WALLS: wf holds the row's flags (RowWalls::flags,
// kept in r.rs); next to a solid row below, populations 2, 5, 6 come back
// from the node's own slots 4, 7, 8 (half-way bounce-back), next to one
// above 4, 7, 8 from 2, 5, 6, so those loads read the row itself.
template <class T, bool WALLS = false>
__device__ __forceinline__ void tb2_gather(PairRow<T> &r, const PairCtx<T> &c, const Tb2Lane &ln,
                                           bool odd, int y, uint32_t wf = 0u) {
    if constexpr (WALLS) {
        const int ym = (y == 0) ? c.ny - 1 : y - 1;
        const int yp = (y == c.ny - 1) ? 0 : y + 1;
        const int64_t e0 = (int64_t)y * c.pitch, em = (int64_t)ym * c.pitch,
                      ep = (int64_t)yp * c.pitch;
        const int64_t pl = c.plane;
        const bool below = (wf & 2u) != 0, above = (wf & 4u) != 0;
        const int64_t o[9] = {e0,
                              pl + e0,
                              below ? 4 * pl + e0 : 2 * pl + em,
                              3 * pl + e0,
                              above ? 2 * pl + e0 : 4 * pl + ep,
                              below ? 7 * pl + e0 : 5 * pl + em,
                              below ? 8 * pl + e0 : 6 * pl + em,
                              above ? 5 * pl + e0 : 7 * pl + ep,
                              above ? 6 * pl + e0 : 8 * pl + ep};
        r.lk = 0u;
        r.rs = wf;
#pragma unroll
        for (int i = 0; i < 9; ++i) r.w[i] = PairIO<T>::ld(c.in, o[i], c.opair);
        r.edge[0] = r.edge[1] = r.edge[2] = T(0);
        if (odd && ln.split) {
#pragma unroll
            for (int i = 0; i < 9; ++i) r.w[i] = Tb2Word<T>::get(c.in, o[i], ln);
        }
        return;
    }
    gather_pair_row<T, false>(r, c, y, 0u);
    if (odd && ln.split) {
        const int ym = (y == 0) ? c.ny - 1 : y - 1;
        const int yp = (y == c.ny - 1) ? 0 : y + 1;
        const int64_t e0 = (int64_t)y * c.pitch, em = (int64_t)ym * c.pitch,
                      ep = (int64_t)yp * c.pitch;
        const int64_t pl = c.plane;
        r.w[0] = Tb2Word<T>::get(c.in, e0, ln);
        r.w[1] = Tb2Word<T>::get(c.in, pl + e0, ln);
        r.w[2] = Tb2Word<T>::get(c.in, 2 * pl + em, ln);
        r.w[3] = Tb2Word<T>::get(c.in, 3 * pl + e0, ln);
        r.w[4] = Tb2Word<T>::get(c.in, 4 * pl + ep, ln);
        r.w[5] = Tb2Word<T>::get(c.in, 5 * pl + em, ln);
        r.w[6] = Tb2Word<T>::get(c.in, 6 * pl + em, ln);
        r.w[7] = Tb2Word<T>::get(c.in, 7 * pl + ep, ln);
        r.w[8] = Tb2Word<T>::get(c.in, 8 * pl + ep, ln);
    }
}

// The pull flags (pull_coeffs_pair) of the row at bit j of a pipeline's
// wall bits sb (bit j + 1 the row behind it in the march, bit j - 1 the row
// ahead).
__device__ __forceinline__ uint32_t wall_flags(uint32_t sb, int j) {
    return ((sb >> j) & 1u) | (((sb >> (j + 1)) & 1u) << 1) | (((sb >> (j - 1)) & 1u) << 2);
}

// A solid row keeps zeros (its slots are never read), as in the one-step
// sweep.
template <class C>
__device__ __forceinline__ void solid_zero(C a[9], C b[9], uint32_t solid) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        a[i] = solid ? C(0) : a[i];
        b[i] = solid ? C(0) : b[i];
    }
}

template <class C> struct Tb2Carry {
    Coeffs<C> kA, kB;     // first step: coefficients of the next row to collide
    C pyA, pyB;           // ... its Phi_y
    C belA, belB;         // ... and that of the row below it
    MidWindow<C> wA, wB;  // first-step results in flight
    Coeffs<C> qA, qB;     // second step: coefficients of the next row to store
    C qyA, qyB, qbelA, qbelB;
    uint32_t sb;          // whole-row walls: bit j, row y + (2 - j) dir solid
};

struct Tb2Params {
    float gx, gy, w1, w2, ph;
};

// The collision coefficients (all but the Phi_y gradient term) and Phi_y
// of a lane's pair in the row between the window (wA, wB) of a previous
// step's post-collision rows and that step's freshly collided row (oa, ob):
// the pull (x neighbours by DPP lane shifts), the moments and the Phi_x
// gradient, as the one-step sweep forms them.
// WALLS: wf bit 0 the row is solid, bit 1 the row behind it (in the
// march's order), bit 2 the row ahead.
template <class C, bool SH, bool UP, bool WALLS = false>
__device__ __forceinline__ void pull_coeffs_pair(Coeffs<C> &ckA, Coeffs<C> &ckB, C &cyA, C &cyB,
                                                 const MidWindow<C> &wA, const MidWindow<C> &wB,
                                                 const C oa[9], const C ob[9],
                                                 const Tb2Params &p, uint32_t wf = 0u) {
    const C gx = p.gx, gy = p.gy, w1 = p.w1, w2 = p.w2, ph = p.ph;
    C fa[9], fb[9];
    MidWindow<C> lw, rw;
    C lf[9], rf[9];
    // node A: x - 1 is the previous lane's node B (it gives 1 and the
    // x + 1 movers of the other two rows: 5 and 8)
    lw.mid[1] = dpp_shr(C(0), wB.mid[1]);
    if (UP) {
        lw.lo[1] = dpp_shr(C(0), wB.lo[1]);
        lf[8] = dpp_shr(C(0), ob[8]);
    } else {
        lw.lo[2] = dpp_shr(C(0), wB.lo[2]);
        lf[5] = dpp_shr(C(0), ob[5]);
    }
    const bool behind = (wf & 2u) != 0, ahead = (wf & 4u) != 0, solid = (wf & 1u) != 0;
    mid_pull<C, UP, WALLS>(fa, wA, oa, lw, lf, wB, ob, behind, ahead);
    // node B: x + 2 is the next lane's node A (3, 6 and 7)
    rw.mid[2] = dpp_shl(C(0), wA.mid[2]);
    if (UP) {
        rw.lo[2] = dpp_shl(C(0), wA.lo[2]);
        rf[7] = dpp_shl(C(0), oa[7]);
    } else {
        rw.lo[1] = dpp_shl(C(0), wA.lo[1]);
        rf[6] = dpp_shl(C(0), oa[6]);
    }
    mid_pull<C, UP, WALLS>(fb, wB, ob, wA, oa, rw, rf, behind, ahead);
    RowState<C, SH> cA, cB;
    node_state<C, SH>(cA, fa, gx, gy, WALLS && solid);
    node_state<C, SH>(cB, fb, gx, gy, WALLS && solid);
    const C left = dpp_shr(C(0), cB.phix);
    const C right = dpp_shl(C(0), cA.phix);
    ckA = collide_coeffs<C, SH>(cA.m, C(0.5) * (cB.phix - left), w1, w2, ph, gx, gy);
    ckB = collide_coeffs<C, SH>(cB.m, C(0.5) * (right - cA.phix), w1, w2, ph, gx, gy);
    cyA = cA.phiy;
    cyB = cB.phiy;
}

// One pipeline row: (b) the moments and coefficients of first-step row
// y + 3 from `raw`, whose registers then take the loads of row `yload`
// (when `load`), (c) from STAGE 1 the first-step collision of row y + 2,
// (d) from STAGE 2 the second-step pull of row y + 1 and its coefficients,
// (e) at STAGE 3 the second-step collision and store of row y.
// WALLS: whole-row walls; lflags are the flags of row yload (RowWalls).
template <int STAGE, class T, class C, bool SH, bool SYNC = true, bool UP = true,
          bool WALLS = false>
__device__ __forceinline__ void tb2_row(Tb2Carry<C> &k, PairRow<T> &raw, const PairCtx<T> &cx,
                                        const Tb2Lane &ln, bool odd, const Tb2Params &p,
                                        const BufAccess<T> &out, int y, bool load, int yload,
                                        bool store, int pitch, int64_t plane, int stage = STAGE,
                                        uint32_t lflags = 0u) {
    const C gx = p.gx, gy = p.gy, w1 = p.w1, w2 = p.w2, ph = p.ph;
    OpenX<C> ox;
    ox.on = false;
    ox.nx = 0;
    ox.u_in = ox.rho_in = ox.rho_out = ox.phi_wall = C(0);
    // (b) row y + 3, then (a) the next loads into the same registers
    C nyA, nyB;
    Coeffs<C> nkA, nkB;
    // whole-row walls: bit j, row y + (3 - j) dir solid
    const uint32_t sb = WALLS ? ((k.sb << 1) | (raw.rs & 1u)) : 0u;
    {
        RowState<C, SH> nA, nB;
        widen_pair<T, C, SH, false, WALLS>(nA, nB, raw, cx, gx, gy, ox);
        if (load) tb2_gather<T, WALLS>(raw, cx, ln, odd, yload, lflags);
        const C left = dpp_shr(C(0), nB.phix);
        const C right = dpp_shl(C(0), nA.phix);
        nkA = collide_coeffs<C, SH>(nA.m, C(0.5) * (nB.phix - left), w1, w2, ph, gx, gy);
        nkB = collide_coeffs<C, SH>(nB.m, C(0.5) * (right - nA.phix), w1, w2, ph, gx, gy);
        nyA = nA.phiy;
        nyB = nB.phiy;
    }
    // (c) collide row y + 2 of the first step
    C oa[9], ob[9];
    if (stage >= 1) {
        // the Phi_y gradient: the row above minus the row below
        const C dya = C(0.5) * (UP ? nyA - k.belA : k.belA - nyA);
        const C dyb = C(0.5) * (UP ? nyB - k.belB : k.belB - nyB);
        reconstruct<C>(oa, k.kA.base, k.kA.bx, k.kA.by, k.kA.bxx, k.kA.byy - ph * dya, k.kA.bxy,
                       k.kA.bxxy, k.kA.bxyy);
        reconstruct<C>(ob, k.kB.base, k.kB.bx, k.kB.by, k.kB.bxx, k.kB.byy - ph * dyb, k.kB.bxy,
                       k.kB.bxxy, k.kB.bxyy);
    }
    // (d) row y + 1 of the second step
    C cyA = C(0), cyB = C(0);
    Coeffs<C> ckA, ckB;
    if (stage >= 2)
        pull_coeffs_pair<C, SH, UP, WALLS>(ckA, ckB, cyA, cyB, k.wA, k.wB, oa, ob, p,
                                           wall_flags(sb, 2));
    // (e) collide row y of the second step and store the window's middle
    if (stage >= 3) {
        const C dya = C(0.5) * (UP ? cyA - k.qbelA : k.qbelA - cyA);
        const C dyb = C(0.5) * (UP ? cyB - k.qbelB : k.qbelB - cyB);
        C sa[9], sb_[9];
        reconstruct<C>(sa, k.qA.base, k.qA.bx, k.qA.by, k.qA.bxx, k.qA.byy - ph * dya, k.qA.bxy,
                       k.qA.bxxy, k.qA.bxyy);
        reconstruct<C>(sb_, k.qB.base, k.qB.bx, k.qB.by, k.qB.bxx, k.qB.byy - ph * dyb, k.qB.bxy,
                       k.qB.bxxy, k.qB.bxyy);
        if (WALLS) solid_zero<C>(sa, sb_, (sb >> 3) & 1u);
        if (store) {
            const int64_t e0 = (int64_t)y * pitch;
#pragma unroll
            for (int i = 0; i < 9; ++i) PairIO<T>::st(out, i * plane + e0, cx.opair, sa[i], sb_[i]);
        }
    }
    // advance the pipeline by one row
    if (stage >= 2) {
        k.qbelA = k.qyA;
        k.qbelB = k.qyB;
        k.qyA = cyA;
        k.qyB = cyB;
        k.qA = ckA;
        k.qB = ckB;
    }
    if (stage >= 1) {
        const bool smid = WALLS && ((sb >> 2) & 1u);
        mid_shift<C, UP, WALLS>(k.wA, oa, smid);
        mid_shift<C, UP, WALLS>(k.wB, ob, smid);
    }
    k.belA = k.pyA;
    k.belB = k.pyB;
    k.pyA = nyA;
    k.pyB = nyB;
    k.kA = nkA;
    k.kB = nkB;
    if (WALLS) k.sb = sb;
    if (SYNC) __builtin_amdgcn_s_barrier();
}

// FP16 storage: the first step's results stay in registers as the words the
// one-step sweep would store (node A's population in the low half, node B's
// in the high one, each rounded once from its exact value), and the second
// step widens them exactly as that sweep widens the words it loads.  The
// window of a lane's pair is then one word per population instead of two
// values.
struct Tb2CarryH {
    Coeffs<float> kA, kB;
    float pyA, pyB, belA, belB;
    MidWindow<uint32_t> w;
    Coeffs<float> qA, qB;
    float qyA, qyB, qbelA, qbelB;
};
// with whole-row walls, the wall bits of the pipeline's rows as well
struct Tb2CarryHW : Tb2CarryH {
    uint32_t sb;  // bit j: row y + (2 - j) dir solid
};

// The nine store words of a pair from its coefficients and Phi_y gradients,
// as the one-step FP16 sweep forms them.
__device__ __forceinline__ void tb2_half_words(uint32_t wd[9], const Coeffs<float> &a, float dya,
                                               const Coeffs<float> &b, float dyb, float ph) {
    HalfPairs pa, pb;
    reconstruct_pairs(pa, a.base, a.bx, a.by, a.bxx, a.byy - ph * dya, a.bxy, a.bxxy, a.bxyy);
    reconstruct_pairs(pb, b.base, b.bx, b.by, b.bxx, b.byy - ph * dyb, b.bxy, b.bxxy, b.bxyy);
    wd[0] = half_out<0, true>(pb, half_out<0, false>(pa));
    wd[1] = half_out<1, true>(pb, half_out<1, false>(pa));
    wd[2] = half_out<2, true>(pb, half_out<2, false>(pa));
    wd[3] = half_out<3, true>(pb, half_out<3, false>(pa));
    wd[4] = half_out<4, true>(pb, half_out<4, false>(pa));
    wd[5] = half_out<5, true>(pb, half_out<5, false>(pa));
    wd[6] = half_out<6, true>(pb, half_out<6, false>(pa));
    wd[7] = half_out<7, true>(pb, half_out<7, false>(pa));
    wd[8] = half_out<8, true>(pb, half_out<8, false>(pa));
}

// One pipeline row with FP16 storage (stages as tb2_row).  WALLS:
// whole-row walls (as tb2_row; the second step's pull row carries the wall
// flags of its neighbours to the widen, which bounces as for loaded rows).
template <int STAGE, bool SYNC = true, bool UP = true, bool WALLS = false, class K>
__device__ __forceinline__ void tb2_row_h(K &k, PairRow<_Float16> &raw,
                                          const PairCtx<_Float16> &cx, const Tb2Lane &ln,
                                          bool odd, const Tb2Params &p,
                                          const BufAccess<_Float16> &out, int y, bool load,
                                          int yload, bool store, int pitch, int64_t plane,
                                          int stage = STAGE, uint32_t lflags = 0u) {
    using C = float;
    constexpr bool SH = true;
    const C gx = p.gx, gy = p.gy, w1 = p.w1, w2 = p.w2, ph = p.ph;
    OpenX<C> ox;
    ox.on = false;
    ox.nx = 0;
    ox.u_in = ox.rho_in = ox.rho_out = ox.phi_wall = C(0);
    // (b) row y + 3 from its stored halves, then (a) the next loads
    C nyA, nyB;
    Coeffs<C> nkA, nkB;
    // whole-row walls: bit j, row y + (3 - j) dir solid
    uint32_t sb = 0u;
    if constexpr (WALLS) sb = (k.sb << 1) | (raw.rs & 1u);
    {
        RowState<C, SH> nA, nB;
        widen_pair<_Float16, C, SH, true, WALLS>(nA, nB, raw, cx, gx, gy, ox);
        if (load) tb2_gather<_Float16, WALLS>(raw, cx, ln, odd, yload, lflags);
        const C left = dpp_shr(C(0), nB.phix);
        const C right = dpp_shl(C(0), nA.phix);
        nkA = collide_coeffs<C, SH>(nA.m, C(0.5) * (nB.phix - left), w1, w2, ph, gx, gy);
        nkB = collide_coeffs<C, SH>(nB.m, C(0.5) * (right - nA.phix), w1, w2, ph, gx, gy);
        nyA = nA.phiy;
        nyB = nB.phiy;
    }
    // (c) collide row y + 2 of the first step into store words
    uint32_t ow[9];
    if (stage >= 1) {
        const C dya = C(0.5) * (UP ? nyA - k.belA : k.belA - nyA);
        const C dyb = C(0.5) * (UP ? nyB - k.belB : k.belB - nyB);
        tb2_half_words(ow, k.kA, dya, k.kB, dyb, ph);
    }
    // (d) the next row of the second step: the words its pull reads (0, 1, 3
    // from its own row, the others from the rows on either side),
    // widened as loaded words are (x neighbours by DPP word shifts)
    C cyA = C(0), cyB = C(0);
    Coeffs<C> ckA, ckB;
    if (stage >= 2) {
        PairRow<_Float16> pr;
        pr.w[0] = k.w.mid[0];
        pr.w[1] = k.w.mid[1];
        pr.w[3] = k.w.mid[2];
        if (UP) {
            pr.w[2] = k.w.lo[0];
            pr.w[5] = k.w.lo[1];
            pr.w[6] = k.w.lo[2];
            pr.w[4] = ow[4];
            pr.w[7] = ow[7];
            pr.w[8] = ow[8];
        } else {
            pr.w[4] = k.w.lo[0];
            pr.w[7] = k.w.lo[1];
            pr.w[8] = k.w.lo[2];
            pr.w[2] = ow[2];
            pr.w[5] = ow[5];
            pr.w[6] = ow[6];
        }
        pr.edge[0] = pr.edge[1] = pr.edge[2] = _Float16(0);
        pr.lk = pr.rs = 0u;
        if constexpr (WALLS) {
            // row y + 1: the words bounced at a wall row ahead are its own
            // words streaming forward (the window's middle); those bounced
            // at a wall row behind are in lo (mid_shift); the widen takes
            // them without shifts, by the row's geometric flags
            const uint32_t behind = (sb >> 3) & 1u, ahead = (sb >> 1) & 1u;
            if (ahead) {
                pr.w[UP ? 4 : 2] = k.w.mid[3];
                pr.w[UP ? 7 : 5] = k.w.mid[4];
                pr.w[UP ? 8 : 6] = k.w.mid[5];
            }
            pr.rs = ((sb >> 2) & 1u) | ((UP ? behind : ahead) << 1) | ((UP ? ahead : behind) << 2);
        }
        RowState<C, SH> cA, cB;
        widen_pair<_Float16, C, SH, true, WALLS>(cA, cB, pr, cx, gx, gy, ox);
        const C left = dpp_shr(C(0), cB.phix);
        const C right = dpp_shl(C(0), cA.phix);
        ckA = collide_coeffs<C, SH>(cA.m, C(0.5) * (cB.phix - left), w1, w2, ph, gx, gy);
        ckB = collide_coeffs<C, SH>(cB.m, C(0.5) * (right - cA.phix), w1, w2, ph, gx, gy);
        cyA = cA.phiy;
        cyB = cB.phiy;
    }
    // (e) collide row y of the second step and store the window's middle
    if (stage >= 3) {
        uint32_t sw[9];
        tb2_half_words(sw, k.qA, C(0.5) * (UP ? cyA - k.qbelA : k.qbelA - cyA), k.qB,
                       C(0.5) * (UP ? cyB - k.qbelB : k.qbelB - cyB), ph);
        if (WALLS) solid_zero<uint32_t>(sw, sw, (sb >> 3) & 1u);
        if (store) {
            const int64_t e0 = (int64_t)y * pitch;
#pragma unroll
            for (int i = 0; i < 9; ++i)
                __builtin_amdgcn_raw_buffer_store_b32(sw[i], out.r, cx.opair,
                                                      (uint32_t)((i * plane + e0) * 2),
                                                      TRT_STORE_CPOL);
        }
    }
    // advance the pipeline by one row
    if (stage >= 2) {
        k.qbelA = k.qyA;
        k.qbelB = k.qyB;
        k.qyA = cyA;
        k.qyB = cyB;
        k.qA = ckA;
        k.qB = ckB;
    }
    if (stage >= 1) mid_shift<uint32_t, UP, WALLS>(k.w, ow, WALLS && ((sb >> 2) & 1u));
    k.belA = k.pyA;
    k.belB = k.pyB;
    k.pyA = nyA;
    k.pyB = nyB;
    k.kA = nkA;
    k.kB = nkB;
    if constexpr (WALLS) k.sb = sb;
    if (SYNC) __builtin_amdgcn_s_barrier();
}

// The pipeline row and carried state of each storage type.
template <int ST> struct Tb2Rows;
template <> struct Tb2Rows<ST_F32> {
    template <bool WALLS> using Carry = Tb2Carry<float>;
    template <int STAGE, bool SYNC, bool UP, bool WALLS>
    __device__ static __forceinline__ void row(Carry<WALLS> &k, PairRow<float> &raw,
                                               const PairCtx<float> &cx, const Tb2Lane &ln,
                                               bool odd, const Tb2Params &p,
                                               const BufAccess<float> &out, int y, bool load,
                                               int yload, bool store, int pitch, int64_t plane,
                                               int stage = STAGE, uint32_t lflags = 0u) {
        tb2_row<STAGE, float, float, true, SYNC, UP, WALLS>(k, raw, cx, ln, odd, p, out, y, load,
                                                            yload, store, pitch, plane, stage,
                                                            lflags);
    }
};
template <> struct Tb2Rows<ST_F16> {
    template <bool WALLS> using Carry = typename std::conditional<WALLS, Tb2CarryHW, Tb2CarryH>::type;
    template <int STAGE, bool SYNC, bool UP, bool WALLS>
    __device__ static __forceinline__ void row(Carry<WALLS> &k, PairRow<_Float16> &raw,
                                               const PairCtx<_Float16> &cx, const Tb2Lane &ln,
                                               bool odd, const Tb2Params &p,
                                               const BufAccess<_Float16> &out, int y, bool load,
                                               int yload, bool store, int pitch, int64_t plane,
                                               int stage = STAGE, uint32_t lflags = 0u) {
        tb2_row_h<STAGE, SYNC, UP, WALLS>(k, raw, cx, ln, odd, p, out, y, load, yload, store,
                                          pitch, plane, stage, lflags);
    }
};

// One wavefront's window through one row block: the six rows that fill the
// pipeline as a short loop (run-time stage: fewer registers than peeled
// copies), then the full pipeline.  The loads run DEPTH rows ahead of their
// use (DEPTH 2: two row buffers, alternating).  SYNC: one workgroup barrier
// per pipeline row (adjacent windows in step); batch work items run
// without.  UP: the march goes up the row block (rows y0 - 6 ... y1 - 1 as
// pipeline rows), else down it (y1 + 5 ... y0), every node computed alike.
// WALLS: the lattice's solid nodes fill whole rows (InstDesc::rowwalls).
template <int ST, int DEPTH, bool SYNC = true, bool UP = true, bool WALLS = false>
__device__ __forceinline__ void sweep_strip_tb2(const InstDesc &d, int strip, int rb, int srcsel) {
    using T = typename Store<ST>::T;
    using R = Tb2Rows<ST>;
    static_assert(ST == ST_F32 || ST == ST_F16, "two steps per pass: FP32 or FP16 storage");
    static_assert(DEPTH == 1 || DEPTH == 2, "loads one or two rows ahead");

    const int lane = threadIdx.x & 63;
    const int nx = d.nx, ny = d.ny, pitch = d.pitch;
    const int64_t plane = d.plane;
    const T *__restrict__ src = static_cast<const T *>(srcsel ? d.buf[1] : d.buf[0]);
    T *__restrict__ dst = static_cast<T *>(srcsel ? d.buf[0] : d.buf[1]);
    const uint64_t bytes = (uint64_t)ny * (uint64_t)pitch * sizeof(T);
    const BufAccess<T> in(src, bytes), out(dst, bytes);
    const LinkAccess lacc(d.links, 0);
    // the lane's pair (Tb2Lane) and whether it is in the stored middle of
    // the window and inside the lattice
    const int xs = strip * kTb2Valid - 4 + 2 * lane;
    int ca = xs % nx;
    if (ca < 0) ca += nx;
    const int cb = ca + 1 == nx ? 0 : ca + 1;
    const bool odd = (nx & 1) != 0;
    const Tb2Lane ln{(ca & 1) != 0 || cb != ca + 1, (uint32_t)ca * (uint32_t)sizeof(T),
                     (uint32_t)cb * (uint32_t)sizeof(T)};
    const int cp = ln.split ? (ca & ~1) : ca;  // the aligned pair loaded (and stored)
    const bool store = lane >= 2 && lane < 62 && xs < nx;
    const Column hcol = column_of(cp, nx, sizeof(T));  // no halo node: unused
    const uint32_t ve[3] = {0u, 0u, 0u};
    const PairCtx<T> cx{in, plane, pitch, ny, (uint32_t)cp * (uint32_t)sizeof(T), (uint32_t)cp,
                        false, ve, hcol, lacc, false, d.lpitch, 0u, false};
    const Tb2Params p{(float)d.gx, (float)d.gy, (float)d.omega1, (float)d.omega2, (float)d.phi};
    const int y0 = rb * d.rows;
    const int y1 = min(y0 + d.rows, ny);
    const auto wrap_row = [&](int v) { v %= ny; return v < 0 ? v + ny : v; };
    // pipeline row y widens row y + 3 dir and loads row y + (3 + DEPTH) dir
    // while one is needed (the block needs rows y0 - 3 ... y1 + 2)
    constexpr int dir = UP ? 1 : -1;
    const auto ld = [&](int y) {
        return UP ? y + 3 + DEPTH <= y1 + 2 : y - 3 - DEPTH >= y0 - 3;
    };
    const auto lrow = [&](int y) { return wrap_row(y + dir * (3 + DEPTH)); };
    // the wall flags of a row to load (0 without walls): rows are loaded in
    // the march's order from the block's first gathered row on, which
    // LoadWalls follows
    LoadWalls<UP, WALLS> lw(d, UP ? y0 - 3 : y1 + 2);
    const auto wfl = [&](int row) -> uint32_t {
        (void)row;
        if constexpr (WALLS) return lw.take(d);
        return 0u;
    };
    const auto lfl = [&](int y) -> uint32_t { return ld(y) ? wfl(lrow(y)) : 0u; };

    typename R::template Carry<WALLS> k{};
    PairRow<T> raw[DEPTH];
    const int ys = UP ? y0 - 6 : y1 + 5;  // the first pipeline row
    tb2_gather<T, WALLS>(raw[0], cx, ln, odd, wrap_row(ys + 3 * dir), wfl(wrap_row(ys + 3 * dir)));
    if (DEPTH == 2)
        tb2_gather<T, WALLS>(raw[DEPTH - 1], cx, ln, odd, wrap_row(ys + 4 * dir),
                             wfl(wrap_row(ys + 4 * dir)));
    constexpr int R1 = DEPTH - 1;
    int y = ys;
    for (int i = 0; i < 6; ++i, y += dir) {
        // both buffers named statically (a run-time index would move them
        // to scratch memory)
        if (DEPTH == 2 && (i & 1))
            R::template row<-1, SYNC, UP, WALLS>(k, raw[R1], cx, ln, odd, p, out, y, ld(y), lrow(y),
                                                 store, pitch, plane, i >> 1, lfl(y));
        else
            R::template row<-1, SYNC, UP, WALLS>(k, raw[0], cx, ln, odd, p, out, y, ld(y), lrow(y),
                                                 store, pitch, plane, i >> 1, lfl(y));
    }
    // the rows of the block, y0 ... y1 - 1 in the march's order
    const auto inside = [&](int v) { return UP ? v < y1 : v >= y0; };
    if (DEPTH == 1) {
        for (; inside(y); y += dir)
            R::template row<3, SYNC, UP, WALLS>(k, raw[0], cx, ln, odd, p, out, y, ld(y), lrow(y),
                                                store, pitch, plane, 3, lfl(y));
    } else {
        for (; inside(y + dir); y += 2 * dir) {
            R::template row<3, SYNC, UP, WALLS>(k, raw[0], cx, ln, odd, p, out, y, ld(y), lrow(y),
                                                store, pitch, plane, 3, lfl(y));
            R::template row<3, SYNC, UP, WALLS>(k, raw[R1], cx, ln, odd, p, out, y + dir,
                                                ld(y + dir), lrow(y + dir), store, pitch, plane, 3,
                                                lfl(y + dir));
        }
        if (inside(y))
            R::template row<3, SYNC, UP, WALLS>(k, raw[0], cx, ln, odd, p, out, y, ld(y), lrow(y),
                                                store, pitch, plane, 3, lfl(y));
    }
}

// A wavefront of a synchronised workgroup with no strip to sweep (the
// lattice has fewer strips than the workgroup has wavefronts): it meets the
// same barriers as its row block's sweeping wavefronts.
__device__ __forceinline__ void idle_rows(const InstDesc &d, int rb) {
    const int y0 = rb * d.rows;
    const int y1 = min(y0 + d.rows, d.ny);
    for (int y = y0; y < y1; ++y) __builtin_amdgcn_s_barrier();
}

// Two-column sweep of one lattice.  Workgroup b covers row block
// b / groups and the strips [g * wpb, g * wpb + wpb) with g = b % groups;
// every wavefront of it runs the same rows and meets one barrier per row, so
// none may leave early: the grid is exactly rowblocks x groups workgroups.
template <int ST, bool LINKED>
__global__ __launch_bounds__(ST == ST_F64 ? 512 : 1024) void sweep_pair_kernel(InstDesc d,
                                                                                 int srcsel,
                                                                                 int remap) {
    int b = blockIdx.x;
    if (remap) b = xcd_remap(b, gridDim.x);
    const int wpb = blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int groups = (d.strips + wpb - 1) / wpb;
    const int rb = b / groups;
    const int strip = (b - rb * groups) * wpb + w;
    if (strip < d.strips)
        sweep_strip2<ST, true, LINKED>(d, strip, rb, srcsel);
    else
        idle_rows(d, rb);
}

// Three time steps per pass (FP32 storage): the two-step pipeline with one
// more step in the middle.  A wavefront's 128-column window loses two
// columns on each side per step (the pull and the Phi_x gradient each
// reach one column further), so it stores its middle kTb3Valid = 116
// columns; a row block of R rows reads R + 10 rows.  Pipeline row y:
// (b) the first-step moments and coefficients of row y + 5 from `raw`,
// then the loads of a later row; (c) the first-step collision of row y + 4;
// (d) the second-step pull and coefficients of row y + 3; (e) the
// second-step collision of row y + 2; (f) the third-step pull and
// coefficients of row y + 1; (g) the third-step collision of row y and its
// store.  Stage k adds part k of these; the first ten pipeline rows of a
// block fill the pipeline.  Every node's arithmetic is the one-step
// sweep's and each step's results are those that sweep stores and loads
// back, so three steps per pass reproduce its bits.
template <class C> struct Tb3Carry {
    Coeffs<C> kA, kB;     // first step: coefficients of the next row to collide
    C pyA, pyB;           // ... its Phi_y
    C belA, belB;         // ... and that of the row behind it
    MidWindow<C> wA, wB;  // first-step results in flight
    Coeffs<C> qA, qB;     // second step: the next row to collide ...
    C qyA, qyB, qbelA, qbelB;
    MidWindow<C> vA, vB;  // second-step results in flight
    Coeffs<C> rA, rB;     // third step: the next row to collide and store
    C ryA, ryB, rbelA, rbelB;
    uint32_t sb;          // whole-row walls: bit j, row y + (4 - j) dir solid
};

// Post-collision populations of a lane's pair from their coefficients and
// Phi_y gradients (dya, dyb: the row ahead minus the row behind, halved).
template <class C>
__device__ __forceinline__ void collide_pair(C oa[9], C ob[9], const Coeffs<C> &a, C dya,
                                             const Coeffs<C> &b, C dyb, C ph) {
    reconstruct<C>(oa, a.base, a.bx, a.by, a.bxx, a.byy - ph * dya, a.bxy, a.bxxy, a.bxyy);
    reconstruct<C>(ob, b.base, b.bx, b.by, b.bxx, b.byy - ph * dyb, b.bxy, b.bxxy, b.bxyy);
}

// WALLS: whole-row walls; lflags are the flags of row yload (RowWalls).
template <int STAGE, bool UP = true, bool SYNC = true, bool WALLS = false>
__device__ __forceinline__ void tb3_row(Tb3Carry<float> &k, PairRow<float> &raw,
                                        const PairCtx<float> &cx, const Tb2Lane &ln, bool odd,
                                        const Tb2Params &p, const BufAccess<float> &out, int y,
                                        bool load, int yload, bool store, int pitch,
                                        int64_t plane, int stage = STAGE, uint32_t lflags = 0u) {
    using C = float;
    constexpr bool SH = true;
    const C gx = p.gx, gy = p.gy, w1 = p.w1, w2 = p.w2, ph = p.ph;
    OpenX<C> ox;
    ox.on = false;
    ox.nx = 0;
    ox.u_in = ox.rho_in = ox.rho_out = ox.phi_wall = C(0);
    // the Phi_y gradient: the row ahead of the march minus the row behind
    const auto grad = [](C ahead, C behind) { return C(0.5) * (UP ? ahead - behind : behind - ahead); };
    // (b) row y + 5, then (a) the next loads into the same registers
    C nyA, nyB;
    Coeffs<C> nkA, nkB;
    // whole-row walls: bit j, row y + (5 - j) dir solid
    const uint32_t sb = WALLS ? ((k.sb << 1) | (raw.rs & 1u)) : 0u;
    {
        RowState<C, SH> nA, nB;
        widen_pair<float, C, SH, false, WALLS>(nA, nB, raw, cx, gx, gy, ox);
        if (load) tb2_gather<float, WALLS>(raw, cx, ln, odd, yload, lflags);
        const C left = dpp_shr(C(0), nB.phix);
        const C right = dpp_shl(C(0), nA.phix);
        nkA = collide_coeffs<C, SH>(nA.m, C(0.5) * (nB.phix - left), w1, w2, ph, gx, gy);
        nkB = collide_coeffs<C, SH>(nB.m, C(0.5) * (right - nA.phix), w1, w2, ph, gx, gy);
        nyA = nA.phiy;
        nyB = nB.phiy;
    }
    // (c) first-step collision of row y + 4
    C oa[9], ob[9];
    if (stage >= 1) collide_pair<C>(oa, ob, k.kA, grad(nyA, k.belA), k.kB, grad(nyB, k.belB), ph);
    // (d) second-step pull and coefficients of row y + 3
    C cyA = C(0), cyB = C(0);
    Coeffs<C> ckA, ckB;
    if (stage >= 2)
        pull_coeffs_pair<C, SH, UP, WALLS>(ckA, ckB, cyA, cyB, k.wA, k.wB, oa, ob, p,
                                           wall_flags(sb, 2));
    // (e) second-step collision of row y + 2
    C sa[9], sb_[9];
    if (stage >= 3)
        collide_pair<C>(sa, sb_, k.qA, grad(cyA, k.qbelA), k.qB, grad(cyB, k.qbelB), ph);
    // (f) third-step pull and coefficients of row y + 1
    C ryA = C(0), ryB = C(0);
    Coeffs<C> rkA, rkB;
    if (stage >= 4)
        pull_coeffs_pair<C, SH, UP, WALLS>(rkA, rkB, ryA, ryB, k.vA, k.vB, sa, sb_, p,
                                           wall_flags(sb, 4));
    // (g) third-step collision of row y and the store of the window's middle
    if (stage >= 5) {
        C ta[9], tb[9];
        collide_pair<C>(ta, tb, k.rA, grad(ryA, k.rbelA), k.rB, grad(ryB, k.rbelB), ph);
        if (WALLS) solid_zero<C>(ta, tb, (sb >> 5) & 1u);
        if (store) {
            const int64_t e0 = (int64_t)y * pitch;
#pragma unroll
            for (int i = 0; i < 9; ++i)
                PairIO<float>::st(out, i * plane + e0, cx.opair, ta[i], tb[i]);
        }
    }
    // advance the pipeline by one row
    if (stage >= 4) {
        k.rbelA = k.ryA;
        k.rbelB = k.ryB;
        k.ryA = ryA;
        k.ryB = ryB;
        k.rA = rkA;
        k.rB = rkB;
    }
    if (stage >= 3) {
        const bool smid = WALLS && ((sb >> 4) & 1u);
        mid_shift<C, UP, WALLS>(k.vA, sa, smid);
        mid_shift<C, UP, WALLS>(k.vB, sb_, smid);
    }
    if (stage >= 2) {
        k.qbelA = k.qyA;
        k.qbelB = k.qyB;
        k.qyA = cyA;
        k.qyB = cyB;
        k.qA = ckA;
        k.qB = ckB;
    }
    if (stage >= 1) {
        const bool smid = WALLS && ((sb >> 2) & 1u);
        mid_shift<C, UP, WALLS>(k.wA, oa, smid);
        mid_shift<C, UP, WALLS>(k.wB, ob, smid);
    }
    k.belA = k.pyA;
    k.belB = k.pyB;
    k.pyA = nyA;
    k.pyB = nyB;
    k.kA = nkA;
    k.kB = nkB;
    if (WALLS) k.sb = sb;
    if (SYNC) __builtin_amdgcn_s_barrier();
}

// Three time steps over row block rb of window `strip` (FP32): as
// sweep_strip_tb2, with ten pipeline rows of fill and the block's rows
// y0 - 5 ... y1 + 4 gathered.  SYNC: one workgroup barrier per pipeline
// row; batch work items run without.
template <int DEPTH, bool UP = true, bool SYNC = true, bool WALLS = false>
__device__ __forceinline__ void sweep_strip_tb3(const InstDesc &d, int strip, int rb, int srcsel) {
    static_assert(DEPTH == 1 || DEPTH == 2, "loads one or two rows ahead");
    using T = float;
    const int lane = threadIdx.x & 63;
    const int nx = d.nx, ny = d.ny, pitch = d.pitch;
    const int64_t plane = d.plane;
    const T *__restrict__ src = static_cast<const T *>(srcsel ? d.buf[1] : d.buf[0]);
    T *__restrict__ dst = static_cast<T *>(srcsel ? d.buf[0] : d.buf[1]);
    const uint64_t bytes = (uint64_t)ny * (uint64_t)pitch * sizeof(T);
    const BufAccess<T> in(src, bytes), out(dst, bytes);
    const LinkAccess lacc(d.links, 0);
    // the lane's pair and whether it is in the stored middle of the window
    // (lanes 3 ... 60) and inside the lattice
    const int xs = strip * kTb3Valid - 6 + 2 * lane;
    int ca = xs % nx;
    if (ca < 0) ca += nx;
    const int cb = ca + 1 == nx ? 0 : ca + 1;
    const bool odd = (nx & 1) != 0;
    const Tb2Lane ln{(ca & 1) != 0 || cb != ca + 1, (uint32_t)ca * (uint32_t)sizeof(T),
                     (uint32_t)cb * (uint32_t)sizeof(T)};
    const int cp = ln.split ? (ca & ~1) : ca;
    const bool store = lane >= 3 && lane < 61 && xs < nx;
    const Column hcol = column_of(cp, nx, sizeof(T));
    const uint32_t ve[3] = {0u, 0u, 0u};
    const PairCtx<T> cx{in, plane, pitch, ny, (uint32_t)cp * (uint32_t)sizeof(T), (uint32_t)cp,
                        false, ve, hcol, lacc, false, d.lpitch, 0u, false};
    const Tb2Params p{(float)d.gx, (float)d.gy, (float)d.omega1, (float)d.omega2, (float)d.phi};
    const int y0 = rb * d.rows;
    const int y1 = min(y0 + d.rows, ny);
    const auto wrap_row = [&](int v) { v %= ny; return v < 0 ? v + ny : v; };
    // pipeline row y widens row y + 5 dir and loads row y + (5 + DEPTH) dir
    // while one is needed (the block needs rows y0 - 5 ... y1 + 4)
    constexpr int dir = UP ? 1 : -1;
    const auto ld = [&](int y) {
        return UP ? y + 5 + DEPTH <= y1 + 4 : y - 5 - DEPTH >= y0 - 5;
    };
    const auto lrow = [&](int y) { return wrap_row(y + dir * (5 + DEPTH)); };
    // the wall flags of a row to load (0 without walls): rows are loaded in
    // the march's order from the block's first gathered row on, which
    // LoadWalls follows
    LoadWalls<UP, WALLS> lw(d, UP ? y0 - 5 : y1 + 4);
    const auto wfl = [&](int row) -> uint32_t {
        (void)row;
        if constexpr (WALLS) return lw.take(d);
        return 0u;
    };
    const auto lfl = [&](int y) -> uint32_t { return ld(y) ? wfl(lrow(y)) : 0u; };

    Tb3Carry<float> k{};
    PairRow<T> raw[DEPTH];
    const int ys = UP ? y0 - 10 : y1 + 9;  // the first pipeline row
    tb2_gather<T, WALLS>(raw[0], cx, ln, odd, wrap_row(ys + 5 * dir), wfl(wrap_row(ys + 5 * dir)));
    if (DEPTH == 2)
        tb2_gather<T, WALLS>(raw[DEPTH - 1], cx, ln, odd, wrap_row(ys + 6 * dir),
                             wfl(wrap_row(ys + 6 * dir)));
    constexpr int R1 = DEPTH - 1;
    int y = ys;
    for (int i = 0; i < 10; ++i, y += dir) {
        // both buffers named statically (a run-time index would move them
        // to scratch memory)
        if (DEPTH == 2 && (i & 1))
            tb3_row<-1, UP, SYNC, WALLS>(k, raw[R1], cx, ln, odd, p, out, y, ld(y), lrow(y), store,
                                         pitch, plane, i >> 1, lfl(y));
        else
            tb3_row<-1, UP, SYNC, WALLS>(k, raw[0], cx, ln, odd, p, out, y, ld(y), lrow(y), store,
                                         pitch, plane, i >> 1, lfl(y));
    }
    const auto inside = [&](int v) { return UP ? v < y1 : v >= y0; };
    if (DEPTH == 1) {
        for (; inside(y); y += dir)
            tb3_row<5, UP, SYNC, WALLS>(k, raw[0], cx, ln, odd, p, out, y, ld(y), lrow(y), store,
                                        pitch, plane, 5, lfl(y));
    } else {
        for (; inside(y + dir); y += 2 * dir) {
            tb3_row<5, UP, SYNC, WALLS>(k, raw[0], cx, ln, odd, p, out, y, ld(y), lrow(y), store,
                                        pitch, plane, 5, lfl(y));
            tb3_row<5, UP, SYNC, WALLS>(k, raw[R1], cx, ln, odd, p, out, y + dir, ld(y + dir),
                                        lrow(y + dir), store, pitch, plane, 5, lfl(y + dir));
        }
        if (inside(y))
            tb3_row<5, UP, SYNC, WALLS>(k, raw[0], cx, ln, odd, p, out, y, ld(y), lrow(y), store,
                                        pitch, plane, 5, lfl(y));
    }
}

// Two time steps per pass (sweep_strip_tb2): workgroup b covers row block
// b / groups and the windows [g * wpb, g * wpb + wpb) with g = b % groups,
// as the two-column sweep; a wavefront without a window meets the R + 6
// barriers of its row block.  FP32: DEPTH 1 fits 168 VGPRs (three
// wavefronts per SIMD), DEPTH 2 210 (two); FP16: 133 (three) and 171 (two).
constexpr int kTb2MaxWaves = 4;
template <int ST, int DEPTH, bool WALLS = false>
__global__ __launch_bounds__(64 * kTb2MaxWaves) void sweep_tb2_kernel(InstDesc d, int srcsel,
                                                                      int remap,
                                                                      int alternate) {
    int b = blockIdx.x;
    if (remap) b = xcd_remap(b, gridDim.x);
    const int wpb = blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int groups = (d.strips + wpb - 1) / wpb;
    const int rb = b / groups;
    const int strip = (b - rb * groups) * wpb + w;
    if (strip < d.strips) {
        // alternate: odd row blocks march down, so that each block boundary
        // is read by both neighbouring blocks at the same end of their runs
        // (both at the start or both at the end) and the second read can
        // hit in L2
        if (alternate && (rb & 1))
            sweep_strip_tb2<ST, DEPTH, true, false, WALLS>(d, strip, rb, srcsel);
        else
            sweep_strip_tb2<ST, DEPTH, true, true, WALLS>(d, strip, rb, srcsel);
    } else {
        const int y0 = rb * d.rows;
        const int y1 = min(y0 + d.rows, d.ny);
        for (int y = y0 - 6; y < y1; ++y) __builtin_amdgcn_s_barrier();
    }
}

// Three time steps per pass: workgroups as for two (sweep_tb2_kernel), R +
// 10 barriers per row block; loads one row ahead (238 VGPRs, two wavefronts
// per SIMD).  WALLS: whole-row walls (InstDesc::rowwalls).
template <bool WALLS>
__global__ __launch_bounds__(64 * kTb2MaxWaves) void sweep_tb3_kernel(InstDesc d, int srcsel,
                                                                      int remap,
                                                                      int alternate) {
    int b = blockIdx.x;
    if (remap) b = xcd_remap(b, gridDim.x);
    const int wpb = blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int groups = (d.strips + wpb - 1) / wpb;
    const int rb = b / groups;
    const int strip = (b - rb * groups) * wpb + w;
    if (strip < d.strips) {
        if (alternate && (rb & 1))
            sweep_strip_tb3<1, false, true, WALLS>(d, strip, rb, srcsel);
        else
            sweep_strip_tb3<1, true, true, WALLS>(d, strip, rb, srcsel);
    } else {
        const int y0 = rb * d.rows;
        const int y1 = min(y0 + d.rows, d.ny);
        for (int y = y0 - 10; y < y1; ++y) __builtin_amdgcn_s_barrier();
    }
}

// Batched three-step pass (FP32): wavefront w takes item w = (member,
// window, row block, -) of the three-step tables; no barriers.  Members
// with whole-row walls take the walled pipeline.
__global__ __launch_bounds__(64 * kTb2MaxWaves) void sweep_tb3_batch_kernel(
    const InstDesc *__restrict__ descs, int ndescs, const int4 *__restrict__ items, int nitems,
    int flip, int remap) {
    int b = blockIdx.x;
    if (remap) b = xcd_remap(b, gridDim.x);
    const int wpb = blockDim.x >> 6;
    const int wave = b * wpb + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= nitems) return;
    const int4 it = items[wave];
    if ((unsigned)it.x >= (unsigned)ndescs) return;
    const InstDesc d = descs[it.x];
    if (d.rowwalls) {
        if (it.z & 1)
            sweep_strip_tb3<1, false, false, true>(d, it.y, it.z, d.cur ^ flip);
        else
            sweep_strip_tb3<1, true, false, true>(d, it.y, it.z, d.cur ^ flip);
    } else {
        if (it.z & 1)
            sweep_strip_tb3<1, false, false>(d, it.y, it.z, d.cur ^ flip);
        else
            sweep_strip_tb3<1, true, false>(d, it.y, it.z, d.cur ^ flip);
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

// Batched one-step sweep: wavefront w takes work item w = (member, strip,
// row block, class); members of class 1 (it.w) read lattice cur ^ flip1,
// the others cur ^ flip0 (members that also take two-step launches advance
// their lattice parity at another rate).
template <int ST, bool MASK, bool BUF>
__global__ __launch_bounds__(256) void sweep_batch_kernel(const InstDesc *__restrict__ descs,
                                                           const int4 *__restrict__ items,
                                                           int nitems, int flip0, int flip1,
                                                           int remap) {
    int b = blockIdx.x;
    if (remap) b = xcd_remap(b, gridDim.x);
    const int wpb = blockDim.x >> 6;
    const int wave = b * wpb + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= nitems) return;
    const int4 it = items[wave];
    const InstDesc d = descs[it.x];
    const int flip = it.w ? flip1 : flip0;
    if (d.cols == 2)
        sweep_strip2<ST, false, MASK>(d, it.y, it.z, d.cur ^ flip);
    else
        sweep_strip<ST, MASK, BUF>(d, it.y, it.z, d.cur ^ flip);
}

// Batched two-step pass: wavefront w takes item w = (member, window, row
// block, -) of the two-step tables (each member's descriptor tiled for the
// pass); items are independent, so no barriers.
template <int ST, int DEPTH>
__global__ __launch_bounds__(64 * kTb2MaxWaves) void sweep_tb2_batch_kernel(
    const InstDesc *__restrict__ descs, int ndescs, const int4 *__restrict__ items, int nitems,
    int flip, int remap) {
    int b = blockIdx.x;
    if (remap) b = xcd_remap(b, gridDim.x);
    const int wpb = blockDim.x >> 6;
    const int wave = b * wpb + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= nitems) return;
    const int4 it = items[wave];
    if ((unsigned)it.x >= (unsigned)ndescs) return;
    const InstDesc d = descs[it.x];
    if (d.rowwalls) {
        sweep_strip_tb2<ST, DEPTH, false, true, true>(d, it.y, it.z, d.cur ^ flip);
        return;
    }
    sweep_strip_tb2<ST, DEPTH, false>(d, it.y, it.z, d.cur ^ flip);
}

template <int ST, bool MASK, bool BUF>
hipError_t launch_single_t(const InstDesc &d, int src, const Launch &l, hipStream_t s) {
    const int waves = d.strips * d.rowblocks;
    const int wpb = single_waves_per_block(d, ST, l);
    const int blocks = (waves + wpb - 1) / wpb;
    sweep_single_kernel<ST, MASK, BUF><<<blocks, 64 * wpb, 0, s>>>(d, src, l.xcd_remap);
    return hipGetLastError();
}

template <int ST, bool MASK, bool BUF>
hipError_t launch_batch_t(const InstDesc *descs, const int4 *items, int nitems, int flip,
                          int flip1, const Launch &l, hipStream_t s) {
    const int wpb = batch_waves_per_block(l);
    const int blocks = (nitems + wpb - 1) / wpb;
    sweep_batch_kernel<ST, MASK, BUF><<<blocks, 64 * wpb, 0, s>>>(descs, items, nitems, flip,
                                                                 flip1, l.xcd_remap);
    return hipGetLastError();
}

template <int ST>
hipError_t launch_pair_t(const InstDesc &d, int src, const Launch &l, hipStream_t s) {
    const int wpb = single_waves_per_block(d, ST, l);
    const int blocks = d.rowblocks * ((d.strips + wpb - 1) / wpb);
    if (d.links)
        sweep_pair_kernel<ST, true><<<blocks, 64 * wpb, 0, s>>>(d, src, l.xcd_remap);
    else
        sweep_pair_kernel<ST, false><<<blocks, 64 * wpb, 0, s>>>(d, src, l.xcd_remap);
    return hipGetLastError();
}

template <int ST, bool MASK>
hipError_t launch_single_b(const InstDesc &d, int src, const Launch &l, bool buf, hipStream_t s) {
    if (d.cols == 2) return launch_pair_t<ST>(d, src, l, s);
    return buf ? launch_single_t<ST, MASK, true>(d, src, l, s)
               : launch_single_t<ST, MASK, false>(d, src, l, s);
}

template <int ST, bool MASK>
hipError_t launch_batch_b(const InstDesc *descs, const int4 *items, int nitems, int flip,
                          int flip1, const Launch &l, bool buf, hipStream_t s) {
    return buf ? launch_batch_t<ST, MASK, true>(descs, items, nitems, flip, flip1, l, s)
               : launch_batch_t<ST, MASK, false>(descs, items, nitems, flip, flip1, l, s);
}

}  // namespace

bool buffer_addressable(const InstDesc &d, int storage) {
    const uint64_t es = storage == ST_F64 ? 8 : (storage == ST_F32 ? 4 : 2);
    return (uint64_t)d.ny * (uint64_t)d.pitch * es <= 0xffffffffull;
}

bool pair_eligible(const InstDesc &d, int storage) {
    // obstacles and open boundaries need the link map; an odd width whose
    // last strip holds a single column would need lane 0 as both edges
    const bool general = d.mask != nullptr || d.xbc != 0;
    return d.nx % kStripWidth2 != 1 && buffer_addressable(d, storage) &&
           (!general || d.links != nullptr);
}

hipError_t launch_sweep(const InstDesc &d, int storage, bool mask, int src, const Launch &l,
                        hipStream_t stream) {
    if (d.cols == 2 && !pair_eligible(d, storage)) return hipErrorInvalidValue;
    // open x boundaries live in the general (mask) kernels
    if (d.xbc) mask = true;
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

// Passes of several steps: FP32 or FP16 lattices, periodic, without a mask
// or with one whose solid nodes fill whole rows (walls parallel to x).
bool tb2_eligible(const InstDesc &d, int storage) {
    const bool open = d.links == nullptr && d.mask == nullptr;
    const bool walls = d.rowwalls != 0 && d.links != nullptr;
    return (storage == ST_F32 || storage == ST_F16) && (open || walls) && d.xbc == 0 &&
           buffer_addressable(d, storage);
}

// Wavefronts from which the two-step pass uses four-wavefront workgroups
// and, in FP32, loads two rows ahead: with at least two rounds of
// wavefronts at two per SIMD, the deeper prefetch outweighs the lost third
// wavefront (4096^2 at 32 rows, 4480 wavefronts: 126.7 against 132.0 us per
// step), below it does not (2048^2, 2304 wavefronts: 40.3 against 35.7).
constexpr long long kTb2DeepWaves = 4096;

InstDesc tb2_desc(const InstDesc &d, const Launch &l) {
    InstDesc t = d;
    t.strips = (d.nx + kTb2Valid - 1) / kTb2Valid;
    if (l.rows_per_wave > 0) {
        t.rows = l.rows_per_wave;
    } else {
        // the longest row block of 32, 24, 16, 12 or 8 rows that still gives
        // 6144 wavefronts, else the longest that gives 2048, else 8 (a block
        // of R rows runs R + 6 pipeline rows).  Measured (us per step, the
        // chosen shape against the best of rows 8..37 x 1, 2, 4 wavefronts
        // per workgroup x loads 1 or 2 rows ahead): FP32 8192^2 32 rows
        // 453.5 / 453.5, 4096^2 16 rows 120.1 / 120.1 (32 rows: 126.0),
        // 3000^2 12 rows 74.2 / 72.2, 2048^2 16 rows 35.8 / 35.1, 1024^2 8
        // rows 12.6 / 12.6; FP16 8192^2 272.8 / 272.8, 4096^2 75.3 / 75.3,
        // 3000^2 46.9 / 46.6, 2048^2 26.1 / 25.2, 1024^2 12.0 / 11.6.  Short
        // blocks read more overlap rows, but the many more wavefronts fill
        // the last round of workgroups on the CUs more evenly.
        static const int kRows[] = {32, 24, 16, 12, 8};
        const auto waves = [&](int r) { return (long long)t.strips * ((d.ny + r - 1) / r); };
        t.rows = 8;
        bool found = false;
        for (long long target : {6144LL, 2048LL}) {
            for (int r : kRows) {
                if (waves(r) >= target) {
                    t.rows = r;
                    found = true;
                    break;
                }
            }
            if (found) break;
        }
    }
    t.rowblocks = (d.ny + t.rows - 1) / t.rows;
    return t;
}

// Loads two rows ahead: two row buffers per wavefront (FP32: 210 VGPRs,
// two wavefronts per SIMD) instead of one (164, three per SIMD).  It pays
// only for FP32 launches of many wavefronts (8192^2 453.5 against 460.2 us
// per step, 4096^2 equal); FP16 gains more from the third wavefront per
// SIMD at every size (4096^2 75.3 against 79.9 us, 8192^2 272.8 against
// 297.1, 2048^2 25.2 against 26.0; the 256-member batch 311.7 against 323.7
// us per step, where FP32 keeps two rows ahead: 454.5 against 474.9).
static int tb2_prefetch(long long waves, int storage, const Launch &l) {
    if (l.prefetch_rows > 0) return l.prefetch_rows;
    return (storage == ST_F32 && waves >= kTb2DeepWaves) ? 2 : 1;
}

int tb2_prefetch_rows(const InstDesc &d, int storage, const Launch &l) {
    const InstDesc t = tb2_desc(d, l);
    return tb2_prefetch((long long)t.strips * t.rowblocks, storage, l);
}

int tb2_batch_prefetch_rows(int items, int storage, const Launch &l) {
    return tb2_prefetch(items, storage, l);
}

int tb2_waves_per_block(const InstDesc &d, int storage, const Launch &l) {
    (void)storage;
    const InstDesc t = tb2_desc(d, l);
    const bool many = (long long)t.strips * t.rowblocks >= kTb2DeepWaves;
    int w = l.waves_per_block > 0 ? l.waves_per_block : (many ? 4 : 1);
    if (w > kTb2MaxWaves) w = kTb2MaxWaves;
    while (w > 1 && w / 2 >= t.strips) w /= 2;
    return w;
}

hipError_t launch_sweep_tb2(const InstDesc &d, int storage, int src, const Launch &l,
                            hipStream_t stream) {
    if (!tb2_eligible(d, storage)) return hipErrorInvalidValue;
    const InstDesc t = tb2_desc(d, l);
    const int wpb = tb2_waves_per_block(d, storage, l);
    const int blocks = t.rowblocks * ((t.strips + wpb - 1) / wpb);
    const bool deep = tb2_prefetch((long long)t.strips * t.rowblocks, storage, l) == 2;
    // Alternating march directions share each row-block boundary's reads
    // through L2: 4096^2 FP32 HBM reads 0.734 -> 0.664 GB per launch, time
    // 128.0 -> 126.4 us per step (48 rows: 149.4 -> 143.6).  Where the pass
    // is further from HBM-bound it measured slower (4096^2 FP16 86.1 ->
    // 87.0, 2048^2 FP32 35.5 -> 36.4, 2048^2 FP16 26.3 -> 26.7), so only
    // deep FP32 launches alternate.
    const int alt = (deep && storage == ST_F32) ? 1 : 0;
    if (storage == ST_F16 && t.rowwalls) {
        if (deep)
            sweep_tb2_kernel<ST_F16, 2, true><<<blocks, 64 * wpb, 0, stream>>>(t, src, l.xcd_remap, alt);
        else
            sweep_tb2_kernel<ST_F16, 1, true><<<blocks, 64 * wpb, 0, stream>>>(t, src, l.xcd_remap, alt);
    } else if (storage == ST_F16) {
        if (deep)
            sweep_tb2_kernel<ST_F16, 2><<<blocks, 64 * wpb, 0, stream>>>(t, src, l.xcd_remap, alt);
        else
            sweep_tb2_kernel<ST_F16, 1><<<blocks, 64 * wpb, 0, stream>>>(t, src, l.xcd_remap, alt);
    } else if (t.rowwalls) {
        if (deep)
            sweep_tb2_kernel<ST_F32, 2, true><<<blocks, 64 * wpb, 0, stream>>>(t, src, l.xcd_remap, alt);
        else
            sweep_tb2_kernel<ST_F32, 1, true><<<blocks, 64 * wpb, 0, stream>>>(t, src, l.xcd_remap, alt);
    } else if (deep) {
        sweep_tb2_kernel<ST_F32, 2><<<blocks, 64 * wpb, 0, stream>>>(t, src, l.xcd_remap, alt);
    } else {
        sweep_tb2_kernel<ST_F32, 1><<<blocks, 64 * wpb, 0, stream>>>(t, src, l.xcd_remap, alt);
    }
    return hipGetLastError();
}

// Wavefronts from which the three-step pass takes four-wavefront
// workgroups in the hardware's round-robin order over the XCDs (4096^2 at
// 48 rows, 3096 wavefronts: 90.3 us per step, against 107.0 with
// contiguous XCD bands and 107.7 with one-wavefront workgroups; 8192^2 and
// 6144^2 at 48 rows: 338.9 / 204.1 against 345.6 / 211.4 with bands),
// below it one-wavefront workgroups in contiguous bands (2048^2 at 24 rows,
// 1548 wavefronts: 29.4 against 31.3 with four per workgroup and 30.8
// without bands).
constexpr long long kTb3ManyWaves = 3072;

bool tb3_eligible(const InstDesc &d, int storage) {
    return storage == ST_F32 && tb2_eligible(d, storage);
}

// Rows that make the pass's four-wavefront workgroups (row blocks x groups
// of four windows) just fit k whole rounds of the workgroups resident at
// once (1024 SIMDs x two wavefronts / four per workgroup = 512), for the
// smallest k = 1, 2, 3 that gives 8 to 192 rows; 0 if none does.  Same-run
// measurements (us per step, such rows in the hardware's XCD order against
// the rule below): 2048^2 21 rows 28.2 against 29.3, 3000^2 42 rows 54.4
// against 61.3, 4096^2 74 rows 88.0 against 89.3, 6144^2 171 rows 201.9
// against 202.5, 8192^2 147 rows 326.6 against 336.5.
static int tb3_round_rows(const InstDesc &d) {
    const int windows = (d.nx + kTb3Valid - 1) / kTb3Valid;
    const int groups = (windows + 3) / 4;
    const int slots = 1024 * 2 / 4;
    for (int k = 1; k <= 3; ++k) {
        const int blocks = k * slots / groups;
        if (blocks < 1) continue;
        const int r = (d.ny + blocks - 1) / blocks;
        if (r >= 8 && r <= 192) return r;
    }
    return 0;
}

InstDesc tb3_desc(const InstDesc &d, const Launch &l) {
    InstDesc t = d;
    t.strips = (d.nx + kTb3Valid - 1) / kTb3Valid;
    if (l.rows_per_wave > 0) {
        t.rows = l.rows_per_wave;
    } else if (tb3_round_rows(d) > 0) {
        t.rows = tb3_round_rows(d);
    } else {
        // lattices too small for whole rounds (below about 1500^2): the
        // longest of 48, 40, 32, 24 or 16 rows that gives 3072
        // wavefronts (four-wavefront workgroups), else the longest of those
        // and 12, 8 that gives 1536 (one-wavefront workgroups), else 8 (2048^2
        // at 8 rows, 4608 wavefronts: 35.6 us per step against 29.0 at 24
        // rows, one wavefront per workgroup).  A block of R rows
        // repeats ten rows of fill, so blocks are longer than in the
        // two-step pass.  Measured (us per step; chosen / best of rows 8 ...
        // 64 x 1, 2, 4 wavefronts per workgroup x XCD order): 8192^2 48 rows
        // 338.9 / 328.3 (64 rows), 6144^2 48 rows 204.1 / 203.6, 4096^2 48
        // rows 90.3 / 90.3, 3000^2 24 rows 61.6 / 55.3 (40 rows, two
        // wavefronts per workgroup), 2048^2 24 rows 29.4 / 28.0 (40 rows);
        // the optimum moves with how evenly the workgroups fill the CUs,
        // which the autotuner searches.
        static const int kRows[] = {48, 40, 32, 24, 16, 12, 8};
        const auto waves = [&](int r) { return (long long)t.strips * ((d.ny + r - 1) / r); };
        t.rows = 8;
        bool found = false;
        for (long long target : {kTb3ManyWaves, 1536LL}) {
            for (int r : kRows) {
                if (target == kTb3ManyWaves && r < 16) break;
                if (waves(r) >= target) {
                    t.rows = r;
                    found = true;
                    break;
                }
            }
            if (found) break;
        }
    }
    t.rowblocks = (d.ny + t.rows - 1) / t.rows;
    return t;
}

// whether the rows in effect are the whole-round rows (none asked for):
// those shapes take four-wavefront workgroups in the hardware's XCD order
static bool tb3_rounds(const InstDesc &d, const Launch &l) {
    return l.rows_per_wave <= 0 && tb3_round_rows(d) > 0;
}

int tb3_xcd_remap(const InstDesc &d, const Launch &l) {
    if (l.remap_asked) return l.xcd_remap;
    if (tb3_rounds(d, l)) return 0;
    const InstDesc t = tb3_desc(d, l);
    return (long long)t.strips * t.rowblocks >= kTb3ManyWaves ? 0 : 1;
}

int tb3_waves_per_block(const InstDesc &d, const Launch &l) {
    const InstDesc t = tb3_desc(d, l);
    const bool many = tb3_rounds(d, l) || (long long)t.strips * t.rowblocks >= kTb3ManyWaves;
    int w = l.waves_per_block > 0 ? l.waves_per_block : (many ? 4 : 1);
    if (w > kTb2MaxWaves) w = kTb2MaxWaves;
    while (w > 1 && w / 2 >= t.strips) w /= 2;
    return w;
}

// The three-step pass loads one row ahead whatever is asked: two rows ahead
// take 256 VGPRs and 33 AGPRs, one wavefront per SIMD.
int tb3_prefetch_rows(const InstDesc &, const Launch &) { return 1; }

hipError_t launch_sweep_tb3(const InstDesc &d, int storage, int src, const Launch &l,
                            hipStream_t stream) {
    if (!tb3_eligible(d, storage)) return hipErrorInvalidValue;
    const InstDesc t = tb3_desc(d, l);
    const int wpb = tb3_waves_per_block(d, l);
    const int blocks = t.rowblocks * ((t.strips + wpb - 1) / wpb);
    // odd row blocks march down, as in the two-step pass: each block
    // boundary's ten shared rows are read by both blocks at the same end
    // of their runs
    if (t.rowwalls)
        sweep_tb3_kernel<true><<<blocks, 64 * wpb, 0, stream>>>(t, src, tb3_xcd_remap(d, l), 1);
    else
        sweep_tb3_kernel<false><<<blocks, 64 * wpb, 0, stream>>>(t, src, tb3_xcd_remap(d, l), 1);
    return hipGetLastError();
}

hipError_t launch_sweep_tb3_batch(const InstDesc *descs, int ndescs, const int4 *items,
                                  int nitems, int storage, int flip, const Launch &l,
                                  hipStream_t stream) {
    if (storage != ST_F32) return hipErrorInvalidValue;
    if (nitems <= 0) return hipSuccess;
    const int wpb = batch_waves_per_block(l);
    const int blocks = (nitems + wpb - 1) / wpb;
    sweep_tb3_batch_kernel<<<blocks, 64 * wpb, 0, stream>>>(descs, ndescs, items, nitems, flip,
                                                            l.xcd_remap);
    return hipGetLastError();
}

hipError_t launch_sweep_batch(const InstDesc *descs, const int4 *items, int nitems, int storage,
                              bool mask, bool buf, int flip, int flip1, const Launch &l,
                              hipStream_t stream) {
    switch (storage * 2 + (mask ? 1 : 0)) {
        case 0: return launch_batch_b<ST_F64, false>(descs, items, nitems, flip, flip1, l, buf, stream);
        case 1: return launch_batch_b<ST_F64, true>(descs, items, nitems, flip, flip1, l, buf, stream);
        case 2: return launch_batch_b<ST_F32, false>(descs, items, nitems, flip, flip1, l, buf, stream);
        case 3: return launch_batch_b<ST_F32, true>(descs, items, nitems, flip, flip1, l, buf, stream);
        case 4: return launch_batch_b<ST_F16, false>(descs, items, nitems, flip, flip1, l, buf, stream);
        case 5: return launch_batch_b<ST_F16, true>(descs, items, nitems, flip, flip1, l, buf, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep_tb2_batch(const InstDesc *descs, int ndescs, const int4 *items,
                                  int nitems, int storage, int flip, bool deep, const Launch &l,
                                  hipStream_t stream) {
    if (nitems <= 0) return hipSuccess;
    const int wpb = batch_waves_per_block(l);
    const int blocks = (nitems + wpb - 1) / wpb;
    const int r = l.xcd_remap;
    const dim3 g(blocks), t(64 * wpb);
    if (storage == ST_F32) {
        if (deep)
            sweep_tb2_batch_kernel<ST_F32, 2><<<g, t, 0, stream>>>(descs, ndescs, items, nitems, flip, r);
        else
            sweep_tb2_batch_kernel<ST_F32, 1><<<g, t, 0, stream>>>(descs, ndescs, items, nitems, flip, r);
    } else if (storage == ST_F16) {
        if (deep)
            sweep_tb2_batch_kernel<ST_F16, 2><<<g, t, 0, stream>>>(descs, ndescs, items, nitems, flip, r);
        else
            sweep_tb2_batch_kernel<ST_F16, 1><<<g, t, 0, stream>>>(descs, ndescs, items, nitems, flip, r);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace trt
