// probe.hip -- the bandwidth ceiling of the sweep's memory access pattern.
//
// A measurement aid, not a step of the method: the kernel below moves a
// population lattice's bytes to the other lattice with the access pattern of
// the two-column sweep and none of its arithmetic.  Same launch shape (row
// blocks of `rows` rows, 128-column strips, workgroups of adjacent strips
// meeting one barrier per row, XCD remap), same loads per row -- each lane
// reads its column pair of the nine population rows from the source rows of
// the pull (y for populations 0, 1, 3; y - 1 for 2, 5, 6; y + 1 for 4, 7, 8),
// the strip's edge lanes also read the three elements beyond the strip and
// gather the halo node beyond it --
// with the next row's loads in flight while the current row is stored, and
// the same non-temporal stores of nine words per lane and row.  Its time per
// launch is what the sweep's access pattern costs on its own, so the sweep's
// time against it says how much of the sweep is memory pattern and how much
// anything else.
#include "kernels.hpp"

namespace trt {

namespace {

template <class T> struct ProbeWord;
template <> struct ProbeWord<_Float16> {
    typedef uint32_t W;
    __device__ static __forceinline__ W ld(const BufAccess<_Float16> &a, int64_t e, uint32_t v) {
        return __builtin_amdgcn_raw_buffer_load_b32(a.r, v, (uint32_t)(e * 2), 0);
    }
    __device__ static __forceinline__ void st(const BufAccess<_Float16> &a, int64_t e, uint32_t v,
                                              W w) {
        __builtin_amdgcn_raw_buffer_store_b32(w, a.r, v, (uint32_t)(e * 2), TRT_STORE_CPOL);
    }
    __device__ static __forceinline__ void mix(W &w, uint32_t x) { w ^= x; }
};
template <> struct ProbeWord<float> {
    typedef uint32_t __attribute__((ext_vector_type(2))) W;
    __device__ static __forceinline__ W ld(const BufAccess<float> &a, int64_t e, uint32_t v) {
        return __builtin_amdgcn_raw_buffer_load_b64(a.r, v, (uint32_t)(e * 4), 0);
    }
    __device__ static __forceinline__ void st(const BufAccess<float> &a, int64_t e, uint32_t v,
                                              W w) {
        __builtin_amdgcn_raw_buffer_store_b64(w, a.r, v, (uint32_t)(e * 4), TRT_STORE_CPOL);
    }
    __device__ static __forceinline__ void mix(W &w, uint32_t x) { w.x ^= x; }
};
template <> struct ProbeWord<double> {
    typedef uint32_t __attribute__((ext_vector_type(4))) W;
    __device__ static __forceinline__ W ld(const BufAccess<double> &a, int64_t e, uint32_t v) {
        return __builtin_amdgcn_raw_buffer_load_b128(a.r, v, (uint32_t)(e * 8), 0);
    }
    __device__ static __forceinline__ void st(const BufAccess<double> &a, int64_t e, uint32_t v,
                                              W w) {
        __builtin_amdgcn_raw_buffer_store_b128(w, a.r, v, (uint32_t)(e * 8), TRT_STORE_CPOL);
    }
    __device__ static __forceinline__ void mix(W &w, uint32_t x) { w.x ^= x; }
};

// Raw bits of one storage element (for folding the edge elements into a
// stored word, so that their loads are kept).
__device__ __forceinline__ uint32_t bits_of(_Float16 v) { return __builtin_bit_cast(unsigned short, v); }
__device__ __forceinline__ uint32_t bits_of(float v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ uint32_t bits_of(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    return (uint32_t)b ^ (uint32_t)(b >> 32);
}

// Source row offset (in elements) of population i for lattice row y: the
// pull reads row y - e_iy.
template <int I>
__device__ __forceinline__ int64_t src_row(int y, int ny, int pitch) {
    constexpr int ey = (I == 2 || I == 5 || I == 6) ? 1 : ((I == 4 || I == 7 || I == 8) ? -1 : 0);
    int r = y - ey;
    if (r < 0) r += ny;
    if (r >= ny) r -= ny;
    return (int64_t)r * pitch;
}

template <class T> struct ProbeRow {
    typename ProbeWord<T>::W w[9];
    uint32_t edge;
};

// An edge lane's halo node: its column and the wrapped columns on either side
// (byte offsets within a row).
struct HaloCols {
    uint32_t om, oc, op;
};

template <class T>
__device__ __forceinline__ void probe_load(ProbeRow<T> &r, const BufAccess<T> &in, int64_t plane,
                                           int pitch, int ny, int y, uint32_t opair, bool edge,
                                           const uint32_t ve[3], const HaloCols &h) {
    using P = ProbeWord<T>;
    r.w[0] = P::ld(in, src_row<0>(y, ny, pitch), opair);
    r.w[1] = P::ld(in, plane + src_row<1>(y, ny, pitch), opair);
    r.w[2] = P::ld(in, 2 * plane + src_row<2>(y, ny, pitch), opair);
    r.w[3] = P::ld(in, 3 * plane + src_row<3>(y, ny, pitch), opair);
    r.w[4] = P::ld(in, 4 * plane + src_row<4>(y, ny, pitch), opair);
    r.w[5] = P::ld(in, 5 * plane + src_row<5>(y, ny, pitch), opair);
    r.w[6] = P::ld(in, 6 * plane + src_row<6>(y, ny, pitch), opair);
    r.w[7] = P::ld(in, 7 * plane + src_row<7>(y, ny, pitch), opair);
    r.w[8] = P::ld(in, 8 * plane + src_row<8>(y, ny, pitch), opair);
    r.edge = 0u;
    if (edge) {
        // the three elements beyond the strip, from the rows the sweep's edge
        // lanes read them from (lane 0: populations 1, 5, 8; lane 63: 3, 6, 7)
        const int64_t e0 = (int64_t)y * pitch;
        const int64_t em = (int64_t)(y == 0 ? ny - 1 : y - 1) * pitch;
        const int64_t ep = (int64_t)(y == ny - 1 ? 0 : y + 1) * pitch;
        uint32_t x = bits_of(in.ld(e0, ve[0])) ^ bits_of(in.ld(em, ve[1])) ^
                     bits_of(in.ld(ep, ve[2]));
        // and the halo node's pull-gather (its Phi_x in the sweep)
        x ^= bits_of(in.ld(e0, h.oc)) ^ bits_of(in.ld(plane + e0, h.om)) ^
             bits_of(in.ld(2 * plane + em, h.oc)) ^ bits_of(in.ld(3 * plane + e0, h.op)) ^
             bits_of(in.ld(4 * plane + ep, h.oc)) ^ bits_of(in.ld(5 * plane + em, h.om)) ^
             bits_of(in.ld(6 * plane + em, h.op)) ^ bits_of(in.ld(7 * plane + ep, h.op)) ^
             bits_of(in.ld(8 * plane + ep, h.om));
        r.edge = x;
    }
}

template <int ST>
__global__ __launch_bounds__(ST == ST_F64 ? 512 : 1024) void pattern_probe_kernel(InstDesc d,
                                                                                  int srcsel,
                                                                                  int remap) {
    using T = typename Store<ST>::T;
    using P = ProbeWord<T>;
    int b = blockIdx.x;
    if (remap) b = xcd_remap(b, gridDim.x);
    const int wpb = blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int groups = (d.strips + wpb - 1) / wpb;
    const int rb = b / groups;
    const int strip = (b - rb * groups) * wpb + w;
    const int ny = d.ny, pitch = d.pitch;
    const int y0 = rb * d.rows;
    const int y1 = min(y0 + d.rows, ny);
    if (strip >= d.strips) {
        // no strip: meet the workgroup's barriers
        for (int y = y0; y < y1; ++y) __builtin_amdgcn_s_barrier();
        return;
    }
    const int lane = threadIdx.x & 63;
    const int64_t plane = d.plane;
    const T *src = static_cast<const T *>(srcsel ? d.buf[1] : d.buf[0]);
    T *dst = static_cast<T *>(srcsel ? d.buf[0] : d.buf[1]);
    const uint64_t bytes = (uint64_t)ny * (uint64_t)pitch * sizeof(T);
    const BufAccess<T> in(src, bytes), out(dst, bytes);
    // the host admits widths that are multiples of 128 only: every lane's
    // pair lies inside the row
    const int x0 = strip * 2 * kStripWidth;
    const uint32_t opair = (uint32_t)(x0 + 2 * lane) * (uint32_t)sizeof(T);
    const bool edge = lane == 0 || lane == 63;
    int hx = lane == 0 ? x0 - 1 : x0 + 2 * kStripWidth;
    if (hx < 0) hx += d.nx;
    if (hx >= d.nx) hx -= d.nx;
    const uint32_t hoff = (uint32_t)hx * (uint32_t)sizeof(T);
    const int hxm = hx == 0 ? d.nx - 1 : hx - 1, hxp = hx == d.nx - 1 ? 0 : hx + 1;
    const HaloCols hc{(uint32_t)hxm * (uint32_t)sizeof(T), hoff,
                      (uint32_t)hxp * (uint32_t)sizeof(T)};
    const int p0 = lane == 0 ? 1 : 3, p1 = lane == 0 ? 5 : 6, p2 = lane == 0 ? 8 : 7;
    const uint32_t ve[3] = {(uint32_t)(p0 * plane * (int64_t)sizeof(T)) + hoff,
                            (uint32_t)(p1 * plane * (int64_t)sizeof(T)) + hoff,
                            (uint32_t)(p2 * plane * (int64_t)sizeof(T)) + hoff};
    ProbeRow<T> cur, nxt;
    probe_load<T>(cur, in, plane, pitch, ny, y0, opair, edge, ve, hc);
    for (int y = y0; y < y1; ++y) {
        const bool more = y + 1 < y1;
        if (more) probe_load<T>(nxt, in, plane, pitch, ny, y + 1, opair, edge, ve, hc);
        P::mix(cur.w[1], cur.edge);
        const int64_t e0 = (int64_t)y * pitch;
#pragma unroll
        for (int i = 0; i < 9; ++i) P::st(out, i * plane + e0, opair, cur.w[i]);
        if (more) cur = nxt;
        __builtin_amdgcn_s_barrier();
    }
}

template <int ST>
hipError_t launch_probe_t(const InstDesc &d, int src, const Launch &l, hipStream_t s) {
    const int wpb = single_waves_per_block(d, ST, l);
    const int blocks = d.rowblocks * ((d.strips + wpb - 1) / wpb);
    pattern_probe_kernel<ST><<<blocks, 64 * wpb, 0, s>>>(d, src, l.xcd_remap);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_pattern_probe(const InstDesc &d, int storage, int src, const Launch &l,
                                hipStream_t stream) {
    if (d.cols != 2 || d.nx % (2 * kStripWidth) != 0 || d.links != nullptr ||
        !buffer_addressable(d, storage))
        return hipErrorInvalidValue;
    switch (storage) {
        case ST_F64: return launch_probe_t<ST_F64>(d, src, l, stream);
        case ST_F32: return launch_probe_t<ST_F32>(d, src, l, stream);
        case ST_F16: return launch_probe_t<ST_F16>(d, src, l, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace trt
