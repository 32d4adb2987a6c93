// fields.hip -- per-node kernels around the sweep: state initialisation and
// read-back, macroscopic fields, and FP64 diagnostics.
//
// The lattice holds the post-collision populations of the previous step, so
// the pre-collision state f(x, t) is obtained by the same pull-gather the
// sweep uses (periodic wrap, half-way bounce-back at solid sources), and
// written by the inverse scatter: f_i(x) goes to node x - e_i, or, when that
// node is solid, to slot opp(i) of x itself.
#include <math.h>

#include "../../include/trtlbm.h"
#include "kernels.hpp"

namespace trt {

namespace {

constexpr int kEx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kEy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

__device__ __forceinline__ double weight(int i) {
    return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
}

__device__ __forceinline__ int wrapi(int a, int n) {
    a %= n;
    return a < 0 ? a + n : a;
}

__device__ __forceinline__ bool is_solid(const uint8_t *mask, int nx, int x, int y) {
    return mask != nullptr && mask[(int64_t)y * nx + x] != 0;
}

// Scatter of one fluid node's pre-collision populations fi[9] (unshifted,
// FP64) into lattice `lat`.  With open x boundaries, the populations that
// enter column 0 through the inflow wall are stored in the slots the gather
// reads them back from (minus the wall's momentum correction), and the
// three that enter the outlet column from outside are not stored: the
// outlet rule determines them.
template <int ST>
__device__ __forceinline__ void scatter_node(const InstDesc &d, void *lat, int x, int y,
                                             const double fi[9]) {
    using T = typename Store<ST>::T;
    T *b = static_cast<T *>(lat);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        double v = Store<ST>::shifted ? fi[i] - weight(i) : fi[i];
        const int tx = x - kEx[i];
        if (d.xbc && tx >= d.nx) continue;
        const int sx = wrapi(tx, d.nx), sy = wrapi(y - kEy[i], d.ny);
        int64_t idx;
        if (d.xbc && tx < 0) {
            v -= (i == 1 ? 2.0 / 3.0 : 1.0 / 6.0) * (d.rho_in * d.u_in);
            idx = kOpp[i] * d.plane + (int64_t)y * d.pitch + x;
        } else if (is_solid(d.mask, d.nx, sx, sy)) {
            idx = kOpp[i] * d.plane + (int64_t)y * d.pitch + x;
        } else {
            idx = i * d.plane + (int64_t)sy * d.pitch + sx;
        }
        b[idx] = (T)v;
    }
}

// Pre-collision populations of node (x, y) in the arithmetic precision,
// including the open x boundaries' rules.
template <int ST>
__device__ __forceinline__ bool gather_state(const InstDesc &d, int srcsel, int x, int y,
                                             typename Store<ST>::C f[9]) {
    using T = typename Store<ST>::T;
    using C = typename Store<ST>::C;
    const int xm = (x == 0) ? d.nx - 1 : x - 1;
    const int xp = (x == d.nx - 1) ? 0 : x + 1;
    const bool solid = gather<T, C, true>(static_cast<const T *>(d.buf[srcsel]), d.plane, d.pitch,
                                          d.mask, d.nx, d.ny, y, xm, x, xp, f, d.xbc != 0);
    if (d.xbc)
        open_x_fix<C, Store<ST>::shifted>(f, x, d.nx, (C)d.u_in, (C)d.rho_in, (C)d.rho_out);
    return solid;
}

// Pre-collision populations of node (x, y), unshifted, FP64.
template <int ST>
__device__ __forceinline__ bool gather_node(const InstDesc &d, int srcsel, int x, int y,
                                            double fo[9]) {
    typename Store<ST>::C f[9];
    const bool solid = gather_state<ST>(d, srcsel, x, y, f);
#pragma unroll
    for (int i = 0; i < 9; ++i)
        fo[i] = Store<ST>::shifted ? (double)f[i] + weight(i) : (double)f[i];
    return solid;
}

template <int ST>
__global__ void set_populations_kernel(InstDesc d, int srcsel, const double *__restrict__ f) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= d.nx || y >= d.ny || is_solid(d.mask, d.nx, x, y)) return;
    const int64_t n = (int64_t)d.nx * d.ny, k = (int64_t)y * d.nx + x;
    double fi[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) fi[i] = f[i * n + k];
    scatter_node<ST>(d, d.buf[srcsel], x, y, fi);
}

template <int ST>
__global__ void init_equilibrium_kernel(InstDesc d, int srcsel, const double *__restrict__ rho,
                                        const double *__restrict__ ux,
                                        const double *__restrict__ uy) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= d.nx || y >= d.ny || is_solid(d.mask, d.nx, x, y)) return;
    const int64_t k = (int64_t)y * d.nx + x;
    double fi[9];
    equilibrium<double>(fi, rho[k], rho[k], ux[k], uy[k]);
    scatter_node<ST>(d, d.buf[srcsel], x, y, fi);
}

template <int ST>
__global__ void get_populations_kernel(InstDesc d, int srcsel, double *__restrict__ f) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= d.nx || y >= d.ny) return;
    const int64_t n = (int64_t)d.nx * d.ny, k = (int64_t)y * d.nx + x;
    double fi[9];
    const bool solid = gather_node<ST>(d, srcsel, x, y, fi);
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i * n + k] = solid ? 0.0 : fi[i];
}

// FP64 moments of the stored state (the storage values widened exactly).
template <int ST>
__device__ __forceinline__ bool node_moments(const InstDesc &d, int srcsel, int x, int y,
                                             Moments<double, Store<ST>::shifted> &m) {
    typename Store<ST>::C f[9];
    const bool solid = gather_state<ST>(d, srcsel, x, y, f);
    double fd[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) fd[i] = (double)f[i];
    m.compute(fd, d.gx, d.gy);
    return solid;
}

template <int ST>
__global__ void macros_kernel(InstDesc d, int srcsel, double *__restrict__ rho,
                              double *__restrict__ ux, double *__restrict__ uy) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= d.nx || y >= d.ny) return;
    const int64_t k = (int64_t)y * d.nx + x;
    Moments<double, Store<ST>::shifted> m;
    const bool solid = node_moments<ST>(d, srcsel, x, y, m);
    if (rho) rho[k] = solid ? 0.0 : m.rho;
    if (ux) ux[k] = solid ? 0.0 : m.ux;
    if (uy) uy[k] = solid ? 0.0 : m.uy;
}

constexpr int kDiagBlocks = 512;
constexpr int kDiagThreads = 256;

struct Acc {
    double v[TRT_NDIAG];
};

__device__ __forceinline__ void acc_init(Acc &a) {
    a.v[0] = a.v[1] = a.v[2] = 0.0;
    a.v[3] = 0.0;
    a.v[4] = a.v[5] = 0.0;
    a.v[6] = INFINITY;
    a.v[7] = 0.0;
}

__device__ __forceinline__ void acc_merge(Acc &a, const Acc &b) {
    a.v[0] += b.v[0];
    a.v[1] += b.v[1];
    a.v[2] += b.v[2];
    a.v[3] = fmax(a.v[3], b.v[3]);
    a.v[4] += b.v[4];
    a.v[5] += b.v[5];
    a.v[6] = fmin(a.v[6], b.v[6]);
}

// Fixed-shape reduction: thread -> nodes is a fixed grid-stride map and the
// tree below has a fixed order, so the result is bitwise reproducible.
__device__ void block_reduce(Acc &a) {
    __shared__ double sh[kDiagThreads / 64][TRT_NDIAG];
    for (int off = 32; off > 0; off >>= 1) {
        Acc o;
#pragma unroll
        for (int j = 0; j < TRT_NDIAG; ++j) o.v[j] = __shfl_down(a.v[j], off);
        acc_merge(a, o);
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
        for (int j = 0; j < TRT_NDIAG; ++j) sh[w][j] = a.v[j];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kDiagThreads / 64; ++k) {
            Acc o;
            for (int j = 0; j < TRT_NDIAG; ++j) o.v[j] = sh[k][j];
            acc_merge(a, o);
        }
    }
}

template <int ST>
__global__ __launch_bounds__(kDiagThreads) void diag_kernel(InstDesc d, int srcsel,
                                                           double *__restrict__ partials) {
    Acc a;
    acc_init(a);
    const int64_t n = (int64_t)d.nx * d.ny;
    for (int64_t k = (int64_t)blockIdx.x * kDiagThreads + threadIdx.x; k < n;
         k += (int64_t)kDiagBlocks * kDiagThreads) {
        const int y = (int)(k / d.nx), x = (int)(k - (int64_t)y * d.nx);
        Moments<double, Store<ST>::shifted> m;
        if (node_moments<ST>(d, srcsel, x, y, m)) continue;
        const double sp = sqrt(m.ux * m.ux + m.uy * m.uy);
        const bool bad = !isfinite(m.rho) || !isfinite(sp) || !(m.rho > 0.0) || !(sp < 1.0);
        a.v[5] += 1.0;
        if (bad) {
            a.v[4] += 1.0;
        }
        if (isfinite(m.rho) && isfinite(sp)) {
            a.v[0] += m.rho;
            a.v[1] += m.rho * m.ux;
            a.v[2] += m.rho * m.uy;
            a.v[3] = fmax(a.v[3], sp);
            a.v[6] = fmin(a.v[6], m.rho);
        }
    }
    block_reduce(a);
    if (threadIdx.x == 0)
        for (int j = 0; j < TRT_NDIAG; ++j) partials[blockIdx.x * TRT_NDIAG + j] = a.v[j];
}

__global__ void diag_final_kernel(const double *__restrict__ partials, double *__restrict__ out,
                                  double time) {
    if (threadIdx.x != 0) return;
    Acc a;
    acc_init(a);
    for (int b = 0; b < kDiagBlocks; ++b) {
        Acc o;
        for (int j = 0; j < TRT_NDIAG; ++j) o.v[j] = partials[b * TRT_NDIAG + j];
        acc_merge(a, o);
    }
    if (a.v[5] == 0.0 || a.v[6] == INFINITY) a.v[6] = 0.0;
    a.v[7] = time;
    for (int j = 0; j < TRT_NDIAG; ++j) out[j] = a.v[j];
}

template <int ST>
__global__ __launch_bounds__(256) void row_mean_kernel(InstDesc d, int srcsel,
                                                       double *__restrict__ out) {
    const int y = blockIdx.x;
    double s = 0.0, cnt = 0.0;
    for (int x = threadIdx.x; x < d.nx; x += 256) {
        Moments<double, Store<ST>::shifted> m;
        if (node_moments<ST>(d, srcsel, x, y, m)) continue;
        s += m.ux;
        cnt += 1.0;
    }
    for (int off = 32; off > 0; off >>= 1) {
        s += __shfl_down(s, off);
        cnt += __shfl_down(cnt, off);
    }
    __shared__ double sh[2][4];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[0][w] = s;
        sh[1][w] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double ts = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
        const double tc = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
        out[y] = tc > 0.0 ? ts / tc : 0.0;
    }
}

// Fixed-order block reduction of K sums (and, for K3MAX, a max in slot 0).
template <int K, bool MAX0>
__device__ void block_reduce_k(double v[K]) {
    __shared__ double sh[kDiagThreads / 64][K];
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const double o = __shfl_down(v[j], off);
            v[j] = (MAX0 && j == 0) ? fmax(v[j], o) : v[j] + o;
        }
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
        for (int j = 0; j < K; ++j) sh[w][j] = v[j];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 1; k < kDiagThreads / 64; ++k)
            for (int j = 0; j < K; ++j) v[j] = (MAX0 && j == 0) ? fmax(v[j], sh[k][j]) : v[j] + sh[k][j];
}

template <int K, bool MAX0>
__global__ void final_reduce_k(const double *__restrict__ partials, double *__restrict__ out) {
    if (threadIdx.x != 0) return;
    double v[K];
    for (int j = 0; j < K; ++j) v[j] = partials[j];
    for (int b = 1; b < kDiagBlocks; ++b)
        for (int j = 0; j < K; ++j)
            v[j] = (MAX0 && j == 0) ? fmax(v[j], partials[b * K + j]) : v[j] + partials[b * K + j];
    for (int j = 0; j < K; ++j) out[j] = v[j];
}

// Momentum exchange with solid nodes (Sec. III.D): every link from a fluid
// node x_f to a solid node x_f + e_i carries 2 e_i f*_i(x_f, t) under
// half-way bounce-back; f* is the lattice after the step (post-collision
// values stored at their own node).  Links leaving through open x ends are
// not wall links.
template <int ST>
__global__ __launch_bounds__(kDiagThreads) void wall_force_kernel(InstDesc d, int src,
                                                                 double *__restrict__ partials) {
    using T = typename Store<ST>::T;
    const T *b = static_cast<const T *>(d.buf[src]);
    double v[2] = {0.0, 0.0};
    const int64_t n = (int64_t)d.nx * d.ny;
    if (d.mask != nullptr) {
        for (int64_t k = (int64_t)blockIdx.x * kDiagThreads + threadIdx.x; k < n;
             k += (int64_t)kDiagBlocks * kDiagThreads) {
            const int y = (int)(k / d.nx), x = (int)(k - (int64_t)y * d.nx);
            if (d.mask[k]) continue;
            for (int i = 1; i < 9; ++i) {
                const int tx = x + kEx[i];
                if (d.xbc && (tx < 0 || tx >= d.nx)) continue;
                if (!is_solid(d.mask, d.nx, wrapi(tx, d.nx), wrapi(y + kEy[i], d.ny))) continue;
                const double fs = (double)b[i * d.plane + (int64_t)y * d.pitch + x] +
                                  (Store<ST>::shifted ? weight(i) : 0.0);
                v[0] += 2.0 * kEx[i] * fs;
                v[1] += 2.0 * kEy[i] * fs;
            }
        }
    }
    block_reduce_k<2, false>(v);
    if (threadIdx.x == 0) {
        partials[blockIdx.x * 2 + 0] = v[0];
        partials[blockIdx.x * 2 + 1] = v[1];
    }
}

// Velocity against a reference field over the fluid nodes: (max over nodes
// and components of |u - u_ref|, sum |u - u_ref|^2, sum |u|^2,
// sum |u_ref|^2); with `update` the reference is then replaced by u.
template <int ST>
__global__ __launch_bounds__(kDiagThreads) void velocity_compare_kernel(
    InstDesc d, int srcsel, double *__restrict__ rux, double *__restrict__ ruy, int update,
    double *__restrict__ partials) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t n = (int64_t)d.nx * d.ny;
    for (int64_t k = (int64_t)blockIdx.x * kDiagThreads + threadIdx.x; k < n;
         k += (int64_t)kDiagBlocks * kDiagThreads) {
        const int y = (int)(k / d.nx), x = (int)(k - (int64_t)y * d.nx);
        Moments<double, Store<ST>::shifted> m;
        if (node_moments<ST>(d, srcsel, x, y, m)) continue;
        const double ax = rux[k], ay = ruy[k];
        const double dx = m.ux - ax, dy = m.uy - ay;
        v[0] = fmax(v[0], fmax(fabs(dx), fabs(dy)));
        v[1] += dx * dx + dy * dy;
        v[2] += m.ux * m.ux + m.uy * m.uy;
        v[3] += ax * ax + ay * ay;
        if (update) {
            rux[k] = m.ux;
            ruy[k] = m.uy;
        }
    }
    block_reduce_k<4, true>(v);
    if (threadIdx.x == 0)
        for (int j = 0; j < 4; ++j) partials[blockIdx.x * 4 + j] = v[j];
}

__global__ void link_map_kernel(InstDesc d, uint16_t *__restrict__ links) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= d.nx || y >= d.ny) return;
    uint32_t b = is_solid(d.mask, d.nx, x, y) ? 1u : 0u;
    for (int i = 1; i < 9; ++i) {
        const int tx = x - kEx[i];
        if (d.xbc && tx < 0) {
            b |= 1u << i;  // beyond the inflow wall: own slot opp(i), plus the wall's correction
        } else if (d.xbc && tx >= d.nx) {
            // beyond the outlet: the outlet rule replaces f_i
        } else if (is_solid(d.mask, d.nx, wrapi(tx, d.nx), wrapi(y - kEy[i], d.ny))) {
            b |= 1u << i;
        }
    }
    links[(int64_t)y * d.lpitch + x] = (uint16_t)b;
}

// Link summary: entry (y, s) is the OR of the codes of row y over columns
// 64 s - 1 ... 64 s + 64, wrapped (entries past the lattice's width cover
// wrapped columns, as the sweep's lanes past the width do).
__global__ void link_summary_kernel(InstDesc d, const uint16_t *__restrict__ links,
                                    uint32_t *__restrict__ sum) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (s >= d.nsum || y >= d.ny) return;
    uint32_t acc = 0u;
    for (int k = -1; k <= 64; ++k) acc |= links[(int64_t)y * d.lpitch + wrapi(64 * s + k, d.nx)];
    sum[(int64_t)y * d.nsum + s] = acc;
}

// Whether the mask's solid nodes fill whole rows: one wavefront per row
// compares every node with the row's first, and a row that differs sets
// *mixed (every writer stores the same 1).
__global__ void mask_rows_kernel(const uint8_t *__restrict__ mask, int nx, int ny,
                                 int *__restrict__ mixed) {
    const int y = blockIdx.x;
    if (y >= ny) return;
    const uint8_t *row = mask + (int64_t)y * nx;
    const bool first = row[0] != 0;
    bool diff = false;
    for (int x = (int)threadIdx.x; x < nx; x += 64) diff |= (row[x] != 0) != first;
    if (__builtin_amdgcn_ballot_w64(diff) != 0 && threadIdx.x == 0) *mixed = 1;
}

dim3 node_grid(const InstDesc &d) { return dim3((d.nx + 63) / 64, (d.ny + 3) / 4); }

#define TRT_DISPATCH(storage, CALL)                 \
    switch (storage) {                              \
        case ST_F64: { constexpr int S = ST_F64; CALL; break; } \
        case ST_F32: { constexpr int S = ST_F32; CALL; break; } \
        case ST_F16: { constexpr int S = ST_F16; CALL; break; } \
        default: return hipErrorInvalidValue;       \
    }

}  // namespace

hipError_t launch_link_map(const InstDesc &d, hipStream_t stream) {
    link_map_kernel<<<node_grid(d), dim3(64, 4), 0, stream>>>(d, const_cast<uint16_t *>(d.links));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    link_summary_kernel<<<dim3((d.nsum + 63) / 64, d.ny), 64, 0, stream>>>(
        d, d.links, const_cast<uint32_t *>(d.rowsum));
    return hipGetLastError();
}

hipError_t launch_mask_rows(const uint8_t *mask, int nx, int ny, int *mixed, hipStream_t stream) {
    hipError_t e = hipMemsetAsync(mixed, 0, sizeof(int), stream);
    if (e != hipSuccess) return e;
    mask_rows_kernel<<<ny, 64, 0, stream>>>(mask, nx, ny, mixed);
    return hipGetLastError();
}

hipError_t launch_set_populations(const InstDesc &d, int storage, int src, const double *f,
                                  hipStream_t stream) {
    TRT_DISPATCH(storage, (set_populations_kernel<S><<<node_grid(d), dim3(64, 4), 0, stream>>>(d, src, f)));
    return hipGetLastError();
}

hipError_t launch_init_equilibrium(const InstDesc &d, int storage, int src, const double *rho,
                                   const double *ux, const double *uy, hipStream_t stream) {
    TRT_DISPATCH(storage, (init_equilibrium_kernel<S><<<node_grid(d), dim3(64, 4), 0, stream>>>(d, src, rho, ux, uy)));
    return hipGetLastError();
}

hipError_t launch_get_populations(const InstDesc &d, int storage, int src, double *f,
                                  hipStream_t stream) {
    TRT_DISPATCH(storage, (get_populations_kernel<S><<<node_grid(d), dim3(64, 4), 0, stream>>>(d, src, f)));
    return hipGetLastError();
}

hipError_t launch_macros(const InstDesc &d, int storage, int src, double *rho, double *ux,
                         double *uy, hipStream_t stream) {
    TRT_DISPATCH(storage, (macros_kernel<S><<<node_grid(d), dim3(64, 4), 0, stream>>>(d, src, rho, ux, uy)));
    return hipGetLastError();
}

int diag_partial_count() { return kDiagBlocks; }

hipError_t launch_diagnostics(const InstDesc &d, int storage, int src, double *partials,
                              double *out, double time, hipStream_t stream) {
    TRT_DISPATCH(storage, (diag_kernel<S><<<kDiagBlocks, kDiagThreads, 0, stream>>>(d, src, partials)));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    diag_final_kernel<<<1, 64, 0, stream>>>(partials, out, time);
    return hipGetLastError();
}

hipError_t launch_wall_force(const InstDesc &d, int storage, int src, double *partials,
                             double *out, hipStream_t stream) {
    TRT_DISPATCH(storage, (wall_force_kernel<S><<<kDiagBlocks, kDiagThreads, 0, stream>>>(d, src, partials)));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    final_reduce_k<2, false><<<1, 64, 0, stream>>>(partials, out);
    return hipGetLastError();
}

hipError_t launch_velocity_compare(const InstDesc &d, int storage, int src, double *ref_ux,
                                   double *ref_uy, bool update, double *partials, double *out,
                                   hipStream_t stream) {
    TRT_DISPATCH(storage, (velocity_compare_kernel<S><<<kDiagBlocks, kDiagThreads, 0, stream>>>(d, src, ref_ux, ref_uy, update ? 1 : 0, partials)));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    final_reduce_k<4, true><<<1, 64, 0, stream>>>(partials, out);
    return hipGetLastError();
}

hipError_t launch_row_mean_ux(const InstDesc &d, int storage, int src, double *out,
                              hipStream_t stream) {
    TRT_DISPATCH(storage, (row_mean_kernel<S><<<d.ny, 256, 0, stream>>>(d, src, out)));
    return hipGetLastError();
}

}  // namespace trt
