// lattice.hpp -- D2Q9 TRT-RLB building blocks shared by the device kernels.
//
// Notation follows Yu et al., arXiv:2312.10318, Sec. II.B: populations f_i,
// velocities e_i in the order (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1)
// (-1,-1) (1,-1), weights w = 4/9, 1/9 x4, 1/36 x4, c_s^2 = 1/3 (lattice
// units, dx = dt = c = 1).
//
// The collision is evaluated in Hermite-coefficient form.  Every term of the
// evolution equation (Eq. 2) -- the third-order equilibrium (Eq. 5), the
// regularized non-equilibrium of orders 1-3 (Eq. 6, with the equilibrium
// moments of Eq. 7), the compensation G_i (Eq. 8) and the force F_i
// (Eq. 11) -- is a combination of the same Hermite polynomials, so the
// post-collision state is
//   f*_i = w_i [ b0 + 3 (e_x b_x + e_y b_y)
//               + 9/2 (H_xx b_xx + 2 H_xy b_xy + H_yy b_yy)
//               + 27/2 (H_xxy b_xxy + H_xyy b_xyy) ]
// with seven coefficients collected once per node:
//   b_x   = j_x + F_x                         (order 1: rho u + (1-1/tau1) A + (1-1/(2tau1)) F)
//   b_xx  = rho u_x^2 + w1 A_xx + phi (2 F_x u_x - dPhi_x)
//   b_xy  = rho u_x u_y + w1 A_xy + phi (F_x u_y + u_x F_y)
//   b_xxy = rho u_x^2 u_y + w2 A_xxy          (and symmetric in x <-> y)
// where w1 = 1 - 1/tau_s1, w2 = 1 - 1/tau_s2, phi = 1 - 1/(2 tau_s1), and the
// A's are the non-equilibrium Hermite moments sum_i H_i (f_i - f_i^eq).  The
// per-direction reconstruction below is that sum with the D2Q9 values of
// H_xx, H_yy (2/3 or -1/3), H_xy (0, +-1), H_xxy = H_xx e_y and
// H_xyy = H_yy e_x (Sec. II.B) substituted.
//
// Shifted storage keeps g_i = f_i - w_i.  Since sum_i w_i = 1,
// sum_i e_i w_i = 0, sum_i e_x^2 w_i = 1/3 and sum_i e_x^2 e_y w_i = 0, every
// formula holds with f replaced by g once rho is replaced by
// delta_rho = rho - 1 wherever it stands alone (the "base" below); the output
// is then f*_i - w_i directly.  This keeps the O(1) rest weights out of the
// low-precision arithmetic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace trt {

enum StorageKind : int { ST_F64 = 0, ST_F32 = 1, ST_F16 = 2 };

template <int ST> struct Store;
template <> struct Store<ST_F64> {
    using T = double;
    using C = double;
    static constexpr bool shifted = false;
};
template <> struct Store<ST_F32> {
    using T = float;
    using C = float;
    static constexpr bool shifted = true;
};
template <> struct Store<ST_F16> {
    using T = _Float16;
    using C = float;
    static constexpr bool shifted = true;
};

// Columns one wavefront produces (one per lane).
constexpr int kStripWidth = 64;

// Everything one instance's sweep needs.  buf[0], buf[1] are the caller's
// two lattices; the step reading buf[s] writes buf[1 - s].
struct InstDesc {
    void *buf[2];
    const uint8_t *mask;  // dense [ny][nx] or null
    // link map [ny][lpitch] of 16-bit codes (null without mask and open
    // boundaries): per node, bit 0 = the node is solid, bit i (1..8) = the
    // pull source x - e_i is a solid node or the inflow wall, so f_i comes
    // back from the node's own slot opp(i) (half-way bounce-back)
    const uint16_t *links;
    int64_t lpitch;  // elements
    // link summary [ny][nsum] (with the link map): for row y and 64-column
    // strip s, the OR of the codes of columns 64 s - 1 ... 64 s + 64 (the
    // strip and the column on either side, wrapped); 0 means the strip's
    // pulls and halo need no link step in that row.  nsum is even, so a
    // 128-column strip k reads entries 2k and 2k + 1.
    const uint32_t *rowsum;
    int32_t nsum;
    // 1: every row of the mask is all solid or all fluid (walls parallel to
    // x) and x is periodic; a row's state is then bit 0 of its first
    // summary entry, and FP32 passes of several steps apply
    int32_t rowwalls;
    // population lattice layout [y][i][x]: f_i of node (x, y) is element
    // y * pitch + i * plane + x
    int64_t plane;        // elements between populations i and i+1 of a node
    int32_t nx, ny, pitch;  // pitch: elements between node rows y and y+1
    int32_t cur;          // lattice holding the state when the descriptor was built
    int32_t strips, rowblocks, rows;
    int32_t cols;         // columns per lane of the sweep: 1 or 2 (two-column strips)
    double omega1, omega2, phi, gx, gy;
    // open x boundaries (xbc = 1): inflow wall at x = -1/2 moving with
    // (u_in, 0) at density rho_in, pressure outlet at x = nx - 1 held at
    // rho_out; xbc = 0: periodic in x
    int32_t xbc;
    int32_t pad2_;
    double u_in, rho_in, rho_out;
};

// Products w_i * X.  In FP32 the rounded weights fl(4/9), fl(1/9), fl(1/36)
// all exceed the true weights by about 7.5e-9 (relative); applied every step
// to every population, that bias accumulates coherently in the momentum
// (about 1e-5 relative after 1000 steps).  The FP32 product is therefore
// formed as fma(w_hi, X, w_lo * X) with w_lo = w - w_hi, which rounds
// w * X correctly up to a tiny term; in FP64 the bias is negligible.
template <class C> struct Wt;
template <> struct Wt<double> {
    __device__ static __forceinline__ double w0(double x) { return (4.0 / 9.0) * x; }
    __device__ static __forceinline__ double w1(double x) { return (1.0 / 9.0) * x; }
    __device__ static __forceinline__ double w5(double x) { return (1.0 / 36.0) * x; }
};
template <> struct Wt<float> {
    static constexpr float h0 = (float)(4.0 / 9.0), h1 = (float)(1.0 / 9.0),
                           h5 = (float)(1.0 / 36.0);
    static constexpr float l0 = (float)(4.0 / 9.0 - (double)h0),
                           l1 = (float)(1.0 / 9.0 - (double)h1),
                           l5 = (float)(1.0 / 36.0 - (double)h5);
    __device__ static __forceinline__ float w0(float x) { return __builtin_fmaf(h0, x, l0 * x); }
    __device__ static __forceinline__ float w1(float x) { return __builtin_fmaf(h1, x, l1 * x); }
    __device__ static __forceinline__ float w5(float x) { return __builtin_fmaf(h5, x, l5 * x); }
};

__device__ __forceinline__ double to_c(double v) { return v; }
__device__ __forceinline__ float to_c(float v) { return v; }
__device__ __forceinline__ float to_c(_Float16 v) { return (float)v; }

template <class T, class C> __device__ __forceinline__ T from_c(C v) { return (T)v; }

// Reciprocal of the density.  FP32: the hardware estimate refined by one
// Newton step (error ~1e-14 before the final rounding), which removes the
// estimate's systematic error for rho close to 1 -- that error would bias
// the velocity coherently from step to step -- at a third of the cost of a
// correctly rounded division.  FP64: correctly rounded division.
__device__ __forceinline__ double recip(double r) { return 1.0 / r; }
__device__ __forceinline__ float recip(float r) {
    const float y = __builtin_amdgcn_rcpf(r);
    const float e = __builtin_fmaf(-r, y, 1.0f);
    return __builtin_fmaf(e, y, y);
}

// Moments of one node (Eqs. 12-13): base = sum_i f_i (shifted: delta rho),
// rho, j = sum_i e_i f_i, and the He-shifted velocity u = j / rho + g / 2
// (F = rho g, so (j + F/2) / rho = j / rho + g / 2); plus the raw moments the
// collision needs, sum e_x^2 f, sum e_y^2 f, sum e_x e_y f, sum e_x^2 e_y f and
// sum e_x e_y^2 f, which share partial sums with rho and j.  Once these are
// formed the nine populations are no longer needed.
template <class C, bool SHIFTED> struct Moments {
    C base, rho, jx, jy, ux, uy;
    C pxx, pyy, pxy, qxxy, qxyy;
    __device__ __forceinline__ void compute(const C f[9], C gx, C gy) {
        const C a13 = f[1] + f[3];
        finish(f[5] + f[6], f[5] - f[6], f[7] + f[8], f[7] - f[8], a13, f[1] - f[3],
               f[2] + f[4], f[2] - f[4], f[0] + a13, gx, gy);
    }
    // The same from the sums and differences of opposite populations
    // (f0a13 = f_0 + (f_1 + f_3)).
    __device__ __forceinline__ void finish(C s56, C d56, C s78, C d78, C a13, C m13, C a24, C m24,
                                           C f0a13, C gx, C gy) {
        const C diag = s56 + s78;
        qxxy = s56 - s78;
        pxy = d56 + d78;
        qxyy = d56 - d78;
        pxx = a13 + diag;
        pyy = a24 + diag;
        jx = m13 + qxyy;
        jy = m24 + qxxy;
        base = f0a13 + (a24 + diag);
        rho = SHIFTED ? C(1) + base : base;
        const C inv = recip(rho);
        ux = jx * inv + C(0.5) * gx;
        uy = jy * inv + C(0.5) * gy;
    }
};

// Sums of FP16 populations held in halves of 32-bit registers, formed in
// FP32 without separate conversions (FP16 to FP32 is exact, so each result
// is the FP32 sum of the converted values): a + b or a - b of the high (HI)
// or low halves of a and b, and h + c of one half of h and an FP32 c.  The
// operands are 32-bit words (uint32_t) or single FP16 values (_Float16, in
// the low half of their register, passed without widening).
template <bool HI, bool NEG, class U>
__device__ __forceinline__ float hsum(U a, U b) {
    static_assert(sizeof(U) == 4 || sizeof(U) == 2, "a word or an FP16 value");
    float r;
    if (HI && NEG)
        asm("v_fma_mix_f32 %0, %1, 1.0, -%2 op_sel:[1,0,1] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(a), "v"(b));
    else if (HI)
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,1] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(a), "v"(b));
    else if (NEG)
        asm("v_fma_mix_f32 %0, %1, 1.0, -%2 op_sel:[0,0,0] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(a), "v"(b));
    else
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[0,0,0] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
template <bool HI, class U>
__device__ __forceinline__ float hadd(U h, float c) {
    float r;
    if (HI)
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(h), "v"(c));
    else
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[0,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(h), "v"(c));
    return r;
}

// f_i from the seven Hermite coefficients (see the file comment).
template <class C>
__device__ __forceinline__ void reconstruct(C f[9], C base, C bx, C by, C bxx, C byy, C bxy,
                                            C bxxy, C bxyy) {
    f[0] = Wt<C>::w0(base - C(1.5) * (bxx + byy));
    const C ax = base + C(3) * bxx - C(1.5) * byy;
    const C dx = C(3) * bx - C(4.5) * bxyy;
    f[1] = Wt<C>::w1(ax + dx);
    f[3] = Wt<C>::w1(ax - dx);
    const C ay = base + C(3) * byy - C(1.5) * bxx;
    const C dy = C(3) * by - C(4.5) * bxxy;
    f[2] = Wt<C>::w1(ay + dy);
    f[4] = Wt<C>::w1(ay - dy);
    const C s = base + C(3) * (bxx + byy);
    const C sp = s + C(9) * bxy, sm = s - C(9) * bxy;
    const C d57 = C(3) * (bx + by) + C(9) * (bxxy + bxyy);
    const C d68 = C(3) * (by - bx) + C(9) * (bxxy - bxyy);
    f[5] = Wt<C>::w5(sp + d57);
    f[7] = Wt<C>::w5(sp - d57);
    f[6] = Wt<C>::w5(sm + d68);
    f[8] = Wt<C>::w5(sm - d68);
}

// FP16 storage.  Opposite directions share the even part of the
// reconstruction above and differ in the sign of its odd part:
// f*_i - w_i = w_i X + s w_i Y with s = +1 for i = 1, 2, 5, 6 and -1 for their
// opposites 3, 4, 7, 8, and f*_0 - w_0 = w_0 X_0.  X and Y are the FP32
// values the reconstruction forms (ax and dx for the pair (1,3), ay and dy
// for (2,4), s +- 9 b_xy and the diagonal odd parts for (5,7) and (6,8));
// here w_i X is formed once per pair and every output is one mixed-precision
// multiply-add, s Y w_i + (w_i X), rounded once from its exact value to FP16
// and written into one half of a 32-bit register.  The FP32 roundings before
// it (of X, Y, w_i X and of w_i itself) lie far below FP16 resolution, so the
// weights need none of the FP32 path's care.
struct HalfPairs {
    float x0;     // X_0
    float wx[4];  // w_i X of the pairs (1,3), (2,4), (5,7), (6,8)
    float y[4];   // their Y
};

__device__ __forceinline__ void reconstruct_pairs(HalfPairs &p, float base, float bx, float by,
                                                  float bxx, float byy, float bxy, float bxxy,
                                                  float bxyy) {
    p.x0 = base - 1.5f * (bxx + byy);
    const float ax = base + 3.0f * bxx - 1.5f * byy;
    p.y[0] = 3.0f * bx - 4.5f * bxyy;
    const float ay = base + 3.0f * byy - 1.5f * bxx;
    p.y[1] = 3.0f * by - 4.5f * bxxy;
    const float s = base + 3.0f * (bxx + byy);
    const float sp = s + 9.0f * bxy, sm = s - 9.0f * bxy;
    p.y[2] = 3.0f * (bx + by) + 9.0f * (bxxy + bxyy);
    p.y[3] = 3.0f * (by - bx) + 9.0f * (bxxy - bxyy);
    p.wx[0] = Wt<float>::h1 * ax;
    p.wx[1] = Wt<float>::h1 * ay;
    p.wx[2] = Wt<float>::h5 * sp;
    p.wx[3] = Wt<float>::h5 * sm;
}

// fma(s a, b, c) rounded once to FP16 into the low (LO) or high half of r;
// the other half of r is kept.  The instructions take FP32 operands.
template <bool NEG>
__device__ __forceinline__ uint32_t mix_lo(float a, float b, float c) {
    uint32_t r;
    if (NEG)
        asm("v_fma_mixlo_f16 %0, -%1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    else
        asm("v_fma_mixlo_f16 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
template <bool NEG>
__device__ __forceinline__ uint32_t mix_hi(uint32_t r, float a, float b, float c) {
    if (NEG)
        asm("v_fma_mixhi_f16 %0, -%1, %2, %3" : "+v"(r) : "v"(a), "v"(b), "v"(c));
    else
        asm("v_fma_mixhi_f16 %0, %1, %2, %3" : "+v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// Population i of one node in the low half of a register (HI: the high half
// of r instead, its low half kept).
template <int I, bool HI>
__device__ __forceinline__ uint32_t half_out(const HalfPairs &p, uint32_t r = 0u) {
    constexpr int k = I == 0 ? 0 : (I == 1 || I == 3) ? 0 : (I == 2 || I == 4) ? 1 : (I == 5 || I == 7) ? 2 : 3;
    constexpr bool neg = I == 3 || I == 4 || I == 7 || I == 8;
    const float w = I == 0 ? Wt<float>::h0 : I < 5 ? Wt<float>::h1 : Wt<float>::h5;
    const float a = I == 0 ? w : p.y[k];
    const float b = I == 0 ? p.x0 : w;
    const float c = I == 0 ? 0.0f : p.wx[k];
    if (HI) return mix_hi<neg>(r, a, b, c);
    return mix_lo<neg>(a, b, c);
}

// Third-order Hermite equilibrium (Eq. 5) in coefficient form: the
// equilibrium moments of Eq. 7 are rho u, rho u u and rho u_x^2 u_y,
// rho u_x u_y^2.  base = rho (or rho - 1 for shifted output).
template <class C>
__device__ __forceinline__ void equilibrium(C f[9], C base, C rho, C ux, C uy) {
    const C rux = rho * ux, ruy = rho * uy;
    const C exy = rux * uy;
    reconstruct<C>(f, base, rux, ruy, rux * ux, ruy * uy, exy, exy * ux, exy * uy);
}

// Hermite coefficients of the post-collision state of one node (Eq. 2),
// except for the y-gradient of Phi, which the sweep adds to b_yy once the
// row above has been gathered (-phi * dPhi_y).
template <class C> struct Coeffs {
    C base, bx, by, bxx, byy, bxy, bxxy, bxyy;
};

template <class C, bool SHIFTED>
__device__ __forceinline__ Coeffs<C> collide_coeffs(const Moments<C, SHIFTED> &m, C dphix, C w1,
                                                    C w2, C phi, C gx, C gy) {
    const C third = C(1) / C(3);
    const C Fx = m.rho * gx, Fy = m.rho * gy;
    // equilibrium Hermite moments (Eq. 7)
    const C rux = m.rho * m.ux, ruy = m.rho * m.uy;
    const C exx = rux * m.ux, eyy = ruy * m.uy, exy = rux * m.uy;
    const C exxy = exy * m.ux, exyy = exy * m.uy;
    // non-equilibrium Hermite moments (Eq. 6) from the raw moments
    const C axx = m.pxx - m.base * third - exx;
    const C ayy = m.pyy - m.base * third - eyy;
    const C axy = m.pxy - exy;
    const C axxy = m.qxxy - m.jy * third - exxy;
    const C axyy = m.qxyy - m.jx * third - exyy;
    // collected Hermite coefficients of f* (relaxation + G_i + F_i)
    Coeffs<C> c;
    c.base = m.base;
    c.bx = m.jx + Fx;
    c.by = m.jy + Fy;
    c.bxx = exx + w1 * axx + phi * (C(2) * Fx * m.ux - dphix);
    c.byy = eyy + w1 * ayy + phi * (C(2) * Fy * m.uy);
    c.bxy = exy + w1 * axy + phi * (Fx * m.uy + m.ux * Fy);
    c.bxxy = exxy + w2 * axxy;
    c.bxyy = exyy + w2 * axyy;
    return c;
}

// Collision of one node, Eq. 2 (the post-collision state is written to f).
template <class C, bool SHIFTED>
__device__ __forceinline__ void collide(C f[9], const Moments<C, SHIFTED> &m, C dphix, C dphiy,
                                        C w1, C w2, C phi, C gx, C gy) {
    Coeffs<C> c = collide_coeffs<C, SHIFTED>(m, dphix, w1, w2, phi, gx, gy);
    reconstruct<C>(f, c.base, c.bx, c.by, c.bxx, c.byy - phi * dphiy, c.bxy, c.bxxy, c.bxyy);
}

// Load of one element at a wave-uniform base plus a per-lane byte offset
// below 4 GiB: this form maps onto the scalar-base + 32-bit vector-offset
// global load, so a lane keeps three column offsets instead of nine 64-bit
// addresses.
// The base goes through readfirstlane so that loop strength reduction cannot
// fold it into per-lane 64-bit induction pointers, and is re-typed as a
// global (address space 1) pointer so that the access stays a global (not a
// flat) memory instruction.
template <class T> using gptr = __attribute__((address_space(1))) T *;

template <class T> __device__ __forceinline__ uint64_t wave_uniform_addr(const T *p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

template <class T>
__device__ __forceinline__ T ld_at(const T *__restrict__ base, uint32_t off) {
    const uint64_t b = wave_uniform_addr(base);
    return *(gptr<const T>)(b + off);
}
template <class T>
__device__ __forceinline__ void st_at(T *__restrict__ base, uint32_t off, T v) {
    const uint64_t b = wave_uniform_addr(base);
    *(gptr<T>)(b + off) = v;
}

// Buffer-instruction access to a lattice of at most 4 GiB: a 128-bit buffer
// resource (base, byte range) in scalar registers, a wave-uniform byte
// offset (population plane and row) in a scalar register and the lane's
// column byte offset in one vector register.  Every access is range-checked
// by the hardware against the lattice size.  The third descriptor word is
// the gfx9-family raw-buffer format (32-bit data format, as used by the ROCm
// composable-kernel library for these targets).
constexpr uint32_t kRawBufferWord3 = 0x00020000u;
// Cache-policy bits of the sweep's population stores.
#ifndef TRT_STORE_CPOL
#define TRT_STORE_CPOL 2  // nt: streaming stores (measured +1.5-2% on the sweep)
#endif

template <class T> struct BufAccess {
    __amdgpu_buffer_rsrc_t r;
    __device__ __forceinline__ BufAccess(const void *base, uint64_t bytes) {
        r = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0,
                                              (int)(uint32_t)(bytes > 0xffffffffull ? 0xffffffffull : bytes),
                                              (int)kRawBufferWord3);
    }
    __device__ __forceinline__ T ld(int64_t elem, uint32_t voff) const;
    __device__ __forceinline__ void st(int64_t elem, uint32_t voff, T v) const;
};
template <> __device__ __forceinline__ float BufAccess<float>::ld(int64_t e, uint32_t v) const {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, (uint32_t)(e * 4), 0));
}
template <> __device__ __forceinline__ void BufAccess<float>::st(int64_t e, uint32_t v, float x) const {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), r, v, (uint32_t)(e * 4), TRT_STORE_CPOL);
}
template <> __device__ __forceinline__ _Float16 BufAccess<_Float16>::ld(int64_t e, uint32_t v) const {
    return __builtin_bit_cast(_Float16,
                              (unsigned short)__builtin_amdgcn_raw_buffer_load_b16(r, v, (uint32_t)(e * 2), 0));
}
template <> __device__ __forceinline__ void BufAccess<_Float16>::st(int64_t e, uint32_t v, _Float16 x) const {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, x), r, v, (uint32_t)(e * 2), TRT_STORE_CPOL);
}
template <> __device__ __forceinline__ double BufAccess<double>::ld(int64_t e, uint32_t v) const {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, (uint32_t)(e * 8), 0));
}
template <> __device__ __forceinline__ void BufAccess<double>::st(int64_t e, uint32_t v, double x) const {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, v, (uint32_t)(e * 8), TRT_STORE_CPOL);
}

// Pointer access (any lattice size): wave-uniform element offset + lane
// byte offset through the global-address-space helpers above.
template <class T> struct PtrAccess {
    T *p;
    __device__ __forceinline__ PtrAccess(const void *base, uint64_t) : p((T *)base) {}
    __device__ __forceinline__ T ld(int64_t e, uint32_t v) const { return ld_at<T>(p + e, v); }
    __device__ __forceinline__ void st(int64_t e, uint32_t v, T x) const { st_at<T>(p + e, v, x); }
};

// Access to the link map through one buffer resource: trt_create refuses
// problems whose map would reach 4 GiB, so the byte range and the byte
// offsets 2 * (row * lpitch + col) below fit in 32 bits.  Offsets are in
// elements (16-bit codes).
struct LinkAccess {
    __amdgpu_buffer_rsrc_t r;
    __device__ __forceinline__ LinkAccess(const uint16_t *base, uint64_t elems) {
        r = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t *>(base), 0,
                                              (int)(uint32_t)(2 * elems), (int)kRawBufferWord3);
    }
    // the code of node (col, row): row_off = row * lpitch
    __device__ __forceinline__ uint32_t ld1(uint32_t row_off, uint32_t col) const {
        return __builtin_amdgcn_raw_buffer_load_b16(r, 2 * col, 2 * row_off, 0);
    }
    // the codes of nodes col (low half) and col + 1 (high half), col even
    __device__ __forceinline__ uint32_t ld2(uint32_t row_off, uint32_t col) const {
        return __builtin_amdgcn_raw_buffer_load_b32(r, 2 * col, 2 * row_off, 0);
    }
};

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

constexpr int kOppDir[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

// The link summary of a row, read with scalar loads (row and strip are
// wave-uniform), so deciding whether a row needs its link codes and own-slot
// loads never waits on vector memory.
struct RowSum {
    const __attribute__((address_space(4))) uint32_t *p;
    int nsum;
    __device__ __forceinline__ RowSum(const uint32_t *q, int n)
        : p((const __attribute__((address_space(4))) uint32_t *)q), nsum(n) {}
    // 64-column strip s of row y
    __device__ __forceinline__ uint32_t one(int y, int s) const {
        return p[(int64_t)y * nsum + s];
    }
    // 128-column strip k of row y (64-column strips 2k and 2k + 1)
    __device__ __forceinline__ uint32_t two(int y, int k) const {
        const int64_t i = (int64_t)y * nsum + 2 * k;
        return p[i] | p[i + 1];
    }
};

template <class T>
__device__ __forceinline__ void open_x_sources(const T *a[9], const T *r0, int64_t plane, int xc,
                                               int nx);

// Pull-gather of the pre-collision populations f_i(x, t) of node (xc, y)
// from the previous step's post-collision lattice: f_i(x, t) =
// f*_i(x - e_i, t - 1), or, when x - e_i is solid, the half-way bounce-back
// value f*_opp(i)(x, t - 1) stored at the node itself (Sec. II.D).
// xm, xp are the wrapped neighbour columns.  Returns whether the node is solid.
template <class T, class C, bool MASK>
__device__ __forceinline__ bool gather(const T *__restrict__ src, int64_t plane, int pitch,
                                       const uint8_t *__restrict__ mask, int nx, int ny, int y,
                                       int xm, int xc, int xp, C f[9], bool xbc = false) {
    const int ym = (y == 0) ? ny - 1 : y - 1;
    const int yp = (y == ny - 1) ? 0 : y + 1;
    const T *r0 = src + (int64_t)y * pitch;
    const T *rm = src + (int64_t)ym * pitch;
    const T *rp = src + (int64_t)yp * pitch;
    const T *a[9] = {r0 + xc,
                     r0 + plane + xm,
                     rm + 2 * plane + xc,
                     r0 + 3 * plane + xp,
                     rp + 4 * plane + xc,
                     rm + 5 * plane + xm,
                     rm + 6 * plane + xp,
                     rp + 7 * plane + xp,
                     rp + 8 * plane + xm};
    bool solid = false;
    if (MASK && mask != nullptr) {
        const uint8_t *mm = mask + (int64_t)ym * nx;
        const uint8_t *m0 = mask + (int64_t)y * nx;
        const uint8_t *mp = mask + (int64_t)yp * nx;
        solid = m0[xc] != 0;
        if (m0[xm]) a[1] = r0 + 3 * plane + xc;
        if (mm[xc]) a[2] = r0 + 4 * plane + xc;
        if (m0[xp]) a[3] = r0 + 1 * plane + xc;
        if (mp[xc]) a[4] = r0 + 2 * plane + xc;
        if (mm[xm]) a[5] = r0 + 7 * plane + xc;
        if (mm[xp]) a[6] = r0 + 8 * plane + xc;
        if (mp[xp]) a[7] = r0 + 5 * plane + xc;
        if (mp[xm]) a[8] = r0 + 6 * plane + xc;
    }
    if (xbc) open_x_sources(a, r0, plane, xc, nx);
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = to_c(a[i][0]);
    return solid;
}

// ---------------------------------------------------------------------------
// Open x boundaries (the creeping flow of Sec. III.D).
//
// Inflow: a half-way bounce-back wall at x = -1/2 moving with (u_in, 0).  A
// population f*_i leaving column 0 through it (e_ix = -1: i = 3, 6, 7)
// returns to the same node as opp(i) with the moving-wall correction
// -2 w_i rho_in (e_i . u_wall) / c_s^2 = +6 w_i rho_in u_in (Ladd's rule),
// so in the pull form column 0 takes f_1, f_5, f_8 from its own slots 3, 7,
// 6 plus 6 w rho_in u_in.  Outflow: the populations entering column nx - 1
// from outside (e_ix = -1: 3, 6, 7) follow Zou and He's pressure rule for a
// prescribed density rho_out and zero transverse velocity, computed from the
// six known ones.  In shifted storage the weights cancel in both rules (w_i
// = w_opp(i); w_2 = w_4; the known sum carries exactly 1 of weight).  Phi
// beyond the inflow wall is the wall's rho_in u_in^3; beyond the outlet it
// equals the last column's.  The body force is not part of either rule.

// Redirect the pull sources of column 0 (inflow: own slots) and column
// nx - 1 (outflow: any valid slot, replaced by open_x_fix).
template <class T>
__device__ __forceinline__ void open_x_sources(const T *a[9], const T *r0, int64_t plane, int xc,
                                               int nx) {
    if (xc == 0) {
        a[1] = r0 + 3 * plane + xc;
        a[5] = r0 + 7 * plane + xc;
        a[8] = r0 + 6 * plane + xc;
    }
    if (xc == nx - 1) a[3] = a[6] = a[7] = r0 + xc;
}

// Complete the boundary columns' pre-collision populations (after the pull
// sources of open_x_sources, widened to C).
template <class C, bool SHIFTED>
__device__ __forceinline__ void open_x_fix(C f[9], int xc, int nx, C u_in, C rho_in, C rho_out) {
    if (xc == 0) {
        const C m1 = C(2.0 / 3.0) * (rho_in * u_in);  // 6 w_1 rho_in u_in
        const C m5 = C(1.0 / 6.0) * (rho_in * u_in);  // 6 w_5 rho_in u_in
        f[1] += m1;
        f[5] += m5;
        f[8] += m5;
    }
    if (xc == nx - 1) {
        const C known = (f[0] + f[2] + f[4]) + C(2) * (f[1] + f[5] + f[8]);
        // rho_out u_x = (sum of the known, counted as Zou and He) - rho_out
        const C rux = SHIFTED ? (known + C(1)) - rho_out : known - rho_out;
        const C half24 = C(0.5) * (f[2] - f[4]);
        f[3] = f[1] - C(2.0 / 3.0) * rux;
        f[7] = f[5] + half24 - C(1.0 / 6.0) * rux;
        f[6] = f[8] - half24 - C(1.0 / 6.0) * rux;
    }
}

}  // namespace trt
