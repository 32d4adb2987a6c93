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

// Columns one wavefront produces: lanes 1..62 write, lanes 0 and 63 supply
// the x-neighbours' Phi_x at the strip edges.
constexpr int kStripWidth = 62;

// Everything one instance's sweep needs.  buf[0], buf[1] are the caller's
// two lattices; the step reading buf[s] writes buf[1 - s].
struct InstDesc {
    void *buf[2];
    const uint8_t *mask;  // dense [ny][nx] or null
    int64_t plane;        // elements between population planes
    int32_t nx, ny, pitch;
    int32_t cur;          // lattice holding the state when the descriptor was built
    int32_t strips, rowblocks, rows;
    int32_t pad_;
    double omega1, omega2, phi, gx, gy;
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

// Correctly rounded reciprocal (the hardware approximation's error is
// systematic for rho close to 1 and would bias the velocity).
__device__ __forceinline__ double recip(double r) { return 1.0 / r; }
__device__ __forceinline__ float recip(float r) { return 1.0f / r; }

// Moments of one node (Eqs. 12-13): base = sum_i f_i (shifted: delta rho),
// rho, j = sum_i e_i f_i, and the He-shifted velocity u = j / rho + g / 2
// (F = rho g, so (j + F/2) / rho = j / rho + g / 2).
template <class C, bool SHIFTED> struct Moments {
    C base, rho, jx, jy, ux, uy;
    __device__ __forceinline__ void compute(const C f[9], C gx, C gy) {
        base = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
        rho = SHIFTED ? C(1) + base : base;
        jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
        jy = (f[2] - f[4]) + (f[5] - f[7]) + (f[6] - f[8]);
        const C inv = recip(rho);
        ux = jx * inv + C(0.5) * gx;
        uy = jy * inv + C(0.5) * gy;
    }
};

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

// Third-order Hermite equilibrium (Eq. 5) in coefficient form: the
// equilibrium moments of Eq. 7 are rho u, rho u u and rho u_x^2 u_y,
// rho u_x u_y^2.  base = rho (or rho - 1 for shifted output).
template <class C>
__device__ __forceinline__ void equilibrium(C f[9], C base, C rho, C ux, C uy) {
    const C rux = rho * ux, ruy = rho * uy;
    const C exy = rux * uy;
    reconstruct<C>(f, base, rux, ruy, rux * ux, ruy * uy, exy, exy * ux, exy * uy);
}

// Collision of one node, Eq. 2 (post-collision state overwrites f).
template <class C, bool SHIFTED>
__device__ __forceinline__ void collide(C f[9], const Moments<C, SHIFTED> &m, C dphix, C dphiy,
                                        C w1, C w2, C phi, C gx, C gy) {
    const C third = C(1) / C(3);
    const C Fx = m.rho * gx, Fy = m.rho * gy;
    // raw moments of the (possibly shifted) populations
    const C pxx = (f[1] + f[3]) + (f[5] + f[6]) + (f[7] + f[8]);
    const C pyy = (f[2] + f[4]) + (f[5] + f[6]) + (f[7] + f[8]);
    const C pxy = (f[5] - f[6]) + (f[7] - f[8]);
    const C qxxy = (f[5] + f[6]) - (f[7] + f[8]);
    const C qxyy = (f[5] - f[6]) + (f[8] - f[7]);
    // equilibrium Hermite moments (Eq. 7)
    const C rux = m.rho * m.ux, ruy = m.rho * m.uy;
    const C exx = rux * m.ux, eyy = ruy * m.uy, exy = rux * m.uy;
    const C exxy = exy * m.ux, exyy = exy * m.uy;
    // non-equilibrium Hermite moments (Eq. 6)
    const C axx = pxx - m.base * third - exx;
    const C ayy = pyy - m.base * third - eyy;
    const C axy = pxy - exy;
    const C axxy = qxxy - m.jy * third - exxy;
    const C axyy = qxyy - m.jx * third - exyy;
    // collected Hermite coefficients of f* (relaxation + G_i + F_i)
    const C bx = m.jx + Fx, by = m.jy + Fy;
    const C bxx = exx + w1 * axx + phi * (C(2) * Fx * m.ux - dphix);
    const C byy = eyy + w1 * ayy + phi * (C(2) * Fy * m.uy - dphiy);
    const C bxy = exy + w1 * axy + phi * (Fx * m.uy + m.ux * Fy);
    const C bxxy = exxy + w2 * axxy;
    const C bxyy = exyy + w2 * axyy;
    reconstruct<C>(f, m.base, bx, by, bxx, byy, bxy, bxxy, bxyy);
}

// Pull-gather of the pre-collision populations f_i(x, t) of node (xc, y)
// from the previous step's post-collision lattice: f_i(x, t) =
// f*_i(x - e_i, t - 1), or, when x - e_i is solid, the half-way bounce-back
// value f*_opp(i)(x, t - 1) stored at the node itself (Sec. II.D).
// xm, xp are the wrapped neighbour columns.  Returns whether the node is solid.
template <class T, class C, bool MASK>
__device__ __forceinline__ bool gather(const T *__restrict__ src, int64_t plane, int pitch,
                                       const uint8_t *__restrict__ mask, int nx, int ny, int y,
                                       int xm, int xc, int xp, C f[9]) {
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
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = to_c(a[i][0]);
    return solid;
}

}  // namespace trt
