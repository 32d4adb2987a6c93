/*
 * trt_oracle.c -- plain FP64 CPU oracle for one time step of the D2Q9
 * two-relaxation-time regularized lattice Boltzmann (TRT-RLB) model of
 * Yu, Qin, Chen, Shu and Yuan, "Two-relaxation-time regularized lattice
 * Boltzmann model for Navier-Stokes equations" (arXiv:2312.10318).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product:
 * only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no code, header, table or helper with the GPU
 * library, and it never calls into it.
 *
 * Style: every quantity is computed the slow, literal way the paper writes
 * it.  The Hermite tensors are rebuilt from their definitions, and every
 * contraction over Cartesian indices (alpha, beta, gamma in {x, y}) is an
 * explicit loop, so the code can be read against the paper term by term.
 * Arithmetic is IEEE FP64, round to nearest; build with -ffp-contract=off so
 * that no multiply-add is fused.
 *
 * Units: lattice units, dx = dt = c = 1, so c_s^2 = 1/3 (Sec. II.B).  This
 * matters: the compensation term G_i (Eq. 8) divides by 6 c_s^6, which equals
 * the 2 c_s^4 its moment identity (Sec. II.C, Eq. 17) needs only at
 * c_s^2 = 1/3.
 *
 * State layout: populations f[i][y][x] (i = 0..8), dense, x fastest, holding
 * the PRE-collision distribution f(x, t).  Solid nodes (mask != 0) hold 0.
 *
 * Readings taken where the paper is silent (numbered as in the design
 * notes of the repository):
 *   R1  The gradient in G_i is a second-order central difference of the
 *       fields rho*u_x^3, rho*u_y^3 taken at the same time level t, with
 *       periodic wrap; at a solid neighbour the field is taken as 0.
 *   R2  The body force is F = rho * g with g an acceleration (Sec. II.D,
 *       the Poiseuille set-up), and dt = 1.
 *   R12 Solid nodes are never collided; their outputs are 0.
 *   R13 A link whose target is a solid node is bounced back half-way, link by
 *       link (Sec. II.D, half-way bounce-back rule), also for diagonal links.
 * Open boundaries in x (the creeping flow of Sec. III.D; orc_step_open):
 *   R17 The inlet is a half-way bounce-back wall at x = -1/2 moving with the
 *       inflow velocity (u_in, 0): a population f*_i leaving column 0
 *       through it returns to the same node as direction opp(i) with the
 *       moving-wall momentum correction -2 w_i rho_w (e_i . u_wall) / c_s^2
 *       (Ladd's moving-wall rule; the paper names the scheme, not the
 *       formula), rho_w the prescribed wall density.
 *   R18 The outlet column nx - 1 has a prescribed density rho_out and zero
 *       transverse velocity: after streaming, its three populations with
 *       e_x = -1 come from Zou and He's pressure rule applied to the six
 *       known ones.  Populations streaming out through x = nx are lost.
 *   R19 Phi beyond the inlet is the wall's, rho_w u_in^3 (x) and 0 (y);
 *       beyond the outlet it equals the last column's (zero gradient).
 *   R20 Moving walls and the outlet rule ignore the body force (the open
 *       case of the paper is unforced).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 9
#define DIM 2

/* D2Q9 velocity set and weights, Sec. II.B (c = 1). */
static const int E[Q][DIM] = {
    {0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1}, {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
static const double WGT[Q] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
/* c_s = c / sqrt(3), Sec. II.B. */
static const double CS2 = 1.0 / 3.0;

static double kron(int a, int b) { return a == b ? 1.0 : 0.0; }

/* Hermite tensors, Sec. II.B, Eq. (3a)-(3d), evaluated from their
 * definitions once, when the library is loaded. */
static double defn_herm2(int i, int a, int b) {
    return (double)E[i][a] * (double)E[i][b] - CS2 * kron(a, b);
}
static double defn_herm3(int i, int a, int b, int c) {
    return (double)E[i][a] * (double)E[i][b] * (double)E[i][c] -
           CS2 * ((double)E[i][a] * kron(b, c) + (double)E[i][b] * kron(c, a) +
                  (double)E[i][c] * kron(a, b));
}
static double H1[Q][DIM], H2[Q][DIM][DIM], H3[Q][DIM][DIM][DIM];
__attribute__((constructor)) static void build_hermite_tables(void) {
    for (int i = 0; i < Q; ++i)
        for (int a = 0; a < DIM; ++a) {
            H1[i][a] = (double)E[i][a];
            for (int b = 0; b < DIM; ++b) {
                H2[i][a][b] = defn_herm2(i, a, b);
                for (int c = 0; c < DIM; ++c) H3[i][a][b][c] = defn_herm3(i, a, b, c);
            }
        }
}
#define herm1(i, a) H1[i][a]
#define herm2(i, a, b) H2[i][a][b]
#define herm3(i, a, b, c) H3[i][a][b][c]

/* Direction opposite to i (e_opp = -e_i). */
static int opposite(int i) {
    for (int j = 0; j < Q; ++j)
        if (E[j][0] == -E[i][0] && E[j][1] == -E[i][1]) return j;
    return -1;
}

/* Third-order Hermite equilibrium, Sec. II.B, Eq. (5):
 *   f_i^eq = w_i rho { 1 + H_a u_a / c_s^2 + H_ab u_a u_b / (2 c_s^4)
 *                        + H_abc u_a u_b u_c / (6 c_s^6) }            */
void orc_feq(double rho, double ux, double uy, double *feq) {
    const double u[DIM] = {ux, uy};
    for (int i = 0; i < Q; ++i) {
        double s1 = 0.0, s2 = 0.0, s3 = 0.0;
        for (int a = 0; a < DIM; ++a) s1 += herm1(i, a) * u[a];
        for (int a = 0; a < DIM; ++a)
            for (int b = 0; b < DIM; ++b) s2 += herm2(i, a, b) * u[a] * u[b];
        for (int a = 0; a < DIM; ++a)
            for (int b = 0; b < DIM; ++b)
                for (int c = 0; c < DIM; ++c) s3 += herm3(i, a, b, c) * u[a] * u[b] * u[c];
        feq[i] = WGT[i] * rho *
                 (1.0 + s1 / CS2 + s2 / (2.0 * CS2 * CS2) + s3 / (6.0 * CS2 * CS2 * CS2));
    }
}

/* Density and velocity with He's change of variables, Sec. II.B, Eqs. (12)-(13):
 *   rho = sum_i f_i,   sum_i e_ia f_i = rho u_a - F_a / 2,   F = rho g.
 * Hence u_a = (sum_i e_ia f_i + F_a / 2) / rho.                      */
void orc_moments(const double *f, double gx, double gy, double *rho_out, double *ux_out,
                 double *uy_out) {
    double rho = 0.0, j[DIM] = {0.0, 0.0};
    for (int i = 0; i < Q; ++i) rho += f[i];
    for (int a = 0; a < DIM; ++a)
        for (int i = 0; i < Q; ++i) j[a] += (double)E[i][a] * f[i];
    const double F[DIM] = {rho * gx, rho * gy};
    *rho_out = rho;
    *ux_out = (j[0] + 0.5 * F[0]) / rho;
    *uy_out = (j[1] + 0.5 * F[1]) / rho;
}

/* Cubic-error compensation source, Sec. II.B, Eqs. (8)-(10):
 *   G_i = -w_i H_ab / (6 c_s^6) (1 - 1/(2 tau1)) d_c Phi_abc,
 *   d_c Phi_abc = d_x(rho u_x^3) delta_ax delta_bx + d_y(rho u_y^3) delta_ay delta_by.
 * dphi[0], dphi[1] are the two gradients d_x(rho u_x^3), d_y(rho u_y^3). */
void orc_source_G(double tau1, double dphix, double dphiy, double *G) {
    double dPhi[DIM][DIM];
    for (int a = 0; a < DIM; ++a)
        for (int b = 0; b < DIM; ++b)
            dPhi[a][b] = dphix * kron(a, 0) * kron(b, 0) + dphiy * kron(a, 1) * kron(b, 1);
    for (int i = 0; i < Q; ++i) {
        double s = 0.0;
        for (int a = 0; a < DIM; ++a)
            for (int b = 0; b < DIM; ++b) s += herm2(i, a, b) * dPhi[a][b];
        G[i] = -WGT[i] * s / (6.0 * CS2 * CS2 * CS2) * (1.0 - 1.0 / (2.0 * tau1));
    }
}

/* Forcing term, Sec. II.B, Eq. (11):
 *   F_i = w_i { H_a F_a / c_s^2 + H_ab (F_a u_b + u_a F_b) / (2 c_s^4) }. */
void orc_source_F(double Fx, double Fy, double ux, double uy, double *Fi) {
    const double F[DIM] = {Fx, Fy};
    const double u[DIM] = {ux, uy};
    for (int i = 0; i < Q; ++i) {
        double s1 = 0.0, s2 = 0.0;
        for (int a = 0; a < DIM; ++a) s1 += herm1(i, a) * F[a];
        for (int a = 0; a < DIM; ++a)
            for (int b = 0; b < DIM; ++b) s2 += herm2(i, a, b) * (F[a] * u[b] + u[a] * F[b]);
        Fi[i] = WGT[i] * (s1 / CS2 + s2 / (2.0 * CS2 * CS2));
    }
}

/* Collision of one node: the right-hand side of the evolution equation,
 * Sec. II.B, Eq. (2), with the off-equilibrium projections of Eq. (6):
 *   A_a   = sum_i H_a   (f_i - f_i^eq)
 *   A_ab  = sum_i H_ab  (f_i - f_i^eq)
 *   A_abc = sum_i H_abc (f_i - f_i^eq)
 *   f*_i = f_i^eq + (1 - 1/tau1) w_i H_a A_a / c_s^2
 *                 + (1 - 1/tau1) w_i H_ab A_ab / (2 c_s^4)
 *                 + (1 - 1/tau2) w_i H_abc A_abc / (6 c_s^6)
 *                 + G_i dt + (1 - 1/(2 tau1)) F_i dt.
 * The moments rho, u are taken from f itself (Eqs. 12-13); dphix, dphiy are
 * the gradients entering G_i; g is the body acceleration (F = rho g).     */
void orc_collide_node(const double *f, double gx, double gy, double dphix, double dphiy,
                      double tau1, double tau2, double *fstar) {
    double rho, ux, uy;
    orc_moments(f, gx, gy, &rho, &ux, &uy);
    double feq[Q], fneq[Q], G[Q], Fi[Q];
    orc_feq(rho, ux, uy, feq);
    for (int i = 0; i < Q; ++i) fneq[i] = f[i] - feq[i];

    double A1[DIM] = {0.0, 0.0}, A2[DIM][DIM], A3[DIM][DIM][DIM];
    for (int a = 0; a < DIM; ++a)
        for (int i = 0; i < Q; ++i) A1[a] += herm1(i, a) * fneq[i];
    for (int a = 0; a < DIM; ++a)
        for (int b = 0; b < DIM; ++b) {
            A2[a][b] = 0.0;
            for (int i = 0; i < Q; ++i) A2[a][b] += herm2(i, a, b) * fneq[i];
        }
    for (int a = 0; a < DIM; ++a)
        for (int b = 0; b < DIM; ++b)
            for (int c = 0; c < DIM; ++c) {
                A3[a][b][c] = 0.0;
                for (int i = 0; i < Q; ++i) A3[a][b][c] += herm3(i, a, b, c) * fneq[i];
            }

    orc_source_G(tau1, dphix, dphiy, G);
    orc_source_F(rho * gx, rho * gy, ux, uy, Fi);

    for (int i = 0; i < Q; ++i) {
        double r1 = 0.0, r2 = 0.0, r3 = 0.0;
        for (int a = 0; a < DIM; ++a) r1 += herm1(i, a) * A1[a];
        for (int a = 0; a < DIM; ++a)
            for (int b = 0; b < DIM; ++b) r2 += herm2(i, a, b) * A2[a][b];
        for (int a = 0; a < DIM; ++a)
            for (int b = 0; b < DIM; ++b)
                for (int c = 0; c < DIM; ++c) r3 += herm3(i, a, b, c) * A3[a][b][c];
        fstar[i] = feq[i] + (1.0 - 1.0 / tau1) * WGT[i] * r1 / CS2 +
                   (1.0 - 1.0 / tau1) * WGT[i] * r2 / (2.0 * CS2 * CS2) +
                   (1.0 - 1.0 / tau2) * WGT[i] * r3 / (6.0 * CS2 * CS2 * CS2) + G[i] +
                   (1.0 - 1.0 / (2.0 * tau1)) * Fi[i];
    }
}

static int wrap(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

/* Density and He-shifted velocity of every node, dense [ny][nx]; solid -> 0. */
void orc_macros(int nx, int ny, const uint8_t *solid, const double *f, double gx, double gy,
                double *rho, double *ux, double *uy) {
    const long n = (long)nx * ny;
#pragma omp parallel for schedule(static) if (n >= 16384)
    for (long k = 0; k < n; ++k) {
        if (solid && solid[k]) {
            rho[k] = ux[k] = uy[k] = 0.0;
            continue;
        }
        double fl[Q];
        for (int i = 0; i < Q; ++i) fl[i] = f[(long)i * n + k];
        orc_moments(fl, gx, gy, &rho[k], &ux[k], &uy[k]);
    }
}

/* Initial state f(x, 0) = f^eq(rho, u) at fluid nodes, 0 at solid nodes. */
void orc_init_equilibrium(int nx, int ny, const uint8_t *solid, const double *rho,
                          const double *ux, const double *uy, double *f) {
    const long n = (long)nx * ny;
#pragma omp parallel for schedule(static) if (n >= 16384)
    for (long k = 0; k < n; ++k) {
        double feq[Q];
        if (solid && solid[k]) {
            for (int i = 0; i < Q; ++i) f[(long)i * n + k] = 0.0;
            continue;
        }
        orc_feq(rho[k], ux[k], uy[k], feq);
        for (int i = 0; i < Q; ++i) f[(long)i * n + k] = feq[i];
    }
}

/* One full time step f(., t) -> f(., t + dt):
 *   1. rho, u at every fluid node (Eqs. 12-13);
 *   2. Phi_x = rho u_x^3, Phi_y = rho u_y^3 (Eq. 9), 0 at solid nodes (R1);
 *   3. d_x Phi_x, d_y Phi_y by central differences at time t (R1);
 *   4. collision at every fluid node (Eq. 2);
 *   5. streaming f_i(x + e_i, t + dt) = f*_i(x, t) with periodic wrap, and
 *      half-way bounce-back f_opp(i)(x, t + dt) = f*_i(x, t) when x + e_i is
 *      solid (Sec. II.D, streaming step and bounce-back rule).
 * fin and fout are [9][ny][nx] and must not overlap.  Returns 0, or -1 when
 * scratch memory cannot be allocated.                                    */
int orc_step(int nx, int ny, const uint8_t *solid, const double *fin, double *fout,
             double tau1, double tau2, double gx, double gy) {
    const long n = (long)nx * ny;
    double *phix = (double *)malloc(sizeof(double) * n);
    double *phiy = (double *)malloc(sizeof(double) * n);
    if (!phix || !phiy) {
        free(phix);
        free(phiy);
        return -1;
    }
    int opp[Q];
    for (int i = 0; i < Q; ++i) opp[i] = opposite(i);

#pragma omp parallel for schedule(static) if (n >= 16384)
    for (long k = 0; k < n; ++k) {
        if (solid && solid[k]) {
            phix[k] = phiy[k] = 0.0;
            continue;
        }
        double fl[Q], rho, ux, uy;
        for (int i = 0; i < Q; ++i) fl[i] = fin[(long)i * n + k];
        orc_moments(fl, gx, gy, &rho, &ux, &uy);
        phix[k] = rho * ux * ux * ux;
        phiy[k] = rho * uy * uy * uy;
    }

#pragma omp parallel for schedule(static) if (n >= 16384)
    for (long k = 0; k < (long)Q * n; ++k) fout[k] = 0.0;

#pragma omp parallel for schedule(static) if (n >= 16384)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            const long k = (long)y * nx + x;
            if (solid && solid[k]) continue;
            double fl[Q], fs[Q];
            for (int i = 0; i < Q; ++i) fl[i] = fin[(long)i * n + k];
            const double dphix =
                0.5 * (phix[(long)y * nx + wrap(x + 1, nx)] - phix[(long)y * nx + wrap(x - 1, nx)]);
            const double dphiy =
                0.5 * (phiy[(long)wrap(y + 1, ny) * nx + x] - phiy[(long)wrap(y - 1, ny) * nx + x]);
            orc_collide_node(fl, gx, gy, dphix, dphiy, tau1, tau2, fs);
            for (int i = 0; i < Q; ++i) {
                const int xd = wrap(x + E[i][0], nx), yd = wrap(y + E[i][1], ny);
                const long kd = (long)yd * nx + xd;
                if (solid && solid[kd])
                    fout[(long)opp[i] * n + k] = fs[i];
                else
                    fout[(long)i * n + kd] = fs[i];
            }
        }
    }
    free(phix);
    free(phiy);
    return 0;
}

/* Post-collision populations fstar[9][ny][nx] of every fluid node (0 at
 * solid nodes) for the state fin, with the Phi gradient of R1 and, when
 * open_x is set, the boundary values of R19 at columns 0 and nx - 1.      */
static int collide_field(int nx, int ny, const uint8_t *solid, const double *fin, double *fstar,
                         double tau1, double tau2, double gx, double gy, int open_x,
                         double u_in, double rho_w) {
    const long n = (long)nx * ny;
    double *px = (double *)malloc(sizeof(double) * n);
    double *py = (double *)malloc(sizeof(double) * n);
    if (!px || !py) {
        free(px);
        free(py);
        return -1;
    }
#pragma omp parallel for schedule(static) if (n >= 16384)
    for (long k = 0; k < n; ++k) {
        double fl[Q], rho, ux, uy;
        px[k] = py[k] = 0.0;
        if (solid && solid[k]) continue;
        for (int i = 0; i < Q; ++i) fl[i] = fin[(long)i * n + k];
        orc_moments(fl, gx, gy, &rho, &ux, &uy);
        px[k] = rho * ux * ux * ux;
        py[k] = rho * uy * uy * uy;
    }
#pragma omp parallel for schedule(static) if (n >= 16384)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            const long k = (long)y * nx + x;
            double fl[Q], fs[Q];
            if (solid && solid[k]) {
                for (int i = 0; i < Q; ++i) fstar[(long)i * n + k] = 0.0;
                continue;
            }
            for (int i = 0; i < Q; ++i) fl[i] = fin[(long)i * n + k];
            /* Phi_x at the two x-neighbours (R1, with R19 at open ends) */
            double left = px[(long)y * nx + wrap(x - 1, nx)];
            double right = px[(long)y * nx + wrap(x + 1, nx)];
            if (open_x && x == 0) left = rho_w * u_in * u_in * u_in;
            if (open_x && x == nx - 1) right = px[k];
            const double below = py[(long)wrap(y - 1, ny) * nx + x];
            const double above = py[(long)wrap(y + 1, ny) * nx + x];
            orc_collide_node(fl, gx, gy, 0.5 * (right - left), 0.5 * (above - below), tau1, tau2,
                             fs);
            for (int i = 0; i < Q; ++i) fstar[(long)i * n + k] = fs[i];
        }
    }
    free(px);
    free(py);
    return 0;
}

/* Post-collision populations fstar[9][ny][nx] of the state fin: the
 * collision of every fluid node as in orc_step (0 at solid nodes), with the
 * open-end values of Phi (R19) when open_x is set.  Returns 0 or -1.     */
int orc_collide(int nx, int ny, const uint8_t *solid, const double *fin, double *fstar,
                double tau1, double tau2, double gx, double gy, int open_x, double u_in,
                double rho_w) {
    return collide_field(nx, ny, solid, fin, fstar, tau1, tau2, gx, gy, open_x, u_in, rho_w);
}

/* Streaming of post-collision populations fstar into the pre-collision
 * state fout with an inflow wall at x = -1/2 and a pressure outlet at
 * x = nx - 1 (R17-R20), periodic in y, half-way bounce-back at solid nodes:
 * f_i(x + e_i) = f*_i(x) inside the lattice, the moving-wall return at the
 * inlet, loss through the outlet, and Zou and He's rule for the outlet's
 * incoming populations.                                                  */
void orc_stream_open(int nx, int ny, const uint8_t *solid, const double *fstar, double *fout,
                     double u_in, double rho_w, double rho_out) {
    const long n = (long)nx * ny;
    for (long k = 0; k < (long)Q * n; ++k) fout[k] = 0.0;
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            const long k = (long)y * nx + x;
            if (solid && solid[k]) continue;
            for (int i = 0; i < Q; ++i) {
                const double v = fstar[(long)i * n + k];
                const int tx = x + E[i][0];
                const int ty = wrap(y + E[i][1], ny);
                const int back = opposite(i);
                if (tx < 0) {
                    /* R17: e_i . u_wall = e_ix u_in */
                    fout[(long)back * n + k] = v - 2.0 * WGT[i] * rho_w * (E[i][0] * u_in) / CS2;
                } else if (tx >= nx) {
                    /* R18: leaves the lattice */
                } else if (solid && solid[(long)ty * nx + tx]) {
                    fout[(long)back * n + k] = v;
                } else {
                    fout[(long)i * n + (long)ty * nx + tx] = v;
                }
            }
        }
    }
    /* R18: Zou and He's pressure rule, e = (1,0):1 (0,1):2 (-1,0):3 (0,-1):4
     * (1,1):5 (-1,1):6 (-1,-1):7 (1,-1):8, with u_y = 0 at the outlet */
    for (int y = 0; y < ny; ++y) {
        const long k = (long)y * nx + (nx - 1);
        if (solid && solid[k]) continue;
        double f[Q];
        for (int i = 0; i < Q; ++i) f[i] = fout[(long)i * n + k];
        const double ux = -1.0 + (f[0] + f[2] + f[4] + 2.0 * (f[1] + f[5] + f[8])) / rho_out;
        fout[3 * n + k] = f[1] - 2.0 / 3.0 * rho_out * ux;
        fout[7 * n + k] = f[5] + 0.5 * (f[2] - f[4]) - 1.0 / 6.0 * rho_out * ux;
        fout[6 * n + k] = f[8] - 0.5 * (f[2] - f[4]) - 1.0 / 6.0 * rho_out * ux;
    }
}

/* One time step with the open x boundaries: orc_collide with the open-end
 * Phi, then orc_stream_open.                                             */
int orc_step_open(int nx, int ny, const uint8_t *solid, const double *fin, double *fout,
                  double tau1, double tau2, double gx, double gy, double u_in, double rho_w,
                  double rho_out) {
    const long n = (long)nx * ny;
    double *fstar = (double *)malloc(sizeof(double) * Q * n);
    if (!fstar) return -1;
    if (collide_field(nx, ny, solid, fin, fstar, tau1, tau2, gx, gy, 1, u_in, rho_w) != 0) {
        free(fstar);
        return -1;
    }
    orc_stream_open(nx, ny, solid, fstar, fout, u_in, rho_w, rho_out);
    free(fstar);
    return 0;
}

/* Momentum handed to the solid nodes during the collision of state f(x, t)
 * (Sec. III.D, momentum exchange): every link from a fluid node x_f to a
 * solid node x_s = x_f + e_i carries e_i [f*_i(x_f, t) + f*_opp(i)(x_s, t)],
 * where under half-way bounce-back the population returned from the wall is
 * f*_i(x_f, t) itself, so the link gives 2 e_i f*_i(x_f, t).  Links leaving
 * through open x ends (open_x) are not wall links.  out[0..1] = (F_x, F_y).
 * Returns 0, or -1 when memory cannot be allocated.                      */
int orc_wall_force(int nx, int ny, const uint8_t *solid, const double *f, double tau1,
                   double tau2, double gx, double gy, int open_x, double u_in, double rho_w,
                   double *out) {
    const long n = (long)nx * ny;
    double *fstar = (double *)malloc(sizeof(double) * Q * n);
    if (!fstar) return -1;
    if (collide_field(nx, ny, solid, f, fstar, tau1, tau2, gx, gy, open_x, u_in, rho_w) != 0) {
        free(fstar);
        return -1;
    }
    double fx = 0.0, fy = 0.0;
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            const long k = (long)y * nx + x;
            if (!solid || solid[k]) continue;
            for (int i = 1; i < Q; ++i) {
                int tx = x + E[i][0];
                if (open_x && (tx < 0 || tx >= nx)) continue;
                tx = wrap(tx, nx);
                const int ty = wrap(y + E[i][1], ny);
                if (!solid[(long)ty * nx + tx]) continue;
                const double returned = fstar[(long)i * n + k];
                fx += E[i][0] * (fstar[(long)i * n + k] + returned);
                fy += E[i][1] * (fstar[(long)i * n + k] + returned);
            }
        }
    }
    out[0] = fx;
    out[1] = fy;
    free(fstar);
    return 0;
}

/* nsteps steps of orc_step_open (in place).  Returns 0 or -1.            */
int orc_run_open(int nx, int ny, const uint8_t *solid, double *f, long nsteps, double tau1,
                 double tau2, double gx, double gy, double u_in, double rho_w, double rho_out) {
    const long len = (long)Q * nx * ny;
    double *tmp = (double *)malloc(sizeof(double) * len);
    if (!tmp) return -1;
    double *a = f, *b = tmp;
    for (long s = 0; s < nsteps; ++s) {
        if (orc_step_open(nx, ny, solid, a, b, tau1, tau2, gx, gy, u_in, rho_w, rho_out) != 0) {
            free(tmp);
            return -1;
        }
        double *t = a;
        a = b;
        b = t;
    }
    if (a != f) memcpy(f, a, sizeof(double) * len);
    free(tmp);
    return 0;
}

/* nsteps steps starting from f (in place, through an internal second
 * lattice).  Returns 0, or -1 when memory cannot be allocated.          */
int orc_run(int nx, int ny, const uint8_t *solid, double *f, long nsteps, double tau1,
            double tau2, double gx, double gy) {
    const long len = (long)Q * nx * ny;
    double *tmp = (double *)malloc(sizeof(double) * len);
    if (!tmp) return -1;
    double *a = f, *b = tmp;
    for (long s = 0; s < nsteps; ++s) {
        if (orc_step(nx, ny, solid, a, b, tau1, tau2, gx, gy) != 0) {
            free(tmp);
            return -1;
        }
        double *t = a;
        a = b;
        b = t;
    }
    if (a != f) memcpy(f, a, sizeof(double) * len);
    free(tmp);
    return 0;
}

/* Threads the OpenMP loops above use (1 without OpenMP). */
int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the number of threads of the OpenMP loops (timing only: the
 * arithmetic of a step does not depend on it). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
