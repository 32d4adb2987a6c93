// A Taylor-Green vortex through the C ABI alone: device buffers from
// hipMalloc, one simulation, the FP64 diagnostics, no Python and no PyTorch.
//
//   taylor_green [n] [f64|f32|f16] [steps]
//
// The vortex u = u0 (-cos kx sin ky, sin kx cos ky), k = 2 pi / n, is an
// exact eigenmode of the incompressible Navier-Stokes equations whose
// amplitude decays as exp(-2 nu k^2 t) (Sec. III.B); the program compares
// the ratio of max |u| after `steps` steps with that decay, checks mass
// conservation, and exits with 0 when both hold (relative difference below
// 5e-3; mass drift below 1e-12 for FP64 storage, 1e-8 for FP32 and 1e-5 for
// FP16, whose rounding of each stored population does not conserve mass
// exactly), 2 when they do not, 1 on an error.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "../../include/trtlbm.h"

#define HIP_OK(x)                                                                   \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess) {                                                     \
            fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                  \
            return 1;                                                               \
        }                                                                           \
    } while (0)
#define TRT_OK_(x)                                                                  \
    do {                                                                            \
        if ((x) != TRT_OK) {                                                        \
            fprintf(stderr, "%s: %s\n", #x, trt_last_error());                      \
            return 1;                                                               \
        }                                                                           \
    } while (0)

int main(int argc, char **argv) {
    const int n = argc > 1 ? atoi(argv[1]) : 64;
    const char *st = argc > 2 ? argv[2] : "f64";
    const long steps = argc > 3 ? atol(argv[3]) : 1000;
    const int storage = !strcmp(st, "f16") ? TRT_F16_SHIFTED
                      : !strcmp(st, "f32") ? TRT_F32_SHIFTED : TRT_F64;
    const double tau = 0.6, lambda = 0.25, u0 = 0.01;
    const double tau2 = 0.5 + lambda / (tau - 0.5);  // magic parameter Lambda_s = 1/4
    const double nu = (tau - 0.5) / 3.0, k = 2.0 * M_PI / n;

    trt_problem p;
    memset(&p, 0, sizeof p);
    p.nx = p.ny = n;
    p.tau_s = tau;
    p.tau_s2 = tau2;
    p.storage = storage;
    const size_t bytes = trt_lattice_bytes(&p);
    if (bytes == 0) {
        fprintf(stderr, "invalid problem: %s\n", trt_last_error());
        return 1;
    }

    // initial fields on the host: rho from the pressure of the vortex
    // (c_s^2 = 1/3), u and v from the eigenmode
    const size_t nn = (size_t)n * n;
    std::vector<double> rho(nn), ux(nn), uy(nn);
    for (int y = 0; y < n; ++y)
        for (int x = 0; x < n; ++x) {
            const size_t i = (size_t)y * n + x;
            ux[i] = -u0 * cos(k * x) * sin(k * y);
            uy[i] = u0 * sin(k * x) * cos(k * y);
            rho[i] = 1.0 - 0.75 * u0 * u0 * (cos(2 * k * x) + cos(2 * k * y));
        }

    void *fa = nullptr, *fb = nullptr;
    double *d_rho = nullptr, *d_ux = nullptr, *d_uy = nullptr, *d_diag = nullptr;
    HIP_OK(hipMalloc(&fa, bytes));
    HIP_OK(hipMalloc(&fb, bytes));
    HIP_OK(hipMalloc(&d_rho, nn * sizeof(double)));
    HIP_OK(hipMalloc(&d_ux, nn * sizeof(double)));
    HIP_OK(hipMalloc(&d_uy, nn * sizeof(double)));
    HIP_OK(hipMalloc(&d_diag, TRT_NDIAG * sizeof(double)));
    HIP_OK(hipMemcpy(d_rho, rho.data(), nn * sizeof(double), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(d_ux, ux.data(), nn * sizeof(double), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(d_uy, uy.data(), nn * sizeof(double), hipMemcpyHostToDevice));

    trt_sim *sim = nullptr;
    TRT_OK_(trt_create(&p, fa, fb, nullptr, &sim));  // the null stream
    TRT_OK_(trt_init_equilibrium(sim, d_rho, d_ux, d_uy));
    double d0[TRT_NDIAG], d1[TRT_NDIAG];
    TRT_OK_(trt_diagnostics(sim, d_diag));
    HIP_OK(hipMemcpy(d0, d_diag, sizeof d0, hipMemcpyDeviceToHost));
    TRT_OK_(trt_step(sim, steps));
    TRT_OK_(trt_diagnostics(sim, d_diag));
    HIP_OK(hipMemcpy(d1, d_diag, sizeof d1, hipMemcpyDeviceToHost));
    trt_destroy(sim);
    HIP_OK(hipFree(fa));
    HIP_OK(hipFree(fb));
    HIP_OK(hipFree(d_rho));
    HIP_OK(hipFree(d_ux));
    HIP_OK(hipFree(d_uy));
    HIP_OK(hipFree(d_diag));

    const double ratio = d1[3] / d0[3];
    const double analytic = exp(-2.0 * nu * k * k * (double)steps);
    const double rel = fabs(ratio / analytic - 1.0);
    const double drift = fabs(d1[0] - d0[0]) / d0[0];
    const double drift_bound = storage == TRT_F64 ? 1e-12 : storage == TRT_F32_SHIFTED ? 1e-8 : 1e-5;
    const bool ok = rel < 5e-3 && drift < drift_bound && d1[4] == 0.0;
    printf("taylor_green n=%d %s (%s): %ld steps, max|u| ratio %.6f, analytic %.6f, "
           "relative difference %.2e, mass drift %.1e, divergent nodes %.0f: %s\n",
           n, st, trt_version(), steps, ratio, analytic, rel, drift, d1[4],
           ok ? "within bounds" : "OUT OF BOUNDS");
    return ok ? 0 : 2;
}
