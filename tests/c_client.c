/* A plain C99 client of the solver's C ABI (test infrastructure).
 *
 * It uses nothing but include/lbm.h and the HIP runtime's C API for device
 * memory: creates a D2Q9 solver on a periodic 96 x 64 grid, initialises it
 * from theta0 = 2 + cos(2 pi x) cos(2 pi y) with the library's fourth-order
 * difference gradient, takes 100 steps (8-step passes), reads theta, u and
 * grad theta, and checks on the host that the total of theta is conserved
 * and that u = -2 nu grad(theta) / theta holds at every node (the Cole-Hopf
 * relation between the two outputs).  With --no-gpu it only exercises the
 * calls that need no device (parameters, sizes, validation).  Prints "ok". */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "lbm.h"

#define CHECK(cond, ...)                          \
    do {                                          \
        if (!(cond)) {                            \
            fprintf(stderr, __VA_ARGS__);         \
            fprintf(stderr, "\n");                \
            return 1;                             \
        }                                         \
    } while (0)

static lb_config make_cfg(int64_t nx, int64_t ny, double eps) {
    lb_config c;
    memset(&c, 0, sizeof c);
    c.dim = 2;
    c.flags = 0;
    c.n[0] = nx;
    c.n[1] = ny;
    c.n[2] = 1;
    c.n[3] = 1;
    c.dx = 1.0 / (double)nx;
    c.nu = 0.01;
    c.dt = eps * c.dx * c.dx / c.nu;
    return c;
}

static int host_checks(void) {
    lb_config c = make_cfg(96, 64, 0.2);
    double p[7];
    CHECK(lb_parameters(&c, p) == LB_OK, "lb_parameters: %s", lb_last_error());
    CHECK(fabs(p[0] - 0.2) < 1e-15, "eps %.17g", p[0]);
    CHECK(fabs(p[1] - 2.0 / 2.2) < 1e-15, "s1 %.17g", p[1]);
    CHECK(lb_num_populations(2) == 9 && lb_num_populations(3) == 19, "q");
    CHECK(lb_state_elements(&c) == 9 * 2 * 4096, "elements %lld",
          (long long)lb_state_elements(&c));
    CHECK(lb_state_bytes(&c) == (size_t)lb_state_elements(&c) * sizeof(double), "bytes");
    lb_config bad = make_cfg(96, 64, 0.6);
    lb_solver* s = NULL;
    double dummy;
    CHECK(lb_create(&bad, NULL, &dummy, &dummy + 1, &s) == LB_ERR_UNSTABLE && s == NULL,
          "unstable eps accepted");
    bad = make_cfg(96, 64, 0.2);
    bad.dim = 5;
    CHECK(lb_create(&bad, NULL, &dummy, &dummy + 1, &s) == LB_ERR_INVALID_ARG, "dim 5 accepted");
    CHECK(strlen(lb_last_error()) > 0, "no error message");
    return 0;
}

static int gpu_run(void) {
    const int64_t nx = 96, ny = 64, V = nx * ny;
    lb_config c = make_cfg(nx, ny, 0.2);
    const size_t sb = lb_state_bytes(&c);
    double *fa = NULL, *fb = NULL, *th0 = NULL, *th = NULL, *u = NULL, *g = NULL;
    CHECK(hipMalloc((void**)&fa, sb) == hipSuccess && hipMalloc((void**)&fb, sb) == hipSuccess,
          "hipMalloc states");
    CHECK(hipMalloc((void**)&th0, V * sizeof(double)) == hipSuccess &&
              hipMalloc((void**)&th, V * sizeof(double)) == hipSuccess &&
              hipMalloc((void**)&u, 2 * V * sizeof(double)) == hipSuccess &&
              hipMalloc((void**)&g, 2 * V * sizeof(double)) == hipSuccess,
          "hipMalloc fields");
    double* h0 = (double*)malloc(V * sizeof(double));
    double* ht = (double*)malloc(V * sizeof(double));
    double* hu = (double*)malloc(2 * V * sizeof(double));
    double* hg = (double*)malloc(2 * V * sizeof(double));
    CHECK(h0 && ht && hu && hg, "malloc");
    const double pi = 3.14159265358979323846;
    double sum0 = 0.0;
    for (int64_t y = 0; y < ny; ++y)
        for (int64_t x = 0; x < nx; ++x) {
            const double v = 2.0 + cos(2.0 * pi * (double)x / (double)nx) *
                                       cos(2.0 * pi * (double)y / (double)ny);
            h0[y * nx + x] = v;
            sum0 += v;
        }
    CHECK(hipMemcpy(th0, h0, V * sizeof(double), hipMemcpyHostToDevice) == hipSuccess, "copy");
    lb_solver* s = NULL;
    CHECK(lb_create(&c, NULL, fa, fb, &s) == LB_OK, "lb_create: %s", lb_last_error());
    CHECK(lb_init(s, th0, NULL, 1) == LB_OK, "lb_init: %s", lb_last_error());
    CHECK(lb_step(s, 100) == LB_OK, "lb_step: %s", lb_last_error());
    CHECK(lb_steps_taken(s) == 100, "steps %lld", (long long)lb_steps_taken(s));
    CHECK(lb_macro(s, th, u, g) == LB_OK, "lb_macro: %s", lb_last_error());
    CHECK(hipDeviceSynchronize() == hipSuccess, "sync");
    CHECK(hipMemcpy(ht, th, V * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(hu, u, 2 * V * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(hg, g, 2 * V * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess,
          "copy back");
    double sum = 0.0, umax = 0.0, err = 0.0;
    for (int64_t k = 0; k < V; ++k) sum += ht[k];
    for (int64_t k = 0; k < 2 * V; ++k) umax = fmax(umax, fabs(hu[k]));
    for (int a = 0; a < 2; ++a)
        for (int64_t k = 0; k < V; ++k)
            err = fmax(err, fabs(-2.0 * c.nu * hg[a * V + k] / ht[k] - hu[a * V + k]));
    CHECK(fabs(sum - sum0) <= 1e-12 * sum0, "theta not conserved: %.17g vs %.17g", sum, sum0);
    CHECK(umax > 1e-3 && err <= 1e-13 * umax, "Cole-Hopf relation: err %.3g, max|u| %.3g", err,
          umax);
    CHECK(lb_destroy(s) == LB_OK, "lb_destroy");
    hipFree(fa);
    hipFree(fb);
    hipFree(th0);
    hipFree(th);
    hipFree(u);
    hipFree(g);
    free(h0);
    free(ht);
    free(hu);
    free(hg);
    return 0;
}

int main(int argc, char** argv) {
    const int no_gpu = argc > 1 && strcmp(argv[1], "--no-gpu") == 0;
    if (host_checks() != 0) return 1;
    if (!no_gpu && gpu_run() != 0) return 1;
    printf("ok\n");
    return 0;
}
