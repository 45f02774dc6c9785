/* Driver for the sanitizer build of the CPU oracle (test infrastructure).
 *
 * Built together with oracle/lbm_oracle.c under -fsanitize=address,undefined
 * by tests/test_oracle_sanitized.py, it calls every exported oracle routine
 * on small grids of each lattice (ragged sizes, one-node axes, the bounded
 * interval) with buffers allocated to their exact sizes, so any read or write
 * past an array, any use of uninitialised heap memory the sanitizers see and
 * any undefined arithmetic ends the run with a report.  Prints "ok" at the end. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_num_threads(void);
void oracle_set_threads(int n);
int oracle_lattice(int d, double eps, int* e, double* M, double* Minv, double* s, double* w,
                   double* ds, double* dw);
int oracle_grad_fd4(int d, const int64_t* n, double dx, const double* theta, double* grad);
int oracle_grad_fd4_transpose(int d, const int64_t* n, double dx, const double* g_grad,
                              double* g_theta);
int oracle_init(int d, const int64_t* n, double dx, double dt, double nu, const double* theta0,
                const double* grad, double* f);
int oracle_run(int d, const int64_t* n, double dx, double dt, double nu, double* f,
               int64_t nsteps);
int oracle_run_dirichlet1(int64_t n, double dx, double dt, double nu, double* f, int64_t nsteps,
                          const double* walls);
int oracle_macro(int d, const int64_t* n, double dx, double dt, double nu, const double* f,
                 double* theta, double* u);
int oracle_grad_theta(int d, const int64_t* n, double dx, double dt, double nu, const double* f,
                      double* grad);
int oracle_collision_matrix(int d, double eps, double* C, double* dC);
int oracle_macro_adjoint(int d, const int64_t* n, double dx, double dt, double nu,
                         const double* f, const double* g_theta, const double* g_u,
                         double* lambda, double* g_eps);
int oracle_adjoint_run(int d, const int64_t* n, double dx, double dt, double nu,
                       const double* f0, int64_t nsteps, double* lambda, double* g_eps);
int oracle_init_adjoint(int d, const int64_t* n, double dx, double dt, double nu,
                        const double* theta0, const double* grad, const double* lambda0,
                        double* g_theta0, double* g_grad, double* g_eps);
int oracle_theta_from_velocity(int d, const int64_t* n, double dx, double nu, const double* u0,
                               double* theta0, double* grad);

static int failures = 0;

static void expect(int rc, const char* what) {
    if (rc != 0) {
        fprintf(stderr, "FAIL %s: rc %d\n", what, rc);
        ++failures;
    }
}

static double* alloc(size_t n, double fill) {
    double* p = (double*)malloc(n * sizeof(double));
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    for (size_t i = 0; i < n; ++i) p[i] = fill + 0.01 * (double)(i % 7);
    return p;
}

static void one_grid(int d, const int64_t* n, double eps) {
    const int q = 1 + 2 * d * d;
    int64_t V = 1;
    for (int a = 0; a < d; ++a) V *= n[a];
    const double dx = 0.1, nu = 0.02, dt = eps * dx * dx / nu;
    double* th = alloc((size_t)V, 1.0);
    double* g = alloc((size_t)(d * V), 0.0);
    double* f = alloc((size_t)(q * V), 0.0);
    double* u = alloc((size_t)(d * V), 0.0);
    double* gt = alloc((size_t)(d * V), 0.0);
    double* lam = alloc((size_t)(q * V), 0.1);
    double* gth = alloc((size_t)V, 0.0);
    double* gg = alloc((size_t)(d * V), 0.0);
    double ge = 0.0;
    expect(oracle_grad_fd4(d, n, dx, th, g), "grad_fd4");
    expect(oracle_grad_fd4_transpose(d, n, dx, g, gth), "grad_fd4_transpose");
    expect(oracle_init(d, n, dx, dt, nu, th, g, f), "init");
    expect(oracle_run(d, n, dx, dt, nu, f, 3), "run");
    expect(oracle_macro(d, n, dx, dt, nu, f, th, u), "macro");
    expect(oracle_macro(d, n, dx, dt, nu, f, NULL, u), "macro (no theta)");
    expect(oracle_grad_theta(d, n, dx, dt, nu, f, gt), "grad_theta");
    expect(oracle_macro_adjoint(d, n, dx, dt, nu, f, th, u, lam, &ge), "macro_adjoint");
    expect(oracle_macro_adjoint(d, n, dx, dt, nu, f, NULL, u, lam, &ge), "macro_adjoint (g_u)");
    expect(oracle_adjoint_run(d, n, dx, dt, nu, f, 3, lam, &ge), "adjoint_run");
    expect(oracle_init_adjoint(d, n, dx, dt, nu, th, g, lam, gth, gg, &ge), "init_adjoint");
    /* a constant gradient field integrates to a periodic potential only when
       it vanishes, so the front end gets u0 = 0 (theta0 = 1) */
    for (int64_t k = 0; k < d * V; ++k) u[k] = 0.0;
    expect(oracle_theta_from_velocity(d, n, dx, nu, u, th, g), "theta_from_velocity");
    if (!isfinite(ge)) {
        fprintf(stderr, "FAIL non-finite eps gradient\n");
        ++failures;
    }
    free(th); free(g); free(f); free(u); free(gt); free(lam); free(gth); free(gg);
}

int main(void) {
    oracle_set_threads(2);
    if (oracle_num_threads() < 1) ++failures;
    for (int d = 1; d <= 4; ++d) {
        const int q = 1 + 2 * d * d;
        int* e = (int*)malloc(sizeof(int) * (size_t)(q * d));
        double* M = alloc((size_t)(q * q), 0.0);
        double* Mi = alloc((size_t)(q * q), 0.0);
        double* C = alloc((size_t)(q * q), 0.0);
        double* dC = alloc((size_t)(q * q), 0.0);
        double* vec[4];
        for (int k = 0; k < 4; ++k) vec[k] = alloc((size_t)q, 0.0);
        /* these two return q on success */
        expect(oracle_lattice(d, 0.11, e, M, Mi, vec[0], vec[1], vec[2], vec[3]) - q, "lattice");
        expect(oracle_collision_matrix(d, 0.11, C, dC) - q, "collision_matrix");
        free(e); free(M); free(Mi); free(C); free(dC);
        for (int k = 0; k < 4; ++k) free(vec[k]);
    }
    const int64_t g1[4] = {7, 1, 1, 1}, g1b[4] = {1, 1, 1, 1};
    const int64_t g2[4] = {5, 3, 1, 1}, g2b[4] = {1, 4, 1, 1};
    const int64_t g3[4] = {4, 3, 2, 1}, g3b[4] = {1, 1, 3, 1};
    const int64_t g4[4] = {3, 2, 2, 3};
    one_grid(1, g1, 0.3);
    one_grid(1, g1b, 0.3);
    one_grid(2, g2, 0.2);
    one_grid(2, g2b, 0.2);
    one_grid(3, g3, 0.1);
    one_grid(3, g3b, 0.1);
    one_grid(4, g4, 0.05);
    /* bounded interval of Example 1: two nodes, then nine */
    for (int64_t n = 2; n <= 9; n += 7) {
        double* f = alloc((size_t)(3 * n), 0.3);
        double* walls = alloc((size_t)(2 * 4), 1.0);
        expect(oracle_run_dirichlet1(n, 0.1, 0.01, 0.5, f, 4, walls), "run_dirichlet1");
        free(f); free(walls);
    }
    if (failures) {
        fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
