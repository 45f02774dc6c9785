/*
 * CPU oracle for the Cole-Hopf fourth-order MRT lattice Boltzmann scheme
 * (Chen, Liu, Chai & Shi, arXiv:2309.02825).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  The product path (the HIP
 * library) never calls it and shares no source with it.
 *
 * Plain, slow, generic double-precision code: the lattice tables and the
 * moment matrix M are typed from Sec. III.A, M^-1 is computed numerically by
 * Gauss-Jordan elimination, the collision is done as explicit q x q
 * matrix-vector products in moment space, and streaming is the literal push
 * f_i(x + e_i, t + dt) = f*_i(x, t).  OpenMP parallelises over nodes only.
 *
 * Conventions
 *   - node index  k = x_0 + n_0 * (x_1 + n_1 * (x_2 + n_2 * x_3))  (x_0 fastest)
 *   - distributions are structure-of-arrays: f[i * V + k], V = prod n
 *   - velocities are kept in lattice units e_i in {-1,0,1}^d; c = dx/dt.
 *     Scaling the rows of M by powers of c leaves M^-1 S M unchanged because
 *     S is diagonal, so M is built from e_i.
 *   - periodic boundaries in every direction (Examples 2-4 of Sec. IV), and
 *     for d = 1 the bounded interval of Example 1 (oracle_run_dirichlet1).
 *
 * Readings of the paper taken here (listed with their justification in the
 * design notes of the repository):
 *   - initialisation f = f^eq - dt * Lambda^{-1} Dbar f^eq uses
 *     Lambda^{-1} = M^-1 S^-1 M (the inverse of the relaxation operator seen
 *     by the distribution), s_0 = 1.
 *   - the velocity is formed from the pre-collision (post-streaming) f.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXD 4
#define OR_MAXQ 33

typedef struct {
    int d, q, nmom;
    int e[OR_MAXQ][OR_MAXD];
    double M[OR_MAXQ][OR_MAXQ];
    double Minv[OR_MAXQ][OR_MAXQ];
    double s[OR_MAXQ];   /* diagonal of S */
    double w[OR_MAXQ];   /* weights */
    double ds[OR_MAXQ];  /* d s / d eps */
    double dw[OR_MAXQ];  /* d w / d eps */
    double eps, s1, s21, s22, w0, w1, wd;
    double ds1;
} or_lattice;

/* ------------------------------------------------------------------------ */
/* Lattice velocities, Sec. III.A.                                           */
/* ------------------------------------------------------------------------ */

/* D1Q3: c_x1 = (0, 1, -1) c. */
static const int D1Q3_E[3][1] = {{0}, {1}, {-1}};

/* D2Q9: c_x1 = (0,1,0,-1,0,1,-1,-1,1) c, c_x2 = (0,0,1,0,-1,1,1,-1,-1) c. */
static const int D2Q9_CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int D2Q9_CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

/* D3Q19 velocity components as printed. */
static const int D3Q19_CX[19] = {0, 1, 0, 0, -1, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1, 0, 0, 0, 0};
static const int D3Q19_CY[19] = {0, 0, 1, 0, 0, -1, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, -1, 1};
static const int D3Q19_CZ[19] = {0, 0, 0, 1, 0, 0, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};

/* Rows of M as exponent tuples (p_1, ..., p_d): row r of M is
 * prod_a e_{i,a}^{p_a}.  Order as printed for d = 1, 2, 3. */
static const int D1_ROWS[3][1] = {{0}, {1}, {2}};
static const int D2_ROWS[9][2] = {{0, 0}, {1, 0}, {0, 1}, {2, 0}, {0, 2},
                                  {1, 1}, {1, 2}, {2, 1}, {2, 2}};
static const int D3_ROWS[19][3] = {
    {0, 0, 0},                                   /* 1 */
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1},             /* c_a */
    {2, 0, 0}, {0, 2, 0}, {0, 0, 2},             /* c_a^2 */
    {1, 1, 0}, {1, 0, 1}, {0, 1, 1},             /* c_a c_b */
    {1, 2, 0}, {2, 1, 0}, {1, 0, 2}, {2, 0, 1},  /* c_a c_b^2, c_a^2 c_b */
    {0, 1, 2}, {0, 2, 1},
    {2, 2, 0}, {2, 0, 2}, {0, 2, 2}};            /* c_a^2 c_b^2 */

/* Kind of each moment row: 0 conserved, 1 first order (s1), 2 diagonal
 * second order (s21, or s2 in 1D), 3 mixed second order (s22), 4 third and
 * fourth order (relaxation rate 1). */
static int row_kind(const int* p, int d) {
    int deg = 0, nz = 0, maxp = 0;
    for (int a = 0; a < d; ++a) {
        deg += p[a];
        if (p[a]) ++nz;
        if (p[a] > maxp) maxp = p[a];
    }
    if (deg == 0) return 0;
    if (deg == 1) return 1;
    if (deg == 2 && nz == 1) return 2;
    if (deg == 2 && nz == 2) return 3;
    return 4;
}

/* General DdQ(1+2d^2) velocity set for d > 3 (Sec. III.A, the d > 3 case):
 * rest, +unit vectors, -unit vectors, then for every pair a < b in
 * lexicographic order the four velocities with (e_a, e_b) =
 * (1,1), (-1,1), (-1,-1), (1,-1).  For d = 2, 3 this rule reproduces the
 * printed tables (checked by the tests). */
static int general_velocities(int d, int e[OR_MAXQ][OR_MAXD]) {
    int q = 0;
    memset(e, 0, sizeof(int) * OR_MAXQ * OR_MAXD);
    ++q;
    for (int a = 0; a < d; ++a) { e[q][a] = 1; ++q; }
    for (int a = 0; a < d; ++a) { e[q][a] = -1; ++q; }
    static const int J1[4] = {1, -1, -1, 1};
    static const int J2[4] = {1, 1, -1, -1};
    for (int a = 0; a < d; ++a)
        for (int b = a + 1; b < d; ++b)
            for (int k = 0; k < 4; ++k) { e[q][a] = J1[k]; e[q][b] = J2[k]; ++q; }
    return q;
}

/* Rows of M for d > 3: 1; c_a; c_a^2; c_a c_b (a<b); c_a c_b^2 (a<b);
 * c_a^2 c_b (a<b); c_a^2 c_b^2 (a<b). */
static int general_rows(int d, int rows[OR_MAXQ][OR_MAXD]) {
    int r = 0;
    memset(rows, 0, sizeof(int) * OR_MAXQ * OR_MAXD);
    ++r;
    for (int a = 0; a < d; ++a) { rows[r][a] = 1; ++r; }
    for (int a = 0; a < d; ++a) { rows[r][a] = 2; ++r; }
    for (int a = 0; a < d; ++a)
        for (int b = a + 1; b < d; ++b) { rows[r][a] = 1; rows[r][b] = 1; ++r; }
    for (int a = 0; a < d; ++a)
        for (int b = a + 1; b < d; ++b) { rows[r][a] = 1; rows[r][b] = 2; ++r; }
    for (int a = 0; a < d; ++a)
        for (int b = a + 1; b < d; ++b) { rows[r][a] = 2; rows[r][b] = 1; ++r; }
    for (int a = 0; a < d; ++a)
        for (int b = a + 1; b < d; ++b) { rows[r][a] = 2; rows[r][b] = 2; ++r; }
    return r;
}

/* Gauss-Jordan inverse with partial pivoting.  Returns 0 on success. */
static int invert(int q, double A[OR_MAXQ][OR_MAXQ], double Ainv[OR_MAXQ][OR_MAXQ]) {
    double T[OR_MAXQ][2 * OR_MAXQ];
    for (int i = 0; i < q; ++i) {
        for (int j = 0; j < q; ++j) {
            T[i][j] = A[i][j];
            T[i][q + j] = (i == j) ? 1.0 : 0.0;
        }
    }
    for (int c = 0; c < q; ++c) {
        int piv = c;
        for (int r = c + 1; r < q; ++r)
            if (fabs(T[r][c]) > fabs(T[piv][c])) piv = r;
        if (fabs(T[piv][c]) < 1e-12) return -1;
        if (piv != c)
            for (int j = 0; j < 2 * q; ++j) { double t = T[c][j]; T[c][j] = T[piv][j]; T[piv][j] = t; }
        double inv = 1.0 / T[c][c];
        for (int j = 0; j < 2 * q; ++j) T[c][j] *= inv;
        for (int r = 0; r < q; ++r) {
            if (r == c) continue;
            double fct = T[r][c];
            if (fct == 0.0) continue;
            for (int j = 0; j < 2 * q; ++j) T[r][j] -= fct * T[c][j];
        }
    }
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j) Ainv[i][j] = T[i][q + j];
    return 0;
}

/* Build the lattice, M, M^-1, S and the weights for a given eps.
 * Parameters from Theorem 2, Sec. III.D (the parameter solution, Bur-Sol):
 *   s1  = 2/(6 eps + 1)
 *   s21 = 24 eps/(6 eps + 1)^2     (called s2 when d = 1)
 *   s22 = 4/(6 eps + 3)
 *   w1  = 1/6 - (d - 1) eps/3,  w_{1+2d} = eps/6  (d > 1);  w1 = 1/6 (d = 1)
 *   w0  = 1 - 2 d w1 - 2 d (d - 1) w_{1+2d}  (weight structure, Sec. III.A)
 * s0 is free because theta is conserved; the oracle uses s0 = 1. */
static int build_lattice(int d, double eps, or_lattice* L) {
    if (d < 1 || d > OR_MAXD) return -1;
    memset(L, 0, sizeof(*L));
    L->d = d;
    int rows[OR_MAXQ][OR_MAXD];
    memset(rows, 0, sizeof(rows));
    if (d == 1) {
        L->q = 3;
        for (int i = 0; i < 3; ++i) L->e[i][0] = D1Q3_E[i][0];
        for (int r = 0; r < 3; ++r) rows[r][0] = D1_ROWS[r][0];
    } else if (d == 2) {
        L->q = 9;
        for (int i = 0; i < 9; ++i) { L->e[i][0] = D2Q9_CX[i]; L->e[i][1] = D2Q9_CY[i]; }
        for (int r = 0; r < 9; ++r) { rows[r][0] = D2_ROWS[r][0]; rows[r][1] = D2_ROWS[r][1]; }
    } else if (d == 3) {
        L->q = 19;
        for (int i = 0; i < 19; ++i) {
            L->e[i][0] = D3Q19_CX[i]; L->e[i][1] = D3Q19_CY[i]; L->e[i][2] = D3Q19_CZ[i];
        }
        for (int r = 0; r < 19; ++r)
            for (int a = 0; a < 3; ++a) rows[r][a] = D3_ROWS[r][a];
    } else {
        L->q = general_velocities(d, L->e);
        if (general_rows(d, rows) != L->q) return -1;
    }
    const int q = L->q;
    L->nmom = q;

    /* M_{r i} = prod_a e_{i a}^{p_{r a}} */
    for (int r = 0; r < q; ++r) {
        for (int i = 0; i < q; ++i) {
            double v = 1.0;
            for (int a = 0; a < d; ++a)
                for (int k = 0; k < rows[r][a]; ++k) v *= (double)L->e[i][a];
            L->M[r][i] = v;
        }
    }
    if (invert(q, L->M, L->Minv) != 0) return -2;

    L->eps = eps;
    const double a6 = 6.0 * eps + 1.0;
    L->s1 = 2.0 / a6;
    L->s21 = 24.0 * eps / (a6 * a6);
    L->s22 = 4.0 / (6.0 * eps + 3.0);
    L->ds1 = -12.0 / (a6 * a6);
    const double ds21 = 24.0 * (1.0 - 6.0 * eps) / (a6 * a6 * a6);
    const double ds22 = -24.0 / ((6.0 * eps + 3.0) * (6.0 * eps + 3.0));
    double dw1, dwd;
    if (d == 1) {
        L->w1 = 1.0 / 6.0; L->wd = 0.0; dw1 = 0.0; dwd = 0.0;
    } else {
        L->w1 = 1.0 / 6.0 - (d - 1) * eps / 3.0; L->wd = eps / 6.0;
        dw1 = -(d - 1) / 3.0; dwd = 1.0 / 6.0;
    }
    L->w0 = 1.0 - 2.0 * d * L->w1 - 2.0 * d * (d - 1) * L->wd;
    const double dw0 = -2.0 * d * dw1 - 2.0 * d * (d - 1) * dwd;

    for (int r = 0; r < q; ++r) {
        switch (row_kind(rows[r], d)) {
            case 0: L->s[r] = 1.0; L->ds[r] = 0.0; break;
            case 1: L->s[r] = L->s1; L->ds[r] = L->ds1; break;
            case 2: L->s[r] = L->s21; L->ds[r] = ds21; break;
            case 3: L->s[r] = L->s22; L->ds[r] = ds22; break;
            default: L->s[r] = 1.0; L->ds[r] = 0.0; break;
        }
    }
    for (int i = 0; i < q; ++i) {
        int n1 = 0;
        for (int a = 0; a < d; ++a) n1 += abs(L->e[i][a]);
        if (n1 == 0) { L->w[i] = L->w0; L->dw[i] = dw0; }
        else if (n1 == 1) { L->w[i] = L->w1; L->dw[i] = dw1; }
        else { L->w[i] = L->wd; L->dw[i] = dwd; }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Grid helpers                                                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    int d;
    int64_t n[OR_MAXD];
    int64_t V;
} or_grid;

static int make_grid(int d, const int64_t* n, or_grid* G) {
    if (d < 1 || d > OR_MAXD) return -1;
    G->d = d;
    G->V = 1;
    for (int a = 0; a < OR_MAXD; ++a) G->n[a] = 1;
    for (int a = 0; a < d; ++a) {
        if (n[a] < 1) return -1;
        G->n[a] = n[a];
        G->V *= n[a];
    }
    return 0;
}

/* Index of the node k shifted by the integer vector sh, periodic wrap. */
static int64_t shifted(const or_grid* G, int64_t k, const int* sh) {
    int64_t idx = 0, stride = 1, rem = k;
    for (int a = 0; a < G->d; ++a) {
        int64_t x = rem % G->n[a];
        rem /= G->n[a];
        int64_t y = (x + sh[a]) % G->n[a];
        if (y < 0) y += G->n[a];
        idx += y * stride;
        stride *= G->n[a];
    }
    return idx;
}

/* ------------------------------------------------------------------------ */
/* Exported API                                                              */
/* ------------------------------------------------------------------------ */

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Lattice description: q, velocities e (q x d, row-major), M and M^-1
 * (q x q, row-major), s (q), w (q), ds/deps (q), dw/deps (q).
 * Returns q, or a negative value on error. */
int oracle_lattice(int d, double eps, int* e_out, double* M_out, double* Minv_out,
                   double* s_out, double* w_out, double* ds_out, double* dw_out) {
    or_lattice L;
    if (build_lattice(d, eps, &L) != 0) return -1;
    const int q = L.q;
    for (int i = 0; i < q; ++i) {
        if (e_out) for (int a = 0; a < d; ++a) e_out[i * d + a] = L.e[i][a];
        if (s_out) s_out[i] = L.s[i];
        if (w_out) w_out[i] = L.w[i];
        if (ds_out) ds_out[i] = L.ds[i];
        if (dw_out) dw_out[i] = L.dw[i];
        for (int j = 0; j < q; ++j) {
            if (M_out) M_out[i * q + j] = L.M[i][j];
            if (Minv_out) Minv_out[i * q + j] = L.Minv[i][j];
        }
    }
    return q;
}

/* Fourth-order central difference of theta along every axis (the reading
 * used when only the field theta0 is given):
 *   d_a theta(x) = (-theta(x+2) + 8 theta(x+1) - 8 theta(x-1) + theta(x-2)) / (12 dx)
 * grad is d x V. */
int oracle_grad_fd4(int d, const int64_t* n, double dx, const double* theta, double* grad) {
    or_grid G;
    if (make_grid(d, n, &G) != 0 || !(dx > 0)) return -1;
    for (int a = 0; a < d; ++a) {
        int p1[OR_MAXD] = {0}, p2[OR_MAXD] = {0}, m1[OR_MAXD] = {0}, m2[OR_MAXD] = {0};
        p1[a] = 1; p2[a] = 2; m1[a] = -1; m2[a] = -2;
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < G.V; ++k) {
            double tp1 = theta[shifted(&G, k, p1)], tp2 = theta[shifted(&G, k, p2)];
            double tm1 = theta[shifted(&G, k, m1)], tm2 = theta[shifted(&G, k, m2)];
            grad[a * G.V + k] = (-tp2 + 8.0 * tp1 - 8.0 * tm1 + tm2) / (12.0 * dx);
        }
    }
    return 0;
}

/* Transpose of oracle_grad_fd4: g_theta += sum_a D_a^T g_grad_a, formed by
 * scattering each stencil tap (no use of the antisymmetry of the stencil). */
int oracle_grad_fd4_transpose(int d, const int64_t* n, double dx, const double* g_grad,
                              double* g_theta) {
    or_grid G;
    if (make_grid(d, n, &G) != 0 || !(dx > 0)) return -1;
    const double c[4] = {-1.0, 8.0, -8.0, 1.0};
    const int off[4] = {2, 1, -1, -2};
    for (int a = 0; a < d; ++a) {
        for (int t = 0; t < 4; ++t) {
            int sh[OR_MAXD] = {0};
            sh[a] = off[t];
            /* serial: the scatter targets of one tap form a permutation, but
             * keep it obviously race free */
            for (int64_t k = 0; k < G.V; ++k)
                g_theta[shifted(&G, k, sh)] += c[t] / (12.0 * dx) * g_grad[a * G.V + k];
        }
    }
    return 0;
}

/* Initial distribution from the first two terms of the fourth-order
 * expansion of f (Theorem 1, Sec. III.C; used as initial condition in
 * Sec. IV):  f = f^eq - dt Lambda^{-1} Dbar f^eq, with f^eq_i = w_i theta0
 * (Sec. III.A), Dbar = diag(c_i . grad) and Lambda^{-1} = M^-1 S^-1 M.
 * Since c_i = (dx/dt) e_i, dt * Dbar f^eq = dx * w_i (e_i . grad theta0). */
int oracle_init(int d, const int64_t* n, double dx, double dt, double nu,
                const double* theta0, const double* grad, double* f) {
    or_grid G;
    or_lattice L;
    if (make_grid(d, n, &G) != 0 || !(dx > 0) || !(dt > 0) || !(nu > 0)) return -1;
    if (build_lattice(d, nu * dt / (dx * dx), &L) != 0) return -1;
    const int q = L.q;
    const int64_t V = G.V;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < V; ++k) {
        double g[OR_MAXQ], y[OR_MAXQ];
        for (int i = 0; i < q; ++i) {
            double eg = 0.0;
            for (int a = 0; a < d; ++a) eg += L.e[i][a] * grad[a * V + k];
            g[i] = L.w[i] * eg;
        }
        for (int r = 0; r < q; ++r) {
            double acc = 0.0;
            for (int i = 0; i < q; ++i) acc += L.M[r][i] * g[i];
            y[r] = acc / L.s[r];
        }
        for (int i = 0; i < q; ++i) {
            double acc = 0.0;
            for (int r = 0; r < q; ++r) acc += L.Minv[i][r] * y[r];
            f[i * V + k] = L.w[i] * theta0[k] - dx * acc;
        }
    }
    return 0;
}

/* One collision at one node in moment space (Sec. III.A evolution equation):
 *   theta = sum_i f_i,  m = M f,  m^eq = M (w theta),
 *   m*_r = m_r - s_r (m_r - m^eq_r),  f* = M^-1 m*. */
static void collide_node(const or_lattice* L, const double* fin, double* fout) {
    const int q = L->q;
    double theta = 0.0;
    for (int i = 0; i < q; ++i) theta += fin[i];
    double mstar[OR_MAXQ];
    for (int r = 0; r < q; ++r) {
        double m = 0.0, meq = 0.0;
        for (int i = 0; i < q; ++i) {
            m += L->M[r][i] * fin[i];
            meq += L->M[r][i] * L->w[i] * theta;
        }
        mstar[r] = m - L->s[r] * (m - meq);
    }
    for (int i = 0; i < q; ++i) {
        double acc = 0.0;
        for (int r = 0; r < q; ++r) acc += L->Minv[i][r] * mstar[r];
        fout[i] = acc;
    }
}

/* Advance f (q x V, pre-collision state at time t) by nsteps time steps:
 * collide at every node, then push f*_i(x) to x + e_i (periodic). */
int oracle_run(int d, const int64_t* n, double dx, double dt, double nu,
               double* f, int64_t nsteps) {
    or_grid G;
    or_lattice L;
    if (make_grid(d, n, &G) != 0 || !(dx > 0) || !(dt > 0) || !(nu > 0) || nsteps < 0)
        return -1;
    if (build_lattice(d, nu * dt / (dx * dx), &L) != 0) return -1;
    const int q = L.q;
    const int64_t V = G.V;
    double* tmp = (double*)malloc(sizeof(double) * (size_t)q * (size_t)V);
    if (!tmp) return -4;
    for (int64_t s = 0; s < nsteps; ++s) {
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < V; ++k) {
            double fin[OR_MAXQ], fout[OR_MAXQ];
            for (int i = 0; i < q; ++i) fin[i] = f[i * V + k];
            collide_node(&L, fin, fout);
            for (int i = 0; i < q; ++i) tmp[i * V + shifted(&G, k, L.e[i])] = fout[i];
        }
        memcpy(f, tmp, sizeof(double) * (size_t)q * (size_t)V);
    }
    free(tmp);
    return 0;
}

/* Example 1 of Sec. IV on the bounded interval: n nodes x_j = j dx,
 * j = 0..n-1, with the end nodes on the boundary, where theta is given.
 * One step: collide at every node, push f*_i to x + e_i where that node
 * exists (populations leaving the interval are dropped), then give each end
 * node the one population the push could not deliver (the one pointing into
 * the interval) the value that makes sum_i f_i equal the boundary theta at
 * the new time:
 *   f_{+1}(x_0)     = theta_left  - f_0(x_0)     - f_{-1}(x_0),
 *   f_{-1}(x_{n-1}) = theta_right - f_0(x_{n-1}) - f_{+1}(x_{n-1}).
 * walls holds 2 * nsteps values, (theta_left, theta_right) at t + dt,
 * t + 2 dt, ...  f is 3 x n (pre-collision), advanced in place. */
int oracle_run_dirichlet1(int64_t n, double dx, double dt, double nu, double* f, int64_t nsteps,
                          const double* walls) {
    or_lattice L;
    if (n < 2 || !(dx > 0) || !(dt > 0) || !(nu > 0) || nsteps < 0 || (nsteps > 0 && !walls))
        return -1;
    if (build_lattice(1, nu * dt / (dx * dx), &L) != 0) return -1;
    const int q = L.q;
    double* tmp = (double*)malloc(sizeof(double) * (size_t)q * (size_t)n);
    if (!tmp) return -4;
    for (int64_t s = 0; s < nsteps; ++s) {
        for (int64_t k = 0; k < n; ++k) {
            double fin[OR_MAXQ], fout[OR_MAXQ];
            for (int i = 0; i < q; ++i) fin[i] = f[i * n + k];
            collide_node(&L, fin, fout);
            for (int i = 0; i < q; ++i) {
                const int64_t to = k + L.e[i][0];
                if (to >= 0 && to < n) tmp[i * n + to] = fout[i];
            }
        }
        for (int i = 0; i < q; ++i) {
            if (L.e[i][0] == 1) {
                double rest = 0.0;
                for (int j = 0; j < q; ++j)
                    if (j != i) rest += tmp[j * n + 0];
                tmp[i * n + 0] = walls[2 * s] - rest;
            } else if (L.e[i][0] == -1) {
                double rest = 0.0;
                for (int j = 0; j < q; ++j)
                    if (j != i) rest += tmp[j * n + n - 1];
                tmp[i * n + n - 1] = walls[2 * s + 1] - rest;
            }
        }
        memcpy(f, tmp, sizeof(double) * (size_t)q * (size_t)n);
    }
    free(tmp);
    return 0;
}

/* Macroscopic output from the pre-collision f (Sec. III.C):
 *   theta = sum_k f_k,  f^ne = f - w theta,
 *   u_a = (2 - s1) sum_k c_{ka} f^ne_k / sum_k f_k,  c_{ka} = (dx/dt) e_{ka}.
 * theta is V, u is d x V; either may be NULL. */
int oracle_macro(int d, const int64_t* n, double dx, double dt, double nu,
                 const double* f, double* theta, double* u) {
    or_grid G;
    or_lattice L;
    if (make_grid(d, n, &G) != 0 || !(dx > 0) || !(dt > 0) || !(nu > 0)) return -1;
    if (build_lattice(d, nu * dt / (dx * dx), &L) != 0) return -1;
    const int q = L.q;
    const int64_t V = G.V;
    const double c = dx / dt;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < V; ++k) {
        double th = 0.0;
        for (int i = 0; i < q; ++i) th += f[i * V + k];
        if (theta) theta[k] = th;
        if (u) {
            for (int a = 0; a < d; ++a) {
                double j = 0.0;
                for (int i = 0; i < q; ++i) j += c * L.e[i][a] * (f[i * V + k] - L.w[i] * th);
                u[a * V + k] = (2.0 - L.s1) * j / th;
            }
        }
    }
    return 0;
}

/* Gradient of theta from the non-equilibrium first moment (Sec. III.C):
 *   grad theta = -(s1 / (dt c_s^2)) sum_k c_k f^ne_k,  c_s^2 = [2 w1 + 4(d-1) w_{1+2d}] c^2. */
int oracle_grad_theta(int d, const int64_t* n, double dx, double dt, double nu,
                      const double* f, double* grad) {
    or_grid G;
    or_lattice L;
    if (make_grid(d, n, &G) != 0 || !(dx > 0) || !(dt > 0) || !(nu > 0)) return -1;
    if (build_lattice(d, nu * dt / (dx * dx), &L) != 0) return -1;
    const int q = L.q;
    const int64_t V = G.V;
    const double c = dx / dt;
    const double cs2 = (2.0 * L.w1 + 4.0 * (d - 1) * L.wd) * c * c;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < V; ++k) {
        double th = 0.0;
        for (int i = 0; i < q; ++i) th += f[i * V + k];
        for (int a = 0; a < d; ++a) {
            double j = 0.0;
            for (int i = 0; i < q; ++i) j += c * L.e[i][a] * (f[i * V + k] - L.w[i] * th);
            grad[a * V + k] = -L.s1 / (dt * cs2) * j;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Discrete adjoint.  The forward map is f^{n+1} = P C f^n with the per-node
 * collision matrix C = I - M^-1 S M (I - w 1^T) and the streaming
 * permutation P.  Its adjoint is lambda^n = C^T P^T lambda^{n+1}; the
 * derivative with respect to eps adds <P^T lambda^{n+1}, (dC/deps) f^n>,
 * where dC/deps = -M^-1 S' M (I - w 1^T) + M^-1 S M w' 1^T.                */
/* ------------------------------------------------------------------------ */

static void collision_matrices(const or_lattice* L, double C[OR_MAXQ][OR_MAXQ],
                               double dC[OR_MAXQ][OR_MAXQ]) {
    const int q = L->q;
    double Mw[OR_MAXQ], Mdw[OR_MAXQ];
    for (int r = 0; r < q; ++r) {
        Mw[r] = 0.0; Mdw[r] = 0.0;
        for (int j = 0; j < q; ++j) { Mw[r] += L->M[r][j] * L->w[j]; Mdw[r] += L->M[r][j] * L->dw[j]; }
    }
    for (int i = 0; i < q; ++i) {
        for (int k = 0; k < q; ++k) {
            double a = 0.0, b = 0.0;
            for (int r = 0; r < q; ++r) {
                double Pk = L->M[r][k] - Mw[r];      /* (M (I - w 1^T))_{rk} */
                a += L->Minv[i][r] * L->s[r] * Pk;
                b += -L->Minv[i][r] * L->ds[r] * Pk + L->Minv[i][r] * L->s[r] * Mdw[r];
            }
            C[i][k] = (i == k ? 1.0 : 0.0) - a;
            dC[i][k] = b;
        }
    }
}

/* Collision matrix and its eps derivative (q x q row-major), for tests. */
int oracle_collision_matrix(int d, double eps, double* C_out, double* dC_out) {
    or_lattice L;
    if (build_lattice(d, eps, &L) != 0) return -1;
    double C[OR_MAXQ][OR_MAXQ], dC[OR_MAXQ][OR_MAXQ];
    collision_matrices(&L, C, dC);
    for (int i = 0; i < L.q; ++i)
        for (int k = 0; k < L.q; ++k) {
            if (C_out) C_out[i * L.q + k] = C[i][k];
            if (dC_out) dC_out[i * L.q + k] = dC[i][k];
        }
    return L.q;
}

/* Adjoint of the macroscopic output.  Given dL/dtheta (V, may be NULL) and
 * dL/du (d x V, may be NULL) at the state f, writes lambda = dL/df (q x V)
 * and adds the explicit eps dependence of u (through s1) to *g_eps. */
int oracle_macro_adjoint(int d, const int64_t* n, double dx, double dt, double nu,
                         const double* f, const double* g_theta, const double* g_u,
                         double* lambda, double* g_eps) {
    or_grid G;
    or_lattice L;
    if (make_grid(d, n, &G) != 0 || !(dx > 0) || !(dt > 0) || !(nu > 0)) return -1;
    if (build_lattice(d, nu * dt / (dx * dx), &L) != 0) return -1;
    const int q = L.q;
    const int64_t V = G.V;
    const double c = dx / dt;
    double ge = 0.0;
    for (int64_t k = 0; k < V; ++k) {
        double th = 0.0;
        for (int i = 0; i < q; ++i) th += f[i * V + k];
        double gt = g_theta ? g_theta[k] : 0.0;
        double lam[OR_MAXQ];
        for (int i = 0; i < q; ++i) lam[i] = gt;
        if (g_u) {
            for (int a = 0; a < d; ++a) {
                double j = 0.0;
                for (int i = 0; i < q; ++i) j += c * L.e[i][a] * (f[i * V + k] - L.w[i] * th);
                const double ua = (2.0 - L.s1) * j / th;
                const double gu = g_u[a * V + k];
                /* d u_a / d f_i = (2 - s1) c e_{ia} / theta - u_a / theta */
                for (int i = 0; i < q; ++i)
                    lam[i] += gu * ((2.0 - L.s1) * c * L.e[i][a] / th - ua / th);
                /* d u_a / d eps = -s1' j / theta */
                ge += gu * (-L.ds1) * j / th;
            }
        }
        for (int i = 0; i < q; ++i) lambda[i * V + k] = lam[i];
    }
    if (g_eps) *g_eps += ge;
    return 0;
}

/* Full reverse sweep.  f0 is the state at step 0 (q x V); the forward
 * trajectory f^0..f^{nsteps-1} is recomputed and stored.  On entry lambda
 * holds dL/df^{nsteps}; on exit it holds dL/df^0.  The eps contribution of
 * the time steps is added to *g_eps. */
int oracle_adjoint_run(int d, const int64_t* n, double dx, double dt, double nu,
                       const double* f0, int64_t nsteps, double* lambda, double* g_eps) {
    or_grid G;
    or_lattice L;
    if (make_grid(d, n, &G) != 0 || !(dx > 0) || !(dt > 0) || !(nu > 0) || nsteps < 0)
        return -1;
    if (build_lattice(d, nu * dt / (dx * dx), &L) != 0) return -1;
    const int q = L.q;
    const int64_t V = G.V;
    const size_t qv = (size_t)q * (size_t)V;
    double* traj = (double*)malloc(sizeof(double) * qv * (size_t)(nsteps > 0 ? nsteps : 1));
    double* mu = (double*)malloc(sizeof(double) * qv);
    if (!traj || !mu) { free(traj); free(mu); return -4; }
    if (nsteps > 0) memcpy(traj, f0, sizeof(double) * qv);
    for (int64_t s = 1; s < nsteps; ++s) {
        memcpy(traj + qv * s, traj + qv * (s - 1), sizeof(double) * qv);
        int rc = oracle_run(d, n, dx, dt, nu, traj + qv * s, 1);
        if (rc) { free(traj); free(mu); return rc; }
    }
    double C[OR_MAXQ][OR_MAXQ], dC[OR_MAXQ][OR_MAXQ];
    collision_matrices(&L, C, dC);
    double ge = 0.0;
    for (int64_t s = nsteps - 1; s >= 0; --s) {
        const double* fn = traj + qv * s;
        /* mu = P^T lambda:  mu_i(x) = lambda_i(x + e_i) */
        for (int64_t k = 0; k < V; ++k)
            for (int i = 0; i < q; ++i) mu[i * V + k] = lambda[i * V + shifted(&G, k, L.e[i])];
        for (int64_t k = 0; k < V; ++k) {
            for (int i = 0; i < q; ++i) {
                double acc = 0.0;
                for (int kk = 0; kk < q; ++kk) acc += dC[i][kk] * fn[kk * V + k];
                ge += mu[i * V + k] * acc;
            }
            for (int kk = 0; kk < q; ++kk) {
                double acc = 0.0;
                for (int i = 0; i < q; ++i) acc += C[i][kk] * mu[i * V + k];
                lambda[kk * V + k] = acc;
            }
        }
    }
    if (g_eps) *g_eps += ge;
    free(traj);
    free(mu);
    return 0;
}

/* Adjoint of oracle_init.  Given lambda0 = dL/df^0, writes g_theta0 (V) and
 * g_grad (d x V, the gradient with respect to the grad-theta0 input), and
 * adds the eps dependence of the initial state to *g_eps. */
int oracle_init_adjoint(int d, const int64_t* n, double dx, double dt, double nu,
                        const double* theta0, const double* grad, const double* lambda0,
                        double* g_theta0, double* g_grad, double* g_eps) {
    or_grid G;
    or_lattice L;
    if (make_grid(d, n, &G) != 0 || !(dx > 0) || !(dt > 0) || !(nu > 0)) return -1;
    if (build_lattice(d, nu * dt / (dx * dx), &L) != 0) return -1;
    const int q = L.q;
    const int64_t V = G.V;
    /* B = M^-1 S^-1 M (maps g to Lambda^{-1} g), dB = M^-1 (S^-1)' M */
    double B[OR_MAXQ][OR_MAXQ], dB[OR_MAXQ][OR_MAXQ];
    for (int i = 0; i < q; ++i)
        for (int k = 0; k < q; ++k) {
            double a = 0.0, b = 0.0;
            for (int r = 0; r < q; ++r) {
                a += L.Minv[i][r] / L.s[r] * L.M[r][k];
                b += L.Minv[i][r] * (-L.ds[r] / (L.s[r] * L.s[r])) * L.M[r][k];
            }
            B[i][k] = a;
            dB[i][k] = b;
        }
    double ge = 0.0;
    for (int64_t k = 0; k < V; ++k) {
        const double* lam = NULL;
        double lv[OR_MAXQ], g[OR_MAXQ], dg[OR_MAXQ];
        for (int i = 0; i < q; ++i) lv[i] = lambda0[i * V + k];
        lam = lv;
        /* f_i = w_i theta0 - dx (B g)_i,  g_i = w_i (e_i . grad) */
        double gt = 0.0;
        for (int i = 0; i < q; ++i) gt += L.w[i] * lam[i];
        if (g_theta0) g_theta0[k] = gt;
        double BtL[OR_MAXQ];
        for (int kk = 0; kk < q; ++kk) {
            double acc = 0.0;
            for (int i = 0; i < q; ++i) acc += B[i][kk] * lam[i];
            BtL[kk] = acc;
        }
        if (g_grad) {
            for (int a = 0; a < d; ++a) {
                double acc = 0.0;
                for (int kk = 0; kk < q; ++kk) acc += BtL[kk] * L.w[kk] * L.e[kk][a];
                g_grad[a * V + k] = -dx * acc;
            }
        }
        for (int i = 0; i < q; ++i) {
            double eg = 0.0;
            for (int a = 0; a < d; ++a) eg += L.e[i][a] * grad[a * V + k];
            g[i] = L.w[i] * eg;
            dg[i] = L.dw[i] * eg;
        }
        for (int i = 0; i < q; ++i) {
            double df = L.dw[i] * theta0[k];
            for (int kk = 0; kk < q; ++kk) df -= dx * (dB[i][kk] * g[kk] + B[i][kk] * dg[kk]);
            ge += lam[i] * df;
        }
    }
    if (g_eps) *g_eps += ge;
    return 0;
}

/* Inverse Cole-Hopf transformation (Sec. II, u = -2 nu grad(theta)/theta):
 * theta0 = exp(-phi/(2 nu)) with grad(phi) = u0, phi = 0 at the origin.
 * phi at node c is the line integral along x_0 (at x_1 = .. = 0) from 0 to
 * c_0, then along x_1 (at x_2 = .. = 0) from 0 to c_1, and so on; each cell
 * [x_j, x_j+1] uses the integral of the cubic through the four nodes
 * j-1..j+2 (periodic):  dx (-u_{j-1} + 13 u_j + 13 u_{j+1} - u_{j+2}) / 24.
 * grad theta0 = -u0 theta0 / (2 nu).  u0 is d x V; grad may be NULL. */
int oracle_theta_from_velocity(int d, const int64_t* n, double dx, double nu, const double* u0,
                               double* theta0, double* grad) {
    or_grid G;
    if (make_grid(d, n, &G) != 0 || !(dx > 0) || !(nu > 0)) return -1;
    const int64_t V = G.V;
    for (int64_t k = 0; k < V; ++k) {
        int64_t c[OR_MAXD] = {0, 0, 0, 0}, rem = k;
        for (int a = 0; a < d; ++a) { c[a] = rem % G.n[a]; rem /= G.n[a]; }
        double phi = 0.0;
        for (int a = 0; a < d; ++a) {
            for (int64_t j = 0; j < c[a]; ++j) {
                double uu[4];
                for (int t = 0; t < 4; ++t) {
                    int64_t p[OR_MAXD] = {0, 0, 0, 0};
                    for (int b = 0; b < a; ++b) p[b] = c[b];
                    int64_t jj = (j - 1 + t) % G.n[a];
                    if (jj < 0) jj += G.n[a];
                    p[a] = jj;
                    int64_t idx = 0, stride = 1;
                    for (int b = 0; b < d; ++b) { idx += p[b] * stride; stride *= G.n[b]; }
                    uu[t] = u0[a * V + idx];
                }
                phi += dx * ((13.0 * (uu[1] + uu[2]) - (uu[0] + uu[3])) / 24.0);
            }
        }
        const double th = exp(-phi / (2.0 * nu));
        theta0[k] = th;
        if (grad)
            for (int a = 0; a < d; ++a) grad[a * V + k] = -u0[a * V + k] * th / (2.0 * nu);
    }
    return 0;
}
