// Device-side lattice definitions and the per-node MRT collision for the
// Cole-Hopf fourth-order MRT-LB scheme (arXiv:2309.02825, Sec. III).
//
// The collision is written in the natural-moment space of Sec. III.A without
// forming M or M^-1:
//   * moments kept: theta = sum f, j_a = sum e_a f, P_aa = sum e_a^2 f and
//     (d > 1) P_ab = sum e_a e_b f (a < b);
//   * post-collision moments (diagonal S, f^eq = w theta):
//       j'_a  = (1 - s1) j_a
//       P'_aa = P_aa - s21 (P_aa - theta/3)    (sum w e_a^2 = 1/3 under Theorem 2)
//       P'_ab = (1 - s22) P_ab
//       third- and fourth-order moments take their equilibrium values
//       (rate 1): sum e_a e_b^2 w theta = 0, sum e_a^2 e_b^2 w theta = 4 w_d theta =: R'
//   * f* = M^-1 m* in closed form.  Every natural-moment basis used here is a
//     set of monomials e_a^p e_b^q ..., so M^-1 factorises into the 1-D map
//     (mu0, mu1, mu2) -> (mu0 - mu2, (mu2 + mu1)/2, (mu2 - mu1)/2) per axis
//     (moments that involve three or more axes vanish on these lattices,
//     whose moving velocities have one or two non-zero components).  This gives
//       rest:        theta - sum_a P'_aa + R' * (number of axis pairs)
//       axis +-a:    (P'_aa +- j'_a)/2 - R' (d - 1)/2
//       edge (a,b):  (e_a e_b P'_ab + R')/4
//     for every d (the D1Q3, D2Q9, D3Q19 and D4Q33 lattices here).
// The same reconstruction, fed with eps-derivatives of the post-collision
// moments, gives (dC/deps) f; the transposed collision C^T is evaluated with
// the dual moments nu = M^-T mu (see collide_adjoint).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// Twin populations.  Theorem 2 relaxes the third-order moments
// sum e_a e_b^2 f and sum e_a^2 e_b f to their equilibrium 0 at rate 1, so
// after every collision the two edge populations of a pair (a, b) with
// opposite velocities are equal: f(-,-) = f(+,+) and f(+,-) = f(-,+) (the
// difference and the sum of those two moments give them).  The collisions
// below produce them as the same rounded value, so a state written by a
// collision holds only 1 + 2d + 2 d(d-1) independent populations per node
// (7 of 9 for D2Q9, 13 of 19 for D3Q19, 21 of 33 for D4Q33).  twin(i) is the
// population whose storage plane holds the value of i in such a state: the
// (+,+) or (-,+) edge of the pair for its (-,-) or (+,-) edge, i itself
// otherwise.
template <int D>
__host__ __device__ constexpr int twin(int i);

// Relaxation rates and weights of Theorem 2 plus the derived constants the
// kernels use.  Filled on the host (lbm_params.cpp).
struct Rates {
    double eps;
    double s1, s21, s22;     // relaxation rates
    double w0, w1, wd;       // weights of rest, axis and edge velocities
    double one_m_s1, one_m_s21, one_m_s22;
    double R4wd;             // 4 w_d (equilibrium of the c_a^2 c_b^2 moments per theta)
    double ucoef;            // (2 - s1) dx / dt
    double gcoef;            // -3 s1 / dx: grad theta = gcoef * sum_i e_i f_i (c_s^2 = c^2/3)
    double dx;               // node spacing
    double inv_s1_m1;        // 1/s1 - 1
    double inv12dx;          // 1 / (12 dx)
    // d/deps of the above
    double ds1, ds21, ds22, dw0, dw1, dwd;
    double dinv_s1;          // d(1/s1)/deps = 3
    double c;                // dx / dt
    // D2Q9 / D3Q19 collisions in folded form (collide_d2q9, collide_d3q19)
    double f_cj;             // (1 - s1) / 2
    double f_cp;             // (1 - s21) / 2
    double f_ct;             // s21 / 6 - 2 (d - 1) w_d
    double f_cq;             // (1 - s22) / 4
};

// Velocity tables in the order of Sec. III.A (a fourth component, zero
// below d = 4, keeps one shape for every lattice).  d = 4 follows the
// general DdQ(1+2d^2) rule: rest, +unit vectors, -unit vectors, then for
// every axis pair a < b (lexicographic) (e_a, e_b) = (+,+) (-,+) (-,-) (+,-).
template <int D> struct Lat;

template <> struct Lat<1> {
    static constexpr int Q = 3;
    static constexpr int NP = 0;  // axis pairs
    static constexpr int E[3][4] = {{0, 0, 0, 0}, {1, 0, 0, 0}, {-1, 0, 0, 0}};
};

template <> struct Lat<2> {
    static constexpr int Q = 9;
    static constexpr int NP = 1;
    static constexpr int E[9][4] = {{0, 0, 0, 0},  {1, 0, 0, 0},   {0, 1, 0, 0},
                                    {-1, 0, 0, 0}, {0, -1, 0, 0},  {1, 1, 0, 0},
                                    {-1, 1, 0, 0}, {-1, -1, 0, 0}, {1, -1, 0, 0}};
};

template <> struct Lat<3> {
    static constexpr int Q = 19;
    static constexpr int NP = 3;
    static constexpr int E[19][4] = {
        {0, 0, 0, 0},  {1, 0, 0, 0},   {0, 1, 0, 0},   {0, 0, 1, 0},  {-1, 0, 0, 0},
        {0, -1, 0, 0}, {0, 0, -1, 0},  {1, 1, 0, 0},   {-1, 1, 0, 0}, {-1, -1, 0, 0},
        {1, -1, 0, 0}, {1, 0, 1, 0},   {-1, 0, 1, 0},  {-1, 0, -1, 0}, {1, 0, -1, 0},
        {0, 1, 1, 0},  {0, -1, 1, 0},  {0, -1, -1, 0}, {0, 1, -1, 0}};
};

template <> struct Lat<4> {
    static constexpr int Q = 33;
    static constexpr int NP = 6;
    static constexpr int E[33][4] = {
        {0, 0, 0, 0},
        {1, 0, 0, 0},   {0, 1, 0, 0},   {0, 0, 1, 0},   {0, 0, 0, 1},
        {-1, 0, 0, 0},  {0, -1, 0, 0},  {0, 0, -1, 0},  {0, 0, 0, -1},
        {1, 1, 0, 0},   {-1, 1, 0, 0},  {-1, -1, 0, 0}, {1, -1, 0, 0},
        {1, 0, 1, 0},   {-1, 0, 1, 0},  {-1, 0, -1, 0}, {1, 0, -1, 0},
        {1, 0, 0, 1},   {-1, 0, 0, 1},  {-1, 0, 0, -1}, {1, 0, 0, -1},
        {0, 1, 1, 0},   {0, -1, 1, 0},  {0, -1, -1, 0}, {0, 1, -1, 0},
        {0, 1, 0, 1},   {0, -1, 0, 1},  {0, -1, 0, -1}, {0, 1, 0, -1},
        {0, 0, 1, 1},   {0, 0, -1, 1},  {0, 0, -1, -1}, {0, 0, 1, -1}};
};

// Edge populations come in groups of four per axis pair, (+,+) (-,+) (-,-)
// (+,-), after the rest and the 2d axis velocities.
template <int D>
__host__ __device__ constexpr int twin(int i) {
    return (i >= 1 + 2 * D && ((i - (1 + 2 * D)) & 3) >= 2) ? i - 2 : i;
}
template <int D>
__host__ __device__ constexpr bool twins_are_opposite() {
    for (int i = 0; i < Lat<D>::Q; ++i) {
        const int t = twin<D>(i);
        if (t == i) continue;
        for (int a = 0; a < 4; ++a)
            if (Lat<D>::E[i][a] != -Lat<D>::E[t][a]) return false;
        if ((Lat<D>::E[i][0] != 0) + (Lat<D>::E[i][1] != 0) + (Lat<D>::E[i][2] != 0) +
                (Lat<D>::E[i][3] != 0) != 2)
            return false;
    }
    return true;
}
static_assert(twins_are_opposite<2>() && twins_are_opposite<3>() && twins_are_opposite<4>(),
              "a twin is the opposite edge velocity of its pair");
// Number of distinct populations of a post-collision state.
template <int D>
__host__ __device__ constexpr int num_independent() {
    int n = 0;
    for (int i = 0; i < Lat<D>::Q; ++i) n += twin<D>(i) == i;
    return n;
}
static_assert(num_independent<2>() == 7 && num_independent<3>() == 13 &&
                  num_independent<4>() == 21 && num_independent<1>() == 3,
              "independent populations after a collision");

// Number of axis pairs as an array extent (at least 1).
template <int D> struct NPairs {
    static constexpr int value = D * (D - 1) / 2 > 0 ? D * (D - 1) / 2 : 1;
};

// Index of the axis pair (a, b), a < b, in lexicographic order.
template <int D>
__host__ __device__ constexpr int pair_index(int a, int b) {
    return a * (2 * D - a - 1) / 2 + (b - a - 1);
}

template <int D> __host__ __device__ constexpr int nnz(int i) {
    return (Lat<D>::E[i][0] != 0) + (Lat<D>::E[i][1] != 0) + (Lat<D>::E[i][2] != 0) +
           (Lat<D>::E[i][3] != 0);
}
template <int D> __host__ __device__ constexpr int first_axis(int i) {
    return Lat<D>::E[i][0] != 0 ? 0 : (Lat<D>::E[i][1] != 0 ? 1 : (Lat<D>::E[i][2] != 0 ? 2 : 3));
}
template <int D> __host__ __device__ constexpr int second_axis(int i) {
    const int a = first_axis<D>(i);
    return (a < 1 && Lat<D>::E[i][1] != 0) ? 1 : ((a < 2 && Lat<D>::E[i][2] != 0) ? 2 : 3);
}

// Signed add: acc + s*v for s in {-1, 0, 1} known at compile time.
#define LBM_SADD(acc, s, v) ((s) == 1 ? (acc) + (v) : ((s) == -1 ? (acc) - (v) : (acc)))

// Moments of a distribution held in registers.
template <int D> struct Moments {
    double theta;
    double j[D];
    double P[D];
    double Pab[NPairs<D>::value];
};

template <int D>
__device__ __forceinline__ void moments(const double (&f)[Lat<D>::Q], Moments<D>& m) {
    constexpr int Q = Lat<D>::Q;
    double th = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) th += f[i];
    m.theta = th;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        double j = 0.0, p = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int e = Lat<D>::E[i][a];
            j = LBM_SADD(j, e, f[i]);
            if (e != 0) p += f[i];
        }
        m.j[a] = j;
        m.P[a] = p;
    }
    if constexpr (D > 1) {
#pragma unroll
        for (int a = 0; a < D; ++a) {
#pragma unroll
            for (int b = a + 1; b < D; ++b) {
                double pab = 0.0;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const int s = Lat<D>::E[i][a] * Lat<D>::E[i][b];
                    pab = LBM_SADD(pab, s, f[i]);
                }
                m.Pab[pair_index<D>(a, b)] = pab;
            }
        }
    } else {
        m.Pab[0] = 0.0;
    }
}

// f = M^-1 m for the moment vector (theta, j, P, Pab, R) with all
// third-order moments zero and every c_a^2 c_b^2 moment equal to R.
template <int D>
__device__ __forceinline__ void reconstruct(double theta, const double (&j)[D], const double (&P)[D],
                                            const double (&Pab)[NPairs<D>::value], double R,
                                            double (&f)[Lat<D>::Q]) {
    constexpr int Q = Lat<D>::Q;
    constexpr int NP = Lat<D>::NP;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int k = nnz<D>(i);
        if (k == 0) {
            double sP = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) sP += P[a];
            f[i] = (theta - sP) + (NP == 0 ? 0.0 : (NP == 1 ? R : (double)NP * R));
        } else if (k == 1) {
            const int a = first_axis<D>(i);
            const int s = Lat<D>::E[i][a];
            const double h = 0.5 * (s == 1 ? P[a] + j[a] : P[a] - j[a]);
            f[i] = (D == 1) ? h : h - (0.5 * (D - 1)) * R;
        } else {
            const int a = first_axis<D>(i);
            const int b = second_axis<D>(i);
            const int s = Lat<D>::E[i][a] * Lat<D>::E[i][b];
            const double pab = Pab[pair_index<D>(a, b)];
            f[i] = 0.25 * (s == 1 ? R + pab : R - pab);
        }
    }
}

// D2Q9 collision with the algebra of collide<D> folded by hand (Sec. III.A,
// Theorem 2).  The six moments share the partial sums over the three
// velocities with e_x = +1 / -1 and e_y = +1 / -1; with
//     hj_a = (1 - s1)/2 j_a,   hP_a = (1 - s21)/2 P_a + (s21/6 - 2 w_d) theta
// the post-collision populations are hP_a +- hj_a on the axis velocities,
// eR +- (1 - s22)/4 P_xy on the diagonals (sign e_x e_y) with eR = w_d theta,
// and (theta - 4 eR) - 2 (hP_x + hP_y) at rest.  Writing the rest population
// with the same rounded eR that the diagonals carry keeps sum_i f_i = theta
// up to unbiased rounding; a separately rounded (1 - 4 w_d) would bias the
// mass at every step (about 1e-16 per step, 1e-12 after 10^4 steps).  The
// products by (1 - s1)/2 and (1 - s22)/4 are fused into the additions that
// form the populations (fma with the sign of e), so that each population
// pair costs two operations: 31 double operations against about 60 for the
// generic form.  The library is built without floating-point contraction, so
// the roundings are the ones written here, in every kernel that calls this.
struct FoldedRates {
    double cj, cp, ct, cq, wd;  // f_cj, f_cp, f_ct, f_cq and w_d of Rates
};
__host__ __device__ __forceinline__ FoldedRates folded(const Rates& r) {
    return FoldedRates{r.f_cj, r.f_cp, r.f_ct, r.f_cq, r.wd};
}

__device__ __forceinline__ void collide_d2q9(double (&f)[9], const FoldedRates& r) {
    const double xp = f[1] + f[5] + f[8], xm = f[3] + f[6] + f[7];
    const double yp = f[2] + f[5] + f[6], ym = f[4] + f[7] + f[8];
    const double jx = xp - xm, Px = xp + xm, jy = yp - ym, Py = yp + ym;
    const double th = f[0] + (f[2] + f[4]) + Px;
    const double Pxy = (f[5] + f[7]) - (f[6] + f[8]);
    const double tt = r.ct * th;
    const double hPx = fma(r.cp, Px, tt), hPy = fma(r.cp, Py, tt);
    const double eR = r.wd * th;
    f[0] = fma(-2.0, hPx + hPy, fma(-4.0, eR, th));
    f[1] = fma(r.cj, jx, hPx);
    f[3] = fma(-r.cj, jx, hPx);
    f[2] = fma(r.cj, jy, hPy);
    f[4] = fma(-r.cj, jy, hPy);
    f[5] = fma(r.cq, Pxy, eR);
    f[7] = f[5];
    f[6] = fma(-r.cq, Pxy, eR);
    f[8] = f[6];
}

// D3Q19 collision folded the same way: with hj_a = (1 - s1)/2 j_a and
// hP_a = (1 - s21)/2 P_a + (s21/6 - 4 w_d) theta the axis populations are
// hP_a +- hj_a, the edge populations of the pair (a, b) are
// eR +- (1 - s22)/4 P_ab (sign e_a e_b) with eR = w_d theta, and the rest
// population is (theta - 12 eR) - 2 (hP_x + hP_y + hP_z), which again keeps
// sum_i f_i = theta up to unbiased rounding.  With the products fused as in
// collide_d2q9, 69 double operations against about 140 for the generic form.
__device__ __forceinline__ void collide_d3q19(double (&f)[19], const FoldedRates& r) {
    // partial sums over the five velocities with e_a = +1 / -1
    const double xp = (f[1] + f[7]) + (f[10] + f[11]) + f[14];
    const double xm = (f[4] + f[8]) + (f[9] + f[12]) + f[13];
    const double yp = (f[2] + f[7]) + (f[8] + f[15]) + f[18];
    const double ym = (f[5] + f[9]) + (f[10] + f[16]) + f[17];
    const double zp = (f[3] + f[11]) + (f[12] + f[15]) + f[16];
    const double zm = (f[6] + f[13]) + (f[14] + f[17]) + f[18];
    const double jx = xp - xm, Px = xp + xm, jy = yp - ym, Py = yp + ym;
    const double jz = zp - zm, Pz = zp + zm;
    const double th =
        ((f[0] + Px) + (f[2] + f[5])) + ((f[3] + f[6]) + ((f[15] + f[16]) + (f[17] + f[18])));
    const double Pxy = (f[7] + f[9]) - (f[8] + f[10]);
    const double Pxz = (f[11] + f[13]) - (f[12] + f[14]);
    const double Pyz = (f[15] + f[17]) - (f[16] + f[18]);
    const double tt = r.ct * th;
    const double hPx = fma(r.cp, Px, tt), hPy = fma(r.cp, Py, tt), hPz = fma(r.cp, Pz, tt);
    const double eR = r.wd * th;
    f[0] = fma(-2.0, (hPx + hPy) + hPz, fma(-12.0, eR, th));
    f[1] = fma(r.cj, jx, hPx);
    f[4] = fma(-r.cj, jx, hPx);
    f[2] = fma(r.cj, jy, hPy);
    f[5] = fma(-r.cj, jy, hPy);
    f[3] = fma(r.cj, jz, hPz);
    f[6] = fma(-r.cj, jz, hPz);
    f[7] = fma(r.cq, Pxy, eR);
    f[9] = f[7];
    f[8] = fma(-r.cq, Pxy, eR);
    f[10] = f[8];
    f[11] = fma(r.cq, Pxz, eR);
    f[13] = f[11];
    f[12] = fma(-r.cq, Pxz, eR);
    f[14] = f[12];
    f[15] = fma(r.cq, Pyz, eR);
    f[17] = f[15];
    f[16] = fma(-r.cq, Pyz, eR);
    f[18] = f[16];
}

// In-place collision f <- C f (Sec. III.A evolution equation, Theorem 2 rates).
template <int D>
__device__ __forceinline__ void collide(double (&f)[Lat<D>::Q], const Rates& r) {
    if constexpr (D == 2) {
        collide_d2q9(f, folded(r));
        return;
    }
    if constexpr (D == 3) {
        collide_d3q19(f, folded(r));
        return;
    }
    Moments<D> m;
    moments<D>(f, m);
    const double th3 = m.theta * (1.0 / 3.0);
    double j[D], P[D], Pab[NPairs<D>::value];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        j[a] = r.one_m_s1 * m.j[a];
        P[a] = m.P[a] - r.s21 * (m.P[a] - th3);
    }
#pragma unroll
    for (int p = 0; p < NPairs<D>::value; ++p) Pab[p] = r.one_m_s22 * m.Pab[p];
    reconstruct<D>(m.theta, j, P, Pab, r.R4wd * m.theta, f);
}

// df = (dC/deps) f at fixed f.
template <int D>
__device__ __forceinline__ void collide_deps(const double (&f)[Lat<D>::Q], const Rates& r,
                                             double (&df)[Lat<D>::Q]) {
    Moments<D> m;
    moments<D>(f, m);
    const double th3 = m.theta * (1.0 / 3.0);
    double j[D], P[D], Pab[NPairs<D>::value];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        j[a] = -r.ds1 * m.j[a];
        P[a] = -r.ds21 * (m.P[a] - th3);
    }
#pragma unroll
    for (int p = 0; p < NPairs<D>::value; ++p) Pab[p] = -r.ds22 * m.Pab[p];
    reconstruct<D>(0.0, j, P, Pab, 4.0 * r.dwd * m.theta, df);
}

// <mu, (dC/deps) f> for D2Q9 through the dual moments nu = M^-T mu (those
// of collide_adjoint below): (dC/deps) f = M^-1 m' with m' holding
// -ds1 j_a, -ds21 (P_a - theta/3), -ds22 P_xy and 4 dw_d theta on the
// c_x^2 c_y^2 row (zero elsewhere), so the product is sum over rows of
// nu_row m'_row.  Equal to sum_i mu_i df_i of collide_deps up to rounding.
// Dual moments nu = M^-T mu of a D2Q9 mu (those of collide_adjoint below),
// shared by the eps part and the folded adjoint collision.  The products by
// 1/2 and 1/4 are exact, so the fused forms round as the plain ones would.
struct Dual2 {
    double rest, nax, nay, naax, naay, nab, naabb;
};
__device__ __forceinline__ Dual2 dual_d2q9(const double (&mu)[9]) {
    const double sx = mu[1] + mu[3], sy = mu[2] + mu[4];
    const double se = mu[5] + mu[7], sd = mu[6] + mu[8];
    Dual2 d;
    d.rest = mu[0];
    d.nax = 0.5 * (mu[1] - mu[3]);
    d.nay = 0.5 * (mu[2] - mu[4]);
    d.naax = fma(0.5, sx, -mu[0]);
    d.naay = fma(0.5, sy, -mu[0]);
    d.nab = 0.25 * (se - sd);
    d.naabb = fma(0.25, se + sd, fma(-0.5, sx + sy, mu[0]));
    return d;
}

__device__ __forceinline__ double eps_part_d2q9(const Dual2& d, const double (&f)[9],
                                                const Rates& r) {
    const double xp = f[1] + f[5] + f[8], xm = f[3] + f[6] + f[7];
    const double yp = f[2] + f[5] + f[6], ym = f[4] + f[7] + f[8];
    const double jx = xp - xm, Px = xp + xm, jy = yp - ym, Py = yp + ym;
    const double th = f[0] + (f[2] + f[4]) + Px;
    const double Pxy = (f[5] + f[7]) - (f[6] + f[8]);
    const double th3 = th * (1.0 / 3.0);
    return (-r.ds1) * (d.nax * jx + d.nay * jy) +
           (-r.ds21) * (d.naax * (Px - th3) + d.naay * (Py - th3)) + (-r.ds22) * (d.nab * Pxy) +
           (4.0 * r.dwd) * (d.naabb * th);
}

// lam = C^T mu for D2Q9 from the dual moments, with the algebra of
// collide_adjoint below folded: with t_a = (1 - s1) nu_a, tt_a =
// (1 - s21) nu_aa and n0 = nu_0 + (s21/3)(nu_xx + nu_yy) + 4 w_d nu_xxyy,
// lam_rest = n0, lam_{+-a} = (n0 + tt_a) +- t_a and the four edges are
// (c +- (1 - s22) nu_xy) +- (t_x +- t_y) with c = n0 + tt_x + tt_y
// (signs e_x e_y, e_x and e_y).  24 operations against about 60.
__device__ __forceinline__ void collide_adjoint_d2q9(const Dual2& d, const Rates& r,
                                                     double (&lam)[9]) {
    const double ttx = r.one_m_s21 * d.naax, tty = r.one_m_s21 * d.naay;
    const double n0 = fma(r.R4wd, d.naabb, fma(r.s21 * (1.0 / 3.0), d.naax + d.naay, d.rest));
    const double bx = n0 + ttx, by = n0 + tty;
    const double tx = r.one_m_s1 * d.nax, ty = r.one_m_s1 * d.nay;
    const double c = bx + tty;
    const double cp = fma(r.one_m_s22, d.nab, c), cm = fma(-r.one_m_s22, d.nab, c);
    const double p = tx + ty, m = tx - ty;
    lam[0] = n0;
    lam[1] = bx + tx;
    lam[3] = bx - tx;
    lam[2] = by + ty;
    lam[4] = by - ty;
    lam[5] = cp + p;
    lam[7] = cp - p;
    lam[6] = cm - m;
    lam[8] = cm + m;
}

// lam = C^T mu.  With C = M^-1 C_m M and C_m = I - S + S (M w) e_0^T,
// C^T mu = M^T C_m^T nu with the dual moments nu = M^-T mu:
//   nu_0   = mu_rest
//   nu_a   = (mu_{+a} - mu_{-a})/2
//   nu_aa  = -mu_rest + (mu_{+a} + mu_{-a})/2
//   nu_ab  = sum_{edges in plane ab} e_a e_b mu / 4
//   nu_aabb= mu_rest - (mu_{+a} + mu_{-a} + mu_{+b} + mu_{-b})/2 + sum_{edges ab} mu / 4
// C_m^T nu keeps (1-s1) nu_a, (1-s21) nu_aa, (1-s22) nu_ab, zeroes the
// rate-1 rows and collects nu_0 + (s21/3) sum nu_aa + 4 w_d sum nu_aabb in
// row 0; M^T maps back to populations.
template <int D>
__device__ __forceinline__ void collide_adjoint(const double (&mu)[Lat<D>::Q], const Rates& r,
                                                double (&lam)[Lat<D>::Q]) {
    if constexpr (D == 2) {
        collide_adjoint_d2q9(dual_d2q9(mu), r, lam);
        return;
    }
    constexpr int Q = Lat<D>::Q;
    double na[D], naa[D], nab[NPairs<D>::value], naabb[NPairs<D>::value];
    const double rest = mu[0];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        double dp = 0.0, sp = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            if (nnz<D>(i) == 1 && first_axis<D>(i) == a) {
                dp = LBM_SADD(dp, Lat<D>::E[i][a], mu[i]);
                sp += mu[i];
            }
        }
        na[a] = 0.5 * dp;
        naa[a] = 0.5 * sp - rest;
    }
    if constexpr (D > 1) {
#pragma unroll
        for (int a = 0; a < D; ++a) {
#pragma unroll
            for (int b = a + 1; b < D; ++b) {
                double se = 0.0, ss = 0.0;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    if (nnz<D>(i) == 2 && Lat<D>::E[i][a] != 0 && Lat<D>::E[i][b] != 0) {
                        ss = LBM_SADD(ss, Lat<D>::E[i][a] * Lat<D>::E[i][b], mu[i]);
                        se += mu[i];
                    }
                }
                const int p = pair_index<D>(a, b);
                nab[p] = 0.25 * ss;
                // mu_{+a} + mu_{-a} = 2 (naa + rest)
                naabb[p] = rest - (naa[a] + rest) - (naa[b] + rest) + 0.25 * se;
            }
        }
    }
    double n0 = rest;
    double snaa = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) snaa += naa[a];
    n0 += r.s21 * (1.0 / 3.0) * snaa;
    if constexpr (D > 1) {
        double sb = 0.0;
#pragma unroll
        for (int p = 0; p < Lat<D>::NP; ++p) sb += naabb[p];
        n0 += r.R4wd * sb;
    }
    double ta[D], taa[D], tab[NPairs<D>::value];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        ta[a] = r.one_m_s1 * na[a];
        taa[a] = r.one_m_s21 * naa[a];
    }
    if constexpr (D > 1) {
#pragma unroll
        for (int p = 0; p < Lat<D>::NP; ++p) tab[p] = r.one_m_s22 * nab[p];
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int k = nnz<D>(i);
        if (k == 0) {
            lam[i] = n0;
        } else if (k == 1) {
            const int a = first_axis<D>(i);
            const double t = Lat<D>::E[i][a] == 1 ? ta[a] : -ta[a];
            lam[i] = n0 + t + taa[a];
        } else {
            const int a = first_axis<D>(i);
            const int b = second_axis<D>(i);
            const double t1 = Lat<D>::E[i][a] == 1 ? ta[a] : -ta[a];
            const double t2 = Lat<D>::E[i][b] == 1 ? ta[b] : -ta[b];
            const double tp = (Lat<D>::E[i][a] * Lat<D>::E[i][b] == 1) ? tab[pair_index<D>(a, b)]
                                                                       : -tab[pair_index<D>(a, b)];
            lam[i] = n0 + t1 + t2 + taa[a] + taa[b] + tp;
        }
    }
}

// Weight of population i.
template <int D>
__device__ __forceinline__ double weight(int i, const Rates& r) {
    const int k = nnz<D>(i);
    return k == 0 ? r.w0 : (k == 1 ? r.w1 : r.wd);
}
template <int D>
__device__ __forceinline__ double dweight(int i, const Rates& r) {
    const int k = nnz<D>(i);
    return k == 0 ? r.dw0 : (k == 1 ? r.dw1 : r.dwd);
}

}  // namespace lbm
