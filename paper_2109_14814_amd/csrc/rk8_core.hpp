// rk8_core.hpp -- pieces shared by the stroboscopic map (rk8.hip) and the
// refinement kernels (refine.hip): the Cooper-Verner order-8 tableau, the
// per-step stage tables of the time-dependent factor w(f) = 1 / (1 + e cos f),
// and the vector fields of the planar elliptic restricted three-body problem:
// pulsating rotating coordinates with the true anomaly as time, and the
// position-momentum form with time t of Sec. 3.3.
#pragma once

#include "ms_internal.hpp"

namespace ms {

constexpr int RK_S = 11;
constexpr double RK_TWO_PI = 6.283185307179586476925286766559;

struct Tableau {
    double a[RK_S][RK_S];
    double b[RK_S];
    double c[RK_S];
};

// Non-zero pattern of the Cooper-Verner tableau (zero terms are dropped at
// compile time; the values themselves come from cv_tableau and are checked
// against this pattern on the host).
constexpr bool RK_NZ[RK_S][RK_S] = {
    {0}, {1}, {1, 1}, {1, 1, 1}, {1, 0, 1, 1}, {1, 0, 1, 1, 1}, {1, 0, 1, 1, 1, 1},
    {1, 0, 0, 0, 1, 1, 1}, {1, 0, 0, 0, 1, 1, 1, 1}, {1, 0, 0, 0, 1, 1, 1, 1, 1}, {0, 0, 0, 0, 1, 1, 1, 1, 1, 1}};
constexpr bool RK_NZB[RK_S] = {1, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1};

// Cooper & Verner (1972), SIAM J. Numer. Anal. 9, the order-8 method with 11
// stages.  Its coefficients lie in Q(sqrt 21); they are formed at compile
// time from RK_SQRT21, the double nearest to sqrt(21) (the host checks that
// sqrt(21.0) rounds to it), each operation rounded once as written.
constexpr double RK_SQRT21 = 4.5825756949558400065880471937280084889844565767679719026072421239;

constexpr Tableau cv_make_tableau()
{
    Tableau T{};
    const double q = RK_SQRT21;
    double (*a)[RK_S] = T.a;
    a[1][0] = 0.5;
    a[2][0] = 0.25; a[2][1] = 0.25;
    a[3][0] = 1.0 / 7.0; a[3][1] = -(7.0 + 3.0 * q) / 98.0; a[3][2] = (21.0 + 5.0 * q) / 49.0;
    a[4][0] = (11.0 + q) / 84.0; a[4][2] = (18.0 + 4.0 * q) / 63.0; a[4][3] = (21.0 - q) / 252.0;
    a[5][0] = (5.0 + q) / 48.0; a[5][2] = (9.0 + q) / 36.0; a[5][3] = (14.0 * q - 231.0) / 360.0; a[5][4] = (63.0 - 7.0 * q) / 80.0;
    a[6][0] = (10.0 - q) / 42.0; a[6][2] = (92.0 * q - 432.0) / 315.0; a[6][3] = (633.0 - 145.0 * q) / 90.0;
    a[6][4] = (115.0 * q - 504.0) / 70.0; a[6][5] = (63.0 - 13.0 * q) / 35.0;
    a[7][0] = 1.0 / 14.0; a[7][4] = (14.0 - 3.0 * q) / 126.0; a[7][5] = (13.0 - 3.0 * q) / 63.0; a[7][6] = 1.0 / 9.0;
    a[8][0] = 1.0 / 32.0; a[8][4] = (91.0 - 21.0 * q) / 576.0; a[8][5] = 11.0 / 72.0;
    a[8][6] = -(385.0 + 75.0 * q) / 1152.0; a[8][7] = (63.0 + 13.0 * q) / 128.0;
    a[9][0] = 1.0 / 14.0; a[9][4] = 1.0 / 9.0; a[9][5] = -(733.0 + 147.0 * q) / 2205.0;
    a[9][6] = (515.0 + 111.0 * q) / 504.0; a[9][7] = -(51.0 + 11.0 * q) / 56.0; a[9][8] = (132.0 + 28.0 * q) / 245.0;
    a[10][4] = (7.0 * q - 42.0) / 18.0; a[10][5] = (28.0 * q - 18.0) / 45.0; a[10][6] = -(273.0 + 53.0 * q) / 72.0;
    a[10][7] = (301.0 + 53.0 * q) / 72.0; a[10][8] = (28.0 - 28.0 * q) / 45.0; a[10][9] = (49.0 - 7.0 * q) / 18.0;
    const double b[RK_S] = {1.0 / 20.0, 0, 0, 0, 0, 0, 0, 49.0 / 180.0, 16.0 / 45.0, 49.0 / 180.0, 1.0 / 20.0};
    const double c[RK_S] = {0.0, 0.5, 0.5, (7.0 + q) / 14.0, (7.0 + q) / 14.0, 0.5, (7.0 - q) / 14.0,
                            (7.0 - q) / 14.0, 0.5, (7.0 + q) / 14.0, 1.0};
    for (int i = 0; i < RK_S; ++i) {
        T.b[i] = b[i];
        T.c[i] = c[i];
    }
    return T;
}

// Host: the tableau; whether sqrt(21.0) rounds to RK_SQRT21 and the zeros
// match RK_NZ.
const Tableau &cv_tableau();
bool cv_pattern_ok();

// Stage values of the time-dependent coefficients, at the abscissa
// f = (n + c_i) h of stage i of step n of one period (h = 2 pi / steps):
//   w(f) = 1 / (1 + e cos f) (pulsating coordinates) and dw/de = -cos f w^2;
//   the separation of the primaries rho = 1 - e cos E(t) and the rate of
//   their true anomaly n(t) = sqrt(1 - e^2) / rho^2 at the time t = f, E the
//   eccentric anomaly (E - e sin E = t, periapse at t = 0).
// All are 2 pi periodic and even in the abscissa, so one period's values
// serve every period and both directions of integration.  The kernels
// compute them on the GPU: the maps a chunk of RK_CHUNK steps at a time
// into LDS, the refinement once per call into its workspace.  Nothing is
// allocated or copied from the host, so every call can be captured.
constexpr int RK_CHUNK = 32;

MS_D double stage_abscissa(int64_t n, double c, int steps)
{
    const double h = RK_TWO_PI / (double)steps;
    return (double)n * h + c * h;
}

// Root of Kepler's equation E - e sin E = M for the primaries' orbit
// (Sec. 3.3, mean anomaly M = t).  E - M is 2 pi periodic in M and lies in
// [-e, e]; Newton's method from E = M + e sin M, kept inside that bracket (a
// step that leaves it is replaced by bisection), converges for every
// 0 <= e < 1.
MS_D double eccentric_anomaly(double M, double e)
{
    const double k = floor(M / RK_TWO_PI + 0.5);
    const double Mr = M - k * RK_TWO_PI;
    double lo = Mr - e, hi = Mr + e;
    double E = Mr + e * sin(Mr);
    if (!(E >= lo && E <= hi)) E = Mr;
    for (int it = 0; it < 100 && e > 0.0; ++it) {
        double sE, cE;
        sincos(E, &sE, &cE);
        const double g = E - e * sE - Mr;
        if (g == 0.0) break;
        if (g < 0.0) lo = E; else hi = E;
        double En = E - g / (1.0 - e * cE);
        if (!(En > lo && En < hi)) En = 0.5 * (lo + hi);
        const bool done = fabs(En - E) <= 2e-16 * (1.0 + fabs(E));
        E = En;
        if (done) break;
    }
    return E + k * RK_TWO_PI;
}

// (rho, n) at time t for eccentricity e.
MS_D double2 kepler_rho_n(double t, double e)
{
    const double rho = 1.0 - e * cos(eccentric_anomaly(t, e));
    return make_double2(rho, sqrt(1.0 - e * e) / (rho * rho));
}

// The block's threads fill the stage values of steps n0 .. n0 + cnt - 1
// (taken mod steps) into s_val[j * RK_S + i]; c_dev: the RK_S abscissae c_i.
template <typename T, typename F>
MS_D void fill_stage_chunk(T *s_val, const double *c_dev, int64_t n0, int cnt, int steps, F &&value)
{
    for (int i = threadIdx.x; i < cnt * RK_S; i += blockDim.x) {
        const int j = i / RK_S, q = i - j * RK_S;
        s_val[i] = value(stage_abscissa((n0 + j) % steps, c_dev[q], steps));
    }
}

struct Model {
    double mu, one_minus_mu;
};

// x^(-1/2) for x = r^2 > 0: the hardware reciprocal square root (about 23
// correct bits) refined by two Newton steps y <- y (3/2 - x y^2 / 2), each of
// which doubles the number of correct bits; the result is within a few ulp
// of the correctly rounded value, for about half the instructions of a
// square root followed by a division.  The force terms m / r^3 = m y^3 and
// the Hessian terms 3 m / r^5 = 3 m y^5 all come from this one value.
MS_D double inv_sqrt(double x)
{
#pragma clang fp contract(fast)
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = fma(y, fma(-h, y * y, 0.5), y);
    y = fma(y, fma(-h, y * y, 0.5), y);
    return y;
}

// Right-hand side at stage weight w: (x', y', w Omega_x + 2 y', w Omega_y - 2 x'),
// Omega = (x^2 + y^2)/2 + (1 - mu)/r1 + mu/r2, r1 = |(x + mu, y)|,
// r2 = |(x - 1 + mu, y)|.
MS_D void rk_field(const Model &md, double w, const double y[4], double k[4])
{
#pragma clang fp contract(fast)
    double x = y[0], yy = y[1];
    double dx1 = x + md.mu, dx2 = x - md.one_minus_mu;
    double yy2 = yy * yy;
    double r1s = dx1 * dx1 + yy2, r2s = dx2 * dx2 + yy2;
    double i1 = inv_sqrt(r1s), i2 = inv_sqrt(r2s);
    double g1 = md.one_minus_mu * (i1 * i1) * i1, g2 = md.mu * (i2 * i2) * i2;   // m_i / r_i^3
    double Ox = x - g1 * dx1 - g2 * dx2;
    double Oy = yy - (g1 + g2) * yy;
    k[0] = y[2];
    k[1] = y[3];
    k[2] = 2.0 * y[3] + w * Ox;
    k[3] = -2.0 * y[2] + w * Oy;
}

// Position-momentum model (Sec. 3.3) at a stage with separation rho and
// frame rate n: z' = J grad H for
//   H = (px^2 + py^2)/2 + n (px y - py x) - (1 - mu)/r1 - mu/r2,
//   r1 = |(x + mu rho, y)|, r2 = |(x - (1 - mu) rho, y)|.
MS_D void pm_field(const Model &md, double rho, double n, const double z[4], double k[4])
{
#pragma clang fp contract(fast)
    double x = z[0], y = z[1];
    double d1 = x + md.mu * rho, d2 = x - md.one_minus_mu * rho;
    double y2 = y * y;
    double r1s = d1 * d1 + y2, r2s = d2 * d2 + y2;
    double i1 = inv_sqrt(r1s), i2 = inv_sqrt(r2s);
    double a1 = md.one_minus_mu * (i1 * i1) * i1, a2 = md.mu * (i2 * i2) * i2;   // m_i / r_i^3
    k[0] = z[2] + n * y;
    k[1] = z[3] - n * x;
    k[2] = n * z[3] - a1 * d1 - a2 * d2;
    k[3] = -n * z[2] - (a1 + a2) * y;
}

// The same field with NC tangent columns v: v' = J Hess(H) v.
template <int NC>
MS_D void pm_field_var(const Model &md, double rho, double n, const double z[4], const double v[NC][4],
                       double k[4], double kv[NC][4])
{
#pragma clang fp contract(fast)
    double x = z[0], y = z[1];
    double d1 = x + md.mu * rho, d2 = x - md.one_minus_mu * rho;
    double y2 = y * y;
    double r1s = d1 * d1 + y2, r2s = d2 * d2 + y2;
    double i1 = inv_sqrt(r1s), i2 = inv_sqrt(r2s);
    double q1 = i1 * i1, q2 = i2 * i2;                                     // 1 / r_i^2
    double a1 = md.one_minus_mu * q1 * i1, a2 = md.mu * q2 * i2;          // m_i / r_i^3
    double b1 = 3.0 * a1 * q1, b2 = 3.0 * a2 * q2;                         // 3 m_i / r_i^5
    double hxx = a1 + a2 - b1 * d1 * d1 - b2 * d2 * d2;
    double hyy = a1 + a2 - (b1 + b2) * y2;
    double hxy = -(b1 * d1 + b2 * d2) * y;
    k[0] = z[2] + n * y;
    k[1] = z[3] - n * x;
    k[2] = n * z[3] - a1 * d1 - a2 * d2;
    k[3] = -n * z[2] - (a1 + a2) * y;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        kv[c][0] = v[c][2] + n * v[c][1];
        kv[c][1] = v[c][3] - n * v[c][0];
        kv[c][2] = n * v[c][3] - hxx * v[c][0] - hxy * v[c][1];
        kv[c][3] = -n * v[c][2] - hxy * v[c][0] - hyy * v[c][1];
    }
}

// Gradient and Hessian of Omega at (x, y).
struct OmegaD {
    double Ox, Oy, Oxx, Oxy, Oyy;
};

MS_D OmegaD omega_derivs(const Model &md, double x, double yy)
{
#pragma clang fp contract(fast)
    double dx1 = x + md.mu, dx2 = x - md.one_minus_mu;
    double yy2 = yy * yy;
    double r1s = dx1 * dx1 + yy2, r2s = dx2 * dx2 + yy2;
    double i1 = inv_sqrt(r1s), i2 = inv_sqrt(r2s);
    double q1 = i1 * i1, q2 = i2 * i2;                                    // 1 / r_i^2
    double g1 = md.one_minus_mu * q1 * i1, g2 = md.mu * q2 * i2;         // (1-mu)/r1^3, mu/r2^3
    double h1 = 3.0 * g1 * q1, h2 = 3.0 * g2 * q2;                        // 3(1-mu)/r1^5, 3 mu/r2^5
    OmegaD o;
    o.Ox = x - g1 * dx1 - g2 * dx2;
    o.Oy = yy - (g1 + g2) * yy;
    o.Oxx = 1.0 - g1 - g2 + h1 * dx1 * dx1 + h2 * dx2 * dx2;
    o.Oyy = 1.0 - g1 - g2 + (h1 + h2) * yy2;
    o.Oxy = (h1 * dx1 + h2 * dx2) * yy;
    return o;
}

}  // namespace ms
