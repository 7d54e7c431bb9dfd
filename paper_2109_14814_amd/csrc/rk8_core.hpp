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

// Host: the tableau in double precision; whether its zeros match RK_NZ.
const Tableau &cv_tableau();
bool cv_pattern_ok();

// Host: device table of one period of stage values, steps x RK_S doubles,
// entry (n, i) at the abscissa f = (n + c_i) h, h = 2 pi / steps.
//   STAGE_W     w(f) = 1 / (1 + e cos f)
//   STAGE_DWDE  dw/de = -cos f w(f)^2
//   STAGE_RHO_N two doubles per entry at the time t = (n + c_i) h: the
//               separation of the primaries rho = 1 - e cos E(t) and the
//               rate of their true anomaly n(t) = sqrt(1 - e^2) / rho^2, E the
//               eccentric anomaly (E - e sin E = t, periapse at t = 0).
// All are 2 pi periodic and even in the abscissa, so one table serves every
// period and both directions of integration.  Cached per (device, e, steps,
// kind) for the life of the process.
enum { STAGE_W = 0, STAGE_DWDE = 1, STAGE_RHO_N = 2 };
int stage_table(double e, int steps, int kind, double **out);

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
