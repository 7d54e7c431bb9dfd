// rk8_core.hpp -- pieces shared by the stroboscopic map (rk8.hip) and the
// refinement kernels (refine.hip): the Cooper-Verner order-8 tableau, the
// per-step stage tables of the time-dependent factor w(f) = 1 / (1 + e cos f),
// and the vector field of the planar elliptic restricted three-body problem in
// pulsating rotating coordinates (the model family of Sec. 3.2-3.3).
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
//   STAGE_W    w(f) = 1 / (1 + e cos f)
//   STAGE_DWDE dw/de = -cos f w(f)^2
// w is 2 pi periodic and even in f, so one table serves every period and
// both directions of integration.  Cached per (device, e, steps, kind) for
// the life of the process.
enum { STAGE_W = 0, STAGE_DWDE = 1 };
int stage_table(double e, int steps, int kind, double **out);

struct Model {
    double mu, one_minus_mu;
};

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
    double r1 = sqrt(r1s), r2 = sqrt(r2s);
    double g1 = md.one_minus_mu / (r1s * r1), g2 = md.mu / (r2s * r2);
    double Ox = x - g1 * dx1 - g2 * dx2;
    double Oy = yy - (g1 + g2) * yy;
    k[0] = y[2];
    k[1] = y[3];
    k[2] = 2.0 * y[3] + w * Ox;
    k[3] = -2.0 * y[2] + w * Oy;
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
    double r1 = sqrt(r1s), r2 = sqrt(r2s);
    double g1 = md.one_minus_mu / (r1s * r1), g2 = md.mu / (r2s * r2);   // (1-mu)/r1^3, mu/r2^3
    double h1 = 3.0 * g1 / r1s, h2 = 3.0 * g2 / r2s;                      // 3(1-mu)/r1^5, 3 mu/r2^5
    OmegaD o;
    o.Ox = x - g1 * dx1 - g2 * dx2;
    o.Oy = yy - (g1 + g2) * yy;
    o.Oxx = 1.0 - g1 - g2 + h1 * dx1 * dx1 + h2 * dx2 * dx2;
    o.Oyy = 1.0 - g1 - g2 + (h1 + h2) * yy2;
    o.Oxy = (h1 * dx1 + h2 * dx2) * yy;
    return o;
}

}  // namespace ms
