// rk8.hip -- stroboscopic map of the planar elliptic restricted three-body
// problem (pulsating rotating coordinates, true anomaly as time), fixed-step
// explicit Runge-Kutta of order 8 (Cooper & Verner 1972, 11 stages).
//
// One thread per state; the tableau is a kernel argument (scalar loads) and
// the stage weights w(f) = 1 / (1 + e cos f) are tabulated per step of one
// period on the host (w is 2 pi periodic and even, so the same table serves
// every period and both directions), read with uniform loads.
#include <math.h>
#include <string.h>

#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "rk8_core.hpp"

namespace ms {

namespace {

constexpr int S = RK_S;
constexpr int RK_BLOCK = 128;

// Cooper & Verner (1972), SIAM J. Numer. Anal. 9, order-8 method with 11
// stages; coefficients in Q(sqrt 21), evaluated once in double precision.
Tableau make_tableau()
{
    Tableau T;
    memset(&T, 0, sizeof T);
    const double q = sqrt(21.0);
    double (*a)[S] = T.a;
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
    const double b[S] = {1.0 / 20.0, 0, 0, 0, 0, 0, 0, 49.0 / 180.0, 16.0 / 45.0, 49.0 / 180.0, 1.0 / 20.0};
    const double c[S] = {0.0, 0.5, 0.5, (7.0 + q) / 14.0, (7.0 + q) / 14.0, 0.5, (7.0 - q) / 14.0, (7.0 - q) / 14.0,
                         0.5, (7.0 + q) / 14.0, 1.0};
    memcpy(T.b, b, sizeof b);
    memcpy(T.c, c, sizeof c);
    return T;
}

// Root of Kepler's equation E - e sin E = M for the primaries' orbit
// (Sec. 3.3, mean anomaly M = t).  E - M is 2 pi periodic in M and lies in
// [-e, e]; Newton's method from E = M + e sin M, kept inside that bracket
// (a step that leaves it is replaced by bisection), converges for every
// 0 <= e < 1.
double eccentric_anomaly(double M, double e)
{
    const double k = floor(M / RK_TWO_PI + 0.5);
    const double Mr = M - k * RK_TWO_PI;
    double lo = Mr - e, hi = Mr + e;
    double E = Mr + e * sin(Mr);
    if (!(E >= lo && E <= hi)) E = Mr;
    for (int it = 0; it < 100 && e > 0.0; ++it) {
        const double g = E - e * sin(E) - Mr;
        if (g == 0.0) break;
        if (g < 0.0) lo = E; else hi = E;
        double En = E - g / (1.0 - e * cos(E));
        if (!(En > lo && En < hi)) En = 0.5 * (lo + hi);
        const bool done = fabs(En - E) <= 2e-16 * (1.0 + fabs(E));
        E = En;
        if (done) break;
    }
    return E + k * RK_TWO_PI;
}

// Stage tables per (device, e, steps per period, kind), kept for the life of
// the process.
std::mutex g_tab_mu;
std::map<std::tuple<int, uint64_t, int, int>, double *> g_tabs;

}  // namespace

const Tableau &cv_tableau()
{
    static const Tableau T = make_tableau();
    return T;
}

bool cv_pattern_ok()
{
    const Tableau &T = cv_tableau();
    for (int i = 0; i < S; ++i) {
        for (int j = 0; j < S; ++j)
            if ((T.a[i][j] != 0.0) != (j < i && RK_NZ[i][j])) return false;
        if ((T.b[i] != 0.0) != RK_NZB[i]) return false;
    }
    return true;
}

int stage_table(double e, int steps, int kind, double **out)
{
    int dev = 0;
    MS_HIP(hipGetDevice(&dev));
    uint64_t eb;
    memcpy(&eb, &e, 8);
    std::lock_guard<std::mutex> lk(g_tab_mu);
    auto key = std::make_tuple(dev, eb, steps, kind);
    auto it = g_tabs.find(key);
    if (it != g_tabs.end()) { *out = it->second; return MS_OK; }
    const Tableau &T = cv_tableau();
    const double h = RK_TWO_PI / (double)steps;
    const int per = kind == STAGE_RHO_N ? 2 : 1;
    std::vector<double> w((size_t)steps * S * per);
    for (int n = 0; n < steps; ++n)
        for (int i = 0; i < S; ++i) {
            const double a = (double)n * h + T.c[i] * h;
            const size_t at = ((size_t)n * S + i) * per;
            if (kind == STAGE_RHO_N) {
                double rho = 1.0 - e * cos(eccentric_anomaly(a, e));
                w[at] = rho;
                w[at + 1] = sqrt(1.0 - e * e) / (rho * rho);
            } else {
                double cf = cos(a);
                double om = 1.0 / (1.0 + e * cf);
                w[at] = kind == STAGE_W ? om : -cf * om * om;
            }
        }
    double *d = nullptr;
    MS_HIP(hipMalloc(&d, w.size() * sizeof(double)));
    hipError_t er = hipMemcpy(d, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice);
    if (er != hipSuccess) { (void)hipFree(d); return hip_fail(er, "copy stage table"); }
    g_tabs[key] = d;
    *out = d;
    return MS_OK;
}

namespace {

__global__ void __launch_bounds__(RK_BLOCK) k_rk8_map(const double *__restrict__ in, double *__restrict__ out,
                                                      int64_t n, Model md, Tableau T, const double *__restrict__ wtab,
                                                      int steps, int64_t nsteps, double h)
{
#pragma clang fp contract(fast)
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    d4 s = load_d4(in + 4 * v);
    double y[4] = {s.x, s.y, s.z, s.w};
    int n_in = 0;
    for (int64_t st = 0; st < nsteps; ++st) {
        const double *w = wtab + (size_t)n_in * S;
        double k[S][4];
#pragma unroll
        for (int i = 0; i < S; ++i) {
            double ys[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double acc = 0.0;
#pragma unroll
                for (int j = 0; j < i; ++j)
                    if (RK_NZ[i][j]) acc += T.a[i][j] * k[j][c];
                ys[c] = y[c] + h * acc;
            }
            rk_field(md, w[i], ys, k[i]);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < S; ++i)
                if (RK_NZB[i]) acc += T.b[i] * k[i][c];
            y[c] = y[c] + h * acc;
        }
        if (++n_in == steps) n_in = 0;
    }
    double2 *o = reinterpret_cast<double2 *>(out + 4 * v);
    o[0] = make_double2(y[0], y[1]);
    o[1] = make_double2(y[2], y[3]);
}

}  // namespace
}  // namespace ms

using namespace ms;

extern "C" int propagate_vertices(const double *in_dev, double *out_dev, int64_t n_vertices, const map_params_t *p,
                                  void *stream)
{
    if (!p || n_vertices < 0 || (n_vertices > 0 && (!in_dev || !out_dev)))
        return fail(MS_E_ARG, "propagate_vertices: bad argument");
    if (p->steps_per_period <= 0) return fail(MS_E_ARG, "propagate_vertices: steps_per_period must be > 0");
    if (!(p->e >= 0.0 && p->e < 1.0) || !(p->mu >= 0.0 && p->mu <= 1.0))
        return fail(MS_E_ARG, "propagate_vertices: need 0 <= e < 1 and 0 <= mu <= 1");
    if (n_vertices == 0) return MS_OK;
    if (!cv_pattern_ok()) return fail(MS_E_ARG, "propagate_vertices: internal tableau pattern mismatch");
    hipStream_t st = (hipStream_t)stream;
    double *wtab = nullptr;
    int rc = stage_table(p->e, p->steps_per_period, STAGE_W, &wtab);
    if (rc) return rc;
    int np = p->n_periods < 0 ? -p->n_periods : p->n_periods;
    int64_t nsteps = (int64_t)p->steps_per_period * np;
    double h = (p->n_periods < 0 ? -6.283185307179586476925286766559 : 6.283185307179586476925286766559) /
               (double)p->steps_per_period;
    if (nsteps == 0) {
        if (in_dev != out_dev) MS_HIP(hipMemcpyAsync(out_dev, in_dev, (size_t)n_vertices * 32, hipMemcpyDeviceToDevice, st));
        return MS_OK;
    }
    Model md{p->mu, 1.0 - p->mu};
    hipLaunchKernelGGL(k_rk8_map, dim3((unsigned)ceil_div(n_vertices, RK_BLOCK)), dim3(RK_BLOCK), 0, st, in_dev,
                       out_dev, n_vertices, md, cv_tableau(), wtab, p->steps_per_period, nsteps, h);
    MS_HIP(hipGetLastError());
    return MS_OK;
}
