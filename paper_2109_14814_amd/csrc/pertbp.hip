// pertbp.hip -- stroboscopic map F of the planar elliptic restricted
// three-body problem in the position-momentum coordinates of Sec. 3.3 (time t,
// frame turning with the primaries but not rescaled, periapse at t = 0), and
// its state transition matrix DF^m (the derivative the parameterization
// formulas of Sec. 7 need).
//
// Same fixed-step order-8 Runge-Kutta method as the pulsating map.  The
// time-dependent coefficients, the separation rho(t) of the primaries and the
// rate n(t) of their true anomaly, come from Kepler's equation; each block
// solves it for the stage times of RK_CHUNK steps at a time into LDS (both
// are 2 pi periodic and even in t, so one period's values serve every period
// and both directions).  Nothing is allocated; every call can be captured.
//
// The map runs one thread per state.  The matrix runs 4 / NC threads per
// state, each carrying the state and NC of the 4 tangent columns (the
// variational equations integrated with the same stages, so the result is
// the exact derivative of the discrete map): NC = 4 computes the field once
// per state (the default for large batches: fastest on gfx950 although it
// runs at one wave per SIMD), NC = 1 keeps the fewest registers live and
// gives small batches four times the threads.
#include <math.h>

#include <string>

#include "rk8_core.hpp"

namespace ms {
namespace {

constexpr int S = RK_S;
constexpr int PM_BLOCK = 128;

// NC = 0: state only.  NC > 0: state and tangent columns g NC .. g NC + NC - 1
// of DF, g = thread index within its state.
template <int NC>
__global__ void __launch_bounds__(PM_BLOCK) k_pm_flow(const double *__restrict__ in, double *out,
                                                      double *__restrict__ stm, int64_t n, Model md, Tableau T,
                                                      double ecc, int steps, int64_t nsteps, double h)
{
#pragma clang fp contract(fast)
    constexpr int G = NC > 0 ? 4 / NC : 1;   // threads per state
    constexpr int NV = NC > 0 ? NC : 1;
    __shared__ double2 s_rn[RK_CHUNK * S];
    __shared__ double s_c[S];
#pragma unroll
    for (int i = 0; i < S; ++i)
        if (threadIdx.x == i) s_c[i] = T.c[i];
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = gid < n * G;      // every thread of the block fills the stage values
    const int64_t p = live ? gid / G : 0;
    const int g = (int)(gid - (gid / G) * G);
    double z[4] = {0.0, 0.0, 0.0, 0.0};
    if (live) {
        const d4 s = load_d4(in + 4 * p);
        z[0] = s.x; z[1] = s.y; z[2] = s.z; z[3] = s.w;
    }
    double v[NV][4];
#pragma unroll
    for (int c = 0; c < NV; ++c)
#pragma unroll
        for (int i = 0; i < 4; ++i) v[c][i] = (i == g * NC + c) ? 1.0 : 0.0;
    int64_t n_in = 0;
    for (int64_t st0 = 0; st0 < nsteps; st0 += RK_CHUNK) {
        const int cnt = nsteps - st0 < RK_CHUNK ? (int)(nsteps - st0) : RK_CHUNK;
        __syncthreads();      // the previous chunk's values are no longer read (and s_c is written)
        fill_stage_chunk(s_rn, s_c, n_in, cnt, steps, [&](double t) { return kepler_rho_n(t, ecc); });
        __syncthreads();
        n_in = (n_in + cnt) % steps;
        if (!live) continue;
        for (int jj = 0; jj < cnt; ++jj) {
            const double2 *row = s_rn + jj * S;
            double k[S][4];
            double kv[S][NV][4];
#pragma unroll
            for (int i = 0; i < S; ++i) {
                double zs[4], vs[NV][4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    double acc = 0.0;
#pragma unroll
                    for (int j = 0; j < i; ++j)
                        if (RK_NZ[i][j]) acc += T.a[i][j] * k[j][c];
                    zs[c] = z[c] + h * acc;
                }
                if constexpr (NC > 0) {
#pragma unroll
                    for (int q = 0; q < NC; ++q)
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            double acc = 0.0;
#pragma unroll
                            for (int j = 0; j < i; ++j)
                                if (RK_NZ[i][j]) acc += T.a[i][j] * kv[j][q][c];
                            vs[q][c] = v[q][c] + h * acc;
                        }
                }
                const double2 rn = row[i];
                if constexpr (NC > 0) pm_field_var<NC>(md, rn.x, rn.y, zs, vs, k[i], kv[i]);
                else pm_field(md, rn.x, rn.y, zs, k[i]);
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double acc = 0.0;
#pragma unroll
                for (int i = 0; i < S; ++i)
                    if (RK_NZB[i]) acc += T.b[i] * k[i][c];
                z[c] = z[c] + h * acc;
            }
            if constexpr (NC > 0) {
#pragma unroll
                for (int q = 0; q < NC; ++q)
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        double acc = 0.0;
#pragma unroll
                        for (int i = 0; i < S; ++i)
                            if (RK_NZB[i]) acc += T.b[i] * kv[i][q][c];
                        v[q][c] = v[q][c] + h * acc;
                    }
            }
        }
    }
    if (!live) return;
    if (out && g == 0) {
        double2 *o = reinterpret_cast<double2 *>(out + 4 * p);
        o[0] = make_double2(z[0], z[1]);
        o[1] = make_double2(z[2], z[3]);
    }
    if constexpr (NC > 0) {
        // Row-major 4 x 4 per state: stm[16 p + 4 i + j] = d out_i / d in_j.
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int i = 0; i < 4; ++i) stm[16 * p + 4 * i + g * NC + q] = v[q][i];
    }
}

int pm_check(const char *who, const double *in_dev, const void *out_dev, int64_t n, const map_params_t *p)
{
    const std::string w(who);
    if (!p || n < 0 || (n > 0 && (!in_dev || !out_dev))) return fail(MS_E_ARG, w + ": bad argument");
    if (p->steps_per_period <= 0) return fail(MS_E_ARG, w + ": steps_per_period must be > 0");
    if (!(p->e >= 0.0 && p->e < 1.0) || !(p->mu >= 0.0 && p->mu <= 1.0))
        return fail(MS_E_ARG, w + ": need 0 <= e < 1 and 0 <= mu <= 1");
    if (!cv_pattern_ok()) return fail(MS_E_ARG, w + ": internal tableau pattern mismatch");
    return MS_OK;
}

template <int NC>
int pm_launch(const double *in, double *out, double *stm, int64_t n, const map_params_t *p, hipStream_t st)
{
    const int np = p->n_periods < 0 ? -p->n_periods : p->n_periods;
    const int64_t nsteps = (int64_t)p->steps_per_period * np;
    const double h = (p->n_periods < 0 ? -RK_TWO_PI : RK_TWO_PI) / (double)p->steps_per_period;
    constexpr int G = NC > 0 ? 4 / NC : 1;
    const int64_t threads = n * G;
    // The launch counts work-items in 32 bits.
    if (n > (((int64_t)1 << 32) - PM_BLOCK) / G) return fail(MS_E_ARG, "pertbp: too many states for one launch");
    Model md{p->mu, 1.0 - p->mu};
    hipLaunchKernelGGL(k_pm_flow<NC>, dim3((unsigned)ceil_div(threads, PM_BLOCK)), dim3(PM_BLOCK), 0, st, in, out,
                       stm, n, md, cv_tableau(), p->e, p->steps_per_period, nsteps, h);
    MS_HIP(hipGetLastError());
    return MS_OK;
}

}  // namespace
}  // namespace ms

using namespace ms;

extern "C" int pertbp_map(const double *in_dev, double *out_dev, int64_t n_states, const map_params_t *p,
                          void *stream)
{
    int rc = pm_check("pertbp_map", in_dev, out_dev, n_states, p);
    if (rc || n_states == 0) return rc;
    return pm_launch<0>(in_dev, out_dev, nullptr, n_states, p, (hipStream_t)stream);
}

extern "C" int pertbp_map_stm(const double *in_dev, double *out_dev, double *stm_dev, int64_t n_states,
                              const map_params_t *p, int32_t cols_per_thread, void *stream)
{
    int rc = pm_check("pertbp_map_stm", in_dev, stm_dev, n_states, p);
    if (rc) return rc;
    // default: four columns per thread (the least work per state) once the
    // batch fills the chip with them, else more threads per state
    if (cols_per_thread == 0) cols_per_thread = n_states >= (1 << 17) ? 4 : n_states >= (1 << 16) ? 2 : 1;
    if (cols_per_thread != 1 && cols_per_thread != 2 && cols_per_thread != 4)
        return fail(MS_E_ARG, "pertbp_map_stm: cols_per_thread must be 0, 1, 2 or 4");
    if (n_states == 0) return MS_OK;
    if (out_dev && (const void *)out_dev < (const void *)(stm_dev + 16 * n_states) &&
        (const void *)stm_dev < (const void *)(out_dev + 4 * n_states))
        return fail(MS_E_ARG, "pertbp_map_stm: out and stm overlap");
    if ((const void *)in_dev < (const void *)(stm_dev + 16 * n_states) &&
        (const void *)stm_dev < (const void *)(in_dev + 4 * n_states))
        return fail(MS_E_ARG, "pertbp_map_stm: in and stm overlap");
    hipStream_t st = (hipStream_t)stream;
    switch (cols_per_thread) {
    case 1: return pm_launch<1>(in_dev, out_dev, stm_dev, n_states, p, st);
    case 2: return pm_launch<2>(in_dev, out_dev, stm_dev, n_states, p, st);
    default: return pm_launch<4>(in_dev, out_dev, stm_dev, n_states, p, st);
    }
}
