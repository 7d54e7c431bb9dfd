// rk8.hip -- stroboscopic map of the planar elliptic restricted three-body
// problem (pulsating rotating coordinates, true anomaly as time), fixed-step
// explicit Runge-Kutta of order 8 (Cooper & Verner 1972, 11 stages).
//
// One thread per state; the tableau is a kernel argument (scalar loads).  The
// stage weights w(f) = 1 / (1 + e cos f) are the same for every state, so
// each block computes them for RK_CHUNK steps at a time into LDS (w is 2 pi
// periodic and even, so the values of one period serve every period and
// both directions); nothing is allocated, and the call can be captured.
#include <math.h>
#include <string.h>

#include "rk8_core.hpp"

namespace ms {

namespace {

constexpr int S = RK_S;
constexpr int RK_BLOCK = 128;

}  // namespace

const Tableau &cv_tableau()
{
    static const Tableau T = cv_make_tableau();
    return T;
}

bool cv_pattern_ok()
{
    if (sqrt(21.0) != RK_SQRT21) return false;
    const Tableau &T = cv_tableau();
    for (int i = 0; i < S; ++i) {
        for (int j = 0; j < S; ++j)
            if ((T.a[i][j] != 0.0) != (j < i && RK_NZ[i][j])) return false;
        if ((T.b[i] != 0.0) != RK_NZB[i]) return false;
    }
    return true;
}

namespace {

__global__ void __launch_bounds__(RK_BLOCK) k_rk8_map(const double *__restrict__ in, double *__restrict__ out,
                                                      int64_t n, Model md, Tableau T, double e, int steps,
                                                      int64_t nsteps, double h)
{
#pragma clang fp contract(fast)
    __shared__ double s_w[RK_CHUNK * S];
    __shared__ double s_c[S];
#pragma unroll
    for (int i = 0; i < S; ++i)
        if (threadIdx.x == i) s_c[i] = T.c[i];
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = v < n;      // every thread of the block fills the weights
    double y[4] = {0.0, 0.0, 0.0, 0.0};
    if (live) {
        const d4 s = load_d4(in + 4 * v);
        y[0] = s.x; y[1] = s.y; y[2] = s.z; y[3] = s.w;
    }
    int64_t n_in = 0;
    for (int64_t st0 = 0; st0 < nsteps; st0 += RK_CHUNK) {
        const int cnt = nsteps - st0 < RK_CHUNK ? (int)(nsteps - st0) : RK_CHUNK;
        __syncthreads();      // the previous chunk's weights are no longer read (and s_c is written)
        fill_stage_chunk(s_w, s_c, n_in, cnt, steps, [&](double f) { return 1.0 / (1.0 + e * cos(f)); });
        __syncthreads();
        if (live) {
            for (int jj = 0; jj < cnt; ++jj) {
                const double *w = s_w + jj * S;
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
            }
        }
        n_in = (n_in + cnt) % steps;
    }
    if (live) {
        double2 *o = reinterpret_cast<double2 *>(out + 4 * v);
        o[0] = make_double2(y[0], y[1]);
        o[1] = make_double2(y[2], y[3]);
    }
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
                       out_dev, n_vertices, md, cv_tableau(), p->e, p->steps_per_period, nsteps, h);
    MS_HIP(hipGetLastError());
    return MS_OK;
}
