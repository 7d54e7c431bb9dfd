// fourier_taylor.hip -- points and partials of Fourier-Taylor
// parameterizations W(theta, s) = sum_k W_k(theta) s^k of a manifold, and of
// their globalization W(theta, s) = F^m(W(theta - m omega, lambda^-m s))
// (Sec. 7).
//
// The coefficients W_k are given by their spectra over theta (theta_spectrum
// of each coefficient row, scaled by 1/N, the pairs (x, y) and (px, py)
// packed as complex sequences).  One wave evaluates one query (theta, s):
// each lane takes frequencies j = lane, lane + 64, ..., sums the series in s
// at j by Horner's rule (the value and its s-derivative together), and adds
// the terms e^{i j theta} V(j) and i j e^{i j theta} V(j); a wave reduction
// gives W, dW/dtheta and dW/ds.  This is the paper's "evaluate in s, FFT
// derivative in theta, interpolate trigonometrically", done in the
// frequency domain so that no per-query transform is needed: the
// trigonometric interpolant of the samples is the sum over their spectrum.
//
// Globalization: the local evaluation at (theta - m omega, lambda^-m s) (the
// s-derivative already scaled by lambda^-m), then F^m and DF^m of the point
// by the position-momentum map, then the two partials multiplied by DF^m.
//
// Refinement (ft_newton): the damped Newton iteration of Sec. 7 on
// f = W_u(theta_u, s_u) - W_s(theta_s, s_s) with Df from the four partials,
// one ft_partials per chart and one decision kernel per iteration.
#include <math.h>

#include <string>

#include "newton.hpp"

namespace ms {
namespace {

constexpr int FT_WAVES = 4;

__global__ void __launch_bounds__(64 * FT_WAVES) k_ft_eval(const double *__restrict__ spec, int N, int P,
                                                           const double *__restrict__ theta,
                                                           const double *__restrict__ s, int64_t nq, double th_off,
                                                           double s_scale, double *w, double *dth, double *ds)
{
    const int64_t q = (int64_t)blockIdx.x * FT_WAVES + threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    if (q >= nq) return;   // whole waves
    const double t = theta[q] - th_off;
    const double sl = s[q] * s_scale;
    if (!isfinite(t) || !isfinite(sl)) {
        if (lane < 4) w[4 * q + lane] = dth[4 * q + lane] = ds[4 * q + lane] = NAN;
        return;
    }
    double aw[4] = {0, 0, 0, 0}, ath[4] = {0, 0, 0, 0}, as[4] = {0, 0, 0, 0};
    for (int j = lane; j < N; j += 64) {
        double v0 = 0, v1 = 0, v2 = 0, v3 = 0, d0 = 0, d1 = 0, d2 = 0, d3 = 0;
        for (int k = P; k >= 0; --k) {
            const d4 c = load_d4(spec + ((int64_t)k * N + j) * 4);
            d0 = d0 * sl + v0; v0 = v0 * sl + c.x;
            d1 = d1 * sl + v1; v1 = v1 * sl + c.y;
            d2 = d2 * sl + v2; v2 = v2 * sl + c.z;
            d3 = d3 * sl + v3; v3 = v3 * sl + c.w;
        }
        const double v[4] = {v0, v1, v2, v3}, dv[4] = {d0, d1, d2, d3};
        const bool nyq = 2 * j == N;
        const double js = 2 * j > N ? (double)(j - N) : (double)j;
        double sn, cs;
        sincos(nyq ? 0.5 * (double)N * t : js * t, &sn, &cs);
        if (nyq) {
            // the cosine mode cos(N theta / 2): real factor on both parts.  It
            // adds nothing to the theta derivative: the derivative is taken
            // at the samples (coefficient j times i j, whose real part is 0
            // at j = N/2) and then interpolated.
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                aw[i] += v[i] * cs;
                as[i] += dv[i] * cs;
            }
        } else {
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const double re = v[2 * p] * cs - v[2 * p + 1] * sn;
                const double im = v[2 * p] * sn + v[2 * p + 1] * cs;
                aw[2 * p] += re;
                aw[2 * p + 1] += im;
                ath[2 * p] += -js * im;      // i js (re + i im)
                ath[2 * p + 1] += js * re;
                as[2 * p] += dv[2 * p] * cs - dv[2 * p + 1] * sn;
                as[2 * p + 1] += dv[2 * p] * sn + dv[2 * p + 1] * cs;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            aw[i] += __shfl_xor(aw[i], off);
            ath[i] += __shfl_xor(ath[i], off);
            as[i] += __shfl_xor(as[i], off);
        }
    // every lane holds the totals after the butterfly reduction
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            w[4 * q + i] = aw[i];
            dth[4 * q + i] = ath[i];
            ds[4 * q + i] = as[i] * s_scale;   // d/ds of W(theta, lambda^-m s)
        }
    }
}

// dth <- M dth, ds <- M ds per query (M row-major 4 x 4).
__global__ void __launch_bounds__(256) k_apply_stm(const double *__restrict__ stm, double *dth, double *ds, int64_t nq)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    const double *M = stm + 16 * q;
    double a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        a[i] = dth[4 * q + i];
        b[i] = ds[4 * q + i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        dth[4 * q + i] = M[4 * i] * a[0] + M[4 * i + 1] * a[1] + M[4 * i + 2] * a[2] + M[4 * i + 3] * a[3];
        ds[4 * q + i] = M[4 * i] * b[0] + M[4 * i + 1] * b[1] + M[4 * i + 2] * b[2] + M[4 * i + 3] * b[3];
    }
}

// Parameters and partials of one side of the Newton problems.
struct FtSide {
    double *th, *s, *w, *dth, *ds, *stm;
};

MS_D void ftn_split(int64_t k, const NewtonState &ns, const FtSide &u, const FtSide &v)
{
    u.th[k] = ns.q[4 * k + 0];
    u.s[k] = ns.q[4 * k + 1];
    v.th[k] = ns.q[4 * k + 2];
    v.s[k] = ns.q[4 * k + 3];
}

__global__ void __launch_bounds__(256) k_ftn_init(const double *x0, NewtonState ns, int64_t K, FtSide u, FtSide v,
                                                  unsigned long long *running)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0) running[0] = running[1] = 0;
    if (k >= K) return;
    newton_init(k, x0, ns);
    ftn_split(k, ns, u, v);
}

// One decision per running problem; counts the problems still running in
// running[par] and clears the other counter for the next iteration.
__global__ void __launch_bounds__(256) k_ftn_update(NewtonState ns, NewtonCfg cfg, int64_t K, FtSide u, FtSide v,
                                                    unsigned long long *running, int par)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0) running[par ^ 1] = 0;
    if (k >= K || ns.status[k] >= 0) return;
    double f[4], M[4][4];
    for (int c = 0; c < 4; ++c) {
        f[c] = u.w[4 * k + c] - v.w[4 * k + c];
        M[c][0] = u.dth[4 * k + c];
        M[c][1] = u.ds[4 * k + c];
        M[c][2] = -v.dth[4 * k + c];
        M[c][3] = -v.ds[4 * k + c];
    }
    newton_decide(k, f, M, ns, cfg);
    if (ns.status[k] < 0) {
        ftn_split(k, ns, u, v);
        atomicAdd(&running[par], 1ull);
    }
}

__global__ void __launch_bounds__(256) k_ftn_finish(NewtonState ns, int64_t K, double *x_out, double *f_out,
                                                    double *r_out, int32_t *st_out, int32_t *tr_out)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    newton_finish(k, ns, x_out, f_out, r_out, st_out, tr_out);
}

// Linear continuation predictor (Sec. 8), one row per thread.
__global__ void __launch_bounds__(256) k_cont_predict(const double *x0, const double *x1, const double *om0,
                                                      const double *om1, const double *dom, int64_t K, double *out)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    double q = 0.0;
    if (x1) {
        if (dom[2 * k] != 0.0) q = dom[2 * k] / (om0[2 * k] - om1[2 * k]);
        else if (dom[2 * k + 1] != 0.0) q = dom[2 * k + 1] / (om0[2 * k + 1] - om1[2 * k + 1]);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const double a = x0[4 * k + c];
        out[4 * k + c] = x1 ? a + q * (a - x1[4 * k + c]) : a;
    }
}

// Workspace layout of ft_newton for K problems (256-byte aligned pieces).
struct FtnLayout {
    size_t total;
    size_t o[24];
};

FtnLayout ftn_layout(int64_t K)
{
    FtnLayout L;
    const size_t d4b = (size_t)K * 32, d1b = (size_t)K * 8, i1b = (size_t)K * 4, d16b = (size_t)K * 128;
    const size_t sizes[] = {d4b, d4b, d4b, d4b, d1b, d1b, i1b, i1b, i1b,     // p q delta fp rp alpha status trials based
                            d1b, d1b, d4b, d4b, d4b, d16b,                   // side u: th s w dth ds stm
                            d1b, d1b, d4b, d4b, d4b, d16b,                   // side s
                            16};                                             // running counters
    size_t at = 0;
    for (size_t i = 0; i < sizeof(sizes) / sizeof(sizes[0]); ++i) {
        L.o[i] = at;
        at += (sizes[i] + 255) & ~(size_t)255;
    }
    L.total = at;
    return L;
}

}  // namespace
}  // namespace ms

using namespace ms;

extern "C" int continuation_predict(const double *x0_dev, const double *omega0_dev, const double *domega_dev,
                                    const double *x1_dev, const double *omega1_dev, int64_t K, double *out_dev,
                                    void *stream)
{
    if (K < 0 || (K > 0 && (!x0_dev || !out_dev || (x1_dev && (!omega0_dev || !omega1_dev || !domega_dev)))))
        return fail(MS_E_ARG, "continuation_predict: bad argument");
    if (K == 0) return MS_OK;
    if (ceil_div(K, 256) > 0x7fffffff) return fail(MS_E_ARG, "continuation_predict: too many rows");
    hipLaunchKernelGGL(k_cont_predict, dim3((unsigned)ceil_div(K, 256)), dim3(256), 0, (hipStream_t)stream, x0_dev,
                       x1_dev, omega0_dev, omega1_dev, domega_dev, K, out_dev);
    MS_HIP(hipGetLastError());
    return MS_OK;
}

extern "C" int ft_newton_workspace_size(int64_t K, size_t *bytes)
{
    if (K < 0 || !bytes) return fail(MS_E_ARG, "ft_newton_workspace_size: bad argument");
    *bytes = ftn_layout(K).total;
    return MS_OK;
}

extern "C" int ft_newton(const double *params_in_dev, double *params_out_dev, int64_t K, const ft_chart_t *U,
                         const ft_chart_t *S, const map_params_t *map, const newton_params_t *np, double *f_dev,
                         double *r_dev, int32_t *status_dev, int32_t *trials_dev, void *ws, size_t ws_bytes,
                         void *stream)
{
    if (K < 0 || !U || !S || !map || !np || (K > 0 && (!params_in_dev || !params_out_dev)))
        return fail(MS_E_ARG, "ft_newton: bad argument");
    if (np->max_trials < 0 || np->max_trials > 100000) return fail(MS_E_ARG, "ft_newton: max_trials out of range");
    if (!(np->alpha0 > 0.0 && np->alpha0 <= 1.0) || !(np->alpha_min > 0.0) || !(np->tol >= 0.0))
        return fail(MS_E_ARG, "ft_newton: need 0 < alpha0 <= 1, alpha_min > 0, tol >= 0");
    if (!U->spec_dev || !S->spec_dev) return fail(MS_E_ARG, "ft_newton: chart spectra missing");
    if (K == 0) return MS_OK;
    if (K > ((int64_t)1 << 28)) return fail(MS_E_ARG, "ft_newton: K too large");
    const FtnLayout L = ftn_layout(K);
    if (!ws || ws_bytes < L.total) return fail(MS_E_WORKSPACE, "ft_newton: workspace too small");
    char *w = (char *)ws;
    NewtonState ns;
    ns.p = (double *)(w + L.o[0]);
    ns.q = (double *)(w + L.o[1]);
    ns.delta = (double *)(w + L.o[2]);
    ns.fp = (double *)(w + L.o[3]);
    ns.rp = (double *)(w + L.o[4]);
    ns.alpha = (double *)(w + L.o[5]);
    ns.status = (int32_t *)(w + L.o[6]);
    ns.trials = (int32_t *)(w + L.o[7]);
    ns.based = (int32_t *)(w + L.o[8]);
    FtSide su{(double *)(w + L.o[9]), (double *)(w + L.o[10]), (double *)(w + L.o[11]), (double *)(w + L.o[12]),
              (double *)(w + L.o[13]), (double *)(w + L.o[14])};
    FtSide ss{(double *)(w + L.o[15]), (double *)(w + L.o[16]), (double *)(w + L.o[17]), (double *)(w + L.o[18]),
              (double *)(w + L.o[19]), (double *)(w + L.o[20])};
    unsigned long long *running = (unsigned long long *)(w + L.o[21]);
    NewtonCfg cfg;
    cfg.tol2 = np->tol * np->tol;
    cfg.alpha0 = np->alpha0;
    cfg.alpha_min = np->alpha_min;
    cfg.max_trials = np->max_trials;
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid((unsigned)ceil_div(K, 256));
    map_params_t mu_map = *map, ms_map = *map;
    mu_map.n_periods = U->n_periods;
    ms_map.n_periods = S->n_periods;
    hipLaunchKernelGGL(k_ftn_init, grid, dim3(256), 0, st, params_in_dev, ns, K, su, ss, running);
    MS_HIP(hipGetLastError());
    for (int it = 0; it <= np->max_trials; ++it) {
        int rc = ft_partials(U->spec_dev, U->n_theta, U->order, su.th, su.s, K, U->omega, U->lambda, &mu_map, su.w,
                             su.dth, su.ds, su.stm, stream);
        if (rc) return rc;
        rc = ft_partials(S->spec_dev, S->n_theta, S->order, ss.th, ss.s, K, S->omega, S->lambda, &ms_map, ss.w,
                         ss.dth, ss.ds, ss.stm, stream);
        if (rc) return rc;
        const int par = it & 1;
        hipLaunchKernelGGL(k_ftn_update, grid, dim3(256), 0, st, ns, cfg, K, su, ss, running, par);
        MS_HIP(hipGetLastError());
        unsigned long long left = 0;
        MS_HIP(hipMemcpyAsync(&left, running + par, sizeof left, hipMemcpyDeviceToHost, st));
        MS_HIP(hipStreamSynchronize(st));
        if (left == 0) break;
    }
    hipLaunchKernelGGL(k_ftn_finish, grid, dim3(256), 0, st, ns, K, params_out_dev, f_dev, r_dev, status_dev,
                       trials_dev);
    MS_HIP(hipGetLastError());
    return MS_OK;
}

extern "C" int ft_partials(const double *spec_dev, int32_t n_theta, int32_t order, const double *theta_dev,
                           const double *s_dev, int64_t n_query, double omega, double lambda,
                           const map_params_t *map, double *w_dev, double *dth_dev, double *ds_dev,
                           double *stm_dev, void *stream)
{
    if (n_query < 0 || n_theta < 1 || order < 0 ||
        (n_query > 0 && (!spec_dev || !theta_dev || !s_dev || !w_dev || !dth_dev || !ds_dev)))
        return fail(MS_E_ARG, "ft_partials: bad argument");
    const int m = map ? map->n_periods : 0;
    if (m != 0 && !stm_dev) return fail(MS_E_ARG, "ft_partials: stm_dev is required when n_periods != 0");
    if (m != 0 && !(lambda > 0.0 && isfinite(lambda) && isfinite(omega)))
        return fail(MS_E_ARG, "ft_partials: need a finite omega and lambda > 0");
    if (n_query == 0) return MS_OK;
    const int64_t blocks = ceil_div(n_query, FT_WAVES);
    if (blocks > 0x7fffffff) return fail(MS_E_ARG, "ft_partials: too many queries for one launch");
    hipStream_t st = (hipStream_t)stream;
    const double th_off = (double)m * omega;
    const double s_scale = m == 0 ? 1.0 : pow(lambda, -(double)m);
    hipLaunchKernelGGL(k_ft_eval, dim3((unsigned)blocks), dim3(64 * FT_WAVES), 0, st, spec_dev, (int)n_theta,
                       (int)order, theta_dev, s_dev, n_query, th_off, s_scale, w_dev, dth_dev, ds_dev);
    MS_HIP(hipGetLastError());
    if (m == 0) return MS_OK;
    int rc = pertbp_map_stm(w_dev, w_dev, stm_dev, n_query, map, 0, stream);
    if (rc) return rc;
    hipLaunchKernelGGL(k_apply_stm, dim3((unsigned)ceil_div(n_query, 256)), dim3(256), 0, st, stm_dev, dth_dev,
                       ds_dev, n_query);
    MS_HIP(hipGetLastError());
    return MS_OK;
}
