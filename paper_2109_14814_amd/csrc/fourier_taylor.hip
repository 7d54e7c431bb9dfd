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
#include <math.h>

#include <string>

#include "ms_internal.hpp"

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

}  // namespace
}  // namespace ms

using namespace ms;

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
