// spectral.hip -- periodic theta operations on the rows of a mesh's vertex
// grid: translation a(theta_i) -> a(theta_i + rho) (the re-alignment of the
// globalised points of Sec. 6.1), theta derivatives (Sec. 7) and
// trigonometric interpolation at arbitrary theta (Sec. 7).
//
// A row is n_theta vertices of one s-value, theta_i = 2 pi i / n_theta, in the
// AoS layout of the mesh (4 doubles per vertex, theta fastest).  Frequencies
// are the signed ones; for even n_theta the coefficient at n_theta / 2 acts
// as the real mode cos(n_theta theta / 2), so real rows stay real.
//
// theta_shift: one workgroup per row.  The two real pairs of a vertex are
// packed as complex sequences z0 = x + i y and z1 = px + i py (the spectral
// multiplier is Hermitian, so it acts on both parts independently); both sit
// in LDS and go through a radix-4 Stockham FFT (a last radix-2 pass for odd
// log2 n_theta), in place: each pass reads its butterflies into registers,
// waits, then writes them back, so one buffer per sequence suffices.  The
// twiddle factors e^{-2 pi i m / N} come from a table of N values made once
// per (device, N) on the host and read through the caches.  The
// multiplier (j k)^order e^{j k rho} is applied between the forward and the
// inverse transform, and the result is scaled by 1 / n_theta on the way out.
//
// theta_interp: one wave per query, the barycentric form of the
// trigonometric interpolant (no transform): with theta = theta_i0 + delta,
//   a(theta) = sin(N delta / 2) / N * sum_i (-1)^d a_i g(delta / 2 + pi d / N),
// d = i0 - i reduced to [-N/2, N/2), g = cot for even N and 1 / sin for odd N.
#include <math.h>

#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "ms_internal.hpp"

namespace ms {
namespace {

constexpr int SP_THREADS = 256;
constexpr int SP_MAX_LOG2 = 11;   // n_theta <= 2048: 2 x 32 KiB of LDS per row
constexpr double SP_PI = 3.141592653589793238462643383279502884;

MS_D double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

MS_D double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
MS_D double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// R-point DFT in place (R = 2 or 4); INV selects the sign of the exponent.
template <int R, bool INV>
MS_D void small_dft(double2 *v)
{
    if constexpr (R == 2) {
        double2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else {
        double2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
        double2 b0 = cadd(v[1], v[3]), b1 = csub(v[1], v[3]);
        // -i b1 (forward) or +i b1 (inverse)
        double2 jb1 = INV ? make_double2(-b1.y, b1.x) : make_double2(b1.y, -b1.x);
        v[0] = cadd(a0, b0);
        v[2] = csub(a0, b0);
        v[1] = cadd(a1, jb1);
        v[3] = csub(a1, jb1);
    }
}

// One Stockham pass of radix R over both sequences: butterfly j reads
// z[j + r N/R], twiddles by e^{-+2 pi i r (j mod Ns) / (Ns R)} (entry
// r (j mod Ns) N / (Ns R) of the table, conjugated for the inverse),
// transforms, and writes z[(j / Ns) Ns R + (j mod Ns) + r Ns].
template <int N, int R, bool INV>
MS_D void stockham_pass(double2 (*z)[N], int Ns, const double2 *__restrict__ tw)
{
    constexpr int NB = N / R;
    constexpr int PER = (NB + SP_THREADS - 1) / SP_THREADS;
    double2 v[2][PER][R];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = threadIdx.x + q * SP_THREADS;
        if (NB % SP_THREADS == 0 || j < NB) {
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int r = 0; r < R; ++r) v[s][q][r] = z[s][j + r * NB];
            const int k = j % Ns;
            if (k != 0) {
                const int stride = N / (Ns * R);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    double2 w = tw[r * k * stride];
                    if (INV) w.y = -w.y;
#pragma unroll
                    for (int s = 0; s < 2; ++s) v[s][q][r] = cmul(v[s][q][r], w);
                }
            }
#pragma unroll
            for (int s = 0; s < 2; ++s) small_dft<R, INV>(v[s][q]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = threadIdx.x + q * SP_THREADS;
        if (NB % SP_THREADS == 0 || j < NB) {
            const int k = j % Ns;
            const int base = (j / Ns) * Ns * R + k;
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int r = 0; r < R; ++r) z[s][base + r * Ns] = v[s][q][r];
        }
    }
    __syncthreads();
}

template <int LOGN, bool INV>
MS_D void fft2(double2 (*z)[1 << LOGN], const double2 *__restrict__ tw)
{
    constexpr int N = 1 << LOGN;
    int Ns = 1;
#pragma unroll
    for (int p = 0; p < LOGN / 2; ++p) {
        stockham_pass<N, 4, INV>(z, Ns, tw);
        Ns *= 4;
    }
    if constexpr (LOGN & 1) stockham_pass<N, 2, INV>(z, Ns, tw);
}

template <int LOGN>
__global__ void __launch_bounds__(SP_THREADS) k_theta_shift(const double *in, double *out,
                                                            const double2 *__restrict__ tw, const double *rho_dev,
                                                            double rho, int order)
{
    constexpr int N = 1 << LOGN;
    __shared__ double2 z[2][N];
    const int64_t row = blockIdx.x;
    const double *src = in + row * (int64_t)N * 4;
    for (int i = threadIdx.x; i < N; i += SP_THREADS) {
        d4 v = load_d4(src + 4 * i);
        z[0][i] = make_double2(v.x, v.y);
        z[1][i] = make_double2(v.z, v.w);
    }
    __syncthreads();
    fft2<LOGN, false>(z, tw);
    const double r = rho_dev ? rho_dev[row] : rho;
    for (int k = threadIdx.x; k < N; k += SP_THREADS) {
        double2 m;
        if (2 * k == N) {
            // the cosine mode: Re[(j N/2)^order e^{j (N/2) rho}]
            const double h = 0.5 * (double)N;
            double sn, cs;
            sincos(h * r, &sn, &cs);
            m = make_double2(order == 0 ? cs : order == 1 ? -h * sn : -h * h * cs, 0.0);
        } else {
            const double ks = 2 * k > N ? (double)(k - N) : (double)k;
            double sn, cs;
            sincos(ks * r, &sn, &cs);
            m = make_double2(cs, sn);
            if (order == 1) m = make_double2(-ks * sn, ks * cs);
            else if (order == 2) m = make_double2(-ks * ks * cs, -ks * ks * sn);
        }
        z[0][k] = cmul(z[0][k], m);
        z[1][k] = cmul(z[1][k], m);
    }
    __syncthreads();
    fft2<LOGN, true>(z, tw);
    const double inv = 1.0 / (double)N;
    double *dst = out + row * (int64_t)N * 4;
    for (int i = threadIdx.x; i < N; i += SP_THREADS) {
        double2 a = z[0][i], b = z[1][i];
        double2 *o = reinterpret_cast<double2 *>(dst + 4 * i);
        o[0] = make_double2(a.x * inv, a.y * inv);
        o[1] = make_double2(b.x * inv, b.y * inv);
    }
}

constexpr int IP_WAVES = 4;

__global__ void __launch_bounds__(64 * IP_WAVES) k_theta_interp(const double *in, int N, int64_t n_rows,
                                                                const int64_t *rows, const double *theta, int64_t nq,
                                                                double *out)
{
    const int64_t q = (int64_t)blockIdx.x * IP_WAVES + threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    if (q >= nq) return;   // whole waves
    const int64_t row = rows[q];
    const double th = theta[q];
    double *o = out + 4 * q;
    if (row < 0 || row >= n_rows || !isfinite(th)) {
        if (lane < 4) o[lane] = NAN;
        return;
    }
    const double *a = in + row * (int64_t)N * 4;
    const double step = 2.0 * SP_PI / (double)N;
    // nearest sample i0 (reduced to [0, N)) and the offset delta from it
    const double i0f = rint(th / step);
    const double delta = th - i0f * step;
    int64_t i0 = (int64_t)fmod(i0f, (double)N);
    if (i0 < 0) i0 += N;
    if (fabs(delta) < 1e-200) {
        if (lane < 4) o[lane] = a[4 * i0 + lane];
        return;
    }
    const bool even = (N & 1) == 0;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = lane; i < N; i += 64) {
        int64_t d = i0 - i;                 // in (-N, N); the kernel is N-periodic in d
        if (2 * d >= N) d -= N;
        else if (2 * d < -N) d += N;
        double sn, cs;
        sincos(0.5 * delta + SP_PI * (double)d / (double)N, &sn, &cs);
        double w = even ? cs / sn : 1.0 / sn;
        if (d & 1) w = -w;
        d4 v = load_d4(a + 4 * i);
        acc[0] += w * v.x;
        acc[1] += w * v.y;
        acc[2] += w * v.z;
        acc[3] += w * v.w;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc[c] += __shfl_xor(acc[c], off);
    if (lane < 4) {
        const double f = sin(0.5 * (double)N * delta) / (double)N;
        double s = lane == 0 ? acc[0] : lane == 1 ? acc[1] : lane == 2 ? acc[2] : acc[3];
        o[lane] = f * s;
    }
}

template <int LOGN>
void launch_shift(const double *in, double *out, const double2 *tw, int64_t n_rows, const double *rho_dev,
                  double rho, int order, hipStream_t st)
{
    hipLaunchKernelGGL(k_theta_shift<LOGN>, dim3((unsigned)n_rows), dim3(SP_THREADS), 0, st, in, out, tw, rho_dev,
                       rho, order);
}

// e^{-2 pi i m / N}, m = 0..N-1, per (device, N), kept for the life of the
// process.  2 m / N is exact for a power of two N, so each entry is the
// rounded cosine and sine of one rounded argument.
std::mutex g_tw_mu;
std::map<std::pair<int, int>, double2 *> g_tw;

int twiddles(int N, const double2 **out)
{
    int dev = 0;
    MS_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_tw_mu);
    auto key = std::make_pair(dev, N);
    auto it = g_tw.find(key);
    if (it != g_tw.end()) { *out = it->second; return MS_OK; }
    std::vector<double2> w(N);
    for (int m = 0; m < N; ++m) {
        const double a = SP_PI * (2.0 * (double)m / (double)N);
        w[m] = make_double2(cos(a), -sin(a));
    }
    double2 *d = nullptr;
    MS_HIP(hipMalloc(&d, (size_t)N * sizeof(double2)));
    hipError_t er = hipMemcpy(d, w.data(), (size_t)N * sizeof(double2), hipMemcpyHostToDevice);
    if (er != hipSuccess) { (void)hipFree(d); return hip_fail(er, "copy twiddle table"); }
    g_tw[key] = d;
    *out = d;
    return MS_OK;
}

}  // namespace
}  // namespace ms

using namespace ms;

extern "C" int theta_shift(const double *in_dev, double *out_dev, int32_t n_theta, int64_t n_rows,
                           const double *rho_dev, double rho, int32_t order, void *stream)
{
    if (n_rows < 0 || (n_rows > 0 && (!in_dev || !out_dev))) return fail(MS_E_ARG, "theta_shift: bad argument");
    if (n_theta < 2 || n_theta > (1 << SP_MAX_LOG2) || (n_theta & (n_theta - 1)))
        return fail(MS_E_ARG, "theta_shift: n_theta must be a power of two in [2, 2048]");
    if (order < 0 || order > 2) return fail(MS_E_ARG, "theta_shift: order must be 0, 1 or 2");
    if (!rho_dev && !isfinite(rho)) return fail(MS_E_ARG, "theta_shift: rho must be finite");
    if (n_rows > 0x7fffffff) return fail(MS_E_ARG, "theta_shift: too many rows for one launch");
    if (n_rows == 0) return MS_OK;
    hipStream_t st = (hipStream_t)stream;
    const double2 *tw = nullptr;
    int rc = twiddles(n_theta, &tw);
    if (rc) return rc;
    int lg = 0;
    while ((1 << lg) < n_theta) ++lg;
    switch (lg) {
    case 1: launch_shift<1>(in_dev, out_dev, tw, n_rows, rho_dev, rho, order, st); break;
    case 2: launch_shift<2>(in_dev, out_dev, tw, n_rows, rho_dev, rho, order, st); break;
    case 3: launch_shift<3>(in_dev, out_dev, tw, n_rows, rho_dev, rho, order, st); break;
    case 4: launch_shift<4>(in_dev, out_dev, tw, n_rows, rho_dev, rho, order, st); break;
    case 5: launch_shift<5>(in_dev, out_dev, tw, n_rows, rho_dev, rho, order, st); break;
    case 6: launch_shift<6>(in_dev, out_dev, tw, n_rows, rho_dev, rho, order, st); break;
    case 7: launch_shift<7>(in_dev, out_dev, tw, n_rows, rho_dev, rho, order, st); break;
    case 8: launch_shift<8>(in_dev, out_dev, tw, n_rows, rho_dev, rho, order, st); break;
    case 9: launch_shift<9>(in_dev, out_dev, tw, n_rows, rho_dev, rho, order, st); break;
    case 10: launch_shift<10>(in_dev, out_dev, tw, n_rows, rho_dev, rho, order, st); break;
    default: launch_shift<11>(in_dev, out_dev, tw, n_rows, rho_dev, rho, order, st); break;
    }
    MS_HIP(hipGetLastError());
    return MS_OK;
}

extern "C" int theta_interp(const double *rows_dev, int32_t n_theta, int64_t n_rows, const int64_t *row_dev,
                            const double *theta_dev, int64_t n_query, double *out_dev, void *stream)
{
    if (n_query < 0 || n_rows < 0 || n_theta < 1 ||
        (n_query > 0 && (!rows_dev || !row_dev || !theta_dev || !out_dev)))
        return fail(MS_E_ARG, "theta_interp: bad argument");
    if (n_query == 0) return MS_OK;
    const int64_t blocks = ceil_div(n_query, IP_WAVES);
    if (blocks > 0x7fffffff) return fail(MS_E_ARG, "theta_interp: too many queries for one launch");
    hipLaunchKernelGGL(k_theta_interp, dim3((unsigned)blocks), dim3(64 * IP_WAVES), 0, (hipStream_t)stream, rows_dev,
                       (int)n_theta, n_rows, row_dev, theta_dev, n_query, out_dev);
    MS_HIP(hipGetLastError());
    return MS_OK;
}
