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
// multiplier is Hermitian, so it acts on both parts independently) and go
// through a Stockham FFT of radix 8 (a last pass of radix 4 or 2 for the
// remaining factor) that keeps both sequences in LDS, in place: each pass
// reads its butterflies into registers, waits, then writes them back.  The
// LDS index is padded by one slot per 8 so that the strided writes of the
// first passes spread over the banks.  The first forward pass reads the row
// straight from global memory and the last inverse pass writes it back
// (scaled by 1 / N); the inverse runs the radices in reverse order, so the
// last forward pass, the multiplier (j k)^order e^{j k rho} and the first
// inverse pass work on the same registers with no LDS round trip between
// them.  The twiddle factors e^{-2 pi i m / N} come from a table of N values
// made once per (device, N) on the host and read through the caches.
//
// theta_interp: one wave per query, the barycentric form of the
// trigonometric interpolant (no transform): with theta = theta_i0 + delta,
//   a(theta) = sin(N delta / 2) / N * sum_i (-1)^d a_i g(delta / 2 + pi d / N),
// d = i0 - i reduced to [-N/2, N/2), g = cot for even N and 1 / sin for odd N.
#include <math.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "ms_internal.hpp"

namespace ms {
namespace {

constexpr int SP_THREADS = 256;
constexpr int SP_MAX_LOG2 = 11;   // n_theta <= 2048: 2 x 36 KiB of LDS per row
constexpr double SP_PI = 3.141592653589793238462643383279502884;
#ifndef SP_RADIX
#define SP_RADIX 8                // largest radix of a pass (4 or 8)
#endif
#ifndef SP_PAD_SHIFT
#define SP_PAD_SHIFT 3            // one pad slot per 2^SP_PAD_SHIFT LDS elements (0: none)
#endif

// LDS slot of element i: padded so that the strided writes of the first
// passes (stride R elements) spread over the banks.
MS_D int pslot(int i) { return SP_PAD_SHIFT ? i + (i >> SP_PAD_SHIFT) : i; }
template <int N>
constexpr int padded_size() { return SP_PAD_SHIFT ? N + (N >> SP_PAD_SHIFT) : N; }

MS_D double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

MS_D double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
MS_D double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// Multiplication by -i (forward) or +i (inverse).
template <bool INV>
MS_D double2 mul_mi(double2 b)
{
    return INV ? make_double2(-b.y, b.x) : make_double2(b.y, -b.x);
}

// 4-point DFT of (a, b, c, d) in place.
template <bool INV>
MS_D void dft4(double2 &a, double2 &b, double2 &c, double2 &d)
{
    double2 a0 = cadd(a, c), a1 = csub(a, c);
    double2 b0 = cadd(b, d), b1 = mul_mi<INV>(csub(b, d));
    a = cadd(a0, b0);
    c = csub(a0, b0);
    b = cadd(a1, b1);
    d = csub(a1, b1);
}

// R-point DFT in place (R = 2, 4 or 8); INV selects the sign of the exponent.
template <int R, bool INV>
MS_D void small_dft(double2 *v)
{
    if constexpr (R == 2) {
        double2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 4) {
        dft4<INV>(v[0], v[1], v[2], v[3]);
    } else {
        // even and odd halves, then X[k] = E[k] + w^k O[k], X[k+4] = E[k] - w^k O[k],
        // w = e^{-+i pi / 4}
        double2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
        double2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
        dft4<INV>(e0, e1, e2, e3);
        dft4<INV>(o0, o1, o2, o3);
        const double h = 0.70710678118654752440084436210484903928;
        // w o1, w^2 o2 = -+i o2, w^3 o3
        double2 t1 = INV ? make_double2((o1.x - o1.y) * h, (o1.x + o1.y) * h)
                         : make_double2((o1.x + o1.y) * h, (o1.y - o1.x) * h);
        double2 t2 = mul_mi<INV>(o2);
        double2 t3 = INV ? make_double2(-(o3.x + o3.y) * h, (o3.x - o3.y) * h)
                         : make_double2((o3.y - o3.x) * h, -(o3.x + o3.y) * h);
        v[0] = cadd(e0, o0);
        v[4] = csub(e0, o0);
        v[1] = cadd(e1, t1);
        v[5] = csub(e1, t1);
        v[2] = cadd(e2, t2);
        v[6] = csub(e2, t2);
        v[3] = cadd(e3, t3);
        v[7] = csub(e3, t3);
    }
}

// Radix of pass p of the forward transform: SP_RADIX while it fits, then 4
// or 2 for the remaining factor.  The inverse transform runs the same radices
// in reverse order, so that its first pass takes exactly the values the last
// forward pass leaves in each thread's registers.
template <int LOGN>
struct Plan {
    static constexpr int LR = SP_RADIX == 8 ? 3 : 2;
    static constexpr int FULL = LOGN / LR;
    static constexpr int REST = LOGN % LR;
    static constexpr int NP = FULL + (REST ? 1 : 0);
    static constexpr int radix(int p) { return p < FULL ? SP_RADIX : (REST == 2 ? 4 : 2); }
    // sub-transform length Ns before forward pass p
    static constexpr int ns_fwd(int p) { return p == 0 ? 1 : ns_fwd(p - 1) * radix(p - 1); }
    static constexpr int radix_inv(int p) { return radix(NP - 1 - p); }
    static constexpr int ns_inv(int p) { return p == 0 ? 1 : ns_inv(p - 1) * radix_inv(p - 1); }
};

// Where a pass takes its inputs from and puts its outputs.
enum { FROM_LDS = 0, FROM_GLOBAL = 1 };

// Stockham pass of radix R, sub-transform length Ns, over both sequences.
// Butterfly j takes element j + r N/R (r = 0..R-1), twiddles it by
// e^{-+2 pi i r (j mod Ns) / (Ns R)} (entry r (j mod Ns) N / (Ns R) of the
// table, conjugated for the inverse), transforms, and gives element
// (j / Ns) Ns R + (j mod Ns) + r Ns.  Inputs come from LDS or, for the first
// forward pass, from the row in global memory; outputs go to LDS or, for the
// last inverse pass, to global memory scaled by 1/N.  With MID the pass is
// the last forward pass fused with the spectral multiplier and the first
// inverse pass (radix R, Ns = 1).  One thread carries both sequences of its
// butterflies, so vertices move between global memory and registers whole.
template <int N, int R, int Ns, bool INV, int SRC, bool TO_GLOBAL, bool MID>
MS_D void pass(double2 (*z)[padded_size<N>()], const double2 *__restrict__ tw, const double *src, double *dst,
               double rho, int order)
{
    constexpr int NB = N / R;
    constexpr int PER = (NB + SP_THREADS - 1) / SP_THREADS;
    double2 v[2][PER][R];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = threadIdx.x + q * SP_THREADS;
        if (NB % SP_THREADS == 0 || j < NB) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int e = j + r * NB;
                if constexpr (SRC == FROM_GLOBAL) {
                    d4 w = load_d4(src + 4 * e);
                    v[0][q][r] = make_double2(w.x, w.y);
                    v[1][q][r] = make_double2(w.z, w.w);
                } else {
                    v[0][q][r] = z[0][pslot(e)];
                    v[1][q][r] = z[1][pslot(e)];
                }
            }
            const int k = j % Ns;
            if (k != 0) {
                constexpr int stride = N / (Ns * R);
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
            if constexpr (MID) {
                // here Ns = N / R, so the outputs are the coefficients k = j + r N/R
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int kk = j + r * NB;
                    double2 m;
                    if (2 * kk == N) {
                        // the cosine mode: Re[(j N/2)^order e^{j (N/2) rho}]
                        const double h = 0.5 * (double)N;
                        double sn, cs;
                        sincos(h * rho, &sn, &cs);
                        m = make_double2(order == 0 ? cs : order == 1 ? -h * sn : -h * h * cs, 0.0);
                    } else {
                        const double ks = 2 * kk > N ? (double)(kk - N) : (double)kk;
                        double sn, cs;
                        sincos(ks * rho, &sn, &cs);
                        m = make_double2(cs, sn);
                        if (order == 1) m = make_double2(-ks * sn, ks * cs);
                        else if (order == 2) m = make_double2(-ks * ks * cs, -ks * ks * sn);
                    }
                    v[0][q][r] = cmul(v[0][q][r], m);
                    v[1][q][r] = cmul(v[1][q][r], m);
                }
                // first inverse pass: the same butterfly j, Ns = 1, no twiddles
#pragma unroll
                for (int s = 0; s < 2; ++s) small_dft<R, true>(v[s][q]);
            }
        }
    }
    // outputs of the fused pass follow the first inverse pass (Ns = 1)
    constexpr int ns_out = MID ? 1 : Ns;
    if constexpr (SRC == FROM_LDS && !TO_GLOBAL) __syncthreads();   // all reads before any write
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = threadIdx.x + q * SP_THREADS;
        if (NB % SP_THREADS == 0 || j < NB) {
            const int base = (j / ns_out) * ns_out * R + j % ns_out;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int e = base + r * ns_out;
                if constexpr (TO_GLOBAL) {
                    const double inv = 1.0 / (double)N;
                    double2 *o = reinterpret_cast<double2 *>(dst + 4 * e);
                    o[0] = make_double2(v[0][q][r].x * inv, v[0][q][r].y * inv);
                    o[1] = make_double2(v[1][q][r].x * inv, v[1][q][r].y * inv);
                } else {
                    z[0][pslot(e)] = v[0][q][r];
                    z[1][pslot(e)] = v[1][q][r];
                }
            }
        }
    }
    if constexpr (!TO_GLOBAL) __syncthreads();
}

template <int LOGN, int P>
MS_D void forward_passes(double2 (*z)[padded_size<1 << LOGN>()], const double2 *tw, const double *src)
{
    using PL = Plan<LOGN>;
    if constexpr (P < PL::NP - 1) {
        constexpr int N = 1 << LOGN;
        constexpr int NS = PL::ns_fwd(P);
        pass<N, PL::radix(P), NS, false, P == 0 ? FROM_GLOBAL : FROM_LDS, false, false>(z, tw, src, nullptr, 0.0, 0);
        forward_passes<LOGN, P + 1>(z, tw, src);
    }
}

template <int LOGN, int P>
MS_D void inverse_passes(double2 (*z)[padded_size<1 << LOGN>()], const double2 *tw, double *dst)
{
    using PL = Plan<LOGN>;
    if constexpr (P < PL::NP) {
        constexpr int N = 1 << LOGN;
        constexpr int NS = PL::ns_inv(P);
        pass<N, PL::radix_inv(P), NS, true, FROM_LDS, P == PL::NP - 1, false>(z, tw, nullptr, dst, 0.0, 0);
        inverse_passes<LOGN, P + 1>(z, tw, dst);
    }
}

// row_map (optional): output row of each input row; a negative entry drops
// the row.
template <int LOGN>
__global__ void __launch_bounds__(SP_THREADS) k_theta_shift(const double *in, double *out,
                                                            const double2 *__restrict__ tw, const double *rho_dev,
                                                            double rho, int order, const int64_t *row_map)
{
    using PL = Plan<LOGN>;
    constexpr int N = 1 << LOGN;
    __shared__ double2 z[2][padded_size<N>()];
    const int64_t row = blockIdx.x;
    const int64_t orow = row_map ? row_map[row] : row;
    if (orow < 0) return;   // the whole block
    const double *src = in + row * (int64_t)N * 4;
    double *dst = out + orow * (int64_t)N * 4;
    const double r = rho_dev ? rho_dev[row] : rho;
    forward_passes<LOGN, 0>(z, tw, src);
    // last forward pass + multiplier + first inverse pass, in registers
    constexpr int PM = PL::NP - 1;
    constexpr int NSM = PL::ns_fwd(PM);
    pass<N, PL::radix(PM), NSM, false, PM == 0 ? FROM_GLOBAL : FROM_LDS, PL::NP == 1, true>(z, tw, src, dst, r,
                                                                                            order);
    inverse_passes<LOGN, 1>(z, tw, dst);
}

// Forward transform only: out(r, j) = (Z0(j), Z1(j)) / N in natural order,
// four doubles per frequency (Re Z0, Im Z0, Re Z1, Im Z1), the layout of the
// input rows.
template <int LOGN>
__global__ void __launch_bounds__(SP_THREADS) k_theta_spectrum(const double *in, double *out,
                                                               const double2 *__restrict__ tw)
{
    using PL = Plan<LOGN>;
    constexpr int N = 1 << LOGN;
    __shared__ double2 z[2][padded_size<N>()];
    const int64_t row = blockIdx.x;
    const double *src = in + row * (int64_t)N * 4;
    double *dst = out + row * (int64_t)N * 4;
    forward_passes<LOGN, 0>(z, tw, src);
    constexpr int PM = PL::NP - 1;
    constexpr int NSM = PL::ns_fwd(PM);
    // the last forward pass (Ns = N / R) writes coefficient j + r N/R of butterfly j
    pass<N, PL::radix(PM), NSM, false, PM == 0 ? FROM_GLOBAL : FROM_LDS, true, false>(z, tw, src, dst, 0.0, 0);
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
    if (!isfinite(i0f)) {       // |theta| beyond any meaningful angle: no index to take
        if (lane < 4) o[lane] = NAN;
        return;
    }
    const double delta = th - i0f * step;
    int64_t i0 = (int64_t)fmod(i0f, (double)N);   // exact, in (-N, N)
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
                  double rho, int order, hipStream_t st, const int64_t *row_map = nullptr)
{
    hipLaunchKernelGGL(k_theta_shift<LOGN>, dim3((unsigned)n_rows), dim3(SP_THREADS), 0, st, in, out, tw, rho_dev,
                       rho, order, row_map);
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

template <int LOGN>
void launch_spectrum(const double *in, double *out, const double2 *tw, int64_t n_rows, hipStream_t st)
{
    hipLaunchKernelGGL(k_theta_spectrum<LOGN>, dim3((unsigned)n_rows), dim3(SP_THREADS), 0, st, in, out, tw);
}

// theta_shift on validated arguments (n_theta a power of two in range).
int shift_rows(const double *in, double *out, int n_theta, int64_t n_rows, const double *rho_dev, double rho,
               int order, const int64_t *row_map, hipStream_t st)
{
    const double2 *tw = nullptr;
    int rc = twiddles(n_theta, &tw);
    if (rc) return rc;
    int lg = 0;
    while ((1 << lg) < n_theta) ++lg;
    switch (lg) {
    case 1: launch_shift<1>(in, out, tw, n_rows, rho_dev, rho, order, st, row_map); break;
    case 2: launch_shift<2>(in, out, tw, n_rows, rho_dev, rho, order, st, row_map); break;
    case 3: launch_shift<3>(in, out, tw, n_rows, rho_dev, rho, order, st, row_map); break;
    case 4: launch_shift<4>(in, out, tw, n_rows, rho_dev, rho, order, st, row_map); break;
    case 5: launch_shift<5>(in, out, tw, n_rows, rho_dev, rho, order, st, row_map); break;
    case 6: launch_shift<6>(in, out, tw, n_rows, rho_dev, rho, order, st, row_map); break;
    case 7: launch_shift<7>(in, out, tw, n_rows, rho_dev, rho, order, st, row_map); break;
    case 8: launch_shift<8>(in, out, tw, n_rows, rho_dev, rho, order, st, row_map); break;
    case 9: launch_shift<9>(in, out, tw, n_rows, rho_dev, rho, order, st, row_map); break;
    case 10: launch_shift<10>(in, out, tw, n_rows, rho_dev, rho, order, st, row_map); break;
    default: launch_shift<11>(in, out, tw, n_rows, rho_dev, rho, order, st, row_map); break;
    }
    MS_HIP(hipGetLastError());
    return MS_OK;
}

// Row copies through a row map (negative entries dropped): the unshifted
// layer of the globalized mesh.
__global__ void __launch_bounds__(256) k_copy_rows(const double *in, double *out, const int64_t *row_map,
                                                   int64_t n_rows, int N)
{
    const int64_t per = (int64_t)N * 2;   // double2 per row
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_rows * per) return;
    const int64_t row = i / per, e = i - row * per;
    const int64_t orow = row_map[row];
    if (orow < 0) return;
    reinterpret_cast<double2 *>(out)[orow * per + e] = reinterpret_cast<const double2 *>(in)[i];
}

}  // namespace
}  // namespace ms

using namespace ms;

extern "C" int globalize_workspace_size(int32_t n_theta, int32_t n_s, int32_t n_max, size_t *bytes)
{
    if (!bytes || n_theta < 1 || n_s < 0 || n_max < 0) return fail(MS_E_ARG, "globalize_workspace_size: bad argument");
    const size_t grid = (size_t)n_s * n_theta * 32;
    const size_t map = (size_t)(n_max + 1) * n_s * 8;
    *bytes = ((grid + 255) & ~(size_t)255) + ((map + 255) & ~(size_t)255);
    return MS_OK;
}

extern "C" int globalize_manifold(const double *grid_dev, const double *s_host, int32_t n_theta, int32_t n_s,
                                  int32_t n_max, double omega, double lambda, const map_params_t *map,
                                  double *out_dev, int64_t out_rows_cap, double *s_out_host, int64_t *n_rows_out,
                                  void *ws, size_t ws_bytes, void *stream)
{
    if (!s_host || !map || !n_rows_out || n_s < 1 || n_max < 0 || (!grid_dev) || (!s_out_host))
        return fail(MS_E_ARG, "globalize_manifold: bad argument");
    if (n_theta < 2 || n_theta > (1 << SP_MAX_LOG2) || (n_theta & (n_theta - 1)))
        return fail(MS_E_ARG, "globalize_manifold: n_theta must be a power of two in [2, 2048]");
    if (map->n_periods != 1 && map->n_periods != -1)
        return fail(MS_E_ARG, "globalize_manifold: map->n_periods must be +1 (unstable) or -1 (stable)");
    if (!(lambda > 0.0) || !isfinite(lambda) || !isfinite(omega))
        return fail(MS_E_ARG, "globalize_manifold: need lambda > 0 and a finite omega");
    for (int k = 0; k < n_s; ++k)
        if (!isfinite(s_host[k]) || (k > 0 && !(s_host[k] > s_host[k - 1])))
            return fail(MS_E_ARG, "globalize_manifold: s must be finite and strictly increasing");
    const int d = map->n_periods;
    // the rows (n, k) and their s values, sorted by s (s = 0 kept once)
    struct Entry { double s; int n, k; };
    std::vector<Entry> ent;
    for (int n = 0; n <= n_max; ++n)
        for (int k = 0; k < n_s; ++k) {
            if (n > 0 && s_host[k] == 0.0) continue;
            ent.push_back({pow(lambda, (double)(d * n)) * s_host[k], n, k});
        }
    std::stable_sort(ent.begin(), ent.end(), [](const Entry &a, const Entry &b) { return a.s < b.s; });
    const int64_t M = (int64_t)ent.size();
    *n_rows_out = M;
    if (!out_dev || out_rows_cap < M) return fail(MS_E_CAPACITY, "globalize_manifold: output holds too few rows");
    size_t need = 0;
    int rc = globalize_workspace_size(n_theta, n_s, n_max, &need);
    if (rc) return rc;
    if (!ws || ws_bytes < need) return fail(MS_E_WORKSPACE, "globalize_manifold: workspace too small");
    std::vector<int64_t> rmap((size_t)(n_max + 1) * n_s, -1);
    for (int64_t r = 0; r < M; ++r) {
        rmap[(size_t)ent[r].n * n_s + ent[r].k] = r;
        s_out_host[r] = ent[r].s;
    }
    double *P = (double *)ws;
    int64_t *rmap_dev = (int64_t *)((char *)ws + (((size_t)n_s * n_theta * 32 + 255) & ~(size_t)255));
    hipStream_t st = (hipStream_t)stream;
    MS_HIP(hipMemcpyAsync(rmap_dev, rmap.data(), rmap.size() * 8, hipMemcpyHostToDevice, st));
    MS_HIP(hipStreamSynchronize(st));   // rmap is a host vector of this call
    const int64_t n_states = (int64_t)n_s * n_theta;
    hipLaunchKernelGGL(k_copy_rows, dim3((unsigned)ceil_div(n_states * 2, 256)), dim3(256), 0, st, grid_dev, out_dev,
                       rmap_dev, (int64_t)n_s, (int)n_theta);
    MS_HIP(hipGetLastError());
    if (n_max > 0) MS_HIP(hipMemcpyAsync(P, grid_dev, (size_t)n_states * 32, hipMemcpyDeviceToDevice, st));
    for (int n = 1; n <= n_max; ++n) {
        // P <- F^d(P) = F^(d n)(grid), then W(theta_i, lambda^(d n) s_k) = P shifted by -d n omega
        if ((rc = pertbp_map(P, P, n_states, map, stream))) return rc;
        if ((rc = shift_rows(P, out_dev, n_theta, n_s, nullptr, -(double)(d * n) * omega, 0,
                             rmap_dev + (size_t)n * n_s, st)))
            return rc;
    }
    return MS_OK;
}

extern "C" int theta_spectrum(const double *in_dev, double *out_dev, int32_t n_theta, int64_t n_rows, void *stream)
{
    if (n_rows < 0 || (n_rows > 0 && (!in_dev || !out_dev))) return fail(MS_E_ARG, "theta_spectrum: bad argument");
    if (n_theta < 2 || n_theta > (1 << SP_MAX_LOG2) || (n_theta & (n_theta - 1)))
        return fail(MS_E_ARG, "theta_spectrum: n_theta must be a power of two in [2, 2048]");
    if (n_rows > 0x7fffffff) return fail(MS_E_ARG, "theta_spectrum: too many rows for one launch");
    if (n_rows == 0) return MS_OK;
    hipStream_t st = (hipStream_t)stream;
    const double2 *tw = nullptr;
    int rc = twiddles(n_theta, &tw);
    if (rc) return rc;
    int lg = 0;
    while ((1 << lg) < n_theta) ++lg;
    switch (lg) {
    case 1: launch_spectrum<1>(in_dev, out_dev, tw, n_rows, st); break;
    case 2: launch_spectrum<2>(in_dev, out_dev, tw, n_rows, st); break;
    case 3: launch_spectrum<3>(in_dev, out_dev, tw, n_rows, st); break;
    case 4: launch_spectrum<4>(in_dev, out_dev, tw, n_rows, st); break;
    case 5: launch_spectrum<5>(in_dev, out_dev, tw, n_rows, st); break;
    case 6: launch_spectrum<6>(in_dev, out_dev, tw, n_rows, st); break;
    case 7: launch_spectrum<7>(in_dev, out_dev, tw, n_rows, st); break;
    case 8: launch_spectrum<8>(in_dev, out_dev, tw, n_rows, st); break;
    case 9: launch_spectrum<9>(in_dev, out_dev, tw, n_rows, st); break;
    case 10: launch_spectrum<10>(in_dev, out_dev, tw, n_rows, st); break;
    default: launch_spectrum<11>(in_dev, out_dev, tw, n_rows, st); break;
    }
    MS_HIP(hipGetLastError());
    return MS_OK;
}

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
    return shift_rows(in_dev, out_dev, n_theta, n_rows, rho_dev, rho, order, nullptr, (hipStream_t)stream);
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
