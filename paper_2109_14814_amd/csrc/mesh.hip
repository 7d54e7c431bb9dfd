// mesh.hip -- mesh handles: triangulation of a vertex grid (Sec. 6.1), the
// mesh statistics used to plan a grid (bounds, mean triangle diameter), and
// error reporting of the ABI.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "ms_internal.hpp"

namespace ms {

static thread_local std::string g_err = "no error";

void set_error(const std::string &msg) { g_err = msg; }

int fail(int code, const std::string &msg)
{
    set_error(msg);
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    char buf[512];
    snprintf(buf, sizeof buf, "HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
    set_error(buf);
    return MS_E_HIP;
}

namespace {

constexpr int MB_BLOCK = 256;
constexpr int MB_GRID = 1024;

// SoA planes -> AoS vertices.
__global__ void __launch_bounds__(MB_BLOCK) k_soa_to_aos(const double *soa, double *aos, int64_t nv)
{
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += stride) {
        double2 a = make_double2(soa[v], soa[nv + v]);
        double2 b = make_double2(soa[2 * nv + v], soa[3 * nv + v]);
        double2 *o = reinterpret_cast<double2 *>(aos + 4 * v);
        o[0] = a;
        o[1] = b;
    }
}

// Statistics of a mesh for grid planning: bounds of the finite triangles'
// vertices, the sum of their longest 4D edges and the counts of finite and
// non-finite triangles, as per-block partials.  (The boxes themselves are
// never stored: the search recomputes them from the vertices.)
struct Partial {
    double lo[4], hi[4];
    double diam_sum;
    long long n_fin_tris, n_bad_tris;
    long long pad;
};

__global__ void __launch_bounds__(MB_BLOCK) k_mesh_stats(MeshView m, Partial *part)
{
    __shared__ double s_lo[4][MB_BLOCK / WAVE], s_hi[4][MB_BLOCK / WAVE], s_sum[MB_BLOCK / WAVE];
    __shared__ long long s_fin[MB_BLOCK / WAVE], s_bad[MB_BLOCK / WAVE];
    double lo[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
    double hi[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
    double dsum = 0.0;
    long long nfin = 0, nbad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m.n_tris; t += stride) {
        int32_t i1, i2, i3;
        tri_vertex_ids(m, (int32_t)t, i1, i2, i3);
        d4 p1 = load_d4(m.V + 4 * (int64_t)i1), p2 = load_d4(m.V + 4 * (int64_t)i2), p3 = load_d4(m.V + 4 * (int64_t)i3);
        double a[3][4] = {{p1.x, p1.y, p1.z, p1.w}, {p2.x, p2.y, p2.z, p2.w}, {p3.x, p3.y, p3.z, p3.w}};
        bool fin = true;
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int d = 0; d < 4; ++d) fin = fin && isfinite(a[j][d]);
        if (fin) {
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                double l = a[0][d], h = a[0][d];
                if (a[1][d] < l) l = a[1][d];
                if (a[2][d] < l) l = a[2][d];
                if (a[1][d] > h) h = a[1][d];
                if (a[2][d] > h) h = a[2][d];
                lo[d] = fmin(lo[d], l);
                hi[d] = fmax(hi[d], h);
            }
            double e = 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double *x = a[j], *y = a[(j + 1) % 3];
                double sq = 0.0;
#pragma unroll
                for (int d = 0; d < 4; ++d) sq += (x[d] - y[d]) * (x[d] - y[d]);
                e = fmax(e, sq);
            }
            dsum += sqrt(e);
            ++nfin;
        } else {
            ++nbad;
        }
    }
    // wave then block reductions
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            lo[d] = fmin(lo[d], __shfl_xor(lo[d], o));
            hi[d] = fmax(hi[d], __shfl_xor(hi[d], o));
        }
        dsum += __shfl_xor(dsum, o);
        nfin += __shfl_xor(nfin, o);
        nbad += __shfl_xor(nbad, o);
    }
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        for (int d = 0; d < 4; ++d) { s_lo[d][w] = lo[d]; s_hi[d][w] = hi[d]; }
        s_sum[w] = dsum; s_fin[w] = nfin; s_bad[w] = nbad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Partial p;
        for (int d = 0; d < 4; ++d) {
            p.lo[d] = s_lo[d][0]; p.hi[d] = s_hi[d][0];
            for (int i = 1; i < MB_BLOCK / WAVE; ++i) { p.lo[d] = fmin(p.lo[d], s_lo[d][i]); p.hi[d] = fmax(p.hi[d], s_hi[d][i]); }
        }
        p.diam_sum = 0; p.n_fin_tris = 0; p.n_bad_tris = 0; p.pad = 0;
        for (int i = 0; i < MB_BLOCK / WAVE; ++i) { p.diam_sum += s_sum[i]; p.n_fin_tris += s_fin[i]; p.n_bad_tris += s_bad[i]; }
        part[blockIdx.x] = p;
    }
}

}  // namespace
}  // namespace ms


namespace ms {
namespace {

// Statistics pass of mesh m on stream st, then the host reduction of its
// per-block partials (synchronises st).
int reduce_info(ms_mesh *m)
{
    if (!m->info_stale) return MS_OK;
    const MeshView &mv = m->view;
    hipStream_t st = m->upd_stream;
    int64_t g = ceil_div(mv.n_tris > 0 ? mv.n_tris : 1, MB_BLOCK);
    if (g > MB_GRID) g = MB_GRID;
    MS_LAUNCH("k_mesh_stats", k_mesh_stats, dim3((unsigned)g), dim3(MB_BLOCK), 0, st, mv, (Partial *)m->scratch);
    MS_HIP(hipGetLastError());
    std::vector<Partial> hp((size_t)g);
    MS_HIP(hipMemcpyAsync(hp.data(), m->scratch, hp.size() * sizeof(Partial), hipMemcpyDeviceToHost, st));
    MS_HIP(hipStreamSynchronize(st));
    ms_mesh_info_t &inf = m->info;
    inf.n_tris = m->view.n_tris;
    for (int d = 0; d < 4; ++d) { inf.lo[d] = INFINITY; inf.hi[d] = -INFINITY; }
    double dsum = 0.0;
    long long nfin = 0, nbad = 0;
    for (const Partial &p : hp) {
        for (int d = 0; d < 4; ++d) { inf.lo[d] = fmin(inf.lo[d], p.lo[d]); inf.hi[d] = fmax(inf.hi[d], p.hi[d]); }
        dsum += p.diam_sum;
        nfin += p.n_fin_tris;
        nbad += p.n_bad_tris;
    }
    inf.n_nonfinite = nbad;
    inf.mean_diam = nfin > 0 ? dsum / (double)nfin : 0.0;
    m->info_stale = 0;
    return MS_OK;
}

}  // namespace
}  // namespace ms

using namespace ms;

extern "C" const char *last_error(void) { return g_err.c_str(); }

extern "C" int mesh_build(const double *verts_dev, int32_t n_theta_v, int32_t n_s_v, int32_t periodic, int32_t layout,
                          const double *theta_host, const double *s_host, void *stream, ms_mesh **out)
{
    if (!out) return fail(MS_E_ARG, "mesh_build: out is NULL");
    *out = nullptr;
    if (n_theta_v < 0 || n_s_v < 0) return fail(MS_E_ARG, "mesh_build: negative grid size");
    if (layout != MS_LAYOUT_AOS && layout != MS_LAYOUT_SOA) return fail(MS_E_ARG, "mesh_build: unknown layout");
    int64_t nv = (int64_t)n_theta_v * n_s_v;
    if (nv > 0 && (!verts_dev || !theta_host || !s_host)) return fail(MS_E_ARG, "mesh_build: NULL vertex/sample array");
    int64_t nq = n_theta_v <= 0 ? 0 : (periodic ? n_theta_v : n_theta_v - 1);
    int64_t ntri = (nq > 0 && n_s_v > 1) ? 2 * nq * (n_s_v - 1) : 0;
    if (ntri > (int64_t)0x7fffffff || nv > (int64_t)0x7fffffff / 4)
        return fail(MS_E_ARG, "mesh_build: more than 2^31 triangles or 2^29 vertices");
    hipStream_t st = (hipStream_t)stream;

    ms_mesh *m = new ms_mesh();
    memset(m, 0, sizeof *m);
    auto cleanup = [&](int rc) {
        mesh_free(m);
        return rc;
    };
    {
        hipError_t e = hipGetDevice(&m->device);
        if (e != hipSuccess) return cleanup(hip_fail(e, "hipGetDevice"));
    }
    const double *V = verts_dev;
    hipError_t e;
    if (layout == MS_LAYOUT_SOA && nv > 0) {
        if ((e = hipMalloc(&m->owned_V, (size_t)nv * 32)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc verts"));
        int64_t g = ceil_div(nv, MB_BLOCK);
        if (g > 4096) g = 4096;
        hipLaunchKernelGGL(k_soa_to_aos, dim3((unsigned)g), dim3(MB_BLOCK), 0, st, verts_dev, m->owned_V, nv);
        V = m->owned_V;
        m->soa_src = verts_dev;
    }
    m->n_verts = nv;
    if ((e = hipMalloc(&m->theta_dev, (size_t)(n_theta_v > 0 ? n_theta_v : 1) * 8)) != hipSuccess)
        return cleanup(hip_fail(e, "hipMalloc theta"));
    if ((e = hipMalloc(&m->s_dev, (size_t)(n_s_v > 0 ? n_s_v : 1) * 8)) != hipSuccess)
        return cleanup(hip_fail(e, "hipMalloc s"));
    if ((e = hipMalloc(&m->scratch, (size_t)(MB_GRID * sizeof(Partial) + MS_COUNT_PARTIALS * 8 + 256))) != hipSuccess)
        return cleanup(hip_fail(e, "hipMalloc scratch"));
    m->counter = (int64_t *)((char *)m->scratch + MB_GRID * sizeof(Partial));
    if (n_theta_v > 0 && (e = hipMemcpyAsync(m->theta_dev, theta_host, (size_t)n_theta_v * 8, hipMemcpyHostToDevice, st)) != hipSuccess)
        return cleanup(hip_fail(e, "copy theta"));
    if (n_s_v > 0 && (e = hipMemcpyAsync(m->s_dev, s_host, (size_t)n_s_v * 8, hipMemcpyHostToDevice, st)) != hipSuccess)
        return cleanup(hip_fail(e, "copy s"));

    MeshView &mv = m->view;
    mv.V = V;
    mv.theta = m->theta_dev;
    mv.s = m->s_dev;
    mv.n_theta_v = n_theta_v;
    mv.n_s_v = n_s_v;
    mv.nq = (int32_t)nq;
    mv.periodic = periodic ? 1 : 0;
    mv.n_tris = (int32_t)ntri;
    mv.inv_nq = nq > 0 ? 1.0 / (double)nq : 0.0;

    m->upd_stream = st;
    m->info_stale = 1;
    int rc = reduce_info(m);
    if (rc) return cleanup(rc);
    *out = m;
    return MS_OK;
}

extern "C" int mesh_free(ms_mesh *m)
{
    if (!m) return MS_OK;
    if (m->owned_V) (void)hipFree(m->owned_V);
    if (m->theta_dev) (void)hipFree(m->theta_dev);
    if (m->s_dev) (void)hipFree(m->s_dev);
    if (m->scratch) (void)hipFree(m->scratch);
    delete m;
    return MS_OK;
}

extern "C" int mesh_update(ms_mesh *m, void *stream)
{
    if (!m) return fail(MS_E_ARG, "mesh_update: NULL mesh");
    m->upd_stream = (hipStream_t)stream;
    m->info_stale = 1;
    if (m->soa_src && m->n_verts > 0) {
        // an SoA mesh searches its own AoS copy: convert the changed planes again
        int64_t g = ceil_div(m->n_verts, MB_BLOCK);
        if (g > 4096) g = 4096;
        hipLaunchKernelGGL(k_soa_to_aos, dim3((unsigned)g), dim3(MB_BLOCK), 0, m->upd_stream, m->soa_src, m->owned_V,
                           m->n_verts);
        MS_HIP(hipGetLastError());
    }
    return MS_OK;
}

extern "C" int mesh_info(const ms_mesh *m, ms_mesh_info_t *out)
{
    if (!m || !out) return fail(MS_E_ARG, "mesh_info: NULL argument");
    int rc = reduce_info(const_cast<ms_mesh *>(m));
    if (rc) return rc;
    *out = m->info;
    return MS_OK;
}

extern "C" int search_default_params(const ms_mesh *A, const ms_mesh *B, double kappa, search_params_t *out)
{
    if (!A || !B || !out) return fail(MS_E_ARG, "search_default_params: NULL argument");
    if (!(kappa > 0.0) || !isfinite(kappa)) return fail(MS_E_ARG, "search_default_params: kappa must be > 0");
    memset(out, 0, sizeof *out);
    int rc;
    if ((rc = reduce_info(const_cast<ms_mesh *>(A))) || (rc = reduce_info(const_cast<ms_mesh *>(B)))) return rc;
    double lo[4], hi[4];
    for (int d = 0; d < 4; ++d) {
        lo[d] = fmin(A->info.lo[d], B->info.lo[d]);
        hi[d] = fmax(A->info.hi[d], B->info.hi[d]);
    }
    // the geometric mean of the two meshes' mean triangle diameters: for
    // meshes of unequal resolution, a cell between the two sizes keeps the
    // coarse mesh's triangles to a few cells each and the fine mesh's cells
    // to a few of its triangles per coarse triangle
    int64_t na = A->info.n_tris - A->info.n_nonfinite, nb = B->info.n_tris - B->info.n_nonfinite;
    const double dA = A->info.mean_diam, dB = B->info.mean_diam;
    double diam = (na > 0 && nb > 0) ? sqrt(dA * dB) : (na > 0 ? dA : (nb > 0 ? dB : 0.0));
    double edge = kappa * diam;
    bool empty = !(lo[0] <= hi[0]);
    if (!(edge > 0.0) || !isfinite(edge)) edge = 1.0;
    out->inv_edge = 1.0 / edge;
    for (int d = 0; d < 4; ++d) {
        out->world_lo[d] = empty ? 0.0 : lo[d];
        double span = empty ? 0.0 : (hi[d] - lo[d]) * out->inv_edge;
        double c = ceil(span);
        out->n_cells[d] = c < 1.0 ? 1 : (c > 4.0e18 ? (int64_t)4e18 : (int64_t)c);
    }
    return MS_OK;
}
