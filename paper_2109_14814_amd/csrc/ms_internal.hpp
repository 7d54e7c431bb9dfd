// ms_internal.hpp -- internal definitions shared by the HIP sources of
// libmsearch.so (never installed; the public ABI is include/msearch.h).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "../../include/msearch.h"

#define MS_HD __host__ __device__ __forceinline__
#define MS_D __device__ __forceinline__

namespace ms {

constexpr int WAVE = 64;

// ----------------------------------------------------------------- errors

void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

#define MS_HIP(call)                                            \
    do {                                                        \
        hipError_t _e = (call);                                 \
        if (_e != hipSuccess) return ::ms::hip_fail(_e, #call); \
    } while (0)

// -------------------------------------------------------------- mesh view

// Device view of a triangulated vertex grid (see mesh_build in msearch.h).
struct MeshView {
    const double *V;       // AoS vertices, 4 doubles each, theta index fastest
    const double *theta;   // n_theta_v samples
    const double *s;       // n_s_v samples
    int32_t n_theta_v, n_s_v;
    int32_t nq;            // quads per s-row
    int32_t periodic;
    int32_t n_tris;
    int32_t pad;
    double inv_nq;         // 1 / nq (0 without quads): the row of a quad without an integer division
};

// Vertex ids (in the AoS array) of triangle t in narrow-phase order.
MS_HD void tri_vertex_ids(const MeshView &m, int32_t t, int32_t &v1, int32_t &v2, int32_t &v3)
{
    int32_t q = t >> 1;
    int32_t h = t & 1;
    int32_t k = q / m.nq;
    int32_t i = q - k * m.nq;
    int32_t i1 = i + 1;
    if (i1 == m.n_theta_v) i1 = 0;   // periodic wrap (i1 == n_theta_v only when periodic)
    int32_t r0 = k * m.n_theta_v, r1 = r0 + m.n_theta_v;
    if (h == 0) { v1 = r0 + i1; v2 = r0 + i;  v3 = r1 + i; }
    else        { v1 = r1 + i;  v2 = r1 + i1; v3 = r0 + i1; }
}

// Row k and column i of quad q = i + k * nq: the quotient from the FP64
// product q * (1 / nq), whose error is far below one for q < 2^31, corrected
// by one step.
MS_D void quad_row_col(const MeshView &m, int32_t q, int32_t &k, int32_t &i)
{
    int32_t kk = (int32_t)((double)q * m.inv_nq);
    int64_t r = (int64_t)q - (int64_t)kk * m.nq;
    if (r < 0) {
        --kk;
        r += m.nq;
    } else if (r >= m.nq) {
        ++kk;
        r -= m.nq;
    }
    k = kk;
    i = (int32_t)r;
}

// tri_vertex_ids with the row found by quad_row_col.
MS_D void tri_vertex_ids_d(const MeshView &m, int32_t t, int32_t &v1, int32_t &v2, int32_t &v3)
{
    int32_t k, i;
    quad_row_col(m, t >> 1, k, i);
    int32_t i1 = i + 1;
    if (i1 == m.n_theta_v) i1 = 0;
    const int32_t r0 = k * m.n_theta_v, r1 = r0 + m.n_theta_v;
    if ((t & 1) == 0) { v1 = r0 + i1; v2 = r0 + i;  v3 = r1 + i; }
    else              { v1 = r1 + i;  v2 = r1 + i1; v3 = r0 + i1; }
}

struct d4 { double x, y, z, w; };

MS_D d4 load_d4(const double *p)
{
    const double2 *q = reinterpret_cast<const double2 *>(p);
    double2 a = q[0], b = q[1];
    return d4{a.x, a.y, b.x, b.y};
}

// 4D box of triangle t (exact min / max per axis of its three vertices,
// Sec. 6.2.2), computed from the vertices wherever it is needed; false when a
// coordinate is not finite (such a triangle takes no part in a search).
MS_D bool tri_box(const MeshView &m, int32_t t, double lo[4], double hi[4])
{
    int32_t i1, i2, i3;
    tri_vertex_ids(m, t, i1, i2, i3);
    const d4 a = load_d4(m.V + 4 * (int64_t)i1), b = load_d4(m.V + 4 * (int64_t)i2),
             c = load_d4(m.V + 4 * (int64_t)i3);
    const double va[4] = {a.x, a.y, a.z, a.w}, vb[4] = {b.x, b.y, b.z, b.w}, vc[4] = {c.x, c.y, c.z, c.w};
    bool fin = true;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        double l = va[d], h = va[d];
        if (vb[d] < l) l = vb[d];
        if (vc[d] < l) l = vc[d];
        if (vb[d] > h) h = vb[d];
        if (vc[d] > h) h = vc[d];
        lo[d] = l;
        hi[d] = h;
        fin = fin && isfinite(va[d]) && isfinite(vb[d]) && isfinite(vc[d]);
    }
    return fin;
}

typedef double dvec2 __attribute__((ext_vector_type(2)));

// Streaming load (data read once): bypasses cache retention.
MS_D d4 load_d4_nt(const double *p)
{
    const dvec2 *q = reinterpret_cast<const dvec2 *>(p);
    dvec2 a = __builtin_nontemporal_load(q);
    dvec2 b = __builtin_nontemporal_load(q + 1);
    return d4{a.x, a.y, b.x, b.y};
}

// ------------------------------------------------------------ grid / keys

struct GridView {
    double wlo[4];
    double inv;
    int64_t n[4];
};

// Cell of coordinate x on one axis: clamp(floor((x - wlo) * inv), 0, n - 1),
// FP64, one rounding per operation (the kernels are built with contraction off).
MS_D int64_t cell_of(double x, double wlo, double inv, int64_t n)
{
    double t = (x - wlo) * inv;
    double f = floor(t);
    if (!(f >= 0.0)) return 0;
    if (f >= (double)n) return n - 1;
    int64_t c = (int64_t)f;
    return c < n ? c : n - 1;
}

MS_D int64_t cell_linear(const int64_t c[4], const int64_t n[4])
{
    return ((c[0] * n[1] + c[1]) * n[2] + c[2]) * n[3] + c[3];
}

// ------------------------------------------------------------- wave utils

MS_D uint64_t ballot(bool p) { return __ballot(p); }

MS_D int lane_id() { return __lane_id(); }

// Number of set bits of m below this lane.
MS_D int mbcnt(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

// Wave-aggregated slot reservation: every lane with `want` gets a distinct
// index in [base, base + popcount); one atomic per wave.
MS_D int64_t wave_reserve(bool want, unsigned long long *counter)
{
    uint64_t m = ballot(want);
    if (m == 0) return -1;
    int leader = __builtin_ctzll(m);
    unsigned long long base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, (unsigned long long)__builtin_popcountll(m));
    base = __shfl(base, leader);
    return want ? (int64_t)(base + (unsigned long long)mbcnt(m)) : -1;
}

MS_D unsigned long long wave_sum_u64(unsigned long long v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// ------------------------------------------------------------ search stats

enum StatIdx {
    ST_ENTRIES = 0, ST_ENTRIES_ALL, ST_CELLS, ST_SLOTS, ST_CAND, ST_MOLLER, ST_DEGEN,
    ST_OUTSIDE, ST_HITS, ST_NONFINITE, ST_OVERFLOW
};

MS_HD int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline int bits_for(uint64_t x)   // bits needed to store values 0..x
{
    int b = 0;
    while (b < 64 && (x >> b) != 0) ++b;
    return b;
}

// ------------------------------------------------------ internal sort API

// Sort of distinct 64-bit keys in two kernels: chunks of 4096 sorted in LDS,
// then every key placed by its rank in the other chunks (cost grows with
// n^2 / 4096; meant for small n such as hit lists).  n from device memory.
int sort_unique_small(const uint64_t *in, uint64_t *tmp, uint64_t *out, const int64_t *n_dev, int64_t cap,
                      int lo_bit, int n_bits, hipStream_t st);   // n = min(*n_dev, cap)

// ------------------------------------------------------------- profiling

// Kernel timing for benchmarks.  While enabled (search_profile_enable),
// prof_pair hands out a start / stop event pair for the next kernel of an
// uncaptured stream; MS_LAUNCH then launches that kernel with
// hipExtLaunchKernelGGL, so the two events carry the dispatch's own start and
// end timestamps.  Otherwise MS_LAUNCH is a plain launch.
bool prof_pair(const char *name, hipStream_t st, hipEvent_t *start, hipEvent_t *stop);

#define MS_LAUNCH(NAME, KERNEL, GRID, BLOCKDIM, SHMEM, STREAM, ...)                                          \
    do {                                                                                                     \
        hipEvent_t ms_e0_, ms_e1_;                                                                           \
        if (::ms::prof_pair(NAME, STREAM, &ms_e0_, &ms_e1_))                                                 \
            hipExtLaunchKernelGGL(KERNEL, GRID, BLOCKDIM, SHMEM, STREAM, ms_e0_, ms_e1_, 0, __VA_ARGS__);     \
        else                                                                                                 \
            hipLaunchKernelGGL(KERNEL, GRID, BLOCKDIM, SHMEM, STREAM, __VA_ARGS__);                          \
    } while (0)

}  // namespace ms

constexpr int MS_COUNT_PARTIALS = 2048;

// The opaque handle of the public ABI.
struct ms_mesh {
    ms::MeshView view;
    double *owned_V;          // AoS copy for MS_LAYOUT_SOA
    const double *soa_src;    // the caller's SoA planes (MS_LAYOUT_SOA), converted again by mesh_update
    int64_t n_verts;
    double *theta_dev, *s_dev;
    int64_t *scratch;         // small device scratch: per-block partials of the statistics pass
    int64_t *counter;         // MS_COUNT_PARTIALS device words (entry counting of workspace queries)
    hipStream_t upd_stream;   // stream of the last mesh_update (vertex values changed there)
    int info_stale;           // bounds / diameter not reduced since the vertices last changed
    ms_mesh_info_t info;
    int device;
    int n_partials;
};
