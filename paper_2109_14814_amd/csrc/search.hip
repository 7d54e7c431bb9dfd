// search.hip -- the mesh-intersection search of Sec. 6.2 on one GPU.
//
// Pipeline (one HIP stream, counts kept in device memory):
//   k_mark      per triangle: overlapped cells (Sec. 6.2.1); per-side hashed
//               occupancy bitmaps
//   k_count     per triangle: cells also touched by the other mesh (a box that
//               holds triangles of only one mesh cannot hold a pair, Sec. 6.3)
//   scan        entry offsets
//   k_emit      entries key = [cell | side | triangle]
//   radix sort  groups entries by cell (A's before B's inside a cell)
//   k_cells     per cell holding both meshes: start, nA, nB
//   scan        pair-slot offsets (sum of nA * nB)
//   k_enum      slot -> (cell, iA, iB); a pair is kept only in its home cell
//               (cell of the componentwise max of the boxes' lower corners) and
//               only if the closed boxes overlap (Sec. 6.2.2)
//   k_narrow    Moller quick test (Sec. 6.2.3), 4x4 solve and inclusion test
//               (Sec. 6.2.4), hit records
//   sort        hits by (triA, triB)
#include <math.h>
#include <string.h>

#include "ms_internal.hpp"

namespace ms {

namespace {

constexpr int BLOCK = 256;
constexpr int MAX_GRID = 2048;
constexpr double TWO_PI = 6.283185307179586476925286766559;

inline unsigned grid_for(int64_t n, int64_t cap = MAX_GRID)
{
    int64_t g = ceil_div(n > 0 ? n : 1, BLOCK);
    return (unsigned)(g < cap ? g : cap);
}

struct KeyLayout {
    int tb;            // triangle bits
    int cell_shift;    // tb + 1
    uint64_t tmask;
};

struct PairView {
    MeshView A, B;
    GridView g;
    KeyLayout kl;
    int32_t nA, nB;      // triangles (entries of B are indexed nA + t in the per-triangle arrays)
    int32_t bm_log2;     // bitmap bits per side = 2^bm_log2
    int32_t pad;
};

MS_D uint32_t bm_hash(uint64_t cell, int log2)
{
    return (uint32_t)((cell * 0x9E3779B97F4A7C15ull) >> (64 - log2));
}

MS_D bool bm_test(const uint64_t *bm, uint32_t h) { return (bm[h >> 6] >> (h & 63)) & 1ull; }

struct CellRange {
    int64_t lo[4], hi[4];
};

// Overlapped cell range of a triangle's box, or false when the triangle is
// flagged non-finite.
MS_D bool tri_cells(const double *box, const GridView &g, CellRange &r)
{
    const double2 *b = reinterpret_cast<const double2 *>(box);
    double2 l01 = b[0], l23 = b[1], h01 = b[2], h23 = b[3];
    double lo[4] = {l01.x, l01.y, l23.x, l23.y}, hi[4] = {h01.x, h01.y, h23.x, h23.y};
    if (!(lo[0] == lo[0])) return false;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        r.lo[d] = cell_of(lo[d], g.wlo[d], g.inv, g.n[d]);
        r.hi[d] = cell_of(hi[d], g.wlo[d], g.inv, g.n[d]);
    }
    return true;
}

MS_D int64_t range_count(const CellRange &r)
{
    return (r.hi[0] - r.lo[0] + 1) * (r.hi[1] - r.lo[1] + 1) * (r.hi[2] - r.lo[2] + 1) * (r.hi[3] - r.lo[3] + 1);
}

// Visit every cell of a range in lexicographic order.
template <typename F>
MS_D void for_cells(const CellRange &r, const int64_t n[4], F &&f)
{
    for (int64_t c0 = r.lo[0]; c0 <= r.hi[0]; ++c0)
        for (int64_t c1 = r.lo[1]; c1 <= r.hi[1]; ++c1)
            for (int64_t c2 = r.lo[2]; c2 <= r.hi[2]; ++c2) {
                int64_t base = ((c0 * n[1] + c1) * n[2] + c2) * n[3];
                for (int64_t c3 = r.lo[3]; c3 <= r.hi[3]; ++c3) f((uint64_t)(base + c3));
            }
}

// Triangle gt of the concatenation [A's triangles, B's triangles]: side, local
// index and box pointer.
MS_D void tri_of(const PairView &pv, int64_t gt, int &side, int32_t &t, const double *&box)
{
    side = gt >= pv.nA;
    t = (int32_t)(side ? gt - pv.nA : gt);
    box = (side ? pv.B.box : pv.A.box) + 8 * (int64_t)t;
}

// ---------------------------------------------------------------- kernels

__global__ void __launch_bounds__(BLOCK) k_init(search_stats_t *stats)
{
    int64_t *s = (int64_t *)stats;
    if (threadIdx.x < 16) s[threadIdx.x] = 0;
}

__global__ void __launch_bounds__(BLOCK) k_mark(PairView pv, uint64_t *bm, search_stats_t *stats)
{
    const int64_t ntot = (int64_t)pv.nA + pv.nB;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long all = 0, bad = 0;
    const size_t words = (size_t)1 << (pv.bm_log2 - 6);
    for (int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gt < ntot; gt += stride) {
        int side; int32_t t; const double *box;
        tri_of(pv, gt, side, t, box);
        CellRange r;
        if (!tri_cells(box, pv.g, r)) { ++bad; continue; }
        all += (unsigned long long)range_count(r);
        uint64_t *mine = bm + (size_t)side * words;
        for_cells(r, pv.g.n, [&](uint64_t c) {
            uint32_t h = bm_hash(c, pv.bm_log2);
            uint64_t bit = 1ull << (h & 63);
            // bits only go from 0 to 1 during this kernel, so a (possibly
            // stale) set bit is final and the atomic can be skipped
            if (!(mine[h >> 6] & bit)) atomicOr((unsigned long long *)&mine[h >> 6], (unsigned long long)bit);
        });
    }
    all = wave_sum_u64(all);
    bad = wave_sum_u64(bad);
    if (lane_id() == 0) {
        if (all) atomicAdd((unsigned long long *)&stats->n_entries_all, all);
        if (bad) atomicAdd((unsigned long long *)&stats->n_nonfinite, bad);
    }
}

__global__ void __launch_bounds__(BLOCK) k_count(PairView pv, const uint64_t *bm, uint32_t *cnt)
{
    const int64_t ntot = (int64_t)pv.nA + pv.nB;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const size_t words = (size_t)1 << (pv.bm_log2 - 6);
    for (int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gt < ntot; gt += stride) {
        int side; int32_t t; const double *box;
        tri_of(pv, gt, side, t, box);
        CellRange r;
        uint32_t c = 0;
        if (tri_cells(box, pv.g, r)) {
            const uint64_t *other = bm + (size_t)(1 - side) * words;
            for_cells(r, pv.g.n, [&](uint64_t cell) { c += bm_test(other, bm_hash(cell, pv.bm_log2)); });
        }
        cnt[gt] = c;
    }
}

// Entries of every triangle at its scanned offset.  When the total exceeds
// the capacity nothing is written and the overflow flag is raised; the
// number of keys to sort (n_eff) is then 0.
__global__ void __launch_bounds__(BLOCK) k_emit(PairView pv, const uint64_t *bm, const int64_t *off, int64_t cap,
                                                uint64_t *keys, int64_t *n_eff, search_stats_t *stats)
{
    const int64_t ntot = (int64_t)pv.nA + pv.nB;
    const int64_t E = off[ntot];
    const bool fits = E <= cap;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *n_eff = fits ? E : 0;
        if (!fits) atomicOr((unsigned long long *)&stats->overflow, 1ull);
    }
    if (!fits) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const size_t words = (size_t)1 << (pv.bm_log2 - 6);
    for (int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gt < ntot; gt += stride) {
        int side; int32_t t; const double *box;
        tri_of(pv, gt, side, t, box);
        CellRange r;
        if (!tri_cells(box, pv.g, r)) continue;
        const uint64_t *other = bm + (size_t)(1 - side) * words;
        int64_t o = off[gt];
        const uint64_t low = ((uint64_t)side << pv.kl.tb) | (uint64_t)t;
        for_cells(r, pv.g.n, [&](uint64_t cell) {
            if (bm_test(other, bm_hash(cell, pv.bm_log2))) keys[o++] = (cell << pv.kl.cell_shift) | low;
        });
    }
}

// First index in [lo, hi) whose key is >= k (keys sorted ascending).
MS_D int64_t lower_bound_u64(const uint64_t *a, int64_t lo, int64_t hi, uint64_t k)
{
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] < k) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

struct CellRec {
    int64_t start;
    int32_t nA, nB;
};

__global__ void __launch_bounds__(BLOCK) k_cells(const uint64_t *keys, const int64_t *n_dev, KeyLayout kl,
                                                 CellRec *cells, int64_t *pairs, search_stats_t *stats)
{
    const int64_t n = *n_dev;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t iters = ceil_div(n, stride);
    for (int64_t it = 0; it < iters; ++it) {
        int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + it * stride;
        bool start = false;
        int64_t nA = 0, nB = 0;
        if (e < n) {
            uint64_t k = keys[e];
            uint64_t cell = k >> kl.cell_shift;
            start = (e == 0) || ((keys[e - 1] >> kl.cell_shift) != cell);
            if (start) {
                uint64_t next = (cell + 1) << kl.cell_shift;
                int64_t end = lower_bound_u64(keys, e + 1, n, next);
                int64_t fb = lower_bound_u64(keys, e, end, (cell << kl.cell_shift) | (1ull << kl.tb));
                nA = fb - e;
                nB = end - fb;
                start = nA > 0 && nB > 0;
            }
        }
        int64_t slot = wave_reserve(start, (unsigned long long *)&stats->n_cells);
        if (start) {
            cells[slot] = CellRec{e, (int32_t)nA, (int32_t)nB};
            pairs[slot] = nA * nB;
        }
    }
}

// Last index c in [0, n) with pre[c] <= x (pre ascending, pre[0] = 0).
MS_D int64_t upper_bound_m1(const int64_t *pre, int64_t n, int64_t x)
{
    int64_t lo = 0, hi = n;   // invariant: pre[lo] <= x < pre[hi] (pre[n] = total)
    while (hi - lo > 1) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (pre[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

struct Box { double lo[4], hi[4]; };

MS_D Box load_box(const double *p)
{
    const double2 *b = reinterpret_cast<const double2 *>(p);
    double2 l01 = b[0], l23 = b[1], h01 = b[2], h23 = b[3];
    return Box{{l01.x, l01.y, l23.x, l23.y}, {h01.x, h01.y, h23.x, h23.y}};
}

__global__ void __launch_bounds__(BLOCK) k_enum(PairView pv, const uint64_t *keys, const CellRec *cells,
                                                const int64_t *pstart, search_stats_t *stats, int64_t *cand,
                                                int64_t cand_cap)
{
    const int64_t ncells = stats->n_cells;
    const int64_t P = pstart[ncells];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t iters = ceil_div(P, stride);
    for (int64_t it = 0; it < iters; ++it) {
        int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + it * stride;
        bool keep = false;
        uint64_t packed = 0;
        if (slot < P) {
            int64_t c = upper_bound_m1(pstart, ncells, slot);
            CellRec cr = cells[c];
            int64_t local = slot - pstart[c];
            int64_t iA = local % cr.nA, iB = local / cr.nA;
            uint64_t kA = keys[cr.start + iA];
            uint64_t kB = keys[cr.start + cr.nA + iB];
            uint64_t cell = kA >> pv.kl.cell_shift;
            int32_t ta = (int32_t)(kA & pv.kl.tmask), tb = (int32_t)(kB & pv.kl.tmask);
            Box a = load_box(pv.A.box + 8 * (int64_t)ta);
            Box b = load_box(pv.B.box + 8 * (int64_t)tb);
            bool ov = true;
            int64_t h[4];
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                ov = ov && (a.lo[d] <= b.hi[d]) && (b.lo[d] <= a.hi[d]);
                double m = a.lo[d] > b.lo[d] ? a.lo[d] : b.lo[d];
                h[d] = cell_of(m, pv.g.wlo[d], pv.g.inv, pv.g.n[d]);
            }
            keep = ov && ((uint64_t)cell_linear(h, pv.g.n) == cell);
            packed = ((uint64_t)(uint32_t)ta << 32) | (uint32_t)tb;
        }
        int64_t idx = wave_reserve(keep, (unsigned long long *)&stats->n_cand);
        if (keep) {
            if (idx < cand_cap) cand[idx] = (int64_t)packed;
            else atomicOr((unsigned long long *)&stats->overflow, 2ull);
        }
    }
}

// ------------------------------------------------------- the pair predicate

struct Tri { double p[3][4]; };

MS_D Tri load_tri(const MeshView &m, int32_t t)
{
    int32_t i1, i2, i3;
    tri_vertex_ids(m, t, i1, i2, i3);
    d4 a = load_d4(m.V + 4 * (int64_t)i1), b = load_d4(m.V + 4 * (int64_t)i2), c = load_d4(m.V + 4 * (int64_t)i3);
    return Tri{{{a.x, a.y, a.z, a.w}, {b.x, b.y, b.z, b.w}, {c.x, c.y, c.z, c.w}}};
}

// Same-side test of Sec. 6.2.3 on the (x, y, p_x) projection: with
// n = (p1 - p2) x (p3 - p2), reject when n.(q_j - p2) is > 0 for all j or < 0
// for all j.
MS_D bool same_side(const Tri &P, const Tri &Q)
{
    const double *p1 = P.p[0], *p2 = P.p[1], *p3 = P.p[2];
    double e1x = p1[0] - p2[0], e1y = p1[1] - p2[1], e1z = p1[2] - p2[2];
    double e2x = p3[0] - p2[0], e2y = p3[1] - p2[1], e2z = p3[2] - p2[2];
    double nx = e1y * e2z - e1z * e2y;
    double ny = e1z * e2x - e1x * e2z;
    double nz = e1x * e2y - e1y * e2x;
    double f[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const double *q = Q.p[j];
        f[j] = (nx * (q[0] - p2[0]) + ny * (q[1] - p2[1])) + nz * (q[2] - p2[2]);
    }
    bool pos = (f[0] > 0.0) && (f[1] > 0.0) && (f[2] > 0.0);
    bool neg = (f[0] < 0.0) && (f[1] < 0.0) && (f[2] < 0.0);
    return pos || neg;
}

// 4x4 system of Sec. 6.2.4, Gaussian elimination with partial pivoting
// (first row of largest magnitude; exact zero pivot = singular).  Row swaps
// are selects on fully unrolled loops, so the matrix stays in registers.
MS_D bool solve_pair(const Tri &P, const Tri &Q, double z[4])
{
    double M[4][4], r[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        M[d][0] = P.p[0][d] - P.p[1][d];
        M[d][1] = P.p[2][d] - P.p[1][d];
        M[d][2] = Q.p[1][d] - Q.p[0][d];
        M[d][3] = Q.p[1][d] - Q.p[2][d];
        r[d] = Q.p[1][d] - P.p[1][d];
    }
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int piv = k;
        double best = fabs(M[k][k]);
#pragma unroll
        for (int i = k + 1; i < 4; ++i) {
            double a = fabs(M[i][k]);
            if (a > best) { best = a; piv = i; }
        }
#pragma unroll
        for (int i = k + 1; i < 4; ++i) {
            bool s = piv == i;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                double x = M[k][j], y = M[i][j];
                M[k][j] = s ? y : x;
                M[i][j] = s ? x : y;
            }
            double x = r[k], y = r[i];
            r[k] = s ? y : x;
            r[i] = s ? x : y;
        }
        ok = ok && (M[k][k] != 0.0);
#pragma unroll
        for (int i = k + 1; i < 4; ++i) {
            double l = M[i][k] / M[k][k];
#pragma unroll
            for (int j = k + 1; j < 4; ++j) M[i][j] = M[i][j] - l * M[k][j];
            r[i] = r[i] - l * r[k];
        }
    }
#pragma unroll
    for (int k = 3; k >= 0; --k) {
        double acc = 0.0;
#pragma unroll
        for (int j = k + 1; j < 4; ++j) acc = acc + M[k][j] * z[j];
        z[k] = (r[k] - acc) / M[k][k];
    }
    return ok;
}

// (theta, s) estimate on triangle t from its barycentrics (Sec. 6.2.4).
MS_D void tri_param(const MeshView &m, int32_t t, double u, double v, double &th, double &s)
{
    int32_t q = t >> 1, h = t & 1;
    int32_t k = q / m.nq, i = q - k * m.nq;
    double th0 = m.theta[i];
    double th1 = (i + 1 < m.n_theta_v) ? m.theta[i + 1] : m.theta[0] + TWO_PI;
    double s0 = m.s[k], s1 = m.s[k + 1];
    if (h == 0) {
        th = (1.0 - u) * th0 + u * th1;
        s = (1.0 - v) * s0 + v * s1;
    } else {
        th = u * th0 + (1.0 - u) * th1;
        s = v * s0 + (1.0 - v) * s1;
    }
    if (m.periodic && th >= TWO_PI) th = th - TWO_PI;
}

enum { PS_AABB = 0, PS_MOLLER = 1, PS_DEGEN = 2, PS_OUTSIDE = 3, PS_HIT = 4 };

// The full pair test without early exits: every stage is evaluated and the
// status is decided at the end (box, Moller, singular, inclusion).
MS_D int pair_status(const Tri &P, const Tri &Q, bool box_ok, double z[4])
{
    bool sep = same_side(P, Q) || same_side(Q, P);
    bool ok = solve_pair(P, Q, z);
    double uv = z[0] + z[1], ab = z[2] + z[3];
    bool in = (z[0] >= 0.0) && (z[1] >= 0.0) && (z[2] >= 0.0) && (z[3] >= 0.0) && (uv <= 1.0) && (ab <= 1.0);
    return !box_ok ? PS_AABB : sep ? PS_MOLLER : !ok ? PS_DEGEN : !in ? PS_OUTSIDE : PS_HIT;
}

MS_D void make_hit(const PairView &pv, const MeshView &A, const MeshView &B, int32_t ta, int32_t tb, const Tri &P,
                   const double z[4], hit_t &h)
{
    double u = z[0], v = z[1], a = z[2], b = z[3];
    h.triA = ta; h.triB = tb; h.flags = 0; h.pad = 0;
    h.u = u; h.v = v; h.a = a; h.b = b;
#pragma unroll
    for (int d = 0; d < 4; ++d) h.X[d] = (P.p[1][d] + u * (P.p[0][d] - P.p[1][d])) + v * (P.p[2][d] - P.p[1][d]);
    tri_param(A, ta, u, v, h.thA, h.sA);
    tri_param(B, tb, a, b, h.thB, h.sB);
    double mg = u;
    mg = fmin(mg, v); mg = fmin(mg, a); mg = fmin(mg, b);
    mg = fmin(mg, 1.0 - (u + v)); mg = fmin(mg, 1.0 - (a + b));
    h.margin = mg;
}

MS_D void wave_count(bool p, int64_t *ctr)
{
    uint64_t m = ballot(p);
    if (m && lane_id() == __builtin_ctzll(m)) atomicAdd((unsigned long long *)ctr, (unsigned long long)__builtin_popcountll(m));
}

MS_D void emit_hit(bool hit, const hit_t &h, uint64_t key, hit_t *hits, uint64_t *hkeys, int64_t cap,
                   search_stats_t *stats)
{
    int64_t idx = wave_reserve(hit, (unsigned long long *)&stats->n_hits);
    if (hit) {
        if (idx < cap) {
            hits[idx] = h;
            if (hkeys) hkeys[idx] = key;
        } else {
            atomicOr((unsigned long long *)&stats->overflow, 4ull);
        }
    }
}

__global__ void __launch_bounds__(BLOCK) k_narrow(PairView pv, const int64_t *cand, int64_t cand_cap,
                                                  hit_t *hits, uint64_t *hkeys, int64_t hits_cap, int tbB,
                                                  search_stats_t *stats)
{
    int64_t n = stats->n_cand;
    if (n > cand_cap) n = cand_cap;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t iters = ceil_div(n, stride);
    for (int64_t it = 0; it < iters; ++it) {
        int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + it * stride;
        int st = PS_AABB;
        int32_t ta = 0, tb = 0;
        double z[4] = {0, 0, 0, 0};
        Tri P;
        if (c < n) {
            uint64_t pk = (uint64_t)cand[c];
            ta = (int32_t)(pk >> 32);
            tb = (int32_t)(pk & 0xffffffffu);
            P = load_tri(pv.A, ta);
            Tri Q = load_tri(pv.B, tb);
            bool sep = same_side(P, Q) || same_side(Q, P);
            if (sep) {
                st = PS_MOLLER;
            } else {
                bool ok = solve_pair(P, Q, z);
                double uv = z[0] + z[1], ab = z[2] + z[3];
                bool in = (z[0] >= 0.0) && (z[1] >= 0.0) && (z[2] >= 0.0) && (z[3] >= 0.0) && (uv <= 1.0) && (ab <= 1.0);
                st = !ok ? PS_DEGEN : !in ? PS_OUTSIDE : PS_HIT;
            }
        }
        wave_count(st == PS_MOLLER, &stats->n_moller);
        wave_count(st == PS_DEGEN, &stats->n_degenerate);
        wave_count(st == PS_OUTSIDE, &stats->n_outside);
        hit_t h;
        if (st == PS_HIT) make_hit(pv, pv.A, pv.B, ta, tb, P, z, h);
        emit_hit(st == PS_HIT, h, ((uint64_t)ta << tbB) | (uint64_t)tb, hits, hkeys, hits_cap, stats);
    }
}

// All pairs, tiled: each thread holds one triangle of A, tiles of B are
// staged in LDS; every stage of the test runs on every pair.
constexpr int AP_TILE = 128;

__global__ void __launch_bounds__(BLOCK) k_allpairs(PairView pv, hit_t *hits, int64_t hits_cap,
                                                    search_stats_t *stats)
{
    __shared__ double s_tri[AP_TILE][12];
    __shared__ double s_box[AP_TILE][8];
    const int64_t a_tiles = ceil_div(pv.nA, BLOCK);
    const int64_t b_tiles = ceil_div(pv.nB, AP_TILE);
    const int64_t n_work = a_tiles * b_tiles;
    for (int64_t w = blockIdx.x; w < n_work; w += gridDim.x) {
        const int64_t at = w % a_tiles, bt = w / a_tiles;
        const int32_t ta = (int32_t)(at * BLOCK + threadIdx.x);
        const bool a_ok = ta < pv.nA;
        Tri P = a_ok ? load_tri(pv.A, ta) : Tri{};
        Box ba = a_ok ? load_box(pv.A.box + 8 * (int64_t)ta) : Box{};
        bool a_fin = a_ok && (ba.lo[0] == ba.lo[0]);
        const int32_t tb0 = (int32_t)(bt * AP_TILE);
        __syncthreads();
        if (threadIdx.x < AP_TILE) {
            int32_t tb = tb0 + threadIdx.x;
            if (tb < pv.nB) {
                Tri Q = load_tri(pv.B, tb);
                Box bb = load_box(pv.B.box + 8 * (int64_t)tb);
                for (int j = 0; j < 3; ++j)
                    for (int d = 0; d < 4; ++d) s_tri[threadIdx.x][4 * j + d] = Q.p[j][d];
                for (int d = 0; d < 4; ++d) { s_box[threadIdx.x][d] = bb.lo[d]; s_box[threadIdx.x][4 + d] = bb.hi[d]; }
            }
        }
        __syncthreads();
        const int nb = (int)((pv.nB - tb0) < AP_TILE ? (pv.nB - tb0) : AP_TILE);
        for (int j = 0; j < nb; ++j) {
            Tri Q;
#pragma unroll
            for (int v = 0; v < 3; ++v)
#pragma unroll
                for (int d = 0; d < 4; ++d) Q.p[v][d] = s_tri[j][4 * v + d];
            bool b_fin = s_box[j][0] == s_box[j][0];
            bool box = true;
#pragma unroll
            for (int d = 0; d < 4; ++d) box = box && (ba.lo[d] <= s_box[j][4 + d]) && (s_box[j][d] <= ba.hi[d]);
            double z[4];
            int st = pair_status(P, Q, box, z);
            bool live = a_fin && b_fin;
            if (!live) st = PS_AABB;
            wave_count(live && st != PS_AABB, &stats->n_cand);
            wave_count(st == PS_MOLLER, &stats->n_moller);
            wave_count(st == PS_DEGEN, &stats->n_degenerate);
            wave_count(st == PS_OUTSIDE, &stats->n_outside);
            hit_t h;
            if (st == PS_HIT) make_hit(pv, pv.A, pv.B, ta, tb0 + j, P, z, h);
            emit_hit(st == PS_HIT, h, 0, hits, nullptr, hits_cap, stats);
        }
    }
}

__global__ void k_min_i64(const int64_t *a, int64_t cap, int64_t *out)
{
    int64_t v = *a;
    *out = v < cap ? v : cap;
}

__global__ void __launch_bounds__(BLOCK) k_hits_place(const hit_t *tmp, const uint64_t *sorted, const int64_t *n_dev,
                                                      int tbB, hit_t *out)
{
    const int64_t n = *n_dev;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const hit_t &h = tmp[i];
        uint64_t key = ((uint64_t)(uint32_t)h.triA << tbB) | (uint32_t)h.triB;
        int64_t pos = lower_bound_u64(sorted, 0, n, key);
        out[pos] = h;
    }
}

// ------------------------------------------------------------- host side

struct Plan {
    int64_t nA, nB, ntot;
    int tb, tbA, tbB;
    int cell_bits;
    int bm_log2;
    int64_t ent_cap, cand_cap, hits_cap;
    // byte offsets into the workspace
    size_t o_bm, o_cnt, o_off, o_keys, o_alt, o_sort, o_scan, o_cells, o_pairs, o_pstart, o_cand, o_htmp,
        o_hkeys, o_halt, o_hsort, o_misc, total;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int key_layout(const ms_mesh *A, const ms_mesh *B, const search_params_t *p, Plan &pl)
{
    pl.nA = A->info.n_tris;
    pl.nB = B->info.n_tris;
    pl.ntot = pl.nA + pl.nB;
    int64_t mx = pl.nA > pl.nB ? pl.nA : pl.nB;
    pl.tb = bits_for(mx > 0 ? (uint64_t)(mx - 1) : 0);
    if (pl.tb == 0) pl.tb = 1;
    pl.tbA = bits_for(pl.nA > 0 ? (uint64_t)(pl.nA - 1) : 0);
    pl.tbB = bits_for(pl.nB > 0 ? (uint64_t)(pl.nB - 1) : 0);
    if (pl.tbB == 0) pl.tbB = 1;
    // total cells, with overflow detection
    unsigned __int128 cells = 1;
    for (int d = 0; d < 4; ++d) {
        if (p->n_cells[d] < 1) return fail(MS_E_ARG, "search: n_cells must be >= 1");
        cells *= (unsigned __int128)p->n_cells[d];
        if (cells > ((unsigned __int128)1 << 64)) return fail(MS_E_KEYBITS, "search: grid has more than 2^64 cells");
    }
    pl.cell_bits = bits_for((uint64_t)(cells - 1));
    if (pl.cell_bits + 1 + pl.tb > 63)
        return fail(MS_E_KEYBITS, "search: cell index + side + triangle needs more than 63 key bits; coarsen the grid");
    if (!(p->inv_edge > 0.0) || !isfinite(p->inv_edge)) return fail(MS_E_ARG, "search: inv_edge must be > 0 and finite");
    for (int d = 0; d < 4; ++d)
        if (!isfinite(p->world_lo[d])) return fail(MS_E_ARG, "search: world_lo must be finite");
    int lg = bits_for((uint64_t)(pl.ntot > 0 ? pl.ntot : 1)) + 4;
    pl.bm_log2 = lg < 12 ? 12 : (lg > 26 ? 26 : lg);
    return MS_OK;
}

void layout_ws(Plan &pl)
{
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
    int passes = (pl.cell_bits + 1 + 7) / 8;
    int hpasses = (pl.tbA + pl.tbB + 7) / 8;
    int max_passes = passes > hpasses ? passes : hpasses;
    if (max_passes < 1) max_passes = 1;
    int64_t cell_cap = pl.ent_cap / 2 + 1;
    pl.o_bm = take(((size_t)2 << pl.bm_log2) / 8);
    pl.o_cnt = take((size_t)(pl.ntot + 1) * 4);
    pl.o_off = take((size_t)(pl.ntot + 1) * 8);
    pl.o_keys = take((size_t)(pl.ent_cap + 1) * 8);
    pl.o_alt = take((size_t)(pl.ent_cap + 1) * 8);
    pl.o_sort = take(sort_ws_bytes(pl.ent_cap > pl.hits_cap ? pl.ent_cap : pl.hits_cap, max_passes));
    pl.o_scan = take(scan_ws_bytes());
    pl.o_cells = take((size_t)cell_cap * sizeof(CellRec));
    pl.o_pairs = take((size_t)cell_cap * 8);
    pl.o_pstart = take((size_t)(cell_cap + 1) * 8);
    pl.o_cand = take((size_t)(pl.cand_cap > 0 ? pl.cand_cap : 1) * 8);
    pl.o_htmp = take((size_t)(pl.hits_cap > 0 ? pl.hits_cap : 1) * sizeof(hit_t));
    pl.o_hkeys = take((size_t)(pl.hits_cap + 1) * 8);
    pl.o_halt = take((size_t)(pl.hits_cap + 1) * 8);
    pl.o_hsort = pl.o_sort;   // the hit sort reuses the entry sort's scratch (the entry sort is done by then)
    pl.o_misc = take(64);
    pl.total = o;
}

__global__ void __launch_bounds__(BLOCK) k_count_all(PairView pv, unsigned long long *total)
{
    const int64_t ntot = (int64_t)pv.nA + pv.nB;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long all = 0;
    for (int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gt < ntot; gt += stride) {
        int side; int32_t t; const double *box;
        tri_of(pv, gt, side, t, box);
        CellRange r;
        if (tri_cells(box, pv.g, r)) all += (unsigned long long)range_count(r);
    }
    all = wave_sum_u64(all);
    if (lane_id() == 0 && all) atomicAdd(total, all);
}

PairView make_pair_view(const ms_mesh *A, const ms_mesh *B, const search_params_t *p, const Plan &pl)
{
    PairView pv;
    memset(&pv, 0, sizeof pv);
    pv.A = A->view;
    pv.B = B->view;
    for (int d = 0; d < 4; ++d) { pv.g.wlo[d] = p->world_lo[d]; pv.g.n[d] = p->n_cells[d]; }
    pv.g.inv = p->inv_edge;
    pv.kl.tb = pl.tb;
    pv.kl.cell_shift = pl.tb + 1;
    pv.kl.tmask = (1ull << pl.tb) - 1;
    pv.nA = (int32_t)pl.nA;
    pv.nB = (int32_t)pl.nB;
    pv.bm_log2 = pl.bm_log2;
    return pv;
}

}  // namespace
}  // namespace ms

using namespace ms;

extern "C" int search_workspace_size(const ms_mesh *A, const ms_mesh *B, const search_params_t *params,
                                     int64_t cand_cap, int64_t hits_cap, void *stream, size_t *bytes)
{
    if (!A || !B || !params || !bytes) return fail(MS_E_ARG, "search_workspace_size: NULL argument");
    if (cand_cap < 0 || hits_cap < 0) return fail(MS_E_ARG, "search_workspace_size: negative capacity");
    Plan pl;
    memset(&pl, 0, sizeof pl);
    int rc = key_layout(A, B, params, pl);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    PairView pv = make_pair_view(A, B, params, pl);
    unsigned long long *ctr = (unsigned long long *)(A->scratch);
    if ((rc = launch_fill_u64((uint64_t *)ctr, 0, 1, st))) return rc;
    hipLaunchKernelGGL(k_count_all, dim3(grid_for(pl.ntot)), dim3(BLOCK), 0, st, pv, ctr);
    MS_HIP(hipGetLastError());
    unsigned long long E = 0;
    MS_HIP(hipMemcpyAsync(&E, ctr, 8, hipMemcpyDeviceToHost, st));
    MS_HIP(hipStreamSynchronize(st));
    pl.ent_cap = (int64_t)E;
    pl.cand_cap = cand_cap;
    pl.hits_cap = hits_cap;
    layout_ws(pl);
    *bytes = pl.total;
    return MS_OK;
}

extern "C" int search_intersections(const ms_mesh *A, const ms_mesh *B, const search_params_t *params, void *ws_dev,
                                    size_t ws_bytes, hit_t *hits_dev, int64_t hits_cap, search_stats_t *stats_dev,
                                    int64_t *cand_dev, int64_t cand_cap, int64_t *needed, void *stream)
{
    if (!A || !B || !params || !stats_dev || (!ws_dev && ws_bytes)) return fail(MS_E_ARG, "search_intersections: NULL argument");
    if (hits_cap < 0 || cand_cap < 0) return fail(MS_E_ARG, "search_intersections: negative capacity");
    if (hits_cap > 0 && !hits_dev) return fail(MS_E_ARG, "search_intersections: hits_dev is NULL");
    const bool want_cand = (params->flags & MS_SEARCH_CANDIDATES) != 0;
    if (want_cand && cand_cap > 0 && !cand_dev) return fail(MS_E_ARG, "search_intersections: cand_dev is NULL");
    if ((params->flags & MS_SEARCH_STRICT) && (A->info.n_nonfinite || B->info.n_nonfinite))
        return fail(MS_E_NONFINITE, "search_intersections: non-finite triangles with MS_SEARCH_STRICT");
    Plan pl;
    memset(&pl, 0, sizeof pl);
    int rc = key_layout(A, B, params, pl);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;

    // Largest entry capacity that fits the workspace for these capacities.
    pl.cand_cap = want_cand ? 0 : cand_cap;
    pl.hits_cap = hits_cap;
    pl.ent_cap = 0;
    layout_ws(pl);
    if (pl.total > ws_bytes) {
        if (needed) { needed[0] = hits_cap; needed[1] = cand_cap; needed[2] = (int64_t)pl.total; }
        return fail(MS_E_WORKSPACE, "search_intersections: workspace smaller than the fixed part");
    }
    {
        // each entry costs 16 B of keys + 8 B cells/pairs + look-back words; grow ent_cap to fit
        int64_t lo = 0, hi = (int64_t)(ws_bytes / 16) + 1;
        while (hi - lo > 1) {
            int64_t mid = lo + (hi - lo) / 2;
            Plan t = pl;
            t.ent_cap = mid;
            layout_ws(t);
            if (t.total <= ws_bytes) lo = mid; else hi = mid;
        }
        pl.ent_cap = lo;
        if (pl.ent_cap > ((int64_t)1 << 30) - 2) pl.ent_cap = ((int64_t)1 << 30) - 2;
        layout_ws(pl);
    }
    char *ws = (char *)ws_dev;
    uint64_t *bm = (uint64_t *)(ws + pl.o_bm);
    uint32_t *cnt = (uint32_t *)(ws + pl.o_cnt);
    int64_t *off = (int64_t *)(ws + pl.o_off);
    uint64_t *keys = (uint64_t *)(ws + pl.o_keys);
    uint64_t *alt = (uint64_t *)(ws + pl.o_alt);
    int max_passes = (pl.cell_bits + 1 + 7) / 8;
    int hpasses = (pl.tbA + pl.tbB + 7) / 8;
    if (hpasses > max_passes) max_passes = hpasses;
    if (max_passes < 1) max_passes = 1;
    SortWs sws;
    sort_ws_carve(ws + pl.o_sort, pl.ent_cap > pl.hits_cap ? pl.ent_cap : pl.hits_cap, max_passes, sws);
    void *scan_ws = ws + pl.o_scan;
    CellRec *cells = (CellRec *)(ws + pl.o_cells);
    int64_t *pairs = (int64_t *)(ws + pl.o_pairs);
    int64_t *pstart = (int64_t *)(ws + pl.o_pstart);
    int64_t *cand = want_cand ? cand_dev : (int64_t *)(ws + pl.o_cand);
    int64_t ccap = cand_cap;
    hit_t *htmp = (hit_t *)(ws + pl.o_htmp);
    uint64_t *hkeys = (uint64_t *)(ws + pl.o_hkeys);
    uint64_t *halt = (uint64_t *)(ws + pl.o_halt);
    int64_t *misc = (int64_t *)(ws + pl.o_misc);   // [0] n_eff entries, [1] n_eff hits
    int64_t cell_cap = pl.ent_cap / 2 + 1;

    PairView pv = make_pair_view(A, B, params, pl);
    hipLaunchKernelGGL(k_init, dim3(1), dim3(BLOCK), 0, st, stats_dev);
    if ((rc = launch_fill_u64(bm, 0, (int64_t)(((size_t)2 << pl.bm_log2) / 64), st))) return rc;
    hipLaunchKernelGGL(k_mark, dim3(grid_for(pl.ntot)), dim3(BLOCK), 0, st, pv, bm, stats_dev);
    hipLaunchKernelGGL(k_count, dim3(grid_for(pl.ntot)), dim3(BLOCK), 0, st, pv, bm, cnt);
    MS_HIP(hipGetLastError());
    if ((rc = scan_u32_to_i64(cnt, off, pl.ntot, &stats_dev->n_entries, scan_ws, st))) return rc;
    hipLaunchKernelGGL(k_emit, dim3(grid_for(pl.ntot)), dim3(BLOCK), 0, st, pv, bm, off, pl.ent_cap, keys, misc,
                       stats_dev);
    MS_HIP(hipGetLastError());
    uint64_t *sorted = keys;
    if ((rc = radix_sort_u64(keys, alt, misc, pl.ent_cap, pl.tb, pl.cell_bits + 1, sws, st, &sorted))) return rc;
    hipLaunchKernelGGL(k_cells, dim3(grid_for(pl.ent_cap)), dim3(BLOCK), 0, st, sorted, misc, pv.kl, cells, pairs,
                       stats_dev);
    MS_HIP(hipGetLastError());
    if ((rc = scan_i64_dev(pairs, pstart, &stats_dev->n_cells, cell_cap, &stats_dev->n_slots, scan_ws, st))) return rc;
    hipLaunchKernelGGL(k_enum, dim3(MAX_GRID), dim3(BLOCK), 0, st, pv, sorted, cells, pstart, stats_dev, cand, ccap);
    MS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_narrow, dim3(MAX_GRID), dim3(BLOCK), 0, st, pv, cand, ccap, htmp, hkeys, hits_cap, pl.tbB,
                       stats_dev);
    hipLaunchKernelGGL(k_min_i64, dim3(1), dim3(1), 0, st, &stats_dev->n_hits, hits_cap, misc + 1);
    MS_HIP(hipGetLastError());
    uint64_t *hsorted = hkeys;
    if (hits_cap > 0) {
        if ((rc = radix_sort_u64(hkeys, halt, misc + 1, hits_cap, 0, pl.tbA + pl.tbB, sws, st, &hsorted))) return rc;
        hipLaunchKernelGGL(k_hits_place, dim3(grid_for(hits_cap, 256)), dim3(BLOCK), 0, st, htmp, hsorted, misc + 1,
                           pl.tbB, hits_dev);
        MS_HIP(hipGetLastError());
    }
    // status: read the counters back
    search_stats_t hs;
    MS_HIP(hipMemcpyAsync(&hs, stats_dev, sizeof hs, hipMemcpyDeviceToHost, st));
    MS_HIP(hipStreamSynchronize(st));
    if (hs.overflow) {
        if (needed) {
            needed[0] = hs.n_hits;
            needed[1] = hs.n_cand;
            Plan t = pl;
            t.ent_cap = hs.n_entries;
            t.hits_cap = hs.n_hits > hits_cap ? hs.n_hits : hits_cap;
            t.cand_cap = want_cand ? 0 : (hs.n_cand > cand_cap ? hs.n_cand : cand_cap);
            layout_ws(t);
            needed[2] = (int64_t)t.total;
        }
        if (hs.overflow & 1) return fail(MS_E_WORKSPACE, "search_intersections: entries exceed the workspace");
        return fail(MS_E_CAPACITY, "search_intersections: candidate or hit capacity exceeded");
    }
    return MS_OK;
}

extern "C" int narrow_allpairs(const ms_mesh *A, const ms_mesh *B, hit_t *hits_dev, int64_t hits_cap,
                               int64_t *n_hits_dev, search_stats_t *stats_dev, void *stream)
{
    if (!A || !B || !n_hits_dev || !stats_dev) return fail(MS_E_ARG, "narrow_allpairs: NULL argument");
    if (hits_cap < 0 || (hits_cap > 0 && !hits_dev)) return fail(MS_E_ARG, "narrow_allpairs: bad hits buffer");
    hipStream_t st = (hipStream_t)stream;
    Plan pl;
    memset(&pl, 0, sizeof pl);
    pl.nA = A->info.n_tris;
    pl.nB = B->info.n_tris;
    PairView pv;
    memset(&pv, 0, sizeof pv);
    pv.A = A->view;
    pv.B = B->view;
    pv.nA = (int32_t)pl.nA;
    pv.nB = (int32_t)pl.nB;
    hipLaunchKernelGGL(k_init, dim3(1), dim3(BLOCK), 0, st, stats_dev);
    int64_t work = ceil_div(pl.nA, BLOCK) * ceil_div(pl.nB, AP_TILE);
    if (work > 0) {
        int64_t g = work < 8192 ? work : 8192;
        hipLaunchKernelGGL(k_allpairs, dim3((unsigned)g), dim3(BLOCK), 0, st, pv, hits_dev, hits_cap, stats_dev);
    }
    hipLaunchKernelGGL(k_min_i64, dim3(1), dim3(1), 0, st, &stats_dev->n_hits, (int64_t)INT64_MAX, n_hits_dev);
    MS_HIP(hipGetLastError());
    return MS_OK;
}
