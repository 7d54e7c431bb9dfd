/*
 * oracle.c -- plain, slow, obviously-correct CPU oracle for the mesh
 * intersection search and the stroboscopic map.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no fast-math, no
 * -march=native), so every floating-point expression is evaluated as written,
 * one IEEE-754 double rounding per operation.
 *
 * Paper: Kumar, Anderson, de la Llave, "Rapid GPU-assisted search and
 * parameterization-based refinement and continuation of connections between
 * tori in periodically perturbed planar circular restricted 3-body problems"
 * (arXiv 2109.14814).  Section references below are to that paper.
 *
 * Contents
 *   1. mesh and triangle definitions              (Sec. 6.1, Sec. 6.2)
 *   2. the pair predicate P: AABB, Moller, 4x4    (Sec. 6.2.2-6.2.4)
 *   3. brute force over all triangle pairs        (Sec. 2.2, the plain definition)
 *   4. uniform-grid search with per-box lists     (Sec. 6.2.1)
 *   5. RK8 stroboscopic map, tangent, invariants  (Sec. 3, Sec. 4.1, Sec. 7)
 *   6. the elliptic problem in position-momentum
 *      coordinates, its flow and state transition
 *      matrix                                      (Sec. 3.3, Sec. 4.1, Sec. 7)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* 1. Meshes (Sec. 6.1)                                                      */
/* ------------------------------------------------------------------------ */

/* Vertex grid W(theta_i, s_k): V[(k*n_theta_v + i)*4 + c], theta fastest.
 * Periodic meshes close in theta: vertex index i+1 is taken mod n_theta_v. */
typedef struct {
    const double *V;
    int32_t n_theta_v, n_s_v, periodic, pad;
    const double *theta;  /* n_theta_v sample values */
    const double *s;      /* n_s_v sample values */
} orc_mesh;

/* Hit record: 16 bytes of ids + 13 doubles = 120 bytes. */
typedef struct {
    int32_t triA, triB;
    uint32_t flags, pad;
    double u, v, a, b;
    double X[4];
    double thA, sA, thB, sB;
    double margin;
} orc_hit;

static const double ORC_2PI = 6.283185307179586476925286766559;

static int64_t quads_theta(const orc_mesh *m)
{
    if (m->n_theta_v <= 0) return 0;
    return m->periodic ? m->n_theta_v : m->n_theta_v - 1;
}

ORC_API int64_t orc_n_tris(const orc_mesh *m)
{
    int64_t nq = quads_theta(m);
    int64_t ns = (int64_t)m->n_s_v - 1;
    if (nq <= 0 || ns <= 0) return 0;
    return 2 * nq * ns;
}

static const double *vtx(const orc_mesh *m, int64_t i, int64_t k)
{
    if (i >= m->n_theta_v) i -= m->n_theta_v;   /* periodic wrap (Sec. 6.1) */
    return m->V + 4 * (k * (int64_t)m->n_theta_v + i);
}

/* Triangle t = 2q + h of quad q = i + k*Nq.  Vertex order of the narrow
 * phase (Sec. 6.2.4), in which p2 is the right-angle corner in parameter space:
 *   h = 0 (T1): p1 = W(i+1,k),   p2 = W(i,k),     p3 = W(i,k+1)
 *   h = 1 (T2): p1 = W(i,k+1),   p2 = W(i+1,k+1), p3 = W(i+1,k)          */
ORC_API void orc_tri_verts(const orc_mesh *m, int64_t t, double p[3][4])
{
    int64_t nq = quads_theta(m);
    int64_t q = t / 2, h = t % 2;
    int64_t i = q % nq, k = q / nq;
    const double *a, *b, *c;
    if (h == 0) { a = vtx(m, i + 1, k); b = vtx(m, i, k); c = vtx(m, i, k + 1); }
    else        { a = vtx(m, i, k + 1); b = vtx(m, i + 1, k + 1); c = vtx(m, i + 1, k); }
    for (int d = 0; d < 4; ++d) { p[0][d] = a[d]; p[1][d] = b[d]; p[2][d] = c[d]; }
}

static int tri_finite(double p[3][4])
{
    for (int j = 0; j < 3; ++j)
        for (int d = 0; d < 4; ++d)
            if (!isfinite(p[j][d])) return 0;
    return 1;
}

/* Exact axis-aligned bounding box of a triangle (Sec. 6.2.2). */
static void tri_box(double p[3][4], double lo[4], double hi[4])
{
    for (int d = 0; d < 4; ++d) {
        double l = p[0][d], h = p[0][d];
        if (p[1][d] < l) l = p[1][d];
        if (p[2][d] < l) l = p[2][d];
        if (p[1][d] > h) h = p[1][d];
        if (p[2][d] > h) h = p[2][d];
        lo[d] = l; hi[d] = h;
    }
}

ORC_API void orc_tri_aabb(const orc_mesh *m, int64_t t, double lo[4], double hi[4])
{
    double p[3][4];
    orc_tri_verts(m, t, p);
    tri_box(p, lo, hi);
}

/* (theta, s) of a point with barycentrics (u, v) on triangle t (Sec. 6.2.4):
 *   T1: ((1-u) th_i + u th_{i+1},  (1-v) s_k + v s_{k+1})
 *   T2: (u th_i + (1-u) th_{i+1},  v s_k + (1-v) s_{k+1})
 * On a periodic mesh th_N = th_0 + 2 pi, and the estimate is wrapped to
 * [0, 2 pi) when it reaches 2 pi. */
static void tri_params(const orc_mesh *m, int64_t t, double u, double v,
                       double *th_out, double *s_out)
{
    int64_t nq = quads_theta(m);
    int64_t q = t / 2, h = t % 2;
    int64_t i = q % nq, k = q / nq;
    double th0 = m->theta[i];
    double th1 = (i + 1 < m->n_theta_v) ? m->theta[i + 1] : m->theta[0] + ORC_2PI;
    double s0 = m->s[k], s1 = m->s[k + 1];
    double th, s;
    if (h == 0) {
        th = (1.0 - u) * th0 + u * th1;
        s = (1.0 - v) * s0 + v * s1;
    } else {
        th = u * th0 + (1.0 - u) * th1;
        s = v * s0 + (1.0 - v) * s1;
    }
    if (m->periodic && th >= ORC_2PI) th = th - ORC_2PI;
    *th_out = th;
    *s_out = s;
}

/* ------------------------------------------------------------------------ */
/* 2. The pair predicate P (Sec. 6.2.2 - 6.2.4)                              */
/* ------------------------------------------------------------------------ */

enum { ST_AABB = 0, ST_MOLLER = 1, ST_DEGENERATE = 2, ST_OUTSIDE = 3, ST_HIT = 4 };

static int boxes_overlap(const double loA[4], const double hiA[4],
                         const double loB[4], const double hiB[4])
{
    for (int d = 0; d < 4; ++d) {
        if (!(loA[d] <= hiB[d])) return 0;   /* closed boxes: touching counts */
        if (!(loB[d] <= hiA[d])) return 0;
    }
    return 1;
}

/* Quick rejection of Moller (Sec. 6.2.3) on the (x, y, p_x) projection:
 * the plane of triangle p has normal n = (p1 - p2) x (p3 - p2); the other
 * triangle q is rejected when all three of its vertices lie strictly on one
 * side, i.e. f_j = n . (q_j - p2) are all > 0 or all < 0.  A zero (or a
 * degenerate projected normal, which gives f = 0) never rejects. */
static int moller_reject(double p[3][4], double q[3][4])
{
    double e1[3], e2[3], n[3], f[3];
    for (int d = 0; d < 3; ++d) { e1[d] = p[0][d] - p[1][d]; e2[d] = p[2][d] - p[1][d]; }
    n[0] = e1[1] * e2[2] - e1[2] * e2[1];
    n[1] = e1[2] * e2[0] - e1[0] * e2[2];
    n[2] = e1[0] * e2[1] - e1[1] * e2[0];
    for (int j = 0; j < 3; ++j) {
        double w0 = q[j][0] - p[1][0], w1 = q[j][1] - p[1][1], w2 = q[j][2] - p[1][2];
        f[j] = (n[0] * w0 + n[1] * w1) + n[2] * w2;
    }
    if (f[0] > 0.0 && f[1] > 0.0 && f[2] > 0.0) return 1;
    if (f[0] < 0.0 && f[1] < 0.0 && f[2] < 0.0) return 1;
    return 0;
}

/* Solve p2 + (p1-p2) u + (p3-p2) v = q2 + (q1-q2) a + (q3-q2) b (Sec. 6.2.4,
 * the 4x4 system of the narrow phase) by Gaussian elimination with partial
 * pivoting: pivot = first row of maximal |entry|; exact zero pivot means the
 * system is singular (returns 0).  z = (u, v, a, b). */
static int solve4(double p[3][4], double q[3][4], double z[4])
{
    double M[4][4], r[4];
    for (int d = 0; d < 4; ++d) {
        M[d][0] = p[0][d] - p[1][d];
        M[d][1] = p[2][d] - p[1][d];
        M[d][2] = q[1][d] - q[0][d];
        M[d][3] = q[1][d] - q[2][d];
        r[d] = q[1][d] - p[1][d];
    }
    for (int k = 0; k < 4; ++k) {
        int piv = k;
        double best = fabs(M[k][k]);
        for (int i = k + 1; i < 4; ++i) {
            if (fabs(M[i][k]) > best) { best = fabs(M[i][k]); piv = i; }
        }
        if (piv != k) {
            for (int j = 0; j < 4; ++j) { double tmp = M[k][j]; M[k][j] = M[piv][j]; M[piv][j] = tmp; }
            double tmp = r[k]; r[k] = r[piv]; r[piv] = tmp;
        }
        if (M[k][k] == 0.0) return 0;
        for (int i = k + 1; i < 4; ++i) {
            double l = M[i][k] / M[k][k];
            for (int j = k + 1; j < 4; ++j) M[i][j] = M[i][j] - l * M[k][j];
            r[i] = r[i] - l * r[k];
        }
    }
    for (int k = 3; k >= 0; --k) {
        double acc = 0.0;
        for (int j = k + 1; j < 4; ++j) acc = acc + M[k][j] * z[j];
        z[k] = (r[k] - acc) / M[k][k];
    }
    return 1;
}

/* Full predicate on one triangle pair; fills *h on a hit.  When `forced` is
 * set every stage is evaluated even after a rejection (the decision is the
 * same; only the work differs). */
static int pair_test(const orc_mesh *A, int64_t ta, double p[3][4],
                     const double loA[4], const double hiA[4],
                     const orc_mesh *B, int64_t tb, double q[3][4],
                     const double loB[4], const double hiB[4],
                     int forced, orc_hit *h)
{
    int box = boxes_overlap(loA, hiA, loB, hiB);
    if (!box && !forced) return ST_AABB;
    int rej = moller_reject(p, q);
    if (!rej || forced) rej = rej | moller_reject(q, p);
    if (rej && !forced) return box ? ST_MOLLER : ST_AABB;
    double z[4];
    int ok = solve4(p, q, z);
    if (!box) return ST_AABB;
    if (rej) return ST_MOLLER;
    if (!ok) return ST_DEGENERATE;
    double u = z[0], v = z[1], a = z[2], b = z[3];
    double uv = u + v, ab = a + b;
    int inside = (u >= 0.0) && (v >= 0.0) && (a >= 0.0) && (b >= 0.0) && (uv <= 1.0) && (ab <= 1.0);
    if (!inside) return ST_OUTSIDE;
    if (h) {
        h->triA = (int32_t)ta; h->triB = (int32_t)tb; h->flags = 0; h->pad = 0;
        h->u = u; h->v = v; h->a = a; h->b = b;
        for (int d = 0; d < 4; ++d)
            h->X[d] = (p[1][d] + u * (p[0][d] - p[1][d])) + v * (p[2][d] - p[1][d]);
        tri_params(A, ta, u, v, &h->thA, &h->sA);
        tri_params(B, tb, a, b, &h->thB, &h->sB);
        double mg = u;
        mg = fmin(mg, v); mg = fmin(mg, a); mg = fmin(mg, b);
        mg = fmin(mg, 1.0 - uv); mg = fmin(mg, 1.0 - ab);
        h->margin = mg;
    }
    return ST_HIT;
}

/* Single-pair entry point (for tests): status code and optional hit. */
ORC_API int orc_pair(const orc_mesh *A, int64_t ta, const orc_mesh *B, int64_t tb, orc_hit *h)
{
    double p[3][4], q[3][4], loA[4], hiA[4], loB[4], hiB[4];
    orc_tri_verts(A, ta, p); orc_tri_verts(B, tb, q);
    tri_box(p, loA, hiA); tri_box(q, loB, hiB);
    return pair_test(A, ta, p, loA, hiA, B, tb, q, loB, hiB, 0, h);
}

/* Raw 4x4 solve of two explicit triangles (for tests). */
ORC_API int orc_solve4(const double *p12, const double *q12, double *z)
{
    double p[3][4], q[3][4];
    memcpy(p, p12, sizeof p); memcpy(q, q12, sizeof q);
    return solve4(p, q, z);
}

ORC_API int orc_moller_reject(const double *p12, const double *q12)
{
    double p[3][4], q[3][4];
    memcpy(p, p12, sizeof p); memcpy(q, q12, sizeof q);
    return moller_reject(p, q) || moller_reject(q, p);
}

/* ------------------------------------------------------------------------ */
/* Growable arrays and the result object                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t n_cand;  int64_t *cand;   /* packed (triA << 32) | triB, ascending */
    int64_t n_hits;  orc_hit *hits;   /* ascending (triA, triB) */
    /* counts[0] pairs examined, [1] AABB pass, [2] Moller reject,
     * [3] degenerate, [4] outside, [5] hits, [6] non-finite tris of A,
     * [7] non-finite tris of B */
    int64_t counts[8];
    int64_t n_entries;   /* grid: (cell, tri) entries */
    int64_t n_slots;     /* grid: sum over boxes of nA * nB */
    int64_t n_boxes;     /* grid: boxes holding both meshes */
} orc_result;

typedef struct { int64_t *p; int64_t n, cap; } vec64;
typedef struct { orc_hit *p; int64_t n, cap; } vechit;

static int v64_push(vec64 *v, int64_t x)
{
    if (v->n == v->cap) {
        int64_t nc = v->cap ? 2 * v->cap : 1024;
        int64_t *np = (int64_t *)realloc(v->p, (size_t)nc * sizeof(int64_t));
        if (!np) return -1;
        v->p = np; v->cap = nc;
    }
    v->p[v->n++] = x;
    return 0;
}

static int vh_push(vechit *v, const orc_hit *x)
{
    if (v->n == v->cap) {
        int64_t nc = v->cap ? 2 * v->cap : 256;
        orc_hit *np = (orc_hit *)realloc(v->p, (size_t)nc * sizeof(orc_hit));
        if (!np) return -1;
        v->p = np; v->cap = nc;
    }
    v->p[v->n++] = *x;
    return 0;
}

ORC_API void orc_result_free(orc_result *r)
{
    free(r->cand); free(r->hits);
    r->cand = NULL; r->hits = NULL; r->n_cand = r->n_hits = 0;
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* Per-mesh triangle boxes and finiteness, computed once. */
typedef struct { double *lo, *hi; unsigned char *fin; int64_t n; } tri_table;

static int table_build(const orc_mesh *m, tri_table *T, int64_t *n_nonfinite)
{
    int64_t n = orc_n_tris(m);
    T->n = n;
    T->lo = (double *)malloc((size_t)(n ? n : 1) * 4 * sizeof(double));
    T->hi = (double *)malloc((size_t)(n ? n : 1) * 4 * sizeof(double));
    T->fin = (unsigned char *)malloc((size_t)(n ? n : 1));
    if (!T->lo || !T->hi || !T->fin) return -1;
    int64_t bad = 0;
#pragma omp parallel for reduction(+ : bad) schedule(static)
    for (int64_t t = 0; t < n; ++t) {
        double p[3][4];
        orc_tri_verts(m, t, p);
        T->fin[t] = (unsigned char)tri_finite(p);
        if (!T->fin[t]) ++bad;
        tri_box(p, T->lo + 4 * t, T->hi + 4 * t);
    }
    *n_nonfinite = bad;
    return 0;
}

static void table_free(tri_table *T) { free(T->lo); free(T->hi); free(T->fin); }

/* Run the full predicate on a sorted unique candidate list; fills hits and
 * the status counters. */
static int narrow_list(const orc_mesh *A, const tri_table *TA, const orc_mesh *B, const tri_table *TB,
                       const int64_t *cand, int64_t n_cand, orc_result *res, int nthreads)
{
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
    vechit *tv = (vechit *)calloc((size_t)nt, sizeof(vechit));
    int64_t cnt[5] = {0, 0, 0, 0, 0};
    int err = 0;
    if (!tv) return -1;
    /* contiguous static chunks keep the concatenation in ascending order */
#pragma omp parallel num_threads(nt) reduction(+ : cnt[:5]) reduction(| : err)
    {
        int me = omp_get_thread_num(), nth = omp_get_num_threads();
        int64_t beg = n_cand * me / nth, end = n_cand * (me + 1) / nth;
        for (int64_t c = beg; c < end; ++c) {
            int64_t ta = (int64_t)((uint64_t)cand[c] >> 32), tb = cand[c] & 0xffffffffLL;
            double p[3][4], q[3][4];
            orc_tri_verts(A, ta, p); orc_tri_verts(B, tb, q);
            orc_hit h;
            int st = pair_test(A, ta, p, TA->lo + 4 * ta, TA->hi + 4 * ta,
                               B, tb, q, TB->lo + 4 * tb, TB->hi + 4 * tb, 0, &h);
            cnt[st] += 1;
            if (st == ST_HIT && vh_push(&tv[me], &h)) err |= 1;
        }
    }
    int64_t tot = 0;
    for (int i = 0; i < nt; ++i) tot += tv[i].n;
    res->hits = (orc_hit *)malloc((size_t)(tot ? tot : 1) * sizeof(orc_hit));
    if (!res->hits) err = 1;
    int64_t o = 0;
    for (int i = 0; i < nt; ++i) {
        if (!err && tv[i].n) memcpy(res->hits + o, tv[i].p, (size_t)tv[i].n * sizeof(orc_hit));
        o += tv[i].n;
        free(tv[i].p);
    }
    free(tv);
    res->n_hits = tot;
    res->counts[2] += cnt[ST_MOLLER];
    res->counts[3] += cnt[ST_DEGENERATE];
    res->counts[4] += cnt[ST_OUTSIDE];
    res->counts[5] += cnt[ST_HIT];
    return err ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* 3. Brute force: H = { (A,B) : P(A,B) } over all pairs (Sec. 2.2)          */
/* ------------------------------------------------------------------------ */

/* Tests every pair of finite triangles.  With forced = 0 the AABB test
 * rejects first; with forced = 1 all stages run on every pair (same result,
 * uniform work).  Non-finite triangles are excluded and counted. */
ORC_API int orc_bruteforce(const orc_mesh *A, const orc_mesh *B, int forced,
                           orc_result *res, int nthreads)
{
    memset(res, 0, sizeof *res);
    tri_table TA, TB;
    if (table_build(A, &TA, &res->counts[6]) || table_build(B, &TB, &res->counts[7])) return -1;
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
    vec64 *cv = (vec64 *)calloc((size_t)nt, sizeof(vec64));
    vechit *hv = (vechit *)calloc((size_t)nt, sizeof(vechit));
    int64_t cnt[5] = {0, 0, 0, 0, 0}, examined = 0;
    int err = 0;
    int64_t na = TA.n, nb = TB.n;
#pragma omp parallel num_threads(nt) reduction(+ : cnt[:5], examined) reduction(| : err)
    {
        int me = omp_get_thread_num(), nth = omp_get_num_threads();
        int64_t beg = na * me / nth, end = na * (me + 1) / nth;
        for (int64_t ta = beg; ta < end; ++ta) {
            if (!TA.fin[ta]) continue;
            double p[3][4];
            orc_tri_verts(A, ta, p);
            for (int64_t tb = 0; tb < nb; ++tb) {
                if (!TB.fin[tb]) continue;
                ++examined;
                const double *loA = TA.lo + 4 * ta, *hiA = TA.hi + 4 * ta;
                const double *loB = TB.lo + 4 * tb, *hiB = TB.hi + 4 * tb;
                if (!forced && !boxes_overlap(loA, hiA, loB, hiB)) { cnt[ST_AABB]++; continue; }
                double q[3][4];
                orc_tri_verts(B, tb, q);
                orc_hit h;
                int st = pair_test(A, ta, p, loA, hiA, B, tb, q, loB, hiB, forced, &h);
                cnt[st]++;
                if (st != ST_AABB && v64_push(&cv[me], (ta << 32) | tb)) err |= 1;
                if (st == ST_HIT && vh_push(&hv[me], &h)) err |= 1;
            }
        }
    }
    int64_t nc = 0, nh = 0;
    for (int i = 0; i < nt; ++i) { nc += cv[i].n; nh += hv[i].n; }
    res->cand = (int64_t *)malloc((size_t)(nc ? nc : 1) * sizeof(int64_t));
    res->hits = (orc_hit *)malloc((size_t)(nh ? nh : 1) * sizeof(orc_hit));
    if (!res->cand || !res->hits) err = 1;
    int64_t oc = 0, oh = 0;
    for (int i = 0; i < nt; ++i) {
        if (!err) {
            if (cv[i].n) memcpy(res->cand + oc, cv[i].p, (size_t)cv[i].n * sizeof(int64_t));
            if (hv[i].n) memcpy(res->hits + oh, hv[i].p, (size_t)hv[i].n * sizeof(orc_hit));
        }
        oc += cv[i].n; oh += hv[i].n;
        free(cv[i].p); free(hv[i].p);
    }
    free(cv); free(hv);
    res->n_cand = nc; res->n_hits = nh;
    res->counts[0] = examined;
    res->counts[1] = examined - cnt[ST_AABB];
    res->counts[2] = cnt[ST_MOLLER];
    res->counts[3] = cnt[ST_DEGENERATE];
    res->counts[4] = cnt[ST_OUTSIDE];
    res->counts[5] = cnt[ST_HIT];
    table_free(&TA); table_free(&TB);
    return err ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* 4. Uniform-grid search (Sec. 6.2.1)                                       */
/* ------------------------------------------------------------------------ */

/* Grid cell of coordinate x on axis d: floor((x - w_lo) * inv_edge) clamped
 * to [0, n_d - 1] (0-based form of the paper's ceiling index). */
static int64_t cell_of(double x, double wlo, double inv_edge, int64_t n)
{
    double t = (x - wlo) * inv_edge;
    double f = floor(t);
    if (!(f >= 0.0)) return 0;
    if (f >= (double)n) return n - 1;
    int64_t c = (int64_t)f;
    return c < n ? c : n - 1;
}

typedef struct { int64_t cell; int64_t tri; int32_t side; int32_t pad; } entry_t;

static int cmp_entry(const void *x, const void *y)
{
    const entry_t *a = (const entry_t *)x, *b = (const entry_t *)y;
    if (a->cell != b->cell) return (a->cell > b->cell) - (a->cell < b->cell);
    if (a->side != b->side) return a->side - b->side;
    return (a->tri > b->tri) - (a->tri < b->tri);
}

/* Cell range [clo, chi] per axis covered by a box, and its number of cells. */
static int64_t tri_cells(const double lo[4], const double hi[4], const double wlo[4],
                         double inv_edge, const int64_t n[4], int64_t clo[4], int64_t chi[4])
{
    int64_t cnt = 1;
    for (int d = 0; d < 4; ++d) {
        clo[d] = cell_of(lo[d], wlo[d], inv_edge, n[d]);
        chi[d] = cell_of(hi[d], wlo[d], inv_edge, n[d]);
        cnt *= chi[d] - clo[d] + 1;
    }
    return cnt;
}

/* Linear id of cell (c0, c1, c2, c3): axis 3 varies fastest. */
static int64_t cell_linear(int64_t c0, int64_t c1, int64_t c2, int64_t c3, const int64_t n[4])
{
    return ((c0 * n[1] + c1) * n[2] + c2) * n[3] + c3;
}

/* The linear ids of the cells of a range, in lexicographic order, written to
 * out[0 .. count) (the per-box list entries of one triangle). */
static void range_cells(const int64_t clo[4], const int64_t chi[4], const int64_t n[4], int64_t *out)
{
    int64_t o = 0;
    for (int64_t c0 = clo[0]; c0 <= chi[0]; ++c0)
        for (int64_t c1 = clo[1]; c1 <= chi[1]; ++c1)
            for (int64_t c2 = clo[2]; c2 <= chi[2]; ++c2)
                for (int64_t c3 = clo[3]; c3 <= chi[3]; ++c3) out[o++] = cell_linear(c0, c1, c2, c3, n);
}

/* The grid search of Sec. 6.2.1 followed by the AABB test, the Moller test
 * and the narrow phase: (1) every triangle's overlapped cells; (2) per-box
 * lists of A and B triangles (built by sorting (cell, side, tri) entries);
 * (3) all A x B pairs in every box that holds both, AABB-tested; (4) the
 * union over boxes (pairs that share several boxes counted once); (5) the
 * Moller test and 4x4 solve on each distinct candidate.  The world origin
 * w_lo, inverse cell edge and cells per axis n[4] are inputs.
 *
 * prune != 0: the world-bound restriction remarked on in Sec. 6.2.1 -- the
 * grid only holds triangles whose box meets the other mesh's box (the box of
 * that mesh's finite vertices); no pair with a triangle outside can have
 * overlapping boxes.  n_entries still counts every finite triangle's cells;
 * n_boxes and n_slots are those of the restricted grid. */
ORC_API int orc_grid_search(const orc_mesh *A, const orc_mesh *B, const double *wlo,
                            double inv_edge, const int64_t *ncell, int prune, orc_result *res, int nthreads)
{
    memset(res, 0, sizeof *res);
    int64_t n[4] = {ncell[0], ncell[1], ncell[2], ncell[3]};
    double prodf = (double)n[0] * (double)n[1] * (double)n[2] * (double)n[3];
    if (prodf > 9.0e18 || n[0] < 1 || n[1] < 1 || n[2] < 1 || n[3] < 1) return -2;
    tri_table T[2];
    if (table_build(A, &T[0], &res->counts[6]) || table_build(B, &T[1], &res->counts[7])) return -1;
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();

    /* each mesh's box over its finite vertices (for the pruning; it holds
     * every finite triangle) */
    int64_t ntri[2] = {T[0].n, T[1].n};
    const orc_mesh *M[2] = {A, B};
    double mlo[2][4], mhi[2][4];
    for (int sd = 0; sd < 2; ++sd) {
        for (int d = 0; d < 4; ++d) { mlo[sd][d] = INFINITY; mhi[sd][d] = -INFINITY; }
        const int64_t nv = ntri[sd] > 0 ? (int64_t)M[sd]->n_theta_v * M[sd]->n_s_v : 0;
        for (int64_t k = 0; k < nv; ++k) {
            const double *x = M[sd]->V + 4 * k;
            if (!(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]) && isfinite(x[3]))) continue;
            for (int d = 0; d < 4; ++d) {
                if (x[d] < mlo[sd][d]) mlo[sd][d] = x[d];
                if (x[d] > mhi[sd][d]) mhi[sd][d] = x[d];
            }
        }
    }

    /* (1) entry counts and offsets (all finite triangles counted; the
     * pruned ones emit nothing) */
    int64_t *off[2];
    int64_t E = 0, E_all = 0;
    for (int sd = 0; sd < 2; ++sd) {
        off[sd] = (int64_t *)malloc((size_t)(ntri[sd] + 1) * sizeof(int64_t));
        if (!off[sd]) return -1;
        int64_t all = 0;
#pragma omp parallel for num_threads(nt) schedule(static) reduction(+ : all)
        for (int64_t t = 0; t < ntri[sd]; ++t) {
            int64_t clo[4], chi[4];
            int64_t c = T[sd].fin[t] ? tri_cells(T[sd].lo + 4 * t, T[sd].hi + 4 * t, wlo, inv_edge, n, clo, chi) : 0;
            all += c;
            if (prune && c && !boxes_overlap(T[sd].lo + 4 * t, T[sd].hi + 4 * t, mlo[1 - sd], mhi[1 - sd])) c = 0;
            off[sd][t] = c;
        }
        E_all += all;
        int64_t run = E;
        for (int64_t t = 0; t < ntri[sd]; ++t) { int64_t c = off[sd][t]; off[sd][t] = run; run += c; }
        off[sd][ntri[sd]] = run;
        E = run;
    }
    res->n_entries = E_all;
    entry_t *ent = (entry_t *)malloc((size_t)(E ? E : 1) * sizeof(entry_t));
    if (!ent) return -1;
    /* (2) emit entries, then group them by box */
    int ent_err = 0;
    for (int sd = 0; sd < 2; ++sd) {
#pragma omp parallel for num_threads(nt) schedule(static) reduction(| : ent_err)
        for (int64_t t = 0; t < ntri[sd]; ++t) {
            if (!T[sd].fin[t] || off[sd][t + 1] == off[sd][t]) continue;    /* non-finite or pruned */
            int64_t clo[4], chi[4];
            int64_t cnt = tri_cells(T[sd].lo + 4 * t, T[sd].hi + 4 * t, wlo, inv_edge, n, clo, chi);
            int64_t *cells = (int64_t *)malloc((size_t)cnt * sizeof(int64_t));
            if (!cells) { ent_err = 1; continue; }
            range_cells(clo, chi, n, cells);
            int64_t o = off[sd][t];
            for (int64_t j = 0; j < cnt; ++j, ++o) {
                ent[o].cell = cells[j];
                ent[o].tri = t; ent[o].side = sd; ent[o].pad = 0;
            }
            free(cells);
        }
        free(off[sd]);
    }
    if (ent_err) { free(ent); table_free(&T[0]); table_free(&T[1]); return -1; }
    qsort(ent, (size_t)E, sizeof(entry_t), cmp_entry);

    /* box boundaries */
    vec64 bstart = {0, 0, 0};
    for (int64_t e = 0; e < E; ++e)
        if (e == 0 || ent[e].cell != ent[e - 1].cell) v64_push(&bstart, e);
    v64_push(&bstart, E);
    int64_t nbox = bstart.n - 1;

    /* (3) all pairs per box that holds both meshes, AABB-tested */
    vec64 *cv = (vec64 *)calloc((size_t)nt, sizeof(vec64));
    int64_t slots = 0, both = 0;
    int err = 0;
#pragma omp parallel for num_threads(nt) schedule(dynamic, 64) reduction(+ : slots, both) reduction(| : err)
    for (int64_t bx = 0; bx < nbox; ++bx) {
        int me = omp_get_thread_num();
        int64_t s0 = bstart.p[bx], s1 = bstart.p[bx + 1];
        int64_t mid = s0;
        while (mid < s1 && ent[mid].side == 0) ++mid;
        int64_t nA = mid - s0, nB = s1 - mid;
        if (nA == 0 || nB == 0) continue;
        both += 1;
        slots += nA * nB;
        for (int64_t ia = s0; ia < mid; ++ia) {
            int64_t ta = ent[ia].tri;
            for (int64_t ib = mid; ib < s1; ++ib) {
                int64_t tb = ent[ib].tri;
                if (boxes_overlap(T[0].lo + 4 * ta, T[0].hi + 4 * ta, T[1].lo + 4 * tb, T[1].hi + 4 * tb))
                    if (v64_push(&cv[me], (ta << 32) | tb)) err |= 1;
            }
        }
    }
    free(ent); free(bstart.p);
    res->n_slots = slots;
    res->n_boxes = both;

    /* (4) union over boxes */
    int64_t tot = 0;
    for (int i = 0; i < nt; ++i) tot += cv[i].n;
    int64_t *all = (int64_t *)malloc((size_t)(tot ? tot : 1) * sizeof(int64_t));
    if (!all) err = 1;
    int64_t o = 0;
    for (int i = 0; i < nt; ++i) {
        if (!err && cv[i].n) memcpy(all + o, cv[i].p, (size_t)cv[i].n * sizeof(int64_t));
        o += cv[i].n; free(cv[i].p);
    }
    free(cv);
    if (err) { free(all); table_free(&T[0]); table_free(&T[1]); return -1; }
    qsort(all, (size_t)tot, sizeof(int64_t), cmp_i64);
    int64_t u = 0;
    for (int64_t i = 0; i < tot; ++i)
        if (i == 0 || all[i] != all[i - 1]) all[u++] = all[i];
    res->cand = all;
    res->n_cand = u;
    res->counts[0] = slots;
    res->counts[1] = u;

    /* (5) narrow phase on the distinct candidates */
    int rc = narrow_list(A, &T[0], B, &T[1], all, u, res, nt);
    table_free(&T[0]); table_free(&T[1]);
    return rc;
}

/* The cell map itself, for its pins: cell_of on one axis, and the linear
 * cell ids of triangle t's entries in the order the grid search emits them
 * (returns their number; writes at most cap of them; -1 for a non-finite
 * triangle). */
ORC_API int64_t orc_cell_of(double x, double wlo, double inv_edge, int64_t n)
{
    return cell_of(x, wlo, inv_edge, n);
}

ORC_API int64_t orc_tri_entries(const orc_mesh *m, int64_t t, const double *wlo, double inv_edge,
                                const int64_t *ncell, int64_t *out, int64_t cap)
{
    double p[3][4], lo[4], hi[4];
    int64_t clo[4], chi[4];
    orc_tri_verts(m, t, p);
    if (!tri_finite(p)) return -1;
    tri_box(p, lo, hi);
    int64_t cnt = tri_cells(lo, hi, wlo, inv_edge, ncell, clo, chi);
    if (cnt <= cap) range_cells(clo, chi, ncell, out);
    return cnt;
}

/* Total (cell, tri) entries for a grid (exact recount, for tests). */
ORC_API int64_t orc_grid_entries(const orc_mesh *m, const double *wlo, double inv_edge, const int64_t *ncell)
{
    int64_t n = orc_n_tris(m), E = 0;
    for (int64_t t = 0; t < n; ++t) {
        double p[3][4], lo[4], hi[4];
        int64_t clo[4], chi[4];
        orc_tri_verts(m, t, p);
        if (!tri_finite(p)) continue;
        tri_box(p, lo, hi);
        E += tri_cells(lo, hi, wlo, inv_edge, ncell, clo, chi);
    }
    return E;
}

/* ------------------------------------------------------------------------ */
/* 5. Stroboscopic map of the planar elliptic RTBP (Sec. 3.3, Sec. 4.1)      */
/* ------------------------------------------------------------------------ */

/* Pulsating rotating coordinates, true anomaly f as independent variable:
 *   x'' - 2 y' = w(f) dOmega/dx,  y'' + 2 x' = w(f) dOmega/dy,
 *   w(f) = 1 / (1 + e cos f),
 *   Omega = (x^2 + y^2)/2 + (1 - mu)/r1 + mu/r2,
 *   r1 = |(x + mu, y)|, r2 = |(x - 1 + mu, y)|.
 * The stroboscopic map F advances f by 2 pi (the period of the primaries). */

/* Cooper & Verner (1972), "Some explicit Runge-Kutta methods of high order",
 * SIAM J. Numer. Anal. 9: the 11-stage explicit method of order 8.
 * Coefficients involve sqrt(21); they are formed here in double precision. */
static double CV_A[11][11], CV_B[11], CV_C[11];
static int cv_ready = 0;

static void cv_init(void)
{
    if (cv_ready) return;
    const double r = sqrt(21.0);
    memset(CV_A, 0, sizeof CV_A);
    double (*a)[11] = CV_A;
    a[1][0] = 1.0 / 2.0;
    a[2][0] = 1.0 / 4.0; a[2][1] = 1.0 / 4.0;
    a[3][0] = 1.0 / 7.0; a[3][1] = (-7.0 - 3.0 * r) / 98.0; a[3][2] = (21.0 + 5.0 * r) / 49.0;
    a[4][0] = (11.0 + r) / 84.0; a[4][2] = (18.0 + 4.0 * r) / 63.0; a[4][3] = (21.0 - r) / 252.0;
    a[5][0] = (5.0 + r) / 48.0; a[5][2] = (9.0 + r) / 36.0; a[5][3] = (-231.0 + 14.0 * r) / 360.0;
    a[5][4] = (63.0 - 7.0 * r) / 80.0;
    a[6][0] = (10.0 - r) / 42.0; a[6][2] = (-432.0 + 92.0 * r) / 315.0; a[6][3] = (633.0 - 145.0 * r) / 90.0;
    a[6][4] = (-504.0 + 115.0 * r) / 70.0; a[6][5] = (63.0 - 13.0 * r) / 35.0;
    a[7][0] = 1.0 / 14.0; a[7][4] = (14.0 - 3.0 * r) / 126.0; a[7][5] = (13.0 - 3.0 * r) / 63.0;
    a[7][6] = 1.0 / 9.0;
    a[8][0] = 1.0 / 32.0; a[8][4] = (91.0 - 21.0 * r) / 576.0; a[8][5] = 11.0 / 72.0;
    a[8][6] = (-385.0 - 75.0 * r) / 1152.0; a[8][7] = (63.0 + 13.0 * r) / 128.0;
    a[9][0] = 1.0 / 14.0; a[9][4] = 1.0 / 9.0; a[9][5] = (-733.0 - 147.0 * r) / 2205.0;
    a[9][6] = (515.0 + 111.0 * r) / 504.0; a[9][7] = (-51.0 - 11.0 * r) / 56.0;
    a[9][8] = (132.0 + 28.0 * r) / 245.0;
    a[10][4] = (-42.0 + 7.0 * r) / 18.0; a[10][5] = (-18.0 + 28.0 * r) / 45.0;
    a[10][6] = (-273.0 - 53.0 * r) / 72.0; a[10][7] = (301.0 + 53.0 * r) / 72.0;
    a[10][8] = (28.0 - 28.0 * r) / 45.0; a[10][9] = (49.0 - 7.0 * r) / 18.0;
    double b[11] = {1.0 / 20.0, 0, 0, 0, 0, 0, 0, 49.0 / 180.0, 16.0 / 45.0, 49.0 / 180.0, 1.0 / 20.0};
    double c[11] = {0.0, 0.5, 0.5, (7.0 + r) / 14.0, (7.0 + r) / 14.0, 0.5,
                    (7.0 - r) / 14.0, (7.0 - r) / 14.0, 0.5, (7.0 + r) / 14.0, 1.0};
    memcpy(CV_B, b, sizeof b);
    memcpy(CV_C, c, sizeof c);
    cv_ready = 1;
}

ORC_API void orc_rk8_tableau(double *a /*11x11*/, double *b, double *c)
{
    cv_init();
    memcpy(a, CV_A, sizeof CV_A); memcpy(b, CV_B, sizeof CV_B); memcpy(c, CV_C, sizeof CV_C);
}

typedef struct { double mu, e; } model_t;

/* Right-hand side; also returns Omega's gradient for reuse. */
static void rhs(const model_t *md, double f, const double y[4], double dy[4])
{
    double mu = md->mu;
    double w = 1.0 / (1.0 + md->e * cos(f));
    double x = y[0], yy = y[1];
    double dx1 = x + mu, dx2 = x - 1.0 + mu;
    double r1 = sqrt(dx1 * dx1 + yy * yy), r2 = sqrt(dx2 * dx2 + yy * yy);
    double r13 = r1 * r1 * r1, r23 = r2 * r2 * r2;
    double Ox = x - (1.0 - mu) * dx1 / r13 - mu * dx2 / r23;
    double Oy = yy - (1.0 - mu) * yy / r13 - mu * yy / r23;
    dy[0] = y[2];
    dy[1] = y[3];
    dy[2] = 2.0 * y[3] + w * Ox;
    dy[3] = -2.0 * y[2] + w * Oy;
}

/* Right-hand side of the variational system: state y plus nd tangent
 * columns Y (4 x nd, column-major: Y[4*j + i]).  Column j gets A(f,y) Y_j,
 * plus dF/de when j == e_col (the parameter column). */
static void rhs_var(const model_t *md, double f, const double *y, const double *Y, int nd, int e_col,
                    double *dy, double *dY)
{
    double mu = md->mu;
    double cf = cos(f);
    double w = 1.0 / (1.0 + md->e * cf);
    double dw_de = -cf * w * w;
    double x = y[0], yy = y[1];
    double dx1 = x + mu, dx2 = x - 1.0 + mu;
    double r1s = dx1 * dx1 + yy * yy, r2s = dx2 * dx2 + yy * yy;
    double r1 = sqrt(r1s), r2 = sqrt(r2s);
    double r13 = r1s * r1, r23 = r2s * r2;
    double r15 = r13 * r1s, r25 = r23 * r2s;
    double Ox = x - (1.0 - mu) * dx1 / r13 - mu * dx2 / r23;
    double Oy = yy - (1.0 - mu) * yy / r13 - mu * yy / r23;
    double Oxx = 1.0 - (1.0 - mu) / r13 - mu / r23 + 3.0 * (1.0 - mu) * dx1 * dx1 / r15 + 3.0 * mu * dx2 * dx2 / r25;
    double Oyy = 1.0 - (1.0 - mu) / r13 - mu / r23 + 3.0 * (1.0 - mu) * yy * yy / r15 + 3.0 * mu * yy * yy / r25;
    double Oxy = 3.0 * (1.0 - mu) * dx1 * yy / r15 + 3.0 * mu * dx2 * yy / r25;
    dy[0] = y[2];
    dy[1] = y[3];
    dy[2] = 2.0 * y[3] + w * Ox;
    dy[3] = -2.0 * y[2] + w * Oy;
    for (int j = 0; j < nd; ++j) {
        const double *v = Y + 4 * j;
        double *dv = dY + 4 * j;
        dv[0] = v[2];
        dv[1] = v[3];
        dv[2] = w * (Oxx * v[0] + Oxy * v[1]) + 2.0 * v[3];
        dv[3] = w * (Oxy * v[0] + Oyy * v[1]) - 2.0 * v[2];
        if (j == e_col) { dv[2] += dw_de * Ox; dv[3] += dw_de * Oy; }
    }
}

/* One RK step of the augmented system (state + nd tangent columns). */
#define MAXD 8
static void rk8_step_var(const model_t *md, double f0, double h, double *y, double *Y, int nd, int e_col)
{
    double k[11][4], K[11][4 * MAXD];
    double ys[4], Ys[4 * MAXD];
    for (int i = 0; i < 11; ++i) {
        for (int c = 0; c < 4; ++c) {
            double acc = 0.0;
            for (int j = 0; j < i; ++j) acc += CV_A[i][j] * k[j][c];
            ys[c] = y[c] + h * acc;
        }
        for (int c = 0; c < 4 * nd; ++c) {
            double acc = 0.0;
            for (int j = 0; j < i; ++j) acc += CV_A[i][j] * K[j][c];
            Ys[c] = Y[c] + h * acc;
        }
        if (nd > 0) rhs_var(md, f0 + CV_C[i] * h, ys, Ys, nd, e_col, k[i], K[i]);
        else rhs(md, f0 + CV_C[i] * h, ys, k[i]);
    }
    for (int c = 0; c < 4; ++c) {
        double acc = 0.0;
        for (int i = 0; i < 11; ++i) acc += CV_B[i] * k[i][c];
        y[c] = y[c] + h * acc;
    }
    for (int c = 0; c < 4 * nd; ++c) {
        double acc = 0.0;
        for (int i = 0; i < 11; ++i) acc += CV_B[i] * K[i][c];
        Y[c] = Y[c] + h * acc;
    }
}

/* F^n_periods by fixed-step RK8, steps_per_period steps per 2 pi of f,
 * starting at f = 0; negative n_periods integrates backwards (h < 0). */
ORC_API int orc_rk8_map(const double *in, double *out, int64_t n, double mu, double e,
                        int32_t steps_per_period, int32_t n_periods, int nthreads)
{
    if (steps_per_period <= 0) return -1;
    cv_init();
    model_t md = {mu, e};
    int64_t nsteps = (int64_t)steps_per_period * (n_periods < 0 ? -n_periods : n_periods);
    double h = (n_periods < 0 ? -ORC_2PI : ORC_2PI) / (double)steps_per_period;
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for num_threads(nt) schedule(dynamic, 16)
    for (int64_t p = 0; p < n; ++p) {
        double y[4] = {in[4 * p], in[4 * p + 1], in[4 * p + 2], in[4 * p + 3]};
        for (int64_t s = 0; s < nsteps; ++s) rk8_step_var(&md, (double)s * h, h, y, NULL, 0, -1);
        for (int c = 0; c < 4; ++c) out[4 * p + c] = y[c];
    }
    return 0;
}

/* F^n and its discrete tangent: dirs is n x nd x 4 (initial tangent columns),
 * e_col the column that also receives dF/de (or -1).  Outputs out (n x 4) and
 * dout (n x nd x 4).  Integrating the variational equations with the same
 * tableau and steps gives exactly the derivative of the discrete map. */
ORC_API int orc_rk8_tangent(const double *in, const double *dirs, int32_t nd, int32_t e_col,
                            double *out, double *dout, int64_t n, double mu, double e,
                            int32_t steps_per_period, int32_t n_periods, int nthreads)
{
    if (steps_per_period <= 0 || nd > MAXD || nd < 0) return -1;
    cv_init();
    model_t md = {mu, e};
    int64_t nsteps = (int64_t)steps_per_period * (n_periods < 0 ? -n_periods : n_periods);
    double h = (n_periods < 0 ? -ORC_2PI : ORC_2PI) / (double)steps_per_period;
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for num_threads(nt) schedule(dynamic, 4)
    for (int64_t p = 0; p < n; ++p) {
        double y[4], Y[4 * MAXD];
        for (int c = 0; c < 4; ++c) y[c] = in[4 * p + c];
        for (int c = 0; c < 4 * nd; ++c) Y[c] = dirs[4 * nd * p + c];
        for (int64_t s = 0; s < nsteps; ++s) rk8_step_var(&md, (double)s * h, h, y, Y, nd, e_col);
        for (int c = 0; c < 4; ++c) out[4 * p + c] = y[c];
        for (int c = 0; c < 4 * nd; ++c) dout[4 * nd * p + c] = Y[c];
    }
    return 0;
}

/* Jacobi integral of the circular problem (e = 0, w = 1):
 * C = 2 Omega - (x'^2 + y'^2). */
ORC_API double orc_jacobi(const double *y, double mu)
{
    double dx1 = y[0] + mu, dx2 = y[0] - 1.0 + mu;
    double r1 = sqrt(dx1 * dx1 + y[1] * y[1]), r2 = sqrt(dx2 * dx2 + y[1] * y[1]);
    double Om = 0.5 * (y[0] * y[0] + y[1] * y[1]) + (1.0 - mu) / r1 + mu / r2;
    return 2.0 * Om - (y[2] * y[2] + y[3] * y[3]);
}

/* Energy balance of the elliptic problem: with E = (x'^2 + y'^2)/2 - w Omega,
 * dE/df = -w'(f) Omega, w' = e sin f / (1 + e cos f)^2.  Integrates the state
 * together with I(f) = integral of -w' Omega by the same RK8 and returns
 * E(end) - E(0) - I(end) in *resid (zero up to truncation and rounding). */
ORC_API int orc_energy_balance(const double *y0, double mu, double e, int32_t steps_per_period,
                               int32_t n_periods, double *resid)
{
    cv_init();
    model_t md = {mu, e};
    int64_t nsteps = (int64_t)steps_per_period * (n_periods < 0 ? -n_periods : n_periods);
    double h = (n_periods < 0 ? -ORC_2PI : ORC_2PI) / (double)steps_per_period;
    double y[5] = {y0[0], y0[1], y0[2], y0[3], 0.0};
    for (int64_t s = 0; s < nsteps; ++s) {
        double f0 = (double)s * h, k[11][5], ys[5];
        for (int i = 0; i < 11; ++i) {
            for (int c = 0; c < 5; ++c) {
                double acc = 0.0;
                for (int j = 0; j < i; ++j) acc += CV_A[i][j] * k[j][c];
                ys[c] = y[c] + h * acc;
            }
            double f = f0 + CV_C[i] * h;
            rhs(&md, f, ys, k[i]);
            double dx1 = ys[0] + mu, dx2 = ys[0] - 1.0 + mu;
            double r1 = sqrt(dx1 * dx1 + ys[1] * ys[1]), r2 = sqrt(dx2 * dx2 + ys[1] * ys[1]);
            double Om = 0.5 * (ys[0] * ys[0] + ys[1] * ys[1]) + (1.0 - mu) / r1 + mu / r2;
            double den = 1.0 + e * cos(f);
            k[i][4] = -(e * sin(f) / (den * den)) * Om;
        }
        for (int c = 0; c < 5; ++c) {
            double acc = 0.0;
            for (int i = 0; i < 11; ++i) acc += CV_B[i] * k[i][c];
            y[c] = y[c] + h * acc;
        }
    }
    double fend = (double)nsteps * h;
    double E[2];
    for (int w = 0; w < 2; ++w) {
        const double *z = w ? y : y0;
        double f = w ? fend : 0.0;
        double dx1 = z[0] + mu, dx2 = z[0] - 1.0 + mu;
        double r1 = sqrt(dx1 * dx1 + z[1] * z[1]), r2 = sqrt(dx2 * dx2 + z[1] * z[1]);
        double Om = 0.5 * (z[0] * z[0] + z[1] * z[1]) + (1.0 - mu) / r1 + mu / r2;
        E[w] = 0.5 * (z[2] * z[2] + z[3] * z[3]) - Om / (1.0 + e * cos(f));
    }
    *resid = E[1] - E[0] - y[4];
    return 0;
}

/* Mismatch of the refinement problem (Sec. 7) between two linear patches
 *   x_u(th1, s1) = bu + th1 du1 + s1 du2,   x_s(th2, s2) = bs + th2 ds1 + s2 ds2,
 *   f = F^{nu}(x_u) - F^{ns}(x_s)   (nu > 0 forward, ns < 0 backward),
 * r = |f|^2, J = df/d(th1, s1, th2, s2, e) from the variational equations,
 * grad = dr/d(...) = 2 J^T f.  patch arrays are 12 doubles: base, d1, d2.
 * Outputs: f (K x 4), r (K), J (K x 4 x 5, row-major), grad (K x 5). */
ORC_API int orc_mismatch(const double *params, int64_t K, const double *pu, const double *ps,
                         double mu, double e, int32_t steps_per_period, int32_t nu, int32_t ns,
                         double *f, double *r, double *J, double *grad, int nthreads)
{
    cv_init();
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
    int err = 0;
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1) reduction(| : err)
    for (int64_t k = 0; k < K; ++k) {
        const double *pr = params + 4 * k;
        double xu[4], xs[4], du[12], ds[12], yu[4], ys[4], Du[12], Ds[12];
        for (int c = 0; c < 4; ++c) {
            xu[c] = pu[c] + pr[0] * pu[4 + c] + pr[1] * pu[8 + c];
            xs[c] = ps[c] + pr[2] * ps[4 + c] + pr[3] * ps[8 + c];
            du[c] = pu[4 + c]; du[4 + c] = pu[8 + c]; du[8 + c] = 0.0;
            ds[c] = ps[4 + c]; ds[4 + c] = ps[8 + c]; ds[8 + c] = 0.0;
        }
        err |= orc_rk8_tangent(xu, du, 3, 2, yu, Du, 1, mu, e, steps_per_period, nu, 1);
        err |= orc_rk8_tangent(xs, ds, 3, 2, ys, Ds, 1, mu, e, steps_per_period, ns, 1);
        double *fk = f + 4 * k, *Jk = J + 20 * k, *gk = grad + 5 * k;
        double rr = 0.0;
        for (int c = 0; c < 4; ++c) { fk[c] = yu[c] - ys[c]; rr += fk[c] * fk[c]; }
        r[k] = rr;
        for (int c = 0; c < 4; ++c) {
            Jk[5 * c + 0] = Du[c];
            Jk[5 * c + 1] = Du[4 + c];
            Jk[5 * c + 2] = -Ds[c];
            Jk[5 * c + 3] = -Ds[4 + c];
            Jk[5 * c + 4] = Du[8 + c] - Ds[8 + c];
        }
        for (int j = 0; j < 5; ++j) {
            double acc = 0.0;
            for (int c = 0; c < 4; ++c) acc += Jk[5 * c + j] * fk[c];
            gk[j] = 2.0 * acc;
        }
    }
    return err ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* 6. The elliptic problem in position-momentum coordinates (Sec. 3.3)        */
/* ------------------------------------------------------------------------ */

/* The primaries move on a Kepler ellipse of semi-major axis 1, eccentricity
 * eps and period 2 pi, with periapse at t = 0, 2 pi, ... (mean anomaly M = t).
 * The frame turns with the line of the primaries but is not rescaled: their
 * separation is rho(t) = 1 - eps cos E(t), E the eccentric anomaly, and they
 * sit at (-mu rho, 0) and ((1 - mu) rho, 0).  With n(t) = d nu / dt (nu the
 * true anomaly) the Hamiltonian is
 *   H = (px^2 + py^2)/2 + n (px y - py x) - (1 - mu)/r1 - mu/r2,
 *   r1 = |(x + mu rho, y)|,  r2 = |(x - (1 - mu) rho, y)|,
 * and the state z = (x, y, px, py) obeys z' = J grad H, J = [[0, I], [-I, 0]]. */

/* Eccentric anomaly: the root of g(E) = E - eps sin E - M.  g is increasing
 * (g' = 1 - eps cos E > 0) and |E - M| = eps |sin E| <= eps, so the root lies
 * in [M - eps, M + eps]; plain bisection until the bracket stops shrinking
 * pins it to the last bit.  M is first reduced to [-pi, pi] (E - M is 2 pi
 * periodic in M). */
static double kepler_E(double M, double eps)
{
    double k = floor(M / ORC_2PI + 0.5);
    double Mr = M - k * ORC_2PI;
    double lo = Mr - eps, hi = Mr + eps;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        if (mid - eps * sin(mid) - Mr < 0.0) lo = mid;
        else hi = mid;
    }
    double glo = fabs(lo - eps * sin(lo) - Mr), ghi = fabs(hi - eps * sin(hi) - Mr);
    return (glo <= ghi ? lo : hi) + k * ORC_2PI;
}

/* E(t), rho(t) = 1 - eps cos E, n(t) = sqrt(1 - eps^2) / rho^2 (the rate of
 * the true anomaly: dE/dt = 1/rho and d nu/dE = sqrt(1 - eps^2)/rho), and
 * nu(t) itself from tan(nu/2) = sqrt((1+eps)/(1-eps)) tan(E/2), continued
 * through the periapse passages. */
ORC_API void orc_pertbp_anomaly(double t, double eps, double *E, double *rho, double *n, double *nu)
{
    double Ea = kepler_E(t, eps);
    double r = 1.0 - eps * cos(Ea);
    double k = floor(Ea / ORC_2PI + 0.5);
    double Er = Ea - k * ORC_2PI;
    double v = 2.0 * atan2(sqrt(1.0 + eps) * sin(0.5 * Er), sqrt(1.0 - eps) * cos(0.5 * Er));
    if (E) *E = Ea;
    if (rho) *rho = r;
    if (n) *n = sqrt(1.0 - eps * eps) / (r * r);
    if (nu) *nu = v + k * ORC_2PI;
}

/* H at (z, t). */
ORC_API double orc_pertbp_hamiltonian(const double *z, double mu, double eps, double t)
{
    double rho, n;
    orc_pertbp_anomaly(t, eps, NULL, &rho, &n, NULL);
    double x = z[0], y = z[1], px = z[2], py = z[3];
    double r1 = sqrt((x + mu * rho) * (x + mu * rho) + y * y);
    double r2 = sqrt((x - (1.0 - mu) * rho) * (x - (1.0 - mu) * rho) + y * y);
    return 0.5 * (px * px + py * py) + n * (px * y - py * x) - (1.0 - mu) / r1 - mu / r2;
}

/* Gradient and Hessian of H in (x, y, px, py) at time t, then
 * z' = J grad H and, for a tangent column v, v' = J Hess(H) v. */
static void pertbp_rhs(double mu, double eps, double t, const double *z, const double *V, int ncol,
                       double *dz, double *dV)
{
    double rho, n;
    orc_pertbp_anomaly(t, eps, NULL, &rho, &n, NULL);
    double x = z[0], y = z[1], px = z[2], py = z[3];
    double d1 = x + mu * rho, d2 = x - (1.0 - mu) * rho;
    double r1s = d1 * d1 + y * y, r2s = d2 * d2 + y * y;
    double r1 = sqrt(r1s), r2 = sqrt(r2s);
    double a1 = (1.0 - mu) / (r1s * r1), a2 = mu / (r2s * r2);                 /* m_i / r_i^3 */
    double b1 = 3.0 * (1.0 - mu) / (r1s * r1s * r1), b2 = 3.0 * mu / (r2s * r2s * r2);   /* 3 m_i / r_i^5 */
    double g[4];                                   /* grad H */
    g[0] = -n * py + a1 * d1 + a2 * d2;
    g[1] = n * px + a1 * y + a2 * y;
    g[2] = px + n * y;
    g[3] = py - n * x;
    dz[0] = g[2];
    dz[1] = g[3];
    dz[2] = -g[0];
    dz[3] = -g[1];
    if (ncol == 0) return;
    double Hs[4][4];                               /* Hess H (symmetric) */
    Hs[0][0] = a1 + a2 - b1 * d1 * d1 - b2 * d2 * d2;
    Hs[1][1] = a1 + a2 - b1 * y * y - b2 * y * y;
    Hs[0][1] = Hs[1][0] = -b1 * d1 * y - b2 * d2 * y;
    Hs[0][2] = Hs[2][0] = 0.0;
    Hs[0][3] = Hs[3][0] = -n;
    Hs[1][2] = Hs[2][1] = n;
    Hs[1][3] = Hs[3][1] = 0.0;
    Hs[2][2] = Hs[3][3] = 1.0;
    Hs[2][3] = Hs[3][2] = 0.0;
    for (int j = 0; j < ncol; ++j) {
        const double *v = V + 4 * j;
        double w[4];
        for (int i = 0; i < 4; ++i) w[i] = Hs[i][0] * v[0] + Hs[i][1] * v[1] + Hs[i][2] * v[2] + Hs[i][3] * v[3];
        double *dv = dV + 4 * j;
        dv[0] = w[2];
        dv[1] = w[3];
        dv[2] = -w[0];
        dv[3] = -w[1];
    }
}

/* One RK8 step of the state with ncol tangent columns (column-major, V[4 j + i]). */
static void pertbp_step(double mu, double eps, double t0, double h, double *z, double *V, int ncol)
{
    double k[11][4], K[11][16], zs[4], Vs[16];
    for (int i = 0; i < 11; ++i) {
        for (int c = 0; c < 4; ++c) {
            double acc = 0.0;
            for (int j = 0; j < i; ++j) acc += CV_A[i][j] * k[j][c];
            zs[c] = z[c] + h * acc;
        }
        for (int c = 0; c < 4 * ncol; ++c) {
            double acc = 0.0;
            for (int j = 0; j < i; ++j) acc += CV_A[i][j] * K[j][c];
            Vs[c] = V[c] + h * acc;
        }
        pertbp_rhs(mu, eps, t0 + CV_C[i] * h, zs, Vs, ncol, k[i], K[i]);
    }
    for (int c = 0; c < 4; ++c) {
        double acc = 0.0;
        for (int i = 0; i < 11; ++i) acc += CV_B[i] * k[i][c];
        z[c] = z[c] + h * acc;
    }
    for (int c = 0; c < 4 * ncol; ++c) {
        double acc = 0.0;
        for (int i = 0; i < 11; ++i) acc += CV_B[i] * K[i][c];
        V[c] = V[c] + h * acc;
    }
}

/* Flow from t0 to t1 in nsteps equal RK8 steps (stage k of step s at time
 * t0 + s h + c_k h, h = (t1 - t0)/nsteps).  out: n x 4.  stm (optional):
 * n x 16, row-major d out_i / d in_j, from the variational equations
 * integrated with the same stages (the exact derivative of the discrete
 * flow).  The stroboscopic map F^m is t0 = 0, t1 = 2 pi m. */
ORC_API int orc_pertbp_flow(const double *in, double *out, double *stm, int64_t n, double mu, double eps,
                            double t0, double t1, int64_t nsteps, int nthreads)
{
    if (nsteps < 0 || !(eps >= 0.0 && eps < 1.0)) return -1;
    cv_init();
    double h = nsteps > 0 ? (t1 - t0) / (double)nsteps : 0.0;
    int ncol = stm ? 4 : 0;
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for num_threads(nt) schedule(dynamic, 4)
    for (int64_t p = 0; p < n; ++p) {
        double z[4], V[16];
        for (int c = 0; c < 4; ++c) z[c] = in[4 * p + c];
        for (int j = 0; j < 4; ++j)
            for (int i = 0; i < 4; ++i) V[4 * j + i] = i == j ? 1.0 : 0.0;
        for (int64_t s = 0; s < nsteps; ++s) pertbp_step(mu, eps, t0 + (double)s * h, h, z, V, ncol);
        for (int c = 0; c < 4; ++c) out[4 * p + c] = z[c];
        if (stm)
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) stm[16 * p + 4 * i + j] = V[4 * j + i];
    }
    return 0;
}

/* Threads the OpenMP loops of this library use. */
ORC_API int orc_max_threads(void) { return omp_get_max_threads(); }
