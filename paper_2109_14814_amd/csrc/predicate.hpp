// predicate.hpp -- the triangle-pair test of the narrow phase (device code).
//
// Same-side (Moller) quick rejection on the (x, y, p_x) projection (Sec.
// 6.2.3), the 4x4 system p2 + (p1-p2) u + (p3-p2) v = q2 + (q1-q2) a +
// (q3-q2) b solved by Gaussian elimination with partial pivoting (Sec. 6.2.4),
// the inclusion test u, v, a, b >= 0, u + v <= 1, a + b <= 1, and the hit
// record (point, (theta, s) estimates, margin).  Every expression is
// evaluated as written with contraction off.
#pragma once

#include "ms_internal.hpp"

namespace ms {

constexpr double TWO_PI_D = 6.283185307179586476925286766559;

struct Tri { double p[3][4]; };

MS_D Tri load_tri(const MeshView &m, int32_t t)
{
    int32_t i1, i2, i3;
    tri_vertex_ids(m, t, i1, i2, i3);
    d4 a = load_d4(m.V + 4 * (int64_t)i1), b = load_d4(m.V + 4 * (int64_t)i2), c = load_d4(m.V + 4 * (int64_t)i3);
    return Tri{{{a.x, a.y, a.z, a.w}, {b.x, b.y, b.z, b.w}, {c.x, c.y, c.z, c.w}}};
}

// With n = (p1 - p2) x (p3 - p2) on the projection, Q is rejected when
// n.(q_j - p2) is > 0 for all three vertices or < 0 for all three.
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

// Pivot = first row of largest magnitude; an exact zero pivot means the
// system is singular (returns false).  Row swaps are selects on fully
// unrolled loops so the matrix stays in registers.
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

MS_D bool inside(const double z[4])
{
    double uv = z[0] + z[1], ab = z[2] + z[3];
    return (z[0] >= 0.0) && (z[1] >= 0.0) && (z[2] >= 0.0) && (z[3] >= 0.0) && (uv <= 1.0) && (ab <= 1.0);
}

// (theta, s) estimate on triangle t from its barycentrics (Sec. 6.2.4).
MS_D void tri_param(const MeshView &m, int32_t t, double u, double v, double &th, double &s)
{
    int32_t q = t >> 1, h = t & 1;
    int32_t k = q / m.nq, i = q - k * m.nq;
    double th0 = m.theta[i];
    double th1 = (i + 1 < m.n_theta_v) ? m.theta[i + 1] : m.theta[0] + TWO_PI_D;
    double s0 = m.s[k], s1 = m.s[k + 1];
    if (h == 0) {
        th = (1.0 - u) * th0 + u * th1;
        s = (1.0 - v) * s0 + v * s1;
    } else {
        th = u * th0 + (1.0 - u) * th1;
        s = v * s0 + (1.0 - v) * s1;
    }
    if (m.periodic && th >= TWO_PI_D) th = th - TWO_PI_D;
}

enum { PS_AABB = 0, PS_MOLLER = 1, PS_DEGEN = 2, PS_OUTSIDE = 3, PS_HIT = 4 };

// The full test without early exits: every stage is evaluated and the
// status decided at the end (box, Moller, singular, inclusion).
MS_D int pair_status_forced(const Tri &P, const Tri &Q, bool box_ok, double z[4])
{
    bool sep = same_side(P, Q) || same_side(Q, P);
    bool ok = solve_pair(P, Q, z);
    bool in = inside(z);
    return !box_ok ? PS_AABB : sep ? PS_MOLLER : !ok ? PS_DEGEN : !in ? PS_OUTSIDE : PS_HIT;
}

MS_D void make_hit(const MeshView &A, const MeshView &B, int32_t ta, int32_t tb, uint32_t tag, const Tri &P,
                   const double z[4], hit_t &h)
{
    double u = z[0], v = z[1], a = z[2], b = z[3];
    h.triA = ta; h.triB = tb; h.flags = tag; h.pad = 0;
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

}  // namespace ms
