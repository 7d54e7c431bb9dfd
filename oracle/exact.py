"""Exact rational evaluation of the triangle-pair test (test infrastructure).

Every double is an exact rational, so the AABB test, the Moller same-side
signs and the 4x4 system of the narrow phase (paper Sec. 6.2.2-6.2.4) can be
evaluated with no rounding at all using fractions.Fraction.  This is used to
pin the floating-point oracle on tiny meshes: both must agree except where the
exact answer sits within rounding distance of a decision boundary.
"""
from __future__ import annotations

from fractions import Fraction as Fr

import numpy as np


def fr(x) -> Fr:
    return Fr(float(x))


def tri_vertex_sets(mesh):
    """Triangles in the narrow-phase vertex order, written independently of
    oracle.c: triangle 2q+h of quad q = i + k*Nq, with
    T1: (W(i+1,k), W(i,k), W(i,k+1)) and T2: (W(i,k+1), W(i+1,k+1), W(i+1,k))."""
    V = mesh.verts
    nt, ns = mesh.n_theta_v, mesh.n_s_v
    nq = nt if mesh.periodic else nt - 1
    out = []
    for k in range(ns - 1):
        for i in range(nq):
            i1 = (i + 1) % nt
            out.append((V[k, i1], V[k, i], V[k + 1, i]))
            out.append((V[k + 1, i], V[k + 1, i1], V[k, i1]))
    # out is in quad order q = i + k*nq, triangle 2q then 2q+1
    return [np.array(t) for t in out]


def aabb_overlap(p, q) -> bool:
    for d in range(4):
        lo_p, hi_p = min(p[:, d]), max(p[:, d])
        lo_q, hi_q = min(q[:, d]), max(q[:, d])
        if lo_p > hi_q or lo_q > hi_p:
            return False
    return True


def moller_signs(p, q):
    """Exact f_j = n . (q_j - p2) on the (x, y, p_x) projection."""
    P = [[fr(p[j][d]) for d in range(3)] for j in range(3)]
    Q = [[fr(q[j][d]) for d in range(3)] for j in range(3)]
    e1 = [P[0][d] - P[1][d] for d in range(3)]
    e2 = [P[2][d] - P[1][d] for d in range(3)]
    n = [e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]]
    return [sum(n[d] * (Q[j][d] - P[1][d]) for d in range(3)) for j in range(3)]


def moller_reject_exact(p, q) -> bool:
    for (x, y) in ((p, q), (q, p)):
        f = moller_signs(x, y)
        if all(v > 0 for v in f) or all(v < 0 for v in f):
            return True
    return False


def solve_exact(p, q):
    """Exact solution z = (u, v, a, b) of p2 + (p1-p2)u + (p3-p2)v = q2 + (q1-q2)a + (q3-q2)b,
    or None when the system is singular."""
    P = [[fr(x) for x in row] for row in p]
    Q = [[fr(x) for x in row] for row in q]
    M = [[P[0][d] - P[1][d], P[2][d] - P[1][d], Q[1][d] - Q[0][d], Q[1][d] - Q[2][d], Q[1][d] - P[1][d]]
         for d in range(4)]
    # Gauss-Jordan with any nonzero pivot (exact arithmetic needs no pivoting strategy)
    for c in range(4):
        r = next((r for r in range(c, 4) if M[r][c] != 0), None)
        if r is None:
            return None
        M[c], M[r] = M[r], M[c]
        piv = M[c][c]
        M[c] = [x / piv for x in M[c]]
        for rr in range(4):
            if rr != c and M[rr][c] != 0:
                fct = M[rr][c]
                M[rr] = [x - fct * y for x, y in zip(M[rr], M[c])]
    return [M[i][4] for i in range(4)]


def margin_exact(z):
    u, v, a, b = z
    return min(u, v, a, b, 1 - u - v, 1 - a - b)


def predicate_exact(p, q):
    """(hit, kind, z, margin) for one pair in exact arithmetic: AABB, Moller, solve, inclusion."""
    if not aabb_overlap(p, q):
        return False, "aabb", None, None
    if moller_reject_exact(p, q):
        return False, "moller", None, None
    z = solve_exact(p, q)
    if z is None:
        return False, "degenerate", None, None
    m = margin_exact(z)
    return (m >= 0), ("hit" if m >= 0 else "outside"), z, m


def bruteforce_exact(meshA, meshB):
    """Exact hit set and per-pair exact margins for every AABB-passing pair."""
    TA = tri_vertex_sets(meshA)
    TB = tri_vertex_sets(meshB)
    hits, info = [], {}
    for ia, p in enumerate(TA):
        for ib, q in enumerate(TB):
            if not aabb_overlap(p, q):
                continue
            res = predicate_exact(p, q)
            info[(ia, ib)] = res
            if res[0]:
                hits.append((ia, ib))
    return hits, info
