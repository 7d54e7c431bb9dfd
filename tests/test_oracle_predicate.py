"""Pins of the oracle's triangle-pair predicate against exact arithmetic and
closed-form plants (paper Sec. 6.1, 6.2.2-6.2.4)."""
from fractions import Fraction as Fr
import math

import numpy as np
import pytest

import oracle
from oracle import exact
import synth


def _planted_affine(theta_star, s_star, theta2_star, s2_star, seed=0):
    """Two affine surfaces on dyadic grids that meet at exactly one point:
    A(th, s) = P + th D1 + s D2 and B(th', s') = Q + th' E1 + s' E2 with
    Q chosen so that A(th*, s*) = B(th'*, s'*)."""
    rng = np.random.default_rng(seed)
    while True:
        D = rng.integers(-4, 5, size=(4, 4)).astype(np.float64)
        if abs(np.linalg.det(D)) > 4:
            break
    P = rng.integers(-8, 9, size=4).astype(np.float64) / 8.0
    D1, D2, E1, E2 = D
    X = P + theta_star * D1 + s_star * D2
    Q = X - theta2_star * E1 - s2_star * E2
    grid = np.arange(5) / 4.0
    A = synth.affine_mesh(P, D1, D2, grid, grid)
    B = synth.affine_mesh(Q, E1, E2, grid, grid)
    return A, B, X


@pytest.mark.parametrize("pts", [
    (0.3125, 0.375, 0.5625, 0.5625),    # T1 on A (local 0.25, 0.5), T1 on B (local 0.25, 0.25)
    (0.4375, 0.375, 0.5625, 0.5625),    # T2 on A (local 0.75, 0.5), T1 on B
    (0.8125, 0.0625, 0.1875, 0.9375),   # T1 (0.25, 0.25) / T2 (0.75, 0.75)
    (0.6875, 0.9375, 0.9375, 0.9375),   # T2 (0.75, 0.75) / T2 (0.75, 0.75)
])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_planted_affine_single_hit(pts, seed):
    th1, s1, th2, s2 = pts
    A, B, X = _planted_affine(th1, s1, th2, s2, seed)
    res = oracle.bruteforce(A, B)
    assert len(res.hits) == 1, res.counts
    h = res.hits[0]
    # the planted parameters are recovered (the mesh is exact for an affine surface)
    assert abs(h["thA"] - th1) < 1e-14 and abs(h["sA"] - s1) < 1e-14
    assert abs(h["thB"] - th2) < 1e-14 and abs(h["sB"] - s2) < 1e-14
    assert np.max(np.abs(h["X"] - X)) < 1e-13
    # barycentrics agree with the exact rational solution
    ta, tb = int(h["triA"]), int(h["triB"])
    z = exact.solve_exact(oracle.tri_verts(A, ta), oracle.tri_verts(B, tb))
    for got, want in zip((h["u"], h["v"], h["a"], h["b"]), z):
        assert abs(got - float(want)) < 1e-14
    assert h["margin"] > 0.05


def test_parameter_formulas_hand_case():
    """One quad per mesh, written out by hand: A is the unit square in the
    (x, y) plane, B the unit square in the (p_x, p_y) plane shifted so that
    they meet at (x, y) = (0.25, 0.5)."""
    th = np.array([0.0, 1.0]); s = np.array([0.0, 1.0])
    A = synth.affine_mesh([0, 0, 0, 0], [1, 0, 0, 0], [0, 1, 0, 0], th, s)
    B = synth.affine_mesh([0.25, 0.5, -0.75, -0.375], [0, 0, 1, 0], [0, 0, 0, 1], th, s)
    res = oracle.bruteforce(A, B)
    assert [(int(h["triA"]), int(h["triB"])) for h in res.hits] == [(0, 1)]
    h = res.hits[0]
    # A's T1 has p2 = W(0,0), p1 = W(1,0), p3 = W(0,1): the point (0.25, 0.5) has u = 0.25, v = 0.5
    assert (h["u"], h["v"]) == (0.25, 0.5)
    # B's T2 has p2 = W(1,1) = (., ., 0.25, 0.625), p1 = W(0,1), p3 = W(1,0); point is (0.75, 0.375) in B's params
    assert (h["a"], h["b"]) == (0.25, 0.625)
    assert (h["thA"], h["sA"], h["thB"], h["sB"]) == (0.25, 0.5, 0.75, 0.375)
    assert list(h["X"]) == [0.25, 0.5, 0.0, 0.0]


def test_inclusive_boundary_vertex_and_edge():
    """Touching counts (closed triangles): a shared vertex is a hit of
    margin 0, in every incident pair."""
    th = np.array([0.0, 1.0]); s = np.array([0.0, 1.0])
    A = synth.affine_mesh([0, 0, 0, 0], [1, 0, 0, 0], [0, 1, 0, 0], th, s)
    # B's corner W(0,0) sits on A's vertex (1, 0): B spans the (p_x, p_y) plane through it
    B = synth.affine_mesh([1, 0, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1], th, s)
    res = oracle.bruteforce(A, B)
    pairs = sorted((int(h["triA"]), int(h["triB"])) for h in res.hits)
    # vertex (1,0) of A is in both of A's triangles; B's W(0,0) is only in B's T1
    assert pairs == [(0, 0), (1, 0)]
    assert all(h["margin"] == 0.0 for h in res.hits)


def test_coplanar_is_degenerate():
    """Two triangles in one 2-plane: the 4x4 system is singular."""
    th = np.array([0.0, 1.0]); s = np.array([0.0, 1.0])
    A = synth.affine_mesh([0, 0, 0, 0], [1, 0, 0, 0], [0, 1, 0, 0], th, s)
    B = synth.affine_mesh([0.25, 0.25, 0, 0], [1, 0, 0, 0], [0, 1, 0, 0], th, s)
    res = oracle.bruteforce(A, B)
    assert len(res.hits) == 0
    assert res.counts["degenerate"] > 0


def test_solve4_matches_library_solve():
    """On well-conditioned random systems the GEPP solve agrees with LAPACK."""
    rng = np.random.default_rng(5)
    for _ in range(200):
        p = rng.standard_normal((3, 4)); q = rng.standard_normal((3, 4))
        M = np.stack([p[0] - p[1], p[2] - p[1], q[1] - q[0], q[1] - q[2]], axis=1)
        if np.linalg.cond(M) > 1e4:
            continue
        ok, z = oracle.solve4(p, q)
        assert ok
        zref = np.linalg.solve(M, q[1] - p[1])
        assert np.max(np.abs(z - zref)) < 1e-12 * max(1.0, np.max(np.abs(zref)))


def test_moller_is_conservative_in_exact_arithmetic():
    """A true intersection point of the two planes inside both triangles is
    never rejected by the same-side test (checked exactly and in FP)."""
    rng = np.random.default_rng(11)
    n_checked = 0
    for _ in range(400):
        p = rng.standard_normal((3, 4))
        u, v = rng.uniform(0, 0.5, size=2)
        a, b = rng.uniform(0, 0.5, size=2)
        X = p[1] + u * (p[0] - p[1]) + v * (p[2] - p[1])
        E = rng.standard_normal((2, 4))
        q1 = X + E[0] * 1.0; q3 = X + E[1] * 1.0
        # q2 such that X = q2 + a (q1 - q2) + b (q3 - q2)
        q2 = (X - a * q1 - b * q3) / (1 - a - b)
        q = np.stack([q1, q2, q3])
        assert not exact.moller_reject_exact(p, q)
        assert not oracle.moller_reject(p, q)
        n_checked += 1
    assert n_checked == 400


def _tiny_random_meshes(seed, n=6, m=6, scale=0.4):
    """Small curved meshes, nearly graphs over (x, y), whose (p_x, p_y)
    components oscillate along different axes so that they cross at a few
    isolated points."""
    rng = np.random.default_rng(seed)
    th = np.linspace(0, 1, n + 1); s = np.linspace(0, 1, m + 1)
    T, S = np.meshgrid(th, s)
    c = rng.uniform(0, 6.3, 8)

    def surf(c, swap):
        x = T + 0.05 * np.sin(3 * S + c[0]); y = S + 0.05 * np.cos(2 * T + c[1])
        if swap:
            z = scale * np.sin(5 * y + c[2]); w = scale * np.cos(4 * x + c[3])
        else:
            z = scale * np.sin(5 * x + c[2]); w = scale * np.cos(4 * y + c[3])
        return np.ascontiguousarray(np.stack([x, y, z, w], -1))
    return (synth.Mesh(surf(c[:4], False), th, s, False),
            synth.Mesh(surf(c[4:], True), th, s, False))


@pytest.mark.parametrize("seed", [0, 1, 2, 4, 5, 6, 7])
def test_fp_predicate_matches_exact_bruteforce(seed):
    """FP-P equals exact-P on every pair except those whose exact margin is
    within 1e-12 of the inclusion boundary; the FP (u, v, a, b) agree with the
    exact ones to 1e-12 on the agreeing hits."""
    A, B = _tiny_random_meshes(seed)
    fp = oracle.bruteforce(A, B)
    ex_hits, info = exact.bruteforce_exact(A, B)
    fp_set = {(int(h["triA"]), int(h["triB"])): h for h in fp.hits}
    ex_set = set(ex_hits)
    for pr in fp_set.keys() ^ ex_set:
        hit, kind, z, m = info[pr]
        assert m is not None and abs(m) < 1e-12, (pr, kind, m)
    for pr in fp_set.keys() & ex_set:
        z = info[pr][2]
        h = fp_set[pr]
        for got, want in zip((h["u"], h["v"], h["a"], h["b"]), z):
            assert abs(got - float(want)) < 1e-12
    # the candidate set is exactly the AABB-overlap set
    assert sorted(info.keys()) == sorted((int(c) >> 32, int(c) & 0xffffffff) for c in fp.cand)
    assert len(ex_set) > 0


def test_curved_plant_second_order():
    """Graph surfaces A = (x, y, g, h) and B = (k, l, z, w) with a designed
    common point: the mesh hit converges to it at second order in the mesh
    spacing (the error of linear interpolation)."""
    x0, y0, z0, w0 = 0.3, 0.45, 0.2, -0.1
    g = lambda x, y: z0 + 0.8 * (x - x0) ** 2 - 0.5 * (y - y0) + 0.3 * (x - x0)
    hh = lambda x, y: w0 + 0.6 * (y - y0) ** 2 + 0.4 * (x - x0) - 0.2 * (y - y0)
    k = lambda z, w: x0 + 0.7 * (w - w0) ** 2 + 0.5 * (z - z0)
    l = lambda z, w: y0 - 0.9 * (z - z0) ** 2 + 0.3 * (w - w0)
    errs = []
    for n in (8, 16, 32, 64):
        u = np.linspace(0, 1, n + 1)
        X, Y = np.meshgrid(u, u)
        A = synth.Mesh(np.ascontiguousarray(np.stack([X, Y, g(X, Y), hh(X, Y)], -1)), u, u, False)
        zz = np.linspace(z0 - 0.5, z0 + 0.5, n + 1); ww = np.linspace(w0 - 0.5, w0 + 0.5, n + 1)
        Z, W = np.meshgrid(zz, ww)
        B = synth.Mesh(np.ascontiguousarray(np.stack([k(Z, W), l(Z, W), Z, W], -1)), zz, ww, False)
        res = oracle.bruteforce(A, B)
        assert len(res.hits) >= 1
        d = min(np.max(np.abs(h["X"] - np.array([x0, y0, z0, w0]))) for h in res.hits)
        dp = min(max(abs(h["thA"] - x0), abs(h["sA"] - y0), abs(h["thB"] - z0), abs(h["sB"] - w0))
                 for h in res.hits)
        errs.append(max(d, dp))
    # the error constant depends on where the point falls inside its triangle,
    # so take the rate over the whole refinement (3 halvings) and bound each level
    rate = math.log2(errs[0] / errs[-1]) / (len(errs) - 1)
    assert rate > 1.8, errs
    assert all(e < 0.5 * (1.0 / n) ** 2 for e, n in zip(errs, (8, 16, 32, 64))), errs


def test_periodic_seam_parameters():
    """A hit in the seam quad (i = N-1) reports theta between th_{N-1} and
    2 pi, wrapped into [0, 2 pi)."""
    N, M = 8, 2
    c = synth.surface_coeffs(3, noise_amp=0.0)
    A = synth.torus_mesh(N, M, c)
    nq = N
    k = 0
    q = (N - 1) + k * nq
    ta = 2 * q                 # T1 of the seam quad
    P = oracle.tri_verts(A, ta)
    u, v = 0.75, 0.125
    X = P[1] + u * (P[0] - P[1]) + v * (P[2] - P[1])
    # B: a small transversal affine patch through X, in general position
    rng = np.random.default_rng(2)
    E = rng.standard_normal((2, 4)) * 0.01
    grid = np.array([-1.0, 1.0])
    B = synth.affine_mesh(X, E[0], E[1], grid, grid)
    res = oracle.bruteforce(A, B)
    mine = [h for h in res.hits if int(h["triA"]) == ta]
    assert mine, res.counts
    h = mine[0]
    th_prev = A.theta[N - 1]
    want = (1 - h["u"]) * th_prev + h["u"] * (A.theta[0] + 2 * math.pi)
    assert abs(h["thA"] - want) < 1e-12 and 0 <= h["thA"] < 2 * math.pi
    assert abs(h["u"] - u) < 1e-9 and abs(h["v"] - v) < 1e-9
    assert abs(h["sA"] - ((1 - h["v"]) * A.s[0] + h["v"] * A.s[1])) < 1e-15
