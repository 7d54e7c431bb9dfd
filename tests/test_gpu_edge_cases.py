"""GPU parity of the narrow phase's edge cases and of the crowded-cell and
large-hit paths, HIP against the oracle on the same vertex bytes (Sec. 6.2.2-
6.2.4): planted affine hits with their exact parameters, margin-0 vertex and
edge contacts reported in every incident pair, coplanar (singular) pairs,
a hit in the periodic seam quad, more than 4096 hits (the hit ordering across
sort chunks) and cells too crowded for the on-chip staging of the
enumeration.  Each test asserts that its path was taken."""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

FLOAT_FIELDS = ("u", "v", "a", "b", "thA", "sA", "thB", "sB", "margin")
TOL = 1e-10


@pytest.fixture(scope="module")
def ms():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_14814_amd as ms
    ms.lib()
    return ms


def _pairs(h):
    return (h["triA"].astype(np.int64) << 32) | h["triB"].astype(np.int64)


def gpu_vs_oracle(ms, A, B, grid=None, kappa=1.0, hits_cap=1 << 10, cand_cap=1 << 16):
    """Search on the GPU and compare with the oracle's brute force and grid
    search: candidates and hits bit-exact, fields within TOL, counters equal.
    Returns (hits, stats, brute-force result)."""
    if grid is None:
        grid = oracle.default_grid([A, B], kappa)
    lo, _, inv, n = grid
    ref = oracle.bruteforce(A, B)
    gref = oracle.grid_search(A, B, lo, inv, n)
    assert np.array_equal(gref.cand, ref.cand) and gref.hits.tobytes() == ref.hits.tobytes()
    ga, gb = ms.Mesh.from_synth(A), ms.Mesh.from_synth(B)
    s = ms.Searcher(ga, gb, ms.make_params(lo, inv, n, ms.MS_SEARCH_CANDIDATES), hits_cap=hits_cap,
                    cand_cap=cand_cap)
    s.run()
    hits, st, cand = s.results()
    print(f"  nA={A.n_tris} nB={B.n_tris} hits={st['n_hits']} cand={st['n_cand']} "
          f"unstaged={st['n_chunks_unstaged']}", flush=True)
    assert st["overflow"] == 0
    assert np.array_equal(np.sort(cand), ref.cand)
    assert np.array_equal(_pairs(hits), ref.hit_pairs)
    for f in FLOAT_FIELDS:
        if len(hits):
            assert np.max(np.abs(hits[f] - ref.hits[f])) <= TOL, f
    if len(hits):
        assert np.max(np.abs(hits["X"] - ref.hits["X"])) <= TOL
    assert st["n_cand"] == len(ref.cand)
    assert st["n_moller"] == ref.counts["moller_reject"]
    assert st["n_degenerate"] == ref.counts["degenerate"]
    assert st["n_outside"] == ref.counts["outside"]
    assert st["n_hits"] == ref.counts["hits"]
    assert st["n_entries_all"] == gref.n_entries
    assert st["n_cells"] == gref.n_boxes and st["n_slots"] == gref.n_slots
    return hits, st, ref


UNIT = np.array([0.0, 1.0])


def _planted_affine(theta_star, s_star, theta2_star, s2_star, seed):
    """Two affine surfaces on dyadic grids meeting at one point (rational data)."""
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
    return synth.affine_mesh(P, D1, D2, grid, grid), synth.affine_mesh(Q, E1, E2, grid, grid), X


@pytest.mark.parametrize("pts", [(0.3125, 0.375, 0.5625, 0.5625), (0.4375, 0.375, 0.5625, 0.5625),
                                 (0.8125, 0.0625, 0.1875, 0.9375), (0.6875, 0.9375, 0.9375, 0.9375)])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_planted_affine_single_hit(ms, pts, seed):
    """One affine hit whose parameters are dyadic: the GPU returns exactly one
    hit, at the planted parameters."""
    A, B, X = _planted_affine(*pts, seed)
    hits, st, _ = gpu_vs_oracle(ms, A, B)
    assert st["n_hits"] == 1
    h = hits[0]
    assert abs(h["thA"] - pts[0]) < 1e-14 and abs(h["sA"] - pts[1]) < 1e-14
    assert abs(h["thB"] - pts[2]) < 1e-14 and abs(h["sB"] - pts[3]) < 1e-14
    assert np.max(np.abs(h["X"] - X)) < 1e-13


def test_hand_case_exact_values(ms):
    """A = unit square in (x, y), B = unit square in (p_x, p_y) through
    (0.25, 0.5, 0, 0): the only hit is (T1 of A, T2 of B) with (u, v) =
    (0.25, 0.5), (a, b) = (0.25, 0.625)."""
    A = synth.affine_mesh([0, 0, 0, 0], [1, 0, 0, 0], [0, 1, 0, 0], UNIT, UNIT)
    B = synth.affine_mesh([0.25, 0.5, -0.75, -0.375], [0, 0, 1, 0], [0, 0, 0, 1], UNIT, UNIT)
    hits, st, _ = gpu_vs_oracle(ms, A, B)
    assert [(int(h["triA"]), int(h["triB"])) for h in hits] == [(0, 1)]
    h = hits[0]
    assert (h["u"], h["v"], h["a"], h["b"]) == (0.25, 0.5, 0.25, 0.625)
    assert (h["thA"], h["sA"], h["thB"], h["sB"]) == (0.25, 0.5, 0.75, 0.375)
    assert list(h["X"]) == [0.25, 0.5, 0.0, 0.0]


def test_vertex_contact_margin_zero_every_incident_pair(ms):
    """B's corner sits on A's vertex (1, 0, 0, 0), which both of A's
    triangles share: both pairs are hits of margin exactly 0."""
    A = synth.affine_mesh([0, 0, 0, 0], [1, 0, 0, 0], [0, 1, 0, 0], UNIT, UNIT)
    B = synth.affine_mesh([1, 0, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1], UNIT, UNIT)
    hits, st, _ = gpu_vs_oracle(ms, A, B)
    assert sorted((int(h["triA"]), int(h["triB"])) for h in hits) == [(0, 0), (1, 0)]
    assert all(h["margin"] == 0.0 for h in hits)


def test_edge_contact_margin_zero_both_sides_of_the_diagonal(ms):
    """B's corner sits at (0.5, 0.5, 0, 0), the midpoint of the diagonal that
    splits A's quad: T1 (u = v = 0.5) and T2 (u = v = 0.5) both report it
    with margin 0."""
    A = synth.affine_mesh([0, 0, 0, 0], [1, 0, 0, 0], [0, 1, 0, 0], UNIT, UNIT)
    B = synth.affine_mesh([0.5, 0.5, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1], UNIT, UNIT)
    hits, st, _ = gpu_vs_oracle(ms, A, B)
    assert sorted(int(h["triA"]) for h in hits) == [0, 1]
    assert all(h["margin"] == 0.0 and h["u"] == 0.5 and h["v"] == 0.5 for h in hits)


def test_coplanar_pairs_are_degenerate(ms):
    """Overlapping triangles in one 2-plane: singular 4x4 systems, counted
    as degenerate, no hit."""
    A = synth.affine_mesh([0, 0, 0, 0], [1, 0, 0, 0], [0, 1, 0, 0], UNIT, UNIT)
    B = synth.affine_mesh([0.25, 0.25, 0, 0], [1, 0, 0, 0], [0, 1, 0, 0], UNIT, UNIT)
    hits, st, ref = gpu_vs_oracle(ms, A, B)
    assert st["n_hits"] == 0
    assert st["n_degenerate"] > 0 and st["n_degenerate"] == ref.counts["degenerate"]


def test_seam_quad_hit(ms):
    """A hit in the periodic seam quad (i = N - 1, joining theta_{N-1} and
    theta_0 + 2 pi): theta wraps into [0, 2 pi)."""
    N = 8
    A = synth.torus_mesh(N, 2, synth.surface_coeffs(3, noise_amp=0.0))
    ta = 2 * (N - 1)
    P = oracle.tri_verts(A, ta)
    u, v = 0.75, 0.125
    X = P[1] + u * (P[0] - P[1]) + v * (P[2] - P[1])
    E = np.random.default_rng(2).standard_normal((2, 4)) * 0.01
    B = synth.affine_mesh(X, E[0], E[1], np.array([-1.0, 1.0]), np.array([-1.0, 1.0]))
    hits, st, _ = gpu_vs_oracle(ms, A, B)
    mine = [h for h in hits if int(h["triA"]) == ta]
    assert mine
    h = mine[0]
    want = (1 - h["u"]) * A.theta[N - 1] + h["u"] * (A.theta[0] + 2 * math.pi)
    assert abs(h["thA"] - want) < 1e-12 and 0 <= h["thA"] < 2 * math.pi
    assert abs(h["u"] - u) < 1e-9 and abs(h["v"] - v) < 1e-9


@pytest.mark.parametrize("kappa", [1.0, 3.0])
def test_more_than_4096_hits(ms, kappa):
    """5,184 isolated crossings: the hit ordering sorts several chunks of
    4096 keys and merges them; the order equals the oracle's."""
    A, B = synth.lattice_plant(32, 288, 36)
    hits, st, _ = gpu_vs_oracle(ms, A, B, kappa=kappa, hits_cap=1 << 13, cand_cap=1 << 16)
    assert st["n_hits"] > 4096
    assert np.all(np.diff(_pairs(hits)) > 0)


@pytest.mark.parametrize("n_cells,power", [((2, 2, 1, 1), 3.0), ((1, 1, 1, 1), 1.0), ((1, 2, 1, 1), 1.0)])
def test_crowded_cells_unstaged_enumeration(ms, n_cells, power):
    """A coarse grid on the lattice plant: a cell holds up to all 2,048 plane
    triangles against tens of thousands of wave triangles, so enumeration
    chunks need more entries than fit on-chip and read their slots from
    device memory (n_chunks_unstaged > 0); with power 3 the plane's
    triangles crowd one column of cells, so staged and unstaged chunks mix."""
    A, B = synth.lattice_plant(32, 96, 12, power=power)
    lo = np.array([-0.02, -0.02, -0.05, -0.05])
    n = np.array(n_cells, np.int64)
    inv = 1.0 / (1.06 / float(max(n[0], n[1])))
    hits, st, _ = gpu_vs_oracle(ms, A, B, grid=(lo, None, inv, n), hits_cap=1 << 10, cand_cap=1 << 16)
    assert st["n_chunks_unstaged"] > 0
    if n_cells == (2, 2, 1, 1):
        chunks = -(-st["n_group_slots"] // 2048)      # the default work tile: 256 threads x 8 slots
        assert st["n_chunks_unstaged"] < chunks        # some chunks were staged
    assert st["n_hits"] > 0
