"""Pins of the oracle's mesh counts and uniform-grid search (paper Sec. 6.1,
6.2, 6.2.1): the grid search must reproduce the all-pairs definition exactly."""
import numpy as np
import pytest

import oracle
import synth


def test_paper_pair_counts():
    """Sec. 6.2: N1 = 1024, N2 = 2048, M1 = M2 = 35 give N(M-1) quads per mesh,
    2,424,307,712 quad pairs and 9,697,230,848 triangle pairs."""
    A = synth.Mesh(np.zeros((35, 1024, 4)), np.zeros(1024), np.zeros(35), True)
    B = synth.Mesh(np.zeros((35, 2048, 4)), np.zeros(2048), np.zeros(35), True)
    ta, tb = oracle.n_tris(A), oracle.n_tris(B)
    assert ta == 2 * 1024 * 34 and tb == 2 * 2048 * 34
    assert (ta // 2) * (tb // 2) == 2_424_307_712
    assert ta * tb == 9_697_230_848


@pytest.mark.parametrize("nt,ns,periodic,want", [
    (64, 65, True, 8192), (512, 513, True, 524288), (2049, 257, False, 1048576),
    (5, 1, True, 0), (1, 5, False, 0), (0, 0, True, 0), (3, 2, False, 4)])
def test_triangle_counts(nt, ns, periodic, want):
    m = synth.Mesh(np.zeros((ns, nt, 4)), np.zeros(nt), np.zeros(ns), periodic)
    assert oracle.n_tris(m) == want == m.n_tris


def test_triangle_vertex_sets_independent_listing():
    """Each triangle's vertex list matches an independent listing of the
    quads of Sec. 6.1 split along W(i+1,k)-W(i,k+1), with the periodic wrap."""
    from oracle import exact
    for periodic in (True, False):
        rng = np.random.default_rng(1)
        V = rng.standard_normal((4, 5, 4))
        m = synth.Mesh(V, np.arange(5.0), np.arange(4.0), periodic)
        ref = exact.tri_vertex_sets(m)
        assert len(ref) == oracle.n_tris(m)
        for t, tri in enumerate(ref):
            assert np.array_equal(oracle.tri_verts(m, t), tri)


def _cfg0(seed=0, n=64):
    return synth.plain_pair(n, n, seed)


@pytest.mark.parametrize("kappa", [0.5, 1.0, 2.0, 4.0])
def test_grid_equals_bruteforce_cfg0(kappa):
    A, B = _cfg0()
    bf = oracle.bruteforce(A, B)
    lo, hi, inv, n = oracle.default_grid([A, B], kappa)
    g = oracle.grid_search(A, B, lo, inv, n)
    assert np.array_equal(g.cand, bf.cand)
    assert g.hits.tobytes() == bf.hits.tobytes()
    assert g.n_entries == oracle.grid_entries(A, lo, inv, n) + oracle.grid_entries(B, lo, inv, n)
    assert len(bf.hits) > 0


def test_grid_invariant_to_world_shift_and_tiny_cells():
    """Results do not depend on the world origin or on the cell edge, down to
    cells much smaller than the triangles."""
    A, B = _cfg0(seed=3, n=24)
    bf = oracle.bruteforce(A, B)
    lo, hi, inv, n = oracle.default_grid([A, B], 1.0)
    for shift, scale in [(0.0, 1.0), (0.37, 1.0), (-0.11, 3.0), (0.05, 0.25)]:
        inv2 = inv * scale
        lo2 = lo - shift / inv2
        n2 = np.ceil((hi - lo2) * inv2).astype(np.int64) + 1
        g = oracle.grid_search(A, B, lo2, inv2, n2)
        assert np.array_equal(g.cand, bf.cand)
        assert g.hits.tobytes() == bf.hits.tobytes()


def test_grid_world_smaller_than_meshes_clamps():
    """Cells outside the world clamp into the border cells: still exact."""
    A, B = _cfg0(seed=4, n=24)
    bf = oracle.bruteforce(A, B)
    lo, hi, inv, n = oracle.default_grid([A, B], 1.0)
    lo2 = lo + 0.4 * (hi - lo)
    n2 = np.maximum(1, (n * 0.3).astype(np.int64))
    g = oracle.grid_search(A, B, lo2, inv, n2)
    assert np.array_equal(g.cand, bf.cand)
    assert g.hits.tobytes() == bf.hits.tobytes()


@pytest.mark.parametrize("crop", [(96, 0), (128, 1), (224, 0), (320, 2), (448, 0)])
def test_grid_equals_bruteforce_on_512_crops(crop):
    """16 x 16 crops of the 512^2 workload, near the s = 0 band where the two
    surfaces meet."""
    A, B = synth.plain_pair(512, 512, 0)
    i0, k0 = crop
    a = synth.crop(A, i0, 16, k0, 16)
    b = synth.crop(B, i0, 16, k0, 16)
    bf = oracle.bruteforce(a, b)
    for kappa in (0.5, 2.0):
        lo, hi, inv, n = oracle.default_grid([a, b], kappa)
        g = oracle.grid_search(a, b, lo, inv, n)
        assert np.array_equal(g.cand, bf.cand)
        assert g.hits.tobytes() == bf.hits.tobytes()
    assert len(bf.cand) > 0


def test_swap_transposes_candidates():
    A, B = _cfg0(seed=1)
    ab = oracle.bruteforce(A, B)
    ba = oracle.bruteforce(B, A)
    t = np.sort(((ba.cand & 0xffffffff) << 32) | (ba.cand >> 32))
    assert np.array_equal(t, ab.cand)
    hab = {(int(h["triA"]), int(h["triB"])): h for h in ab.hits}
    hba = {(int(h["triB"]), int(h["triA"])): h for h in ba.hits}
    for k in hab.keys() ^ hba.keys():
        h = hab.get(k, None)
        h = h if h is not None else hba[k]
        assert abs(h["margin"]) < 1e-12
    for k in hab.keys() & hba.keys():
        assert abs(hab[k]["u"] - hba[k]["a"]) < 1e-10 and abs(hab[k]["b"] - hba[k]["v"]) < 1e-10


def test_nonfinite_vertices_are_excluded_and_counted():
    A, B = _cfg0(seed=2, n=16)
    A.verts = A.verts.copy()
    A.verts[3, 5, 2] = np.nan       # touches up to 6 triangles
    A.verts[7, 0, 0] = np.inf
    bf = oracle.bruteforce(A, B)
    assert bf.counts["nonfinite_A"] == 12
    lo, hi, inv, n = oracle.default_grid([A, B], 1.0)
    g = oracle.grid_search(A, B, lo, inv, n)
    assert np.array_equal(g.cand, bf.cand)
    assert g.hits.tobytes() == bf.hits.tobytes()
    bad = set()
    for t in range(oracle.n_tris(A)):
        if not np.all(np.isfinite(oracle.tri_verts(A, t))):
            bad.add(t)
    assert len(bad) == 12
    assert not any((int(c) >> 32) in bad for c in bf.cand)


def test_empty_meshes():
    A, B = _cfg0(n=8)
    E = synth.Mesh(np.zeros((1, 8, 4)), np.zeros(8), np.zeros(1), True)
    for x, y in ((A, E), (E, B), (E, E)):
        r = oracle.bruteforce(x, y)
        assert len(r.cand) == 0 and len(r.hits) == 0
        lo, hi, inv, n = oracle.default_grid([A, B], 1.0)
        g = oracle.grid_search(x, y, lo, inv, n)
        assert len(g.cand) == 0 and len(g.hits) == 0


# --------------------------------------------------- world-bound pruning

def _shifted_pair(n, shift, seed=0):
    """The plain pair with B moved along x, so that part of each mesh lies
    outside the other's box."""
    A, B = synth.plain_pair(n, n, seed)
    V = B.verts.copy()
    V[..., 0] += shift
    return A, synth.Mesh(V, B.theta, B.s, B.periodic)


def _tri_boxes(m):
    boxes = []
    for t in range(oracle.n_tris(m)):
        v = oracle.tri_verts(m, t)
        boxes.append((v.min(axis=0), v.max(axis=0), bool(np.all(np.isfinite(v)))))
    return boxes


def _pruned_stats_numpy(A, B, grid):
    """Boxes and slots of the restricted grid of Sec. 6.2.1, counted
    independently: the triangles whose box meets the other mesh's box (over
    its finite vertices), their cells, and per cell nA * nB."""
    lo, _, inv, n = grid
    bx = [_tri_boxes(A), _tri_boxes(B)]
    mb = []
    for m in (A, B):
        v = m.verts.reshape(-1, 4)
        v = v[np.all(np.isfinite(v), axis=1)]
        mb.append((v.min(axis=0), v.max(axis=0)))
    counts = {}
    kept = [0, 0]
    for sd, (m, boxes) in enumerate(zip((A, B), bx)):
        olo, ohi = mb[1 - sd]
        for t, (tlo, thi, fin) in enumerate(boxes):
            if not fin or not (np.all(tlo <= ohi) and np.all(olo <= thi)):
                continue
            kept[sd] += 1
            for c in oracle.tri_entries(m, t, lo, inv, n):
                counts.setdefault(int(c), [0, 0])[sd] += 1
    both = [v for v in counts.values() if v[0] and v[1]]
    return len(both), sum(a * b for a, b in both), kept


@pytest.mark.parametrize("shift", [0.0, 0.9, 1.7])
def test_pruning_keeps_hits_and_candidates(shift):
    """The restricted grid finds the same candidates and hits (no pair with a
    triangle outside the other mesh's box has overlapping boxes), counts the
    same entries before the restriction, and its boxes and slots are those
    of the triangles that meet the other mesh's box."""
    A, B = _shifted_pair(24, shift)
    grid = oracle.default_grid([A, B], 1.0)
    full = oracle.grid_search(A, B, grid[0], grid[2], grid[3])
    pr = oracle.grid_search(A, B, grid[0], grid[2], grid[3], prune=True)
    assert np.array_equal(pr.cand, full.cand)
    assert np.array_equal(pr.hits["triA"], full.hits["triA"]) and np.array_equal(pr.hits["triB"], full.hits["triB"])
    assert pr.n_entries == full.n_entries
    nb, ns, kept = _pruned_stats_numpy(A, B, grid)
    assert (pr.n_boxes, pr.n_slots) == (nb, ns)
    if shift == 0.0:
        assert (pr.n_boxes, pr.n_slots) == (full.n_boxes, full.n_slots)
    else:
        # the shifted pair loses triangles on both sides (and slots, where
        # a lost triangle shared a cell with the other mesh)
        assert kept[0] < oracle.n_tris(A) and kept[1] < oracle.n_tris(B)
        assert pr.n_slots <= full.n_slots


def test_pruning_with_nonfinite_triangles():
    """A vertex made NaN leaves the mesh's box and removes its triangles:
    the restricted grid still equals the independent count."""
    A, B = _shifted_pair(16, 1.2, seed=3)
    V = A.verts.copy()
    V[3, 5, 1] = np.nan
    A = synth.Mesh(V, A.theta, A.s, A.periodic)
    grid = oracle.default_grid([A, B], 1.5)
    full = oracle.grid_search(A, B, grid[0], grid[2], grid[3])
    pr = oracle.grid_search(A, B, grid[0], grid[2], grid[3], prune=True)
    assert np.array_equal(pr.cand, full.cand)
    nb, ns, _ = _pruned_stats_numpy(A, B, grid)
    assert (pr.n_boxes, pr.n_slots) == (nb, ns)
