"""GPU parity of the layer search (Sec. 5 / 6.2): the half-layer pairs of an
unstable and a stable mesh, each half-layer a column sub-mesh sharing the
vertices, searched as one batch; per pair against the oracle (brute force
on the same half-layer meshes) and against plain searches."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

FLOAT_FIELDS = ("u", "v", "a", "b", "thA", "sA", "thB", "sB", "margin")


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


def assert_same_hits(got, want):
    assert np.array_equal(_pairs(got), _pairs(want)), (len(got), len(want))
    for f in FLOAT_FIELDS:
        if len(got):
            assert np.max(np.abs(got[f] - want[f])) <= 1e-10, f


def half(mesh, k):
    return synth.Mesh(np.ascontiguousarray(mesh.verts[k[0]:k[1] + 1]), mesh.theta, mesh.s[k[0]:k[1] + 1].copy(),
                      mesh.periodic)


@pytest.mark.parametrize("seed,kappa", [(0, 1.0), (3, 2.0)])
def test_layer_search_matches_oracle_per_pair(ms, seed, kappa):
    lp = synth.layered_pair(64, 96, 6, 3, seed)
    U, S = ms.Mesh.from_synth(lp.U), ms.Mesh.from_synth(lp.S)
    ls = ms.LayerSearch(U, S, lp.D_u, lp.lam_u, lp.D_s, lp.lam_s, lp.n_layers, kappa=kappa, hits_cap=1 << 14)
    ls.run(True)
    per_pair, st = ls.results()
    assert st["overflow"] == 0 and len(per_pair) == 24
    tot_c = tot_h = 0
    for p, hits in zip(oracle.layer_pairs(lp.n_layers), per_pair):
        n, a, m, b = p
        ku = oracle.half_layer_columns(lp.U.s, lp.D_u, lp.lam_u, False, n, a)
        ks = oracle.half_layer_columns(lp.S.s, lp.D_s, lp.lam_s, True, m, b)
        ref = oracle.bruteforce(half(lp.U, ku), half(lp.S, ks))
        assert_same_hits(hits, ref.hits)
        tot_c += len(ref.cand)
        tot_h += len(ref.hits)
    assert st["n_cand"] == tot_c and st["n_hits"] == tot_h
    assert tot_h > 0


def test_layer_search_equals_plain_searches(ms):
    """A larger layered pair (8 layers, 64 half-layer pairs): the batched
    layer search, eager and as a graph, gives each pair's plain search."""
    lp = synth.layered_pair(256, 384, 12, 8, 5)
    U, S = ms.Mesh.from_synth(lp.U), ms.Mesh.from_synth(lp.S)
    ls = ms.LayerSearch(U, S, lp.D_u, lp.lam_u, lp.D_s, lp.lam_s, lp.n_layers, kappa=1.5, hits_cap=1 << 16)
    got = []
    for use_graph in (False, True):
        ls.run(use_graph)
        got.append(ls.results())
    (h0, st0), (h1, st1) = got
    assert st0 == st1
    tot = 0
    for (a, b), p, x0, x1 in zip(ls.meshes, ls.params, h0, h1):
        hits, st, _ = ms.search(a, b, p, hits_cap=1 << 12, cand_cap=1 << 18)
        assert_same_hits(x0, hits)
        assert_same_hits(x1, hits)
        tot += len(hits)
    assert tot == st0["n_hits"] and tot > 0


def test_pruned_layer_search(ms):
    """The layer search with and without world-bound pruning: the same hits
    and candidates per pair; the cells and slots of each pair equal the
    oracle's restricted grid."""
    lp = synth.layered_pair(64, 96, 6, 3, 2)
    U, S = ms.Mesh.from_synth(lp.U), ms.Mesh.from_synth(lp.S)
    ls_p = ms.LayerSearch(U, S, lp.D_u, lp.lam_u, lp.D_s, lp.lam_s, lp.n_layers, kappa=1.5, hits_cap=1 << 14)
    ls_f = ms.LayerSearch(U, S, lp.D_u, lp.lam_u, lp.D_s, lp.lam_s, lp.n_layers, kappa=1.5, hits_cap=1 << 14,
                          prune=False)
    ls_p.run(True)
    ls_f.run(True)
    hp, stp = ls_p.results()
    hf, stf = ls_f.results()
    for x, y in zip(hp, hf):
        assert_same_hits(x, y)
    assert stp["n_cand"] == stf["n_cand"] and stp["n_entries_all"] == stf["n_entries_all"]
    cells = slots = 0
    for (a, b), p in zip(ls_p.meshes, ls_p.params):
        assert p.flags & ms.MS_SEARCH_PRUNE
    for p in oracle.layer_pairs(lp.n_layers):
        n, sa, m, sb = p
        ku = oracle.half_layer_columns(lp.U.s, lp.D_u, lp.lam_u, False, n, sa)
        ks = oracle.half_layer_columns(lp.S.s, lp.D_s, lp.lam_s, True, m, sb)
        A, B = half(lp.U, ku), half(lp.S, ks)
        g = oracle.default_grid([A, B], 1.5)
        ref = oracle.grid_search(A, B, g[0], g[2], g[3], prune=True)
        cells += ref.n_boxes
        slots += ref.n_slots
    assert (stp["n_cells"], stp["n_slots"]) == (cells, slots)
    assert stp["n_slots"] <= stf["n_slots"]


def test_full_size_layer_search_equals_plain_searches(ms):
    """The layer search at the paper's shape (112 half-layer pairs, 25M
    triangles: more tiles than k_mark's grid, so each block marks a run of
    two tiles), at its tuned tuple with world-bound pruning: every pair's
    hits equal its plain search's (same grid, tile and pruning, its own
    table size), and the batch's counts equal the plain searches' sums."""
    lp = synth.layered_pair(1024, 2048, 34, 14, 0)
    U, S = ms.Mesh.from_synth(lp.U), ms.Mesh.from_synth(lp.S)
    ls = ms.LayerSearch(U, S, lp.D_u, lp.lam_u, lp.D_s, lp.lam_s, lp.n_layers, hits_cap=1 << 16)
    assert len(ls.meshes) == 112
    assert sum(a.n_tris + b.n_tris for a, b in ls.meshes) > 512 * 32768
    ls.run(True)
    per_pair, st = ls.results()
    sums = dict.fromkeys(("n_cand", "n_hits", "n_cells", "n_slots"), 0)
    for (a, b), p, got in zip(ls.meshes, ls.params, per_pair):
        q = type(p).from_buffer_copy(p)
        q.table_log2 = 0
        hits, pst, _ = ms.search(a, b, q, hits_cap=1 << 12, cand_cap=1 << 18)
        assert_same_hits(got, hits)
        for k in sums:
            sums[k] += pst[k]
    assert all(st[k] == v for k, v in sums.items()), (st, sums)
    assert st["n_hits"] > 0
