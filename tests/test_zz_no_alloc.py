"""The search entry point that allocates nothing (search_intersections_noalloc,
its workspace a fixed device array inside the library) against the search
with a caller workspace (search_intersections), through the C ABI: two calls
in a row on the same fixed array, the second with smaller meshes.  Both run
the same kernels, so hit records, candidate sets and the exact counters must
be identical; the hits are also held to the oracle's."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

EXACT = ("n_entries_all", "n_cells", "n_slots", "n_cand", "n_moller", "n_degenerate", "n_outside", "n_hits",
         "n_nonfinite", "overflow")
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


def _noalloc(ms, ga, gb, p, hits_cap, cand_cap):
    import torch
    hits = torch.empty(hits_cap * ms.HIT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    stats = torch.zeros(16, dtype=torch.int64, device="cuda")
    cand = torch.empty(cand_cap, dtype=torch.int64, device="cuda")
    ms.search_noalloc(ga, gb, p, hits, stats, cand)
    torch.cuda.synchronize()
    st = {k: int(v) for k, v in zip(ms.STATS_FIELDS, stats.cpu().numpy())}
    nh = min(st["n_hits"], hits_cap)
    h = np.frombuffer(hits[: nh * ms.HIT_DTYPE.itemsize].cpu().numpy().tobytes(), dtype=ms.HIT_DTYPE)
    c = np.sort(cand[: min(st["n_cand"], cand_cap)].cpu().numpy())
    return h, st, c


@pytest.mark.parametrize("n", [(512, 512, 1.5), (64, 64, 2.0)], ids=["512x512", "64x64"])
def test_noalloc_equals_workspace_search(ms, n):
    """First call 512x512 quads per surface (the table size lowered to fit the
    fixed array), second 64x64: each equal to the workspace search."""
    nt, ns, kappa = n
    A, B = synth.plain_pair(nt, ns, 0)
    ga, gb = ms.Mesh.from_synth(A), ms.Mesh.from_synth(B)
    p = ms.default_params(ga, gb, kappa)
    p.flags = ms.MS_SEARCH_CANDIDATES
    print(f"noalloc case {nt}x{ns} kappa {kappa}", flush=True)
    s = ms.Searcher(ga, gb, p, hits_cap=1 << 12, cand_cap=1 << 18)
    s.run()
    want_h, want_st, want_c = s.results()
    want_c = np.sort(want_c)
    got_h, got_st, got_c = _noalloc(ms, ga, gb, p, 1 << 12, 1 << 18)
    for k in EXACT:
        assert got_st[k] == want_st[k], (k, got_st[k], want_st[k])
    assert got_st["overflow"] == 0
    assert np.array_equal(got_c, want_c)
    assert got_h.tobytes() == want_h.tobytes()
    if nt == 64:
        ref = oracle.bruteforce(A, B)
        assert np.array_equal(_pairs(got_h), _pairs(ref.hits))
        for f in FLOAT_FIELDS:
            assert np.max(np.abs(got_h[f] - ref.hits[f])) <= 1e-10 if len(got_h) else True
        assert np.array_equal(got_c, ref.cand)


def test_noalloc_rejects_what_does_not_fit(ms):
    """An explicit hashed table of 2^25 per side needs more than the fixed
    array: a clear MS_E_WORKSPACE, nothing queued."""
    import torch
    A, B = synth.plain_pair(64, 64, 1)
    ga, gb = ms.Mesh.from_synth(A), ms.Mesh.from_synth(B)
    p = ms.default_params(ga, gb, 2.0)
    p.table_log2 = 25
    hits = torch.empty(16 * ms.HIT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    stats = torch.zeros(16, dtype=torch.int64, device="cuda")
    with pytest.raises(ms.MSearchError) as ei:
        ms.search_noalloc(ga, gb, p, hits, stats)
    assert ei.value.code == ms.MS_E_WORKSPACE
    assert "fixed scratch" in str(ei.value)
