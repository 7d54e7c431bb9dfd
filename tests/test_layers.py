"""The method of layers (Sec. 5): the half-layer pair schedule and the
half-layer column ranges, oracle pins and the C-ABI host functions against
the oracle (no GPU needed)."""
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "layers_sec6_4.txt")


def golden():
    out = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            out[k] = int(v)
    return out


def test_oracle_schedule_matches_the_paper_counts():
    g = golden()
    pairs = oracle.layer_pairs(g["layers"])
    assert len(pairs) == g["total_pairs"] == g["layers"] * g["pairs_per_layer"]
    assert len(set(pairs)) == len(pairs)


def test_oracle_schedule_structure():
    """(U_n, S_n) and (U_n, S_(n-1)) for n >= 1, every sign combination once."""
    for L in range(0, 6):
        pairs = oracle.layer_pairs(L)
        want = {(n, a, m, b) for n in range(1, L + 1) for m in (n, n - 1) for a in (1, -1) for b in (1, -1)}
        assert set(pairs) == want
        assert [p[0] for p in pairs] == sorted(p[0] for p in pairs)


def test_layered_workload_has_the_paper_shape():
    """A half-layer pair of the paper-shaped synthetic meshes spans the quad
    pairs of the paper's half-layer meshes."""
    g = golden()
    su = synth.layered_s(0.05, 1.35, False, 1, g["layers"], 34)
    ss = synth.layered_s(0.05, 1 / 1.35, True, 0, g["layers"], 34)
    ku = oracle.half_layer_columns(su, 0.05, 1.35, False, 7, 1)
    ks = oracle.half_layer_columns(ss, 0.05, 1 / 1.35, True, 6, -1)
    assert (ku[1] - ku[0]) == (ks[1] - ks[0]) == 34
    assert (1024 * (ku[1] - ku[0])) * (2048 * (ks[1] - ks[0])) == g["quad_pairs_per_pair"]


@pytest.mark.parametrize("stable", [False, True])
def test_oracle_half_layers_tile_the_mesh(stable):
    """Half-layers of one sign share only their boundary columns, cover
    every column from b_0 out, and hold exactly the samples whose |s| lies
    between the layer's boundaries."""
    D, lam = 0.05, (1 / 1.35 if stable else 1.35)
    first = 0 if stable else 1
    s = synth.layered_s(D, lam, stable, first, 5, 6)
    for sign in (1, -1):
        prev = None
        for n in range(first, 6):
            k0, k1 = oracle.half_layer_columns(s, D, lam, stable, n, sign)
            lo, hi = oracle.half_layer_interval(D, lam, stable, n, sign)
            assert np.all((s[k0:k1 + 1] >= lo - 1e-15) & (s[k0:k1 + 1] <= hi + 1e-15))
            if prev is not None:
                assert (k0 == prev[1]) if sign > 0 else (k1 == prev[0])
            prev = (k0, k1)
    with pytest.raises(ValueError):
        oracle.half_layer_columns(s, D * 1.01, lam, stable, 2, 1)


@pytest.fixture(scope="module")
def ms():
    import paper_2109_14814_amd as m
    if not os.path.exists(m.LIB_PATH):
        pytest.skip("libmsearch.so not built")
    return m


def test_capi_layer_pairs_match_oracle(ms):
    for L in range(0, 21):
        got = ms.layer_pairs(L)
        want = oracle.layer_pairs(L)
        assert [tuple(int(x) for x in p) for p in got] == want
    import ctypes
    n = ctypes.c_int32()
    buf = np.zeros(4, dtype=ms.LAYER_PAIR_DTYPE)
    assert ms.lib().layer_pairs(2, buf.ctypes.data_as(ctypes.c_void_p), 4, ctypes.byref(n)) == ms.MS_E_CAPACITY
    assert n.value == 16


@pytest.mark.parametrize("stable", [False, True])
def test_capi_half_layer_columns_match_oracle(ms, stable):
    D, lam = 0.05, (1 / 1.35 if stable else 1.35)
    first = 0 if stable else 1
    s = synth.layered_s(D, lam, stable, first, 14, 34)
    for n in range(first, 15):
        for sign in (1, -1):
            assert ms.half_layer_columns(s, D, lam, stable, n, sign) == \
                oracle.half_layer_columns(s, D, lam, stable, n, sign)
            lo, hi = ms.half_layer_bounds(D, lam, stable, n)
            olo, ohi = oracle.half_layer_interval(D, lam, stable, n, 1)
            assert abs(lo - olo) <= 1e-15 * ohi and abs(hi - ohi) <= 1e-15 * ohi


def test_capi_half_layer_errors(ms):
    s = synth.layered_s(0.05, 1.35, False, 1, 3, 4)
    with pytest.raises(ms.MSearchError):
        ms.half_layer_columns(s, 0.051, 1.35, False, 2, 1)          # boundaries not samples
    with pytest.raises(ms.MSearchError):
        ms.half_layer_columns(s[::-1].copy(), 0.05, 1.35, False, 2, 1)   # decreasing
    with pytest.raises(ms.MSearchError):
        ms.half_layer_columns(s, 0.05, 1.0, False, 2, 1)            # lambda = 1
    with pytest.raises(ms.MSearchError):
        ms.half_layer_columns(s, 0.05, 1.35, False, 2, 0)           # sign
