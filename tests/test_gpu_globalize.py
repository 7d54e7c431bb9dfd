"""GPU parity of the globalized manifold mesh (Sec. 6.1: F^n images shifted
back in theta, rows sorted by s) against the oracle, for an unstable and a
stable grid of the Jupiter-Europa problem; rows within 1e-10 (the oracle maps
the base grid n periods at once, the library one period per layer, so the
two differ by rounding only); s values and row order exact."""
import numpy as np
import pytest

import synth
from oracle import spectral

pytestmark = pytest.mark.gpu

MU, ECC = 2.527e-5, 0.0094


@pytest.fixture(scope="module")
def ms():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_14814_amd as ms
    ms.lib()
    return ms


def _grid(N, s, base, seed):
    rng = np.random.default_rng(seed)
    th = 2 * np.pi * np.arange(N) / N
    d1, d2 = rng.standard_normal(4), rng.standard_normal(4)
    g = np.zeros((len(s), N, 4))
    for k, sk in enumerate(s):
        g[k] = base[None, :] + 1e-3 * (np.cos(th)[:, None] * d1 + np.sin(2 * th)[:, None] * d2) + sk * d2[None, :]
    return g


@pytest.mark.parametrize("direction,lam,stable", [(1, 1.35, False), (-1, 1 / 1.35, True)])
def test_globalized_mesh_matches_oracle(ms, direction, lam, stable):
    base = synth.periapse_position_momentum(np.array(synth.STABLE_BASE if stable else synth.UNSTABLE_BASE), ECC)
    D, K = 0.02, 3
    s = np.array([k * D / K for k in range(-K, K + 1)])
    g = _grid(64, s, base, 3)
    rows, sv = ms.globalize(g, s, 3, 0.61, lam, direction, MU, ECC, 1000)
    ref, ref_s, _ = spectral.globalize(g, s, 3, 0.61, lam, direction, MU, ECC, 1000)
    assert np.array_equal(sv, ref_s)
    assert np.max(np.abs(rows.cpu().numpy() - ref)) < 1e-10


def test_larger_grid_sampled_rows(ms):
    """256 samples per row, 35 s values, 6 layers: the rows of two base rows
    (which the oracle globalizes on their own: rows are independent)."""
    base = synth.periapse_position_momentum(np.array(synth.UNSTABLE_BASE), ECC)
    D, K = 0.02, 17
    s = np.array([k * D / K for k in range(-K, K + 1)])
    g = _grid(256, s, base, 4)
    rows, sv = ms.globalize(g, s, 6, 0.61, 1.35, 1, MU, ECC, 1000)
    rows = rows.cpu().numpy()
    assert rows.shape[0] == 35 + 6 * 34
    for k in (3, K + 5):
        ref, ref_s, src = spectral.globalize(g[k:k + 1], s[k:k + 1], 6, 0.61, 1.35, 1, MU, ECC, 1000)
        for r, sr in zip(ref, ref_s):
            i = int(np.nonzero(sv == sr)[0][0])
            assert np.max(np.abs(rows[i] - r)) < 1e-10


def test_capacity_and_errors(ms):
    import ctypes as C
    import torch
    s = np.array([-0.01, 0.0, 0.01])
    g = torch.tensor(_grid(16, s, np.array([0.9, 0.0, 0.0, 0.97]), 1), device="cuda")
    nb = C.c_size_t()
    ms.lib().globalize_workspace_size(16, 3, 2, C.byref(nb))
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    out = torch.empty((4, 16, 4), dtype=torch.float64, device="cuda")
    s_out = np.empty(7)
    m = C.c_int64()
    mp = ms.MapParams(MU, ECC, 100, 1)
    rc = ms.lib().globalize_manifold(C.c_void_p(g.data_ptr()), s.ctypes.data_as(C.c_void_p), 16, 3, 2, 0.5, 1.35,
                                     C.byref(mp), C.c_void_p(out.data_ptr()), 4, s_out.ctypes.data_as(C.c_void_p),
                                     C.byref(m), C.c_void_p(ws.data_ptr()), nb.value, None)
    assert rc == -2 and m.value == 7                    # MS_E_CAPACITY, rows needed
    with pytest.raises(ms.MSearchError):
        ms.globalize(g, s[::-1].copy(), 2, 0.5, 1.35, 1, MU, ECC, 100)      # s not increasing
    with pytest.raises(ms.MSearchError):
        ms.globalize(g, s, 2, 0.5, 1.35, 2, MU, ECC, 100)                    # direction not +-1
    rows, sv = ms.globalize(g, s, 0, 0.5, 1.35, 1, MU, ECC, 100)
    assert np.array_equal(rows.cpu().numpy(), g.cpu().numpy()) and np.array_equal(sv, s)
