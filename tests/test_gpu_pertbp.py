"""GPU parity of the position-momentum elliptic problem (Sec. 3.3): the map
F^m and its state transition matrix DF^m through the C ABI against the
oracle, on Jupiter-Europa states near the seeds of the propagated patches.
States within 1e-10; matrix entries within 1e-10 of the largest entry of
their matrix (entries reach ~1e2 after three periods)."""
import numpy as np
import pytest

import oracle
import synth

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


def _states(n, seed, stable=False):
    return synth.pm_random_states(n, seed, ECC, synth.STABLE_BASE if stable else synth.UNSTABLE_BASE, 1e-3)


def _close_stm(got, ref):
    scale = np.maximum(1.0, np.abs(ref).max(axis=(1, 2)))
    return np.max(np.abs(got - ref).max(axis=(1, 2)) / scale)


@pytest.mark.parametrize("n,n_periods,stable", [(300, 3, False), (257, -3, True), (1, 1, False)])
def test_map_matches_oracle(ms, n, n_periods, stable):
    z = _states(n, 31 + n, stable)
    ref = oracle.pertbp_map(z, MU, ECC, 4000, n_periods)
    got = ms.pertbp_map(z, MU, ECC, 4000, n_periods).cpu().numpy()
    assert np.max(np.abs(got - ref)) < 1e-10


@pytest.mark.parametrize("cols", [1, 2, 4])
@pytest.mark.parametrize("n_periods,stable", [(3, False), (-3, True)])
def test_stm_matches_oracle(ms, cols, n_periods, stable):
    n = 67                      # several blocks at 4 threads per state, ragged tail
    z = _states(n, 40 + cols, stable)
    ref_out, ref_M = oracle.pertbp_map(z, MU, ECC, 4000, n_periods, stm=True)
    out, M = ms.pertbp_map_stm(z, MU, ECC, 4000, n_periods, cols_per_thread=cols)
    assert np.max(np.abs(out.cpu().numpy() - ref_out)) < 1e-10
    assert _close_stm(M.cpu().numpy(), ref_M) < 1e-10


def test_stm_columns_agree_bitwise(ms):
    """The split of the 4 columns over threads changes nothing in the arithmetic."""
    z = _states(100, 50)
    _, a = ms.pertbp_map_stm(z, MU, ECC, 1000, 2, cols_per_thread=1)
    _, b = ms.pertbp_map_stm(z, MU, ECC, 1000, 2, cols_per_thread=2)
    _, c = ms.pertbp_map_stm(z, MU, ECC, 1000, 2, cols_per_thread=4)
    out = ms.pertbp_map(z, MU, ECC, 1000, 2)
    o2, _ = ms.pertbp_map_stm(z, MU, ECC, 1000, 2)
    assert np.max(np.abs((a - b).cpu().numpy())) < 1e-12 and np.max(np.abs((a - c).cpu().numpy())) < 1e-12
    assert np.max(np.abs((out - o2).cpu().numpy())) < 1e-13


def test_bench_size_sampled(ms):
    """The benchmark's workload (2 x 2049 x 257 states, F^3 and F^-3), compared
    on a seeded sample the oracle maps one by one."""
    (mu_mesh, _), (ms_mesh, _) = synth.propagated_patches(2048, 256, 0)
    Vu = synth.periapse_position_momentum(mu_mesh.verts.reshape(-1, 4), ECC)
    got = ms.pertbp_map(Vu, MU, ECC, 4000, 3).cpu().numpy()
    idx = np.concatenate([np.random.default_rng(5).choice(Vu.shape[0], 64, replace=False), [0, Vu.shape[0] - 1]])
    ref = oracle.pertbp_map(Vu[idx], MU, ECC, 4000, 3)
    assert np.max(np.abs(got[idx] - ref)) < 1e-10
    Vs = synth.periapse_position_momentum(ms_mesh.verts.reshape(-1, 4), ECC)
    zs = Vs[:: 9973]
    _, M = ms.pertbp_map_stm(zs, MU, ECC, 4000, -3)
    _, ref_M = oracle.pertbp_map(zs, MU, ECC, 4000, -3, stm=True)
    assert _close_stm(M.cpu().numpy(), ref_M) < 1e-10


def test_edge_cases(ms):
    import torch
    z = _states(5, 60)
    # zero periods: identity map and identity matrix
    out, M = ms.pertbp_map_stm(z, MU, ECC, 100, 0)
    assert np.array_equal(out.cpu().numpy(), z)
    assert np.array_equal(M.cpu().numpy(), np.broadcast_to(np.eye(4), (5, 4, 4)))
    assert np.array_equal(ms.pertbp_map(z, MU, ECC, 100, 0).cpu().numpy(), z)
    # empty input
    e = np.zeros((0, 4))
    assert ms.pertbp_map(e, MU, ECC, 100, 1).shape == (0, 4)
    assert ms.pertbp_map_stm(e, MU, ECC, 100, 1)[1].shape == (0, 4, 4)
    # in place
    t = torch.tensor(z, device="cuda")
    ref = ms.pertbp_map(z, MU, ECC, 500, 1).cpu().numpy()
    ms.pertbp_map(t, MU, ECC, 500, 1, out=t)
    assert np.array_equal(t.cpu().numpy(), ref)
    # eccentricity zero and a large one
    for eps in (0.0, 0.6):
        ref = oracle.pertbp_map(z, MU, eps, 2000, 1)
        assert np.max(np.abs(ms.pertbp_map(z, MU, eps, 2000, 1).cpu().numpy() - ref)) < 1e-10
    # only the matrix
    _, M1 = ms.pertbp_map_stm(z, MU, ECC, 500, 1, want_out=False)
    _, M2 = ms.pertbp_map_stm(z, MU, ECC, 500, 1)
    assert torch.equal(M1, M2)


def test_errors(ms):
    z = _states(4, 61)
    with pytest.raises(ms.MSearchError):
        ms.pertbp_map(z, MU, 1.0, 100, 1)
    with pytest.raises(ms.MSearchError):
        ms.pertbp_map(z, MU, ECC, 0, 1)
    with pytest.raises(ms.MSearchError):
        ms.pertbp_map_stm(z, MU, ECC, 100, 1, cols_per_thread=3)
