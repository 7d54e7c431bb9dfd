"""GPU parity of the RK8 stroboscopic map against the oracle (same states,
4000 steps per period, F^{+-3}), within 1e-10."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

MU, ECC = 2.528e-5, 0.0094


@pytest.fixture(scope="module")
def ms():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_14814_amd as ms
    ms.lib()
    return ms


@pytest.mark.parametrize("n_periods,base", [(3, synth.UNSTABLE_BASE), (-3, synth.STABLE_BASE), (1, synth.UNSTABLE_BASE)])
def test_map_matches_oracle(ms, n_periods, base):
    y0 = synth.random_states(300, 21, base, 1e-3)
    ref = oracle.rk8_map(y0, MU, ECC, 4000, n_periods)
    got = ms.propagate(y0, MU, ECC, 4000, n_periods).cpu().numpy()
    assert np.max(np.abs(got - ref)) < 1e-10


def test_map_full_patch_sampled(ms):
    """The full 2049 x 257 propagated patch, compared on a seeded sample of
    vertices the oracle maps one by one."""
    (mu_mesh, _), _ = synth.propagated_patches(2048, 256, 0)
    V = mu_mesh.verts.reshape(-1, 4)
    got = ms.propagate(V, MU, ECC, 4000, 3).cpu().numpy()
    idx = np.random.default_rng(3).choice(V.shape[0], 256, replace=False)
    idx = np.concatenate([idx, [0, V.shape[0] - 1]])
    ref = oracle.rk8_map(V[idx], MU, ECC, 4000, 3)
    assert np.max(np.abs(got[idx] - ref)) < 1e-10


def test_map_edge_cases(ms):
    y0 = synth.random_states(5, 1, synth.UNSTABLE_BASE, 1e-3)
    # zero periods is the identity; in-place works
    assert np.array_equal(ms.propagate(y0, MU, ECC, 4000, 0).cpu().numpy(), y0)
    import torch
    t = torch.as_tensor(y0).cuda()
    ms.propagate(t, MU, ECC, 400, 1, out=t)
    assert np.max(np.abs(t.cpu().numpy() - oracle.rk8_map(y0, MU, ECC, 400, 1))) < 1e-10
    # the equilateral point is fixed
    L4 = np.array([[0.5 - MU, np.sqrt(3) / 2, 0.0, 0.0]])
    assert np.max(np.abs(ms.propagate(L4, MU, ECC, 400, 1).cpu().numpy() - L4)) < 1e-13
    with pytest.raises(ms.MSearchError):
        ms.propagate(y0, MU, 1.5, 400, 1)
