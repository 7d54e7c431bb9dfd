"""GPU parity of the spectral theta operations (Sec. 6.1 translation, Sec. 7
derivative and trigonometric interpolation) through the C ABI against the
oracle (numpy FFT).  Bar: 1e-12 x max|a| x (N/2)^order, from the rounding of
two length-N transforms (error ~ log2(N) eps per coefficient) and the factor
k^order the derivative applies to the highest coefficients."""
import numpy as np
import pytest

from oracle import spectral

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ms():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_14814_amd as ms
    ms.lib()
    return ms


def _rows(n_rows, N, seed, smooth):
    rng = np.random.default_rng(seed)
    if not smooth:
        return rng.standard_normal((n_rows, N, 4))
    # a few low modes plus a small full-band part
    th = 2 * np.pi * np.arange(N) / N
    K = min(8, N // 2 - 1) if N > 2 else 0
    out = np.zeros((n_rows, N, 4))
    for k in range(K + 1):
        c = rng.standard_normal((n_rows, 1, 4))
        s = rng.standard_normal((n_rows, 1, 4))
        out += c * np.cos(k * th)[None, :, None] + s * np.sin(k * th)[None, :, None]
    return out + 1e-6 * rng.standard_normal((n_rows, N, 4))


def _tol(ref_rows, N, order):
    return 1e-12 * max(1.0, np.abs(ref_rows).max()) * max(1.0, N / 2) ** order


@pytest.mark.parametrize("N", [2, 4, 8, 32, 128, 512, 1024, 2048])
@pytest.mark.parametrize("order", [0, 1, 2])
def test_shift_matches_oracle(ms, N, order):
    rows = _rows(37, N, N + order, smooth=(N % 3 == 0 or N >= 512))
    for rho in (0.31, -5.7):
        got = ms.theta_shift(rows, rho, order).cpu().numpy()
        ref = spectral.shift_derivative(rows, rho, order)
        assert np.max(np.abs(got - ref)) < _tol(rows, N, order)


@pytest.mark.parametrize("N", [16, 2048])
def test_per_row_shift_and_random_data(ms, N):
    rows = _rows(53, N, 7, smooth=False)
    rho = np.random.default_rng(8).uniform(-4, 4, 53)
    for order in (0, 1):
        got = ms.theta_shift(rows, rho, order).cpu().numpy()
        ref = spectral.shift_derivative(rows, rho, order)
        assert np.max(np.abs(got - ref)) < _tol(rows, N, order)


def test_grid_shift_is_a_roll_and_in_place(ms):
    import torch
    N = 256
    rows = _rows(9, N, 3, smooth=False)
    t = torch.tensor(rows, device="cuda")
    ms.theta_shift(t, 2 * np.pi * 5 / N, 0, out=t)
    assert np.max(np.abs(t.cpu().numpy() - np.roll(rows, -5, axis=1))) < 1e-12


def test_mesh_sized_rows(ms):
    """A 2048-sample theta grid with 2049 s-rows, the shape of a globalised
    layer mesh, compared on a seeded sample of rows."""
    N, M = 2048, 2049
    rows = _rows(M, N, 11, smooth=True)
    rho = np.random.default_rng(12).uniform(-3, 3, M)
    got = ms.theta_shift(rows, rho, 0).cpu().numpy()
    idx = np.concatenate([np.random.default_rng(13).choice(M, 40, replace=False), [0, M - 1]])
    ref = spectral.shift_derivative(rows[idx], rho[idx], 0)
    assert np.max(np.abs(got[idx] - ref)) < _tol(rows, N, 0)


@pytest.mark.parametrize("N", [1, 2, 7, 64, 65, 2048, 3000])
def test_interp_matches_oracle(ms, N):
    rows = _rows(5, N, 20 + N, smooth=(N > 8))
    rng = np.random.default_rng(N)
    q_rows = rng.integers(0, 5, 300)
    theta = rng.uniform(-10, 10, 300)
    theta[:5] = 2 * np.pi * np.array([0, 1, N - 1, 3 * N, -2]) / N      # on grid points
    theta[5] = theta[6] + 1e-13                                          # very near one
    got = ms.theta_interp(rows, q_rows, theta).cpu().numpy()
    ref = np.stack([spectral.interpolate(rows[r], t) for r, t in zip(q_rows, theta)])
    scale = max(1.0, np.abs(rows).max())
    assert np.max(np.abs(got - ref)) < 1e-11 * scale


def test_interp_out_of_range_is_nan(ms):
    rows = _rows(3, 16, 1, smooth=True)
    got = ms.theta_interp(rows, [0, 3, -1, 1, 2], [0.2, 0.2, 0.2, float("nan"), 1e308]).cpu().numpy()
    assert np.all(np.isfinite(got[0])) and np.all(np.isnan(got[1:]))


def test_edges_and_errors(ms):
    assert ms.theta_shift(np.zeros((0, 8, 4)), 0.3).shape == (0, 8, 4)
    assert ms.theta_interp(np.zeros((2, 8, 4)), [], []).shape == (0, 4)
    with pytest.raises(ms.MSearchError):
        ms.theta_shift(np.zeros((3, 12, 4)), 0.3)          # not a power of two
    with pytest.raises(ms.MSearchError):
        ms.theta_shift(np.zeros((3, 4096, 4)), 0.3)        # above 2048
    with pytest.raises(ms.MSearchError):
        ms.theta_shift(np.zeros((3, 8, 4)), 0.3, order=3)
    # rho = 0, order 0 is the identity up to rounding
    rows = _rows(4, 64, 2, smooth=False)
    assert np.max(np.abs(ms.theta_shift(rows, 0.0).cpu().numpy() - rows)) < 1e-13
