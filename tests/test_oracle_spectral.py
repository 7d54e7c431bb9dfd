"""Pins of the oracle's spectral theta operations (paper Sec. 6.1 translation,
Sec. 7 derivative and trigonometric interpolation): closed forms on
trigonometric polynomials, exact grid shifts, the cosine mode at N/2, a
brute-force DFT, and real outputs."""
import math

import numpy as np
import pytest

from oracle import spectral


def _trig_poly(seed, K):
    """a(theta) = sum_{k<=K} c_k cos(k theta) + s_k sin(k theta) per coordinate,
    with its first two derivatives, as callables of theta (any shape)."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((K + 1, 4)) / (1 + np.arange(K + 1))[:, None]
    s = rng.standard_normal((K + 1, 4)) / (1 + np.arange(K + 1))[:, None]
    k = np.arange(K + 1)[:, None]

    def f(th, d=0):
        th = np.asarray(th, dtype=np.float64)[..., None, None]
        if d == 0:
            v = c * np.cos(k * th) + s * np.sin(k * th)
        elif d == 1:
            v = -k * c * np.sin(k * th) + k * s * np.cos(k * th)
        else:
            v = -k * k * (c * np.cos(k * th) + s * np.sin(k * th))
        return v.sum(axis=-2)
    return f


def _grid(N):
    return 2 * np.pi * np.arange(N) / N


@pytest.mark.parametrize("N", [16, 64, 127, 1024])
@pytest.mark.parametrize("order", [0, 1, 2])
def test_shift_and_derivative_of_trig_polynomials(N, order):
    """Band-limited data (degree < N/2): the operation is exact, so it equals
    the closed form d^order a(theta_i + rho) for any rho."""
    K = (N - 1) // 2 if N % 2 else N // 2 - 1
    f = _trig_poly(N + order, K)
    rows = f(_grid(N))
    for rho in (0.0, 0.37, -2.9, 11.0):
        got = spectral.shift_derivative(rows, rho, order)
        ref = f(_grid(N) + rho, order)
        scale = max(1.0, np.abs(ref).max())
        assert np.max(np.abs(got - ref)) < 1e-12 * scale * max(1, K) ** order


def test_per_row_shifts():
    N = 64
    f = _trig_poly(3, 20)
    rhos = np.array([0.1, -0.4, 2.0])
    rows = np.stack([f(_grid(N))] * 3)
    got = spectral.shift_derivative(rows, rhos, 0)
    for r, rho in enumerate(rhos):
        assert np.max(np.abs(got[r] - f(_grid(N) + rho))) < 1e-13


@pytest.mark.parametrize("N", [32, 33])
def test_grid_shift_is_a_roll(N):
    """rho = 2 pi m / N moves every sample m places, whatever the data (for
    even N the cosine mode (-1)^i rolls into (-1)^m (-1)^i, which is what
    its multiplier cos(N rho / 2) = (-1)^m gives)."""
    rows = np.random.default_rng(N).standard_normal((N, 4))
    for m in (1, 5, -3):
        got = spectral.shift_derivative(rows, 2 * np.pi * m / N, 0)
        ref = np.roll(rows, -m, axis=0)
        assert np.max(np.abs(got - ref)) < 1e-13


def test_cosine_mode_at_half_n():
    """Samples (-1)^i of cos(N theta / 2) (even N) shift to cos(N (theta_i + rho)/2)
    and differentiate to -(N/2) sin(N (theta_i + rho)/2)."""
    N = 16
    th = _grid(N)
    rows = np.repeat(np.cos(N * th / 2)[:, None], 4, axis=1)
    for rho in (0.1, 0.7):
        s0 = spectral.shift_derivative(rows, rho, 0)
        s1 = spectral.shift_derivative(rows, rho, 1)
        assert np.max(np.abs(s0 - np.cos(N * (th + rho) / 2)[:, None])) < 1e-13
        assert np.max(np.abs(s1 + N / 2 * np.sin(N * (th + rho) / 2)[:, None])) < 1e-12


@pytest.mark.parametrize("N", [8, 9])
def test_against_brute_force_dft(N):
    """The same operation from an explicit N x N DFT matrix (no FFT)."""
    rows = np.random.default_rng(7).standard_normal((N, 4))
    i = np.arange(N)
    F = np.exp(-2j * np.pi * np.outer(i, i) / N)
    for rho, order in ((0.3, 0), (1.1, 1), (-0.4, 2)):
        A = F @ rows
        m = spectral.multiplier(N, rho, order)
        ref = (np.conj(F) @ (A * m[:, None])) / N
        assert np.max(np.abs(ref.imag)) < 1e-12            # a real result
        got = spectral.shift_derivative(rows, rho, order)
        assert np.max(np.abs(got - ref.real)) < 1e-12


def test_multiplier_is_hermitian():
    """m(-k) = conj(m(k)), so real rows stay real."""
    for N in (16, 17):
        m = spectral.multiplier(N, 0.77, 1)
        k = np.arange(1, N)
        assert np.max(np.abs(m[N - k] - np.conj(m[k]))) < 1e-15


@pytest.mark.parametrize("N", [64, 65])
def test_interpolation(N):
    K = N // 2 - 1
    f = _trig_poly(11, K)
    rows = f(_grid(N))
    # at the grid points it returns the samples
    assert np.max(np.abs(spectral.interpolate(rows, _grid(N)) - rows)) < 1e-13
    # between them, the polynomial itself
    th = np.random.default_rng(2).uniform(-7, 7, 50)
    assert np.max(np.abs(spectral.interpolate(rows, th) - f(th))) < 1e-12
    # and it agrees with a shift: value at theta_3 + rho = row 3 of the shifted row
    rho = 0.123
    assert np.max(np.abs(spectral.interpolate(rows, _grid(N)[3] + rho) -
                         spectral.shift_derivative(rows, rho)[3])) < 1e-13
