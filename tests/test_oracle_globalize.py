"""Pins of the oracle's globalized mesh (paper Sec. 6.1): no globalization
returns the grid; the s-set is the sorted union of lambda^n s_k with s = 0
once and contains the layer boundaries +-lambda^n D; a grid of copies of a
fixed point of the map stays that point at every layer; every row is the
theta shift of F^n of a base row, and shifts of rows that F only rotates
(a circle of fixed radius in the two-body problem) bring them back to the
base row exactly up to truncation."""
import math

import numpy as np

from oracle import spectral

MU_EM = 0.0121505856


def _grid(N, s):
    th = 2 * np.pi * np.arange(N) / N
    g = np.zeros((len(s), N, 4))
    for k, sk in enumerate(s):
        g[k, :, 0] = 0.8 + 0.01 * sk + 1e-3 * np.cos(th)
        g[k, :, 1] = 1e-3 * np.sin(th)
        g[k, :, 3] = 0.9
    return g


def test_no_globalization_is_the_grid():
    s = np.linspace(-0.05, 0.05, 7)
    g = _grid(16, s)
    mesh, sv, src = spectral.globalize(g, s, 0, 0.3, 1.4, 1, MU_EM, 0.0, 200)
    assert np.array_equal(mesh, g) and np.array_equal(sv, s)


def test_s_set_is_the_sorted_union():
    D, lam, K, n_max = 0.05, 1.4, 3, 4
    s = np.array([k * D / K for k in range(-K, K + 1)])
    g = _grid(8, s)
    _, sv, src = spectral.globalize(g, s, n_max, 0.3, lam, 1, MU_EM, 0.0, 50)
    brute = sorted({lam ** n * sk for n in range(n_max + 1) for sk in s if not (n > 0 and sk == 0.0)})
    assert np.array_equal(sv, np.array(brute))
    assert np.all(np.diff(sv) > 0) and np.sum(sv == 0.0) == 1
    for n in range(n_max + 1):
        for b in (D * lam ** n, -D * lam ** n):
            assert np.min(np.abs(sv - b)) <= 1e-15 * abs(b)
    # stable direction: lam < 1 and F^-1
    _, sv2, _ = spectral.globalize(g, s, 2, 0.3, 1 / lam, -1, MU_EM, 0.0, 50)
    assert np.max(np.abs(sv2 - np.array(sorted({(1 / lam) ** (-n) * sk for n in range(3) for sk in s
                                                 if not (n > 0 and sk == 0.0)})))) < 1e-15


def test_fixed_point_rows_stay():
    """At e = 0 the equilateral point is a fixed point of F (in this frame
    q = (1/2 - mu, sqrt(3)/2), p = (-q_y, q_x)): rows of copies stay put."""
    q = np.array([0.5 - MU_EM, math.sqrt(3) / 2])
    L4 = np.array([q[0], q[1], -q[1], q[0]])
    s = np.array([-0.01, 0.0, 0.01])
    g = np.broadcast_to(L4, (3, 16, 4)).copy()
    mesh, _, _ = spectral.globalize(g, s, 3, 0.7, 1.3, 1, MU_EM, 0.0, 400)
    assert np.max(np.abs(mesh - L4)) < 1e-11


def test_rotated_circle_comes_back():
    """mu = 0, e = 0: a circular orbit of radius a is turned by
    omega = 2 pi (a^-1.5 - 1) per period in this frame, so with that omega
    the shift undoes F exactly (the rows are one Fourier mode)."""
    a = 0.7
    om = 2 * np.pi * (a ** -1.5 - 1.0)
    N = 32
    th = 2 * np.pi * np.arange(N) / N
    w = a ** -1.5
    # p = v + J q with the rotating-frame velocity v = a (w - 1)(-sin, cos), J q = a (-sin, cos)
    row = np.stack([a * np.cos(th), a * np.sin(th), -a * w * np.sin(th), a * w * np.cos(th)], axis=1)
    s = np.array([0.0, 0.01])
    g = np.stack([row, row])
    mesh, sv, src = spectral.globalize(g, s, 3, om, 1.5, 1, 0.0, 0.0, 2000)
    for r in range(mesh.shape[0]):
        assert np.max(np.abs(mesh[r] - row)) < 1e-11
