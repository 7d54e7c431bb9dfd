"""Fourier-Taylor parameterizations and their globalized partials (paper
Sec. 7).

TEST INFRASTRUCTURE ONLY: used by tests/ and the CPU-baseline leg of the
benchmark.

A local parameterization is W(theta, s) = sum_k W_k(theta) s^k with each
coefficient stored as its values at theta_i = 2 pi i / N: an array
coeffs[k, i, c] of shape (P+1, N, 4).  Its partials at a point follow the
paper's recipe step by step: evaluate the series in s at every theta_i, take
the theta derivative of those values by FFT (multiply coefficient j by i j),
differentiate the series term by term for the s derivative, and interpolate
all three trigonometrically at theta.

The globalized manifold is W(theta, s) = F^m(W(theta - m omega, lambda^-m s))
(m > 0 unstable, m < 0 stable, with the stable multiplier), and its partials
are the state transition matrix DF^m applied to the local partials, the s one
scaled by lambda^-m.  F is the stroboscopic map of the position-momentum
problem (oracle.pertbp_map).
"""
from __future__ import annotations

import numpy as np

from . import spectral


def series_rows(coeffs: np.ndarray, s: float):
    """Values sum_k W_k(theta_i) s^k and s-derivatives sum_k k W_k(theta_i)
    s^(k-1) at every theta_i (two (N, 4) arrays), by Horner's rule."""
    c = np.asarray(coeffs, dtype=np.float64)
    v = np.zeros(c.shape[1:])
    dv = np.zeros(c.shape[1:])
    for k in range(c.shape[0] - 1, -1, -1):
        dv = dv * s + v
        v = v * s + c[k]
    return v, dv


def local(coeffs: np.ndarray, theta: float, s: float):
    """(W, dW/dtheta, dW/ds) at (theta, s), each a 4-vector."""
    v, dv = series_rows(coeffs, s)
    w = spectral.interpolate(v, theta)
    dth = spectral.interpolate(spectral.shift_derivative(v, 0.0, 1), theta)
    ds = spectral.interpolate(dv, theta)
    return w, dth, ds


def globalized(coeffs: np.ndarray, theta: float, s: float, m: int, omega: float, lam: float, mu: float,
               eps: float, steps_per_period: int):
    """(W, dW/dtheta, dW/ds) of the globalized parameterization at (theta, s):
    the local ones at (theta - m omega, lam^-m s) carried by F^m and DF^m."""
    from . import pertbp_map
    w, dth, ds = local(coeffs, theta - m * omega, lam ** (-m) * s)
    out, M = pertbp_map(w[None], mu, eps, steps_per_period, m, stm=True)
    return out[0], M[0] @ dth, lam ** (-m) * (M[0] @ ds)
