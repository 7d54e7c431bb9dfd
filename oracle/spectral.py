"""Spectral operations on periodic theta samples (paper Sec. 6.1 and Sec. 7).

TEST INFRASTRUCTURE ONLY: used by tests/ and the CPU-baseline leg of the
benchmark.  Plain numpy; numpy's FFT serves as the library primitive.

A row holds a(theta_i) at theta_i = 2 pi i / N, i = 0..N-1, for each of the
four coordinates (x, y, px, py) of a mesh: rows are arrays (..., N, 4) with
theta along axis -2, the layout of a mesh's vertex grid (theta fastest).

Frequencies are the signed ones: k for k < N/2, k - N for k > N/2.  For even N
the coefficient at k = N/2 stands for the real mode cos(N theta / 2) (half of
it at +N/2 and half at -N/2), which keeps every result real; this is the
reading of the paper's sum over k = 0..N-1 that a real periodic function
needs.
"""
from __future__ import annotations

import numpy as np


def _signed_k(N: int) -> np.ndarray:
    k = np.arange(N, dtype=np.float64)
    k[k > N / 2] -= N
    return k


def multiplier(N: int, rho, order: int) -> np.ndarray:
    """Spectral multiplier (j k)^order e^{j k rho} per signed frequency k
    (shape (..., N) for an array rho); at k = N/2 (even N) its real part,
    the action on cos(N theta / 2)."""
    k = _signed_k(N)
    r = np.asarray(rho, dtype=np.float64)[..., None]
    m = (1j * k) ** order * np.exp(1j * k * r)
    if N % 2 == 0:
        m[..., N // 2] = m[..., N // 2].real
    return m


def shift_derivative(rows: np.ndarray, rho, order: int = 0) -> np.ndarray:
    """d^order/dtheta^order of a(theta_i + rho) for every row (Sec. 6.1: FFT,
    multiply coefficient k by e^{j k rho}, inverse FFT; Sec. 7: multiply by
    j k for the derivative).  rows (..., N, 4); rho a scalar or one value per
    row (shape rows.shape[:-2])."""
    a = np.asarray(rows, dtype=np.float64)
    N = a.shape[-2]
    A = np.fft.fft(a, axis=-2)
    m = multiplier(N, rho, order)
    out = np.fft.ifft(A * m[..., :, None], axis=-2)
    return out.real


def interpolate(rows: np.ndarray, theta) -> np.ndarray:
    """Trigonometric interpolation (Sec. 7): the value at theta of the real
    trigonometric polynomial through a row's samples,
    (1/N) sum_k a^(k) e^{j k theta} over the signed k (k = N/2 as the cosine
    mode).  rows (N, 4), theta scalar or array; returns (..., 4)."""
    a = np.asarray(rows, dtype=np.float64)
    N = a.shape[0]
    A = np.fft.fft(a, axis=0)
    k = _signed_k(N)
    th = np.asarray(theta, dtype=np.float64)[..., None]
    e = np.exp(1j * k * th)
    if N % 2 == 0:
        e[..., N // 2] = np.cos(N / 2 * th[..., 0])
    return (e @ A).real / N


def globalize(grid, s, n_max: int, omega: float, lam: float, direction: int, mu: float, eps: float,
              steps_per_period: int):
    """The globalized mesh of Sec. 6.1 from a fundamental-domain grid
    grid (n_s, N, 4) = W(theta_i, s_k) (s increasing).  For n = 0..n_max the
    points F^{d n}(W(theta_i, s_k)) = W(theta_i + d n omega, lam^{d n} s_k)
    (d = +1 for an unstable manifold with the map F, -1 for a stable one with
    F^-1 and its own lam) are shifted back by rho = -d n omega, giving
    W(theta_i, lam^{d n} s_k).  The rows are returned sorted by their s
    values, with the row s = 0 (the torus) kept once.  Returns (mesh (M, N,
    4), s (M,), source (M, 2) = (n, k) of each row).  F is the position-momentum
    map (oracle.pertbp_map), applied to the base grid n times at once."""
    from . import pertbp_map
    g = np.asarray(grid, dtype=np.float64)
    n_s, N = g.shape[0], g.shape[1]
    sv = np.asarray(s, dtype=np.float64)
    rows, svals, src = [], [], []
    for n in range(n_max + 1):
        if n == 0:
            P = g.copy()
        else:
            P = pertbp_map(g.reshape(-1, 4), mu, eps, steps_per_period, direction * n).reshape(g.shape)
            P = shift_derivative(P, -direction * n * omega, 0)
        for k in range(n_s):
            if n > 0 and sv[k] == 0.0:
                continue
            rows.append(P[k])
            svals.append(lam ** (direction * n) * sv[k])
            src.append((n, k))
    order = sorted(range(len(svals)), key=lambda i: svals[i])
    return (np.stack([rows[i] for i in order]), np.array([svals[i] for i in order]),
            np.array([src[i] for i in order]))
