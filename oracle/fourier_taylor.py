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


def newton(coeffs_u, coeffs_s, params, chart_u, chart_s, mu: float, eps: float, steps_per_period: int,
           max_trials: int = 40, tol: float = 1e-12, alpha0: float = 1.0, alpha_min: float = 2.0 ** -30,
           history: bool = False):
    """Damped Newton on the globalized charts (paper Sec. 7):
        f(x) = W_u(theta_u, s_u) - W_s(theta_s, s_s),
        Df = [dW_u/dtheta, dW_u/ds, -dW_s/dtheta, -dW_s/ds],
        x <- x - alpha Df^{-1} f,
    for every row x = (theta_u, s_u, theta_s, s_s) of params.  chart_u and
    chart_s are (m, omega, lambda) of each chart's globalization.  alpha
    starts at alpha0 after every accepted point and is halved after every
    trial point whose r = |f|^2 is not below the current one; a row stops
    when r <= tol^2, after max_trials trial points, when alpha < alpha_min,
    on a singular Df, or on a non-finite f at the start (the rules of
    damped_newton).  Returns (x, f, r, status, trials[, accepted r's])."""
    from . import NEWTON_CONVERGED, NEWTON_LIMIT, NEWTON_NONFINITE, NEWTON_SINGULAR, NEWTON_STALLED, gepp4
    P = np.ascontiguousarray(params, dtype=np.float64).reshape(-1, 4)
    K = P.shape[0]
    xo = np.empty_like(P); fo = np.full((K, 4), np.nan); ro = np.full(K, np.nan)
    status = np.empty(K, np.int32); trials = np.zeros(K, np.int32)
    hist = []
    tol2 = tol * tol

    def evaluate(q):
        wu, tu, su = globalized(coeffs_u, q[0], q[1], *chart_u, mu, eps, steps_per_period)
        ws, ts, ss = globalized(coeffs_s, q[2], q[3], *chart_s, mu, eps, steps_per_period)
        return wu - ws, np.stack([tu, su, -ts, -ss], axis=1)

    for k in range(K):
        q = P[k].copy()
        based, st, tr = False, -1, 0
        p = fp = delta = None
        rp = alpha = 0.0
        seq = []
        while True:
            f, J = evaluate(q)
            r = float(np.dot(f, f))
            if not based:
                accept = True
                if not np.isfinite(r):
                    st = NEWTON_NONFINITE
            else:
                tr += 1
                accept = r < rp
            if accept and st == -1:
                p, fp, rp, alpha, based = q.copy(), f.copy(), r, alpha0, True
                seq.append(r)
                if r <= tol2:
                    st = NEWTON_CONVERGED
                else:
                    ok, z = gepp4(J, -f)
                    if not ok:
                        st = NEWTON_SINGULAR
                    else:
                        delta = z
            elif st == -1:
                alpha = alpha * 0.5
                if alpha < alpha_min:
                    st = NEWTON_STALLED
            if st == -1 and tr >= max_trials:
                st = NEWTON_LIMIT
            if st != -1:
                break
            q = np.array([p[c] + alpha * delta[c] for c in range(4)])
        xo[k] = p if based else q
        if based:
            fo[k] = fp; ro[k] = rp
        status[k] = st; trials[k] = tr
        hist.append(seq)
    out = (xo, fo, ro, status, trials)
    return out + (hist,) if history else out


def planted_charts(N: int, order: int, seed: int, root, chart_u, chart_s, mu: float, eps: float,
                   steps_per_period: int, base_u, base_s):
    """Two charts whose globalizations meet at the parameters `root`
    (theta_u, s_u, theta_s, s_s): seeded smooth coefficients around the base
    points, then the stable chart's s^0 coefficient shifted by the constant
    that carries its local point at the root onto F^{-m_s} of the unstable
    globalized point (a constant added to W_0 adds it at every (theta, s))."""
    from . import pertbp_map
    rng = np.random.default_rng(seed)
    th = 2 * np.pi * np.arange(N) / N

    def coeffs(base):
        c = np.zeros((order + 1, N, 4))
        c[0] = np.asarray(base, dtype=np.float64)[None, :]
        for k in range(order + 1):
            for q in range(min(4, N // 2)):
                amp = (1e-3 if k == 0 else 1e-2 / (k + 1) ** 2) / (1 + q) ** 2
                c[k] += amp * (rng.standard_normal(4)[None, :] * np.cos(q * th)[:, None]
                               + rng.standard_normal(4)[None, :] * np.sin(q * th)[:, None])
        return c
    cu, cs = coeffs(base_u), coeffs(base_s)
    pu = globalized(cu, root[0], root[1], *chart_u, mu, eps, steps_per_period)[0]
    m_s, om_s, lam_s = chart_s
    local_s = local(cs, root[2] - m_s * om_s, lam_s ** (-m_s) * root[3])[0]
    target = pertbp_map(pu[None], mu, eps, steps_per_period, -m_s)[0]
    cs[0] += (target - local_s)[None, :]
    return cu, cs


def continuation_predict(x0, omega0, domega, x1=None, omega1=None):
    """Initial guess for the connection at rotation numbers
    (omega_u, omega_s) = omega0 + domega (paper Sec. 8): x0 itself on a first
    step (no earlier solution x1), else the linear predictor
        x = x0 + q (x0 - x1),  q = domega_u / (omega_u0 - omega_u1),
    with q = domega_s / (omega_s0 - omega_s1) instead when domega_u = 0 (and
    q = 0 when both are 0).  Rows: x (K, 4) = (theta_u, s_u, theta_s, s_s),
    omega (K, 2) = (omega_u, omega_s)."""
    x0 = np.asarray(x0, dtype=np.float64).reshape(-1, 4)
    if x1 is None:
        return x0.copy()
    x1 = np.asarray(x1, dtype=np.float64).reshape(-1, 4)
    o0 = np.asarray(omega0, dtype=np.float64).reshape(-1, 2)
    o1 = np.asarray(omega1, dtype=np.float64).reshape(-1, 2)
    d = np.asarray(domega, dtype=np.float64).reshape(-1, 2)
    out = np.empty_like(x0)
    for k in range(x0.shape[0]):
        if d[k, 0] != 0.0:
            q = d[k, 0] / (o0[k, 0] - o1[k, 0])
        elif d[k, 1] != 0.0:
            q = d[k, 1] / (o0[k, 1] - o1[k, 1])
        else:
            q = 0.0
        out[k] = x0[k] + q * (x0[k] - x1[k])
    return out
