"""Pins of the oracle's Fourier-Taylor evaluation and globalized partials
(paper Sec. 7): a parameterization with closed-form coefficients (values and
both partials known exactly), Horner against numpy's polynomial evaluation,
the globalized partials against central differences of the globalized
parameterization, and m = 0 reducing to the local one."""
import numpy as np
import pytest

from oracle import fourier_taylor as ft

MU, ECC = 2.527e-5, 0.0094


def closed_form(N, P, seed):
    """W_k(theta) = a_k cos(q_k theta + phi_k) per coordinate, q_k < N/2; returns
    the sampled coefficients and callables for W, dW/dtheta, dW/ds."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((P + 1, 4)) / (1.0 + np.arange(P + 1))[:, None] ** 2
    q = rng.integers(0, N // 2, (P + 1, 4)).astype(float)
    ph = rng.uniform(0, 2 * np.pi, (P + 1, 4))
    th = 2 * np.pi * np.arange(N) / N
    coeffs = a[:, None, :] * np.cos(q[:, None, :] * th[None, :, None] + ph[:, None, :])
    k = np.arange(P + 1)[:, None]

    def W(t, s):
        return np.sum(s ** k * a * np.cos(q * t + ph), axis=0)

    def Wth(t, s):
        return np.sum(-(s ** k) * a * q * np.sin(q * t + ph), axis=0)

    def Ws(t, s):
        kk = np.arange(1, P + 1)[:, None]
        return np.sum(kk * s ** (kk - 1) * a[1:] * np.cos(q[1:] * t + ph[1:]), axis=0)
    return coeffs, W, Wth, Ws


@pytest.mark.parametrize("N,P", [(16, 3), (64, 10), (65, 6), (512, 20)])
def test_local_closed_form(N, P):
    coeffs, W, Wth, Ws = closed_form(N, P, N + P)
    rng = np.random.default_rng(1)
    for t, s in zip(rng.uniform(-4, 8, 12), rng.uniform(-0.9, 0.9, 12)):
        w, dth, ds = ft.local(coeffs, t, s)
        scale = max(1.0, N / 2)
        assert np.max(np.abs(w - W(t, s))) < 1e-12
        assert np.max(np.abs(dth - Wth(t, s))) < 1e-12 * scale
        assert np.max(np.abs(ds - Ws(t, s))) < 1e-12 * P


def test_horner_rows():
    rng = np.random.default_rng(2)
    c = rng.standard_normal((7, 5, 4))
    v, dv = ft.series_rows(c, 0.37)
    for i in range(5):
        for comp in range(4):
            p = np.polynomial.Polynomial(c[:, i, comp])
            assert v[i, comp] == pytest.approx(p(0.37), abs=1e-14)
            assert dv[i, comp] == pytest.approx(p.deriv()(0.37), abs=1e-13)


def _surface(N, P, seed, base):
    """Small smooth coefficients around a base point of the Jupiter-Europa problem."""
    rng = np.random.default_rng(seed)
    th = 2 * np.pi * np.arange(N) / N
    c = np.zeros((P + 1, N, 4))
    c[0] = np.asarray(base)[None, :] + 1e-3 * (np.cos(th)[:, None] * rng.standard_normal(4)
                                               + np.sin(2 * th)[:, None] * rng.standard_normal(4))
    for k in range(1, P + 1):
        c[k] = 1e-2 / k ** 2 * (rng.standard_normal(4)[None, :] * np.cos(k * th)[:, None]
                                 + rng.standard_normal(4)[None, :])
    return c


@pytest.mark.parametrize("m,lam", [(2, 1.35), (-2, 1 / 1.35)])
def test_globalized_partials_by_differences(m, lam):
    import synth
    base = synth.periapse_position_momentum(np.array(synth.UNSTABLE_BASE if m > 0 else synth.STABLE_BASE), ECC)
    c = _surface(32, 5, 3, base)
    omega, t, s = 0.7, 1.1, 0.04
    w, dth, ds = ft.globalized(c, t, s, m, omega, lam, MU, ECC, 1000)
    h = 1e-6
    fd_th = (ft.globalized(c, t + h, s, m, omega, lam, MU, ECC, 1000)[0]
             - ft.globalized(c, t - h, s, m, omega, lam, MU, ECC, 1000)[0]) / (2 * h)
    fd_s = (ft.globalized(c, t, s + h, m, omega, lam, MU, ECC, 1000)[0]
            - ft.globalized(c, t, s - h, m, omega, lam, MU, ECC, 1000)[0]) / (2 * h)
    assert np.max(np.abs(dth - fd_th)) < 1e-6 * max(1.0, np.abs(fd_th).max())
    assert np.max(np.abs(ds - fd_s)) < 1e-6 * max(1.0, np.abs(fd_s).max())


def test_zero_periods_is_local():
    c = _surface(16, 4, 5, (0.9, 0.0, 0.0, 0.97))
    g = ft.globalized(c, 0.3, 0.1, 0, 0.5, 1.35, MU, ECC, 100)
    l_ = ft.local(c, 0.3, 0.1)
    for a, b in zip(g, l_):
        assert np.array_equal(a, b)


def test_newton_finds_a_planted_root():
    """Charts built to meet at a known parameter point: damped Newton from a
    perturbed start converges to it, with r falling quadratically."""
    import synth
    bu = synth.periapse_position_momentum(np.array(synth.UNSTABLE_BASE), ECC)
    bs = synth.periapse_position_momentum(np.array(synth.STABLE_BASE), ECC)
    chart_u, chart_s = (2, 0.61, 1.35), (-2, 0.47, 1 / 1.35)
    root = np.array([1.3, 0.02, 4.1, -0.015])
    cu, cs = ft.planted_charts(32, 4, 11, root, chart_u, chart_s, MU, ECC, 1000, bu, bs)
    f, _ = (ft.globalized(cu, root[0], root[1], *chart_u, MU, ECC, 1000)[0]
            - ft.globalized(cs, root[2], root[3], *chart_s, MU, ECC, 1000)[0]), None
    assert np.max(np.abs(f)) < 1e-12
    x0 = root + np.array([2e-4, -1e-4, 1.5e-4, 1e-4])
    x, fo, r, st, tr, hist = ft.newton(cu, cs, x0[None], chart_u, chart_s, MU, ECC, 1000, tol=1e-12, history=True)
    assert st[0] == 0 and np.max(np.abs(x[0] - root)) < 1e-9
    seq = hist[0]
    assert len(seq) >= 3 and seq[2] < 1e-3 * seq[1] and seq[1] < 1e-2 * seq[0]


def test_continuation_predictor():
    """Exact for solutions that move linearly along the line of rotation
    numbers; the s ratio when omega_u does not change; x0 on a first step."""
    rng = np.random.default_rng(6)
    a, b = rng.standard_normal((5, 4)), rng.standard_normal((5, 4))
    dirn = np.array([[0.3, -0.2]] * 5)
    w0 = np.array([[0.61, 0.47]] * 5)
    x = lambda t: a + t * b                          # the solution at omega = w0 + t dirn
    w1 = w0 - 0.01 * dirn
    got = ft.continuation_predict(x(0.0), w0, 0.02 * dirn, x(-0.01), w1)
    assert np.max(np.abs(got - x(0.02))) < 1e-13
    only_s = np.array([[0.0, 0.4]] * 5)
    got = ft.continuation_predict(x(0.0), w0, 0.05 * only_s, x(-0.02), w0 - 0.02 * only_s)
    assert np.max(np.abs(got - x(0.05))) < 1e-13
    assert np.array_equal(ft.continuation_predict(x(0.0), w0, 0.02 * dirn), x(0.0))
    assert np.array_equal(ft.continuation_predict(x(0.0), w0, 0 * dirn, x(-0.01), w1), x(0.0))
