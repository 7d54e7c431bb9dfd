"""Pins of the oracle's RK8 stroboscopic map (paper Sec. 3, 4.1) and its
tangent (Sec. 7): order conditions of the published tableau, the closed-form
Kepler flow, first integrals, reversibility and finite differences."""
from fractions import Fraction as Fr
import math

import numpy as np
import pytest

import oracle
import synth

MU = 2.528e-5
ECC = 0.0094


# ---------------------------------------------------------------- tableau ---

def _trees(n, memo={}):
    """Rooted trees with n nodes, each a sorted tuple of child subtrees."""
    if n in memo:
        return memo[n]
    if n == 1:
        memo[1] = [()]
        return memo[1]
    out = set()

    def build(rem, acc):
        if rem == 0:
            out.add(tuple(sorted(acc)))
            return
        for k in range(1, rem + 1):
            for t in _trees(k):
                build(rem - k, acc + [t])
    build(n - 1, [])
    memo[n] = sorted(out)
    return memo[n]


def _gamma(t):
    n = 1 + sum(_order(c) for c in t)
    g = n
    for c in t:
        g *= _gamma(c)
    return g


def _order(t):
    return 1 + sum(_order(c) for c in t)


def test_tableau_satisfies_all_order_conditions_to_8():
    """The oracle's Cooper-Verner coefficients (as the doubles it uses, taken
    exactly as rationals) satisfy every Butcher order condition b.Phi(t) =
    1/gamma(t) for the 200 rooted trees of order <= 8 up to their rounding,
    and miss the order-9 conditions (so the check has teeth)."""
    a, b, c = oracle.rk8_tableau()
    s = len(b)
    A = [[Fr(float(a[i, j])) for j in range(s)] for i in range(s)]
    B = [Fr(float(x)) for x in b]
    for i in range(s):
        assert abs(float(sum(A[i])) - c[i]) < 1e-14
        assert all(A[i][j] == 0 for j in range(i, s))   # explicit
    cache = {}

    def phi(t):
        if t in cache:
            return cache[t]
        v = [Fr(1)] * s
        for ch in t:
            w = phi(ch)
            aw = [sum(A[i][j] * w[j] for j in range(s)) for i in range(s)]
            v = [v[i] * aw[i] for i in range(s)]
        cache[t] = v
        return v
    n_trees = 0
    for n in range(1, 9):
        for t in _trees(n):
            val = sum(B[i] * phi(t)[i] for i in range(s))
            assert abs(float(val - Fr(1, _gamma(t)))) < 1e-14, (n, t)
            n_trees += 1
    assert n_trees == 200
    worst9 = max(abs(float(sum(B[i] * phi(t)[i] for i in range(s)) - Fr(1, _gamma(t)))) for t in _trees(9))
    assert worst9 > 1e-6


# ----------------------------------------------------------------- Kepler ---

def _kepler_rotating(y0, T):
    """Closed-form flow of the mu = 0, e = 0 problem (Kepler in a frame
    rotating at unit rate): rotate to inertial, propagate with Lagrange's f and
    g functions and Kepler's equation in the eccentric-anomaly difference,
    rotate back."""
    x, y, vx, vy = y0
    X0 = np.array([x, y]); V0 = np.array([vx - y, vy + x])
    r0 = np.linalg.norm(X0); v2 = V0 @ V0
    a = 1.0 / (2.0 / r0 - v2)
    n = a ** -1.5
    sig = X0 @ V0
    M = n * T
    dE = M
    for _ in range(100):
        F = dE - (1 - r0 / a) * math.sin(dE) + sig / math.sqrt(a) * (1 - math.cos(dE)) - M
        dF = 1 - (1 - r0 / a) * math.cos(dE) + sig / math.sqrt(a) * math.sin(dE)
        step = F / dF
        dE -= step
        if abs(step) < 1e-16:
            break
    f = 1 - a / r0 * (1 - math.cos(dE))
    g = T - (dE - math.sin(dE)) / n
    X = f * X0 + g * V0
    r = np.linalg.norm(X)
    fd = -math.sqrt(a) * math.sin(dE) / (r * r0)
    gd = 1 - a / r * (1 - math.cos(dE))
    V = fd * X0 + gd * V0
    c, s = math.cos(T), math.sin(T)
    xr = np.array([c * X[0] + s * X[1], -s * X[0] + c * X[1]])
    Vr = np.array([c * V[0] + s * V[1], -s * V[0] + c * V[1]])
    vr = Vr - np.array([-xr[1], xr[0]])
    return np.array([xr[0], xr[1], vr[0], vr[1]])


def test_kepler_closed_form_and_eighth_order():
    a, ecc = 0.8, 0.1
    X0 = np.array([a * (1 - ecc), 0.0]); V0 = np.array([0.0, math.sqrt((1 + ecc) / (a * (1 - ecc)))])
    y0 = np.array([X0[0], X0[1], V0[0] + X0[1], V0[1] - X0[0]])
    exact = _kepler_rotating(y0, 2 * math.pi)
    errs = []
    for S in (24, 48, 96):
        y = oracle.rk8_map(y0[None, :], 0.0, 0.0, S, 1)[0]
        errs.append(np.max(np.abs(y - exact)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert all(r > 7.0 for r in rates), (errs, rates)
    y = oracle.rk8_map(y0[None, :], 0.0, 0.0, 4000, 1)[0]
    assert np.max(np.abs(y - exact)) < 1e-12


# --------------------------------------------------------- first integrals ---

def test_jacobi_constant_conserved_when_circular():
    y0 = synth.random_states(8, 3, synth.UNSTABLE_BASE, 1e-3)
    y3 = oracle.rk8_map(y0, MU, 0.0, 4000, 3)
    for a, b in zip(y0, y3):
        assert abs(oracle.jacobi(a, MU) - oracle.jacobi(b, MU)) < 1e-12
    # and it is not conserved once e > 0 (the check would see a dropped term)
    ye = oracle.rk8_map(y0, MU, ECC, 4000, 3)
    assert max(abs(oracle.jacobi(a, MU) - oracle.jacobi(b, MU)) for a, b in zip(y0, ye)) > 1e-6


@pytest.mark.parametrize("n_periods", [3, -3])
def test_energy_balance_elliptic(n_periods):
    """d/df[(x'^2 + y'^2)/2 - w Omega] = -w'(f) Omega, integrated alongside."""
    for y0 in synth.random_states(4, 5, synth.STABLE_BASE, 1e-3):
        assert abs(oracle.energy_balance(y0, MU, ECC, 4000, n_periods)) < 1e-12


# ------------------------------------------------------------ symmetries ---

def test_time_reversal_symmetry():
    """R(x, y, x', y') = (x, -y, -x', y') maps F to its inverse (w is even in f)."""
    R = np.array([1.0, -1.0, -1.0, 1.0])
    y0 = synth.random_states(6, 7, synth.UNSTABLE_BASE, 1e-3)
    lhs = R * oracle.rk8_map(y0, MU, ECC, 4000, 1)
    rhs = oracle.rk8_map(R * y0, MU, ECC, 4000, -1)
    assert np.max(np.abs(lhs - rhs)) < 1e-11


def test_inverse_map_roundtrip_and_richardson():
    y0 = synth.random_states(6, 9, synth.STABLE_BASE, 1e-3)
    y3 = oracle.rk8_map(y0, MU, ECC, 4000, 3)
    back = oracle.rk8_map(y3, MU, ECC, 4000, -3)
    assert np.max(np.abs(back - y0)) < 1e-11
    fine = oracle.rk8_map(y0, MU, ECC, 16000, 3)
    assert np.max(np.abs(fine - y3)) < 1e-11


# ---------------------------------------------------------------- tangent ---

def test_tangent_matches_central_differences():
    """DF^3 v and dF^3/de against central differences with h = 1e-6."""
    y0 = synth.random_states(3, 13, synth.UNSTABLE_BASE, 1e-3)
    rng = np.random.default_rng(4)
    dirs = rng.standard_normal((3, 2, 4))
    dirs = np.concatenate([dirs, np.zeros((3, 1, 4))], axis=1)   # column 2: d/de
    S, P = 4000, 3
    y, D = oracle.rk8_tangent(y0, dirs, 2, MU, ECC, S, P)
    h = 1e-6
    for j in range(2):
        fp = oracle.rk8_map(y0 + h * dirs[:, j], MU, ECC, S, P)
        fm = oracle.rk8_map(y0 - h * dirs[:, j], MU, ECC, S, P)
        fd = (fp - fm) / (2 * h)
        rel = np.max(np.abs(fd - D[:, j])) / np.max(np.abs(D[:, j]))
        assert rel < 1e-7, rel
    fp = oracle.rk8_map(y0, MU, ECC + h, S, P)
    fm = oracle.rk8_map(y0, MU, ECC - h, S, P)
    fd = (fp - fm) / (2 * h)
    rel = np.max(np.abs(fd - D[:, 2])) / np.max(np.abs(D[:, 2]))
    assert rel < 1e-7, rel
    assert np.max(np.abs(y - oracle.rk8_map(y0, MU, ECC, S, P))) < 1e-12


def test_mismatch_gradient_is_twice_jt_f():
    (mu_mesh, pu), (ms_mesh, ps) = synth.propagated_patches(4, 4, 0)
    params = np.array([[1e-4, -2e-4, 3e-4, 5e-5], [0.0, 0.0, 0.0, 0.0]])
    f, r, J, g = oracle.mismatch(params, pu, ps, MU, ECC, 400, 1, -1)
    assert np.allclose(r, np.sum(f * f, axis=1), rtol=0, atol=0)
    h = 1e-6
    for k in range(4):
        dp = np.zeros(4); dp[k] = h
        fp, rp, _, _ = oracle.mismatch(params + dp, pu, ps, MU, ECC, 400, 1, -1)
        fm, rm, _, _ = oracle.mismatch(params - dp, pu, ps, MU, ECC, 400, 1, -1)
        assert np.max(np.abs((fp - fm) / (2 * h) - J[:, :, k])) < 1e-7 * np.max(np.abs(J[:, :, k]))
        assert np.max(np.abs((rp - rm) / (2 * h) - g[:, k])) < 1e-7 * max(1e-12, np.max(np.abs(g[:, k])))


# ---------------------------------------------------- closed-form fixed points ---

@pytest.mark.parametrize("mu", [MU, 0.01])
@pytest.mark.parametrize("ecc", [0.0, ECC])
def test_equilateral_points_are_fixed(mu, ecc):
    """The triangular libration points (1/2 - mu, +-sqrt(3)/2) at rest are
    equilibria of the pulsating-coordinate equations for every e, so F fixes
    them (a misplaced primary or a wrong mass weight moves them)."""
    for sgn in (1.0, -1.0):
        L = np.array([[0.5 - mu, sgn * math.sqrt(3.0) / 2.0, 0.0, 0.0]])
        y = oracle.rk8_map(L, mu, ecc, 400, 1)
        assert np.max(np.abs(y - L)) < 1e-13


def test_mass_ratio_mirror_symmetry():
    """Rotating by pi while exchanging the primaries (mu -> 1 - mu) is a
    symmetry: F_{1-mu}(-y) = -F_mu(y)."""
    y0 = synth.random_states(5, 17, (0.3, 0.4, 0.1, -0.2), 0.2)
    mu = 0.3
    a = oracle.rk8_map(y0, mu, ECC, 800, 1)
    b = oracle.rk8_map(-y0, 1.0 - mu, ECC, 800, 1)
    # some of these orbits pass near a primary, which amplifies rounding
    scale = np.maximum(1.0, np.max(np.abs(a), axis=1, keepdims=True))
    assert np.max(np.abs(a + b) / scale) < 1e-10
    # and mu alone matters (the check is sensitive to the mass weights)
    c = oracle.rk8_map(-y0, mu, ECC, 800, 1)
    assert np.max(np.abs(a + c)) > 1e-3
