"""Pins of the oracle's refinement pieces (paper Sec. 7): the 4 x 4 solve by
Gaussian elimination with partial pivoting, and the damped Newton iteration
on mismatch problems with planted roots (quadratic convergence, recovery of
the root, monotone accepted residuals)."""
import math

import numpy as np
import pytest

import oracle
import synth

MU, ECC = 2.528e-5, 0.0094


def test_gepp4_against_library_solve_and_singular_systems():
    rng = np.random.default_rng(1)
    for _ in range(50):
        M = rng.standard_normal((4, 4))
        b = rng.standard_normal(4)
        ok, z = oracle.gepp4(M, b)
        assert ok
        assert np.max(np.abs(M @ z - b)) < 1e-12 * np.linalg.cond(M)
        assert np.max(np.abs(z - np.linalg.solve(M, b))) < 1e-10
    # a zero leading entry needs a row exchange
    M = np.array([[0.0, 1, 2, 3], [1, 0, 1, 0], [2, 1, 0, 1], [0, 0, 1, 1]])
    ok, z = oracle.gepp4(M, np.array([1.0, 2, 3, 4]))
    assert ok and np.allclose(M @ z, [1, 2, 3, 4], atol=1e-14)
    # singular: repeated rows, and a zero column
    assert oracle.gepp4(np.ones((4, 4)), np.ones(4)) == (False, None)
    Z = rng.standard_normal((4, 4)); Z[:, 2] = 0.0
    assert oracle.gepp4(Z, np.ones(4))[0] is False


def _planted(K, seed, steps):
    return synth.planted_refinement(K, seed, lambda x, n: oracle.rk8_map(x, MU, ECC, steps, n))


@pytest.mark.parametrize("steps", [400, 4000])
def test_newton_recovers_planted_roots(steps):
    pr = _planted(3, 0, steps)
    rng = np.random.default_rng(5)
    start = pr.roots + rng.uniform(-1e-4, 1e-4, size=pr.roots.shape)
    x, f, r, st, tr = oracle.damped_newton(start, pr.patch_u, pr.patches_s, MU, ECC, steps, 3, -3)
    assert np.all(st == oracle.NEWTON_CONVERGED), st
    assert np.all(r <= 1e-24)
    # the planted root holds up to the integration error of F^-3 o F^6 vs F^3
    assert np.max(np.abs(x - pr.roots)) < 1e-10


def test_newton_converges_quadratically():
    pr = _planted(4, 2, 400)
    rng = np.random.default_rng(6)
    start = pr.roots + rng.uniform(-3e-4, 3e-4, size=pr.roots.shape)
    *_, st, tr, hist = oracle.damped_newton(start, pr.patch_u, pr.patches_s, MU, ECC, 400, 3, -3, history=True)
    assert np.all(st == oracle.NEWTON_CONVERGED)
    checked = 0
    for seq in hist:
        nf = [math.sqrt(v) for v in seq]
        assert all(b < a for a, b in zip(nf, nf[1:]))          # accepted points decrease r
        for a, b in zip(nf, nf[1:]):
            if a < 1e-4 and b > 1e-11:                         # above the rounding floor
                assert b <= 1e4 * a * a, (a, b)
                checked += 1
    assert checked >= 3


def test_newton_backtracks_from_far_starts():
    """From starts far outside the quadratic basin the step is halved until r
    decreases; accepted residuals are strictly decreasing and every row ends
    with a documented status."""
    pr = _planted(4, 3, 400)
    rng = np.random.default_rng(7)
    start = pr.roots + rng.uniform(-3e-2, 3e-2, size=pr.roots.shape)
    x, f, r, st, tr, hist = oracle.damped_newton(start, pr.patch_u, pr.patches_s, MU, ECC, 400, 3, -3,
                                                 max_trials=60, history=True)
    assert set(st.tolist()) <= {0, 1, 2}
    for seq in hist:
        assert all(b < a for a, b in zip(seq, seq[1:]))
    assert np.any(tr > np.array([len(s) - 1 for s in hist]))   # some trial was rejected


def test_newton_stops_on_singular_jacobian_and_trial_limit():
    pr = _planted(1, 4, 400)
    # a patch with a zero direction: the first column of Df is exactly zero
    bad = synth.Patch(pr.patch_u.base, np.zeros(4), pr.patch_u.d2)
    x, f, r, st, tr = oracle.damped_newton(pr.roots + 1e-5, bad, pr.patches_s, MU, ECC, 400, 3, -3)
    assert st[0] == oracle.NEWTON_SINGULAR and tr[0] == 0
    assert np.array_equal(x, pr.roots + 1e-5)
    x, f, r, st, tr = oracle.damped_newton(pr.roots + 1e-4, pr.patch_u, pr.patches_s, MU, ECC, 400, 3, -3,
                                           max_trials=1)
    assert st[0] == oracle.NEWTON_LIMIT and tr[0] == 1
    assert np.isfinite(r[0])
