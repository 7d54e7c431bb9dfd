"""Pins of the oracle's position-momentum elliptic problem (paper Sec. 3.3):
Kepler's equation and the anomaly rates, the fixed change of coordinates at
periapse that carries the (separately pinned) pulsating-coordinate map onto
this one, the closed-form two-body flow, the first integral of the circular
case, time reversal, and the state transition matrix (symplectic, equal to
finite differences of the map, and carried by the same change of
coordinates onto the pulsating tangent map)."""
import math

import numpy as np
import pytest

import oracle
import synth

MU_JE, ECC_JE = 2.527e-5, 0.0094     # Jupiter-Europa values of Sec. 3.3
MU_EM = 0.0121505856                  # a larger mass ratio, to exercise the second primary

# States of regular orbits for mu = MU_EM (no close passage in a few periods):
# a near-circular orbit about the large primary, and two wider ones.
REGULAR = np.array([[0.3 - MU_EM, 0.0, 0.0, 1.526], [-0.5, 0.1, 0.2, -0.9], [0.0, 0.6, -0.7, 0.0]])


def _C(eps):
    """Matrix of the periapse change of coordinates (pulsating (x, y, x', y')
    -> position-momentum (x, y, px, py)), written out from its definition:
    q = (1 - eps) xi, p = (1 - eps) n0 xi' + n0 (-q_y, q_x)."""
    n0 = math.sqrt(1 - eps * eps) / (1 - eps) ** 2
    a = 1 - eps
    return np.array([[a, 0, 0, 0],
                     [0, a, 0, 0],
                     [0, -n0 * a, a * n0, 0],
                     [n0 * a, 0, 0, a * n0]])


# ------------------------------------------------------------ the anomalies

@pytest.mark.parametrize("eps", [0.0, ECC_JE, 0.3, 0.9])
def test_kepler_equation_and_rates(eps):
    ts = np.concatenate([np.linspace(-7.0, 13.0, 41), [0.0, math.pi, 2 * math.pi]])
    for t in ts:
        E, rho, n, nu = oracle.pertbp_anomaly(t, eps)
        assert abs(E - eps * math.sin(E) - t) <= 4e-16 * (1 + abs(t))
        assert rho == pytest.approx(1 - eps * math.cos(E), abs=1e-15)
        # n is d nu / dt: compare with a central difference of nu (h^2 error)
        h = 1e-5
        nd = (oracle.pertbp_anomaly(t + h, eps)[3] - oracle.pertbp_anomaly(t - h, eps)[3]) / (2 * h)
        assert n == pytest.approx(nd, rel=1e-7)
        # symmetry: E odd, rho and n even in t
        Em, rhom, nm, num = oracle.pertbp_anomaly(-t, eps)
        assert Em == pytest.approx(-E, abs=1e-14)
        assert rhom == pytest.approx(rho, rel=4e-15) and nm == pytest.approx(n, rel=1e-13)
    # closed forms at periapse and apoapse
    _, rho0, n0, nu0 = oracle.pertbp_anomaly(0.0, eps)
    assert rho0 == pytest.approx(1 - eps) and nu0 == 0.0
    assert n0 == pytest.approx(math.sqrt(1 - eps ** 2) / (1 - eps) ** 2, rel=1e-15)
    Epi, rhopi, npi, nupi = oracle.pertbp_anomaly(math.pi, eps)
    assert Epi == pytest.approx(math.pi, abs=1e-15) and nupi == pytest.approx(math.pi, abs=1e-14)
    assert npi == pytest.approx(math.sqrt(1 - eps ** 2) / (1 + eps) ** 2, rel=1e-14)
    # the true anomaly advances by 2 pi per period
    assert oracle.pertbp_anomaly(2 * math.pi, eps)[3] == pytest.approx(2 * math.pi, abs=1e-13)
    if eps == 0.0:
        assert n0 == 1.0 and rho0 == 1.0


# --------------------------------------------- conjugacy to the pulsating map

@pytest.mark.parametrize("eps", [0.0, ECC_JE, 0.2])
@pytest.mark.parametrize("n_periods", [1, -2])
def test_periapse_conjugacy_with_pulsating_map(eps, n_periods):
    """Both frames place periapse at time 0: the pulsating map (its own pins in
    test_oracle_rk8) and this one describe the same motion, so
    F_pm(C z) = C F_puls(z) up to the two integrations' truncation errors."""
    C = _C(eps)
    got = oracle.pertbp_map(REGULAR @ C.T, MU_EM, eps, 2000, n_periods)
    ref = oracle.rk8_map(REGULAR, MU_EM, eps, 2000, n_periods) @ C.T
    assert np.max(np.abs(got - ref)) < 1e-11


def test_periapse_conjugacy_of_the_matrices():
    """DF_pm(C z) = C DF_puls(z) C^-1 (C is linear)."""
    eps = 0.2
    C = _C(eps)
    z = REGULAR
    _, M = oracle.pertbp_map(z @ C.T, MU_EM, eps, 2000, 1, stm=True)
    dirs = np.broadcast_to(np.eye(4), (z.shape[0], 4, 4))
    _, D = oracle.rk8_tangent(z, dirs, -1, MU_EM, eps, 2000, 1)
    Cinv = np.linalg.inv(C)
    for p in range(z.shape[0]):
        ref = C @ D[p].T @ Cinv            # D[p][j] is the image of unit vector j
        assert np.max(np.abs(M[p] - ref)) < 1e-9 * max(1.0, np.abs(ref).max())


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("eps", [0.0, 0.3])
def test_two_body_flow_in_the_turning_frame(eps):
    """mu = 0 leaves a Kepler problem about the origin seen from a frame that
    turns by the true anomaly nu(t): a circular inertial orbit of radius a,
    Q(t) = a (cos(w t + phi), sin(w t + phi)), w = a^-1.5, gives
    q = R(-nu) Q and p = R(-nu) dQ/dt, between two times that are not
    periapses."""
    def state(t, a, phi):
        w = a ** -1.5
        Q = a * np.array([math.cos(w * t + phi), math.sin(w * t + phi)])
        P = a * w * np.array([-math.sin(w * t + phi), math.cos(w * t + phi)])
        nu = oracle.pertbp_anomaly(t, eps)[3]
        R = np.array([[math.cos(nu), math.sin(nu)], [-math.sin(nu), math.cos(nu)]])
        return np.concatenate([R @ Q, R @ P])
    t0, t1 = 0.4, 2.9
    for a, phi in [(0.5, 0.3), (1.7, -2.0), (0.9, 1.0)]:
        got = oracle.pertbp_flow(state(t0, a, phi)[None], 0.0, eps, t0, t1, 3000)[0]
        assert np.max(np.abs(got - state(t1, a, phi))) < 1e-11


def test_circular_case_keeps_its_hamiltonian():
    """eps = 0 makes H time independent (n = 1, rho = 1): a first integral.
    (The drift left is the method's truncation error: it falls by 2^9 per
    halving of the step, 3.6e-10 at 2000 steps per period here.)"""
    z = REGULAR
    out = oracle.pertbp_map(z, MU_EM, 0.0, 4000, 3)
    for p in range(z.shape[0]):
        h0 = oracle.pertbp_hamiltonian(z[p], MU_EM, 0.0, 0.0)
        h1 = oracle.pertbp_hamiltonian(out[p], MU_EM, 0.0, 6 * math.pi)
        assert abs(h1 - h0) < 5e-12 * max(1.0, abs(h0))


def test_eccentric_case_hamiltonian_balance():
    """For eps > 0, dH/dt along a solution is the explicit time derivative
    dH/dt|_z; integrating it by Simpson's rule over a stored trajectory
    matches H(end) - H(start)."""
    eps, mu = 0.2, MU_EM
    z0 = REGULAR[0]
    ts = np.linspace(0.0, 2.0, 401)
    traj = [z0]
    for a, b in zip(ts[:-1], ts[1:]):
        traj.append(oracle.pertbp_flow(traj[-1][None], mu, eps, a, b, 8)[0])
    dHdt = []
    for t, z in zip(ts, traj):
        h = 1e-5
        dHdt.append((oracle.pertbp_hamiltonian(z, mu, eps, t + h) - oracle.pertbp_hamiltonian(z, mu, eps, t - h)) / (2 * h))
    dHdt = np.array(dHdt)
    dt = ts[1] - ts[0]
    simpson = dt / 3 * (dHdt[0] + dHdt[-1] + 4 * dHdt[1:-1:2].sum() + 2 * dHdt[2:-1:2].sum())
    dH = oracle.pertbp_hamiltonian(traj[-1], mu, eps, ts[-1]) - oracle.pertbp_hamiltonian(z0, mu, eps, 0.0)
    assert abs(dH - simpson) < 1e-7
    assert abs(dH) > 1e-3          # H really changes when eps > 0


def test_time_reversal():
    """n and rho are even in t and H is invariant under
    R (x, y, px, py) = (x, -y, -px, py) with t -> -t, so F^-1 = R F R."""
    eps = ECC_JE
    R = np.diag([1.0, -1.0, -1.0, 1.0])
    z = synth.pm_random_states(6, 4, eps)
    back = oracle.pertbp_map(z, MU_JE, eps, 2000, -1)
    ref = oracle.pertbp_map(z @ R, MU_JE, eps, 2000, 1) @ R
    assert np.max(np.abs(back - ref)) < 1e-11
    # and F^-1 F = id
    fw = oracle.pertbp_map(z, MU_JE, eps, 2000, 1)
    assert np.max(np.abs(oracle.pertbp_map(fw, MU_JE, eps, 2000, -1) - z)) < 1e-11


def test_zero_steps_is_identity():
    z = synth.pm_random_states(3, 5, ECC_JE)
    out, M = oracle.pertbp_flow(z, MU_JE, ECC_JE, 0.0, 1.0, 0, stm=True)
    assert np.array_equal(out, z) and np.array_equal(M, np.broadcast_to(np.eye(4), (3, 4, 4)))


# ------------------------------------------------- state transition matrix

def test_stm_is_symplectic():
    """The flow of a Hamiltonian system is symplectic: M^T J M = J, det M = 1."""
    J = np.block([[np.zeros((2, 2)), np.eye(2)], [-np.eye(2), np.zeros((2, 2))]])
    z = np.concatenate([synth.pm_random_states(4, 6, ECC_JE), synth.pm_random_states(4, 7, ECC_JE, synth.STABLE_BASE)])
    _, M = oracle.pertbp_map(z, MU_JE, ECC_JE, 2000, 2, stm=True)
    for m in M:
        assert np.max(np.abs(m.T @ J @ m - J)) < 1e-9 * np.abs(m).max() ** 2
        assert np.linalg.det(m) == pytest.approx(1.0, abs=1e-8)


def test_stm_matches_finite_differences():
    z = synth.pm_random_states(3, 8, ECC_JE)
    _, M = oracle.pertbp_map(z, MU_JE, ECC_JE, 1000, 1, stm=True)
    h = 1e-6
    for j in range(4):
        dz = np.zeros(4)
        dz[j] = h
        fd = (oracle.pertbp_map(z + dz, MU_JE, ECC_JE, 1000, 1) - oracle.pertbp_map(z - dz, MU_JE, ECC_JE, 1000, 1)) / (2 * h)
        assert np.max(np.abs(M[:, :, j] - fd)) < 1e-6 * max(1.0, np.abs(fd).max())
