"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds no arithmetic of the search or of the map: it only draws
random numbers and evaluates the closed-form test surfaces that stand in for
the manifold meshes of the paper (whose Jupiter-Europa manifolds are not
available).  Both the CPU oracle and the HIP path consume the exact bytes
produced here.

Mesh convention (paper Sec. 6.1): a mesh is a grid of vertices W(theta_i, s_k)
stored as an (n_s_v, n_theta_v, 4) float64 array (theta index fastest, the
four coordinates (x, y, p_x, p_y) contiguous), with the sample values
theta[n_theta_v] and s[n_s_v].  A periodic mesh has n_theta_v = N samples
theta_i = 2 pi i / N; quad (i, k) joins theta index i and (i+1) mod N.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclasses.dataclass
class Mesh:
    verts: np.ndarray          # (n_s_v, n_theta_v, 4) float64, C-contiguous
    theta: np.ndarray          # (n_theta_v,) float64
    s: np.ndarray              # (n_s_v,) float64
    periodic: bool

    @property
    def n_theta_v(self) -> int:
        return int(self.verts.shape[1])

    @property
    def n_s_v(self) -> int:
        return int(self.verts.shape[0])

    @property
    def n_quads_theta(self) -> int:
        return self.n_theta_v if self.periodic else max(self.n_theta_v - 1, 0)

    @property
    def n_tris(self) -> int:
        return 2 * self.n_quads_theta * max(self.n_s_v - 1, 0)


# ---------------------------------------------------------------------------
# Closed-form torus-like surfaces (plain search workloads)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class SurfaceCoeffs:
    phi: float
    psi: float
    alpha: np.ndarray   # (4, 5) noise amplitudes in [-1, 1]
    beta: np.ndarray    # (4, 5) noise phases in [0, 2 pi)
    gamma: np.ndarray   # (4, 5) noise s-frequencies in [-pi, pi]
    noise_amp: float = 1e-2


def surface_coeffs(seed: int, noise_amp: float = 1e-2) -> SurfaceCoeffs:
    """Draw (phi, psi, alpha, beta, gamma) in that order from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    phi = float(rng.uniform(0.0, TWO_PI))
    psi = float(rng.uniform(0.0, TWO_PI))
    alpha = rng.uniform(-1.0, 1.0, size=(4, 5))
    beta = rng.uniform(0.0, TWO_PI, size=(4, 5))
    gamma = rng.uniform(-math.pi, math.pi, size=(4, 5))
    return SurfaceCoeffs(phi, psi, alpha, beta, gamma, noise_amp)


def eval_surface(c: SurfaceCoeffs, th: np.ndarray, s: np.ndarray) -> np.ndarray:
    """K(theta, s) = ((1+0.3 s) cos th, (1+0.3 s) sin th, s cos(2 th + phi),
    s sin(th + psi)) + sum_m (amp/5) alpha_{c,m} cos(m th + gamma_{c,m} s + beta_{c,m}).

    th and s broadcast against each other; returns (..., 4)."""
    th = np.asarray(th, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    th, s = np.broadcast_arrays(th, s)
    r = 1.0 + 0.3 * s
    out = np.empty(th.shape + (4,), dtype=np.float64)
    out[..., 0] = r * np.cos(th)
    out[..., 1] = r * np.sin(th)
    out[..., 2] = s * np.cos(2.0 * th + c.phi)
    out[..., 3] = s * np.sin(th + c.psi)
    w = c.noise_amp / 5.0
    for comp in range(4):
        acc = np.zeros(th.shape, dtype=np.float64)
        for m in range(5):
            acc += c.alpha[comp, m] * np.cos((m + 1) * th + c.gamma[comp, m] * s + c.beta[comp, m])
        out[..., comp] += w * acc
    return out


def torus_mesh(n_quads_theta: int, n_quads_s: int, coeffs: SurfaceCoeffs) -> Mesh:
    """Periodic N x M-quad mesh over theta in [0, 2 pi) x s in [0, 1]:
    theta_i = 2 pi i / N (N samples), s_k = k / M (M + 1 samples)."""
    N, M = int(n_quads_theta), int(n_quads_s)
    theta = TWO_PI * np.arange(N, dtype=np.float64) / N
    s = np.arange(M + 1, dtype=np.float64) / M
    verts = eval_surface(coeffs, theta[None, :], s[:, None])
    return Mesh(np.ascontiguousarray(verts), theta, s, True)


def plain_pair(n_quads_theta: int, n_quads_s: int, seed: int = 0,
               noise_amp: float = 1e-2) -> tuple[Mesh, Mesh]:
    """The plain-search workload: surface A from seed, surface B from seed+1."""
    a = torus_mesh(n_quads_theta, n_quads_s, surface_coeffs(seed, noise_amp))
    b = torus_mesh(n_quads_theta, n_quads_s, surface_coeffs(seed + 1, noise_amp))
    return a, b


def layered_s(D: float, lam: float, stable: bool, first: int, last: int, m_quads: int,
              m_core: int = 4) -> np.ndarray:
    """s samples of a manifold mesh whose columns contain the half-layer
    boundaries b_n = D lam^n (unstable) or D / lam^n (stable) for
    n = first-1 .. last: every half-layer [b_(n-1), b_n] (and its mirror) in
    m_quads quads, the core |s| < b_(first-1) in m_core quads; increasing."""
    b = [D / lam ** n if stable else D * lam ** n for n in range(first - 1, last + 1)]
    pos = [np.array([b[0]])]
    for n in range(1, len(b)):
        pos.append(np.linspace(b[n - 1], b[n], m_quads + 1)[1:])
    pos = np.concatenate(pos)
    core = np.linspace(-b[0], b[0], m_core + 1)[1:-1]
    return np.concatenate([-pos[::-1], core, pos])


def layered_mesh(n_theta: int, s: np.ndarray, coeffs: SurfaceCoeffs, eps: float = 0.0, shift: float = 0.0,
                 D: float = 1.0, lam: float = 2.0) -> Mesh:
    """Periodic mesh over theta_i = 2 pi i / n_theta and the given s samples;
    the surface is the closed form P at sigma = s / max|s| (bounded), plus
    eps * (0, 0, sin(2 theta - shift), cos(2 pi l(s))) with l(s) =
    log(|s| / D) / |log lam| the continuous layer index (layer n is
    n - 1 <= l <= n).  With eps != 0 it meets the eps = 0 surface
    transversally at the isolated points theta = shift / 2 + k pi / 2,
    l = n - 3/4 and n - 1/4: eight in every half-layer."""
    theta = TWO_PI * np.arange(n_theta, dtype=np.float64) / n_theta
    s = np.asarray(s, dtype=np.float64)
    sigma = s / np.max(np.abs(s))
    th, sg = theta[None, :], sigma[:, None]
    verts = eval_surface(coeffs, th, sg)
    if eps:
        ell = np.log(np.maximum(np.abs(s), 1e-300) / D) / abs(math.log(lam))
        th2, el2 = np.broadcast_arrays(th, ell[:, None])
        verts[..., 2] += eps * np.sin(2.0 * th2 - shift)
        verts[..., 3] += eps * np.cos(TWO_PI * el2)
    return Mesh(np.ascontiguousarray(verts), theta, s.copy(), True)


@dataclasses.dataclass
class LayeredPair:
    U: Mesh            # unstable-manifold mesh, layers 1..n_layers
    S: Mesh            # stable-manifold mesh, layers 0..n_layers
    D_u: float
    lam_u: float
    D_s: float
    lam_s: float
    n_layers: int


def layered_pair(n_theta_u: int, n_theta_s: int, m_quads: int, n_layers: int, seed: int = 0,
                 D_u: float = 0.05, lam_u: float = 1.35, D_s: float = 0.05, lam_s: float = 1 / 1.35,
                 m_core: int = 4) -> LayeredPair:
    """The layer-search workload of Sec. 5 / 6.4 in synthetic form: an
    unstable mesh with n_theta_u theta samples and the stable one with
    n_theta_s, each half-layer m_quads quads in s (the paper: 1024 / 2048
    samples, 35 columns, 14 layers).  Both surfaces share the closed form of
    `seed`; the stable one is displaced as in layered_mesh (shift drawn from
    seed + 1), so the two cross at isolated points inside every half-layer
    pair (U_n^a, S_n^a) (sigma = s / max|s| agrees between the meshes because
    both reach the same max|s|)."""
    su = layered_s(D_u, lam_u, False, 1, n_layers, m_quads, m_core)
    ss = layered_s(D_s, lam_s, True, 0, n_layers, m_quads, m_core)
    c = surface_coeffs(seed)
    shift = float(np.random.default_rng(seed + 1).uniform(0.0, TWO_PI))
    U = layered_mesh(n_theta_u, su, c)
    S = layered_mesh(n_theta_s, ss, c, eps=0.05, shift=shift, D=D_s, lam=lam_s)
    return LayeredPair(U, S, D_u, lam_u, D_s, lam_s, n_layers)


def crop(mesh: Mesh, i0: int, ni: int, k0: int, nk: int) -> Mesh:
    """Non-periodic crop of ni x nk quads starting at quad (i0, k0)."""
    idx = (np.arange(i0, i0 + ni + 1) % mesh.n_theta_v)
    v = mesh.verts[k0:k0 + nk + 1][:, idx]
    th = mesh.theta[idx].copy()
    # keep theta increasing across the periodic seam
    for j in range(1, len(th)):
        while th[j] <= th[j - 1]:
            th[j] += TWO_PI
    return Mesh(np.ascontiguousarray(v), th, mesh.s[k0:k0 + nk + 1].copy(), False)


# ---------------------------------------------------------------------------
# Batched continuation family
# ---------------------------------------------------------------------------

def family_sizes(n_pairs: int, seed: int) -> list[tuple[int, int, int, int]]:
    """Per pair (N_A, M_A, N_B, M_B): N ~ logU[32, 1024], M ~ logU[16, 128],
    independent per surface, rounded to the nearest integer."""
    rng = np.random.default_rng(seed + 7919)
    out = []
    for _ in range(n_pairs):
        row = []
        for _surf in range(2):
            n = int(round(math.exp(rng.uniform(math.log(32.0), math.log(1024.0)))))
            m = int(round(math.exp(rng.uniform(math.log(16.0), math.log(128.0)))))
            row += [n, m]
        out.append(tuple(row))
    return out


def family(n_pairs: int = 256, seed: int = 0, drift: float = 1e-3,
           sizes: list | None = None) -> list[tuple[Mesh, Mesh]]:
    """A torus-family-like sequence of mesh pairs: member m uses
    phi_m = phi_0 + drift m and psi_m = psi_0 + drift m, noise fixed."""
    ca0 = surface_coeffs(seed)
    cb0 = surface_coeffs(seed + 1)
    if sizes is None:
        sizes = family_sizes(n_pairs, seed)
    pairs = []
    for m, (na, ma, nb, mb) in enumerate(sizes):
        ca = dataclasses.replace(ca0, phi=ca0.phi + drift * m, psi=ca0.psi + drift * m)
        cb = dataclasses.replace(cb0, phi=cb0.phi + drift * m, psi=cb0.psi + drift * m)
        pairs.append((torus_mesh(na, ma, ca), torus_mesh(nb, mb, cb)))
    return pairs


# ---------------------------------------------------------------------------
# Affine and graph-surface plants (closed-form intersections)
# ---------------------------------------------------------------------------

def affine_mesh(p0, d_theta, d_s, theta, s) -> Mesh:
    """Non-periodic mesh of the affine surface W(th, s) = p0 + th d_theta + s d_s
    sampled at the given (increasing) theta and s values."""
    theta = np.asarray(theta, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    p0 = np.asarray(p0, dtype=np.float64)
    d1 = np.asarray(d_theta, dtype=np.float64)
    d2 = np.asarray(d_s, dtype=np.float64)
    v = p0[None, None, :] + theta[None, :, None] * d1[None, None, :] + s[:, None, None] * d2[None, None, :]
    return Mesh(np.ascontiguousarray(v), theta.copy(), s.copy(), False)


def lattice_plant(n_plane: int, n_wave: int, m: int, amp: float = 0.02, power: float = 1.0, seed: int = 0):
    """Many isolated crossings, for large hit counts and crowded cells.

    A is the plane (x, y, 0, 0) over [0, 1]^2 on an n_plane x n_plane quad
    grid whose x samples are (i / n_plane)^power (power > 1 crowds A's
    triangles towards x = 0).  B is the graph
      (x, y, amp sin(2 pi m x + phi), amp sin(2 pi m y + psi)) + small tilt
    over [-0.01, 1.01]^2 on an n_wave x n_wave quad grid.  The two meet near
    the (2m)^2 common zeros of the two sines in the unit square: about
    (2m)^2 triangle pairs intersect.  phi, psi and the tilt are seeded."""
    rng = np.random.default_rng(seed)
    phi, psi = rng.uniform(0.1, 0.9, 2) * TWO_PI
    tilt = rng.uniform(-1e-3, 1e-3, 2)
    xa = (np.arange(n_plane + 1) / n_plane) ** power
    ya = np.arange(n_plane + 1) / n_plane
    VA = np.zeros((n_plane + 1, n_plane + 1, 4))
    VA[:, :, 0] = xa[None, :]
    VA[:, :, 1] = ya[:, None]
    A = Mesh(np.ascontiguousarray(VA), xa.copy(), ya.copy(), False)
    g = np.linspace(-0.01, 1.01, n_wave + 1)
    X, Y = np.meshgrid(g, g)
    VB = np.stack([X, Y, amp * np.sin(TWO_PI * m * X + phi) + tilt[0] * Y,
                   amp * np.sin(TWO_PI * m * Y + psi) + tilt[1] * X], -1)
    B = Mesh(np.ascontiguousarray(VB), g.copy(), g.copy(), False)
    return A, B


# ---------------------------------------------------------------------------
# Propagated-mesh patches (stroboscopic map workloads)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Patch:
    base: np.ndarray   # (4,)
    d1: np.ndarray     # (4,) unit, theta-like direction
    d2: np.ndarray     # (4,) unit, s-like direction, orthogonal to d1


def patch_dirs(seed: int, base) -> Patch:
    """Two seeded Gaussian directions in R^4, Gram-Schmidt orthonormalised."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((2, 4))
    d1 = g[0] / np.linalg.norm(g[0])
    d2 = g[1] - np.dot(g[1], d1) * d1
    d2 = d2 / np.linalg.norm(d2)
    return Patch(np.asarray(base, dtype=np.float64), d1, d2)


UNSTABLE_BASE = (0.92, 0.0, 0.0, 0.05)
STABLE_BASE = (1.08, 0.0, 0.0, -0.05)


def patch_vertices(p: Patch, n_theta_v: int, n_s_v: int, half_width: float = 1e-3) -> Mesh:
    """Grid base + alpha_i d1 + beta_j d2, alpha in linspace(-w, w, n_theta_v),
    beta in linspace(-w, w, n_s_v); non-periodic; (theta, s) = (alpha, beta)."""
    al = np.linspace(-half_width, half_width, n_theta_v)
    be = np.linspace(-half_width, half_width, n_s_v)
    v = p.base[None, None, :] + al[None, :, None] * p.d1[None, None, :] + be[:, None, None] * p.d2[None, None, :]
    return Mesh(np.ascontiguousarray(v), al, be, False)


def propagated_patches(n_quads_theta: int = 2048, n_quads_s: int = 256, seed: int = 0):
    """Unstable and stable seed patches before propagation: (Mesh, Patch) x 2."""
    pu = patch_dirs(seed, UNSTABLE_BASE)
    ps = patch_dirs(seed + 1, STABLE_BASE)
    mu = patch_vertices(pu, n_quads_theta + 1, n_quads_s + 1)
    ms = patch_vertices(ps, n_quads_theta + 1, n_quads_s + 1)
    return (mu, pu), (ms, ps)


def random_states(n: int, seed: int, center=UNSTABLE_BASE, spread: float = 1e-2) -> np.ndarray:
    """n seeded phase-space points around `center` (uniform box of half-width spread)."""
    rng = np.random.default_rng(seed)
    c = np.asarray(center, dtype=np.float64)
    return np.ascontiguousarray(c[None, :] + rng.uniform(-spread, spread, size=(n, 4)))


def periapse_position_momentum(states: np.ndarray, eps: float) -> np.ndarray:
    """Pulsating-coordinate states (x, y, x', y') at periapse (f = 0) rewritten
    as states (x, y, px, py) of the non-pulsating position-momentum frame at
    t = 0: positions scale by the separation 1 - eps, velocities by
    (1 - eps) n0 with n0 = sqrt(1 - eps^2) / (1 - eps)^2 the rate of the true
    anomaly, and p = v + n0 (-y, x).  Used to seed both frames with the same
    physical points."""
    z = np.asarray(states, dtype=np.float64)
    n0 = math.sqrt(1.0 - eps * eps) / (1.0 - eps) ** 2
    q = (1.0 - eps) * z[..., :2]
    v = (1.0 - eps) * n0 * z[..., 2:]
    p = v + n0 * np.stack([-q[..., 1], q[..., 0]], axis=-1)
    return np.ascontiguousarray(np.concatenate([q, p], axis=-1))


def pm_random_states(n: int, seed: int, eps: float, center=UNSTABLE_BASE, spread: float = 1e-2) -> np.ndarray:
    """random_states mapped to the position-momentum frame at periapse."""
    return periapse_position_momentum(random_states(n, seed, center, spread), eps)


# ---------------------------------------------------------------------------
# Planted refinement problems (known roots of the mismatch)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class PlantedRefinement:
    patch_u: Patch            # shared unstable-side patch
    patches_s: list           # one stable-side patch per root
    roots: np.ndarray         # (K, 4) parameters (th1, s1, th2, s2) of the planted roots
    n_periods: int            # the roots solve F^n(x_u) = F^-n(x_s)


def planted_refinement(K: int, seed: int, map_forward, n_periods: int = 3, spread: float = 5e-4):
    """K refinement problems with known roots: points p_k = x_u(th1_k, s1_k)
    of the unstable patch are drawn; the k-th stable patch is centred at
    F^{2n}(p_k), so that F^n(x_u(th1_k, s1_k)) = F^-n(x_s(0, 0)) up to the
    integration error.  `map_forward(states, n_periods)` evaluates F^n on an
    (m, 4) array (the caller supplies it; this module draws numbers only)."""
    (_, pu), (_, ps) = propagated_patches(2, 2, seed)
    rng = np.random.default_rng(seed + 100)
    stars = rng.uniform(-spread, spread, size=(K, 2))
    xu = pu.base[None, :] + stars[:, :1] * pu.d1[None, :] + stars[:, 1:2] * pu.d2[None, :]
    y = np.asarray(map_forward(xu, 2 * n_periods), dtype=np.float64).reshape(K, 4)
    patches = [Patch(y[k].copy(), ps.d1.copy(), ps.d2.copy()) for k in range(K)]
    roots = np.concatenate([stars, np.zeros((K, 2))], axis=1)
    return PlantedRefinement(pu, patches, roots, n_periods)
