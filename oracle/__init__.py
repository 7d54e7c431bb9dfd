"""CPU oracle for the mesh-intersection search and the stroboscopic map.

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU-baseline
leg of the benchmark.  The product path never imports this package, and this
package imports nothing from the product path.

Python side of the plain C oracle in oracle.c (loaded through ctypes); see
that file for the definitions and their sources in the paper.  exact.py holds
the rational-arithmetic checks, spectral.py the FFT translation, derivative
and trigonometric interpolation in theta, fourier_taylor.py the Fourier-Taylor
charts, their globalized partials and the chart-based Newton.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

HIT_DTYPE = np.dtype([
    ("triA", np.int32), ("triB", np.int32), ("flags", np.uint32), ("pad", np.uint32),
    ("u", np.float64), ("v", np.float64), ("a", np.float64), ("b", np.float64),
    ("X", np.float64, (4,)),
    ("thA", np.float64), ("sA", np.float64), ("thB", np.float64), ("sB", np.float64),
    ("margin", np.float64),
])
assert HIT_DTYPE.itemsize == 120

# pair_test status codes
ST_AABB, ST_MOLLER, ST_DEGENERATE, ST_OUTSIDE, ST_HIT = range(5)


class _Mesh(C.Structure):
    _fields_ = [("V", C.c_void_p), ("n_theta_v", C.c_int32), ("n_s_v", C.c_int32),
                ("periodic", C.c_int32), ("pad", C.c_int32),
                ("theta", C.c_void_p), ("s", C.c_void_p)]


class _Result(C.Structure):
    _fields_ = [("n_cand", C.c_int64), ("cand", C.POINTER(C.c_int64)),
                ("n_hits", C.c_int64), ("hits", C.c_void_p),
                ("counts", C.c_int64 * 8),
                ("n_entries", C.c_int64), ("n_slots", C.c_int64), ("n_boxes", C.c_int64)]


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIB") or _build.ensure_built()   # ORACLE_LIB: the sanitizer build
        L = C.CDLL(path)
        P, I64, I32, D = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        L.orc_n_tris.argtypes = [C.POINTER(_Mesh)]; L.orc_n_tris.restype = I64
        L.orc_tri_verts.argtypes = [C.POINTER(_Mesh), I64, P]; L.orc_tri_verts.restype = None
        L.orc_tri_aabb.argtypes = [C.POINTER(_Mesh), I64, P, P]; L.orc_tri_aabb.restype = None
        L.orc_pair.argtypes = [C.POINTER(_Mesh), I64, C.POINTER(_Mesh), I64, P]; L.orc_pair.restype = C.c_int
        L.orc_solve4.argtypes = [P, P, P]; L.orc_solve4.restype = C.c_int
        L.orc_moller_reject.argtypes = [P, P]; L.orc_moller_reject.restype = C.c_int
        L.orc_bruteforce.argtypes = [C.POINTER(_Mesh), C.POINTER(_Mesh), C.c_int, C.POINTER(_Result), C.c_int]
        L.orc_bruteforce.restype = C.c_int
        L.orc_grid_search.argtypes = [C.POINTER(_Mesh), C.POINTER(_Mesh), P, D, P, C.c_int, C.POINTER(_Result), C.c_int]
        L.orc_grid_search.restype = C.c_int
        L.orc_grid_entries.argtypes = [C.POINTER(_Mesh), P, D, P]; L.orc_grid_entries.restype = I64
        L.orc_cell_of.argtypes = [D, D, D, I64]; L.orc_cell_of.restype = I64
        L.orc_tri_entries.argtypes = [C.POINTER(_Mesh), I64, P, D, P, P, I64]; L.orc_tri_entries.restype = I64
        L.orc_result_free.argtypes = [C.POINTER(_Result)]; L.orc_result_free.restype = None
        L.orc_rk8_tableau.argtypes = [P, P, P]; L.orc_rk8_tableau.restype = None
        L.orc_rk8_map.argtypes = [P, P, I64, D, D, I32, I32, C.c_int]; L.orc_rk8_map.restype = C.c_int
        L.orc_rk8_tangent.argtypes = [P, P, I32, I32, P, P, I64, D, D, I32, I32, C.c_int]
        L.orc_rk8_tangent.restype = C.c_int
        L.orc_jacobi.argtypes = [P, D]; L.orc_jacobi.restype = D
        L.orc_energy_balance.argtypes = [P, D, D, I32, I32, P]; L.orc_energy_balance.restype = C.c_int
        L.orc_mismatch.argtypes = [P, I64, P, P, D, D, I32, I32, I32, P, P, P, P, C.c_int]
        L.orc_mismatch.restype = C.c_int
        L.orc_pertbp_anomaly.argtypes = [D, D, P, P, P, P]; L.orc_pertbp_anomaly.restype = None
        L.orc_pertbp_hamiltonian.argtypes = [P, D, D, D]; L.orc_pertbp_hamiltonian.restype = D
        L.orc_pertbp_flow.argtypes = [P, P, P, I64, D, D, D, D, I64, C.c_int]
        L.orc_pertbp_flow.restype = C.c_int
        L.orc_max_threads.argtypes = []; L.orc_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class OMesh:
    """Holds numpy buffers alive for the C view of a mesh."""

    def __init__(self, mesh):
        self.V = np.ascontiguousarray(mesh.verts, dtype=np.float64)
        self.theta = np.ascontiguousarray(mesh.theta, dtype=np.float64)
        self.s = np.ascontiguousarray(mesh.s, dtype=np.float64)
        assert self.V.shape == (len(self.s), len(self.theta), 4)
        self.c = _Mesh(self.V.ctypes.data, len(self.theta), len(self.s), int(bool(mesh.periodic)), 0,
                       self.theta.ctypes.data, self.s.ctypes.data)

    @property
    def ref(self):
        return C.byref(self.c)


def n_tris(mesh) -> int:
    return int(lib().orc_n_tris(OMesh(mesh).ref))


def tri_verts(mesh, t: int) -> np.ndarray:
    om = OMesh(mesh)
    out = np.empty((3, 4))
    lib().orc_tri_verts(om.ref, int(t), _ptr(out))
    return out


def tri_aabb(mesh, t: int):
    om = OMesh(mesh)
    lo = np.empty(4); hi = np.empty(4)
    lib().orc_tri_aabb(om.ref, int(t), _ptr(lo), _ptr(hi))
    return lo, hi


def pair(meshA, ta: int, meshB, tb: int):
    """Status code of the predicate on one pair, and the hit record if any."""
    a, b = OMesh(meshA), OMesh(meshB)
    h = np.zeros(1, dtype=HIT_DTYPE)
    st = lib().orc_pair(a.ref, int(ta), b.ref, int(tb), _ptr(h))
    return int(st), (h[0] if st == ST_HIT else None)


def solve4(p: np.ndarray, q: np.ndarray):
    p = np.ascontiguousarray(p, dtype=np.float64); q = np.ascontiguousarray(q, dtype=np.float64)
    z = np.zeros(4)
    ok = lib().orc_solve4(_ptr(p), _ptr(q), _ptr(z))
    return bool(ok), z


def moller_reject(p: np.ndarray, q: np.ndarray) -> bool:
    p = np.ascontiguousarray(p, dtype=np.float64); q = np.ascontiguousarray(q, dtype=np.float64)
    return bool(lib().orc_moller_reject(_ptr(p), _ptr(q)))


class SearchResult:
    def __init__(self, res: _Result):
        self.cand = np.ctypeslib.as_array(res.cand, shape=(res.n_cand,)).copy() if res.n_cand else np.zeros(0, np.int64)
        if res.n_hits:
            buf = (C.c_char * (res.n_hits * HIT_DTYPE.itemsize)).from_address(res.hits)
            self.hits = np.frombuffer(bytes(buf), dtype=HIT_DTYPE).copy()
        else:
            self.hits = np.zeros(0, dtype=HIT_DTYPE)
        c = list(res.counts)
        self.counts = dict(examined=c[0], aabb_pass=c[1], moller_reject=c[2], degenerate=c[3],
                           outside=c[4], hits=c[5], nonfinite_A=c[6], nonfinite_B=c[7])
        self.n_entries = int(res.n_entries)
        self.n_slots = int(res.n_slots)
        self.n_boxes = int(res.n_boxes)

    @property
    def hit_pairs(self) -> np.ndarray:
        return (self.hits["triA"].astype(np.int64) << 32) | self.hits["triB"].astype(np.int64)


def bruteforce(meshA, meshB, forced: bool = False, nthreads: int = 0) -> SearchResult:
    """All pairs: C = AABB-overlapping pairs, H = pairs satisfying P (sorted)."""
    a, b = OMesh(meshA), OMesh(meshB)
    res = _Result()
    rc = lib().orc_bruteforce(a.ref, b.ref, int(forced), C.byref(res), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"orc_bruteforce failed ({rc})")
    out = SearchResult(res)
    lib().orc_result_free(C.byref(res))
    return out


def grid_search(meshA, meshB, w_lo, inv_edge: float, n_cells, nthreads: int = 0, prune: bool = False) -> SearchResult:
    """Uniform-grid search with per-box lists (paper Sec. 6.2.1), then the
    AABB, Moller and narrow-phase tests; C and H are sorted and distinct.
    prune: the world-bound restriction of Sec. 6.2.1 (triangles whose box
    misses the other mesh's box take no part in the grid)."""
    a, b = OMesh(meshA), OMesh(meshB)
    wl = np.ascontiguousarray(w_lo, dtype=np.float64)
    nc = np.ascontiguousarray(n_cells, dtype=np.int64)
    res = _Result()
    rc = lib().orc_grid_search(a.ref, b.ref, _ptr(wl), float(inv_edge), _ptr(nc), int(bool(prune)), C.byref(res),
                               int(nthreads))
    if rc != 0:
        raise RuntimeError(f"orc_grid_search failed ({rc})")
    out = SearchResult(res)
    lib().orc_result_free(C.byref(res))
    return out


def grid_entries(mesh, w_lo, inv_edge: float, n_cells) -> int:
    om = OMesh(mesh)
    wl = np.ascontiguousarray(w_lo, dtype=np.float64)
    nc = np.ascontiguousarray(n_cells, dtype=np.int64)
    return int(lib().orc_grid_entries(om.ref, _ptr(wl), float(inv_edge), _ptr(nc)))


def cell_of(x: float, w_lo: float, inv_edge: float, n: int) -> int:
    """Cell of coordinate x on one axis of the grid (Sec. 6.2.1, 0-based
    floor form, clamped to [0, n - 1])."""
    return int(lib().orc_cell_of(float(x), float(w_lo), float(inv_edge), int(n)))


def tri_entries(mesh, t: int, w_lo, inv_edge: float, n_cells) -> np.ndarray | None:
    """Linear cell ids of triangle t's grid entries, in the grid search's
    emission order; None for a non-finite triangle."""
    om = OMesh(mesh)
    wl = np.ascontiguousarray(w_lo, dtype=np.float64)
    nc = np.ascontiguousarray(n_cells, dtype=np.int64)
    cnt = int(lib().orc_tri_entries(om.ref, int(t), _ptr(wl), float(inv_edge), _ptr(nc), None, 0))
    if cnt < 0:
        return None
    out = np.zeros(max(cnt, 1), np.int64)
    lib().orc_tri_entries(om.ref, int(t), _ptr(wl), float(inv_edge), _ptr(nc), _ptr(out), cnt)
    return out[:cnt]


def max_threads() -> int:
    return int(lib().orc_max_threads())


def rk8_tableau():
    a = np.zeros((11, 11)); b = np.zeros(11); c = np.zeros(11)
    lib().orc_rk8_tableau(_ptr(a), _ptr(b), _ptr(c))
    return a, b, c


def rk8_map(states: np.ndarray, mu: float, e: float, steps_per_period: int, n_periods: int,
            nthreads: int = 0) -> np.ndarray:
    x = np.ascontiguousarray(states, dtype=np.float64).reshape(-1, 4)
    out = np.empty_like(x)
    rc = lib().orc_rk8_map(_ptr(x), _ptr(out), x.shape[0], float(mu), float(e), int(steps_per_period),
                           int(n_periods), int(nthreads))
    if rc != 0:
        raise RuntimeError("orc_rk8_map failed")
    return out.reshape(np.shape(states))


def rk8_tangent(states: np.ndarray, dirs: np.ndarray, e_col: int, mu: float, e: float,
                steps_per_period: int, n_periods: int, nthreads: int = 0):
    """states (n,4), dirs (n, nd, 4): returns (F^n(states), DF^n dirs [+ dF/de in column e_col])."""
    x = np.ascontiguousarray(states, dtype=np.float64).reshape(-1, 4)
    d = np.ascontiguousarray(dirs, dtype=np.float64).reshape(x.shape[0], -1, 4)
    nd = d.shape[1]
    out = np.empty_like(x); dout = np.empty_like(d)
    rc = lib().orc_rk8_tangent(_ptr(x), _ptr(d), nd, int(e_col), _ptr(out), _ptr(dout), x.shape[0],
                               float(mu), float(e), int(steps_per_period), int(n_periods), int(nthreads))
    if rc != 0:
        raise RuntimeError("orc_rk8_tangent failed")
    return out, dout


def jacobi(state, mu: float) -> float:
    y = np.ascontiguousarray(state, dtype=np.float64)
    return float(lib().orc_jacobi(_ptr(y), float(mu)))


def pertbp_anomaly(t: float, eps: float):
    """(E, rho, n, nu) of the primaries' orbit at time t (Sec. 3.3): eccentric
    anomaly, separation 1 - eps cos E, rate of the true anomaly, true anomaly."""
    v = [C.c_double() for _ in range(4)]
    lib().orc_pertbp_anomaly(float(t), float(eps), *[C.byref(x) for x in v])
    return tuple(x.value for x in v)


def pertbp_hamiltonian(state, mu: float, eps: float, t: float) -> float:
    z = np.ascontiguousarray(state, dtype=np.float64)
    return float(lib().orc_pertbp_hamiltonian(_ptr(z), float(mu), float(eps), float(t)))


def pertbp_flow(states: np.ndarray, mu: float, eps: float, t0: float, t1: float, nsteps: int,
                stm: bool = False, nthreads: int = 0):
    """Flow of the position-momentum elliptic problem from t0 to t1 in nsteps
    RK8 steps; returns out (n,4) or (out, stm (n,4,4)) with stm[p, i, j] =
    d out_i / d in_j."""
    x = np.ascontiguousarray(states, dtype=np.float64).reshape(-1, 4)
    out = np.empty_like(x)
    M = np.empty((x.shape[0], 4, 4)) if stm else None
    rc = lib().orc_pertbp_flow(_ptr(x), _ptr(out), _ptr(M) if stm else None, x.shape[0], float(mu), float(eps),
                               float(t0), float(t1), int(nsteps), int(nthreads))
    if rc != 0:
        raise RuntimeError("orc_pertbp_flow failed")
    return (out, M) if stm else out


def pertbp_map(states: np.ndarray, mu: float, eps: float, steps_per_period: int, n_periods: int,
               stm: bool = False, nthreads: int = 0):
    """Stroboscopic map F^n_periods at periapse (t from 0 to 2 pi n_periods)."""
    return pertbp_flow(states, mu, eps, 0.0, 2.0 * np.pi * n_periods, steps_per_period * abs(n_periods),
                       stm=stm, nthreads=nthreads)


def energy_balance(state, mu: float, e: float, steps_per_period: int, n_periods: int) -> float:
    y = np.ascontiguousarray(state, dtype=np.float64)
    r = np.zeros(1)
    lib().orc_energy_balance(_ptr(y), float(mu), float(e), int(steps_per_period), int(n_periods), _ptr(r))
    return float(r[0])


def mismatch(params: np.ndarray, patch_u, patch_s, mu: float, e: float, steps_per_period: int,
             n_u: int, n_s: int, nthreads: int = 0):
    """f, r, J, grad of f = F^{n_u}(x_u(th1,s1)) - F^{n_s}(x_s(th2,s2)) (n_s < 0)."""
    p = np.ascontiguousarray(params, dtype=np.float64).reshape(-1, 4)
    K = p.shape[0]
    pu = np.ascontiguousarray(np.concatenate([patch_u.base, patch_u.d1, patch_u.d2]), dtype=np.float64)
    ps = np.ascontiguousarray(np.concatenate([patch_s.base, patch_s.d1, patch_s.d2]), dtype=np.float64)
    f = np.empty((K, 4)); r = np.empty(K); J = np.empty((K, 4, 5)); g = np.empty((K, 5))
    rc = lib().orc_mismatch(_ptr(p), K, _ptr(pu), _ptr(ps), float(mu), float(e), int(steps_per_period),
                            int(n_u), int(n_s), _ptr(f), _ptr(r), _ptr(J), _ptr(g), int(nthreads))
    if rc != 0:
        raise RuntimeError("orc_mismatch failed")
    return f, r, J, g


def gepp4(M, rhs):
    """Solve M z = rhs for a 4 x 4 system by Gaussian elimination with partial
    pivoting, in plain double arithmetic: the pivot of column k is the first
    row (from k down) of largest magnitude; an exact zero pivot means the
    system is singular.  Returns (ok, z) with z None when singular."""
    A = [[float(M[i][j]) for j in range(4)] for i in range(4)]
    r = [float(x) for x in rhs]
    for k in range(4):
        piv, best = k, abs(A[k][k])
        for i in range(k + 1, 4):
            if abs(A[i][k]) > best:
                piv, best = i, abs(A[i][k])
        if piv != k:
            A[k], A[piv] = A[piv], A[k]
            r[k], r[piv] = r[piv], r[k]
        if A[k][k] == 0.0:
            return False, None
        for i in range(k + 1, 4):
            l = A[i][k] / A[k][k]
            for j in range(k + 1, 4):
                A[i][j] = A[i][j] - l * A[k][j]
            r[i] = r[i] - l * r[k]
    z = [0.0] * 4
    for k in range(3, -1, -1):
        acc = 0.0
        for j in range(k + 1, 4):
            acc = acc + A[k][j] * z[j]
        z[k] = (r[k] - acc) / A[k][k]
    return True, np.array(z)


NEWTON_CONVERGED, NEWTON_LIMIT, NEWTON_STALLED, NEWTON_SINGULAR, NEWTON_NONFINITE = 0, 1, 2, 3, 4


def damped_newton(params, patch_u, patch_s, mu: float, e: float, steps_per_period: int, n_u: int, n_s: int,
                  max_trials: int = 40, tol: float = 1e-12, alpha0: float = 1.0, alpha_min: float = 2.0 ** -30,
                  history: bool = False):
    """Damped Newton refinement of mesh hits (paper Sec. 7):
        x <- x - alpha Df(x)^{-1} f(x),
    with f the mismatch of `mismatch` and Df its first four Jacobian columns.
    The paper picks alpha by trial and error; here alpha starts at alpha0
    after every accepted point and is halved after every trial point whose
    r = |f|^2 is not below the current r (the current point is kept).  Per
    row: stop when r <= tol^2 (converged), after max_trials trial points,
    when alpha < alpha_min, on a singular Df, or on a non-finite f at the
    start.  patch_u / patch_s: one patch for all rows, or a list with one
    per row.  Returns (x, f, r, status, trials[, accepted r sequences])."""
    P = np.ascontiguousarray(params, dtype=np.float64).reshape(-1, 4)
    K = P.shape[0]
    xo = np.empty_like(P); fo = np.full((K, 4), np.nan); ro = np.full(K, np.nan)
    status = np.empty(K, np.int32); trials = np.zeros(K, np.int32)
    hist = []
    tol2 = tol * tol
    for k in range(K):
        q = P[k].copy()
        based, st, tr = False, -1, 0
        p = fp = delta = None
        rp = alpha = 0.0
        seq = []
        pu_k = patch_u[k] if isinstance(patch_u, (list, tuple)) else patch_u
        ps_k = patch_s[k] if isinstance(patch_s, (list, tuple)) else patch_s
        while True:
            f, r, J, _ = mismatch(q[None, :], pu_k, ps_k, mu, e, steps_per_period, n_u, n_s, nthreads=1)
            f, r, J = f[0], float(r[0]), J[0]
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
                    ok, z = gepp4(J[:, :4], -f)
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


def default_grid(meshes, kappa: float):
    """World = box of all finite vertices; edge = kappa x the geometric mean
    over the meshes of each mesh's mean longest 4D triangle edge (a mesh
    without finite triangles left out); cells per axis = max(1, ceil(span x
    inv_edge)).  Returns (w_lo, w_hi, inv_edge, n_cells).  Test helper: the
    grid only decides which pairs are examined (Sec. 6.2.1), never the hit
    set."""
    import math
    lo = np.full(4, np.inf); hi = np.full(4, -np.inf)
    means = []
    for m in meshes:
        v = m.verts
        fin = np.all(np.isfinite(v.reshape(-1, 4)), axis=1)
        if fin.any():
            vv = v.reshape(-1, 4)[fin]
            lo = np.minimum(lo, vv.min(axis=0)); hi = np.maximum(hi, vv.max(axis=0))
        if m.n_tris == 0:
            continue
        w = np.concatenate([v, v[:, :1]], axis=1) if m.periodic else v
        a = w[:-1, :-1]; b = w[:-1, 1:]; c = w[1:, :-1]; d = w[1:, 1:]   # (i,k) (i+1,k) (i,k+1) (i+1,k+1)
        nrm = lambda x: np.sqrt(np.sum(x * x, axis=-1))
        e_diag = nrm(b - c)
        t1 = np.maximum(np.maximum(nrm(b - a), nrm(c - a)), e_diag)
        t2 = np.maximum(np.maximum(nrm(c - d), nrm(b - d)), e_diag)
        allt = np.concatenate([t1.ravel(), t2.ravel()])
        allt = allt[np.isfinite(allt)]
        if allt.size:
            means.append(float(allt.sum()) / allt.size)
    if len(means) == 2:
        gm = math.sqrt(means[0] * means[1])
    elif means:
        gm = float(np.prod(means)) ** (1.0 / len(means))
    else:
        gm = 0.0
    edge = kappa * gm
    if not (edge > 0.0 and math.isfinite(edge)):
        edge = 1.0
    inv = 1.0 / edge
    n = np.array([max(1, int(math.ceil((hi[d] - lo[d]) * inv))) for d in range(4)], dtype=np.int64)
    return lo, hi, inv, n


# ---------------------------------------------------------------------------
# The method of layers (Sec. 5)
# ---------------------------------------------------------------------------

def layer_pairs(n_layers: int) -> list[tuple[int, int, int, int]]:
    """The half-layer pairs a search up to layer L examines (Sec. 5, Sec. 6.2):
    for n = 1..L, U_n^a against S_n^b and S_(n-1)^b, a, b in {+1, -1}, as
    tuples (n, a, m, b); ordered by n, a (+ first), m (n first), b (+ first)."""
    out = []
    for n in range(1, n_layers + 1):
        for a in (1, -1):
            for m in (n, n - 1):
                for b in (1, -1):
                    out.append((n, a, m, b))
    return out


def half_layer_interval(D: float, lam: float, stable: bool, layer: int, sign: int) -> tuple[float, float]:
    """The s interval of half-layer `layer` of sign `sign` (Sec. 5): unstable
    |s| in [D lam^(n-1), D lam^n], stable |s| in [D / lam^(n-1), D / lam^n];
    returned as (lo, hi) in s, lo < hi."""
    if stable:
        ends = (D / lam ** (layer - 1), D / lam ** layer)
    else:
        ends = (D * lam ** (layer - 1), D * lam ** layer)
    a, b = min(ends), max(ends)
    return (a, b) if sign > 0 else (-b, -a)


def half_layer_columns(s, D: float, lam: float, stable: bool, layer: int, sign: int,
                       rel: float = 1e-12) -> tuple[int, int]:
    """The columns of a mesh (s samples increasing) whose s lie in the
    half-layer's interval (the boundaries admitted within a relative `rel`):
    (first, last).  Raises ValueError when fewer than two samples lie in it or
    a boundary is not a sample."""
    s = np.asarray(s, dtype=np.float64)
    lo, hi = half_layer_interval(D, lam, stable, layer, sign)
    tol = rel * max(abs(lo), abs(hi))
    inside = np.nonzero((s >= lo - tol) & (s <= hi + tol))[0]
    if len(inside) < 2 or abs(s[inside[0]] - lo) > tol or abs(s[inside[-1]] - hi) > tol:
        raise ValueError("half-layer boundaries are not samples of the mesh")
    return int(inside[0]), int(inside[-1])
