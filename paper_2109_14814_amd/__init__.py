"""Python binding of libmsearch.so (the MI355X mesh-intersection search and
stroboscopic-map library; C ABI in include/msearch.h).

Argument marshalling only: every step of the search and of the map runs in
the library's HIP kernels.  PyTorch provides device memory and the current
HIP stream.  Importing this package does not need a GPU; calling into the
library does, and fails loudly when the library is not built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import tune as _tune

_HERE = os.path.dirname(os.path.abspath(__file__))
# MSEARCH_LIB selects another build of the same library (the host-sanitizer build of the CPU checks)
LIB_PATH = os.environ.get("MSEARCH_LIB") or os.path.join(_HERE, "libmsearch.so")

MS_OK, MS_E_ARG, MS_E_CAPACITY, MS_E_HIP, MS_E_NONFINITE, MS_E_KEYBITS, MS_E_WORKSPACE = 0, -1, -2, -3, -4, -5, -6
MS_LAYOUT_AOS, MS_LAYOUT_SOA = 0, 1
MS_SEARCH_CANDIDATES, MS_SEARCH_STRICT, MS_SEARCH_PRUNE = 1, 2, 4
MS_ENUM_WIDE, MS_ENUM_HALF, MS_ENUM_QUARTER = 1, 2, 3

# Exported entry points (the C ABI of include/msearch.h).
EXPORTS = ("last_error", "mesh_build", "mesh_free", "mesh_info", "mesh_update", "search_default_params",
           "search_workspace_size", "search_intersections", "search_intersections_async",
           "search_intersections_noalloc", "narrow_allpairs", "propagate_vertices",
           "search_profile_enable", "search_profile_read", "batch_create", "batch_search", "batch_needed",
           "batch_free", "search_batched_workspace_size", "search_intersections_batched", "refine_workspace_size", "refine_grad", "refine_newton", "layer_pairs",
           "half_layer_bounds", "half_layer_columns", "pertbp_map", "pertbp_map_stm", "theta_shift", "theta_interp", "theta_spectrum",
           "ft_partials", "ft_newton_workspace_size", "ft_newton", "continuation_predict",
           "globalize_workspace_size", "globalize_manifold")

MS_REFINE_RESIDUAL, MS_REFINE_ADJOINT, MS_REFINE_TANGENT, MS_REFINE_NEWTON = 0, 1, 2, 3
NEWTON_STATUS = {0: "converged", 1: "trial limit", 2: "step too small", 3: "singular", 4: "non-finite"}

HIT_DTYPE = np.dtype([
    ("triA", np.int32), ("triB", np.int32), ("flags", np.uint32), ("pad", np.uint32),
    ("u", np.float64), ("v", np.float64), ("a", np.float64), ("b", np.float64),
    ("X", np.float64, (4,)),
    ("thA", np.float64), ("sA", np.float64), ("thB", np.float64), ("sB", np.float64),
    ("margin", np.float64),
])
STATS_FIELDS = ("n_entries", "n_entries_all", "n_cells", "n_slots", "n_cand", "n_moller", "n_degenerate",
                "n_outside", "n_hits", "n_nonfinite", "overflow", "n_groups", "n_group_slots",
                "n_chunks_unstaged")


class MSearchError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class SearchParams(C.Structure):
    _fields_ = [("world_lo", C.c_double * 4), ("inv_edge", C.c_double), ("n_cells", C.c_int64 * 4),
                ("flags", C.c_int32), ("table_log2", C.c_int32), ("enum_shape", C.c_int32), ("reserved", C.c_int32)]


class MeshInfo(C.Structure):
    _fields_ = [("n_tris", C.c_int64), ("n_nonfinite", C.c_int64), ("lo", C.c_double * 4),
                ("hi", C.c_double * 4), ("mean_diam", C.c_double)]


class MapParams(C.Structure):
    _fields_ = [("mu", C.c_double), ("e", C.c_double), ("steps_per_period", C.c_int32), ("n_periods", C.c_int32)]


class NewtonParams(C.Structure):
    _fields_ = [("max_trials", C.c_int32), ("tol", C.c_double), ("alpha0", C.c_double), ("alpha_min", C.c_double)]


class FtChart(C.Structure):
    _fields_ = [("spec_dev", C.c_void_p), ("n_theta", C.c_int32), ("order", C.c_int32), ("n_periods", C.c_int32),
                ("reserved", C.c_int32), ("omega", C.c_double), ("lam", C.c_double)]


_lib = None


def lib():
    """Load libmsearch.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it first (python -m paper_2109_14814_amd.build)")
        L = C.CDLL(LIB_PATH)
        P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.last_error.argtypes = []; L.last_error.restype = C.c_char_p
        L.mesh_build.argtypes = [P, I32, I32, I32, I32, P, P, P, C.POINTER(P)]; L.mesh_build.restype = C.c_int
        L.mesh_free.argtypes = [P]; L.mesh_free.restype = C.c_int
        L.mesh_info.argtypes = [P, C.POINTER(MeshInfo)]; L.mesh_info.restype = C.c_int
        L.search_default_params.argtypes = [P, P, D, C.POINTER(SearchParams)]
        L.search_default_params.restype = C.c_int
        L.search_workspace_size.argtypes = [P, P, C.POINTER(SearchParams), I64, I64, P, C.POINTER(C.c_size_t)]
        L.search_workspace_size.restype = C.c_int
        L.search_intersections.argtypes = [P, P, C.POINTER(SearchParams), P, C.c_size_t, P, I64, P, P, I64, P, P]
        L.search_intersections.restype = C.c_int
        L.search_intersections_async.argtypes = [P, P, C.POINTER(SearchParams), P, C.c_size_t, P, I64, P, P, I64, P]
        L.search_intersections_async.restype = C.c_int
        L.search_intersections_noalloc.argtypes = [P, P, C.POINTER(SearchParams), P, I64, P, P, I64, P]
        L.search_intersections_noalloc.restype = C.c_int
        L.narrow_allpairs.argtypes = [P, P, P, I64, P, P, P]; L.narrow_allpairs.restype = C.c_int
        L.propagate_vertices.argtypes = [P, P, I64, C.POINTER(MapParams), P]
        L.propagate_vertices.restype = C.c_int
        L.pertbp_map.argtypes = [P, P, I64, C.POINTER(MapParams), P]
        L.pertbp_map.restype = C.c_int
        L.pertbp_map_stm.argtypes = [P, P, P, I64, C.POINTER(MapParams), I32, P]
        L.pertbp_map_stm.restype = C.c_int
        L.theta_shift.argtypes = [P, P, I32, I64, P, D, I32, P]
        L.theta_shift.restype = C.c_int
        L.theta_interp.argtypes = [P, I32, I64, P, P, I64, P, P]
        L.theta_interp.restype = C.c_int
        L.theta_spectrum.argtypes = [P, P, I32, I64, P]
        L.theta_spectrum.restype = C.c_int
        L.ft_partials.argtypes = [P, I32, I32, P, P, I64, D, D, C.POINTER(MapParams), P, P, P, P, P]
        L.ft_partials.restype = C.c_int
        L.ft_newton_workspace_size.argtypes = [I64, C.POINTER(C.c_size_t)]
        L.ft_newton_workspace_size.restype = C.c_int
        L.ft_newton.argtypes = [P, P, I64, C.POINTER(FtChart), C.POINTER(FtChart), C.POINTER(MapParams),
                                C.POINTER(NewtonParams), P, P, P, P, P, C.c_size_t, P]
        L.ft_newton.restype = C.c_int
        L.continuation_predict.argtypes = [P, P, P, P, P, I64, P, P]
        L.continuation_predict.restype = C.c_int
        L.globalize_workspace_size.argtypes = [I32, I32, I32, C.POINTER(C.c_size_t)]
        L.globalize_workspace_size.restype = C.c_int
        L.globalize_manifold.argtypes = [P, P, I32, I32, I32, D, D, C.POINTER(MapParams), P, I64, P,
                                         C.POINTER(I64), P, C.c_size_t, P]
        L.globalize_manifold.restype = C.c_int
        L.mesh_update.argtypes = [P, P]; L.mesh_update.restype = C.c_int
        L.batch_create.argtypes = [I32, P, P, P, I64, I64, P, C.POINTER(P), C.POINTER(C.c_size_t)]
        L.batch_create.restype = C.c_int
        L.batch_search.argtypes = [P, P, C.c_size_t, P, I64, P, P, I32, P]; L.batch_search.restype = C.c_int
        L.batch_needed.argtypes = [P, P, P]; L.batch_needed.restype = C.c_int
        L.batch_free.argtypes = [P]; L.batch_free.restype = C.c_int
        L.search_batched_workspace_size.argtypes = [I32, P, P, P, I64, P, C.POINTER(C.c_size_t)]
        L.search_batched_workspace_size.restype = C.c_int
        L.search_intersections_batched.argtypes = [I32, P, P, P, P, C.c_size_t, P, I64, P, P, I32, P]
        L.search_intersections_batched.restype = C.c_int
        L.search_profile_enable.argtypes = [C.c_int]; L.search_profile_enable.restype = C.c_int
        L.search_profile_read.argtypes = [C.c_char_p, C.c_size_t, P, C.c_int, C.POINTER(C.c_int)]
        L.search_profile_read.restype = C.c_int
        MP = C.POINTER(MapParams)
        L.refine_workspace_size.argtypes = [I64, MP, MP, I32, I32, C.POINTER(C.c_size_t)]
        L.refine_workspace_size.restype = C.c_int
        L.refine_grad.argtypes = [P, I64, P, P, I32, MP, MP, I32, I32, P, P, P, P, P, C.c_size_t, P]
        L.refine_grad.restype = C.c_int
        L.refine_newton.argtypes = [P, P, I64, P, P, I32, MP, MP, C.POINTER(NewtonParams), P, P, P, P, P,
                                    C.c_size_t, P]
        L.refine_newton.restype = C.c_int
        L.layer_pairs.argtypes = [I32, P, I32, C.POINTER(C.c_int32)]; L.layer_pairs.restype = C.c_int
        L.half_layer_bounds.argtypes = [D, D, I32, I32, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.half_layer_bounds.restype = C.c_int
        L.half_layer_columns.argtypes = [P, I32, D, D, I32, I32, I32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.half_layer_columns.restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != MS_OK:
        raise MSearchError(rc, lib().last_error().decode())


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_bytes(n: int):
    torch = _torch()
    return torch.empty(max(int(n), 1), dtype=torch.uint8, device="cuda")


def _workspace(n: int):
    """A search workspace, zeroed once so that the work counters of its
    first search are not inflated by leftover occupancy marks."""
    torch = _torch()
    return torch.zeros(max(int(n), 1), dtype=torch.uint8, device="cuda")


class Mesh:
    """A triangulated vertex grid resident in HBM (mesh_build).

    verts: (n_s_v, n_theta_v, 4) float64 (numpy or torch); theta, s: sample values."""

    def __init__(self, verts, theta, s, periodic: bool, layout: int = MS_LAYOUT_AOS):
        torch = _torch()
        self.periodic = bool(periodic)
        self.layout = layout
        v = torch.as_tensor(verts, dtype=torch.float64)
        if layout == MS_LAYOUT_SOA:
            v = v.permute(2, 0, 1)
        self.verts = v.contiguous().to("cuda")
        n_s_v, n_theta_v = (self.verts.shape[1], self.verts.shape[2]) if layout == MS_LAYOUT_SOA else \
            (self.verts.shape[0], self.verts.shape[1])
        self.theta = np.ascontiguousarray(theta, dtype=np.float64)
        self.s = np.ascontiguousarray(s, dtype=np.float64)
        assert len(self.theta) == n_theta_v and len(self.s) == n_s_v
        h = C.c_void_p()
        _check(lib().mesh_build(C.c_void_p(self.verts.data_ptr()), n_theta_v, n_s_v, int(bool(periodic)), layout,
                                self.theta.ctypes.data_as(C.c_void_p), self.s.ctypes.data_as(C.c_void_p),
                                _stream(), C.byref(h)))
        self.handle = h
        inf = MeshInfo()
        _check(lib().mesh_info(h, C.byref(inf)))
        self.n_tris = int(inf.n_tris)
        self.n_nonfinite = int(inf.n_nonfinite)
        self.lo = np.array(inf.lo[:]); self.hi = np.array(inf.hi[:])
        self.mean_diam = float(inf.mean_diam)

    def update(self):
        """Recompute the triangle boxes after self.verts changed in place."""
        _check(lib().mesh_update(self.handle, _stream()))

    def info(self) -> dict:
        """Counts, bounds and mean triangle diameter (mesh_info; waits for a
        pending update)."""
        inf = MeshInfo()
        _check(lib().mesh_info(self.handle, C.byref(inf)))
        self.lo = np.array(inf.lo[:]); self.hi = np.array(inf.hi[:])
        self.mean_diam = float(inf.mean_diam)
        self.n_nonfinite = int(inf.n_nonfinite)
        return {"n_tris": int(inf.n_tris), "n_nonfinite": self.n_nonfinite, "lo": self.lo, "hi": self.hi,
                "mean_diam": self.mean_diam}

    @classmethod
    def from_synth(cls, m, layout: int = MS_LAYOUT_AOS):
        return cls(m.verts, m.theta, m.s, m.periodic, layout)

    def columns(self, k0: int, k1: int) -> "Mesh":
        """The mesh over s-columns k0..k1 of this one (a half-layer), sharing
        its device vertices (AoS layout)."""
        if self.layout != MS_LAYOUT_AOS:
            raise ValueError("column sub-meshes need the AoS layout")
        return Mesh(self.verts[k0:k1 + 1], self.theta, self.s[k0:k1 + 1], self.periodic)

    def close(self):
        if getattr(self, "handle", None):
            lib().mesh_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def default_params(A: Mesh, B: Mesh, kappa: float) -> SearchParams:
    p = SearchParams()
    _check(lib().search_default_params(A.handle, B.handle, float(kappa), C.byref(p)))
    return p


def make_params(w_lo, inv_edge: float, n_cells, flags: int = 0, table_log2: int = 0, enum_shape: int = 0) -> SearchParams:
    p = SearchParams()
    for d in range(4):
        p.world_lo[d] = float(w_lo[d])
        p.n_cells[d] = int(n_cells[d])
    p.inv_edge = float(inv_edge)
    p.flags = int(flags)
    p.table_log2 = int(table_log2)
    p.enum_shape = int(enum_shape)
    return p


def _stats_dict(buf) -> dict:
    arr = buf.view(_torch().int64).cpu().numpy()
    return {k: int(arr[i]) for i, k in enumerate(STATS_FIELDS)}


class Searcher:
    """Device buffers for repeated searches of one mesh pair."""

    def __init__(self, A: Mesh, B: Mesh, params: SearchParams, hits_cap: int = 1 << 16,
                 cand_cap: int = 1 << 20):
        self.A, self.B, self.params = A, B, params
        self.hits_cap, self.cand_cap = int(hits_cap), int(cand_cap)
        self.stats = _dev_bytes(16 * 8)
        self._alloc()

    def _alloc(self):
        nb = C.c_size_t()
        _check(lib().search_workspace_size(self.A.handle, self.B.handle, C.byref(self.params), self.cand_cap,
                                           self.hits_cap, _stream(), C.byref(nb)))
        self.ws_bytes = int(nb.value)
        self.ws = _workspace(self.ws_bytes)
        self.hits = _dev_bytes(self.hits_cap * HIT_DTYPE.itemsize)
        want_cand = bool(self.params.flags & MS_SEARCH_CANDIDATES)
        self.cand = _dev_bytes(self.cand_cap * 8) if want_cand else None

    def _call(self, needed):
        cand_ptr = C.c_void_p(self.cand.data_ptr()) if self.cand is not None else None
        return lib().search_intersections(self.A.handle, self.B.handle, C.byref(self.params),
                                          C.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                                          C.c_void_p(self.hits.data_ptr()), self.hits_cap,
                                          C.c_void_p(self.stats.data_ptr()), cand_ptr, self.cand_cap,
                                          needed, _stream())

    def run(self, retry: bool = True) -> None:
        """One search.  On a capacity error, grow the buffers to the reported
        needs and search again (when retry is set).  A candidate overflow
        only bounds the hit count from below, so a second growth may follow."""
        needed = (C.c_int64 * 3)()
        rc = self._call(needed)
        for _ in range(3 if retry else 0):
            if rc not in (MS_E_CAPACITY, MS_E_WORKSPACE):
                break
            self.hits_cap = max(self.hits_cap, int(needed[0]))
            self.cand_cap = max(self.cand_cap, int(needed[1]))
            self._alloc()
            rc = self._call(needed)
        _check(rc)

    def run_async(self) -> None:
        """Queue one search without waiting (overflow only in the stats;
        check_overflow() after synchronising)."""
        cand_ptr = C.c_void_p(self.cand.data_ptr()) if self.cand is not None else None
        _check(lib().search_intersections_async(self.A.handle, self.B.handle, C.byref(self.params),
                                                C.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                                                C.c_void_p(self.hits.data_ptr()), self.hits_cap,
                                                C.c_void_p(self.stats.data_ptr()), cand_ptr, self.cand_cap, _stream()))

    def check_overflow(self) -> None:
        """Raise if the last search overflowed a buffer."""
        st = _stats_dict(self.stats)
        if st["overflow"]:
            raise MSearchError(MS_E_CAPACITY, f"search overflowed its buffers (flags {st['overflow']}); "
                                              "run() grows them")

    def results(self):
        """(hits structured array sorted by (triA, triB), stats dict, candidates or None)."""
        st = _stats_dict(self.stats)
        nh = min(st["n_hits"], self.hits_cap)
        hits = np.frombuffer(self.hits[: nh * HIT_DTYPE.itemsize].cpu().numpy().tobytes(), dtype=HIT_DTYPE)
        cand = None
        if self.cand is not None:
            nc = min(st["n_cand"], self.cand_cap)
            cand = self.cand[: nc * 8].view(_torch().int64).cpu().numpy().copy()
        return hits, st, cand


KAPPAS = _tune.KAPPAS


def _time_ms(fn, reps: int) -> float:
    torch = _torch()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _device_tag() -> str:
    torch = _torch()
    pr = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(pr, "gcnArchName", "") or pr.name
    return f"{arch.split(':')[0]}x{pr.multi_processor_count}"


def tuned_params(A: Mesh, B: Mesh, choice: dict, flags: int = 0) -> SearchParams:
    """The search parameters of a tuned choice (tune.tune)."""
    p = default_params(A, B, choice["kappa"])
    p.table_log2 = int(choice["table_log2"])
    p.enum_shape = int(choice["enum_shape"])
    p.flags = int(flags)
    return p


def autotune(pairs, batch: bool = False, reps: int | None = None, hits_cap: int = 1 << 16,
             cand_cap: int = 1 << 20, use_cache: bool = True, cache_path: str | None = None, flags: int = 0):
    """The tuned (kappa, table_log2, enum_shape) of a plain search of one
    pair or of a batched search of many (tune.tune: joint sweep, cached per
    size bucket), timed with the search flags `flags`.  Returns (choice,
    per-pair parameters, timings)."""
    if reps is None:
        reps = 3 if batch else 20

    def measure(kappa, table, shape):
        ch = {"kappa": kappa, "table_log2": table, "enum_shape": shape}
        params = [tuned_params(a, b, ch, flags) for a, b in pairs]
        if batch:
            bt = Batch(pairs, params, hits_cap=hits_cap, cand_cap=cand_cap)
            bt.run_checked(True)
            t = _time_ms(lambda: bt.run(True), reps)
            bt.close()
            return t
        s = Searcher(pairs[0][0], pairs[0][1], params[0], hits_cap, cand_cap)
        s.run()
        t = _time_ms(s.run_async, reps)
        s.check_overflow()
        return t

    choice, times = _tune.tune(pairs, measure, _device_tag() + (f"|flags{flags}" if flags else ""), batch, use_cache,
                               cache_path)
    return choice, [tuned_params(a, b, choice, flags) for a, b in pairs], times


def autotune_kappa(A: Mesh, B: Mesh, hits_cap: int = 1 << 10, cand_cap: int = 1 << 20, use_cache: bool = True):
    """The tuned choice for one mesh pair: (choice, parameters, timings)."""
    choice, params, times = autotune([(A, B)], False, hits_cap=hits_cap, cand_cap=cand_cap, use_cache=use_cache)
    return choice, params[0], times


def autotune_batch_kappa(pairs, hits_cap: int = 1 << 16, cand_cap: int = 1 << 22, use_cache: bool = True,
                         flags: int = 0):
    """The tuned choice for a batch (one choice for every pair, one captured
    graph per trial): (choice, per-pair parameters, timings)."""
    return autotune(pairs, True, hits_cap=hits_cap, cand_cap=cand_cap, use_cache=use_cache, flags=flags)


LAYER_PAIR_DTYPE = np.dtype([("u_layer", "<i4"), ("u_sign", "<i4"), ("s_layer", "<i4"), ("s_sign", "<i4")])


def layer_pairs(n_layers: int) -> np.ndarray:
    """The 8 n_layers half-layer pairs of a search up to layer n_layers
    (layer_pairs)."""
    out = np.zeros(max(8 * int(n_layers), 1), dtype=LAYER_PAIR_DTYPE)
    n = C.c_int32()
    _check(lib().layer_pairs(int(n_layers), out.ctypes.data_as(C.c_void_p), len(out), C.byref(n)))
    return out[: n.value]


def half_layer_bounds(D: float, lam: float, stable: bool, layer: int) -> tuple[float, float]:
    lo, hi = C.c_double(), C.c_double()
    _check(lib().half_layer_bounds(float(D), float(lam), int(bool(stable)), int(layer), C.byref(lo), C.byref(hi)))
    return lo.value, hi.value


def half_layer_columns(s, D: float, lam: float, stable: bool, layer: int, sign: int) -> tuple[int, int]:
    """Columns (k0, k1) of a mesh with s samples `s` forming the half-layer
    (half_layer_columns)."""
    s = np.ascontiguousarray(s, dtype=np.float64)
    k0, k1 = C.c_int32(), C.c_int32()
    _check(lib().half_layer_columns(s.ctypes.data_as(C.c_void_p), len(s), float(D), float(lam), int(bool(stable)),
                                    int(layer), int(sign), C.byref(k0), C.byref(k1)))
    return k0.value, k1.value


class LayerSearch:
    """The connection search of Sec. 5 / 6.2 up to layer n_layers: the
    half-layer pairs of an unstable mesh U (multiplier lam_u, fundamental
    domain D_u) and a stable mesh S (lam_s, D_s), each half-layer a column
    sub-mesh sharing the vertices, searched together as one batch."""

    def __init__(self, U: Mesh, S: Mesh, D_u: float, lam_u: float, D_s: float, lam_s: float, n_layers: int,
                 kappa=None, hits_cap: int = 1 << 16, cand_cap: int = 1 << 22, prune: bool = True):
        self.pairs = layer_pairs(n_layers)
        cache = {}

        def half(mesh, stable, D, lam, layer, sign):
            key = (stable, layer, sign)
            if key not in cache:
                cache[key] = mesh.columns(*half_layer_columns(mesh.s, D, lam, stable, layer, sign))
            return cache[key]

        self.meshes = [(half(U, False, D_u, lam_u, int(p["u_layer"]), int(p["u_sign"])),
                        half(S, True, D_s, lam_s, int(p["s_layer"]), int(p["s_sign"]))) for p in self.pairs]
        self.halves = cache
        # world-bound pruning (Sec. 6.2.1): a half-layer's triangles outside
        # the other half-layer's box take no part (the hits do not change)
        flags = MS_SEARCH_PRUNE if prune else 0
        if kappa is None:
            self.tuned, params, self.kappa_times = autotune_batch_kappa(self.meshes, hits_cap=hits_cap,
                                                                        cand_cap=cand_cap, flags=flags)
            self.kappa = self.tuned["kappa"]
        else:
            self.kappa, self.kappa_times, self.tuned = float(kappa), {}, None
            params = [default_params(a, b, self.kappa) for a, b in self.meshes]
            for p in params:
                p.flags = flags
        self.params = params
        self.batch = Batch(self.meshes, params, hits_cap=hits_cap, cand_cap=cand_cap)

    def run(self, use_graph: bool = True) -> None:
        self.batch.run_checked(use_graph)

    def results(self):
        """(per-pair hit arrays, in the order of self.pairs; stats)."""
        return self.batch.results()


def profile_enable(on: bool = True):
    _check(lib().search_profile_enable(int(bool(on))))


def profile_read():
    """[(kernel name, ms)] of every kernel launched by mesh updates and searches
    since the previous read, while profiling is enabled (dispatch timestamps)."""
    cap = 256
    names = C.create_string_buffer(8192)
    arr = (C.c_double * cap)()
    n = C.c_int()
    _check(lib().search_profile_read(names, 8192, arr, cap, C.byref(n)))
    nm = names.value.decode().split(",") if n.value else []
    return list(zip(nm, arr[: n.value]))


def search(A: Mesh, B: Mesh, params: SearchParams, hits_cap: int = 1 << 16, cand_cap: int = 1 << 20):
    s = Searcher(A, B, params, hits_cap, cand_cap)
    s.run()
    return s.results()


def search_noalloc(A: Mesh, B: Mesh, params: SearchParams, hits, stats, cand=None) -> None:
    """Queue search_intersections_noalloc into caller-owned device buffers
    (hits: hits_cap x 120 bytes, stats: 128 bytes, cand: optional int64
    tensor); the library's fixed scratch is the workspace."""
    hits_cap = hits.numel() * hits.element_size() // HIT_DTYPE.itemsize
    cand_ptr = C.c_void_p(cand.data_ptr()) if cand is not None else None
    cand_cap = cand.numel() if cand is not None else 0
    _check(lib().search_intersections_noalloc(A.handle, B.handle, C.byref(params), C.c_void_p(hits.data_ptr()),
                                              int(hits_cap), C.c_void_p(stats.data_ptr()), cand_ptr, int(cand_cap),
                                              _stream()))


class Batch:
    """Many mesh pairs searched by one pass of the pipeline (batch_create /
    batch_search); with use_graph the kernel sequence is a captured HIP graph."""

    def __init__(self, pairs, params, hits_cap: int = 1 << 16, cand_cap: int = 1 << 20):
        self.pairs = list(pairs)
        self.params = list(params)
        n = len(self.pairs)
        self._A = (C.c_void_p * n)(*[a.handle for a, _ in self.pairs])
        self._B = (C.c_void_p * n)(*[b.handle for _, b in self.pairs])
        self._P = (SearchParams * n)(*self.params)
        self.hits_cap, self.cand_cap = int(hits_cap), int(cand_cap)
        self.handle = None
        self.stats = _dev_bytes(16 * 8)
        self.offsets = _torch().zeros(n + 1, dtype=_torch().int64, device="cuda")
        self._create()

    def _create(self):
        if self.handle:
            lib().batch_free(self.handle)
        h = C.c_void_p()
        nb = C.c_size_t()
        _check(lib().batch_create(len(self.pairs), self._A, self._B, self._P, self.hits_cap, self.cand_cap,
                                  _stream(), C.byref(h), C.byref(nb)))
        self.handle = h
        self.ws_bytes = int(nb.value)
        self.ws = _workspace(self.ws_bytes)
        self.hits = _dev_bytes(self.hits_cap * HIT_DTYPE.itemsize)

    def run(self, use_graph: bool = True) -> None:
        """Queue one search of every pair (no host synchronisation)."""
        _check(lib().batch_search(self.handle, C.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                                  C.c_void_p(self.hits.data_ptr()), self.hits_cap,
                                  C.c_void_p(self.offsets.data_ptr()), C.c_void_p(self.stats.data_ptr()),
                                  int(bool(use_graph)), _stream()))

    def run_checked(self, use_graph: bool = True) -> None:
        """Search, and on a capacity overflow re-plan with the reported sizes and search again."""
        for _ in range(3):
            self.run(use_graph)
            st = self.stats_dict()
            if st["overflow"] == 0:
                return
            needed = (C.c_int64 * 3)()
            sh = (C.c_int64 * 16)(*self.stats.view(_torch().int64).cpu().tolist())
            _check(lib().batch_needed(self.handle, sh, needed))
            self.hits_cap = max(self.hits_cap, int(needed[0]))
            self.cand_cap = max(self.cand_cap, int(needed[1]))
            self._create()
        raise MSearchError(MS_E_CAPACITY, "batch: capacity still exceeded after re-planning")

    def stats_dict(self) -> dict:
        return _stats_dict(self.stats)

    def results(self):
        """(list of per-pair hit arrays sorted by (triA, triB), stats dict)."""
        st = self.stats_dict()
        nh = min(st["n_hits"], self.hits_cap)
        hits = np.frombuffer(self.hits[: nh * HIT_DTYPE.itemsize].cpu().numpy().tobytes(), dtype=HIT_DTYPE)
        off = self.offsets.cpu().numpy()
        return [hits[off[i]:off[i + 1]] for i in range(len(self.pairs))], st

    def close(self):
        if getattr(self, "handle", None):
            lib().batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def search_batched(pairs, params, hits_cap: int = 1 << 16, use_graph: bool = True, buffers=None):
    """search_intersections_batched of the C ABI: every (A, B) mesh pair of
    `pairs` with its own grid; returns (per-pair hit arrays sorted by (triA,
    triB), stats dict, buffers).  Pass the returned buffers back to repeat the
    search on the same buffers (the library then reuses its plan and graph);
    they are re-sized when the counts outgrow them."""
    torch = _torch()
    n = len(pairs)
    A = (C.c_void_p * n)(*[a.handle for a, _ in pairs])
    B = (C.c_void_p * n)(*[b.handle for _, b in pairs])
    P = (SearchParams * n)(*params)
    if buffers is None:
        nb = C.c_size_t()
        _check(lib().search_batched_workspace_size(n, A, B, P, int(hits_cap), _stream(), C.byref(nb)))
        buffers = {"ws": _workspace(nb.value), "hits": _dev_bytes(int(hits_cap) * HIT_DTYPE.itemsize),
                   "hits_cap": int(hits_cap), "offs": torch.zeros(n + 1, dtype=torch.int64, device="cuda"),
                   "stats": _dev_bytes(16 * 8)}
    b = buffers
    for _ in range(3):
        _check(lib().search_intersections_batched(n, A, B, P, C.c_void_p(b["ws"].data_ptr()), b["ws"].numel(),
                                                  C.c_void_p(b["hits"].data_ptr()), b["hits_cap"],
                                                  C.c_void_p(b["offs"].data_ptr()), C.c_void_p(b["stats"].data_ptr()),
                                                  int(bool(use_graph)), _stream()))
        st = _stats_dict(b["stats"])
        if st["overflow"] == 0:
            break
        b["hits_cap"] = max(b["hits_cap"], st["n_hits"])
        nb = C.c_size_t()
        _check(lib().search_batched_workspace_size(n, A, B, P, b["hits_cap"], _stream(), C.byref(nb)))
        b["ws"] = _workspace(max(nb.value, b["ws"].numel()))
        b["hits"] = _dev_bytes(b["hits_cap"] * HIT_DTYPE.itemsize)
    else:
        raise MSearchError(MS_E_CAPACITY, "search_batched: capacity still exceeded")
    nh = min(st["n_hits"], b["hits_cap"])
    hits = np.frombuffer(b["hits"][: nh * HIT_DTYPE.itemsize].cpu().numpy().tobytes(), dtype=HIT_DTYPE)
    off = b["offs"].cpu().numpy()
    return [hits[off[i]:off[i + 1]] for i in range(n)], st, b


def narrow_allpairs(A: Mesh, B: Mesh, hits_cap: int = 1 << 16):
    """All pairs with the full test on every pair: (hits in the order the
    kernel wrote them, stats)."""
    torch = _torch()
    hits = _dev_bytes(hits_cap * HIT_DTYPE.itemsize)
    nh = torch.zeros(1, dtype=torch.int64, device="cuda")
    stats = _dev_bytes(16 * 8)
    _check(lib().narrow_allpairs(A.handle, B.handle, C.c_void_p(hits.data_ptr()), int(hits_cap),
                                 C.c_void_p(nh.data_ptr()), C.c_void_p(stats.data_ptr()), _stream()))
    st = _stats_dict(stats)
    n = min(int(nh.item()), hits_cap)
    h = np.frombuffer(hits[: n * HIT_DTYPE.itemsize].cpu().numpy().tobytes(), dtype=HIT_DTYPE)
    return h, st


def propagate(states, mu: float, e: float, steps_per_period: int, n_periods: int, out=None):
    """F^n_periods of (n, 4) states on the GPU (torch float64 cuda tensor in, tensor out)."""
    torch = _torch()
    x = torch.as_tensor(states, dtype=torch.float64).to("cuda").contiguous()
    assert x.shape[-1] == 4
    if out is None:
        out = torch.empty_like(x)
    p = MapParams(float(mu), float(e), int(steps_per_period), int(n_periods))
    _check(lib().propagate_vertices(C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()), x.numel() // 4,
                                    C.byref(p), _stream()))
    return out


def pertbp_map(states, mu: float, eps: float, steps_per_period: int, n_periods: int, out=None):
    """F^n_periods of (n, 4) position-momentum states (x, y, px, py) of the
    elliptic problem of Sec. 3.3 on the GPU (pertbp_map of the C ABI)."""
    torch = _torch()
    x = torch.as_tensor(states, dtype=torch.float64).to("cuda").contiguous()
    assert x.shape[-1] == 4
    if out is None:
        out = torch.empty_like(x)
    p = MapParams(float(mu), float(eps), int(steps_per_period), int(n_periods))
    _check(lib().pertbp_map(C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()), x.numel() // 4, C.byref(p),
                            _stream()))
    return out


def pertbp_map_stm(states, mu: float, eps: float, steps_per_period: int, n_periods: int,
                   cols_per_thread: int = 0, want_out: bool = True):
    """(F^n(states), DF^n) on the GPU (pertbp_map_stm of the C ABI): out (n, 4)
    (None unless want_out) and stm (n, 4, 4) with stm[p, i, j] = d out_i / d in_j."""
    torch = _torch()
    x = torch.as_tensor(states, dtype=torch.float64).to("cuda").contiguous().reshape(-1, 4)
    out = torch.empty_like(x) if want_out else None
    stm = torch.empty((x.shape[0], 4, 4), dtype=torch.float64, device="cuda")
    p = MapParams(float(mu), float(eps), int(steps_per_period), int(n_periods))
    _check(lib().pertbp_map_stm(C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()) if out is not None else None,
                                C.c_void_p(stm.data_ptr()), x.shape[0], C.byref(p), int(cols_per_thread),
                                _stream()))
    return out, stm


def theta_shift(rows, rho, order: int = 0, out=None):
    """d^order/dtheta^order of a(theta_i + rho) for rows (..., n_theta, 4)
    (a cuda float64 tensor or array; rho a number or one value per row):
    theta_shift of the C ABI."""
    torch = _torch()
    x = torch.as_tensor(rows, dtype=torch.float64).to("cuda").contiguous()
    assert x.shape[-1] == 4 and x.dim() >= 2
    n_theta = x.shape[-2]
    n_rows = x.numel() // (4 * n_theta) if x.numel() else int(np.prod(x.shape[:-2]))
    if out is None:
        out = torch.empty_like(x)
    if np.ndim(rho) == 0 and not torch.is_tensor(rho):
        rd, rv = None, float(rho)
    else:
        rd = torch.as_tensor(rho, dtype=torch.float64).to("cuda").contiguous().reshape(-1)
        if rd.numel() != n_rows:
            raise ValueError("rho: one value per row")
        rv = 0.0
    _check(lib().theta_shift(_ptr(x), _ptr(out), int(n_theta), int(n_rows), _ptr(rd), rv, int(order), _stream()))
    return out


def theta_interp(rows, row_index, theta):
    """Trigonometric interpolation: values (n_query, 4) at theta[q] of row
    row_index[q] of rows (n_rows, n_theta, 4): theta_interp of the C ABI."""
    torch = _torch()
    x = torch.as_tensor(rows, dtype=torch.float64).to("cuda").contiguous()
    assert x.shape[-1] == 4 and x.dim() == 3
    r = torch.as_tensor(row_index, dtype=torch.int64).to("cuda").contiguous().reshape(-1)
    t = torch.as_tensor(theta, dtype=torch.float64).to("cuda").contiguous().reshape(-1)
    if r.numel() != t.numel():
        raise ValueError("one row index per theta")
    out = torch.empty((t.numel(), 4), dtype=torch.float64, device="cuda")
    _check(lib().theta_interp(_ptr(x), int(x.shape[1]), int(x.shape[0]), _ptr(r), _ptr(t), t.numel(), _ptr(out),
                              _stream()))
    return out


def theta_spectrum(rows, out=None):
    """Spectra of rows (..., n_theta, 4): (Z0, Z1) / n_theta per frequency as
    4 doubles (theta_spectrum of the C ABI)."""
    torch = _torch()
    x = torch.as_tensor(rows, dtype=torch.float64).to("cuda").contiguous()
    assert x.shape[-1] == 4 and x.dim() >= 2
    n_theta = x.shape[-2]
    n_rows = int(np.prod(x.shape[:-2])) if x.dim() > 2 else 1
    if out is None:
        out = torch.empty_like(x)
    _check(lib().theta_spectrum(_ptr(x), _ptr(out), int(n_theta), n_rows, _stream()))
    return out


def globalize(grid, s, n_max: int, omega: float, lam: float, direction: int, mu: float, eps: float,
              steps_per_period: int):
    """Globalized manifold mesh of Sec. 6.1 (globalize_manifold of the C ABI)
    from a fundamental-domain grid (n_s, n_theta, 4) at the increasing s
    values s; direction +1 (unstable, F) or -1 (stable, F^-1).  Returns
    (rows (M, n_theta, 4) cuda tensor, s values (M,) numpy array)."""
    torch = _torch()
    g = torch.as_tensor(grid, dtype=torch.float64).to("cuda").contiguous()
    assert g.dim() == 3 and g.shape[-1] == 4
    n_s, n_theta = g.shape[0], g.shape[1]
    sv = np.ascontiguousarray(s, dtype=np.float64)
    if sv.shape != (n_s,):
        raise ValueError("one s value per grid row")
    cap = n_s * (int(n_max) + 1)
    out = torch.empty((cap, n_theta, 4), dtype=torch.float64, device="cuda")
    s_out = np.empty(cap)
    nb = C.c_size_t()
    _check(lib().globalize_workspace_size(n_theta, n_s, int(n_max), C.byref(nb)))
    ws = _dev_bytes(nb.value)
    m = C.c_int64()
    mp = MapParams(float(mu), float(eps), int(steps_per_period), int(direction))
    _check(lib().globalize_manifold(_ptr(g), sv.ctypes.data_as(C.c_void_p), n_theta, n_s, int(n_max), float(omega),
                                    float(lam), C.byref(mp), _ptr(out), cap, s_out.ctypes.data_as(C.c_void_p),
                                    C.byref(m), _ptr(ws), nb.value, _stream()))
    return out[: m.value], s_out[: m.value]


class FourierTaylor:
    """A Fourier-Taylor chart W(theta, s) = sum_k W_k(theta) s^k from its
    sampled coefficients coeffs (order + 1, n_theta, 4); the spectra are
    computed once on the GPU."""

    def __init__(self, coeffs):
        torch = _torch()
        c = torch.as_tensor(coeffs, dtype=torch.float64).to("cuda").contiguous()
        assert c.dim() == 3 and c.shape[-1] == 4
        self.order, self.n_theta = c.shape[0] - 1, c.shape[1]
        self.spec = theta_spectrum(c)

    def partials(self, theta, s, m: int = 0, omega: float = 0.0, lam: float = 1.0, mu: float = 0.0,
                 eps: float = 0.0, steps_per_period: int = 1):
        """(W, dW/dtheta, dW/ds), each (n, 4), at the parameters (theta, s) of
        the chart globalized by m periods (m = 0: the local chart)."""
        torch = _torch()
        t = torch.as_tensor(theta, dtype=torch.float64).to("cuda").contiguous().reshape(-1)
        sv = torch.as_tensor(s, dtype=torch.float64).to("cuda").contiguous().reshape(-1)
        if t.numel() != sv.numel():
            raise ValueError("one s per theta")
        n = t.numel()
        w, dth, ds = (torch.empty((n, 4), dtype=torch.float64, device="cuda") for _ in range(3))
        stm = torch.empty((n, 16), dtype=torch.float64, device="cuda") if m != 0 else None
        mp = MapParams(float(mu), float(eps), int(steps_per_period), int(m))
        _check(lib().ft_partials(_ptr(self.spec), int(self.n_theta), int(self.order), _ptr(t), _ptr(sv), n,
                                 float(omega), float(lam), C.byref(mp), _ptr(w), _ptr(dth), _ptr(ds), _ptr(stm),
                                 _stream()))
        return w, dth, ds


def ft_newton(params, chart_u: "FourierTaylor", glob_u, chart_s: "FourierTaylor", glob_s, mu: float, eps: float,
              steps_per_period: int, max_trials: int = 40, tol: float = 1e-12, alpha0: float = 1.0,
              alpha_min: float = 2.0 ** -30):
    """Damped Newton on two globalized Fourier-Taylor charts (ft_newton of the
    C ABI); glob_u / glob_s are (m, omega, lambda).  Returns (x, f, r, status,
    trials) as cuda tensors."""
    torch = _torch()
    x = torch.as_tensor(params, dtype=torch.float64).reshape(-1, 4).to("cuda").contiguous()
    K = x.shape[0]
    cu = FtChart(chart_u.spec.data_ptr(), chart_u.n_theta, chart_u.order, int(glob_u[0]), 0, float(glob_u[1]),
                 float(glob_u[2]))
    cs = FtChart(chart_s.spec.data_ptr(), chart_s.n_theta, chart_s.order, int(glob_s[0]), 0, float(glob_s[1]),
                 float(glob_s[2]))
    mp = MapParams(float(mu), float(eps), int(steps_per_period), 0)
    nb = C.c_size_t()
    _check(lib().ft_newton_workspace_size(K, C.byref(nb)))
    ws = _dev_bytes(nb.value)
    xo = torch.empty_like(x)
    f = torch.empty((K, 4), dtype=torch.float64, device="cuda")
    r = torch.empty((K,), dtype=torch.float64, device="cuda")
    st = torch.empty((K,), dtype=torch.int32, device="cuda")
    tr = torch.empty((K,), dtype=torch.int32, device="cuda")
    npar = NewtonParams(int(max_trials), float(tol), float(alpha0), float(alpha_min))
    _check(lib().ft_newton(_ptr(x), _ptr(xo), K, C.byref(cu), C.byref(cs), C.byref(mp), C.byref(npar), _ptr(f),
                           _ptr(r), _ptr(st), _ptr(tr), _ptr(ws), nb.value, _stream()))
    return xo, f, r, st, tr


def continuation_predict(x0, omega0, domega, x1=None, omega1=None):
    """Initial guesses for a continuation step (continuation_predict of the C
    ABI): rows x (K, 4), omega (K, 2).  Returns a cuda tensor (K, 4)."""
    torch = _torch()
    dev = lambda a, w: torch.as_tensor(a, dtype=torch.float64).to("cuda").contiguous().reshape(-1, w)
    a0 = dev(x0, 4)
    K = a0.shape[0]
    o0, d = dev(omega0, 2), dev(domega, 2)
    a1 = dev(x1, 4) if x1 is not None else None
    o1 = dev(omega1, 2) if x1 is not None else None
    if any(t.shape[0] != K for t in (o0, d) + ((a1, o1) if a1 is not None else ())):
        raise ValueError("one row per problem in every argument")
    out = torch.empty_like(a0)
    _check(lib().continuation_predict(_ptr(a0), _ptr(o0), _ptr(d), _ptr(a1), _ptr(o1), K, _ptr(out), _stream()))
    return out


# ------------------------------------------------------------- refinement

def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p()


def _patches(P):
    """(12,) or (n, 12) patch rows (base, d1, d2) -> (cuda float64 tensor, stride)."""
    torch = _torch()
    t = torch.as_tensor(P, dtype=torch.float64).reshape(-1, 12).to("cuda").contiguous()
    return t, (0 if t.shape[0] == 1 else 1)


def patch_row(patch) -> np.ndarray:
    """Row (base, d1, d2) of an object with base, d1, d2 attributes."""
    return np.concatenate([np.asarray(patch.base, np.float64), np.asarray(patch.d1, np.float64),
                           np.asarray(patch.d2, np.float64)])


def refine_grad(params, U, S, fwd: MapParams, bwd: MapParams, mode: int, ckpt_every: int = 100):
    """Mismatch f, r and (mode) its gradient / Jacobian for K parameter rows
    (th1, s1, th2, s2): refine_grad of the C ABI.  Returns a dict of cuda
    tensors: f (K,4), r (K,), grad (K,5) in adjoint and tangent modes, J
    (K,4,5) in tangent mode."""
    torch = _torch()
    x = torch.as_tensor(params, dtype=torch.float64).reshape(-1, 4).to("cuda").contiguous()
    K = x.shape[0]
    u, su = _patches(U)
    v, sv = _patches(S)
    if su != sv or (su == 1 and (u.shape[0] != K or v.shape[0] != K)):
        raise ValueError("patches: one shared row each, or one row per hit on both sides")
    ck = int(ckpt_every) if mode == MS_REFINE_ADJOINT else 1
    nb = C.c_size_t()
    _check(lib().refine_workspace_size(K, C.byref(fwd), C.byref(bwd), ck, int(mode), C.byref(nb)))
    ws = _dev_bytes(nb.value)
    out = {"f": torch.empty((K, 4), dtype=torch.float64, device="cuda"),
           "r": torch.empty((K,), dtype=torch.float64, device="cuda")}
    if mode in (MS_REFINE_ADJOINT, MS_REFINE_TANGENT):
        out["grad"] = torch.empty((K, 5), dtype=torch.float64, device="cuda")
    if mode == MS_REFINE_TANGENT:
        out["J"] = torch.empty((K, 4, 5), dtype=torch.float64, device="cuda")
    _check(lib().refine_grad(_ptr(x), K, _ptr(u), _ptr(v), su, C.byref(fwd), C.byref(bwd), ck, int(mode),
                             _ptr(out["f"]), _ptr(out["r"]), _ptr(out.get("grad")), _ptr(out.get("J")),
                             _ptr(ws), nb.value, _stream()))
    return out


def refine_newton(params, U, S, fwd: MapParams, bwd: MapParams, max_trials: int = 40, tol: float = 1e-12,
                  alpha0: float = 1.0, alpha_min: float = 2.0 ** -30):
    """Damped Newton refinement of K parameter rows (refine_newton of the C
    ABI).  Returns (x, f, r, status, trials) as cuda tensors."""
    torch = _torch()
    x = torch.as_tensor(params, dtype=torch.float64).reshape(-1, 4).to("cuda").contiguous()
    K = x.shape[0]
    u, su = _patches(U)
    v, sv = _patches(S)
    if su != sv or (su == 1 and (u.shape[0] != K or v.shape[0] != K)):
        raise ValueError("patches: one shared row each, or one row per hit on both sides")
    nb = C.c_size_t()
    _check(lib().refine_workspace_size(K, C.byref(fwd), C.byref(bwd), 1, MS_REFINE_NEWTON, C.byref(nb)))
    ws = _dev_bytes(nb.value)
    xo = torch.empty_like(x)
    f = torch.empty((K, 4), dtype=torch.float64, device="cuda")
    r = torch.empty((K,), dtype=torch.float64, device="cuda")
    st = torch.empty((K,), dtype=torch.int32, device="cuda")
    tr = torch.empty((K,), dtype=torch.int32, device="cuda")
    npar = NewtonParams(int(max_trials), float(tol), float(alpha0), float(alpha_min))
    _check(lib().refine_newton(_ptr(x), _ptr(xo), K, _ptr(u), _ptr(v), su, C.byref(fwd), C.byref(bwd),
                               C.byref(npar), _ptr(f), _ptr(r), _ptr(st), _ptr(tr), _ptr(ws), nb.value, _stream()))
    return xo, f, r, st, tr


def _mismatch_fn():
    torch = _torch()

    class MismatchFn(torch.autograd.Function):
        """r = |F^{n_u}(x_u(th1, s1)) - F^{n_s}(x_s(th2, s2))|^2 per row of
        params, as a differentiable function of params (K, 4) and the
        eccentricity e (0-dim tensor).  forward: refine_grad residual mode;
        backward: the discrete adjoint (refine_grad adjoint mode)."""

        @staticmethod
        def forward(ctx, params, e, U, S, mu, steps_per_period, n_u, n_s, ckpt_every):
            ev = float(e.detach().cpu())
            fwd = MapParams(float(mu), ev, int(steps_per_period), int(n_u))
            bwd = MapParams(float(mu), ev, int(steps_per_period), int(n_s))
            out = refine_grad(params.detach(), U, S, fwd, bwd, MS_REFINE_RESIDUAL)
            ctx.save_for_backward(params.detach())
            ctx.maps = (fwd, bwd, U, S, int(ckpt_every))
            ctx.e_shape = e.shape
            return out["r"]

        @staticmethod
        def backward(ctx, grad_r):
            (params,) = ctx.saved_tensors
            fwd, bwd, U, S, ck = ctx.maps
            g = refine_grad(params, U, S, fwd, bwd, MS_REFINE_ADJOINT, ck)["grad"]
            gr = grad_r.to(g.dtype)
            g_params = gr[:, None] * g[:, :4]
            g_e = (gr * g[:, 4]).sum().reshape(ctx.e_shape)
            return g_params, g_e, None, None, None, None, None, None, None

    return MismatchFn


_MISMATCH = None


def mismatch_r(params, e, U, S, mu: float, steps_per_period: int, n_u: int, n_s: int, ckpt_every: int = 100):
    """Differentiable r (K,) through MismatchFn (adjoint backward)."""
    global _MISMATCH
    if _MISMATCH is None:
        _MISMATCH = _mismatch_fn()
    return _MISMATCH.apply(params, e, U, S, mu, steps_per_period, n_u, n_s, ckpt_every)
