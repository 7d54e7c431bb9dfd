"""Autotuner of the search's work shape.

Three knobs decide how much work a search does, never what it finds: the
cell edge of the uniform grid (kappa times the meshes' mean triangle
diameter, Sec. 6.2.1), the size of the hashed occupancy tables (table_log2)
and the enumeration's work tile (enum_shape).  The tuner times the search
over them and keeps the fastest choice, first over kappa at the default
table and tile, then over table size and tile around the two best kappas.
Choices are cached per size bucket (device, pair count and triangles per
side, each to the nearest power of two) in a JSON file, so that a later
search of the same bucket skips the sweep.

The timing itself is the caller's (`measure`), so this module holds no GPU
code: the package passes a closure that runs the plain or batched search.
"""
from __future__ import annotations

import json
import math
import os

KAPPAS = (0.25, 0.35, 0.5, 0.75, 1.0, 1.5, 2.0, 3.0, 4.0)
BATCH_KAPPAS = (1.0, 1.5, 2.0, 3.0)
SHAPES = (1, 2, 3)          # MS_ENUM_WIDE, MS_ENUM_HALF, MS_ENUM_QUARTER
MAX_TABLE = 27              # the largest table_log2 the library takes (its automatic choice stops at 25)
DEFAULT_SHAPE = 2
CACHE_PATH = os.environ.get("MSEARCH_TUNE_CACHE") or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                                   "tune_cache.json")


def auto_table_log2(n_tris_total: int) -> int:
    """The table size the library picks when table_log2 = 0: bits of the
    triangle count plus 2, within [12, 25]."""
    lg = int(max(n_tris_total, 1)).bit_length() + 2
    return min(max(lg, 12), 25)


def _lg(x: float) -> int:
    return int(round(math.log2(max(x, 1))))


def bucket(pairs, device: str) -> str:
    """Cache key of a search of `pairs` [(A, B), ...] (objects with n_tris)."""
    n_a = sum(a.n_tris for a, _ in pairs)
    n_b = sum(b.n_tris for _, b in pairs)
    return f"{device}|pairs~2^{_lg(len(pairs))}|A~2^{_lg(n_a)}|B~2^{_lg(n_b)}"


def load_cache(path: str | None = None) -> dict:
    path = path or CACHE_PATH
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store(key: str, entry: dict, path: str | None = None) -> None:
    """Adds one choice to the cache file (written whole, through a temporary
    file, so that a reader never sees half of it)."""
    path = path or CACHE_PATH
    data = load_cache(path)
    data[key] = entry
    tmp = path + ".tmp"
    try:
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass          # a read-only install keeps working without its cache


def sweep(measure, kappas, tables, shapes=SHAPES, default_table: int = 0, tie: float = 0.03):
    """The joint sweep.  measure(kappa, table_log2, enum_shape) -> ms.
    Stage 1 times every kappa at (default_table, DEFAULT_SHAPE); stage 2 every
    (table, shape) of `tables` x `shapes` at the two fastest kappas.  Of the
    choices within `tie` of the fastest, the one with the smallest kappa, then
    the default table, then the default tile is kept, so that near-ties
    resolve the same way every time.  Returns (choice, {str(config): ms})."""
    times = {}

    def run(k, t, s):
        key = (k, t, s)
        if key not in times:
            times[key] = float(measure(k, t, s))
        return times[key]

    for k in kappas:
        run(k, default_table, DEFAULT_SHAPE)
    best_k = sorted(kappas, key=lambda k: (times[(k, default_table, DEFAULT_SHAPE)], k))[:2]
    for k in best_k:
        for t in tables:
            for s in shapes:
                run(k, t, s)
    fastest = min(times.values())
    near = [c for c, v in times.items() if v <= fastest * (1.0 + tie)]
    k, t, s = min(near, key=lambda c: (c[0], c[1] != default_table, c[2] != DEFAULT_SHAPE, times[c]))
    choice = {"kappa": k, "table_log2": t, "enum_shape": s, "ms": times[(k, t, s)], "configs": len(times)}
    return choice, {f"kappa={c[0]},table={c[1]},shape={c[2]}": round(v, 5) for c, v in times.items()}


def tune(pairs, measure, device: str, batch: bool, use_cache: bool = True, path: str | None = None):
    """The cached joint choice for `pairs`: (choice, timings); timings are
    empty on a cache hit.  choice["cache"] says which."""
    key = bucket(pairs, device)
    if use_cache:
        hit = load_cache(path).get(key)
        if hit and all(f in hit for f in ("kappa", "table_log2", "enum_shape")):
            return dict(hit, cache="hit", key=key), {}
    auto = auto_table_log2(sum(a.n_tris + b.n_tris for a, b in pairs))
    tables = sorted({max(12, auto - 1), auto, min(MAX_TABLE, auto + 1)})
    choice, times = sweep(measure, BATCH_KAPPAS if batch else KAPPAS, tables, default_table=auto)
    if use_cache:
        store(key, dict(choice), path)
    return dict(choice, cache="miss", key=key), times
