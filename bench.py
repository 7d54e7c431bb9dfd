"""Benchmark of the mesh-intersection search on one MI355X.

One step = one pass of the search hot path over the 512 x 512-quad workload
(two seeded torus-like surfaces of 524,288 triangles each, FP64): both
meshes' vertices refreshed in place (mesh_update), then the full keyed-grid
search from the HBM-resident vertices (cell occupancy, entries in cells that
both meshes occupy, grouping by hashed cell with counts and a scan -- no
sort --, slot enumeration with the same-cell, home-cell and box tests, the
Moller test, the 4x4 narrow phase, hits sorted by (pair, triA, triB)).
Prints one JSON line.

The cell edge is picked by the package's autotuner unless --kappa is given.

Side legs (reported in the same line): the all-pairs forced test rate on the
64 x 64 workload, the 256-pair continuation family searched pair by pair
(plain) and in one captured graph (batched), the RK8 map rate, the
refinement kernels (residual, tangent, discrete adjoint, damped Newton) on
128 planted problems, and a plain 1 GiB device copy (the HBM reference that
also scales the hardware counters); the CPU oracle is timed on a bounded
sample as the baseline.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("tri-pair tests/s + ms per 512² mesh-pair search; batched vs plain meshes/s (FP64)")
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(kernel: str, st: dict, mesh_sizes) -> float | None:
    """Bytes a kernel must move per launch, each byte counted once (no
    re-reads): the per-unit figures times the units of one launch."""
    E, nc, C, H = st["n_entries"], st["n_groups"], st["n_cand"], st["n_hits"]
    ntot = sum(nt for nt, _ in mesh_sizes)
    nvtot = sum(nv for _, nv in mesh_sizes)
    table = {
        "k_mark": 32.0 * nvtot + 8.0 * ntot,          # vertices read once, compact cell ranges written
        "k_keys": 8.0 * ntot + 16.0 * E,              # cell ranges read, entries and their group ranks written
        # entries, ranks and hashed cells read; grouped entries and their boxes written
        "k_scatter": 88.0 * E,
        # grouped entries, their boxes and their groups; the 6 vertices of every candidate; hit records
        "k_enum": 72.0 * E + 24.0 * nc + 192.0 * C + 120.0 * H,
    }
    return table.get(kernel)


# FP64 flops per unit of work, counted from the method as written: every
# add, subtract, multiply, divide and square root is one flop (a multiply-add
# is two), whatever instructions the kernels spend on it.
#   Runge-Kutta step: the stage sums of the 11-stage method (39 non-zero
#   a_ij, 5 non-zero b_i) over 4 state components are 396 flops per step.
#   Pulsating field (Sec. 3.2), per stage: the two offsets 2, y^2 1, the two
#   squared distances 4, per primary r = sqrt(r^2), r^3 and m / r^3 4 (8),
#   Omega_x 4, Omega_y 3, the two Coriolis rows 6: 28.
#   Position-momentum field (Sec. 3.3), per stage: offsets 4, y^2 1, squared
#   distances 4, m / r^3 per primary 8, the four rows 13: 30.
#   Its variational terms with 4 tangent columns, per stage: 1 / r^2 and
#   3 m / r^5 per primary 6, the Hessian entries 13 (a1 + a2 formed once),
#   J Hess v 14 per column (56): 75; the stage sums of the 16 tangent
#   components add 1584 per step.
#   Triangle-pair test (Sec. 6.2.3-6.2.4), forced (no early exit): the
#   Moller same-side test 39 each way (edges 6, normal 9, three signed
#   distances 24), the 4x4 system 20 to form, 46 to eliminate (6 divisions)
#   and 20 to back-substitute (4 divisions), inclusion 2: 166 per pair.
FP64_PEAK_TFLOPS = 78.6
RK_FLOPS = {
    "k_rk8_map": 396 + 11 * 28,                      # per vertex-step: 704
    "k_pm_flow<0>": 396 + 11 * 30,                   # per state-step: 726
    "k_pm_flow<4>": 396 + 11 * 30 + 11 * 75 + 1584,  # per state-step with DF: 3135
}
PAIR_TEST_FLOPS = 166
# Peak issue rate of FP64 vector instructions: a wave64 instruction occupies
# a 16-lane SIMD for 4 cycles; 256 CUs x 4 SIMDs at 2.4 GHz.
FP64_WAVE_INSTS_PER_S = 256 * 4 * 2.4e9 / 4

SEARCH_SOURCES = ("mesh.hip", "small_sort.hip", "search.hip", "predicate.hpp", "ms_internal.hpp")
# The sources each kernel family is built from (counters are valid only for these).
SOURCE_GROUPS = {
    "search": SEARCH_SOURCES,
    "rk8": ("rk8.hip", "rk8_core.hpp", "ms_internal.hpp"),
    "pertbp": ("pertbp.hip", "rk8.hip", "rk8_core.hpp", "ms_internal.hpp"),
}


def source_digest(group: str = "search") -> str:
    """Digest of the sources of a kernel family (the hardware counters in
    profiles/ are valid only for the sources they were taken on)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2109_14814_amd", "csrc")
    for f in SOURCE_GROUPS[group]:
        h.update(os.path.basename(f).encode())
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


FP64_FILE = os.path.join(ROOT, "profiles", "fp64_valu_counters.txt")


def fp64_counters(kernel: str) -> dict | None:
    """Per-dispatch FP64 VALU instruction counts of `kernel` from the
    committed rocprofv3 summary, or None when it is missing or was taken on
    other sources."""
    if not os.path.exists(FP64_FILE):
        return None
    cols = None
    for line in open(FP64_FILE):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "kernel":
            cols = f
            continue
        if cols and f[0] == kernel and len(f) == len(cols):
            row = dict(zip(cols, f))
            if row["digest"] != source_digest(row["group"]):
                return None
            return {k: float(v) for k, v in row.items() if k not in ("kernel", "group", "digest")}
    return None


def fp64_issue(kernel: str, launch_s: float) -> dict:
    """Issue fraction of `kernel`: its FP64 VALU wave-instructions per
    dispatch (counters) over what the chip can issue in the launch's
    duration; None without valid counters."""
    c = fp64_counters(kernel)
    if c is None or launch_s <= 0:
        return {"issue_frac": None, "fp64_insts_per_launch": None}
    return {"issue_frac": round(c["fp64_insts"] / (launch_s * FP64_WAVE_INSTS_PER_S), 4),
            "fp64_insts_per_launch": c["fp64_insts"]}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "search_512x512_traffic.txt")


def file_digest(path: str) -> str:
    import hashlib
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


SPECTRAL_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "theta_shift_4096x2048_traffic.txt")


def spectral_traffic(kernel: str) -> float | None:
    """HBM bytes per launch of a spectral kernel from its committed counter
    summary, or None when it is missing or was taken on other sources."""
    if not os.path.exists(SPECTRAL_TRAFFIC_FILE):
        return None
    digest, rows = None, {}
    for line in open(SPECTRAL_TRAFFIC_FILE):
        f = line.split()
        if len(f) >= 2 and f[0] == "source_digest":
            digest = f[1]
        elif len(f) == 5 and f[0].startswith("k_"):
            try:
                rows[f[0]] = float(f[4])
            except ValueError:
                pass
    src = os.path.join(ROOT, "paper_2109_14814_amd", "csrc", "spectral.hip")
    if digest != file_digest(src):
        return None
    return rows.get(kernel)


def measured_traffic(kernel: str) -> float | None:
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, KiB per dispatch, each scaled by the
    same counter's reading on a plain copy of known size), or None when the
    summary is missing or was taken on other sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    digest, rows = None, {}
    for line in open(TRAFFIC_FILE):
        f = line.split()
        if len(f) >= 2 and f[0] == "source_digest":
            digest = f[1]
        elif len(f) == 7 and f[0].startswith("k_"):
            try:
                rows[f[0]] = float(f[6])
            except ValueError:
                pass
    if digest != source_digest():
        return None
    return rows.get(kernel)


BATCH_COUNTERS_FILE = os.path.join(ROOT, "profiles", "search_batched_counters.txt")


def batch_counters(leg: str, kernel: str) -> dict | None:
    """Executed VALU instructions and HBM bytes per batched dispatch of
    `kernel` in `leg` ("family" or "layers") from the committed counter
    summary, or None when it is missing or was taken on other sources."""
    if not os.path.exists(BATCH_COUNTERS_FILE):
        return None
    digest, rows = None, {}
    for line in open(BATCH_COUNTERS_FILE):
        f = line.split()
        if len(f) >= 2 and f[0] == "source_digest":
            digest = f[1]
        elif len(f) == 8 and f[1].startswith("k_"):
            try:
                rows[(f[0], f[1])] = {"valu": float(f[3]) * float(f[4]), "traffic": float(f[7])}
            except ValueError:
                pass
    if digest != source_digest():
        return None
    return rows.get((leg, kernel))


def batch_roofline(ms, batch, pairs, leg: str) -> dict:
    """Dominant kernel of one batched search (launched without a graph, so
    that every dispatch carries its own start / stop events): its
    algorithmic bytes (the same table as the plain search, summed over the
    batch's meshes and counts) over its dispatch duration, its measured
    traffic, and its VALU issue fraction from the committed counters; the
    bound is the busier of HBM and VALU issue, as for the plain search."""
    import torch
    ms.profile_enable(True)
    batch.run(False)
    torch.cuda.synchronize()
    rows = ms.profile_read()
    ms.profile_enable(False)
    per = {}
    for name, t in rows:
        per[name] = per.get(name, 0.0) + t
    st = batch.stats_dict()
    sizes = [(m.n_tris, len(m.theta) * len(m.s)) for pr in pairs for m in pr]
    cands = [k for k in per if algorithmic_bytes(k, st, sizes) is not None]
    dom = max(cands, key=per.get)
    b = algorithmic_bytes(dom, st, sizes)
    t = per[dom] * 1e-3
    gbs = b / t / 1e9
    cnt = batch_counters(leg, dom)
    traffic = cnt["traffic"] if cnt else None
    hbm = {"achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 5),
           "traffic": traffic, "traffic_frac": round(traffic / t / 1e9 / HBM_PEAK_GBS, 5) if traffic else None}
    out = {"kernel": dom, "launch_ms": round(per[dom], 5), "bytes_per_launch": b,
           "kernels_ms": {k: round(v, 5) for k, v in per.items()}}
    valu_frac = cnt["valu"] * 64 / t / VALU_LANE_OPS_PER_S if cnt else None
    if valu_frac is not None and valu_frac > max(hbm["frac"], hbm["traffic_frac"] or 0.0):
        out.update({"bound": "alu", "achieved": round(valu_frac * VALU_LANE_OPS_PER_S / 1e12, 3),
                    "peak": round(VALU_LANE_OPS_PER_S / 1e12, 2), "unit": "TOP/s", "frac": round(valu_frac, 4),
                    "basis": "executed VALU lane operations (SQ_INSTS_VALU x 64, committed counters) per launch",
                    "traffic": traffic, "hbm": hbm})
    else:
        out.update({"bound": "hbm", **hbm, "valu_issue_frac": round(valu_frac, 4) if valu_frac is not None else None})
    return out


SQ_FILE = os.path.join(ROOT, "profiles", "search_512x512_sq_counters.txt")
# 32-bit VALU lane operations per second without FMA or packed forms: 16 lanes
# per SIMD per cycle, 4 SIMDs per CU, 256 CUs at 2.4 GHz.
VALU_LANE_OPS_PER_S = 256 * 4 * 16 * 2.4e9


def sq_valu_per_dispatch(kernel: str) -> float | None:
    """SQ_INSTS_VALU per dispatch of a search kernel from the committed
    counter summary, or None when it is missing or was taken on other
    sources."""
    import re
    if not os.path.exists(SQ_FILE):
        return None
    digest, rows = None, {}
    for line in open(SQ_FILE):
        f = line.split()
        if "source_digest" in f:
            digest = f[f.index("source_digest") + 1]
        elif len(f) >= 4 and f[0].startswith("k_"):
            try:
                rows[re.sub(r"<.*>", "", f[0])] = float(f[2]) * float(f[3])
            except ValueError:
                pass
    if digest != source_digest():
        return None
    return rows.get(kernel)


def search_roofline(kernel: str, launch_ms: float, alg_bytes: float) -> dict:
    """Roofline of the dominant search kernel against the unit its counters
    show busiest: HBM (algorithmic bytes, and the measured traffic) or the
    VALU issue rate (executed VALU instructions from the SQ counters: the
    cell hashing and bit tests have no algorithmic flop count)."""
    t = launch_ms * 1e-3
    gbs = alg_bytes / t / 1e9
    traffic = measured_traffic(kernel)
    hbm = {"achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 5),
           "traffic": traffic, "traffic_frac": round(traffic / t / 1e9 / HBM_PEAK_GBS, 5) if traffic else None}
    valu = sq_valu_per_dispatch(kernel)
    out = {"kernel": kernel, "avg_launch_ms": round(launch_ms, 6), "bytes_per_launch": alg_bytes,
           "source_digest": source_digest()}
    if valu is not None and valu * 64 / t / VALU_LANE_OPS_PER_S > max(hbm["frac"], hbm["traffic_frac"] or 0.0):
        tops = valu * 64 / t / 1e12
        out.update({"bound": "alu", "achieved": round(tops, 3), "peak": round(VALU_LANE_OPS_PER_S / 1e12, 2),
                    "unit": "TOP/s", "frac": round(tops * 1e12 / VALU_LANE_OPS_PER_S, 4),
                    "basis": "executed VALU lane operations (SQ_INSTS_VALU x 64, committed counters) per launch",
                    "traffic": traffic, "hbm": hbm})
    else:
        out.update({"bound": "hbm", **hbm})
    return out


def per_pair_params(p):
    """The batch's tuned parameters for one pair searched on its own: the
    same grid and tile, the hashed tables sized for the pair (table_log2 =
    0), not for the whole batch (hundreds of batch-sized workspaces would
    not fit in memory)."""
    q = type(p).from_buffer_copy(p)
    q.table_log2 = 0
    return q


def time_search(ms, A, B, searcher, steps, warmup, profile=False):
    """ms per step (mesh_update x 2 + one queued search); with profile, also
    the per-dispatch kernel durations of every step."""
    import torch
    for _ in range(warmup):
        A.update(); B.update(); searcher.run_async()
    torch.cuda.synchronize()
    searcher.check_overflow()
    kern = {}
    if profile:
        ms.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        A.update(); B.update(); searcher.run_async()
        if profile:
            for name, t in ms.profile_read():
                kern.setdefault(name, []).append(t)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if profile:
        ms.profile_enable(False)
    searcher.check_overflow()
    return (t1 - t0) / steps * 1e3, kern


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=512, help="quads per axis of each surface")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--kappa", type=float, default=0.0, help="cell edge / mean triangle diameter (0 = autotune)")
    ap.add_argument("--legs", default="search,allpairs,family,layers,rk8,pertbp,spectral,globalize,ft,refine,copy,cpu")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    legs = set(args.legs.split(","))

    import numpy as np
    import torch

    import paper_2109_14814_amd as ms
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    ms.lib()

    # ------------------------------------------------ main leg: 512^2 search
    Am, Bm = synth.plain_pair(args.n, args.n, args.seed)
    A, B = ms.Mesh.from_synth(Am), ms.Mesh.from_synth(Bm)
    mesh_sizes = [(A.n_tris, Am.verts.shape[0] * Am.verts.shape[1]), (B.n_tris, Bm.verts.shape[0] * Bm.verts.shape[1])]
    logical_pairs = A.n_tris * B.n_tris
    if args.kappa > 0:
        kappa, params, sweep, tuned = args.kappa, ms.default_params(A, B, args.kappa), {}, None
    else:
        tuned, params, sweep = ms.autotune_kappa(A, B, hits_cap=1 << 10)
        kappa = tuned["kappa"]
        log(f"tuned ({tuned['cache']}): kappa {kappa}, table_log2 {tuned['table_log2']}, enum_shape "
            f"{tuned['enum_shape']}" + "".join(f"; {k}: {v:.4f} ms" for k, v in sweep.items()))
    searcher = ms.Searcher(A, B, params, hits_cap=1 << 10, cand_cap=1 << 20)   # run() grows it if needed
    searcher.run()
    ms_step_prof, kern = time_search(ms, A, B, searcher, args.steps, args.warmup, profile=True)
    hits, st, _ = searcher.results()
    log(f"search: {ms_step_prof:.4f} ms/step with per-kernel events, kappa={kappa}, stats={st}")
    ms_step, _ = time_search(ms, A, B, searcher, args.steps, args.warmup, profile=False)
    log(f"search: {ms_step:.4f} ms/step (timed region, no events)")
    value = logical_pairs / (ms_step * 1e-3)

    kern_avg = {k: sum(v) / len(v) for k, v in kern.items()}
    kern_launches = {k: len(v) / args.steps for k, v in kern.items()}
    kern_total = {k: sum(v) / args.steps for k, v in kern.items()}
    dominant = max((k for k in kern_total if algorithmic_bytes(k, st, mesh_sizes) is not None),
                   key=lambda k: kern_total[k])
    roofline = search_roofline(dominant, kern_avg[dominant], algorithmic_bytes(dominant, st, mesh_sizes))

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "tri-pairs/s (logical |A||B| per second, 512^2 search)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"plain search, two seeded torus surfaces of {args.n}x{args.n} quads "
                               f"({A.n_tris} triangles each), FP64, seed {args.seed}",
                   "kappa": kappa, "table_log2": params.table_log2, "enum_shape": params.enum_shape,
                   "world_cells": list(params.n_cells)},
        "ms_per_step_with_kernel_events": ms_step_prof,
        "search_tris_per_s": (A.n_tris + B.n_tris) / (ms_step * 1e-3),
        "tuned": tuned,
        "tune_sweep_ms": sweep,
        "search_stats": st,
        "kernels_ms_avg": {k: round(v, 6) for k, v in kern_avg.items()},
        "kernels_ms_per_step": {k: round(v, 6) for k, v in kern_total.items()},
        "kernels_launches_per_step": kern_launches,
        "roofline": roofline,
    }
    # rooflines of the other legs' main kernels (filled in by the legs below)
    leg_roof = {}
    out["leg_rooflines"] = leg_roof

    # ------------------------------------------- all-pairs forced test rate
    if "allpairs" in legs:
        a0, b0 = synth.plain_pair(64, 64, args.seed)
        A0, B0 = ms.Mesh.from_synth(a0), ms.Mesh.from_synth(b0)
        ms.narrow_allpairs(A0, B0)
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            h0, st0 = ms.narrow_allpairs(A0, B0)
        torch.cuda.synchronize()
        t_ap = (time.perf_counter() - t0) / reps
        pairs0 = A0.n_tris * B0.n_tris
        out["allpairs_tests_per_s"] = pairs0 / t_ap
        out["allpairs_ms"] = t_ap * 1e3
        tf = pairs0 * PAIR_TEST_FLOPS / t_ap / 1e12
        leg_roof["k_allpairs"] = {"bound": "alu", "achieved": round(tf, 2), "peak": FP64_PEAK_TFLOPS,
                                  "unit": "TFLOP/s", "frac": round(tf / FP64_PEAK_TFLOPS, 4),
                                  "flops_per_pair": PAIR_TEST_FLOPS, **fp64_issue("k_allpairs", t_ap)}
        log(f"allpairs: {t_ap * 1e3:.3f} ms for {pairs0} pairs -> {pairs0 / t_ap:.3e} tests/s")

    # ------------------------------------- family: plain per-pair searches
    if "family" in legs:
        fam = synth.family(256, args.seed)
        gp = [(ms.Mesh.from_synth(a), ms.Mesh.from_synth(b)) for a, b in fam]
        ftuned, fparams, fsweep = ms.autotune_batch_kappa(gp)
        fkappa = ftuned["kappa"]
        log(f"family: tuned ({ftuned['cache']}) {ftuned}" + "".join(f"; {k}: {v:.3f} ms" for k, v in fsweep.items()))
        srch = [ms.Searcher(ga, gb, per_pair_params(p), hits_cap=1 << 12, cand_cap=1 << 18)
                for (ga, gb), p in zip(gp, fparams)]
        for s in srch:
            s.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in srch:
            s.run()
        torch.cuda.synchronize()
        t_f = time.perf_counter() - t0
        plain_stats = [s.results()[1] for s in srch]
        bt = ms.Batch(gp, fparams, hits_cap=1 << 16, cand_cap=1 << 22)
        bt.run_checked(True)
        torch.cuda.synchronize()
        reps = 10
        t0 = time.perf_counter()
        for _ in range(reps):
            bt.run(True)
        torch.cuda.synchronize()
        t_b = (time.perf_counter() - t0) / reps
        bst = bt.stats_dict()
        same = bst["overflow"] == 0 and all(bst[k] == sum(p[k] for p in plain_stats)
                                            for k in ("n_cand", "n_hits", "n_cells", "n_slots"))
        out["family_kappa"] = fkappa
        out["family_tuned"] = ftuned
        out["family_plain_meshes_per_s"] = len(srch) / t_f
        out["family_plain_ms_total"] = t_f * 1e3
        out["family_batched_meshes_per_s"] = len(srch) / t_b
        out["family_batched_ms_total"] = t_b * 1e3
        out["family_batched_over_plain"] = t_f / t_b
        out["family_batched_counts_equal_plain"] = bool(same)
        out["family_tris_total"] = int(sum(ga.n_tris + gb.n_tris for ga, gb in gp))
        out["family_batched_tris_per_s"] = out["family_tris_total"] / t_b
        leg_roof["family_batched"] = batch_roofline(ms, bt, gp, "family")
        log(f"family: 256 plain searches in {t_f * 1e3:.2f} ms, batched graph {t_b * 1e3:.2f} ms, counts equal={same}")
        del bt, srch, gp

    # ---------------- the layer search of Sec. 5 / 6.4 at the paper's shape
    if "layers" in legs:
        lp = synth.layered_pair(1024, 2048, 34, 14, args.seed)
        U, S = ms.Mesh.from_synth(lp.U), ms.Mesh.from_synth(lp.S)
        ls = ms.LayerSearch(U, S, lp.D_u, lp.lam_u, lp.D_s, lp.lam_s, lp.n_layers, hits_cap=1 << 16)
        log(f"layers: tuned {ls.tuned}" + "".join(f"; {k}: {v:.3f} ms" for k, v in ls.kappa_times.items()))
        ls.run(True)
        torch.cuda.synchronize()
        reps = 10
        t0 = time.perf_counter()
        for _ in range(reps):
            ls.batch.run(True)
        torch.cuda.synchronize()
        t_l = (time.perf_counter() - t0) / reps
        lst = ls.batch.stats_dict()
        srch = [ms.Searcher(a, b, per_pair_params(p), hits_cap=1 << 12, cand_cap=1 << 18)
                for (a, b), p in zip(ls.meshes, ls.params)]
        for sr in srch:
            sr.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for sr in srch:
            sr.run()
        torch.cuda.synchronize()
        t_p = time.perf_counter() - t0
        pst = [sr.results()[1] for sr in srch]
        same = lst["overflow"] == 0 and all(lst[k] == sum(q[k] for q in pst) for k in ("n_cand", "n_hits", "n_cells", "n_slots"))
        quads = int(sum((a.n_tris // 2) * (b.n_tris // 2) for a, b in ls.meshes))
        out["layers_pairs"] = len(ls.meshes)
        out["layers_kappa"] = ls.kappa
        out["layers_tuned"] = ls.tuned
        out["layers_batched_ms"] = t_l * 1e3
        out["layers_plain_ms"] = t_p * 1e3
        out["layers_quad_pairs"] = quads
        out["layers_quad_pairs_per_s"] = quads / t_l
        out["layers_hits"] = int(lst["n_hits"])
        out["layers_counts_equal_plain"] = bool(same)
        # the same search without world-bound pruning, same tuned tuple
        lsu = ms.LayerSearch(U, S, lp.D_u, lp.lam_u, lp.D_s, lp.lam_s, lp.n_layers, kappa=ls.kappa, hits_cap=1 << 16,
                             prune=False)
        for pu, pt in zip(lsu.params, ls.params):
            pu.table_log2, pu.enum_shape = pt.table_log2, pt.enum_shape
        lsu.batch = ms.Batch(lsu.meshes, lsu.params, hits_cap=1 << 16, cand_cap=1 << 22)
        lsu.run(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            lsu.batch.run(True)
        torch.cuda.synchronize()
        t_u = (time.perf_counter() - t0) / reps
        ust = lsu.batch.stats_dict()
        out["layers_batched_ms_unpruned"] = t_u * 1e3
        out["layers_pruned_counts_equal_unpruned"] = bool(ust["n_hits"] == lst["n_hits"] and ust["n_cand"] == lst["n_cand"])
        log(f"layers: without world-bound pruning {t_u * 1e3:.2f} ms (hits {ust['n_hits']}, candidates equal "
            f"{ust['n_cand'] == lst['n_cand']})")
        del lsu
        leg_roof["layers_batched"] = batch_roofline(ms, ls.batch, ls.meshes, "layers")
        log(f"layers: {len(ls.meshes)} half-layer pairs ({quads:.3e} quad pairs) batched in {t_l * 1e3:.2f} ms, "
            f"pair by pair {t_p * 1e3:.2f} ms, {lst['n_hits']} hits, counts equal={same}")
        del ls, srch, U, S

    # ---------------- propagated patches: F^+-3, boxes, search, refinement
    if "rk8" in legs:
        MU, ECC, STEPS = 2.528e-5, 0.0094, 4000
        gmap = lambda x, n: ms.propagate(torch.tensor(np.ascontiguousarray(x)).cuda(), MU, ECC, STEPS, n)
        pr = synth.planted_refinement(1, args.seed, lambda x, n: gmap(x, n).cpu().numpy())
        mu_mesh = synth.patch_vertices(pr.patch_u, 2049, 257)
        ms_mesh = synth.patch_vertices(pr.patches_s[0], 2049, 257)
        gu, gs = ms.Mesh.from_synth(mu_mesh), ms.Mesh.from_synth(ms_mesh)
        base_u, base_s = gu.verts.clone(), gs.verts.clone()
        ms.propagate(base_u.view(-1, 4)[:1024], MU, ECC, STEPS, 1)    # stage table, warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ms.propagate(base_u.view(-1, 4), MU, ECC, STEPS, 3, out=gu.verts.view(-1, 4))
        ms.propagate(base_s.view(-1, 4), MU, ECC, STEPS, -3, out=gs.verts.view(-1, 4))
        torch.cuda.synchronize()
        t_rk = time.perf_counter() - t0
        t0 = time.perf_counter()
        gu.update(); gs.update()
        # the propagated patches are a regime of their own (millions of
        # box-overlapping pairs): their own tuned tuple
        ptuned, pp, _ = ms.autotune_kappa(gu, gs, hits_cap=1 << 14, cand_cap=1 << 22)
        t0 = time.perf_counter()
        sp = ms.Searcher(gu, gs, pp, hits_cap=1 << 14, cand_cap=1 << 22)
        sp.run()
        hp, stp, _ = sp.results()
        t_s = time.perf_counter() - t0
        sp.run()
        torch.cuda.synchronize()
        t_q = ms._time_ms(sp.run_async, 5)
        out["propagated_search_ms"] = t_q
        out["propagated_search_tuned"] = ptuned
        out["propagated_search_stats"] = stp
        x0 = np.stack([hp["thA"], hp["sA"], hp["thB"], hp["sB"]], axis=1)
        t0 = time.perf_counter()
        xr, _, rr, sr, tr = ms.refine_newton(x0, ms.patch_row(pr.patch_u), ms.patch_row(pr.patches_s[0]),
                                             ms.MapParams(MU, ECC, STEPS, 3), ms.MapParams(MU, ECC, STEPS, -3),
                                             max_trials=30)
        sr = sr.cpu().numpy()
        t_r = time.perf_counter() - t0
        vsteps = 2 * base_u.numel() // 4 * STEPS * 3
        out["rk8_vertex_steps_per_s"] = vsteps / t_rk
        tf = vsteps * RK_FLOPS["k_rk8_map"] / t_rk / 1e12
        leg_roof["k_rk8_map"] = {"bound": "alu", "achieved": round(tf, 2), "peak": FP64_PEAK_TFLOPS,
                                 "unit": "TFLOP/s", "frac": round(tf / FP64_PEAK_TFLOPS, 4),
                                 "flops_per_vertex_step": RK_FLOPS["k_rk8_map"], **fp64_issue("k_rk8_map", t_rk / 2)}
        out["rk8_ms_F3_and_Fm3_two_patches"] = t_rk * 1e3
        out["propagated_search_ms_incl_setup"] = t_s * 1e3
        out["propagated_hits"] = int(len(hp))
        out["propagated_refine_ms"] = t_r * 1e3
        out["propagated_refined_converged"] = int(np.sum(sr == 0))
        out["propagated_root_error"] = float(np.max(np.abs(xr.cpu().numpy() - pr.roots[0]))) if len(hp) else None
        log(f"propagated: F^3 + F^-3 of 2 x {base_u.numel() // 4} vertices in {t_rk * 1e3:.1f} ms, search "
            f"{t_q:.2f} ms ({t_s * 1e3:.2f} ms with set-up; {len(hp)} hits, {stp['n_cand']} candidates, tuned "
            f"kappa {ptuned['kappa']}, tile {ptuned['enum_shape']}), refine {t_r * 1e3:.1f} ms "
            f"({int(np.sum(sr == 0))} converged)")
        del gu, gs, base_u, base_s, sp

    # ------------- the position-momentum model of Sec. 3.3: F^+-3 and DF^3
    if "pertbp" in legs:
        MU, ECC, STEPS = 2.527e-5, 0.0094, 4000
        (mu_mesh, _), (ms_mesh, _) = synth.propagated_patches(2048, 256, args.seed)
        zu = torch.tensor(synth.periapse_position_momentum(mu_mesh.verts.reshape(-1, 4), ECC)).cuda()
        zs = torch.tensor(synth.periapse_position_momentum(ms_mesh.verts.reshape(-1, 4), ECC)).cuda()
        ou, os_ = torch.empty_like(zu), torch.empty_like(zs)
        ms.pertbp_map(zu[:1024], MU, ECC, STEPS, 1)          # stage table, warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ms.pertbp_map(zu, MU, ECC, STEPS, 3, out=ou)
        ms.pertbp_map(zs, MU, ECC, STEPS, -3, out=os_)
        torch.cuda.synchronize()
        t_pm = time.perf_counter() - t0
        vsteps = (zu.shape[0] + zs.shape[0]) * STEPS * 3
        out["pertbp_vertex_steps_per_s"] = vsteps / t_pm
        tf = vsteps * RK_FLOPS["k_pm_flow<0>"] / t_pm / 1e12
        leg_roof["k_pm_flow<0>"] = {"bound": "alu", "achieved": round(tf, 2), "peak": FP64_PEAK_TFLOPS,
                                    "unit": "TFLOP/s", "frac": round(tf / FP64_PEAK_TFLOPS, 4),
                                    "flops_per_state_step": RK_FLOPS["k_pm_flow<0>"],
                                    **fp64_issue("k_pm_flow<0>", t_pm / 2)}
        out["pertbp_ms_F3_and_Fm3_two_patches"] = t_pm * 1e3
        n_stm = 1 << 18
        zst = zu[:n_stm].contiguous()
        stm_t = {}
        for cols in (1, 2, 4):
            ms.pertbp_map_stm(zst[:256], MU, ECC, STEPS, 1, cols_per_thread=cols)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ms.pertbp_map_stm(zst, MU, ECC, STEPS, 3, cols_per_thread=cols)
            torch.cuda.synchronize()
            stm_t[cols] = time.perf_counter() - t0
        best = min(stm_t, key=stm_t.get)
        out["pertbp_stm_vertex_steps_per_s"] = n_stm * STEPS * 3 / stm_t[best]
        tf = n_stm * STEPS * 3 * RK_FLOPS["k_pm_flow<4>"] / stm_t[4] / 1e12
        leg_roof["k_pm_flow<4>"] = {"bound": "alu", "achieved": round(tf, 2), "peak": FP64_PEAK_TFLOPS,
                                    "unit": "TFLOP/s", "frac": round(tf / FP64_PEAK_TFLOPS, 4),
                                    "flops_per_state_step": RK_FLOPS["k_pm_flow<4>"],
                                    **fp64_issue("k_pm_flow<4>", stm_t[4])}
        out["pertbp_stm_ms_by_cols_per_thread"] = {str(k): v * 1e3 for k, v in stm_t.items()}
        log(f"pertbp: F^3 + F^-3 of 2 x {zu.shape[0]} states in {t_pm * 1e3:.1f} ms "
            f"({vsteps / t_pm:.3e} vertex-steps/s); DF^3 of {n_stm} states in "
            + ", ".join(f"{v * 1e3:.1f} ms ({k} cols/thread)" for k, v in stm_t.items()))
        del zu, zs, ou, os_, zst

    # ------------- spectral theta operations (Sec. 6.1 translation, Sec. 7)
    if "spectral" in legs:
        N_TH, M_ROWS = 2048, 4096
        rng = np.random.default_rng(args.seed)
        rows = torch.randn((M_ROWS, N_TH, 4), dtype=torch.float64, device="cuda",
                           generator=torch.Generator(device="cuda").manual_seed(args.seed))
        rho = torch.tensor(rng.uniform(-np.pi, np.pi, M_ROWS), device="cuda")
        dst = torch.empty_like(rows)
        sp_t = {}
        for order in (0, 1):
            ms.theta_shift(rows, rho, order, out=dst)
            torch.cuda.synchronize()
            reps = 10
            t0 = time.perf_counter()
            for _ in range(reps):
                ms.theta_shift(rows, rho, order, out=dst)
            torch.cuda.synchronize()
            sp_t[order] = (time.perf_counter() - t0) / reps
        nbytes = 2 * rows.numel() * 8
        out["spectral_shift_ms"] = sp_t[0] * 1e3
        out["spectral_shift_GBps"] = nbytes / sp_t[0] / 1e9
        gbs = nbytes / sp_t[0] / 1e9
        leg_roof["k_theta_shift<11>"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                                         "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                                         "traffic": spectral_traffic("k_theta_shift<11>"),
                                         "bytes_per_launch": nbytes}
        out["spectral_derivative_ms"] = sp_t[1] * 1e3
        nq = 1 << 16
        qr = torch.tensor(rng.integers(0, M_ROWS, nq), device="cuda")
        qt = torch.tensor(rng.uniform(0, 2 * np.pi, nq), device="cuda")
        ms.theta_interp(rows, qr, qt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ms.theta_interp(rows, qr, qt)
        torch.cuda.synchronize()
        t_i = time.perf_counter() - t0
        out["spectral_interp_queries_per_s"] = nq / t_i
        log(f"spectral: shift of {M_ROWS} rows x {N_TH} samples in {sp_t[0] * 1e3:.3f} ms "
            f"({nbytes / sp_t[0] / 1e9:.0f} GB/s algorithmic), derivative {sp_t[1] * 1e3:.3f} ms; "
            f"{nq} interpolations in {t_i * 1e3:.2f} ms")
        del rows, dst

    # ------------- globalized manifold mesh (Sec. 6.1): 14 layers of a 2048 x 35 grid
    if "globalize" in legs:
        N_TH, K_S, N_MAX = 2048, 17, 14
        s_grid = np.array([k * 0.02 / K_S for k in range(-K_S, K_S + 1)])
        th = 2 * np.pi * np.arange(N_TH) / N_TH
        base = synth.periapse_position_momentum(np.array(synth.UNSTABLE_BASE), 0.0094)
        rng = np.random.default_rng(args.seed)
        d1, d2 = rng.standard_normal(4), rng.standard_normal(4)
        grid = (base[None, None, :] + 1e-3 * (np.cos(th)[None, :, None] * d1 + np.sin(2 * th)[None, :, None] * d2)
                + s_grid[:, None, None] * d2[None, None, :])
        g_dev = torch.tensor(grid, device="cuda")
        ms.globalize(g_dev, s_grid, 1, 0.61, 1.35, 1, 2.527e-5, 0.0094, 4000)      # tables, warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rows_g, s_g = ms.globalize(g_dev, s_grid, N_MAX, 0.61, 1.35, 1, 2.527e-5, 0.0094, 4000)
        torch.cuda.synchronize()
        t_gl = time.perf_counter() - t0
        out["globalize_ms"] = t_gl * 1e3
        out["globalize_rows"] = int(rows_g.shape[0])
        out["globalize_state_steps_per_s"] = N_MAX * grid.shape[0] * N_TH * 4000 / t_gl
        log(f"globalize: {N_MAX} layers of a {grid.shape[0]} x {N_TH} grid -> {rows_g.shape[0]} rows in "
            f"{t_gl * 1e3:.1f} ms ({out['globalize_state_steps_per_s']:.3e} state-steps/s)")
        del g_dev, rows_g

    # ------------- Fourier-Taylor chart partials, local and through F^3 (Sec. 7)
    if "ft" in legs:
        N_TH, ORDER, NQ = 2048, 25, 4096
        rng = np.random.default_rng(args.seed)
        th = 2 * np.pi * np.arange(N_TH) / N_TH
        base = synth.periapse_position_momentum(np.array(synth.UNSTABLE_BASE), 0.0094)
        coeffs = np.zeros((ORDER + 1, N_TH, 4))
        coeffs[0] = base[None, :]
        for k in range(ORDER + 1):
            for q in range(8):
                amp = (1e-3 if k == 0 else 1e-2 / (k + 1) ** 2) / (1 + q) ** 2
                coeffs[k] += amp * (rng.standard_normal(4)[None, :] * np.cos(q * th)[:, None]
                                    + rng.standard_normal(4)[None, :] * np.sin(q * th)[:, None])
        chart = ms.FourierTaylor(coeffs)
        qt = torch.tensor(rng.uniform(0, 2 * np.pi, NQ), device="cuda")
        qs = torch.tensor(rng.uniform(-0.05, 0.05, NQ), device="cuda")
        chart.partials(qt[:64], qs[:64])
        chart.partials(qt[:64], qs[:64], 3, 0.61, 1.35, 2.527e-5, 0.0094, 4000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        chart.partials(qt, qs)
        torch.cuda.synchronize()
        t_loc = time.perf_counter() - t0
        t0 = time.perf_counter()
        chart.partials(qt, qs, 3, 0.61, 1.35, 2.527e-5, 0.0094, 4000)
        torch.cuda.synchronize()
        t_glob = time.perf_counter() - t0
        out["ft_local_partials_per_s"] = NQ / t_loc
        out["ft_global_partials_ms"] = t_glob * 1e3
        # damped Newton on two charts made to meet at a known point: the stable
        # chart's s^0 coefficient is shifted so that its local point at the
        # root is F^2 of the unstable chart's globalized point (GPU map)
        MU_JE, ECC_JE, ST = 2.527e-5, 0.0094, 4000
        gu, gs = (2, 0.61, 1.35), (-2, 0.47, 1 / 1.35)
        root = np.array([1.3, 0.02, 4.1, -0.015])
        cs = coeffs.copy()
        cs[0] += (synth.periapse_position_momentum(np.array(synth.STABLE_BASE), ECC_JE) - base)[None, :]
        pu = chart.partials([root[0]], [root[1]], *gu, MU_JE, ECC_JE, ST)[0]
        loc_s = ms.FourierTaylor(cs).partials([root[2] - gs[0] * gs[1]], [gs[2] ** (-gs[0]) * root[3]])[0]
        target = ms.pertbp_map(pu, MU_JE, ECC_JE, ST, -gs[0])
        cs[0] += (target - loc_s).cpu().numpy()[0][None, :]
        chart_s = ms.FourierTaylor(cs)
        KN = 256
        x0 = root[None, :] + rng.uniform(-3e-4, 3e-4, (KN, 4))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xn, fn, rn, stn, trn = ms.ft_newton(x0, chart, gu, chart_s, gs, MU_JE, ECC_JE, ST, tol=1e-12)
        torch.cuda.synchronize()
        t_newton = time.perf_counter() - t0
        stn = stn.cpu().numpy()
        out["ft_newton_ms"] = t_newton * 1e3
        out["ft_newton_converged"] = int(np.sum(stn == 0))
        out["ft_newton_max_root_error"] = float(np.max(np.abs(xn.cpu().numpy() - root)))
        out["ft_newton_max_trials_used"] = int(trn.cpu().numpy().max())
        log(f"fourier-taylor: {NQ} local chart partials (N={N_TH}, order {ORDER}) in {t_loc * 1e3:.3f} ms; "
            f"globalized through F^3 / DF^3 in {t_glob * 1e3:.1f} ms; Newton on {KN} starts "
            f"{t_newton * 1e3:.1f} ms ({int(np.sum(stn == 0))} converged, root error "
            f"{out['ft_newton_max_root_error']:.1e})")
        del chart, chart_s

    # ------------------------- plain device copy (HBM reference, counter scale)
    if "copy" in legs:
        nbytes = 1 << 30
        src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        reps = 10
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        t_c = e0.elapsed_time(e1) / reps * 1e-3
        out["copy_bytes"] = 2 * nbytes
        out["copy_GBps"] = 2 * nbytes / t_c / 1e9
        log(f"copy: {nbytes >> 20} MiB in {t_c * 1e3:.3f} ms -> {2 * nbytes / t_c / 1e9:.1f} GB/s (read+write)")
        del src, dst

    # ------------------------------- refinement: tangent, adjoint, Newton
    if "refine" in legs:
        MU, ECC, STEPS, K = 2.528e-5, 0.0094, 4000, 128

        def gpu_map(x, n):
            return ms.propagate(torch.tensor(x, device="cuda"), MU, ECC, STEPS, n).cpu().numpy()

        pr = synth.planted_refinement(K, args.seed, gpu_map)
        U = np.repeat(ms.patch_row(pr.patch_u)[None, :], K, axis=0)
        S = np.stack([ms.patch_row(p) for p in pr.patches_s])
        rng = np.random.default_rng(args.seed + 1)
        x0 = pr.roots + rng.uniform(-1e-4, 1e-4, size=pr.roots.shape)
        fwd, bwd = ms.MapParams(MU, ECC, STEPS, 3), ms.MapParams(MU, ECC, STEPS, -3)
        res = {}
        for name, fn in (("residual", lambda: ms.refine_grad(x0, U, S, fwd, bwd, ms.MS_REFINE_RESIDUAL)),
                         ("tangent", lambda: ms.refine_grad(x0, U, S, fwd, bwd, ms.MS_REFINE_TANGENT)),
                         ("adjoint", lambda: ms.refine_grad(x0, U, S, fwd, bwd, ms.MS_REFINE_ADJOINT, 100)),
                         ("newton", lambda: ms.refine_newton(x0, U, S, fwd, bwd, max_trials=30))):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            res[name] = (time.perf_counter() - t0) * 1e3
            if name == "newton":
                xg, _, rg, sg, tg = (t.cpu().numpy() for t in r)
        out["refine_hits"] = K
        out["refine_ms"] = {k: round(v, 3) for k, v in res.items()}
        out["refine_adjoint_grads_per_s"] = K / (res["adjoint"] * 1e-3)
        out["refine_newton_converged"] = int(np.sum(sg == 0))
        out["refine_newton_max_trials_used"] = int(tg.max())
        out["refine_newton_max_root_error"] = float(np.max(np.abs(xg - pr.roots)))
        log(f"refine: K={K} residual {res['residual']:.1f} ms, tangent {res['tangent']:.1f} ms, adjoint "
            f"{res['adjoint']:.1f} ms, newton {res['newton']:.1f} ms ({int(np.sum(sg == 0))} converged)")

    # ------------------------------------------- CPU oracle baseline (bounded)
    if "cpu" in legs:
        import oracle
        lo, _, inv, n = oracle.default_grid([Am, Bm], kappa)
        reps, t_cpu = 0, 0.0
        t0 = time.perf_counter()
        while t_cpu < 10.0 and reps < 50:
            oracle.grid_search(Am, Bm, lo, inv, n)
            reps += 1
            t_cpu = time.perf_counter() - t0
        per = t_cpu / reps
        out["cpu_baseline"] = {"value": logical_pairs / per, "unit": "tri-pairs/s (logical, 512^2 search)",
                               "cores": oracle.max_threads(), "kind": "oracle",
                               "sample": f"{reps} full 512^2 grid searches (same grid), {per * 1e3:.1f} ms each"}
        log(f"cpu oracle: {per * 1e3:.1f} ms per search on {oracle.max_threads()} threads")
        # the oracle of the other rows on bounded samples of their workloads
        # (each a few seconds), in the units of the GPU legs
        from oracle import fourier_taylor as oft
        from oracle import spectral as osp
        ob = {}
        y0 = synth.random_states(8192, args.seed, synth.UNSTABLE_BASE, 1e-3)
        t0 = time.perf_counter()
        oracle.rk8_map(y0, 2.528e-5, 0.0094, 4000, 1)
        dt = time.perf_counter() - t0
        ob["rk8_map"] = {"value": 8192 * 4000 / dt, "unit": "vertex-steps/s",
                         "sample": f"F^1 of 8192 states, 4000 steps ({dt:.2f} s)"}
        z0 = synth.pm_random_states(512, args.seed, 0.0094, synth.UNSTABLE_BASE, 1e-3)
        t0 = time.perf_counter()
        oracle.pertbp_map(z0, 2.527e-5, 0.0094, 4000, 1)
        dt = time.perf_counter() - t0
        ob["pertbp_map"] = {"value": 512 * 4000 / dt, "unit": "state-steps/s",
                            "sample": f"F^1 of 512 states, 4000 steps ({dt:.2f} s)"}
        t0 = time.perf_counter()
        oracle.pertbp_map(z0[:128], 2.527e-5, 0.0094, 4000, 1, stm=True)
        dt = time.perf_counter() - t0
        ob["pertbp_stm"] = {"value": 128 * 4000 / dt, "unit": "state-steps/s (with DF)",
                            "sample": f"DF^1 of 128 states, 4000 steps ({dt:.2f} s)"}
        rows = np.random.default_rng(args.seed).standard_normal((2048, 2048, 4))
        rho = np.random.default_rng(args.seed + 1).uniform(-np.pi, np.pi, 2048)
        t0 = time.perf_counter()
        osp.shift_derivative(rows, rho, 0)
        dt = time.perf_counter() - t0
        ob["theta_shift"] = {"value": rows.nbytes * 2 / dt / 1e9, "unit": "GB/s (read + write once)",
                             "sample": f"2048 rows x 2048 samples ({dt:.2f} s)"}
        c = np.random.default_rng(args.seed).standard_normal((26, 2048, 4)) * 1e-3
        t0 = time.perf_counter()
        for q in range(1024):
            oft.local(c, 0.1 * q, 0.01)
        dt = time.perf_counter() - t0
        ob["ft_local_partials"] = {"value": 1024 / dt, "unit": "points/s (order 25, N = 2048)",
                                   "sample": f"1024 points ({dt:.2f} s)"}
        out["oracle_baselines"] = ob
        log("cpu oracle, other rows: " + ", ".join(f"{k} {v['value']:.3g} {v['unit']}" for k, v in ob.items()))

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
