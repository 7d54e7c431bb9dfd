"""The committed counter summaries that bench.py reads: they parse, their
derived columns follow from the raw ones, and the method's flop counts of
the Runge-Kutta and pair-test kernels add up as itemised."""
import os

import bench


def _rows(path):
    cols, rows = None, []
    for line in open(path):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "kernel":
            cols = f
        elif cols and f[0].startswith("k_") and len(f) == len(cols):
            rows.append(dict(zip(cols, f)))
    return rows


def test_fp64_counters_are_consistent():
    rows = _rows(bench.FP64_FILE)
    names = {r["kernel"] for r in rows}
    assert {"k_allpairs", "k_enum", "k_rk8_map", "k_pm_flow<0>", "k_pm_flow<4>"} <= names
    for r in rows:
        parts = sum(float(r[c]) for c in ("fma_f64", "mul_f64", "add_f64", "trans_f64"))
        assert abs(parts - float(r["fp64_insts"])) <= 4, r["kernel"]
        frac = float(r["fp64_insts"]) / (float(r["dur_us"]) * 1e-6 * bench.FP64_WAVE_INSTS_PER_S)
        assert abs(frac - float(r["issue_frac_counter_run"])) < 1e-3, r["kernel"]
        assert float(r["fp64_insts"]) <= float(r["valu"])
        assert r["group"] in bench.SOURCE_GROUPS


def test_traffic_rows_follow_the_scale():
    digest = None
    for line in open(bench.TRAFFIC_FILE):
        f = line.split()
        if f and f[0] == "source_digest":
            digest = f[1]
        elif len(f) == 7 and f[0].startswith("k_") and f[1].isdigit():
            want = (float(f[2]) * float(f[4]) + float(f[3]) * float(f[5])) * 1024
            assert abs(want - float(f[6])) <= 1e-4 * want + 2048, f[0]
    assert digest is not None and len(digest) == 16


def test_method_flop_counts():
    assert bench.RK_FLOPS["k_rk8_map"] == 396 + 11 * 28 == 704
    assert bench.RK_FLOPS["k_pm_flow<0>"] == 396 + 11 * 30 == 726
    assert bench.RK_FLOPS["k_pm_flow<4>"] == 3135
    # pair test: Moller 2 x (6 + 9 + 3 x 8), solve 20 + (27 + 14 + 5) + (2 + 4 + 6 + 8), inclusion 2
    assert bench.PAIR_TEST_FLOPS == 2 * (6 + 9 + 3 * 8) + 20 + (27 + 14 + 5) + (2 + 4 + 6 + 8) + 2
    assert abs(bench.FP64_WAVE_INSTS_PER_S * 64 * 2 / 1e12 - bench.FP64_PEAK_TFLOPS) < 0.05


def test_profile_files_exist():
    for f in ("search_512x512_kernel_stats.txt", "search_512x512_sq_counters.txt", "search_512x512_traffic.txt",
              "fp64_valu_counters.txt"):
        assert os.path.exists(os.path.join(bench.ROOT, "profiles", f)), f


def test_batched_counters_parse_and_read_back():
    """The batched searches' summary: its traffic column follows from the
    scaled FETCH_SIZE / WRITE_SIZE columns, every leg has its dominant
    kernels, and bench.batch_counters returns the row while the digest
    matches the sources."""
    path = bench.BATCH_COUNTERS_FILE
    digest, fscale, wscale, rows = None, None, None, []
    for line in open(path):
        f = line.split()
        if f and f[0] == "source_digest":
            digest = f[1]
        elif line.startswith("#   its FETCH_SIZE"):
            nums = [float(x.rstrip("),")) for x in line.replace("(", " ").split() if x.rstrip("),").replace(".", "", 1).isdigit()]
            fscale, wscale = nums[1], nums[3]
        elif len(f) == 8 and f[1].startswith("k_"):
            rows.append(f)
    assert digest is not None and len(digest) == 16 and fscale and wscale
    legs = {(r[0], r[1]) for r in rows}
    for leg in ("family", "layers"):
        assert {(leg, k) for k in ("k_mark", "k_keys", "k_scatter", "k_enum")} <= legs
    for r in rows:
        want = (float(r[5]) * fscale + float(r[6]) * wscale) * 1024
        assert abs(want - float(r[7])) <= 1e-4 * want + 2048, r[:2]
    if digest == bench.source_digest():
        got = bench.batch_counters("family", "k_keys")
        row = next(r for r in rows if r[0] == "family" and r[1] == "k_keys")
        assert got["traffic"] == float(row[7]) and got["valu"] == float(row[3]) * float(row[4])
