"""Host-side measurement and tuning logic (no GPU): the counter calibration
arithmetic, the trace summary's choice of the timed launches, the kernel
source hash, and the tuner's coordinate search and cache."""
import json

import pytest

import bench


def write_csv(path, header, rows):
    import csv
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        for r in rows:
            w.writerow(r)


def test_pmc_summary_scales_by_the_copy_kernel(tmp_path):
    """Counters are KiB per dispatch; each is divided by what it reads for
    the 1 GiB copy kernel per byte of it."""
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    fetch, write = tmp_path / "f", tmp_path / "w"
    fetch.mkdir()
    write.mkdir()
    gib_kib = bench.CALIB_BYTES / 1024
    write_csv(fetch / "run_counter_collection.csv", hdr,
              [("synth_copy_kernel(x)", "FETCH_SIZE", 0.5 * gib_kib),
               ("crum::k_diff<true>(y)", "FETCH_SIZE", 100.0),
               ("crum::k_diff<true>(y)", "FETCH_SIZE", 300.0),
               ("other", "FETCH_SIZE", 7.0)])
    write_csv(write / "run_counter_collection.csv", hdr,
              [("synth_copy_kernel(x)", "WRITE_SIZE", 1.0 * gib_kib),
               ("crum::k_diff<true>(y)", "WRITE_SIZE", 2.0),
               ("crum::k_diff<true>(y)", "WRITE_SIZE", 2.0)])
    res = bench.pmc_summary(str(fetch), str(write), "many_allocs")
    assert res["FETCH_SIZE"]["calibration_factor"] == 0.5
    assert res["FETCH_SIZE"]["k_diff_dispatches"] == 2
    # (100 + 300) KiB / 2 launches / 0.5
    assert res["FETCH_SIZE"]["k_diff_bytes_per_launch"] == pytest.approx(400 * 1024)
    assert res["WRITE_SIZE"]["k_diff_bytes_per_launch"] == pytest.approx(2 * 1024)
    assert res["traffic_bytes_per_launch"] == round(400 * 1024 + 2 * 1024)
    assert res["kernel_source_hash"] == bench.kernel_source_hash()


def test_trace_summary_takes_the_last_steps(tmp_path):
    """k_diff launches after the header that closes the last untimed
    snapshot are the timed ones."""
    hdr = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    rows = []
    t = 0
    for snap in range(5):  # 2 untimed + 3 timed snapshots, 2 diffs each
        dur = 1000 if snap < 2 else 3000
        for _ in range(2):
            rows.append(("crum::k_diff<true>", t, t + dur))
            t += 10000
        rows.append(("crum::k_header", t, t + 10))
        t += 10000
    write_csv(tmp_path / "run_kernel_trace.csv", hdr, rows)
    out = bench.trace_summary(str(tmp_path), 3)
    assert "6, average duration 0.0030 ms" in out


def test_trace_summary_reports_timed_drain_copies(tmp_path):
    """Device-to-host copies of at least 4 KiB that start after the last
    untimed snapshot's header are summed into bytes, time and GB/s."""
    hdr = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    rows, copies = [], []
    t = 0
    for snap in range(3):  # 1 untimed + 2 timed
        rows.append(("crum::k_diff<true>", t, t + 1000))
        rows.append(("crum::k_pack<0, 4, 0>", t + 2000, t + 2500))
        copies.append(("MEMORY_COPY_DEVICE_TO_HOST", t + 3000, t + 4000, 1 << 20))
        copies.append(("MEMORY_COPY_DEVICE_TO_HOST", t + 4000, t + 4100, 40))
        copies.append(("MEMORY_COPY_HOST_TO_DEVICE", t + 4100, t + 4200, 1 << 20))
        rows.append(("crum::k_header", t + 5000, t + 5100))
        t += 10000
    write_csv(tmp_path / "run_kernel_trace.csv", hdr, rows)
    write_csv(tmp_path / "run_memory_copy_trace.csv",
              ["Direction", "Start_Timestamp", "End_Timestamp", "Size"], copies)
    out = bench.trace_summary(str(tmp_path), 2)
    assert "k_pack (snapshot pack) launches in the timed snapshots: 2" in out
    assert "2 copies, summed duration 0.002 ms" in out
    assert "2097152 bytes (from the trace): 1048.58 GB/s" in out
    # a trace without sizes: the rate comes from the images' bytes
    write_csv(tmp_path / "run_memory_copy_trace.csv",
              ["Kind", "Direction", "Start_Timestamp", "End_Timestamp"],
              [("MEMORY_COPY", d, a, b) for d, a, b, _ in copies])
    out = bench.trace_summary(str(tmp_path), 2, image_bytes=1 << 20)
    assert "2097152 bytes (2 images of 1048576 bytes)" in out


def test_trace_summary_of_the_grouped_plan(tmp_path):
    """With the plan's group count, the k_diff launches of its warm-up
    launches are skipped and those of its timed launches averaged; later
    launches (the other plans, the plain snapshots) are left out."""
    hdr = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    rows = []
    t = 0
    for launch, dur in enumerate([1000, 4000, 4000, 9000]):  # warm-up, 2 timed, later
        for _ in range(3):  # 3 groups
            rows.append(("void crum::k_diff<true>(...)", t, t + dur))
            t += 10000
    write_csv(tmp_path / "run_kernel_trace.csv", hdr, rows)
    out = bench.trace_summary(str(tmp_path), 2, plan_groups=3, warmup=1)
    assert "timed launches (3 groups each): 6, average duration 0.0040 ms" in out


def test_kernel_hash_ignores_comments(tmp_path, monkeypatch):
    src = tmp_path / "paper_1808_00117_amd" / "csrc"
    src.mkdir(parents=True)
    for f in ("crum_kernels.hip", "crum_dev.h", "gf2.h"):
        (src / f).write_text("int a; // one\n/* two\n lines */\nint b;\n\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h1 = bench.kernel_source_hash()
    (src / "gf2.h").write_text("int a; // changed comment\n\nint b;\n")
    assert bench.kernel_source_hash() == h1
    (src / "gf2.h").write_text("int a;\nint c;\n")
    assert bench.kernel_source_hash() != h1


def test_autotune_search_and_cache(tmp_path, monkeypatch):
    """Coordinate search finds the minimum of a separable objective and the
    cache round-trips per device key and workload."""
    from paper_1808_00117_amd import autotune
    state = {"a": 1, "b": 1}
    monkeypatch.setattr(autotune, "current", lambda ctx: dict(state))
    monkeypatch.setattr(autotune, "apply", lambda ctx, p: state.update(p))
    monkeypatch.setattr(autotune, "device_key", lambda: "test-device|hip0")
    best, trials, stats = autotune.search(
        None, lambda: (state["a"] - 3) ** 2 + (state["b"] - 5) ** 2 + 1.0,
        {"a": [1, 2, 3, 4], "b": [2, 5, 8]}, repeats=3)
    assert best == {"a": 3, "b": 5} and state == best
    assert stats["default_s"] == 21.0 and stats["best_s"] == 1.0 and stats["spread_s"] == 0
    assert trials[0]["params"] == {"a": 1, "b": 1}
    assert min(t["seconds"] for t in trials) == 1.0
    path = str(tmp_path / "cache.json")
    autotune.save("batched", best, trials, path)
    autotune.save("other", {"a": 9}, [], path)
    assert autotune.load("batched", path) == best
    assert autotune.load("missing", path) is None
    assert autotune.load("batched", str(tmp_path / "none.json")) is None
    assert set(json.load(open(path))["test-device|hip0"]) == {"batched", "other"}


def test_autotune_keeps_only_gains_above_the_noise(monkeypatch):
    """The default shapes' runs spread over 0.2 s: a candidate 0.1 s faster
    is noise and is not kept; one 0.5 s faster is."""
    import itertools

    from paper_1808_00117_amd import autotune
    state = {"a": 0}
    monkeypatch.setattr(autotune, "current", lambda ctx: dict(state))
    monkeypatch.setattr(autotune, "apply", lambda ctx, p: state.update(p))
    jitter = itertools.cycle([0.0, 0.1, 0.2])
    base = {0: 10.0, 1: 9.9, 2: 9.5}
    best, trials, stats = autotune.search(None, lambda: base[state["a"]] + next(jitter),
                                          {"a": [1]}, repeats=3)
    assert best == {"a": 0} and abs(stats["spread_s"] - 0.2) < 1e-9
    best, trials, stats = autotune.search(None, lambda: base[state["a"]] + next(jitter),
                                          {"a": [2]}, repeats=3)
    assert best == {"a": 2} and stats["gain"] > 1.0


def test_autotune_class_keys():
    from paper_1808_00117_amd import autotune
    assert autotune.class_key("snapshot", 17179869184, 65536) == "snapshot|p65536|b34"
    assert autotune.class_key("snapshot", (1 << 26) + 5, 4096) == "snapshot|p4096|b26"
    assert autotune.class_key("plan", 70977024000) == "plan|b36"


def test_cpu_baseline_reports_one_and_all_threads():
    """The CPU baseline times the unchanged oracle on one thread and on
    several threads over the same host-regenerated sample."""
    import bench
    from synth import scenarios as sc
    res = bench.cpu_baseline(sc.plain(nbytes=2 << 20), 0.2, threads=2)
    assert res["kind"] == "oracle" and res["cores"] == 2 and res["unit"] == "GB/s"
    assert res["value"] > 0 and res["single_core"]["cores"] == 1
    assert res["single_core"]["value"] > 0
    assert res["host"]["threads_available"] >= 1
