#!/usr/bin/env python3
"""Snapshot throughput benchmark (one MI355X).

A step is one incremental snapshot of the whole workload: quiesce, diff of
every page against its HBM shadow, bitmap, prefix sum, pack with CRC-32C,
image header, and the drain of the image to pinned host memory, ending when
the image has landed.  Inputs are resident in HBM before the timed region.

Default workload (the one the headline metric is quoted on): 64 device
allocations with log-uniform sizes (4 KiB-1 GiB draws scaled by one factor
to 16 GiB total), 64 KiB pages, dirty pages in clustered runs (start
probability 0.003 per page, geometric run length with mean 32, about 9 %
dirty), and an fp32 SAXPY loop over 4096x4096 elements co-running on a second
stream.  Shadow update is off so every step does the same work.

Device and pinned buffers, streams, events and the co-runner graph come from
the HIP runtime directly (paper_1808_00117_amd.hip); torch is not imported, so
the process runs on the system ROCm runtime, whose device-to-host copies use
the SDMA engines rather than compute units.

Prints one JSON line (see the fields below).  `--config plain` runs the
64 MiB / 4 KiB / 5 % workload instead.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
LINK_PEAK_GBS = 63.0       # PCIe 5.0 x16 per direction after 128b/130b encoding
METRIC = "snapshot GB/s (diff+CRC+compact+drain)"


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="headline",
                    choices=["headline", "many", "plain", "batched", "served", "managed",
                             "persist", "lazy", "diff_sizes"],
                    help="headline (default): the batched 256-request workload, batched vs "
                         "plain, then the 16 GiB many-allocations snapshot beside its "
                         "co-runner (diff roofline, drain, pack, restore) and the CPU oracle")
    ap.add_argument("--lazy-step", type=int, default=8 << 20,
                    help="lazy: bytes per touch of the sequential sweep")
    ap.add_argument("--persist-dir", default=None,
                    help="persist: directory for the checkpoint files ($TMPDIR/crum_persist)")
    ap.add_argument("--app-ms", type=float, default=500.0,
                    help="persist: application compute time between checkpoints")
    ap.add_argument("--writer-threads", type=int, default=4)
    ap.add_argument("--duration", type=float, default=60.0, help="served: trace seconds")
    ap.add_argument("--slots", type=int, default=6, help="served: concurrent request slots")
    ap.add_argument("--rate", type=float, default=200.0, help="served: arrivals per second")
    ap.add_argument("--policy", type=int, default=0,
                    help="served: 0 adaptive, 1 two-stage, 2 pipelined snapshot admission")
    ap.add_argument("--tune", action="store_true",
                    help="batched: run the autotuner and store the result in the tuning cache")
    ap.add_argument("--requests", type=int, default=256, help="batched: number of requests")
    ap.add_argument("--tune-cache", default=None,
                    help="tuning cache path (default: the package's tuning_cache.json)")
    ap.add_argument("--no-corunner", action="store_true")
    ap.add_argument("--seed-base", type=int, default=1000,
                    help="configuration k draws its scenario with seed SEED_BASE + k (1000: "
                         "the reported inputs; 2000 and 3000: variance runs)")
    ap.add_argument("--param", action="append", default=[], metavar="NAME=VALUE",
                    help="set a context parameter (names as in autotune.PARAMS)")
    ap.add_argument("--diff-prio", type=int, default=None,
                    help="issue priority of the diff kernel's waves (0..3)")
    ap.add_argument("--cold", action="store_true",
                    help="plain workload: rotate over 8 independent (current, shadow) pairs "
                         "(1 GiB working set, larger than the 256 MB last-level cache)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="wall time of each CPU oracle baseline leg, one thread and all "
                         "threads (0 disables them)")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="threads of the all-core oracle leg (0: every usable hardware "
                         "thread, at most 16)")
    ap.add_argument("--quick", action="store_true",
                    help="skip the untimed reference phases (for profiler runs)")
    ap.add_argument("--pmc-calibrate", action="store_true",
                    help="run a 1 GiB plain copy kernel first (counter calibration)")
    ap.add_argument("--trace-summary", metavar="DIR",
                    help="summarise a rocprofv3 --kernel-trace --stats run of this script")
    ap.add_argument("--plan-groups", type=int, default=0,
                    help="with --trace-summary of a --config batched run: the grouped "
                         "plan's group count (its first launches' diffs are summarised)")
    ap.add_argument("--image-bytes", type=int, default=0,
                    help="--trace-summary: bytes of one timed snapshot's image, for the drain "
                         "rate when the copy trace carries no sizes")
    ap.add_argument("--pmc-table", metavar="DIR",
                    help="per-kernel mean counter values of one rocprofv3 --pmc run")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of "
                         "this script and print the JSON that the roofline 'traffic' reads")
    return ap.parse_args()


def kernel_source_hash() -> str:
    """Hash of the device code's sources without comments and blank lines, so
    that counters taken on a kernel stay valid across comment edits only."""
    import re
    h = hashlib.sha256()
    for f in ("crum_kernels.hip", "crum_dev.h", "gf2.h"):
        with open(os.path.join(ROOT, "paper_1808_00117_amd", "csrc", f)) as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        lines = (re.sub(r"//.*", "", ln).rstrip() for ln in text.splitlines())
        h.update("\n".join(ln for ln in lines if ln).encode())
    return h.hexdigest()[:16]


CALIB_BYTES = 1 << 30


def pmc_summary(fetch_dir: str, write_dir: str, workload: str) -> dict:
    """Per-launch HBM traffic of k_diff from two rocprofv3 --pmc runs, each
    counter scaled by what it reads for the 1 GiB plain copy kernel."""
    import csv
    import glob

    def per_kernel(d, counter):
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not files:
            raise FileNotFoundError(f"no counter_collection.csv under {d}")
        out = {}
        for f in files:
            for r in csv.DictReader(open(f)):
                if r.get("Counter_Name") != counter:
                    continue
                name = r["Kernel_Name"]
                out.setdefault(name, []).append(float(r["Counter_Value"]) * 1024.0)  # KiB
        return out

    res = {"workload": workload, "kernel_source_hash": kernel_source_hash()}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        pk = per_kernel(d, counter)
        calib = [v for k, vs in pk.items() if "synth_copy_kernel" in k for v in vs]
        diff = [v for k, vs in pk.items() if "k_diff" in k for v in vs]
        if not calib or not diff:
            raise RuntimeError(f"{counter}: missing calibration or k_diff dispatches")
        factor = statistics.median(calib) / CALIB_BYTES
        res[counter] = {"calibration_factor": round(factor, 4),
                        "k_diff_dispatches": len(diff),
                        "k_diff_bytes_raw_total": sum(diff),
                        "k_diff_bytes_per_launch": sum(diff) / len(diff) / factor}
    res["traffic_bytes_per_launch"] = round(res["FETCH_SIZE"]["k_diff_bytes_per_launch"] +
                                            res["WRITE_SIZE"]["k_diff_bytes_per_launch"])
    # the snapshot pack (k_pack<0, ...>): counter bytes summed over its launches
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        pk = per_kernel(d, counter)
        pack = [v for k, vs in pk.items() if "k_pack<0" in k for v in vs]
        heads = sum(len(vs) for k, vs in pk.items() if "k_header" in k)
        if pack:
            res[counter]["k_pack_dispatches"] = len(pack)
            res[counter]["k_pack_snapshots"] = heads
            res[counter]["k_pack_bytes_total"] = sum(pack) / res[counter]["calibration_factor"]
    return res


def pmc_table(d: str, kernels=("k_pack<0", "k_pack<1", "k_diff", "k_scatter")) -> str:
    """Markdown table of a rocprofv3 --pmc run: per kernel (matched by name
    prefix) the dispatch count and the mean of each counter per dispatch."""
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    acc = {}
    for f in files:
        for r in csv.DictReader(open(f)):
            name = r["Kernel_Name"]
            key = next((k for k in kernels if k in name), None)
            if key is None:
                continue
            per = acc.setdefault(key, {})
            per.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    counters = sorted({c for per in acc.values() for c in per})
    out = ["| kernel | dispatches | " + " | ".join(counters) + " |",
           "|---|---:|" + "---:|" * len(counters)]
    for k in kernels:
        if k not in acc:
            continue
        per = acc[k]
        n = max(len(v) for v in per.values())
        out.append(f"| `{k}` | {n} | " + " | ".join(
            f"{statistics.mean(per[c]):.4g}" if c in per else "" for c in counters) + " |")
    return "\n".join(out)


def trace_summary(d: str, steps: int, image_bytes: int = 0, plan_groups: int = 0,
                  warmup: int = 0) -> str:
    """Markdown summary of a rocprofv3 kernel-trace run of this script: the
    per-kernel stats table, and the k_diff launches of the last `steps`
    snapshots (the timed region), which is what the bench's avg_launch_ms
    covers.  With plan_groups (a `--config batched` run without --tune): the
    first plan_groups * (warmup + steps) k_diff launches of the run are the
    grouped plan's, the last plan_groups * steps of them its timed launches,
    which is what the batched block's diff_roofline covers."""
    import csv
    import glob

    def find(pat):
        f = glob.glob(os.path.join(d, "**", pat), recursive=True)
        return f[0] if f else None

    out = []
    ks = find("*kernel_stats.csv")
    if ks:
        out.append("| kernel | calls | avg us | total ms | % |")
        out.append("|---|---:|---:|---:|---:|")
        for r in csv.DictReader(open(ks)):
            out.append(f"| `{r['Name'][:70]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                       f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f} |")
    ms = find("*memory_copy_stats.csv")
    if ms:
        out.append("")
        out.append("| copy | calls | avg us | total ms |")
        out.append("|---|---:|---:|---:|")
        for r in csv.DictReader(open(ms)):
            out.append(f"| {r['Name']} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                       f"{float(r['TotalDurationNs']) / 1e6:.2f} |")
    kt = find("*kernel_trace.csv")
    t_lo = t_hi = None
    if kt:
        rows = [r for r in csv.DictReader(open(kt))]
        diff = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]))
                      for r in rows if "k_diff" in r["Kernel_Name"])
        heads = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]))
                       for r in rows if "k_header" in r["Kernel_Name"])
        if plan_groups:
            n0, n1 = plan_groups * warmup, plan_groups * (warmup + steps)
            if len(diff) >= n1:
                sel = diff[n0:n1]
                avg = statistics.mean(b - a for a, b in sel) / 1e6
                out.append("")
                out.append(f"k_diff launches of the grouped plan's {steps} timed launches "
                           f"({plan_groups} groups each): {len(sel)}, average duration "
                           f"{avg:.4f} ms, summed {sum(b - a for a, b in sel) / 1e6:.3f} ms")
            return "\n".join(out)
        if diff and len(heads) >= steps:
            t0 = heads[-steps - 1][0] if len(heads) > steps else 0
            sel = [(a, b) for a, b in diff if a > t0]
            avg = statistics.mean(b - a for a, b in sel) / 1e6
            out.append("")
            out.append(f"k_diff launches in the last {steps} snapshots (timed region): "
                       f"{len(sel)}, average duration {avg:.4f} ms")
            # from the first timed diff: the previous snapshot's copies are done
            t_lo, t_hi = sel[0][0] - 1, heads[-1][1]
        packs = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]))
                       for r in rows if "k_pack<0" in r["Kernel_Name"])
        if packs and t_lo is not None:
            sel = [(a, b) for a, b in packs if t_lo < a < t_hi]
            if sel:
                tot = sum(b - a for a, b in sel) / 1e6
                out.append(f"k_pack (snapshot pack) launches in the timed snapshots: {len(sel)}, "
                           f"summed duration {tot:.4f} ms ({tot / steps:.4f} ms per snapshot)")
    mt = find("*memory_copy_trace.csv")
    if mt and t_lo is not None:
        rows = [r for r in csv.DictReader(open(mt))]
        cols = list(rows[0].keys()) if rows else []
        size_col = next((c for c in cols if "size" in c.lower() or "bytes" in c.lower()), None)
        dir_col = next((c for c in cols if c.lower() in ("direction", "kind", "operation")), None)

        def is_d2h(r):
            v = " ".join(str(r.get(c, "")) for c in cols if c in ("Direction", "Kind",
                                                                     "Operation"))
            return "DEVICE_TO_HOST" in v.upper()
        sel = [r for r in rows if is_d2h(r) and
               t_lo < int(r["Start_Timestamp"]) and int(r["End_Timestamp"]) <= t_hi + 10**9]
        if size_col:
            sel = [r for r in sel if int(r[size_col]) >= 4096]
        if sel:
            dur = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in sel) / 1e9
            span = (max(int(r["End_Timestamp"]) for r in sel) -
                    min(int(r["Start_Timestamp"]) for r in sel)) / 1e9
            what = "of at least 4 KiB " if size_col else ""
            line = (f"device-to-host copies {what}from the first timed snapshot's diff on "
                    f"({dir_col}): {len(sel)} copies, summed duration {dur * 1e3:.3f} ms, "
                    f"first start to last end {span * 1e3:.3f} ms")
            nbytes = sum(int(r[size_col]) for r in sel) if size_col else steps * image_bytes
            if nbytes:
                gbs = nbytes / dur / 1e9
                line += (f"; {nbytes} bytes "
                         f"({'from the trace' if size_col else f'{steps} images of {image_bytes} bytes'}): "
                         f"{gbs:.2f} GB/s over the copies' durations = "
                         f"{gbs / LINK_PEAK_GBS:.3f} of the {LINK_PEAK_GBS:.1f} GB/s host link")
            out.append(line)
    return "\n".join(out)


def load_traffic(workload: str, launches_bytes: float):
    """HBM traffic of the diff kernel from committed rocprofv3 counter runs,
    if they were taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"diff_{workload}_pmc.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("traffic_bytes_per_launch")


def cpu_baseline(scn, budget_s: float, threads: int = 0) -> dict:
    """Time the CPU oracle (as it stands: plain single-threaded C) on a
    bounded sample of the same workload: whole regions in table order up to
    1 GiB, regenerated on the host (untimed).  Two legs of about `budget_s`
    seconds each: one thread snapshotting the sample repeatedly, then
    `threads` threads (default: every hardware thread this process may use,
    at most 16) each snapshotting the same sample repeatedly and independently
    (the oracle call releases the GIL; the inputs are only read).  Reported as
    scanned GB/s: sample bytes x snapshots / wall time."""
    import threading

    import oracle
    from synth import scenarios as sc

    regs, total, dirty = [], 0, 0
    for i, r in enumerate(scn.regions):
        if total + r.nbytes > (1 << 30) and regs:
            continue
        cur, sh = sc.materialize_host(scn, i)
        regs.append((cur, sh, r.id))
        total += r.nbytes
        dirty += int(r.dirty_pages.size)
        if total >= (1 << 30) - (64 << 20):
            break
    P = scn.page_size
    G = total // P
    cap = oracle.prefix_bytes(len(regs), G) + dirty * P + ((4 * dirty + 7) // 8) * 8
    oracle.crc32c(b"")  # the oracle's CRC table is built before any thread starts

    def leg(n_threads):
        counts = [0] * n_threads
        stop_at = [0.0]

        def worker(k):
            while True:
                st, img, _ = oracle.snapshot(regs, P, image_cap=cap)
                assert st.code == oracle.OK and st.n_dirty == dirty
                del img
                counts[k] += 1
                if time.perf_counter() >= stop_at[0]:
                    return
        t0 = time.perf_counter()
        stop_at[0] = t0 + budget_s
        ths = [threading.Thread(target=worker, args=(k,)) for k in range(n_threads)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        wall = time.perf_counter() - t0
        return total * sum(counts) / wall / 1e9, sum(counts), wall

    host = host_cpu()
    if threads <= 0:
        threads = max(1, min(16, host["threads_available"] or 1))
    one_gbs, one_n, one_s = leg(1)
    all_gbs, all_n, all_s = leg(threads)
    sample = (f"{len(regs)} whole regions in table order, {total / 2**30:.2f} GiB scanned, "
              f"{dirty} dirty {P // 1024} KiB pages")
    return {"value": round(all_gbs, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "host": host,
            "sample": f"{sample}; {threads} threads each snapshotting the sample independently, "
                      f"{all_n} snapshots in {all_s:.1f} s",
            "single_core": {"value": round(one_gbs, 3), "unit": "GB/s", "cores": 1,
                            "sample": f"{sample}; {one_n} snapshots in {one_s:.1f} s"}}


def settle_copy_engines(H, dev_ptr: int, host_ptr: int, nbytes: int = 256 << 20,
                        limit_s: float = 20.0) -> dict:
    """Wait until device-to-host copies run at a steady rate.  Shortly after
    a process allocates (or another process frees) tens of GB of device
    memory, pinned copies on this system run at about half rate for a few
    seconds (the copy engines are shared with the kernel driver's background work),
    then at full rate for good.  Repeats a `nbytes` copy until three in a row
    are within 3 % of the best rate seen and above 45 GB/s, or `limit_s`."""
    s = H.Stream()
    t0 = time.perf_counter()
    rates = []
    while True:
        a, b = H.Event(), H.Event()
        a.record(s)
        H.check(H.hip().hipMemcpyAsync(host_ptr, dev_ptr, nbytes, H.hipMemcpyDeviceToHost,
                                       s.handle), "hipMemcpyAsync")
        b.record(s)
        rates.append(nbytes / (a.elapsed_ms(b) * 1e-3) / 1e9)
        best = max(rates)
        if len(rates) >= 3 and best > 45.0 and all(r >= 0.97 * best for r in rates[-3:]):
            break
        if time.perf_counter() - t0 > limit_s:
            break
    out = {"seconds": round(time.perf_counter() - t0, 2), "copies": len(rates),
           "first_gbs": round(rates[0], 1), "final_gbs": round(rates[-1], 1)}
    log(f"[bench] copy engines settled: {out}")
    return out


def link_reference(H, staging_ptr: int, host_ptr: int, nbytes: int = 1 << 30) -> dict:
    """A plain pinned device-to-host hipMemcpyAsync of `nbytes` (best of 3),
    and the GPU's PCIe link state as the kernel's sysfs reports it."""
    s = H.Stream()
    best = 0.0
    for _ in range(3):
        a, b = H.Event(), H.Event()
        a.record(s)
        H.check(H.hip().hipMemcpyAsync(host_ptr, staging_ptr, nbytes, H.hipMemcpyDeviceToHost,
                                       s.handle), "hipMemcpyAsync")
        b.record(s)
        best = max(best, nbytes / (a.elapsed_ms(b) * 1e-3) / 1e9)
    link = {}
    import glob
    for dev in sorted(glob.glob("/sys/class/drm/card*/device")):
        try:
            vendor = open(os.path.join(dev, "vendor")).read().strip()
            if vendor != "0x1002":
                continue
            link = {k: open(os.path.join(dev, k)).read().strip()
                    for k in ("current_link_speed", "current_link_width", "max_link_speed",
                              "max_link_width")}
            break
        except OSError:
            continue
    return {"pinned_copy_gbs": round(best, 2), "pinned_copy_bytes": nbytes,
            "pcie_link": link or None}


def materialize_raw(scn, H):
    """Device buffers (current, shadow) per region, filled by the generator
    kernels: current = generator bytes, shadow = copy with the page mutations."""
    import numpy as np
    import synth
    pairs = []
    for r in scn.regions:
        cur = H.DeviceBuffer(r.nbytes)
        synth.fill_dev(cur.ptr, r.nbytes, r.fill_seed, r.fill_region, 0, 0)
        sh = None
        if r.has_shadow:
            sh = H.DeviceBuffer(r.nbytes)
            H.memcpy_dtod(sh.ptr, cur.ptr, r.nbytes)
            if r.dirty_pages.size:
                pages = np.ascontiguousarray(r.dirty_pages, np.int64)
                d_pages = H.DeviceBuffer(pages.nbytes)
                H.memcpy_htod(d_pages.ptr, pages.ctypes.data, pages.nbytes)
                synth.mutate_dev(sh.ptr, r.nbytes, scn.page_size, d_pages.ptr, int(pages.size),
                                 int(pages.max()), r.mut_kind, scn.mut_seed, r.fill_region, 0)
                H.device_synchronize()
                d_pages.free()
        pairs.append((cur, sh))
    H.device_synchronize()
    return pairs


def host_cpu() -> dict:
    """The host the CPU baseline ran on: CPU model and the hardware threads
    this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        threads = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        threads = os.cpu_count()
    out = {"cpu_model": model, "threads_available": threads, "nproc": os.cpu_count()}
    try:
        import subprocess
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        f = dict((k.strip(), v.strip()) for k, v in
                 (ln.split(":", 1) for ln in txt.splitlines() if ":" in ln))
        out["lscpu"] = {k: f.get(k) for k in ("Model name", "Socket(s)", "Core(s) per socket",
                                              "Thread(s) per core", "CPU(s)")}
        out["physical_cores"] = int(f["Socket(s)"]) * int(f["Core(s) per socket"])
    except Exception:
        pass
    return out


def read_ceiling(H, scn, pairs, stream, reps: int = 7) -> dict:
    """Practical HBM read rate of this GPU: the plain two-stream read kernel
    of the generator library over the largest region and its shadow (the
    diff's traffic without its bookkeeping), median of `reps` launches timed
    with HIP events."""
    import synth
    i = max(range(len(scn.regions)), key=lambda k: scn.regions[k].nbytes)
    nb = scn.regions[i].nbytes // 16384 * 16384
    blocks = 2048
    out = H.DeviceBuffer(4 * blocks * 256)
    e0, e1 = H.Event(), H.Event()
    v = []
    for r in range(reps + 2):
        e0.record(stream)
        synth.read2_dev(pairs[i][0].ptr, pairs[i][1].ptr, nb, out.ptr, blocks * 256, blocks,
                        stream.handle)
        e1.record(stream)
        ms = e0.elapsed_ms(e1)
        if r >= 2:
            v.append(ms)
    out.free()
    ms = statistics.median(v)
    gbs = 2 * nb / (ms * 1e-3) / 1e9
    return {"kernel": "synth_read2_kernel: one wave per 16 KiB unit, 4 non-temporal 16-byte "
                      "loads per buffer in flight", "bytes": 2 * nb, "ms": round(ms, 4),
            "achieved": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}


def copy_ceiling(H, src_ptr: int, dst_ptr: int, nbytes: int, stream, reps: int = 7) -> dict:
    """Practical HBM copy rate of this GPU (read + write): the generator
    library's streaming copy kernel (one wave per 16 KiB, 16 non-temporal
    loads per lane in flight, non-temporal stores, 4096 workgroups) over
    `nbytes` (rounded down to 16 KiB), median of `reps` launches timed with
    HIP events.  The pack's traffic has the same read/write mix."""
    import synth
    nb = nbytes // 16384 * 16384
    e0, e1 = H.Event(), H.Event()
    v = []
    for r in range(reps + 2):
        e0.record(stream)
        synth.lib.copy2_dev(dst_ptr, src_ptr, nb, 4096, 16, True, stream.handle)
        e1.record(stream)
        ms = e0.elapsed_ms(e1)
        if r >= 2:
            v.append(ms)
    ms = statistics.median(v)
    gbs = 2 * nb / (ms * 1e-3) / 1e9
    return {"kernel": "synth_copy2_kernel<16, true>: one wave per 16 KiB unit, 16 "
                      "non-temporal 16-byte loads per lane in flight, non-temporal stores",
            "bytes": 2 * nb, "ms": round(ms, 4), "achieved": round(gbs, 1),
            "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}


def percentile(v, q):
    v = sorted(v)
    return v[min(len(v) - 1, int(round(q * (len(v) - 1))))]


def bench_batched(args) -> dict:
    """Batched workload: 256 requests (1-32 allocations each, request totals
    log-uniform 1 MiB-2 GiB, 4 KiB or 64 KiB pages, dirty fraction U(1%, 50%)
    in runs of mean 16) snapshotted by one plan launch (captured graphs, one
    per group of requests), against 256 one-at-a-time plain snapshots of the
    same requests into the same host offsets; images compared byte for byte.
    Three plans are timed: the grouped plan (tuned shapes, caller's order),
    the same plan smallest request first, and a one-graph plan (a single group
    holding all 256 requests: one persistent diff, one drain).  Returns the
    result dict."""
    import numpy as np

    import paper_1808_00117_amd as crum
    import paper_1808_00117_amd.hip as H
    from paper_1808_00117_amd import autotune
    from synth import scenarios as sc

    crum.lib()
    reqs = sc.batched(seed=args.seed_base + 4, n_requests=args.requests)
    N = sum(r.total_bytes for r in reqs)
    Dsum = sum(r.n_dirty for r in reqs)
    log(f"[batched] {len(reqs)} requests, {N / 1e9:.1f} GB scanned, "
        f"{sum(r.n_dirty * r.page_size for r in reqs) / 1e9:.1f} GB dirty")
    t0 = time.perf_counter()
    pairs = [materialize_raw(r, H) for r in reqs]
    log(f"[batched] materialised in {time.perf_counter() - t0:.1f} s")
    tables = []
    for r, pr in zip(reqs, pairs):
        tables.append([(c.ptr, s.ptr if s else 0, g.nbytes, g.id) for (c, s), g in
                       zip(pr, r.regions)])
    sizes = [crum.crum_image_bytes(len(r.regions), r.total_pages, r.n_dirty, r.page_size)
             for r in reqs]
    total = sum((b + 4095) // 4096 * 4096 for b in sizes)
    cap = total + (64 << 20)
    staging = H.DeviceBuffer(cap)
    h_images = H.PinnedBuffer(cap)
    status = H.PinnedBuffer(40 * len(reqs))
    settle = settle_copy_engines(H, staging.ptr, h_images.ptr)
    ctx = crum.crum_ctx_create(0)
    stream = H.Stream()
    plan_reqs = [(t, r.page_size, 0, 5) for t, r in zip(tables, reqs)]

    def make_plan():
        return crum.Plan(ctx, plan_reqs, staging.ptr, cap, h_images.ptr, cap)

    def launch(plan):
        t = time.perf_counter()
        rc = plan.launch(stream.handle, status.ptr)
        assert rc == 0, rc
        stream.synchronize()
        return time.perf_counter() - t

    cache = args.tune_cache or autotune.DEFAULT_CACHE
    tune_key = autotune.class_key("plan", N)
    tuned = autotune.load(tune_key, cache)

    def mean_request_latency(plan):
        """Mean over requests of the time from launch start to the end of the
        drain of the request's group, in seconds."""
        gr = plan.groups()
        gt = plan.group_times()
        return sum((gr[g + 1] - gr[g]) * gt[g] for g in range(len(gt))) / len(reqs) / 1e3

    def digests():
        """Per request: status code and the image's two checksums (meta_crc
        covers header, table and bitmap; crcs_crc covers every page CRC)."""
        img = h_images.numpy(cap)
        out = []
        for code, _, _, _, b, off in crum.read_request_statuses(status.ptr, len(reqs)):
            out.append((code, b, img[off + 56:off + 64].tobytes() if code == 0 else b""))
        return out

    if args.tune:
        # objective: mean request completion time (latency), which also
        # tracks the makespan since the batch is drain-bound; every candidate
        # must give the same images as the first
        ref = []

        def trial():
            plan = make_plan()
            launch(plan)  # warm
            launch(plan)
            t = mean_request_latency(plan)
            plan.destroy()
            dg = digests()
            if not ref:
                ref.append(dg)
            assert dg == ref[0], "a tuning candidate changed the images"
            return t
        space = {"chunk_bytes": [4 << 20, 16 << 20, 64 << 20, 256 << 20],
                 "chunk_max_bytes": [64 << 20, 256 << 20, 1 << 30, 4 << 30],
                 "pack_blocks": [512, 1024, 2048],
                 "diff_blocks": [512, 1024, 2048]}
        best, trials, stats = autotune.search(ctx, trial, space, repeats=3, log=log)
        autotune.save(tune_key, best, trials, cache, stats)
        log(f"[autotune] {tune_key}: {stats}")
        tuned = best
    if tuned:
        autotune.apply(ctx, tuned)
    params = autotune.current(ctx)

    def timed(plan):
        """Warm-up and timed launches of a plan: makespans, per-request
        latencies (launch start to the end of the request's group drain) and
        the last statuses.  The context's timing sums restart after the
        warm-up launches."""
        order, gr = plan.order(), plan.groups()
        group_of = np.zeros(len(reqs), np.int64)
        for g in range(len(gr) - 1):
            for pos in range(gr[g], gr[g + 1]):
                group_of[order[pos]] = g
        for _ in range(args.warmup):
            launch(plan)
        crum.crum_ctx_timing_reset(ctx)
        sts = crum.read_request_statuses(status.ptr, len(reqs))
        for q, (code, _, D, G, ib, off) in enumerate(sts):
            assert code == 0 and D == reqs[q].n_dirty and ib == sizes[q], (q, sts[q])
        mk, lat = [], []
        for _ in range(args.steps):
            mk.append(launch(plan))
            gt = plan.group_times()
            lat.extend(gt[g] for g in group_of)
        return mk, lat, sts, len(gr) - 1

    # the grouped plan with its diff launches timed (each group's diff
    # kernel records the device wall clock at its start and end)
    crum.crum_ctx_set_timing(ctx, crum.TIMING_DIFF)
    t_create = time.perf_counter()
    plan = make_plan()
    create_ms = 1e3 * (time.perf_counter() - t_create)
    crum.crum_ctx_set_timing(ctx, 0)
    mk, lat_b, sts, n_groups = timed(plan)
    n_pd, pd_ms = crum.crum_ctx_timing(ctx, 0)
    offsets = [st[5] for st in sts]
    batched_image = h_images.numpy(cap)[: max(o + b for o, b in zip(offsets, sizes))].copy()
    plan.destroy()

    # one graph for the whole batch: a single group (one persistent diff
    # over every unit of the 256 requests, one scan, one pack, one drain)
    crum.crum_ctx_set_param(ctx, crum.CRUM_PARAM_CHUNK_BYTES, N)
    crum.crum_ctx_set_param(ctx, crum.CRUM_PARAM_CHUNK_MAX_BYTES, N)
    plan = make_plan()
    mk_1, lat_1, sts_1, n_groups_1 = timed(plan)
    img_1 = h_images.numpy(cap)
    same_1 = all(np.array_equal(img_1[st[5]:st[5] + b], batched_image[o:o + b])
                 for st, o, b in zip(sts_1, offsets, sizes))
    assert same_1 and n_groups_1 == 1, "one-graph images differ from the grouped plan's"
    plan.destroy()
    autotune.apply(ctx, {"chunk_bytes": params["chunk_bytes"],
                         "chunk_max_bytes": params["chunk_max_bytes"]})

    # the same plan with the smallest requests first: same images, each at
    # its own offset
    crum.crum_ctx_set_param(ctx, crum.CRUM_PARAM_PLAN_ORDER, 1)
    plan = make_plan()
    mk_s, lat_s, sts_s, n_groups_s = timed(plan)
    img_s = h_images.numpy(cap)
    same_s = all(np.array_equal(img_s[st[5]:st[5] + b], batched_image[o:o + b])
                 for st, o, b in zip(sts_s, offsets, sizes))
    assert same_s, "smallest-first images differ from the given-order ones"
    plan.destroy()
    crum.crum_ctx_set_param(ctx, crum.CRUM_PARAM_PLAN_ORDER, params.get("plan_order", 0))

    # one-at-a-time plain path, same host offsets
    worst = max(crum.crum_image_bytes(len(r.regions), r.total_pages, r.total_pages,
                                      r.page_size) for r in reqs)
    pstage = H.DeviceBuffer(worst)
    pstatus = H.PinnedBuffer(64)
    pctx = crum.crum_ctx_create(0)  # the plain path with its default shapes

    def plain_all():
        lat = []
        t0 = time.perf_counter()
        for q, r in enumerate(reqs):
            tab = crum.region_table(tables[q])
            rc = crum.crum_snapshot(pctx, tab, r.page_size, 0, 5, pstage.ptr, worst,
                                    h_images.ptr + offsets[q], cap - offsets[q], stream.handle,
                                    pstatus.ptr)
            assert rc == 0
            stream.synchronize()
            st = crum.read_status(pstatus.ptr)
            assert st.code == 0 and st.image_bytes == sizes[q]
            lat.append(time.perf_counter() - t0)
        return time.perf_counter() - t0, lat

    plain_all()  # warm
    h_images.numpy(cap)[:] = 0
    t_plain, lat_p = plain_all()
    same = all(np.array_equal(h_images.numpy(cap)[o:o + b], batched_image[o:o + b])
               for o, b in zip(offsets, sizes))
    assert same, "batched and plain images differ"
    mk_ms = 1e3 * statistics.median(mk)
    # the plan's diff bytes per launch: both copies of every region with a
    # shadow (regions without one are flagged without loads) and one flag
    # byte per diff unit
    us_max = crum.crum_ctx_get_param(ctx, crum.CRUM_PARAM_DIFF_UNIT_SHIFT)
    plan_diff_bytes = 0
    for r in reqs:
        us = min(r.page_size.bit_length() - 1, us_max)
        for g in r.regions:
            plan_diff_bytes += (2 * g.nbytes if g.has_shadow else 0) + (g.nbytes >> us)
    pd_gbs = plan_diff_bytes * args.steps / (pd_ms * 1e-3) / 1e9 if pd_ms > 0 else None
    result = {
        "metric": "snapshot GB/s (diff+CRC+compact+drain), batched vs plain",
        "value": round(N / (statistics.median(mk)) / 1e9, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mk_ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic (seeded SplitMix64 bytes, PCG64 scenario)",
        "config": {"workload": f"{len(reqs)} snapshot requests, 1-32 allocations each, "
                               "request totals log-uniform 1 MiB-2 GiB, 4/64 KiB pages, dirty "
                               "U(1%,50%) in runs of mean 16",
                   "scanned_bytes": N, "dirty_pages": Dsum, "image_bytes": sum(sizes),
                   "groups": n_groups, "params": params, "tuned": bool(tuned),
                   "tuning_class": tune_key,
                   "settle": settle},
        "batched": {"makespan_ms": round(mk_ms, 2),
                    "gbs": round(N / statistics.median(mk) / 1e9, 2),
                    "groups": n_groups,
                    "plan_create_ms": round(create_ms, 1),
                    "makespans_ms": [round(1e3 * v, 1) for v in mk],
                    "latency_ms": {"p50": round(percentile(lat_b, 0.5), 2),
                                   "p90": round(percentile(lat_b, 0.9), 2),
                                   "p99": round(percentile(lat_b, 0.99), 2)},
                    "drain_gbs": round(sum(sizes) / statistics.median(mk) / 1e9, 2),
                    "diff_roofline": {
                        "kernel": "k_diff", "bound": "hbm",
                        "achieved": round(pd_gbs, 1) if pd_gbs else None,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(pd_gbs / HBM_PEAK_GBS, 4) if pd_gbs else None,
                        "launches": n_pd,
                        "avg_launch_ms": round(pd_ms / max(n_pd, 1), 4),
                        "algorithmic_bytes_per_step": plan_diff_bytes,
                        "what": "the plan's persistent diff launches (one per group), "
                                "timed by the device wall clock the diff kernel records at "
                                "its start and end, summed over the timed launches"}},
        "batched_smallest_first": {
            "makespan_ms": round(1e3 * statistics.median(mk_s), 2),
            "gbs": round(N / statistics.median(mk_s) / 1e9, 2),
            "latency_ms": {"p50": round(percentile(lat_s, 0.5), 2),
                           "p90": round(percentile(lat_s, 0.9), 2),
                           "p99": round(percentile(lat_s, 0.99), 2)},
            "groups": n_groups_s, "same_images": same_s},
        "batched_one_graph": {
            "makespan_ms": round(1e3 * statistics.median(mk_1), 2),
            "gbs": round(N / statistics.median(mk_1) / 1e9, 2),
            "latency_ms": {"p50": round(percentile(lat_1, 0.5), 2),
                           "p90": round(percentile(lat_1, 0.9), 2),
                           "p99": round(percentile(lat_1, 0.99), 2)},
            "groups": n_groups_1, "same_images": same_1,
            "what": "all 256 requests in one captured graph (one persistent diff, one "
                    "scan, one pack), drained by one copy when the graph ends"},
        "plain": {"makespan_ms": round(1e3 * t_plain, 2),
                  "gbs": round(N / t_plain / 1e9, 2),
                  "latency_ms": {"p50": round(1e3 * percentile(lat_p, 0.5), 2),
                                 "p90": round(1e3 * percentile(lat_p, 0.9), 2),
                                 "p99": round(1e3 * percentile(lat_p, 0.99), 2)}},
        "bit_exact_vs_plain": same,
    }
    crum.crum_ctx_destroy(ctx)
    crum.crum_ctx_destroy(pctx)

    for pr in pairs:
        for c, sh in pr:
            c.free()
            if sh:
                sh.free()
    for b in (staging, h_images, status, pstage, pstatus):
        b.free()
    return result


def run_leg(args, config: str) -> dict:
    """Run `bench.py --config <config>` with this run's steps, warmup and
    parameters in a child process (no CPU baseline there) and return its
    JSON line."""
    import subprocess
    cmd = [sys.executable, "-u", os.path.abspath(__file__), "--config", config,
           "--steps", str(args.steps), "--warmup", str(args.warmup), "--cpu-seconds", "0"]
    for kv in args.param:
        cmd += ["--param", kv]
    if args.tune_cache:
        cmd += ["--tune-cache", args.tune_cache]
    if args.no_corunner:
        cmd.append("--no-corunner")
    if args.seed_base != 1000:
        cmd += ["--seed-base", str(args.seed_base)]
    log(f"[bench] leg: {' '.join(cmd[2:])}")
    r = subprocess.run(cmd, stdout=subprocess.PIPE, text=True)
    if r.returncode != 0:
        raise SystemExit(f"bench leg {config} failed with status {r.returncode}")
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    if not lines:
        raise SystemExit(f"bench leg {config} printed no result")
    return json.loads(lines[-1])


HEADLINE_METRIC = ("snapshot GB/s (diff+CRC+compact+drain) and p99 latency, batched vs plain")


def bench_headline(args):
    """The default line.  Headline: the batched workload (256 snapshot
    requests, 71 GB scanned), one plan launch per step against the same 256
    requests snapshotted one at a time by the plain path: GB/s, makespan and
    p50/p99 request latency of both, images equal byte for byte.  Then the
    16 GiB many-allocations snapshot beside its SAXPY co-runner, which gives
    the diff kernel's roofline (HIP events around each launch over its timed
    snapshots), the drain against the host link, the pack, verify and
    scatter rates, and a verified restore; then the CPU oracle on one thread
    and on all threads.  The two GPU legs run as child processes of this
    one (this process does not use the GPU).  One JSON line."""
    # Each leg runs in a process of its own: in one process, the streams the
    # first leg leaves behind change how the second leg's snapshot and
    # co-runner streams share the device's hardware queues (the co-runner's
    # kernels then land between a diff launch's timing events), and the
    # first leg's 160 GB of buffers would be freed or held in its way.
    b = run_leg(args, "batched")
    log(f"[bench] batched leg: {b['value']} GB/s, p99 {b['batched']['latency_ms']['p99']} ms "
        f"vs plain {b['plain']['latency_ms']['p99']} ms")
    m = run_leg(args, "many")
    cpu = None
    if args.cpu_seconds > 0:
        from synth import scenarios as sc
        log("[bench] CPU oracle baseline ...")
        cpu = cpu_baseline(sc.many_allocs(seed=args.seed_base + 2), args.cpu_seconds,
                           args.cpu_threads)
    bat, pl = b["batched"], b["plain"]
    roof = dict(m["roofline"])
    roof["workload"] = ("the 16 GiB many-allocations snapshot (64 regions, 64 KiB pages) "
                        "beside the SAXPY co-runner: its own timed snapshots in this run")
    many = {k: m[k] for k in ("value", "unit", "ms_per_step", "latency_ms", "config", "restore",
                              "roofline_alone", "drain", "pack", "diff_and_crc", "header",
                              "breakdown_timed", "overlap")}
    many["metric"] = m["metric"]
    many["steps"] = m["steps"]
    result = {
        "metric": HEADLINE_METRIC,
        "value": b["value"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": b["steps"],
        "warmup": b["warmup"],
        "ms_per_step": b["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": b["data"],
        "config": dict(b["config"], parallelism="single GPU",
                       step="one plan launch snapshotting all 256 requests, ending when "
                            "every image has landed in pinned host memory"),
        "latency_ms": bat["latency_ms"],
        "batched": bat,
        "batched_smallest_first": b["batched_smallest_first"],
        "batched_one_graph": b["batched_one_graph"],
        "plain": pl,
        "bit_exact_vs_plain": b["bit_exact_vs_plain"],
        "vs_plain": {"gbs_ratio": round(b["value"] / pl["gbs"], 3),
                     "p50_ratio": round(bat["latency_ms"]["p50"] / pl["latency_ms"]["p50"], 3),
                     "p99_ratio": round(bat["latency_ms"]["p99"] / pl["latency_ms"]["p99"], 3)},
        "roofline": roof,
        "drain": m["drain"],
        "pack": m["pack"],
        "diff_and_crc": m["diff_and_crc"],
        "many_allocs": many,
        "cpu_baseline": cpu,
    }
    print(json.dumps(result), flush=True)


def bench_served(args):
    """Served workload: 32 clients with persistent device state (log-uniform
    64 MiB-8 GiB, 64 KiB pages, resident shadows), open-loop Poisson arrivals
    at 200 req/s, snapshot:restore 4:1, a 64 GiB pinned budget.  The same trace
    runs through the serving loop with several slots and with one slot (the
    plain one-request-at-a-time path)."""
    import threading

    import paper_1808_00117_amd as crum
    import paper_1808_00117_amd.hip as H
    import synth
    from synth import scenarios as sc

    crum.lib()
    P = 64 * 1024
    sizes = sc.served_clients(seed=args.seed_base + 5)
    trace = sc.served_trace(seed=args.seed_base + 5, duration=args.duration, rate=args.rate)
    warm = min(5.0, args.duration / 6)
    # offered device-to-host load: expected dirty bytes of the snapshots per second
    offered = sum(sizes[c] * f for t, c, k, f in trace if k == 1) / args.duration
    log(f"[served] {len(sizes)} clients, {sum(sizes) / 2**30:.1f} GiB, {len(trace)} requests "
        f"over {args.duration:.0f} s, offered D2H {offered / 1e9:.1f} GB/s")
    cur = [H.DeviceBuffer(n) for n in sizes]
    sh = [H.DeviceBuffer(n) for n in sizes]
    clients = [([(c.ptr, s.ptr, n, 500 + i)], P) for i, (c, s, n) in enumerate(zip(cur, sh, sizes))]
    fracs = [f for _, _, _, f in trace]
    BASE = 1 << 40
    probe_dev, probe_host = H.DeviceBuffer(256 << 20), H.PinnedBuffer(256 << 20)
    settles = []

    def reset_state():
        for i, (c, s, n) in enumerate(zip(cur, sh, sizes)):
            synth.fill_dev(c.ptr, n, args.seed_base + 5, i, 0, 0)
            H.memcpy_dtod(s.ptr, c.ptr, n)
        H.device_synchronize()

    last_sel = {}

    def prepare(user, client, kind, tag, stream):
        n = sizes[client]
        if kind == 1:
            f = 0.0 if tag >= BASE else fracs[tag]
            last_sel[client] = (tag, f)
            if f > 0:
                synth.mutate_frac_dev(cur[client].ptr, n, P, tag, f, tag, client, stream)
        else:
            sel, f = last_sel[client]
            if f > 0:
                synth.clobber_frac_dev(cur[client].ptr, n, P, sel, f, 777, client, stream)

    def run(n_slots):
        reset_state()
        last_sel.clear()
        srv = crum.Server(clients, n_slots, 64 << 30, prepare=prepare)
        srv.set_policy(args.policy)
        for i in range(len(sizes)):  # untimed base image per client
            srv.submit(i, 1, BASE + i)
        srv.poll(wait_all=True)
        settles.append(settle_copy_engines(H, probe_dev.ptr, probe_host.ptr))
        t0 = srv.time()

        def driver():
            for i, (t, c, kind, _) in enumerate(trace):
                dt = t0 + t - srv.time()
                if dt > 0:
                    time.sleep(dt)
                srv.submit(c, kind, i)
        th = threading.Thread(target=driver)
        th.start()
        th.join()
        done = srv.poll(wait_all=True, max_n=1 << 16)
        t_end = srv.time()
        srv.destroy()
        recs = [d for d in done if d["tag"] < BASE]
        assert all(d["code"] == 0 for d in recs), [d for d in recs if d["code"] != 0][:3]
        win = [d for d in recs if d["arrival_s"] - t0 >= warm]
        lat = [1e3 * (d["done_s"] - d["arrival_s"]) for d in win]
        snaps = [d for d in win if d["kind"] == 1]
        span = max(d["done_s"] for d in win) - (t0 + warm)
        scanned = sum(sizes[d["client"]] for d in snaps)
        drained = sum(d["image_bytes"] for d in snaps)
        return {"slots": n_slots, "requests": len(win),
                "latency_ms": {"p50": round(percentile(lat, 0.5), 2),
                               "p90": round(percentile(lat, 0.9), 2),
                               "p99": round(percentile(lat, 0.99), 2)},
                "snapshot_gbs": round(scanned / span / 1e9, 2),
                "drain_gbs": round(drained / span / 1e9, 2),
                "restore_h2d_gbs": round(sum(d["image_bytes"] for d in win if d["kind"] == 2)
                                         / span / 1e9, 2),
                "tail_s": round(t_end - t0 - args.duration, 2)}

    served = run(args.slots)
    log(f"[served] {served}")
    plain = run(1)
    log(f"[served] plain {plain}")
    result = {
        "metric": "snapshot GB/s and p99 latency, served vs plain",
        "value": served["snapshot_gbs"], "unit": "GB/s", "n_gpus": 1, "steps": len(trace),
        "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8",
        "data": "synthetic (seeded SplitMix64 bytes, PCG64 trace)",
        "config": {"workload": f"{len(sizes)} clients log-uniform 64 MiB-8 GiB "
                               f"({sum(sizes) / 2**30:.1f} GiB), 64 KiB pages, Poisson "
                               f"{args.rate:g} req/s, "
                               f"snapshot:restore 4:1, dirty U(2%,30%), 64 GiB pinned budget",
                   "duration_s": args.duration, "excluded_s": warm, "policy": args.policy,
                   "offered_d2h_gbs": round(offered / 1e9, 2), "settle": settles},
        "served": served, "plain": plain,
    }
    print(json.dumps(result), flush=True)


def mount_of(path: str) -> dict:
    """File system type and device of the mount holding `path` (/proc/mounts)."""
    path = os.path.realpath(path)
    best = None
    try:
        for line in open("/proc/mounts"):
            dev, mnt, fstype = line.split()[:3]
            if (path == mnt or path.startswith(mnt.rstrip("/") + "/")) and \
                    (best is None or len(mnt) > len(best[1])):
                best = (dev, mnt, fstype)
    except OSError:
        pass
    return {"device": best[0], "mount": best[1], "fstype": best[2]} if best else {}


def bench_persist(args):
    """Phase two: checkpoints of the 16 GiB many-allocations workload written
    to files.  Naive: each checkpoint snapshots, then writes its image and
    waits (the application is paused for both).  Overlapped: the image goes
    to a writer thread pool and the application resumes; two pinned image
    buffers alternate, so a checkpoint waits only if the write from two
    checkpoints back has not finished.  Between checkpoints the application
    computes (SAXPY graphs) for --app-ms."""
    import numpy as np

    import oracle
    import paper_1808_00117_amd as crum
    import paper_1808_00117_amd.hip as H
    import synth
    from synth import scenarios as sc

    crum.lib()
    scn = sc.many_allocs(seed=args.seed_base + 2)
    P, N, D, G, R = scn.page_size, scn.total_bytes, scn.n_dirty, scn.total_pages, len(scn.regions)
    pairs = materialize_raw(scn, H)
    table = crum.region_table([(c.ptr, s.ptr if s else 0, r.nbytes, r.id)
                               for (c, s), r in zip(pairs, scn.regions)])
    ib = crum.crum_image_bytes(R, G, D, P)
    cap = crum.crum_image_bytes(R, G, G, P)
    staging = H.DeviceBuffer(cap)
    bufs = [H.PinnedBuffer(cap), H.PinnedBuffer(cap)]
    status = H.PinnedBuffer(64)
    settle = settle_copy_engines(H, staging.ptr, bufs[0].ptr)
    ctx = crum.crum_ctx_create(0)
    s1, s2 = H.Stream(), H.Stream()
    d = args.persist_dir or os.path.join(os.environ.get("TMPDIR", "/tmp"), "crum_persist")
    os.makedirs(d, exist_ok=True)
    fs = mount_of(d)
    writer = crum.Writer(n_threads=args.writer_threads, chunk_bytes=64 << 20)
    n_sax = 4096 * 4096
    x, y = H.DeviceBuffer(4 * n_sax), H.DeviceBuffer(4 * n_sax)
    H.check(H.hip().hipMemset(x.ptr, 0x3F, 4 * n_sax), "hipMemset")
    H.check(H.hip().hipMemset(y.ptr, 0x3E, 4 * n_sax), "hipMemset")
    graph = H.Graph(s2, lambda st: [synth.saxpy_loop_dev(y.ptr, x.ptr, 1.0001, n_sax, 1, 4096,
                                                          st.handle) for _ in range(16)])

    def app():
        t_end = time.perf_counter() + args.app_ms * 1e-3
        while time.perf_counter() < t_end:
            graph.launch(s2)
            s2.synchronize()

    def snap(buf, seq):
        rc = crum.crum_snapshot(ctx, table, P, 0, seq, staging.ptr, cap, buf.ptr, cap,
                                s1.handle, status.ptr)
        assert rc == 0, rc
        s1.synchronize()
        st = crum.read_status(status.ptr)
        assert st.code == 0 and st.n_dirty == D and st.image_bytes == ib, st

    snap(bufs[0], 1)
    K = args.steps
    writes = []
    log(f"[persist] {K} checkpoints of {ib / 1e9:.2f} GB images to {d} ({fs})")
    # naive: snapshot + synchronous write
    naive = []
    snap_only = []

    def drain_gbs():
        n, ms_ = crum.crum_ctx_timing(ctx, 2)
        crum.crum_ctx_timing_reset(ctx)
        return round(ib * K / (ms_ * 1e-3) / 1e9, 2) if ms_ else None
    crum.crum_ctx_timing_reset(ctx)
    crum.crum_ctx_set_timing(ctx, crum.TIMING_DRAIN)
    for i in range(K):
        app()
        t = time.perf_counter()
        snap(bufs[0], 100 + i)
        snap_only.append(time.perf_counter() - t)
        st = writer.poll(writer.submit(os.path.join(d, f"naive{i % 2}.crum"), bufs[0].ptr, ib))
        assert st["code"] == 0, st
        writes.append(st)
        naive.append(time.perf_counter() - t)
    drain_naive = drain_gbs()
    # overlapped: snapshot, hand the image to the writer, resume
    over, waits, submits, pending = [], [], [], [None, None]
    t_all = time.perf_counter()
    for i in range(K):
        app()
        t = time.perf_counter()
        b = i % 2
        if pending[b] is not None:
            st = writer.poll(pending[b])
            assert st["code"] == 0, st
            writes.append(st)
        waits.append(time.perf_counter() - t)
        snap(bufs[b], 200 + i)
        t_sub = time.perf_counter()
        pending[b] = writer.submit(os.path.join(d, f"over{b}.crum"), bufs[b].ptr, ib)
        submits.append(time.perf_counter() - t_sub)
        over.append(time.perf_counter() - t)
    last = (K - 1) % 2
    for b in (1 - last, last):
        if pending[b] is not None:
            st = writer.poll(pending[b])
            assert st["code"] == 0, st
            writes.append(st)
    t_all = time.perf_counter() - t_all
    drain_over = drain_gbs()
    crum.crum_ctx_set_timing(ctx, False)
    # the last file equals its image and parses
    back = np.fromfile(os.path.join(d, f"over{last}.crum"), np.uint8)
    same = bool(np.array_equal(back, bufs[last].numpy(ib)))
    rc, hdr = oracle.parse(back)
    assert same and rc == oracle.OK and hdr["seq"] == 200 + K - 1
    del back
    for f in os.listdir(d):
        if f.endswith(".crum"):
            os.remove(os.path.join(d, f))
    writer.destroy()
    wr = [w["bytes"] / w["seconds"] / 1e9 for w in writes]
    ms = lambda v: round(1e3 * v, 2)  # noqa: E731
    result = {
        "metric": "checkpoint pause (snapshot + persist to a file), overlapped vs naive",
        "value": ms(statistics.median(over)), "unit": "ms", "n_gpus": 1, "steps": K,
        "warmup": 1, "ms_per_step": ms(statistics.median(over)), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic (seeded SplitMix64 bytes, PCG64 scenario)",
        "config": {"workload": "64 allocations scaled to 16 GiB, 64 KiB pages, clustered "
                               "dirty runs; each checkpoint's image written to a file",
                   "image_bytes": ib, "app_ms_between": args.app_ms,
                   "writer_threads": args.writer_threads, "dir": d, "filesystem": fs,
                   "settle": settle},
        "overlapped": {"pause_ms": {"p50": ms(statistics.median(over)), "max": ms(max(over))},
                       "buffer_wait_ms_max": ms(max(waits)),
                       "submit_ms_max": ms(max(submits)), "total_s": round(t_all, 2),
                       "drain_gbs": drain_over},
        "naive": {"pause_ms": {"p50": ms(statistics.median(naive)), "max": ms(max(naive))},
                  "snapshot_part_ms_p50": ms(statistics.median(snap_only)),
                  "drain_gbs": drain_naive},
        "persist_gbs": {"p50": round(statistics.median(wr), 2), "min": round(min(wr), 2),
                        "direct": bool(writes[-1]["direct"])},
        "file_equals_image": same,
    }
    crum.crum_ctx_destroy(ctx)
    print(json.dumps(result), flush=True)


def bench_diff_sizes(args):
    """The diff kernel alone by launch size, page size and units per wave:
    one 8 GiB region pair (current and shadow, equal, so nothing is dirty),
    snapshotted in the diff-first order (one diff launch per snapshot) over
    its first 64 and 256 MiB, 1, 2 and 4 GiB and the whole 8 GiB, with 4 KiB and
    64 KiB pages, CRUM_PARAM_DIFF_GROUP 1, 2 and 4 (4 KiB units per wave; with
    64 KiB pages the units are 16 KiB and one per wave whatever the group).
    A 5 s pause after the allocation lets the copy engines and HBM settle.
    One JSON line per case: event-timed average launch and the HBM rate of
    its algorithmic bytes (2 x span + one flag byte per unit)."""
    import paper_1808_00117_amd as crum
    import paper_1808_00117_amd.hip as H
    import synth

    N = 8 << 30
    cur, sh = H.DeviceBuffer(N), H.DeviceBuffer(N)
    synth.fill_dev(cur.ptr, N, args.seed_base + 11, 0, 0, 0)
    H.memcpy_dtod(sh.ptr, cur.ptr, N)
    H.device_synchronize()
    time.sleep(5)
    s = H.Stream()
    status = H.PinnedBuffer(64)
    reps = max(3, args.steps // 4)
    try:
        for span in (64 << 20, 256 << 20, 1 << 30, 2 << 30, 4 << 30, N):
            table = crum.region_table([(cur.ptr, sh.ptr, span, 1)])
            for P in (4096, 65536):
                cap = crum.crum_image_prefix_bytes(1, span // P) + 4096
                staging = H.DeviceBuffer(cap)
                for group in ((1, 2, 4) if P == 4096 else (1,)):
                    ctx = crum.crum_ctx_create(0)
                    try:
                        crum.crum_ctx_set_param(ctx, crum.CRUM_PARAM_EAGER, 0)
                        crum.crum_ctx_set_param(ctx, crum.CRUM_PARAM_DIFF_GROUP, group)

                        def snap():
                            rc = crum.crum_snapshot(ctx, table, P, 0, 1, staging.ptr, cap, 0, 0,
                                                    s.handle, status.ptr)
                            s.synchronize()
                            st = crum.read_status(status.ptr)
                            if rc != 0 or st.code != 0 or st.n_dirty != 0:
                                raise RuntimeError(f"diff_sizes: rc {rc}, {st}")
                        for _ in range(3):
                            snap()
                        crum.crum_ctx_timing_reset(ctx)
                        crum.crum_ctx_set_timing(ctx, crum.TIMING_DIFF)
                        for _ in range(reps):
                            snap()
                        n, ms = crum.crum_ctx_timing(ctx, 0)
                    finally:
                        crum.crum_ctx_destroy(ctx)
                    unit = min(P, 1 << 14)
                    gbs = (2 * span + span // unit) * n / (ms * 1e-3) / 1e9
                    print(json.dumps({"config": "diff_sizes", "span_bytes": span, "page": P,
                                      "unit": unit, "diff_group": group, "launches": n,
                                      "avg_launch_ms": round(ms / n, 4),
                                      "achieved_gbs": round(gbs, 1),
                                      "frac": round(gbs / 8000, 4)}), flush=True)
                staging.free()
    finally:
        cur.free()
        sh.free()


def bench_lazy(args):
    """On-demand restore of the 16 GiB many-allocations image (section 4.2's
    read-fault readahead, with touches announced by the caller) against the
    full restore.  The targets are the shadow buffers, which hold the old
    bytes of the dirty pages; restoring makes them equal to the current
    buffers, and applying the page mutation again (an XOR) resets them.
    Measured: time to the first restored access (open + a touch of one
    dirty page, which fetches that 64 KiB page),
    a sequential sweep of every region in --lazy-step touches plus finish,
    and 1024 random 64 KiB touches."""
    import numpy as np

    import paper_1808_00117_amd as crum
    import paper_1808_00117_amd.hip as H
    import synth
    from synth import scenarios as sc

    crum.lib()
    scn = sc.many_allocs(seed=args.seed_base + 2)
    P, N, D, G, R = scn.page_size, scn.total_bytes, scn.n_dirty, scn.total_pages, len(scn.regions)
    pairs = materialize_raw(scn, H)
    table = crum.region_table([(c.ptr, s.ptr, r.nbytes, r.id)
                               for (c, s), r in zip(pairs, scn.regions)])
    targets = crum.region_table([(s.ptr, 0, r.nbytes, r.id)
                                 for (c, s), r in zip(pairs, scn.regions)])
    ib = crum.crum_image_bytes(R, G, D, P)
    staging = H.DeviceBuffer(ib)
    himg = H.PinnedBuffer(ib)
    status = H.PinnedBuffer(64)
    settle = settle_copy_engines(H, staging.ptr, himg.ptr, min(256 << 20, ib))
    ctx = crum.crum_ctx_create(0)
    s1 = H.Stream()
    assert crum.crum_snapshot(ctx, table, P, 0, 5, staging.ptr, ib, himg.ptr, ib, s1.handle,
                              status.ptr) == 0
    s1.synchronize()
    st = crum.read_status(status.ptr)
    assert st.code == 0 and st.n_dirty == D and st.image_bytes == ib, st
    d_pages = []
    for r in scn.regions:
        pg = np.ascontiguousarray(r.dirty_pages, np.int64)
        buf = H.DeviceBuffer(max(pg.nbytes, 8))
        if pg.size:
            H.memcpy_htod(buf.ptr, pg.ctypes.data, pg.nbytes)
        d_pages.append((buf, pg))

    def reset():
        """Old bytes back into the dirty pages of the targets."""
        for (c, sh), r, (buf, pg) in zip(pairs, scn.regions, d_pages):
            if pg.size:
                synth.mutate_dev(sh.ptr, r.nbytes, P, buf.ptr, int(pg.size), int(pg.max()),
                                 r.mut_kind, scn.mut_seed, r.fill_region, 0)
        H.device_synchronize()

    def n_differing():
        """Pages where the targets differ from the current buffers (a snapshot
        kept on the device)."""
        assert crum.crum_snapshot(ctx, table, P, 0, 6, staging.ptr, ib, 0, 0, s1.handle,
                                  status.ptr) == 0
        s1.synchronize()
        return crum.read_status(status.ptr).n_dirty

    def ok(code_addr=status.ptr):
        st_ = crum.read_status(code_addr)
        assert st_.code == 0, st_

    assert n_differing() == D
    # the first access: the first dirty page of the largest region (a fault
    # whose window is that one page)
    ri_first = int(np.argmax([r.nbytes if r.dirty_pages.size else 0 for r in scn.regions]))
    pg_first = int(scn.regions[ri_first].dirty_pages[0])
    trials = 2 if args.quick else 4
    full, first, open_ms, sweep, rand = [], [], [], [], []
    stats = {}
    rng = np.random.default_rng(11)
    sizes = np.array([r.nbytes for r in scn.regions], np.float64)
    for t in range(trials + 1):
        # full restore
        reset()
        t0 = time.perf_counter()
        assert crum.crum_restore(ctx, targets, himg.ptr, ib, crum.CRUM_VERIFY, staging.ptr, ib,
                                 s1.handle, status.ptr) == 0
        s1.synchronize()
        t1 = time.perf_counter()
        ok()
        if t == 0:
            assert n_differing() == 0
        else:
            full.append(t1 - t0)
        # on demand: first access, then a sequential sweep and finish
        reset()
        t0 = time.perf_counter()
        lz = crum.Lazy(ctx, targets, himg.ptr, ib, crum.CRUM_VERIFY, 2 << 20, staging.ptr, ib,
                       s1.handle, status.ptr)
        s1.synchronize()
        t_open = time.perf_counter()
        ok()
        assert lz.touch(ri_first, pg_first * P, P, s1.handle, status.ptr) == 1
        s1.synchronize()
        t1 = time.perf_counter()
        for ri, r in enumerate(scn.regions):
            for off in range(0, r.nbytes, args.lazy_step):
                lz.touch(ri, off, min(args.lazy_step, r.nbytes - off), s1.handle, 0)
        lz.finish(s1.handle, status.ptr)
        s1.synchronize()
        t2 = time.perf_counter()
        ok()
        sw = lz.stats()
        lz.close()
        if t == 0:
            assert n_differing() == 0
            stats["sweep"] = sw
        else:
            open_ms.append(t_open - t0)
            first.append(t1 - t0)
            sweep.append(t2 - t0)
        # on demand: random single-page accesses
        reset()
        lz = crum.Lazy(ctx, targets, himg.ptr, ib, crum.CRUM_VERIFY, 2 << 20, staging.ptr, ib,
                       s1.handle, status.ptr)
        s1.synchronize()
        picks = []
        for _ in range(1024):
            ri = int(rng.choice(R, p=sizes / sizes.sum()))
            picks.append((ri, int(rng.integers(0, scn.regions[ri].nbytes // P)) * P))
        t0 = time.perf_counter()
        for ri, off in picks:
            lz.touch(ri, off, P, s1.handle, 0)
        s1.synchronize()
        t1 = time.perf_counter()
        rs = lz.stats()
        lz.finish(s1.handle, status.ptr)
        s1.synchronize()
        ok()
        lz.close()
        if t == 0:
            assert n_differing() == 0
        else:
            rand.append(t1 - t0)
            stats["random"] = rs
    ms = lambda v: round(1e3 * statistics.median(v), 3)  # noqa: E731
    sw = stats["sweep"]
    result = {
        "metric": "restart latency: time until the first access of a restored image can run",
        "value": ms(first), "unit": "ms", "n_gpus": 1, "steps": trials, "warmup": 1,
        "ms_per_step": ms(first), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8",
        "data": "synthetic (seeded SplitMix64 bytes, PCG64 scenario)",
        "config": {"workload": "on-demand restore of the image of 64 allocations scaled to "
                               "16 GiB, 64 KiB pages, clustered dirty runs",
                   "image_bytes": ib, "dirty_pages": D, "small_region_bytes": 2 << 20,
                   "sweep_step_bytes": args.lazy_step, "verify": True, "settle": settle},
        "full_restore_ms": ms(full),
        "on_demand": {
            "open_ms": ms(open_ms),
            "first_access_ms": ms(first),
            "first_access": f"region {ri_first} page {pg_first}: one 64 KiB page fetched",
            "sweep_plus_finish_ms": ms(sweep),
            "sweep": {"faults": sw["faults"], "copies": sw["copies"],
                      "pages_fetched_by_touches_and_finish": sw["pages_fetched"],
                      "image_gbs": round(ib / (statistics.median(sweep)) / 1e9, 2)},
            "random_1024_pages": {"ms": ms(rand), "faults": stats["random"]["faults"],
                                  "copies": stats["random"]["copies"],
                                  "bytes_fetched": stats["random"]["bytes_fetched"],
                                  "fraction_of_image_pages": round(
                                      stats["random"]["pages_fetched"] / max(D, 1), 4)},
        },
        "checked": "targets equal the current buffers after every first trial (snapshot "
                   "finds 0 differing pages)",
    }
    crum.crum_ctx_destroy(ctx)
    print(json.dumps(result), flush=True)


def fill_managed_host(buf, scn, region_index, pages, threads=16):
    """Write the generator bytes of the listed pages from host threads."""
    from concurrent.futures import ThreadPoolExecutor

    import synth
    r = scn.regions[region_index]
    P = scn.page_size

    def one(p):
        synth.fill_host(P, r.fill_seed, r.fill_region, int(p) * P, out=buf.numpy(int(p) * P, P))
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(one, pages))


def fill_managed_device(buf, scn, region_index, pages):
    """Prefetch the listed pages to the device (runs coalesced), then write
    their generator bytes with a device kernel."""
    import paper_1808_00117_amd.hip as H
    import synth
    r = scn.regions[region_index]
    P = scn.page_size
    pages = sorted(int(p) for p in pages)
    i, prefetch_rc = 0, set()
    while i < len(pages):
        j = i
        while j + 1 < len(pages) and pages[j + 1] == pages[j] + 1:
            j += 1
        prefetch_rc.add(buf.prefetch(pages[i] * P, (j - i + 1) * P, 0, 0))
        synth.fill_dev(buf.ptr + pages[i] * P, (j - i + 1) * P, r.fill_seed, r.fill_region,
                       pages[i] * P, 0)
        i = j + 1
    H.device_synchronize()
    return sorted(prefetch_rc)


def bench_managed(args):
    """Managed-memory workload: one 32 GiB hipMallocManaged region, 2 MiB
    pages; 70 % of pages written last by host threads, 30 % prefetched to the
    device and written by a kernel; the HBM shadow differs on 20 % of pages
    by a 256-byte span.  The image must not depend on residency: it is
    checked on sampled pages against bytes regenerated on the host, its
    bitmap against the chosen set, and its checksums by the oracle's parser."""
    import numpy as np

    import oracle
    import paper_1808_00117_amd as crum
    import paper_1808_00117_amd.hip as H
    import synth
    from synth import scenarios as sc

    crum.lib()
    scn = sc.managed(seed=args.seed_base + 3)
    r = scn.regions[0]
    P, G, N, D = scn.page_size, scn.total_pages, scn.total_bytes, scn.n_dirty
    dev_pages = scn.meta["device_pages"]
    host_pages = np.setdiff1d(np.arange(G), dev_pages)
    t0 = time.perf_counter()
    cur = H.ManagedBuffer(N)
    attrs = H.pointer_attributes(cur.ptr)
    log(f"[managed] pointer attributes {attrs}")
    if not cur.device_mapped():
        raise SystemExit("managed allocation is not mapped for the device; not launching")
    fill_managed_host(cur, scn, 0, host_pages)
    t_host = time.perf_counter() - t0
    prefetch_rc = fill_managed_device(cur, scn, 0, dev_pages)
    sh = H.DeviceBuffer(N)
    synth.fill_dev(sh.ptr, N, r.fill_seed, r.fill_region, 0, 0)
    pages_d = H.DeviceBuffer(8 * r.dirty_pages.size)
    pd = np.ascontiguousarray(r.dirty_pages, np.int64)
    H.memcpy_htod(pages_d.ptr, pd.ctypes.data, pd.nbytes)
    synth.mutate_dev(sh.ptr, N, P, pages_d.ptr, pd.size, int(pd.max()), r.mut_kind, scn.mut_seed,
                     r.fill_region, 0)
    H.device_synchronize()
    log(f"[managed] filled in {time.perf_counter() - t0:.1f} s (host part {t_host:.1f} s); "
        f"prefetch status {prefetch_rc}")

    def residency(pages):
        locs = {}
        for p in pages[:: max(1, len(pages) // 32)]:
            rc, loc = cur.last_prefetch_location(int(p) * P, P)
            locs[f"rc{rc}:loc{loc}"] = locs.get(f"rc{rc}:loc{loc}", 0) + 1
        return locs
    res_before = {"device_pages": residency(dev_pages), "host_pages": residency(host_pages)}
    image_bytes = crum.crum_image_bytes(1, G, D, P)
    cap = crum.crum_image_bytes(1, G, G, P)
    staging = H.DeviceBuffer(cap)
    himg = H.PinnedBuffer(cap)
    status = H.PinnedBuffer(64)
    settle = settle_copy_engines(H, staging.ptr, himg.ptr)
    ctx = crum.crum_ctx_create(0)
    s1 = H.Stream()
    table = crum.region_table([(cur.ptr, sh.ptr, N, r.id)])

    def snap():
        rc = crum.crum_snapshot(ctx, table, P, 0, 3, staging.ptr, cap, himg.ptr, cap, s1.handle,
                                status.ptr)
        assert rc == 0
        s1.synchronize()
        st = crum.read_status(status.ptr)
        assert st.code == 0 and st.n_dirty == D and st.image_bytes == image_bytes, st

    snap()
    for _ in range(args.warmup):
        snap()
    crum.crum_ctx_timing_reset(ctx)
    crum.crum_ctx_set_timing(ctx, True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        snap()
    t_total = time.perf_counter() - t0
    crum.crum_ctx_set_timing(ctx, False)
    n_diff, diff_ms = crum.crum_ctx_timing(ctx, 0)
    n_dr, drain_ms = crum.crum_ctx_timing(ctx, 2)
    # parity on the image: checksums and layout by the oracle's parser, the
    # bitmap against the chosen set, sampled pages and CRCs against bytes
    # regenerated on the host
    img = himg.numpy(image_bytes)
    rc, hdr = oracle.parse(img)
    assert rc == oracle.OK and hdr["n_dirty"] == D
    W = (G + 63) // 64
    bm = np.frombuffer(img[96:96 + 8 * W].tobytes(), np.uint64)
    got = np.flatnonzero(np.unpackbits(bm.view(np.uint8), bitorder="little"))
    assert np.array_equal(got, r.dirty_pages), "bitmap differs from the chosen set"
    data_off = hdr["data_off"]
    rng = np.random.default_rng(5)
    for k in rng.choice(D, size=24, replace=False):
        g = int(r.dirty_pages[k])
        page = img[data_off + k * P: data_off + (k + 1) * P]
        exp = synth.fill_host(P, r.fill_seed, r.fill_region, g * P)
        assert np.array_equal(page, exp), f"page {g}"
        crc = int(np.frombuffer(img[data_off + D * P + 4 * k: data_off + D * P + 4 * k + 4]
                                .tobytes(), np.uint32)[0])
        assert crc == oracle.crc32c(exp)
    res_after = {"device_pages": residency(dev_pages), "host_pages": residency(host_pages)}
    value = N * args.steps / t_total / 1e9
    result = {
        "metric": "snapshot GB/s (diff+CRC+compact+drain), managed memory",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * t_total / args.steps, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic (seeded SplitMix64 bytes, PCG64 scenario)",
        "config": {"workload": "one 32 GiB hipMallocManaged region, 2 MiB pages, 70% of pages "
                               "written last by host threads, 30% prefetched to the device and "
                               "written by a kernel, shadow differs on 20% of pages (256-byte "
                               "spans)", "scanned_bytes": N, "dirty_pages": D,
                   "image_bytes": image_bytes, "settle": settle},
        "diff": {"achieved_gbs": round(2 * N * args.steps / (diff_ms * 1e-3) / 1e9, 1),
                 "launches": n_diff},
        "drain": {"achieved_gbs": round(image_bytes * args.steps / (drain_ms * 1e-3) / 1e9, 2)
                  if drain_ms else None},
        "residency": {"pointer_attributes": {k: v for k, v in attrs.items()
                                             if k in ("type", "isManaged", "allocationFlags")},
                      "before": res_before, "after": res_after,
                      "prefetch_status": prefetch_rc},
        "parity": "bitmap exact; 24 sampled pages and CRCs equal to host-regenerated bytes; "
                  "image checksums verified by the oracle parser",
    }
    untracked_image = img.copy()
    result["tracked"] = managed_tracked_leg(args, scn, cur, sh, table, ctx, staging, himg, cap,
                                            status, s1, untracked_image, t_total / args.steps)
    crum.crum_ctx_destroy(ctx)
    print(json.dumps(result), flush=True)


def managed_tracked_leg(args, scn, cur, sh, table, ctx, staging, himg, cap, status, s1,
                        untracked_image, untracked_s):
    """Host write tracking (paper section 3.2, Algorithm 1) on the managed
    workload.  The host-written pages are written through a tracker's view
    and flushed into the managed region; the snapshot then reads only the
    candidate pages: those flushed since the last snapshot, and every
    device-written page (the device's writes are not tracked).

    Set-up (untimed): the view gets the shadow's bytes of every host page and
    is flushed (the state at the last snapshot); the device pages are written
    again by their kernel; the pending set is cleared.  Then the application
    writes each host page that changed since (the scenario's dirty host pages,
    with their current bytes) through the view, and a flush moves them into
    the region.  The managed region then holds exactly the bytes of the
    untracked runs, and the tracked image must equal theirs byte for byte."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import paper_1808_00117_amd as crum
    import synth
    from synth import scenarios as sc

    r = scn.regions[0]
    P, G, N, D = scn.page_size, scn.total_pages, scn.total_bytes, scn.n_dirty
    W = (G + 63) // 64
    dev_pages = np.asarray(scn.meta["device_pages"], np.int64)
    host_pages = np.setdiff1d(np.arange(G), dev_pages)
    dirty_host = np.intersect1d(r.dirty_pages, host_pages)
    threads = 16
    t0 = time.perf_counter()
    tr = crum.Tracker(N, P)
    try:
        v = tr.view()
        dirty_set = set(int(x) for x in r.dirty_pages)

        def write_shadow(p):
            page = v[p * P:(p + 1) * P]
            synth.fill_host(P, r.fill_seed, r.fill_region, p * P, out=page)
            if p in dirty_set:
                sc._mutate_one(page, P, p, r.mut_kind, scn.mut_seed, r.fill_region)
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(write_shadow, (int(p) for p in host_pages)))
        tr.flush(cur.ptr, threads)
        fill_managed_device(cur, scn, 0, dev_pages)
        tr.pending(clear=True)
        f0 = tr.stats()["faults"]
        t_setup = time.perf_counter() - t0

        # the application's writes since the last snapshot, then the flush of
        # Algorithm 1 before the next call into the GPU runtime
        t0 = time.perf_counter()

        def write_current(p):
            synth.fill_host(P, r.fill_seed, r.fill_region, p * P, out=v[p * P:(p + 1) * P])
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(write_current, (int(p) for p in dirty_host)))
        t_writes = time.perf_counter() - t0
        faults = tr.stats()["faults"] - f0
        t0 = time.perf_counter()
        n_flushed = tr.flush(cur.ptr, threads)
        t_flush = time.perf_counter() - t0
        pend = tr.pending(clear=False)
        pend_pages = np.flatnonzero(np.unpackbits(pend.view(np.uint8), bitorder="little"))
        assert np.array_equal(pend_pages, dirty_host), "pending set differs from the writes"
        cand = pend.copy()
        for p in dev_pages:
            cand[p >> 6] |= np.uint64(1) << np.uint64(p & 63)
        n_cand = int(np.unpackbits(cand.view(np.uint8)).sum())
        image_bytes = untracked_image.size

        def snap():
            rc = crum.crum_snapshot_tracked(ctx, table, P, 0, 3, cand, staging.ptr, cap,
                                            himg.ptr, himg.nbytes, s1.handle, status.ptr)
            assert rc == 0, rc
            s1.synchronize()
            st = crum.read_status(status.ptr)
            assert st.code == 0 and st.n_dirty == D and st.image_bytes == image_bytes, st

        snap()
        same = bool(np.array_equal(himg.numpy(image_bytes), untracked_image))
        assert same, "tracked image differs from the untracked one"
        for _ in range(args.warmup):
            snap()
        lat = []
        for _ in range(args.steps):
            t = time.perf_counter()
            snap()
            lat.append(time.perf_counter() - t)
        ms = 1e3 * statistics.median(lat)
        return {
            "what": "host-written pages written through a write-protected view and flushed "
                    "into the managed region (Algorithm 1); the snapshot reads only pages "
                    "flushed since the last snapshot and the device-written pages",
            "candidate_pages": n_cand, "of_pages": G,
            "candidate_bytes_read": n_cand * P, "pages_flushed": int(n_flushed),
            "write_faults": int(faults),
            "snapshot_ms": round(ms, 2),
            "snapshot_ms_untracked": round(1e3 * untracked_s, 2),
            "speedup": round(1e3 * untracked_s / ms, 3),
            "gbs": round(N / (ms * 1e-3) / 1e9, 2),
            "app_writes_ms": round(1e3 * t_writes, 1),
            "flush_ms": round(1e3 * t_flush, 1),
            "flush_gbs": round(n_flushed * P / max(t_flush, 1e-9) / 1e9, 2),
            "setup_s": round(t_setup, 1),
            "same_image_as_untracked": same,
        }
    finally:
        tr.destroy()


def main():
    args = parse_args()
    if args.pmc_summary:
        wl = "plain" if args.config == "plain" else "many_allocs"
        print(json.dumps(pmc_summary(args.pmc_summary[0], args.pmc_summary[1], wl), indent=1))
        return
    if args.trace_summary:
        print(trace_summary(args.trace_summary, args.steps, args.image_bytes, args.plan_groups,
                            args.warmup))
        return
    if args.pmc_table:
        print(pmc_table(args.pmc_table))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the snapshot path has no cross-GPU step and "
              "is measured on one device only (each GPU would snapshot its own regions "
              "independently).", file=sys.stderr)
        sys.exit(2)
    if args.config == "headline":
        return bench_headline(args)
    if args.config == "batched":
        print(json.dumps(bench_batched(args)), flush=True)
        return
    if args.config == "served":
        return bench_served(args)
    if args.config == "managed":
        return bench_managed(args)
    if args.config == "persist":
        return bench_persist(args)
    if args.config == "lazy":
        return bench_lazy(args)
    if args.config == "diff_sizes":
        return bench_diff_sizes(args)
    print(json.dumps(bench_many(args)), flush=True)


def bench_many(args, with_cpu: bool = True) -> dict:
    """The single-request workloads (`--config many`, the 16 GiB
    many-allocations snapshot beside a SAXPY co-runner, or `--config plain`,
    the 64 MiB one): K timed snapshots, the diff kernel's roofline, the
    drain against the host link, pack and header times, and a verified
    restore of the last image.  Returns the result dict."""
    import numpy as np

    import paper_1808_00117_amd as crum
    import paper_1808_00117_amd.hip as H
    import synth
    from synth import scenarios as sc

    crum.lib()
    if H.device_count() < 1:
        raise RuntimeError("bench.py needs a GPU")

    if args.config == "many":
        scn = sc.many_allocs(seed=args.seed_base + 2)
        workload = "many_allocs"
        wl_name = "64 allocations log-uniform 4KiB-1GiB scaled to 16 GiB, 64 KiB pages, " \
                  "clustered dirty runs (p_start 0.003, mean 32)"
    else:
        scn = sc.plain(seed=args.seed_base + 1)
        workload = "plain"
        wl_name = "one 64 MiB allocation, 4 KiB pages, 5% of pages dirty"
        if args.cold:
            workload = "plain_cold"
            wl_name += "; 8 independent copies rotated per step (1 GiB working set)"
    copies = 8 if (args.config == "plain" and args.cold) else 1
    P = scn.page_size
    N = scn.total_bytes
    D = scn.n_dirty
    G = scn.total_pages
    R = len(scn.regions)
    log(f"[bench] workload={workload} N={N} G={G} D={D} R={R}")

    if args.pmc_calibrate:
        a, b = H.DeviceBuffer(CALIB_BYTES), H.DeviceBuffer(CALIB_BYTES)
        synth.copy_dev(b.ptr, a.ptr, CALIB_BYTES, 0)
        H.device_synchronize()
        a.free()
        b.free()
    t0 = time.perf_counter()
    pair_sets = [materialize_raw(scn, H) for _ in range(copies)]
    log(f"[bench] materialised in {time.perf_counter() - t0:.1f} s")
    tables = [crum.region_table([(c.ptr, s.ptr if s else 0, r.nbytes, r.id)
                                 for (c, s), r in zip(pairs, scn.regions)])
              for pairs in pair_sets]
    step_no = [0]
    image_bytes = crum.crum_image_bytes(R, G, D, P)
    # capacity for an image with every page dirty: the snapshot then runs in
    # its chunk-pipelined order when the pages span several chunks (ENOSPC
    # impossible)
    cap = crum.crum_image_bytes(R, G, G, P)
    staging = H.DeviceBuffer(cap)
    h_image = H.PinnedBuffer(cap)
    status = H.PinnedBuffer(64)
    settle = settle_copy_engines(H, staging.ptr, h_image.ptr, min(256 << 20, cap))
    ctx = crum.crum_ctx_create(0)
    if args.diff_prio is not None:
        crum.crum_ctx_set_param(ctx, crum.CRUM_PARAM_DIFF_PRIORITY, args.diff_prio)
    from paper_1808_00117_amd import autotune
    for kv in args.param:
        k, v = kv.split("=")
        autotune.apply(ctx, {k: int(v)})
    s1, s2 = H.Stream(), H.Stream()
    ceiling = read_ceiling(H, scn, pair_sets[0], s1) if args.config == "many" else None
    # the largest region's current bytes copied into staging: the pack's bytes
    big = max(range(R), key=lambda k: scn.regions[k].nbytes)
    c_ceiling = copy_ceiling(H, pair_sets[0][big][0].ptr, staging.ptr,
                             min(D * P, scn.regions[big].nbytes), s1) \
        if args.config == "many" else None

    # co-runner: an application stream of fp32 SAXPY passes (y = a*x + y over
    # 4096x4096 elements), one kernel per pass, captured once as a graph of
    # PASSES kernels and replayed on its own stream
    n_sax = 4096 * 4096
    x = H.DeviceBuffer(4 * n_sax)
    y = H.DeviceBuffer(4 * n_sax)
    H.check(H.hip().hipMemset(x.ptr, 0x3F, 4 * n_sax), "hipMemset")
    H.check(H.hip().hipMemset(y.ptr, 0x3E, 4 * n_sax), "hipMemset")
    PASSES = 16

    def capture(st):
        for _ in range(PASSES):
            synth.saxpy_loop_dev(y.ptr, x.ptr, 1.0001, n_sax, 1, 4096, st.handle)
    graph = H.Graph(s2, capture)
    H.device_synchronize()
    sax_bytes_per_pass = 3 * 4 * n_sax

    def read_status():
        return crum.read_status(status.ptr)

    def run_snapshot(eager=True):
        crum.crum_ctx_set_param(ctx, crum.CRUM_PARAM_EAGER, 1 if eager else 0)
        c = cap if eager else image_bytes
        table = tables[step_no[0] % copies]
        step_no[0] += 1
        rc = crum.crum_snapshot(ctx, table, P, 0, 1, staging.ptr, c, h_image.ptr, c, s1.handle,
                                status.ptr)
        assert rc == 0, rc
        s1.synchronize()

    def corun(replays):
        for _ in range(replays):
            graph.launch(s2)

    # correctness of one step before timing (status, D, and both orders agree)
    run_snapshot()
    st = read_status()
    assert st.code == 0 and st.n_dirty == D and st.image_bytes == image_bytes, st
    if not args.quick:
        first_image = h_image.numpy(image_bytes).copy()
        run_snapshot(eager=False)
        assert read_status().n_dirty == D
        assert np.array_equal(h_image.numpy(image_bytes), first_image), "orders disagree"
        del first_image

    for _ in range(args.warmup):
        run_snapshot()

    # reference phases (outside the timed region)
    def median_ms(fn, n=5, record=None):
        v = []
        for _ in range(n):
            t = time.perf_counter()
            fn()
            v.append(time.perf_counter() - t)
        if record is not None:
            record.extend(round(1e3 * x, 3) for x in v)
        return 1e3 * statistics.median(v)
    # one flag byte per diff unit of min(P, 2^DIFF_UNIT_SHIFT) bytes
    unit_shift = min(P.bit_length() - 1,
                     crum.crum_ctx_get_param(ctx, crum.CRUM_PARAM_DIFF_UNIT_SHIFT))
    diff_bytes_step = 2 * N + (N >> unit_shift)
    crum.crum_ctx_timing_reset(ctx)
    crum.crum_ctx_set_timing(ctx, crum.TIMING_DIFF | crum.TIMING_DRAIN)
    n_alone = 1 if args.quick else 5
    alone_list = []
    snap_alone_ms = median_ms(run_snapshot, n_alone, alone_list)
    crum.crum_ctx_set_timing(ctx, False)
    n_da, da_ms = crum.crum_ctx_timing(ctx, 0)
    _, dr_alone_ms = crum.crum_ctx_timing(ctx, 2)
    # no drain copies in the direct order (the kernels write the host image)
    drain_alone_gbs = image_bytes * n_alone / (dr_alone_ms * 1e-3) / 1e9 if dr_alone_ms else None
    diff_alone_gbs = diff_bytes_step * n_alone / (da_ms * 1e-3) / 1e9
    checked_ms = float("nan") if args.quick else median_ms(lambda: run_snapshot(eager=False))
    corun_on = args.config == "many" and not args.no_corunner
    graph_ms, sax_alone_gbs = float("nan"), float("nan")
    if corun_on:
        e0, e1 = H.Event(), H.Event()
        probe = 1 if args.quick else 20
        e0.record(s2)
        corun(probe)
        e1.record(s2)
        graph_ms = e0.elapsed_ms(e1) / probe
        sax_alone_gbs = sax_bytes_per_pass * PASSES / (graph_ms * 1e-3) / 1e9
    link_ref = link_reference(H, staging.ptr, h_image.ptr, min(1 << 30, cap))
    log(f"[bench] snapshot alone {snap_alone_ms:.2f} ms (diff-first order {checked_ms:.2f} ms); "
        f"saxpy alone {sax_alone_gbs:.0f} GB/s ({graph_ms:.3f} ms per graph)")

    # timed region: exactly K steps, with the co-runner application issuing
    # SAXPY graphs continuously from its own host thread (at most two graphs
    # queued ahead, so it stops promptly when the last step ends)
    import threading
    stop = threading.Event()
    sax_graphs = [0]
    sax_time = [0.0]

    def corunner():
        evs = []
        while not stop.is_set():
            a, b = H.Event(), H.Event()
            a.record(s2)
            graph.launch(s2)
            b.record(s2)
            evs.append((a, b))
            if len(evs) > 2:
                a0, b0 = evs.pop(0)
                sax_time[0] += a0.elapsed_ms(b0)
                sax_graphs[0] += 1
        for a0, b0 in evs:
            sax_time[0] += a0.elapsed_ms(b0)
            sax_graphs[0] += 1

    # Timing events cost host time per record: for short snapshots only the
    # diff launches are timed inside the timed region, and pack / drain /
    # header are timed in a separate pass afterwards.
    breakdown_in_timed = snap_alone_ms > 5.0
    mask_rest = crum.TIMING_PACK | crum.TIMING_DRAIN | crum.TIMING_SCAN | crum.TIMING_HEADER
    crum.crum_ctx_timing_reset(ctx)
    crum.crum_ctx_set_timing(ctx, crum.TIMING_DIFF | (mask_rest if breakdown_in_timed else 0))
    lat = []
    H.device_synchronize()
    th = threading.Thread(target=corunner, daemon=True) if corun_on else None
    if th:
        th.start()
        time.sleep(0.005)
    t_start = time.perf_counter()
    for _ in range(args.steps):
        t = time.perf_counter()
        run_snapshot()
        lat.append(time.perf_counter() - t)
    if th:
        stop.set()
        th.join()
    H.device_synchronize()
    t_total = time.perf_counter() - t_start
    crum.crum_ctx_set_timing(ctx, False)

    timing = {}
    for cls, name in enumerate(["diff", "pack", "drain", "scan", "header"]):
        timing[name] = crum.crum_ctx_timing(ctx, cls)
    st = read_status()
    assert st.code == 0 and st.n_dirty == D, st
    n_breakdown = args.steps
    if not breakdown_in_timed:
        crum.crum_ctx_timing_reset(ctx)
        crum.crum_ctx_set_timing(ctx, mask_rest)
        n_breakdown = min(args.steps, 10)
        for _ in range(n_breakdown):
            run_snapshot()
        crum.crum_ctx_set_timing(ctx, False)
        for cls, name in enumerate(["diff", "pack", "drain", "scan", "header"]):
            if cls:
                timing[name] = crum.crum_ctx_timing(ctx, cls)

    n_diff, diff_ms = timing["diff"]
    diff_gbs = diff_bytes_step * args.steps / (diff_ms * 1e-3) / 1e9
    n_dr, drain_ms = timing["drain"]
    drain_gbs = image_bytes * n_breakdown / (drain_ms * 1e-3) / 1e9 if drain_ms else None
    n_pk, pack_ms = timing["pack"]
    pack_bytes = 2 * D * P + 4 * D
    pack_gbs = pack_bytes * n_breakdown / (pack_ms * 1e-3) / 1e9
    n_hd, header_ms = timing["header"]
    # the two HBM-bound kernels of the path together: diff and pack (with its
    # CRC) bytes of one snapshot over their summed time per snapshot
    dc_ms = diff_ms / args.steps + pack_ms / n_breakdown
    dc_gbs = (diff_bytes_step + pack_bytes) / (dc_ms * 1e-3) / 1e9
    sax_with = None
    if sax_graphs[0]:
        sax_with = sax_bytes_per_pass * PASSES * sax_graphs[0] / (sax_time[0] * 1e-3) / 1e9

    ms_step = 1e3 * t_total / args.steps
    value = N * args.steps / t_total / 1e9
    lat_ms = sorted(1e3 * v for v in lat)
    p50 = statistics.median(lat_ms)
    p99 = lat_ms[min(len(lat_ms) - 1, int(round(0.99 * (len(lat_ms) - 1))))]
    p90 = lat_ms[min(len(lat_ms) - 1, int(round(0.90 * (len(lat_ms) - 1))))]

    # restore (inverse path, outside the timed snapshot steps): the image just
    # taken, uploaded from pinned host memory, every page CRC verified before
    # any write, then scattered into the regions (their bytes already equal
    # the image's pages, so the workload is unchanged for the next step)
    crum.crum_ctx_timing_reset(ctx)
    crum.crum_ctx_set_timing(ctx, crum.TIMING_VERIFY | crum.TIMING_SCATTER)
    rest_lat = []
    for i in range(2 if args.quick else 6):
        t = time.perf_counter()
        rc = crum.crum_restore(ctx, tables[0], h_image.ptr, image_bytes, crum.CRUM_VERIFY,
                               staging.ptr, cap, s1.handle, status.ptr)
        assert rc == 0, rc
        s1.synchronize()
        if i:
            rest_lat.append(time.perf_counter() - t)
        rst = read_status()
        assert rst.code == 0 and rst.n_dirty == D, rst
    crum.crum_ctx_set_timing(ctx, False)
    n_v, verify_ms = crum.crum_ctx_timing(ctx, 5)
    n_sc, scatter_ms = crum.crum_ctx_timing(ctx, 6)
    rest_ms = 1e3 * statistics.median(rest_lat)
    restore = {
        "ms": round(rest_ms, 3),
        "image_gbs": round(image_bytes / (rest_ms * 1e-3) / 1e9, 2),
        "link_frac": round(image_bytes / (rest_ms * 1e-3) / 1e9 / LINK_PEAK_GBS, 4),
        "verify_gbs": round((D * P + 4 * D) * n_v / max(verify_ms * 1e-3, 1e-12) / 1e9, 1)
        if n_v else None,
        "scatter_gbs": round(2 * D * P * n_sc / max(scatter_ms * 1e-3, 1e-12) / 1e9, 1)
        if n_sc else None,
        "verify_frac": round((D * P + 4 * D) * n_v / max(verify_ms * 1e-3, 1e-12) / 1e9 /
                             HBM_PEAK_GBS, 4) if n_v else None,
        "scatter_frac": round(2 * D * P * n_sc / max(scatter_ms * 1e-3, 1e-12) / 1e9 /
                              HBM_PEAK_GBS, 4) if n_sc else None,
        "what": "H2D of the image from pinned memory, CRC verify of every page, scatter",
    }

    traffic = load_traffic(workload, diff_bytes_step * args.steps / max(n_diff, 1))
    result = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic (seeded SplitMix64 bytes, PCG64 scenario)",
        "config": {
            "workload": wl_name,
            "regions": R,
            "page_size": P,
            "scanned_bytes": N,
            "total_pages": G,
            "dirty_pages": D,
            "image_bytes": image_bytes,
            "staging_capacity": cap,
            "order": ("direct (image built in the pinned host image)"
                      if cap <= crum.crum_ctx_get_param(ctx, crum.CRUM_PARAM_DIRECT_BYTES)
                      else "chunk-pipelined" if N > crum.crum_ctx_get_param(
                          ctx, crum.CRUM_PARAM_CHUNK_BYTES)
                      else "chunked, one chunk (the whole image drained in one copy "
                           "behind the header)"),
            "co_runner": (f"fp32 SAXPY 4096x4096: graphs of {PASSES} single-pass kernels "
                          f"issued continuously on a second stream by a second host thread "
                          f"({sax_graphs[0]} graphs during the timed steps)") if corun_on else None,
            "parallelism": "single GPU",
            "params": autotune.current(ctx),
            "settle": settle,
        },
        "latency_ms": {"p50": round(p50, 3), "p90": round(p90, 3), "p99": round(p99, 3)},
        "restore": restore,
        "roofline": {
            "bound": "hbm",
            "kernel": "k_diff",
            "achieved": round(diff_gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(diff_gbs / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_step": diff_bytes_step,
            "avg_launch_ms": round(diff_ms / max(n_diff, 1), 4),
            "launches": n_diff,
            "measured_with": "co-runner active" if corun_on else "alone",
            "practical_ceiling": ceiling,
            "frac_of_ceiling": round(diff_gbs / ceiling["achieved"], 4) if ceiling else None,
        },
        "roofline_alone": {"kernel": "k_diff", "achieved": round(diff_alone_gbs, 1),
                           "frac": round(diff_alone_gbs / HBM_PEAK_GBS, 4),
                           "avg_launch_ms": round(da_ms / max(n_da, 1), 4),
                           "what": "same snapshot steps without the co-runner"},
        "drain": {"achieved": round(drain_gbs, 2) if drain_gbs else None,
                  "peak": LINK_PEAK_GBS, "unit": "GB/s",
                  "frac": round(drain_gbs / LINK_PEAK_GBS, 4) if drain_gbs else None,
                  "copies": n_dr, "reference": link_ref,
                  "what": None if drain_gbs else "no drain copies: the image was built in "
                                                   "the pinned host image (direct order)"},
        "pack": {"achieved": round(pack_gbs, 1), "unit": "GB/s", "peak": HBM_PEAK_GBS,
                 "frac": round(pack_gbs / HBM_PEAK_GBS, 4), "launches": n_pk,
                 "avg_launch_ms": round(pack_ms / max(n_pk, 1), 4),
                 "practical_ceiling": c_ceiling,
                 "frac_of_ceiling": round(pack_gbs / c_ceiling["achieved"], 4)
                 if c_ceiling else None,
                 "algorithmic_bytes_per_step": pack_bytes,
                 "what": None if drain_gbs else "direct order: the pack's stores cross the "
                                                "host link into the pinned image"},
        "diff_and_crc": {"achieved": round(dc_gbs, 1), "unit": "GB/s", "peak": HBM_PEAK_GBS,
                         "frac": round(dc_gbs / HBM_PEAK_GBS, 4),
                         "ms_per_snapshot": round(dc_ms, 4),
                         "algorithmic_bytes_per_step": diff_bytes_step + pack_bytes,
                         "what": "k_diff and k_pack (copy + CRC-32C) together: both kernels' "
                                 "algorithmic bytes of one snapshot over their summed launch "
                                 "durations per snapshot"},
        "header": {"avg_launch_ms": round(header_ms / max(n_hd, 1), 4)},
        "breakdown_timed": "in the timed steps" if breakdown_in_timed else
                           f"separate pass of {n_breakdown} snapshots after the timed steps",
        "overlap": {
            "snapshot_ms_alone": round(snap_alone_ms, 3),
            "snapshot_ms_alone_each": alone_list,
            "drain_gbs_alone": round(drain_alone_gbs, 2) if drain_alone_gbs else None,
            "snapshot_ms_with_corunner": round(p50, 3) if corun_on else None,
            "snapshot_ms_diff_first_order": round(checked_ms, 3),
            "saxpy_gbs_alone": round(sax_alone_gbs, 1) if corun_on else None,
            "saxpy_gbs_with_snapshot": round(sax_with, 1) if sax_with else None,
        },
    }
    if args.cpu_seconds > 0 and with_cpu:
        log("[bench] CPU oracle baseline ...")
        result["cpu_baseline"] = cpu_baseline(scn, args.cpu_seconds, args.cpu_threads)
    else:
        result["cpu_baseline"] = None
    crum.crum_ctx_destroy(ctx)
    for pairs in pair_sets:
        for c, s in pairs:
            c.free()
            if s:
                s.free()
    for b in (staging, h_image, status, x, y):
        b.free()
    return result


if __name__ == "__main__":
    main()
