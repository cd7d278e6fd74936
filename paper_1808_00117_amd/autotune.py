"""Autotuner for launch and pipeline shapes.

Searches the context parameters that shape the device work (diff unit size,
non-temporal loads, diff and pack grid sizes, chunk or group sizes) by timing
a caller-supplied workload, and keeps the winners in a JSON cache keyed by the
device (compute capability, compute units, HIP runtime version) and by the
workload class: ``snapshot|p<page size>|b<k>`` for single snapshots scanning
2^k..2^(k+1) bytes, ``plan|b<k>`` for plans.  A candidate value is kept only
when it beats the best so far by more than the run-to-run spread of the
default shapes, so noise never becomes a tuned shape.  The library reads the
same file (``crum_ctx_create``'s tuning_cache argument) and applies a class's
shapes to the calls of that class, so C callers get them too.
"""
from __future__ import annotations

import ctypes
import itertools
import json
import os
import time
from typing import Callable, Dict, Iterable, List, Optional

from . import _lib as C

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuning_cache.json")

PARAMS = {
    "diff_unit_shift": C.CRUM_PARAM_DIFF_UNIT_SHIFT,
    "diff_nontemporal": C.CRUM_PARAM_DIFF_NONTEMPORAL,
    "diff_blocks": C.CRUM_PARAM_DIFF_BLOCKS,
    "pack_blocks": C.CRUM_PARAM_PACK_BLOCKS,
    "chunk_bytes": C.CRUM_PARAM_CHUNK_BYTES,
    "chunk_max_bytes": C.CRUM_PARAM_CHUNK_MAX_BYTES,
    "drain_chunk_bytes": C.CRUM_PARAM_DRAIN_CHUNK_BYTES,
    "piece_shift": C.CRUM_PARAM_PIECE_SHIFT,
    "pack_depth": C.CRUM_PARAM_PACK_DEPTH,
    "diff_priority": C.CRUM_PARAM_DIFF_PRIORITY,
    "crc_variant": C.CRUM_PARAM_CRC_VARIANT,
    "plan_order": C.CRUM_PARAM_PLAN_ORDER,
    "direct_bytes": C.CRUM_PARAM_DIRECT_BYTES,
    "chunk_growth": C.CRUM_PARAM_CHUNK_GROWTH,
    "pack_nt_store": C.CRUM_PARAM_PACK_NT_STORE,
    "pack_prefetch": C.CRUM_PARAM_PACK_PREFETCH,
    "pack_nt_load": C.CRUM_PARAM_PACK_NT_LOAD,
    "diff_group": C.CRUM_PARAM_DIFF_GROUP,
    "eager": C.CRUM_PARAM_EAGER,
}


def class_key(kind: str, nbytes: int, page_size: int = 0) -> str:
    """Cache key of a workload class: kind "snapshot" (one page size) or
    "plan", and k = floor(log2(scanned bytes))."""
    k = max(0, int(nbytes).bit_length() - 1)
    if kind == "snapshot":
        return f"snapshot|p{int(page_size)}|b{k}"
    if kind == "plan":
        return f"plan|b{k}"
    raise ValueError(kind)


# hipDeviceAttribute_t values (hip_runtime_api.h, ROCm 7)
_ATTR_CC_MAJOR, _ATTR_CC_MINOR, _ATTR_CUS = 23, 61, 63


def device_key() -> str:
    """'cc<major>.<minor>-<CUs>cu|hip<runtime version>' of device 0 (the
    marketing name can be empty, so the key uses the compute capability that
    HIP reports, 9.5 for gfx950, and the compute unit count)."""
    from . import hip as H
    h = H.hip()
    ver = ctypes.c_int(0)
    h.hipRuntimeGetVersion.restype = ctypes.c_int
    h.hipRuntimeGetVersion.argtypes = [ctypes.POINTER(ctypes.c_int)]
    h.hipRuntimeGetVersion(ctypes.byref(ver))
    h.hipDeviceGetAttribute.restype = ctypes.c_int
    h.hipDeviceGetAttribute.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int]

    def attr(a):
        v = ctypes.c_int(-1)
        h.hipDeviceGetAttribute(ctypes.byref(v), a, 0)
        return v.value
    return f"cc{attr(_ATTR_CC_MAJOR)}.{attr(_ATTR_CC_MINOR)}-{attr(_ATTR_CUS)}cu|hip{ver.value}"


def apply(ctx: int, params: Dict[str, int]) -> None:
    for k, v in params.items():
        C.crum_ctx_set_param(ctx, PARAMS[k], int(v))


def current(ctx: int) -> Dict[str, int]:
    return {k: C.crum_ctx_get_param(ctx, p) for k, p in PARAMS.items()}


def load(workload: str, path: str = DEFAULT_CACHE) -> Optional[Dict[str, int]]:
    try:
        with open(path) as f:
            cache = json.load(f)
    except (OSError, ValueError):
        return None
    entry = cache.get(device_key(), {}).get(workload)
    return dict(entry["params"]) if entry else None


def save(workload: str, params: Dict[str, int], table: List, path: str = DEFAULT_CACHE,
         stats: Optional[Dict[str, float]] = None) -> None:
    try:
        with open(path) as f:
            cache = json.load(f)
    except (OSError, ValueError):
        cache = {}
    entry = {"params": params, "trials": table}
    if stats:
        entry.update(stats)
    cache.setdefault(device_key(), {})[workload] = entry
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def search(ctx: int, run: Callable[[], float], space: Dict[str, Iterable[int]],
           repeats: int = 3, log: Optional[Callable[[str], None]] = None):
    """Coordinate search: starting from the context's current parameters,
    sweep one parameter at a time over its candidate values (others fixed at
    their best so far), scoring each by the median of `repeats` runs of
    `run()` (which returns seconds and must rebuild any state that depends on
    the parameters).  The default shapes are measured first; the spread of
    their runs (slowest minus fastest) is the noise margin, and a candidate
    replaces the best so far only when it is faster by more than that margin.
    Returns (best params, trials, stats) with stats = {default_s, best_s,
    spread_s, gain}."""
    best = current(ctx)
    trials = []

    def measure(params):
        apply(ctx, params)
        ts = sorted(run() for _ in range(repeats))
        t = ts[len(ts) // 2]
        trials.append({"params": dict(params), "seconds": t, "runs": ts})
        if log:
            log(f"[autotune] {params} -> {t * 1e3:.2f} ms")
        return t, ts[-1] - ts[0]

    default_t, spread = measure(best)
    best_t = default_t
    for name, values in space.items():
        for v in values:
            if best.get(name) == v:
                continue
            cand = dict(best)
            cand[name] = v
            t, _ = measure(cand)
            if t < best_t - spread:
                best, best_t = cand, t
    apply(ctx, best)
    stats = {"default_s": default_t, "best_s": best_t, "spread_s": spread,
             "gain": default_t / best_t if best_t else 1.0}
    return best, trials, stats
