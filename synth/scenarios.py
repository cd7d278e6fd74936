"""Seeded scenario descriptions for the snapshot workloads.

A scenario lists regions (size, generator stream) and, per region, the pages
whose *shadow* is mutated; the current bytes are always pure generator output,
so the exact dirty set is the chosen page set by construction (every mutation
changes at least one byte).  All choices come from
``numpy.random.Generator(PCG64(seed))``.

Workloads (sizes as the benchmark configurations state them):

* :func:`plain`        -- one 64 MiB allocation, 4 KiB pages, exactly 5 % of
                          pages mutated (1-16 words each).
* :func:`many_allocs`  -- 64 allocations, log-uniform 4 KiB-1 GiB, scaled by
                          one common factor to 16 GiB total, 64 KiB pages;
                          clustered dirty runs (start Bernoulli(0.003), length
                          geometric with mean 32).
* :func:`managed`      -- one 32 GiB region, 2 MiB pages, 30 % of pages
                          device-resident, 20 % of pages with a 256-byte span
                          rewritten.
* :func:`batched`      -- 256 requests of 1-32 allocations, request totals
                          log-uniform 1 MiB-2 GiB, 4 KiB or 64 KiB pages,
                          dirty fraction U(1 %, 50 %) in clustered runs
                          (geometric mean 16).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

KiB, MiB, GiB = 1 << 10, 1 << 20, 1 << 30

MUT_WORDS = 0
MUT_SPAN = 1


@dataclass
class RegionSpec:
    id: int
    nbytes: int
    fill_seed: int
    fill_region: int
    dirty_pages: np.ndarray          # sorted int64 page indices whose shadow differs
    mut_kind: int = MUT_WORDS
    has_shadow: bool = True


@dataclass
class Scenario:
    name: str
    seed: int
    page_size: int
    mut_seed: int
    regions: List[RegionSpec]
    meta: Dict = field(default_factory=dict)

    @property
    def total_bytes(self) -> int:
        return sum(r.nbytes for r in self.regions)

    @property
    def total_pages(self) -> int:
        return sum(r.nbytes // self.page_size for r in self.regions)

    @property
    def n_dirty(self) -> int:
        return sum(int(r.dirty_pages.size) if r.has_shadow else r.nbytes // self.page_size
                   for r in self.regions)

    def dirty_global(self) -> np.ndarray:
        """Expected dirty set as sorted global page indices (table order)."""
        out = []
        g = 0
        for r in self.regions:
            n = r.nbytes // self.page_size
            if r.has_shadow:
                out.append(g + r.dirty_pages)
            else:
                out.append(g + np.arange(n, dtype=np.int64))
            g += n
        return np.concatenate(out) if out else np.zeros(0, np.int64)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def clustered_runs(rng: np.random.Generator, n_pages: int, start_p: float,
                   mean_len: float) -> np.ndarray:
    """Union of runs: each page starts a run with probability start_p; run
    lengths are geometric (support >= 1) with the given mean; runs are cut at
    the region end.  Returns sorted unique page indices."""
    if n_pages == 0:
        return np.zeros(0, np.int64)
    starts = np.flatnonzero(rng.random(n_pages) < start_p)
    if starts.size == 0:
        return np.zeros(0, np.int64)
    lens = rng.geometric(1.0 / mean_len, size=starts.size)
    # mark [start, start+len) on a difference array
    diff = np.zeros(n_pages + 1, np.int64)
    np.add.at(diff, starts, 1)
    np.add.at(diff, np.minimum(starts + lens, n_pages), -1)
    return np.flatnonzero(np.cumsum(diff[:-1]) > 0).astype(np.int64)


def plain(seed: int = 1001, nbytes: int = 64 * MiB, page_size: int = 4 * KiB,
          frac: float = 0.05) -> Scenario:
    rng = _rng(seed)
    G = nbytes // page_size
    n_dirty = int(round(frac * G))
    pages = np.sort(rng.choice(G, size=n_dirty, replace=False)).astype(np.int64)
    reg = RegionSpec(id=1, nbytes=nbytes, fill_seed=seed, fill_region=0, dirty_pages=pages)
    return Scenario("plain", seed, page_size, seed + 7919, [reg],
                    {"frac": frac})


def many_allocs(seed: int = 1002, n: int = 64, page_size: int = 64 * KiB,
                total: Optional[int] = 16 * GiB, start_p: float = 0.003,
                mean_run: float = 32.0) -> Scenario:
    """64 allocations log-uniform in 4 KiB-1 GiB.  With `total`, the draws are
    scaled by one common factor so the sizes sum to exactly `total` bytes (each
    rounded to whole pages, the largest one absorbing the rounding)."""
    rng = _rng(seed)
    raw = np.exp2(12 + 18 * rng.random(n))
    if total is None:
        sizes = np.maximum(1, np.ceil(raw / page_size)).astype(np.int64) * page_size
    else:
        assert total % page_size == 0
        scaled = raw * (total / raw.sum())
        pages = np.maximum(1, np.round(scaled / page_size)).astype(np.int64)
        pages[np.argmax(pages)] += total // page_size - pages.sum()
        assert pages.min() >= 1
        sizes = pages * page_size
    regs = []
    for i, sz in enumerate(sizes):
        dp = clustered_runs(rng, int(sz) // page_size, start_p, mean_run)
        regs.append(RegionSpec(id=100 + i, nbytes=int(sz), fill_seed=seed, fill_region=i,
                               dirty_pages=dp))
    return Scenario("many_allocs", seed, page_size, seed + 7919, regs,
                    {"scaled_total": total})


def managed(seed: int = 1003, nbytes: int = 32 * GiB, page_size: int = 2 * MiB,
            device_frac: float = 0.30, dirty_frac: float = 0.20) -> Scenario:
    rng = _rng(seed)
    G = nbytes // page_size
    n_dev = int(round(device_frac * G))
    dev_pages = np.sort(rng.choice(G, size=n_dev, replace=False)).astype(np.int64)
    n_dirty = int(round(dirty_frac * G))
    dirty = np.sort(rng.choice(G, size=n_dirty, replace=False)).astype(np.int64)
    reg = RegionSpec(id=7, nbytes=nbytes, fill_seed=seed, fill_region=0, dirty_pages=dirty,
                     mut_kind=MUT_SPAN)
    return Scenario("managed", seed, page_size, seed + 7919, [reg],
                    {"device_pages": dev_pages})


def batched(seed: int = 1004, n_requests: int = 256, min_total: int = 1 * MiB,
            max_total: int = 2 * GiB, max_allocs: int = 32, mean_run: float = 16.0,
            frac_lo: float = 0.01, frac_hi: float = 0.50) -> List[Scenario]:
    """Per request: page size 4 KiB or 64 KiB (p = 0.5), k ~ U{1..max_allocs}
    allocations, a request total log-uniform in [min_total, max_total] split at
    uniform page-aligned cut points (k reduced when there are fewer pages),
    dirty fraction f ~ U(frac_lo, frac_hi) in runs with start probability
    -ln(1-f)/mean_run and geometric lengths of mean `mean_run`."""
    rng = _rng(seed)
    out = []
    for q in range(n_requests):
        P = 4 * KiB if rng.random() < 0.5 else 64 * KiB
        k = int(rng.integers(1, max_allocs + 1))
        lo, hi = math.log2(min_total), math.log2(max_total)
        tot = 2.0 ** (lo + (hi - lo) * rng.random())
        n_pages = max(1, int(round(tot / P)))
        k = min(k, n_pages)
        cuts = np.sort(rng.choice(np.arange(1, n_pages), size=k - 1, replace=False)) \
            if k > 1 else np.zeros(0, np.int64)
        bounds = np.concatenate([[0], cuts, [n_pages]]).astype(np.int64)
        f = frac_lo + (frac_hi - frac_lo) * rng.random()
        start_p = -math.log(1.0 - f) / mean_run
        regs = []
        for i in range(k):
            npg = int(bounds[i + 1] - bounds[i])
            dp = clustered_runs(rng, npg, start_p, mean_run)
            regs.append(RegionSpec(id=q * 64 + i, nbytes=npg * P, fill_seed=seed,
                                   fill_region=q * 64 + i, dirty_pages=dp))
        out.append(Scenario(f"batched[{q}]", seed, P, seed + 7919 + q, regs,
                            {"request": q, "dirty_frac": f}))
    return out


def materialize_host(scn: Scenario, index: int, shadow: bool = True):
    """Host copies (current, shadow-or-None) of one region, as uint8 arrays."""
    from .lib import fill_host, mutate_host
    r = scn.regions[index]
    cur = fill_host(r.nbytes, r.fill_seed, r.fill_region)
    if not (shadow and r.has_shadow):
        return cur, None
    sh = cur.copy()
    mutate_host(sh, scn.page_size, r.dirty_pages, r.mut_kind, scn.mut_seed, r.fill_region)
    return cur, sh


def host_page(scn: Scenario, index: int, page: int, shadow: bool):
    """One page of a region, regenerated on the host without the whole region."""
    from .lib import fill_host, mutate_host
    r = scn.regions[index]
    P = scn.page_size
    buf = fill_host(P, r.fill_seed, r.fill_region, byte_off=page * P)
    if shadow and r.has_shadow:
        pos = np.searchsorted(r.dirty_pages, page)
        if pos < r.dirty_pages.size and r.dirty_pages[pos] == page:
            # mutate a one-page view: the rule depends on the page index only
            tmp = np.zeros(P, np.uint8)
            tmp[:] = buf
            _mutate_one(tmp, P, page, r.mut_kind, scn.mut_seed, r.fill_region)
            buf = tmp
    return buf


def _mutate_one(page_buf: np.ndarray, P: int, page: int, kind: int, ms: int, region: int):
    from .lib import host_lib
    host_lib().synth_mutate_page_host(page_buf.ctypes.data, P, kind, ms, region, page)


def served_clients(seed: int = 1005, n_clients: int = 32, min_bytes: int = 64 * MiB,
                   max_bytes: int = 8 * GiB, page_size: int = 64 * KiB,
                   cap_total: int = 120 * GiB) -> List[int]:
    """Client state sizes: log-uniform in [min_bytes, max_bytes], rounded up to
    whole pages; the draw is repeated if the total exceeds cap_total."""
    rng = _rng(seed)
    lo, hi = math.log2(min_bytes), math.log2(max_bytes)
    while True:
        raw = np.exp2(lo + (hi - lo) * rng.random(n_clients))
        sizes = [int(math.ceil(x / page_size)) * page_size for x in raw]
        if sum(sizes) <= cap_total:
            return sizes


def served_trace(seed: int = 1005, n_clients: int = 32, rate: float = 200.0,
                 duration: float = 60.0, snapshot_share: float = 0.8,
                 frac_lo: float = 0.02, frac_hi: float = 0.30):
    """Open-loop Poisson arrivals at `rate` requests/s over `duration` s; each
    request picks a client uniformly and is a snapshot with probability
    `snapshot_share` (4:1), else a restore; snapshots carry the fraction of the
    client's pages changed before them, U(frac_lo, frac_hi).
    Returns a list of (arrival_s, client, kind, frac) with kind 1 snapshot,
    2 restore."""
    rng = _rng(seed + 17)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            return out
        c = int(rng.integers(0, n_clients))
        snap = rng.random() < snapshot_share
        f = float(frac_lo + (frac_hi - frac_lo) * rng.random()) if snap else 0.0
        out.append((t, c, 1 if snap else 2, f))
