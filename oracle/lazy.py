"""Oracle of the on-demand (lazy) restore's fetch rule -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module; the product never does.

Section 4.2 (the HYPRE discussion) describes how the application's copy of a
unified-memory region is filled on read faults: a small region is read whole
at its first fault; in a large region the first fault reads only the page
that holds the faulting address, and every later fault of the same region
reads twice as many pages as the fault before it (1, 2, 4, ... pages),
relying on spatial locality.

Restated for restoring a delta image: the pages packed in the image are
"absent" until fetched; every other page already holds its bytes.  An access
(region, byte offset, length) faults when one of the pages it covers is an
absent image page.  The fault starts at the first such page (the faulting
address, the lowest one the access reaches), and its window is
max(2^f, pages up to the end of the access) pages long, where f counts the
region's earlier faults, clipped at the region's end; a small region's window
is the whole region.  Every image page in the window is fetched.  An access
that finds nothing absent is not a fault.  Finishing fetches what is left.

Readings where the paper is silent: "small" means at most ``small_bytes``
bytes; the window reaches at least to the end of the access, so one access
never takes two faults; the counter never resets.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Set, Tuple


class LazyModel:
    """region_bytes: lengths of the regions in table order (multiples of
    page_size); image_pages: global page numbers packed in the image (pages
    numbered across regions in table order)."""

    def __init__(self, region_bytes: Sequence[int], page_size: int, image_pages,
                 small_bytes: int):
        self.P = page_size
        self.n_pages = [b // page_size for b in region_bytes]
        self.region_bytes = list(region_bytes)
        self.first: List[int] = []
        g = 0
        for n in self.n_pages:
            self.first.append(g)
            g += n
        self.image: Set[int] = set(int(x) for x in image_pages)
        self.small_bytes = small_bytes
        self.fetched: Set[int] = set()
        self.faults: Dict[int, int] = {}
        self.windows: List[Tuple[int, int, int]] = []  # (region, first page, end page)

    def touch(self, region: int, offset: int, length: int) -> int:
        """Apply one access; returns the number of pages it fetched."""
        assert length > 0 and 0 <= offset and offset + length <= self.region_bytes[region]
        base = self.first[region]
        lo = base + offset // self.P
        hi = base + (offset + length - 1) // self.P + 1  # one past the last page
        absent = [g for g in range(lo, hi) if g in self.image and g not in self.fetched]
        if not absent:
            return 0
        f = self.faults.get(region, 0)
        end_of_region = base + self.n_pages[region]
        if self.region_bytes[region] <= self.small_bytes:
            w0, w1 = base, end_of_region
        else:
            w0 = absent[0]
            w1 = min(max(w0 + (1 << f), hi), end_of_region)
        new = [g for g in range(w0, w1) if g in self.image and g not in self.fetched]
        self.fetched.update(new)
        self.faults[region] = f + 1
        self.windows.append((region, w0, w1))
        return len(new)

    def finish(self) -> int:
        new = self.image - self.fetched
        self.fetched |= new
        return len(new)

    def fetched_bitmap(self, total_pages: int):
        """The fetched set as 64-bit words (bit g % 64 of word g // 64)."""
        words = [0] * ((total_pages + 63) // 64)
        for g in self.fetched:
            words[g >> 6] |= 1 << (g & 63)
        return words
