"""Pins of the lazy-restore fetch model (section 4.2's read-fault readahead)
by closed forms and special cases, not by re-running its rule."""
import math

import numpy as np
import pytest

from oracle.lazy import LazyModel

P = 4096


def sweep(model, region, n_pages, step_pages=1):
    fault_pages = []
    for p in range(0, n_pages, step_pages):
        if model.touch(region, p * P, step_pages * P):
            fault_pages.append(p)
    return fault_pages


@pytest.mark.parametrize("n", [1, 2, 3, 7, 8, 100, 1000, 4097])
def test_sequential_sweep_faults_at_powers_of_two(n):
    """A page-by-page sweep of an all-image region: after k faults the first
    1 + 2 + ... + 2^(k-1) = 2^k - 1 pages are present, so faults happen at
    pages 2^k - 1 and there are ceil(log2(n + 1)) of them."""
    m = LazyModel([n * P], P, range(n), small_bytes=0)
    faults = sweep(m, 0, n)
    assert faults == [(1 << k) - 1 for k in range(len(faults))]
    assert len(faults) == math.ceil(math.log2(n + 1))
    assert m.fetched == set(range(n))


def test_small_region_is_fetched_whole():
    m = LazyModel([16 * P, 64 * P], P, range(80), small_bytes=16 * P)
    assert m.touch(0, 5 * P + 17, 1) == 16
    assert m.fetched == set(range(16))
    assert sweep(m, 0, 16) == []          # nothing left to fault on
    assert m.touch(1, 0, 1) == 1          # the larger region starts at one page
    assert m.fetched == set(range(17))


def test_clean_pages_never_fault():
    image = [3, 4, 10]
    m = LazyModel([32 * P], P, image, small_bytes=0)
    assert m.touch(0, 0, 3 * P) == 0      # pages 0..2: none in the image
    assert m.touch(0, 20 * P, 12 * P) == 0
    assert m.fetched == set() and m.faults == {}
    # the first fault starts at page 3 (the lowest absent page reached) and,
    # with 2^0 = 1 page, ends at the access's last page
    assert m.touch(0, 0, 5 * P) == 2
    assert m.fetched == {3, 4}
    # the second fault has a 2-page window starting at page 10
    assert m.touch(0, 10 * P, 1) == 1
    assert m.windows[-1] == (0, 10, 12)


def test_window_clipped_at_region_end_and_counted_per_region():
    m = LazyModel([8 * P, 8 * P], P, range(16), small_bytes=0)
    # interleaved sweeps: each region faults at its own 0, 1, 3, 7
    f0, f1 = [], []
    for p in range(8):
        if m.touch(0, p * P, P):
            f0.append(p)
        if m.touch(1, p * P, P):
            f1.append(p)
    assert f0 == [0, 1, 3, 7] and f1 == [0, 1, 3, 7]
    # region 1's last window (8 pages from page 7) stops at the region's end
    assert (1, 8 + 7, 16) in m.windows


def test_long_access_is_one_fault():
    m = LazyModel([64 * P], P, range(64), small_bytes=0)
    assert m.touch(0, 2 * P + 5, 20 * P) == 21   # pages 2..22
    assert m.faults == {0: 1}
    assert m.touch(0, 40 * P, 1) == 2            # second fault: 2 pages
    assert m.fetched == set(range(2, 23)) | {40, 41}


def test_finish_fetches_the_rest_and_random_touches_cover_their_range():
    rng = np.random.default_rng(7)
    n = [37, 1, 200, 5]
    image = sorted(rng.choice(sum(n), size=120, replace=False).tolist())
    m = LazyModel([k * P for k in n], P, image, small_bytes=5 * P)
    first = np.concatenate([[0], np.cumsum(n)[:-1]])
    before = set()
    for _ in range(200):
        r = int(rng.integers(0, len(n)))
        off = int(rng.integers(0, n[r] * P))
        ln = int(rng.integers(1, n[r] * P - off + 1))
        m.touch(r, off, ln)
        lo, hi = first[r] + off // P, first[r] + (off + ln - 1) // P
        # every image page the access covers is present afterwards
        assert {g for g in image if lo <= g <= hi} <= m.fetched
        assert before <= m.fetched <= set(image)
        before = set(m.fetched)
    m.finish()
    assert m.fetched == set(image)
