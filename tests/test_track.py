"""Host write tracking (paper section 3.2, Algorithm 1): CPU tests of the
tracker behind crum_track_*: a new view is all dirty, a write to a clean page
faults once and marks it dirty, reads never do, a flush copies exactly the
dirty pages and clears them, the pending set collects flushed pages until it
is cleared, and writes racing with a flush are never lost."""
import ctypes
import subprocess
import sys
import threading

import numpy as np
import pytest

import paper_1808_00117_amd as crum

P = 4096


def bits_to_pages(words):
    return np.flatnonzero(np.unpackbits(np.asarray(words, np.uint64).view(np.uint8),
                                        bitorder="little"))


@pytest.fixture
def tracker():
    t = crum.Tracker(37 * P, P)
    yield t
    t.destroy()


def test_new_view_is_all_dirty_and_writable(tracker):
    st = tracker.stats()
    assert st["pages"] == 37 and st["dirty_pages"] == 37 and st["pending_pages"] == 0
    v = tracker.view()
    v[:] = 7  # every page writable: no fault
    assert tracker.stats()["faults"] == 0
    assert list(bits_to_pages(tracker.dirty())) == list(range(37))


def test_flush_copies_dirty_pages_and_clears_them(tracker):
    v = tracker.view()
    v[:] = np.arange(v.size, dtype=np.uint64).astype(np.uint8)
    dst = np.zeros(v.size, np.uint8)
    assert tracker.flush(dst.ctypes.data, 2) == 37
    assert np.array_equal(dst, v)
    st = tracker.stats()
    assert st["dirty_pages"] == 0 and st["pending_pages"] == 37 and st["flushed_pages"] == 37
    assert list(bits_to_pages(tracker.pending(clear=True))) == list(range(37))
    assert tracker.stats()["pending_pages"] == 0
    # nothing dirty: a flush copies nothing
    dst[:] = 0
    assert tracker.flush(dst.ctypes.data) == 0
    assert not dst.any()


def test_write_to_clean_page_faults_once_and_marks_it(tracker):
    v = tracker.view()
    dst = np.zeros(v.size, np.uint8)
    tracker.flush(dst.ctypes.data)
    tracker.pending(clear=True)
    f0 = tracker.stats()["faults"]
    v[3 * P + 100] = 1          # first write: one fault
    v[3 * P + 200: 3 * P + 300] = 2
    v[20 * P + P - 1] = 3
    assert tracker.stats()["faults"] == f0 + 2
    assert list(bits_to_pages(tracker.dirty())) == [3, 20]
    assert tracker.flush(dst.ctypes.data) == 2
    assert np.array_equal(dst, v)
    assert list(bits_to_pages(tracker.pending())) == [3, 20]


def test_reads_do_not_mark_pages(tracker):
    v = tracker.view()
    dst = np.zeros(v.size, np.uint8)
    tracker.flush(dst.ctypes.data)
    f0 = tracker.stats()["faults"]
    s = int(v.sum()) + int(v[5 * P])
    assert s >= 0
    assert tracker.stats()["faults"] == f0 and tracker.stats()["dirty_pages"] == 0


def test_read_then_write_is_dirty(tracker):
    v = tracker.view()
    dst = np.zeros(v.size, np.uint8)
    tracker.flush(dst.ctypes.data)
    tracker.pending(clear=True)
    x = int(v[9 * P + 5])
    v[9 * P + 5] = (x + 1) & 255
    assert list(bits_to_pages(tracker.dirty())) == [9]
    tracker.flush(dst.ctypes.data)
    assert dst[9 * P + 5] == (x + 1) & 255


def test_pending_accumulates_over_flushes_until_cleared(tracker):
    v = tracker.view()
    dst = np.zeros(v.size, np.uint8)
    tracker.flush(dst.ctypes.data)
    tracker.pending(clear=True)
    v[P] = 1
    tracker.flush(dst.ctypes.data)
    v[30 * P] = 1
    tracker.flush(dst.ctypes.data)
    assert list(bits_to_pages(tracker.pending())) == [1, 30]
    assert list(bits_to_pages(tracker.pending(clear=True))) == [1, 30]
    assert len(bits_to_pages(tracker.pending())) == 0


def test_writes_racing_with_flushes_are_not_lost():
    """Writer threads store into random pages while flushes run: after the
    writers stop and a last flush, the real region equals the view."""
    n = 512
    t = crum.Tracker(n * P, P)
    try:
        v = t.view()
        dst = np.zeros(v.size, np.uint8)
        t.flush(dst.ctypes.data, 4)
        stop = threading.Event()

        def writer(seed):
            rng = np.random.default_rng(seed)
            while not stop.is_set():
                p = int(rng.integers(0, n))
                o = int(rng.integers(0, P - 64))
                v[p * P + o: p * P + o + 64] = rng.integers(0, 256, 64, dtype=np.uint8)

        ths = [threading.Thread(target=writer, args=(s,)) for s in range(4)]
        for th in ths:
            th.start()
        for _ in range(50):
            t.flush(dst.ctypes.data, 4)
        stop.set()
        for th in ths:
            th.join()
        t.flush(dst.ctypes.data, 4)
        assert np.array_equal(dst, v)
        assert t.stats()["dirty_pages"] == 0
    finally:
        t.destroy()


def test_two_trackers_and_large_pages():
    a = crum.Tracker(8 * P, P)
    b = crum.Tracker(4 * (64 << 10), 64 << 10)
    try:
        da, db = np.zeros(a.nbytes, np.uint8), np.zeros(b.nbytes, np.uint8)
        a.flush(da.ctypes.data)
        b.flush(db.ctypes.data)
        a.view()[2 * P] = 9
        b.view()[(64 << 10) * 3 + 17] = 9
        assert list(bits_to_pages(a.dirty())) == [2]
        assert list(bits_to_pages(b.dirty())) == [3]
    finally:
        a.destroy()
        b.destroy()


def test_argument_errors():
    L = crum.lib()
    h = ctypes.c_void_p()
    E = crum.CRUM_EINVAL
    assert L.crum_track_create(3 * P, 3000, ctypes.byref(h)) == E      # not a power of two
    assert L.crum_track_create(3 * P + 1, P, ctypes.byref(h)) == E     # not whole pages
    assert L.crum_track_create(0, P, ctypes.byref(h)) == E
    assert L.crum_track_create(P, P, None) == E
    assert L.crum_track_flush(None, None, 1, None) == E
    t = crum.Tracker(P, P)
    try:
        assert L.crum_track_flush(t.handle, None, 1, None) == E
        d = np.zeros(P, np.uint8)
        assert L.crum_track_flush(t.handle, d.ctypes.data, 0, None) == E
        assert L.crum_track_pending(t.handle, None, 1, 0) == E
    finally:
        t.destroy()


def test_faults_outside_views_still_crash():
    """The handler passes faults it does not own on: a process that reads an
    unmapped address after creating a tracker still dies of SIGSEGV."""
    code = ("import ctypes, paper_1808_00117_amd as crum\n"
            "t = crum.Tracker(4096, 4096)\n"
            "ctypes.string_at(8)\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, timeout=120,
                       cwd=crum.__path__[0] + "/..")
    assert r.returncode == -11, (r.returncode, r.stderr[-500:])
