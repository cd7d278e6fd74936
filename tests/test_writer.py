"""The image writer (host code, no GPU): the file holds exactly the bytes of
the buffer for every size, alignment, chunking and flag combination, several
writes may be in flight at once, and failures are reported with errno."""
import ctypes
import os

import numpy as np
import pytest

import oracle

KiB, MiB = 1 << 10, 1 << 20


def aligned(nbytes: int, offset: int = 0, seed: int = 0):
    """Random bytes in a buffer whose data starts `offset` bytes past a 4 KiB
    boundary (keeps the owning array alive with the view)."""
    raw = np.empty(nbytes + 2 * 4096, np.uint8)
    start = (-raw.ctypes.data) % 4096 + offset
    v = raw[start:start + nbytes]
    v[:] = np.random.default_rng(seed).integers(0, 256, nbytes, dtype=np.uint8)
    return raw, v


@pytest.fixture(scope="module")
def crum():
    import paper_1808_00117_amd as crum
    crum.lib()
    return crum


@pytest.mark.parametrize("nbytes", [0, 1, 4095, 4096, 4097, 3 * MiB + 123, 8 * MiB])
@pytest.mark.parametrize("flags", [0, 1, 2, 3])
def test_file_equals_buffer(crum, tmp_path, nbytes, flags):
    w = crum.Writer(n_threads=3, chunk_bytes=1 * MiB, flags=flags)
    try:
        _, buf = aligned(nbytes, seed=nbytes + flags)
        path = tmp_path / f"img_{nbytes}_{flags}.bin"
        t = w.submit(str(path), buf.ctypes.data, nbytes)
        st = w.poll(t)
        assert st["code"] == crum.CRUM_OK and st["err"] == 0 and st["bytes"] == nbytes
        assert st["seconds"] >= 0
        assert np.array_equal(np.fromfile(path, np.uint8), buf)
    finally:
        w.destroy()


def test_unaligned_buffer_and_small_chunks(crum, tmp_path):
    """A buffer off the 4 KiB grid never uses the direct descriptor; chunks
    of one page each land at their offsets."""
    w = crum.Writer(n_threads=4, chunk_bytes=4 * KiB, flags=crum.CRUM_WRITE_DIRECT)
    try:
        _, buf = aligned(100 * KiB + 7, offset=8, seed=3)
        path = tmp_path / "u.bin"
        st = w.poll(w.submit(str(path), buf.ctypes.data, buf.size))
        assert st["code"] == 0 and st["direct"] == 0
        assert np.array_equal(np.fromfile(path, np.uint8), buf)
    finally:
        w.destroy()


def test_many_writes_in_flight(crum, tmp_path):
    w = crum.Writer(n_threads=4, chunk_bytes=64 * KiB, flags=crum.CRUM_WRITE_SYNC)
    try:
        bufs, tickets = [], []
        for i in range(12):
            raw, b = aligned(200 * KiB + 4096 * i + (i % 3), seed=100 + i)
            bufs.append((raw, b))
            tickets.append(w.submit(str(tmp_path / f"m{i}.bin"), b.ctypes.data, b.size))
        # collect out of order; a collected ticket is forgotten
        for i in reversed(range(12)):
            st = w.poll(tickets[i])
            assert st["code"] == 0 and st["bytes"] == bufs[i][1].size
            assert np.array_equal(np.fromfile(tmp_path / f"m{i}.bin", np.uint8), bufs[i][1])
        with pytest.raises(ValueError):
            w.poll(tickets[0])
    finally:
        w.destroy()


def test_poll_without_wait(crum, tmp_path):
    w = crum.Writer(n_threads=1, chunk_bytes=1 * MiB, flags=0)
    try:
        _, b = aligned(32 * MiB, seed=9)
        t = w.submit(str(tmp_path / "nw.bin"), b.ctypes.data, b.size)
        st = None
        for _ in range(100000):
            st = w.poll(t, wait=False)
            if st is not None:
                break
        if st is None:
            st = w.poll(t)
        assert st["code"] == 0 and st["bytes"] == b.size
    finally:
        w.destroy()


def test_oracle_image_round_trip(crum, tmp_path):
    """An image made by the oracle, persisted and read back, still parses."""
    rng = np.random.default_rng(5)
    P = 4 * KiB
    cur = rng.integers(0, 256, 40 * P, dtype=np.uint8)
    sh = cur.copy()
    sh[::3 * P] ^= 1
    st, img, _ = oracle.snapshot([(cur, sh, 9)], P, seq=4)
    raw, b = aligned(img.size)
    b[:] = img
    w = crum.Writer()
    try:
        path = tmp_path / "img.crum"
        assert w.poll(w.submit(str(path), b.ctypes.data, b.size))["code"] == 0
        back = np.fromfile(path, np.uint8)
        rc, hdr = oracle.parse(back)
        assert rc == oracle.OK and hdr["n_dirty"] == st.n_dirty and np.array_equal(back, img)
    finally:
        w.destroy()


def test_errors(crum, tmp_path):
    lib = crum.lib()
    h = ctypes.c_void_p()
    for n, c, f in [(0, MiB, 0), (1, 0, 0), (1, 1000, 0), (1, MiB, 4), (300, MiB, 0)]:
        assert lib.crum_writer_create(n, c, f, ctypes.byref(h)) == crum.CRUM_EINVAL
    w = crum.Writer(n_threads=2)
    try:
        _, b = aligned(4096)
        with pytest.raises(OSError):
            w.submit(str(tmp_path / "missing_dir" / "x.bin"), b.ctypes.data, b.size)
        t = ctypes.c_uint64()
        assert lib.crum_writer_submit(w.handle, None, b.ctypes.data, 1, ctypes.byref(t)) == \
            crum.CRUM_EINVAL
        assert lib.crum_writer_submit(w.handle, os.fsencode(str(tmp_path / "n.bin")), None, 5,
                                      ctypes.byref(t)) == crum.CRUM_EINVAL
        with pytest.raises(ValueError):
            w.poll(12345)
    finally:
        w.destroy()


def test_overwrite_shorter_and_longer(crum, tmp_path):
    """Writing over an existing file leaves exactly the new bytes, whether
    the new image is shorter or longer than the old file."""
    w = crum.Writer(n_threads=2, chunk_bytes=64 * KiB, flags=crum.CRUM_WRITE_SYNC)
    try:
        path = tmp_path / "over.bin"
        for n, seed in [(300 * KiB + 5, 1), (100 * KiB + 3, 2), (500 * KiB, 3), (0, 4),
                        (7, 5)]:
            _, b = aligned(n, seed=seed)
            assert w.poll(w.submit(str(path), b.ctypes.data, n))["code"] == 0
            assert np.array_equal(np.fromfile(path, np.uint8), b)
    finally:
        w.destroy()
