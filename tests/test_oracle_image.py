"""Image format pins: round trip, every single-bit flip in the metadata is
caught by meta_crc, the CRC array by crcs_crc, pads and lengths by the parser,
and page corruption by per-page CRC verification at restore."""
import struct

import numpy as np
import pytest

import oracle

P = 4096


def _regs(counts, dirty, seed=0):
    rng = np.random.default_rng(seed)
    regs = []
    g = 0
    for rid, n in enumerate(counts):
        cur = rng.integers(0, 256, n * P, dtype=np.uint8)
        sh = cur.copy()
        for i in range(n):
            if g + i in dirty:
                sh[i * P + int(rng.integers(0, P))] ^= np.uint8(0x5A)
        g += n
        regs.append((cur, sh, 77 + 3 * rid))
    return regs


def _img(counts=(3, 4), dirty=(0, 2, 5), seq=99):
    regs = _regs(counts, set(dirty))
    st, img, bm = oracle.snapshot(regs, P, seq=seq)
    assert st.code == oracle.OK
    return regs, st, img


def test_round_trip_header_fields():
    regs, st, img = _img()
    rc, h = oracle.parse(img)
    assert rc == oracle.OK
    assert img[:8].tobytes() == b"CRUMIMG1"
    assert h["version"] == 1 and h["page_size"] == P and h["n_regions"] == 2
    assert h["total_pages"] == 7 and h["n_dirty"] == 3 and h["seq"] == 99
    assert h["data_off"] == 4096 and h["flags"] == 0
    assert len(img) == 4096 + 3 * P + 16  # 3 CRCs = 12 bytes, padded to 16
    table = struct.unpack_from("<8Q", img.tobytes(), 64)
    assert table == (77, 3 * P, 0, 0, 80, 4 * P, 3, 0)
    (word,) = struct.unpack_from("<Q", img.tobytes(), 128)
    assert word == 0b100101
    # packed pages are the current bytes of global pages 0, 2, 5 (region 1 page 2)
    pages = [regs[0][0][0:P], regs[0][0][2 * P:3 * P], regs[1][0][2 * P:3 * P]]
    for k, pg in enumerate(pages):
        assert np.array_equal(img[4096 + k * P:4096 + (k + 1) * P], pg)
        (c,) = struct.unpack_from("<I", img.tobytes(), 4096 + 3 * P + 4 * k)
        assert c == oracle.crc32c(pg)


def test_every_metadata_bit_flip_is_detected():
    _, _, img = _img()
    prefix_end = 64 + 32 * 2 + 8 * 1
    for byte in range(prefix_end):
        for bit in range(8):
            bad = img.copy()
            bad[byte] ^= np.uint8(1 << bit)
            rc, _ = oracle.parse(bad)
            assert rc == oracle.EFORMAT, (byte, bit)


def test_pad_and_crc_array_flips_are_detected():
    _, st, img = _img()
    D = st.n_dirty
    crc_start = 4096 + D * P
    for pos in [200, 1000, 4095, crc_start, crc_start + 5, crc_start + 4 * D, len(img) - 1]:
        bad = img.copy()
        bad[pos] ^= np.uint8(0x10)
        assert oracle.parse(bad)[0] == oracle.EFORMAT, pos


def test_truncated_or_extended_image_rejected():
    _, _, img = _img()
    for n in [0, 8, 63, 64, 4095, 4096, len(img) - 1]:
        assert oracle.parse(img[:n])[0] == oracle.EFORMAT, n
    longer = np.concatenate([img, np.zeros(8, np.uint8)])
    assert oracle.parse(longer)[0] == oracle.EFORMAT


def test_page_corruption_found_by_verify_only():
    regs, st, img = _img()
    for k in range(st.n_dirty):
        bad = img.copy()
        bad[4096 + k * P + 17] ^= np.uint8(1)
        assert oracle.parse(bad)[0] == oracle.OK  # pages are not in meta_crc
        dst = [(s.copy(), None, rid) for _, s, rid in regs]
        before = [d.copy() for d, _, _ in dst]
        res = oracle.restore(dst, bad, flags=oracle.VERIFY)
        assert res.code == oracle.ECRC and res.first_bad == k
        for (d, _, _), b in zip(dst, before):
            assert np.array_equal(d, b)  # nothing written
        # without VERIFY the corrupt page is written as is
        res = oracle.restore(dst, bad, flags=0)
        assert res.code == oracle.OK


def test_lowest_bad_slot_reported():
    regs, st, img = _img(dirty=(0, 1, 2, 3, 4, 5, 6))
    bad = img.copy()
    for k in (5, 2, 6):
        bad[4096 + k * P] ^= np.uint8(0x80)
    res = oracle.restore([(s.copy(), None, rid) for _, s, rid in regs], bad, oracle.VERIFY)
    assert res.code == oracle.ECRC and res.first_bad == 2


def test_restore_table_mismatch():
    regs, _, img = _img()
    dst = [(s.copy(), None, rid) for _, s, rid in regs]
    assert oracle.restore(dst[:1], img).code == oracle.EMISMATCH
    wrong_id = [dst[0], (dst[1][0], None, 12345)]
    assert oracle.restore(wrong_id, img).code == oracle.EMISMATCH
    wrong_len = [dst[0], (dst[1][0][:P], None, dst[1][2])]
    assert oracle.restore(wrong_len, img).code == oracle.EMISMATCH


@pytest.mark.parametrize("G", [0, 1, 63, 64, 65, 500])
def test_prefix_bytes(G):
    for R in [0, 1, 5, 200]:
        assert oracle.prefix_bytes(R, G) == -(-(64 + 32 * R + 8 * (-(-G // 64))) // 4096) * 4096
