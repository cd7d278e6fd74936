"""Pure-Python brute force for tiny snapshot images -- TEST INFRASTRUCTURE.

Independent of ``crum_oracle.c`` (no shared code, tables or constants beyond
the published CRC-32C polynomial and the image layout definition).  Used only
on inputs of a few pages to pin the C oracle:

* CRC-32C by the bit-at-a-time rule (reflected polynomial 0x82F63B78, init and
  final XOR 0xFFFFFFFF), no table;
* dirty test by ``bytes`` equality, with a missing shadow meaning every page
  is dirty (the paper's shadow regions start with every page dirty, section
  3.2);
* compaction by walking pages in global order;
* the image written field by field with ``struct``;
* restore by the same walk in reverse.
"""
from __future__ import annotations

import struct
from functools import lru_cache
from typing import List, Optional, Sequence, Tuple

POLY_REFLECTED = 0x82F63B78


@lru_cache(maxsize=65536)
def crc32c_bitwise(data: bytes) -> int:
    c = 0xFFFFFFFF
    for b in data:
        c ^= b
        for _ in range(8):
            if c & 1:
                c = (c >> 1) ^ POLY_REFLECTED
            else:
                c >>= 1
    return c ^ 0xFFFFFFFF


def _ceil_div(a: int, b: int) -> int:
    return -(-a // b)


def _round_up(a: int, b: int) -> int:
    return _ceil_div(a, b) * b


def snapshot(regions: Sequence[Tuple[bytes, Optional[bytes], int]], page_size: int,
             seq: int = 0) -> Tuple[bytes, List[int]]:
    """regions: (current bytes, shadow bytes or None, id).  Returns (image, dirty g list)."""
    P = page_size
    dirty_g: List[int] = []
    pages: List[bytes] = []
    table = []
    g = 0
    for cur, shadow, rid in regions:
        n = len(cur) // P
        table.append((rid, len(cur), g))
        for i in range(n):
            page = bytes(cur[i * P:(i + 1) * P])
            if shadow is None or page != bytes(shadow[i * P:(i + 1) * P]):
                dirty_g.append(g)
                pages.append(page)
            g += 1
    G = g
    D = len(pages)
    R = len(regions)
    W = _ceil_div(G, 64)
    words = [0] * W
    for gg in dirty_g:
        words[gg // 64] |= 1 << (gg % 64)
    prefix_end = 64 + 32 * R + 8 * W
    data_off = _round_up(prefix_end, 4096)
    crcs = b"".join(struct.pack("<I", crc32c_bitwise(p)) for p in pages)
    crcs_crc = crc32c_bitwise(crcs)
    base_flag = 1 if all(sh is None for _, sh, _ in regions) else 0

    def header(meta_crc: int) -> bytes:
        h = b"CRUMIMG1" + struct.pack("<IIII", 1, P, R, base_flag)
        h += struct.pack("<QQQQ", G, D, seq, data_off)
        h += struct.pack("<II", meta_crc, crcs_crc)
        for rid, ln, first in table:
            h += struct.pack("<QQQQ", rid, ln, first, 0)
        for w in words:
            h += struct.pack("<Q", w)
        return h

    meta_crc = crc32c_bitwise(header(0))
    meta = header(meta_crc)
    assert len(meta) == prefix_end
    img = meta + bytes(data_off - prefix_end) + b"".join(pages) + crcs
    img += bytes(_round_up(4 * D, 8) - 4 * D)
    return img, dirty_g


def restore(regions: Sequence[Tuple[bytearray, int]], image: bytes) -> None:
    """Copy packed pages back into the (current bytearray, id) regions."""
    P, R = struct.unpack_from("<II", image, 12)
    G, D, _seq, data_off = struct.unpack_from("<QQQQ", image, 24)
    assert R == len(regions)
    W = _ceil_div(G, 64)
    words = struct.unpack_from("<%dQ" % W, image, 64 + 32 * R) if W else ()
    k = 0
    g = 0
    for cur, _rid in regions:
        for i in range(len(cur) // P):
            if (words[g // 64] >> (g % 64)) & 1:
                cur[i * P:(i + 1) * P] = image[data_off + k * P:data_off + (k + 1) * P]
                k += 1
            g += 1
    assert k == D
