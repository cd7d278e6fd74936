"""CPU oracle for the incremental GPU snapshot -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product package never does, and the
two share no code.  Two independent implementations live here:

* ``crum_oracle.c`` (built into ``liboracle.so``): plain, single-threaded C --
  memcmp diff, ascending compaction, byte-table CRC-32C, image v1 serialiser
  and parser, restore.  Wrapped by the functions below.
* ``brute.py``: pure-Python brute force (bitwise CRC-32C, bytes compare,
  ``struct`` image writer) used on tiny inputs to pin the C oracle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ENOSPC, ECRC, EFORMAT, EHIP, EMISMATCH = 0, -1, -2, -3, -4, -5, -6
UPDATE_SHADOW, VERIFY = 1, 2


class _Region(ctypes.Structure):
    _fields_ = [("cur", ctypes.c_void_p), ("shadow", ctypes.c_void_p),
                ("len", ctypes.c_uint64), ("id", ctypes.c_uint64)]


class _Status(ctypes.Structure):
    _fields_ = [("code", ctypes.c_int32), ("first_bad", ctypes.c_uint32),
                ("n_dirty", ctypes.c_uint64), ("total_pages", ctypes.c_uint64),
                ("image_bytes", ctypes.c_uint64)]


class _Header(ctypes.Structure):
    _fields_ = [("version", ctypes.c_uint32), ("page_size", ctypes.c_uint32),
                ("n_regions", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("total_pages", ctypes.c_uint64), ("n_dirty", ctypes.c_uint64),
                ("seq", ctypes.c_uint64), ("data_off", ctypes.c_uint64),
                ("meta_crc", ctypes.c_uint32), ("crcs_crc", ctypes.c_uint32)]


@dataclass
class Status:
    code: int
    first_bad: int
    n_dirty: int
    total_pages: int
    image_bytes: int


_lib = None


def build(verbose: bool = False) -> None:
    """Compile liboracle.so in-tree with gcc (no GPU code)."""
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-fPIC", "-shared", "-o", SO + ".tmp",
           os.path.join(_HERE, "crum_oracle.c")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(SO + ".tmp", SO)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(SO):
            raise RuntimeError(f"{SO} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(SO)
        L.orc_crc32c.restype = ctypes.c_uint32
        L.orc_crc32c.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
        L.orc_validate.restype = ctypes.c_int
        L.orc_validate.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32]
        L.orc_prefix_bytes.restype = ctypes.c_uint64
        L.orc_prefix_bytes.argtypes = [ctypes.c_uint32, ctypes.c_uint64]
        L.orc_snapshot.restype = ctypes.c_int
        L.orc_snapshot.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                   ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                                   ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                   ctypes.c_uint64, ctypes.POINTER(_Status)]
        L.orc_parse.restype = ctypes.c_int
        L.orc_parse.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(_Header)]
        L.orc_snapshot_stream.restype = ctypes.c_int
        L.orc_snapshot_stream.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                          ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                          ctypes.c_uint64, ctypes.POINTER(_Status)]
        L.orc_restore.restype = ctypes.c_int
        L.orc_restore.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                                  ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(_Status)]
        _lib = L
    return _lib


def _buf(a) -> int:
    if a is None:
        return 0
    if isinstance(a, int):
        return a
    assert isinstance(a, np.ndarray) and a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data


def _regions(regions) -> "ctypes.Array":
    """regions: sequence of (cur, shadow_or_None, id) with numpy uint8 buffers,
    or (cur_ptr, shadow_ptr, len, id) tuples of raw host addresses."""
    arr = (_Region * max(1, len(regions)))()
    for i, reg in enumerate(regions):
        if len(reg) == 4:
            cur, sh, ln, rid = reg
            arr[i] = _Region(cur or None, sh or None, ln, rid)
        else:
            cur, sh, rid = reg
            arr[i] = _Region(_buf(cur) or None, _buf(sh) or None, cur.size, rid)
    return arr


def _status(st: _Status) -> Status:
    return Status(st.code, st.first_bad, st.n_dirty, st.total_pages, st.image_bytes)


def crc32c(data) -> int:
    """Standard CRC-32C of a bytes-like object or uint8 array."""
    a = np.frombuffer(bytes(data), dtype=np.uint8) if not isinstance(data, np.ndarray) else data
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return lib().orc_crc32c(a.ctypes.data if a.size else None, a.size)


def validate(regions, page_size: int) -> int:
    arr = _regions(regions)
    return lib().orc_validate(arr if regions else None, len(regions), page_size)


def prefix_bytes(n_regions: int, total_pages: int) -> int:
    return lib().orc_prefix_bytes(n_regions, total_pages)


def snapshot(regions, page_size: int, flags: int = 0, seq: int = 0,
             staging_cap: Optional[int] = None, image_cap: Optional[int] = None):
    """Run the oracle snapshot.

    Returns (Status, image bytes as a numpy uint8 array (empty unless OK),
    bitmap as a numpy uint64 array).  Default capacities are unbounded.
    """
    G = sum(int(r[2] if len(r) == 4 else r[0].size) // page_size for r in regions) \
        if page_size else 0
    W = (G + 63) // 64
    total_cap = prefix_bytes(len(regions), G) + G * page_size + ((4 * G + 7) // 8) * 8
    if image_cap is None:
        image_cap = total_cap
    if staging_cap is None:
        staging_cap = G * page_size
    # every image byte is written by the C code (header, pads, pages, CRCs)
    image = np.empty(max(1, min(image_cap, total_cap)), dtype=np.uint8)
    bitmap = np.zeros(max(1, W), dtype=np.uint64)
    st = _Status()
    arr = _regions(regions)
    lib().orc_snapshot(arr if regions else None, len(regions), page_size, flags, seq,
                       staging_cap, image.ctypes.data, image_cap, bitmap.ctypes.data, W,
                       ctypes.byref(st))
    s = _status(st)
    img = image[: s.image_bytes].copy() if s.code == OK else np.zeros(0, np.uint8)
    return s, img, bitmap[:W].copy()


class _StreamRegion(ctypes.Structure):
    _fields_ = [("len", ctypes.c_uint64), ("id", ctypes.c_uint64),
                ("has_shadow", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


def snapshot_stream(regions, page_size: int, src_fn: int, src_user: int, seq: int = 0,
                    image_cap: Optional[int] = None):
    """The snapshot with region bytes handed in one page at a time.

    regions: sequence of (len, id, has_shadow); src_fn: address of a C
    function ``int src(void* user, uint32_t region, uint64_t page, uint8_t*
    cur, uint8_t* shadow_or_NULL)`` (for example ``synth.lib.PageSource``);
    src_user: its first argument.  Returns (Status, image, bitmap) like
    :func:`snapshot`.  The default capacity holds the image whatever D is;
    the buffer is reserved with np.empty, so only the image's own bytes are
    ever touched."""
    G = sum(int(ln) // page_size for ln, _, _ in regions) if page_size else 0
    W = (G + 63) // 64
    full = prefix_bytes(len(regions), G) + G * page_size + ((4 * G + 7) // 8) * 8
    if image_cap is None:
        image_cap = full
    image = np.empty(max(1, min(image_cap, full)), dtype=np.uint8)
    bitmap = np.zeros(max(1, W), dtype=np.uint64)
    arr = (_StreamRegion * max(1, len(regions)))()
    for i, (ln, rid, has_sh) in enumerate(regions):
        arr[i] = _StreamRegion(ln, rid, 1 if has_sh else 0, 0)
    st = _Status()
    lib().orc_snapshot_stream(arr if regions else None, len(regions), page_size, seq, src_fn,
                              src_user, image.ctypes.data, min(image_cap, full),
                              bitmap.ctypes.data, W, ctypes.byref(st))
    s = _status(st)
    img = image[: s.image_bytes] if s.code == OK else np.zeros(0, np.uint8)
    return s, img, bitmap[:W].copy()


def parse(image) -> tuple:
    """Returns (code, header dict)."""
    a = np.ascontiguousarray(np.frombuffer(bytes(image), np.uint8)
                             if not isinstance(image, np.ndarray) else image, dtype=np.uint8)
    h = _Header()
    rc = lib().orc_parse(a.ctypes.data if a.size else None, a.size, ctypes.byref(h))
    return rc, {f: getattr(h, f) for f, _ in _Header._fields_}


def restore(regions, image: np.ndarray, flags: int = 0) -> Status:
    """Restore the image into the regions' current (and optionally shadow) buffers."""
    a = np.ascontiguousarray(image, dtype=np.uint8)
    st = _Status()
    arr = _regions(regions)
    lib().orc_restore(arr if regions else None, len(regions),
                      a.ctypes.data if a.size else None, a.size, flags, ctypes.byref(st))
    return _status(st)
