"""ctypes binding of libcrum.so: argument marshalling only.

Every function of ``include/crum.h`` is exposed under the same name with the
same argument order; pointers are Python ints (for example ``tensor.data_ptr()``
of a device or pinned tensor) and streams are raw ``hipStream_t`` handles
(``torch.cuda.current_stream().cuda_stream``).  There is no fallback: when the
shared library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libcrum.so")

CRUM_OK, CRUM_EINVAL, CRUM_ENOSPC, CRUM_ECRC = 0, -1, -2, -3
CRUM_EFORMAT, CRUM_EHIP, CRUM_EMISMATCH = -4, -5, -6
CRUM_EIO, CRUM_EAGAIN = -7, -8
CRUM_ELIMIT = -9
CRUM_NOALLOC_SCRATCH_BYTES, CRUM_NOALLOC_MAX_REGIONS = 64 << 20, 2048
CRUM_UPDATE_SHADOW, CRUM_VERIFY = 1, 2
CRUM_PARAM_DIFF_BLOCKS, CRUM_PARAM_PACK_BLOCKS = 1, 2
CRUM_PARAM_CHUNK_BYTES, CRUM_PARAM_CHUNK_MAX_BYTES = 3, 4
CRUM_PARAM_EAGER, CRUM_PARAM_DRAIN_CHUNK_BYTES = 5, 6
CRUM_PARAM_DIFF_UNIT_SHIFT, CRUM_PARAM_DIFF_NONTEMPORAL = 7, 8
CRUM_PARAM_PIECE_SHIFT, CRUM_PARAM_PACK_DEPTH, CRUM_PARAM_DIFF_PRIORITY = 9, 10, 11
CRUM_PARAM_CRC_VARIANT, CRUM_PARAM_PLAN_ORDER = 12, 13
CRUM_PARAM_DIRECT_BYTES = 14
CRUM_PARAM_CHUNK_GROWTH, CRUM_PARAM_PACK_NT_STORE, CRUM_PARAM_PACK_PREFETCH = 15, 16, 17
CRUM_PARAM_PACK_NT_LOAD, CRUM_PARAM_DIFF_GROUP = 18, 19

CODE_NAMES = {0: "CRUM_OK", -1: "CRUM_EINVAL", -2: "CRUM_ENOSPC", -3: "CRUM_ECRC",
              -4: "CRUM_EFORMAT", -5: "CRUM_EHIP", -6: "CRUM_EMISMATCH", -7: "CRUM_EIO",
              -8: "CRUM_EAGAIN", -9: "CRUM_ELIMIT"}


class crum_region(ctypes.Structure):
    _fields_ = [("base", ctypes.c_void_p), ("shadow", ctypes.c_void_p),
                ("len", ctypes.c_uint64), ("id", ctypes.c_uint64)]


class crum_status(ctypes.Structure):
    _fields_ = [("code", ctypes.c_int32), ("first_bad", ctypes.c_uint32),
                ("n_dirty", ctypes.c_uint64), ("total_pages", ctypes.c_uint64),
                ("image_bytes", ctypes.c_uint64)]


class crum_request(ctypes.Structure):
    _fields_ = [("regions", ctypes.c_void_p), ("n_regions", ctypes.c_uint32),
                ("page_size", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("seq", ctypes.c_uint64)]


class crum_client(ctypes.Structure):
    _fields_ = [("regions", ctypes.c_void_p), ("n_regions", ctypes.c_uint32),
                ("page_size", ctypes.c_uint32)]


class crum_server_completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("tag", ctypes.c_uint64), ("client", ctypes.c_uint32),
                ("kind", ctypes.c_uint32), ("code", ctypes.c_int32),
                ("meta_crc", ctypes.c_uint32), ("crcs_crc", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("n_dirty", ctypes.c_uint64),
                ("image_bytes", ctypes.c_uint64), ("arrival_s", ctypes.c_double),
                ("start_s", ctypes.c_double), ("done_s", ctypes.c_double)]


PREPARE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                              ctypes.c_uint64, ctypes.c_void_p)
CRUM_REQ_SNAPSHOT, CRUM_REQ_RESTORE = 1, 2
CRUM_SERVE_ADAPTIVE, CRUM_SERVE_TWO_STAGE, CRUM_SERVE_PIPELINED = 0, 1, 2


class crum_write_status(ctypes.Structure):
    _fields_ = [("code", ctypes.c_int32), ("err", ctypes.c_int32), ("bytes", ctypes.c_uint64),
                ("direct", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("seconds", ctypes.c_double)]


CRUM_WRITE_DIRECT, CRUM_WRITE_SYNC = 1, 2


class crum_lazy_info(ctypes.Structure):
    _fields_ = [("pages_total", ctypes.c_uint64), ("pages_fetched", ctypes.c_uint64),
                ("faults", ctypes.c_uint64), ("copies", ctypes.c_uint64),
                ("bytes_fetched", ctypes.c_uint64)]


class crum_request_status(ctypes.Structure):
    _fields_ = [("status", crum_status), ("image_offset", ctypes.c_uint64)]


_P = ctypes.c_void_p
_U32, _U64, _I = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
_SIGS = {
    "crum_ctx_create": (_I, [_I, ctypes.c_char_p, ctypes.POINTER(_P)]),
    "crum_ctx_tuned_classes": (_I, [_P, ctypes.POINTER(_U32)]),
    "crum_tuning_check": (_I, [ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(_U32)]),
    "crum_ctx_destroy": (None, [_P]),
    "crum_image_prefix_bytes": (_I, [_U32, _U64, ctypes.POINTER(_U64)]),
    "crum_image_bytes": (_I, [_U32, _U64, _U64, _U32, ctypes.POINTER(_U64)]),
    "crum_snapshot": (_I, [_P, _P, _U32, _U32, _U32, _U64, _P, _U64, _P, _U64, _P, _P]),
    "crum_restore": (_I, [_P, _P, _U32, _P, _U64, _U32, _P, _U64, _P, _P]),
    "crum_plan_create": (_I, [_P, _P, _U32, _P, _U64, _P, _U64, ctypes.POINTER(_P)]),
    "crum_plan_launch": (_I, [_P, _P, _P]),
    "crum_plan_groups": (_I, [_P, ctypes.POINTER(_U32), _P, _U32]),
    "crum_plan_group_times": (_I, [_P, _P, _U32]),
    "crum_plan_order": (_I, [_P, _P, _U32]),
    "crum_plan_destroy": (None, [_P]),
    "crum_server_create": (_I, [_I, _P, _U32, _U32, _U64, ctypes.POINTER(_P)]),
    "crum_server_set_prepare": (_I, [_P, _P, _P]),
    "crum_server_set_policy": (_I, [_P, _I]),
    "crum_server_submit": (_I, [_P, _U32, _U32, _U64, ctypes.POINTER(_U64)]),
    "crum_server_poll": (_I, [_P, _P, _U32, ctypes.POINTER(_U32), _I]),
    "crum_server_time": (ctypes.c_double, [_P]),
    "crum_server_pinned_used": (_I, [_P, ctypes.POINTER(_U64)]),
    "crum_server_latest_image": (_I, [_P, _U32, ctypes.POINTER(_P), ctypes.POINTER(_U64)]),
    "crum_server_destroy": (None, [_P]),
    "crum_ctx_set_param": (_I, [_P, _I, _U64]),
    "crum_ctx_get_param": (_I, [_P, _I, ctypes.POINTER(_U64)]),
    "crum_ctx_set_timing": (_I, [_P, _I]),
    "crum_ctx_timing": (_I, [_P, _I, ctypes.POINTER(_U64), ctypes.POINTER(ctypes.c_double)]),
    "crum_ctx_timing_reset": (_I, [_P]),
    "crum_writer_create": (_I, [_U32, _U64, _U32, ctypes.POINTER(_P)]),
    "crum_writer_submit": (_I, [_P, ctypes.c_char_p, _P, _U64, ctypes.POINTER(_U64)]),
    "crum_writer_poll": (_I, [_P, _U64, _I, _P]),
    "crum_writer_destroy": (None, [_P]),
    "crum_lazy_open": (_I, [_P, _P, _U32, _P, _U64, _U32, _U64, _P, _U64, _P, _P,
                            ctypes.POINTER(_P)]),
    "crum_lazy_touch": (_I, [_P, _U32, _U64, _U64, _P, _P, ctypes.POINTER(_U64)]),
    "crum_lazy_finish": (_I, [_P, _P, _P]),
    "crum_lazy_stats": (_I, [_P, _P]),
    "crum_lazy_fetched": (_I, [_P, _P, _U64]),
    "crum_lazy_close": (None, [_P]),
    "crum_track_create": (_I, [_U64, _U32, ctypes.POINTER(_P)]),
    "crum_track_view": (_P, [_P]),
    "crum_track_flush": (_I, [_P, _P, _U32, ctypes.POINTER(_U64)]),
    "crum_track_pending": (_I, [_P, _P, _U64, _I]),
    "crum_track_dirty": (_I, [_P, _P, _U64]),
    "crum_track_stats": (_I, [_P, _P]),
    "crum_track_destroy": (None, [_P]),
    "crum_snapshot_tracked": (_I, [_P, _P, _U32, _U32, _U32, _U64, _P, _U64, _P, _U64, _P,
                                   _U64, _P, _P]),
    "crum_snapshot_noalloc": (_I, [_P, _P, _U32, _U32, _U32, _U64, _P, _U64, _P, _U64, _P,
                                   _P]),
}

_lib = None


def lib():
    """Load libcrum.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO):
            raise RuntimeError(f"{SO} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(SO)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def region_table(regions: Sequence) -> "ctypes.Array":
    """regions: (base_ptr, shadow_ptr_or_0, len, id) tuples -> crum_region array."""
    arr = (crum_region * max(1, len(regions)))()
    for i, (base, shadow, ln, rid) in enumerate(regions):
        arr[i] = crum_region(base or None, shadow or None, ln, rid)
    return arr


def crum_ctx_create(device: int = 0, tuning_cache: Optional[str] = None) -> int:
    h = _P()
    path = tuning_cache.encode() if tuning_cache else None
    rc = lib().crum_ctx_create(device, path, ctypes.byref(h))
    if rc != CRUM_OK:
        raise RuntimeError(f"crum_ctx_create failed: {CODE_NAMES.get(rc, rc)}")
    return h.value


def crum_ctx_tuned_classes(ctx: int) -> int:
    n = _U32()
    rc = lib().crum_ctx_tuned_classes(ctx, ctypes.byref(n))
    if rc != CRUM_OK:
        raise RuntimeError(CODE_NAMES.get(rc, rc))
    return n.value


def crum_tuning_check(path: str, device_key: str):
    """(code, number of classes) of a tuning cache file for a device key."""
    n = _U32()
    rc = lib().crum_tuning_check(path.encode(), device_key.encode(), ctypes.byref(n))
    return rc, n.value


def crum_ctx_destroy(ctx: int) -> None:
    lib().crum_ctx_destroy(ctx)


def crum_image_prefix_bytes(n_regions: int, total_pages: int) -> int:
    out = _U64()
    rc = lib().crum_image_prefix_bytes(n_regions, total_pages, ctypes.byref(out))
    if rc != CRUM_OK:
        raise ValueError(CODE_NAMES.get(rc, rc))
    return out.value


def crum_image_bytes(n_regions: int, total_pages: int, n_dirty: int, page_size: int) -> int:
    out = _U64()
    rc = lib().crum_image_bytes(n_regions, total_pages, n_dirty, page_size, ctypes.byref(out))
    if rc != CRUM_OK:
        raise ValueError(CODE_NAMES.get(rc, rc))
    return out.value


def crum_snapshot(ctx: int, regions, page_size: int, flags: int, seq: int, d_staging: int,
                  staging_bytes: int, h_image: int, h_image_bytes: int, stream: int,
                  h_status: int) -> int:
    """regions: sequence of (base, shadow, len, id) or a crum_region array."""
    arr = regions if isinstance(regions, ctypes.Array) else region_table(regions)
    n = len(regions)
    return lib().crum_snapshot(ctx, ctypes.cast(arr, _P) if n else None, n, page_size, flags,
                               seq, d_staging, staging_bytes, h_image or None, h_image_bytes,
                               stream or None, h_status)


def crum_snapshot_noalloc(ctx: int, regions, page_size: int, flags: int, seq: int,
                          d_staging: int, staging_bytes: int, h_image: int, h_image_bytes: int,
                          stream: int, h_status: int) -> int:
    """As crum_snapshot, through the entry point that allocates nothing."""
    arr = regions if isinstance(regions, ctypes.Array) else region_table(regions)
    n = len(regions)
    return lib().crum_snapshot_noalloc(ctx, ctypes.cast(arr, _P) if n else None, n, page_size,
                                       flags, seq, d_staging, staging_bytes, h_image or None,
                                       h_image_bytes, stream or None, h_status)


def crum_snapshot_tracked(ctx: int, regions, page_size: int, flags: int, seq: int,
                          candidates, d_staging: int, staging_bytes: int, h_image: int,
                          h_image_bytes: int, stream: int, h_status: int) -> int:
    """candidates: a uint64 numpy array (the candidate bitmap, host memory)."""
    import numpy as np
    arr = regions if isinstance(regions, ctypes.Array) else region_table(regions)
    n = len(regions)
    cand = np.ascontiguousarray(candidates, dtype=np.uint64)
    return lib().crum_snapshot_tracked(ctx, ctypes.cast(arr, _P) if n else None, n, page_size,
                                       flags, seq, cand.ctypes.data if cand.size else None,
                                       cand.size, d_staging, staging_bytes, h_image or None,
                                       h_image_bytes, stream or None, h_status)


class crum_track_info(ctypes.Structure):
    _fields_ = [("pages", ctypes.c_uint64), ("dirty_pages", ctypes.c_uint64),
                ("pending_pages", ctypes.c_uint64), ("faults", ctypes.c_uint64),
                ("flushed_pages", ctypes.c_uint64)]


class Tracker:
    """Owns a crum_track: a host view of `nbytes` whose writes are tracked
    per page of `page_size` bytes."""

    def __init__(self, nbytes: int, page_size: int):
        h = _P()
        rc = lib().crum_track_create(nbytes, page_size, ctypes.byref(h))
        if rc != CRUM_OK:
            raise RuntimeError(f"crum_track_create: {CODE_NAMES.get(rc, rc)}")
        self.handle, self.nbytes, self.page_size = h.value, nbytes, page_size
        self.n_pages = nbytes // page_size
        self.ptr = lib().crum_track_view(self.handle)

    def view(self):
        """The view as a writable uint8 numpy array (no copy)."""
        import numpy as np
        return np.ctypeslib.as_array((ctypes.c_uint8 * self.nbytes).from_address(self.ptr))

    def flush(self, dst: int, n_threads: int = 1) -> int:
        n = _U64()
        rc = lib().crum_track_flush(self.handle, dst, n_threads, ctypes.byref(n))
        if rc != CRUM_OK:
            raise RuntimeError(f"crum_track_flush: {CODE_NAMES.get(rc, rc)}")
        return n.value

    def _bits(self, fn, *extra):
        import numpy as np
        w = np.zeros(max(1, (self.n_pages + 63) // 64), np.uint64)
        rc = fn(self.handle, w.ctypes.data, w.size, *extra)
        if rc != CRUM_OK:
            raise RuntimeError(CODE_NAMES.get(rc, rc))
        return w

    def pending(self, clear: bool = False):
        return self._bits(lib().crum_track_pending, 1 if clear else 0)

    def dirty(self):
        return self._bits(lib().crum_track_dirty)

    def stats(self) -> dict:
        info = crum_track_info()
        rc = lib().crum_track_stats(self.handle, ctypes.byref(info))
        if rc != CRUM_OK:
            raise RuntimeError(CODE_NAMES.get(rc, rc))
        return {f: getattr(info, f) for f, _ in crum_track_info._fields_}

    def destroy(self) -> None:
        if self.handle:
            lib().crum_track_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def crum_restore(ctx: int, regions, h_image: int, image_bytes: int, flags: int,
                 d_staging: int, staging_bytes: int, stream: int, h_status: int) -> int:
    arr = regions if isinstance(regions, ctypes.Array) else region_table(regions)
    n = len(regions)
    return lib().crum_restore(ctx, ctypes.cast(arr, _P) if n else None, n, h_image or None,
                              image_bytes, flags, d_staging, staging_bytes, stream or None,
                              h_status)


class Plan:
    """Owns a crum_plan and the ctypes arrays it was created from.

    requests: sequence of (regions, page_size, flags, seq) where regions is a
    sequence of (base, shadow, len, id)."""

    def __init__(self, ctx: int, requests, d_staging: int, staging_bytes: int, h_images: int,
                 h_images_bytes: int):
        self._tables = [region_table(regs) for regs, _, _, _ in requests]
        self.n = len(requests)
        arr = (crum_request * max(1, self.n))()
        for i, ((regs, ps, flags, seq), tab) in enumerate(zip(requests, self._tables)):
            arr[i] = crum_request(ctypes.cast(tab, _P) if len(regs) else None, len(regs), ps,
                                  flags, 0, seq)
        self._reqs = arr
        h = _P()
        rc = lib().crum_plan_create(ctx, ctypes.cast(arr, _P) if self.n else None, self.n,
                                    d_staging, staging_bytes, h_images or None, h_images_bytes,
                                    ctypes.byref(h))
        if rc != CRUM_OK:
            raise RuntimeError(f"crum_plan_create: {CODE_NAMES.get(rc, rc)}")
        self.handle = h.value

    def launch(self, stream: int, h_status: int) -> int:
        return lib().crum_plan_launch(self.handle, stream or None, h_status)

    def order(self):
        """Caller's index of the request at each processing position."""
        arr = (_U32 * max(1, self.n))()
        lib().crum_plan_order(self.handle, ctypes.cast(arr, _P), self.n)
        return [arr[i] for i in range(self.n)]

    def groups(self):
        n = _U32()
        lib().crum_plan_groups(self.handle, ctypes.byref(n), None, 0)
        arr = (_U32 * (n.value + 1))()
        lib().crum_plan_groups(self.handle, ctypes.byref(n), ctypes.cast(arr, _P), n.value + 1)
        return list(arr)

    def group_times(self):
        n = len(self.groups()) - 1
        arr = (ctypes.c_double * max(1, n))()
        rc = lib().crum_plan_group_times(self.handle, ctypes.cast(arr, _P), n)
        if rc != CRUM_OK:
            raise RuntimeError(CODE_NAMES.get(rc, rc))
        return list(arr)[:n]

    def destroy(self) -> None:
        if self.handle:
            lib().crum_plan_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Server:
    """Owns a crum_server.  clients: sequence of (regions, page_size) where
    regions is a sequence of (base, shadow, len, id)."""

    def __init__(self, clients, n_slots: int, pinned_budget: int, device: int = 0,
                 prepare=None):
        self._tables = [region_table(regs) for regs, _ in clients]
        arr = (crum_client * max(1, len(clients)))()
        for i, ((regs, ps), tab) in enumerate(zip(clients, self._tables)):
            arr[i] = crum_client(ctypes.cast(tab, _P) if len(regs) else None, len(regs), ps)
        self._clients = arr
        h = _P()
        rc = lib().crum_server_create(device, ctypes.cast(arr, _P), len(clients), n_slots,
                                      pinned_budget, ctypes.byref(h))
        if rc != CRUM_OK:
            raise RuntimeError(f"crum_server_create: {CODE_NAMES.get(rc, rc)}")
        self.handle = h.value
        self._prepare = None
        if prepare is not None:
            self._prepare = PREPARE_FN(prepare)
            lib().crum_server_set_prepare(self.handle, ctypes.cast(self._prepare, _P), None)

    def set_policy(self, policy: int) -> None:
        rc = lib().crum_server_set_policy(self.handle, policy)
        if rc != CRUM_OK:
            raise ValueError(CODE_NAMES.get(rc, rc))

    def submit(self, client: int, kind: int, tag: int = 0) -> int:
        i = _U64()
        rc = lib().crum_server_submit(self.handle, client, kind, tag, ctypes.byref(i))
        if rc != CRUM_OK:
            raise RuntimeError(f"crum_server_submit: {CODE_NAMES.get(rc, rc)}")
        return i.value

    def poll(self, wait_all: bool = False, max_n: int = 4096):
        arr = (crum_server_completion * max_n)()
        n = _U32()
        rc = lib().crum_server_poll(self.handle, ctypes.cast(arr, _P), max_n, ctypes.byref(n),
                                    1 if wait_all else 0)
        if rc != CRUM_OK:
            raise RuntimeError(f"crum_server_poll: {CODE_NAMES.get(rc, rc)}")
        out = []
        for i in range(n.value):
            c = arr[i]
            out.append({f: getattr(c, f) for f, _ in crum_server_completion._fields_})
        if wait_all and n.value == max_n:
            out.extend(self.poll(True, max_n))
        return out

    def time(self) -> float:
        return lib().crum_server_time(self.handle)

    def pinned_used(self) -> int:
        v = _U64()
        lib().crum_server_pinned_used(self.handle, ctypes.byref(v))
        return v.value

    def latest_image(self, client: int):
        p, n = _P(), _U64()
        rc = lib().crum_server_latest_image(self.handle, client, ctypes.byref(p), ctypes.byref(n))
        if rc != CRUM_OK:
            return None
        return p.value, n.value

    def destroy(self) -> None:
        if self.handle:
            lib().crum_server_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def read_request_statuses(addr: int, n: int):
    arr = (crum_request_status * max(1, n)).from_address(addr)
    return [(arr[i].status.code, arr[i].status.first_bad, arr[i].status.n_dirty,
             arr[i].status.total_pages, arr[i].status.image_bytes, arr[i].image_offset)
            for i in range(n)]


def crum_ctx_set_param(ctx: int, param: int, value: int) -> None:
    rc = lib().crum_ctx_set_param(ctx, param, value)
    if rc != CRUM_OK:
        raise ValueError(f"crum_ctx_set_param({param}, {value}): {CODE_NAMES.get(rc, rc)}")


def crum_ctx_get_param(ctx: int, param: int) -> int:
    v = _U64()
    rc = lib().crum_ctx_get_param(ctx, param, ctypes.byref(v))
    if rc != CRUM_OK:
        raise ValueError(CODE_NAMES.get(rc, rc))
    return v.value


TIMING_DIFF, TIMING_PACK, TIMING_DRAIN, TIMING_SCAN, TIMING_HEADER = 1, 2, 4, 8, 16
TIMING_VERIFY, TIMING_SCATTER = 32, 64


def crum_ctx_set_timing(ctx: int, classes) -> None:
    """classes: True (every class), False (off) or a bit mask of TIMING_*."""
    if classes is True:
        classes = -1
    elif classes is False:
        classes = 0
    rc = lib().crum_ctx_set_timing(ctx, int(classes))
    if rc != CRUM_OK:
        raise ValueError(CODE_NAMES.get(rc, rc))


def crum_ctx_timing(ctx: int, which: int):
    n, ms = _U64(), ctypes.c_double()
    rc = lib().crum_ctx_timing(ctx, which, ctypes.byref(n), ctypes.byref(ms))
    if rc != CRUM_OK:
        raise RuntimeError(CODE_NAMES.get(rc, rc))
    return n.value, ms.value


def crum_ctx_timing_reset(ctx: int) -> None:
    rc = lib().crum_ctx_timing_reset(ctx)
    if rc != CRUM_OK:
        raise RuntimeError(CODE_NAMES.get(rc, rc))


def read_status(addr: int) -> crum_status:
    """Copy a crum_status out of (pinned) host memory at addr."""
    st = crum_status()
    ctypes.memmove(ctypes.byref(st), addr, ctypes.sizeof(st))
    return st


class Writer:
    """Owns a crum_writer: persists host images to files on a thread pool."""

    def __init__(self, n_threads: int = 4, chunk_bytes: int = 64 << 20,
                 flags: int = CRUM_WRITE_DIRECT | CRUM_WRITE_SYNC):
        h = _P()
        rc = lib().crum_writer_create(n_threads, chunk_bytes, flags, ctypes.byref(h))
        if rc != CRUM_OK:
            raise ValueError(f"crum_writer_create: {CODE_NAMES.get(rc, rc)}")
        self.handle = h.value

    def submit(self, path: str, image_ptr: int, nbytes: int) -> int:
        t = _U64()
        rc = lib().crum_writer_submit(self.handle, os.fsencode(path), image_ptr or None, nbytes,
                                      ctypes.byref(t))
        if rc != CRUM_OK:
            raise OSError(f"crum_writer_submit({path}): {CODE_NAMES.get(rc, rc)}")
        return t.value

    def poll(self, ticket: int, wait: bool = True):
        """dict of the write's status, or None while it runs (wait=False)."""
        st = crum_write_status()
        rc = lib().crum_writer_poll(self.handle, ticket, 1 if wait else 0, ctypes.byref(st))
        if rc == CRUM_EAGAIN:
            return None
        if rc != CRUM_OK:
            raise ValueError(f"crum_writer_poll: {CODE_NAMES.get(rc, rc)}")
        return {f: getattr(st, f) for f, _ in crum_write_status._fields_}

    def destroy(self) -> None:
        if self.handle:
            lib().crum_writer_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class ImageError(Exception):
    """An image refused by the host-side checks; .code is the CRUM_ code."""

    def __init__(self, code: int):
        super().__init__(CODE_NAMES.get(code, code))
        self.code = code


class Lazy:
    """Owns a crum_lazy session (on-demand restore of an image).

    Raises ValueError for argument errors; an image error found on the host
    (EFORMAT, EMISMATCH, ENOSPC) is raised as ImageError with the status."""

    def __init__(self, ctx: int, regions, h_image: int, image_bytes: int, flags: int,
                 small_bytes: int, d_staging: int, staging_bytes: int, stream: int,
                 h_status: int):
        self._table = regions if isinstance(regions, ctypes.Array) else region_table(regions)
        n = len(regions)
        h = _P()
        rc = lib().crum_lazy_open(ctx, ctypes.cast(self._table, _P) if n else None, n,
                                  h_image or None, image_bytes, flags, small_bytes, d_staging,
                                  staging_bytes, stream or None, h_status, ctypes.byref(h))
        self.handle = h.value or 0
        if rc in (CRUM_EFORMAT, CRUM_EMISMATCH, CRUM_ENOSPC):
            raise ImageError(rc)
        if rc != CRUM_OK:
            raise ValueError(f"crum_lazy_open: {CODE_NAMES.get(rc, rc)}")

    def touch(self, region: int, offset: int, length: int, stream: int, h_status: int = 0) -> int:
        """Returns the number of pages the access fetched (0: not a fault)."""
        n = _U64()
        rc = lib().crum_lazy_touch(self.handle, region, offset, length, stream or None,
                                   h_status or None, ctypes.byref(n))
        if rc != CRUM_OK:
            raise ValueError(f"crum_lazy_touch: {CODE_NAMES.get(rc, rc)}")
        return n.value

    def finish(self, stream: int, h_status: int) -> None:
        rc = lib().crum_lazy_finish(self.handle, stream or None, h_status)
        if rc != CRUM_OK:
            raise ValueError(f"crum_lazy_finish: {CODE_NAMES.get(rc, rc)}")

    def stats(self) -> dict:
        st = crum_lazy_info()
        rc = lib().crum_lazy_stats(self.handle, ctypes.byref(st))
        if rc != CRUM_OK:
            raise ValueError(f"crum_lazy_stats: {CODE_NAMES.get(rc, rc)}")
        return {f: getattr(st, f) for f, _ in crum_lazy_info._fields_}

    def fetched(self, n_words: int):
        """The fetched-page bitmap as a list of n_words ints."""
        arr = (ctypes.c_uint64 * max(1, n_words))()
        rc = lib().crum_lazy_fetched(self.handle, ctypes.cast(arr, _P), n_words)
        if rc != CRUM_OK:
            raise ValueError(f"crum_lazy_fetched: {CODE_NAMES.get(rc, rc)}")
        return list(arr)[:n_words]

    def close(self) -> None:
        if self.handle:
            lib().crum_lazy_close(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
