"""Convenience layer over the C ABI using torch tensors as plain buffers.

Torch provides device memory, pinned host memory and streams; every step of
the snapshot and restore runs in libcrum's HIP kernels.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

from . import _lib as C


@dataclass
class Status:
    code: int
    first_bad: int
    n_dirty: int
    total_pages: int
    image_bytes: int

    @property
    def name(self) -> str:
        return C.CODE_NAMES.get(self.code, str(self.code))


def _ptr(t) -> int:
    if t is None:
        return 0
    if isinstance(t, int):
        return t
    if t.numel() == 0:
        # torch reports address 0 for any empty tensor; an empty view still
        # names a buffer, and a shadow given for a zero-length region must
        # stay a shadow (None is the way to say "no shadow")
        return t.untyped_storage().data_ptr() + t.storage_offset() * t.element_size()
    return t.data_ptr()


def _nbytes(t) -> int:
    return t.numel() * t.element_size()


def regions_of(pairs: Sequence[Tuple[object, Optional[object], int]]):
    """[(current tensor, shadow tensor or None, id)] -> (base, shadow, len, id) tuples."""
    out = []
    for cur, sh, rid in pairs:
        out.append((_ptr(cur), _ptr(sh), _nbytes(cur), rid))
    return out


class Snapshotter:
    """One libcrum context plus a pinned status buffer."""

    def __init__(self, device: int = 0):
        import torch

        self._torch = torch
        self.ctx = C.crum_ctx_create(device)
        self.status_buf = torch.zeros(64, dtype=torch.uint8, pin_memory=True)

    def close(self) -> None:
        if self.ctx:
            C.crum_ctx_destroy(self.ctx)
            self.ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self, stream) -> int:
        if stream is None:
            return self._torch.cuda.current_stream().cuda_stream
        return stream if isinstance(stream, int) else stream.cuda_stream

    def status(self) -> Status:
        st = C.read_status(self.status_buf.data_ptr())
        return Status(st.code, st.first_bad, st.n_dirty, st.total_pages, st.image_bytes)

    def snapshot(self, regions, page_size: int, staging, h_image=None, flags: int = 0,
                 seq: int = 0, stream=None, sync: bool = True):
        """Enqueue a snapshot. Returns the enqueue code; with sync=True waits
        for the stream and returns (code, Status)."""
        regs = regions if regions and isinstance(regions[0], tuple) and \
            isinstance(regions[0][0], int) else regions_of(regions)
        s = self._stream(stream)
        rc = C.crum_snapshot(self.ctx, regs, page_size, flags, seq, _ptr(staging),
                             _nbytes(staging), _ptr(h_image),
                             _nbytes(h_image) if h_image is not None else 0, s,
                             self.status_buf.data_ptr())
        if not sync:
            return rc
        if rc == C.CRUM_OK:
            self._torch.cuda.synchronize()
        return rc, self.status()

    def restore(self, regions, h_image, image_bytes: int, staging, flags: int = 0,
                stream=None, sync: bool = True):
        regs = regions if regions and isinstance(regions[0], tuple) and \
            isinstance(regions[0][0], int) else regions_of(regions)
        s = self._stream(stream)
        rc = C.crum_restore(self.ctx, regs, _ptr(h_image), image_bytes, flags, _ptr(staging),
                            _nbytes(staging), s, self.status_buf.data_ptr())
        if not sync:
            return rc
        if rc == C.CRUM_OK:
            self._torch.cuda.synchronize()
        return rc, self.status()
