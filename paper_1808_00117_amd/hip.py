"""Minimal HIP runtime plumbing without torch: device and pinned buffers,
streams, events and graph capture through ctypes.

It binds the HIP runtime that libcrum itself is linked against.  In a process
that never imports torch this is the system ROCm runtime, which executes
device-to-host hipMemcpyAsync on the SDMA copy engines; torch wheels bundle
their own runtime, whose device-to-host copies run as blit kernels on the
compute units.  Argument marshalling only.
"""
from __future__ import annotations

import ctypes
from typing import Optional

from . import _lib

_hip = None

hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice = 1, 2, 3
hipStreamNonBlocking = 1
hipStreamCaptureModeGlobal = 0


def hip():
    global _hip
    if _hip is None:
        _lib.lib()  # resolves libamdhip64 through libcrum's own dependency
        h = ctypes.CDLL("libamdhip64.so.7")
        V, S, I = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
        sigs = {
            "hipMalloc": [ctypes.POINTER(V), S],
            "hipFree": [V],
            "hipHostMalloc": [ctypes.POINTER(V), S, ctypes.c_uint],
            "hipHostFree": [V],
            "hipMemcpy": [V, V, S, I],
            "hipMemcpyAsync": [V, V, S, I, V],
            "hipMemsetAsync": [V, I, S, V],
            "hipMemset": [V, I, S],
            "hipStreamCreateWithFlags": [ctypes.POINTER(V), ctypes.c_uint],
            "hipStreamDestroy": [V],
            "hipStreamSynchronize": [V],
            "hipDeviceSynchronize": [],
            "hipEventCreate": [ctypes.POINTER(V)],
            "hipEventDestroy": [V],
            "hipEventRecord": [V, V],
            "hipEventSynchronize": [V],
            "hipEventElapsedTime": [ctypes.POINTER(ctypes.c_float), V, V],
            "hipStreamBeginCapture": [V, I],
            "hipStreamEndCapture": [V, ctypes.POINTER(V)],
            "hipGraphInstantiate": [ctypes.POINTER(V), V, V, V, S],
            "hipGraphLaunch": [V, V],
            "hipGraphExecDestroy": [V],
            "hipGraphDestroy": [V],
            "hipGetDeviceCount": [ctypes.POINTER(I)],
            "hipMemGetInfo": [ctypes.POINTER(S), ctypes.POINTER(S)],
            "hipMallocManaged": [ctypes.POINTER(V), S, ctypes.c_uint],
            "hipMemPrefetchAsync": [V, S, I, V],
            "hipMemAdvise": [V, S, I, I],
            "hipMemRangeGetAttribute": [V, S, I, V, S],
            "hipPointerGetAttributes": [V, V],
            "hipGetLastError": [],
        }
        for name, args in sigs.items():
            f = getattr(h, name)
            f.restype = ctypes.c_int
            f.argtypes = args
        _hip = h
    return _hip


def check(rc: int, what: str) -> None:
    """Raise on a failed HIP call.  HIP also keeps the failure as the calling
    thread's last error, which the next launch check (hipGetLastError, as in
    libcrum's kernel launchers) would report as its own; a caller that goes on
    after catching this error must not see it there, so it is cleared here."""
    if rc != 0:
        hip().hipGetLastError()
        raise RuntimeError(f"{what} failed with hipError {rc}")


def device_count() -> int:
    n = ctypes.c_int(0)
    if hip().hipGetDeviceCount(ctypes.byref(n)) != 0:
        return 0
    return n.value


class DeviceBuffer:
    def __init__(self, nbytes: int):
        p = ctypes.c_void_p()
        check(hip().hipMalloc(ctypes.byref(p), max(nbytes, 16)), f"hipMalloc({nbytes})")
        self.ptr, self.nbytes = p.value, nbytes

    def free(self) -> None:
        if self.ptr:
            hip().hipFree(self.ptr)
            self.ptr = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


hipMemAttachGlobal = 1
hipMemAdviseSetPreferredLocation = 3
hipMemRangeAttributeLastPrefetchLocation = 4
hipCpuDeviceId = -1


class PointerAttributes(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int), ("device", ctypes.c_int),
                ("devicePointer", ctypes.c_void_p), ("hostPointer", ctypes.c_void_p),
                ("isManaged", ctypes.c_int), ("allocationFlags", ctypes.c_uint)]


def pointer_attributes(ptr: int) -> dict:
    a = PointerAttributes()
    check(hip().hipPointerGetAttributes(ctypes.byref(a), ptr), "hipPointerGetAttributes")
    return {"type": a.type, "device": a.device, "devicePointer": a.devicePointer or 0,
            "hostPointer": a.hostPointer or 0, "isManaged": a.isManaged,
            "allocationFlags": a.allocationFlags}


class ManagedBuffer:
    """hipMallocManaged memory (host and device may both touch it)."""

    def __init__(self, nbytes: int):
        p = ctypes.c_void_p()
        check(hip().hipMallocManaged(ctypes.byref(p), max(nbytes, 16), hipMemAttachGlobal),
              f"hipMallocManaged({nbytes})")
        self.ptr, self.nbytes = p.value, nbytes

    def device_mapped(self) -> bool:
        """True when the runtime reports the allocation mapped into the
        device's address space at the same address (the condition for a
        kernel to read it through this pointer)."""
        a = pointer_attributes(self.ptr)
        return a["devicePointer"] == self.ptr

    def prefetch(self, offset: int, nbytes: int, device: int, stream: int = 0) -> int:
        """hipMemPrefetchAsync of a sub-range; returns the HIP status."""
        return hip().hipMemPrefetchAsync(self.ptr + offset, nbytes, device, stream)

    def last_prefetch_location(self, offset: int, nbytes: int):
        """(HIP status, location) of hipMemRangeGetAttribute(LastPrefetchLocation).
        The query can leave an error in the runtime's last-error slot, which a
        later launch check would report as its own: the slot is read and
        cleared here, and a nonzero value is returned as the status when the
        call itself reported success."""
        v = ctypes.c_int(-99)
        rc = hip().hipMemRangeGetAttribute(ctypes.byref(v), 4,
                                           hipMemRangeAttributeLastPrefetchLocation,
                                           self.ptr + offset, nbytes)
        last = hip().hipGetLastError()
        return (rc or last), v.value

    def numpy(self, offset: int, n: int):
        import numpy as np
        return np.ctypeslib.as_array((ctypes.c_uint8 * n).from_address(self.ptr + offset))

    def free(self) -> None:
        if self.ptr:
            hip().hipFree(self.ptr)
            self.ptr = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class PinnedBuffer:
    def __init__(self, nbytes: int):
        p = ctypes.c_void_p()
        check(hip().hipHostMalloc(ctypes.byref(p), max(nbytes, 16), 0), f"hipHostMalloc({nbytes})")
        self.ptr, self.nbytes = p.value, nbytes

    def numpy(self, n: Optional[int] = None):
        import numpy as np
        n = self.nbytes if n is None else n
        return np.ctypeslib.as_array((ctypes.c_uint8 * n).from_address(self.ptr))

    def free(self) -> None:
        if self.ptr:
            hip().hipHostFree(self.ptr)
            self.ptr = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Stream:
    def __init__(self):
        s = ctypes.c_void_p()
        check(hip().hipStreamCreateWithFlags(ctypes.byref(s), hipStreamNonBlocking),
              "hipStreamCreateWithFlags")
        self.handle = s.value

    def synchronize(self) -> None:
        check(hip().hipStreamSynchronize(self.handle), "hipStreamSynchronize")


class Event:
    def __init__(self):
        e = ctypes.c_void_p()
        check(hip().hipEventCreate(ctypes.byref(e)), "hipEventCreate")
        self.handle = e.value

    def record(self, stream: Stream) -> None:
        check(hip().hipEventRecord(self.handle, stream.handle), "hipEventRecord")

    def elapsed_ms(self, end: "Event") -> float:
        check(hip().hipEventSynchronize(end.handle), "hipEventSynchronize")
        ms = ctypes.c_float()
        check(hip().hipEventElapsedTime(ctypes.byref(ms), self.handle, end.handle),
              "hipEventElapsedTime")
        return ms.value


class Graph:
    """Capture work issued by `fn(stream)` on `stream` into an executable graph."""

    def __init__(self, stream: Stream, fn):
        h = hip()
        check(h.hipStreamBeginCapture(stream.handle, hipStreamCaptureModeGlobal),
              "hipStreamBeginCapture")
        fn(stream)
        g = ctypes.c_void_p()
        check(h.hipStreamEndCapture(stream.handle, ctypes.byref(g)), "hipStreamEndCapture")
        ex = ctypes.c_void_p()
        check(h.hipGraphInstantiate(ctypes.byref(ex), g, None, None, 0), "hipGraphInstantiate")
        self.graph, self.exec = g.value, ex.value

    def launch(self, stream: Stream) -> None:
        check(hip().hipGraphLaunch(self.exec, stream.handle), "hipGraphLaunch")


def device_synchronize() -> None:
    check(hip().hipDeviceSynchronize(), "hipDeviceSynchronize")


def memcpy_dtoh(dst_host: int, src_dev: int, n: int) -> None:
    check(hip().hipMemcpy(dst_host, src_dev, n, hipMemcpyDeviceToHost), "hipMemcpy D2H")


def memcpy_dtod(dst: int, src: int, n: int) -> None:
    check(hip().hipMemcpy(dst, src, n, hipMemcpyDeviceToDevice), "hipMemcpy D2D")


def memcpy_htod(dst_dev: int, src_host: int, n: int) -> None:
    check(hip().hipMemcpy(dst_dev, src_host, n, hipMemcpyHostToDevice), "hipMemcpy H2D")
