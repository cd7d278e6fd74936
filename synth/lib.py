"""Loaders and thin wrappers for the synthetic-input generators."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
HOST_SO = os.path.join(_HERE, "libsynth_host.so")
DEV_SO = os.path.join(_HERE, "libsynth_dev.so")

HIP_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]

_host = None
_dev = None

M_GOLD = 0x9E3779B97F4A7C15
M_REGION = 0xD1B54A32D192ED03
M_PAGE = 0x8CB92BA72F3D8DD7
U64 = (1 << 64) - 1


def build(verbose: bool = False) -> None:
    """Compile both generator libraries in-tree (host C with gcc, HIP with hipcc)."""
    src_c = os.path.join(_HERE, "csrc", "synth_host.c")
    src_h = os.path.join(_HERE, "csrc", "synth_dev.hip")
    cmds = [
        ["gcc", "-O2", "-fPIC", "-shared", "-o", HOST_SO + ".tmp", src_c],
        ["hipcc", *HIP_FLAGS, "-o", DEV_SO + ".tmp", src_h],
    ]
    for cmd, out in zip(cmds, [HOST_SO, DEV_SO]):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


def host_lib():
    global _host
    if _host is None:
        if not os.path.exists(HOST_SO):
            raise RuntimeError(f"{HOST_SO} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(HOST_SO)
        lib.synth_word.restype = ctypes.c_uint64
        lib.synth_word.argtypes = [ctypes.c_uint64] * 3
        lib.synth_fill_host.restype = None
        lib.synth_fill_host.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                        ctypes.c_uint64, ctypes.c_uint64]
        lib.synth_mutate_page_host.restype = None
        lib.synth_mutate_page_host.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                                               ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        lib.synth_mutate_host.restype = None
        lib.synth_mutate_host.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                          ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64,
                                          ctypes.c_uint64]
        _host = lib
    return _host


def dev_lib():
    global _dev
    if _dev is None:
        if not os.path.exists(DEV_SO):
            raise RuntimeError(f"{DEV_SO} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(DEV_SO)
        lib.synth_fill_dev.restype = ctypes.c_int
        lib.synth_fill_dev.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                       ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p]
        lib.synth_mutate_dev.restype = ctypes.c_int
        lib.synth_mutate_dev.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                         ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64,
                                         ctypes.c_uint64, ctypes.c_void_p]
        for nm in ("synth_mutate_frac_dev", "synth_clobber_frac_dev"):
            f = getattr(lib, nm)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                          ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p]
        lib.synth_copy_dev.restype = ctypes.c_int
        lib.synth_copy_dev.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                       ctypes.c_void_p]
        lib.synth_copy2_dev.restype = ctypes.c_int
        lib.synth_copy2_dev.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                        ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_void_p]
        lib.synth_read2_dev.restype = ctypes.c_int
        lib.synth_read2_dev.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                        ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                                        ctypes.c_void_p]
        lib.synth_saxpy_loop.restype = ctypes.c_int
        lib.synth_saxpy_loop.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_float,
                                         ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_void_p]
        _dev = lib
    return _dev


def splitmix_words(seed: int, region: int, j) -> np.ndarray:
    """numpy SplitMix64 output function over counters seed*G + region*R + j (uint64)."""
    j = np.asarray(j, dtype=np.uint64)
    base = np.uint64(((seed * M_GOLD) + (region * M_REGION)) & U64)
    with np.errstate(over="ignore"):
        z = base + j
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def fill_host(nbytes: int, seed: int, region: int, byte_off: int = 0, out=None) -> np.ndarray:
    """Generator bytes [byte_off, byte_off+nbytes) of a region stream, in host memory."""
    if out is None:
        out = np.empty(nbytes, dtype=np.uint8)
    assert out.dtype == np.uint8 and out.flags.c_contiguous and out.size >= nbytes
    host_lib().synth_fill_host(out.ctypes.data, nbytes, seed, region, byte_off)
    return out


def mutate_host(buf: np.ndarray, page_size: int, pages, kind: int, ms: int, region: int) -> None:
    """Apply the page mutation rule to the listed pages of a host region buffer (in place)."""
    pages = np.ascontiguousarray(pages, dtype=np.int64)
    assert buf.dtype == np.uint8 and buf.flags.c_contiguous
    if pages.size:
        assert pages.min() >= 0 and (int(pages.max()) + 1) * page_size <= buf.size
    host_lib().synth_mutate_host(buf.ctypes.data, page_size, pages.ctypes.data, pages.size,
                                 kind, ms, region)


class _SrcRegion(ctypes.Structure):
    _fields_ = [("nbytes", ctypes.c_uint64), ("fill_seed", ctypes.c_uint64),
                ("fill_region", ctypes.c_uint64), ("mutated", ctypes.c_void_p),
                ("n_mutated", ctypes.c_uint64), ("mut_kind", ctypes.c_int32),
                ("has_shadow", ctypes.c_int32)]


class _Src(ctypes.Structure):
    _fields_ = [("page_size", ctypes.c_uint64), ("mut_seed", ctypes.c_uint64),
                ("n_regions", ctypes.c_uint64), ("regions", ctypes.c_void_p)]


class PageSource:
    """A scenario as a C page source (``synth_page_source``): ``fn`` is the
    function's address and ``user`` the address of its argument block, valid
    while this object lives.  Region i of the scenario is source region i."""

    def __init__(self, scn):
        self._lists = [np.ascontiguousarray(r.dirty_pages, dtype=np.int64) for r in scn.regions]
        self._regs = (_SrcRegion * max(1, len(scn.regions)))()
        for i, (r, lst) in enumerate(zip(scn.regions, self._lists)):
            self._regs[i] = _SrcRegion(r.nbytes, r.fill_seed, r.fill_region,
                                       lst.ctypes.data if lst.size else None, lst.size,
                                       r.mut_kind, 1 if r.has_shadow else 0)
        self._src = _Src(scn.page_size, scn.mut_seed, len(scn.regions),
                         ctypes.cast(self._regs, ctypes.c_void_p))
        self.fn = ctypes.cast(host_lib().synth_page_source, ctypes.c_void_p).value
        self.user = ctypes.addressof(self._src)
        self.regions = [(r.nbytes, r.id, bool(r.has_shadow)) for r in scn.regions]
        self.page_size = scn.page_size


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise RuntimeError(f"{what} failed with code {rc}")


def fill_dev(ptr: int, nbytes: int, seed: int, region: int, byte_off: int = 0, stream: int = 0):
    """Fill device memory at ptr (8-byte aligned, nbytes % 8 == 0) with generator bytes."""
    _check(dev_lib().synth_fill_dev(ptr, nbytes, seed, region, byte_off, stream), "synth_fill_dev")


def mutate_dev(ptr: int, region_bytes: int, page_size: int, d_pages_ptr: int, n_pages: int,
               max_page: int, kind: int, ms: int, region: int, stream: int = 0) -> None:
    """Apply the page mutation rule on the device. d_pages_ptr: int64 device array."""
    if n_pages and (max_page + 1) * page_size > region_bytes:
        raise ValueError("mutated page beyond region end")
    _check(dev_lib().synth_mutate_dev(ptr, page_size, d_pages_ptr, n_pages, kind, ms, region,
                                      stream), "synth_mutate_dev")


def frac_threshold(f: float) -> int:
    return min((1 << 64) - 1, int(f * (1 << 64)))


def mutate_frac_dev(ptr: int, nbytes: int, page_size: int, sel_seed: int, frac: float, ms: int,
                    region: int, stream: int = 0) -> None:
    """Word mutation of the pages selected by hash with probability `frac`."""
    _check(dev_lib().synth_mutate_frac_dev(ptr, nbytes, page_size, sel_seed, frac_threshold(frac),
                                           ms, region, stream), "synth_mutate_frac_dev")


def clobber_frac_dev(ptr: int, nbytes: int, page_size: int, sel_seed: int, frac: float,
                     seed: int, region: int, stream: int = 0) -> None:
    """Overwrite the same hash-selected pages with bytes of another stream."""
    _check(dev_lib().synth_clobber_frac_dev(ptr, nbytes, page_size, sel_seed,
                                            frac_threshold(frac), seed, region, stream),
           "synth_clobber_frac_dev")


def copy_dev(dst: int, src: int, nbytes: int, stream: int = 0) -> None:
    """Plain device copy kernel (16-byte aligned pointers and size)."""
    _check(dev_lib().synth_copy_dev(dst, src, nbytes, stream), "synth_copy_dev")


def copy2_dev(dst: int, src: int, nbytes: int, blocks: int, depth: int = 16,
              nt_store: bool = False, stream: int = 0) -> None:
    """Reference streaming copy (nbytes a multiple of 16 KiB)."""
    _check(dev_lib().synth_copy2_dev(dst, src, nbytes, blocks, depth, 1 if nt_store else 0,
                                     stream), "synth_copy2_dev")


def read2_dev(a: int, b: int, nbytes: int, out: int, out_words: int, blocks: int,
              stream: int = 0) -> None:
    """Reference streaming read of two buffers (nbytes a multiple of 16 KiB)."""
    _check(dev_lib().synth_read2_dev(a, b, nbytes, out, out_words, blocks, stream),
           "synth_read2_dev")


def saxpy_loop_dev(y_ptr: int, x_ptr: int, a: float, n: int, iters: int, blocks: int,
                   stream: int) -> None:
    _check(dev_lib().synth_saxpy_loop(y_ptr, x_ptr, a, n, iters, blocks, stream),
           "synth_saxpy_loop")
