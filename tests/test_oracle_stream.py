"""Pin the oracle's streamed-input snapshot (region bytes handed in one page
at a time by a source) to things other than itself:

* the pure-Python brute force, on tiny scenarios small enough for it;
* the in-memory oracle on the same scenarios materialised whole, over every
  workload shape the GPU tests stream (many allocations with clustered runs,
  256-byte spans on 2 MiB pages, batched requests of 4 KiB and 64 KiB pages,
  a region without shadow, zero-length regions);
* the scenario's chosen dirty set (each mutation changes bytes), so a page
  dropped or added by either pass fails;
* ENOSPC with the needed size, and a failing source reported as EINVAL.
"""
import ctypes

import numpy as np
import pytest

import oracle
from oracle import brute
from synth import scenarios as sc
from synth.lib import PageSource

KiB, MiB = 1 << 10, 1 << 20


def _materialised(scn):
    regs = []
    for i, r in enumerate(scn.regions):
        c, s = sc.materialize_host(scn, i)
        regs.append((c, s, r.id))
    return regs


def _stream(scn, seq=0, image_cap=None):
    src = PageSource(scn)
    return oracle.snapshot_stream(src.regions, scn.page_size, src.fn, src.user, seq=seq,
                                  image_cap=image_cap)


def _bits(bitmap, G):
    return np.flatnonzero(np.unpackbits(bitmap.view(np.uint8), bitorder="little")[:G])


def test_stream_equals_brute_force_on_tiny_scenarios():
    rng = np.random.default_rng(5)
    for trial in range(6):
        P = 4 * KiB
        counts = [int(c) for c in rng.integers(0, 5, size=int(rng.integers(1, 4)))]
        regs = []
        for i, n in enumerate(counts):
            dp = np.sort(rng.choice(max(n, 1), size=int(rng.integers(0, n + 1)),
                                    replace=False)).astype(np.int64) if n else np.zeros(0, np.int64)
            regs.append(sc.RegionSpec(id=40 + i, nbytes=n * P, fill_seed=77, fill_region=i,
                                      dirty_pages=dp, mut_kind=trial % 2,
                                      has_shadow=not (trial == 3 and i == 0)))
        scn = sc.Scenario("tiny", 77, P, 99, regs)
        st, img, bm = _stream(scn, seq=trial)
        assert st.code == oracle.OK
        host = [(c.tobytes(), None if s is None else s.tobytes(), rid)
                for c, s, rid in _materialised(scn)]
        bimg, dirty_g = brute.snapshot(host, P, seq=trial)
        assert img.tobytes() == bimg
        assert list(_bits(bm, scn.total_pages)) == list(dirty_g)
        assert list(dirty_g) == list(scn.dirty_global())


@pytest.mark.parametrize("name", ["many", "managed", "batched4k", "batched64k", "noshadow"])
def test_stream_equals_in_memory_oracle(name):
    if name == "many":
        scn = sc.many_allocs(total=96 * MiB)
    elif name == "managed":
        scn = sc.managed(nbytes=64 * MiB)
    elif name.startswith("batched"):
        reqs = sc.batched(seed=1004, n_requests=40, max_total=24 * MiB)
        want = 4 * KiB if name == "batched4k" else 64 * KiB
        scn = next(r for r in reqs if r.page_size == want and len(r.regions) > 2)
    else:
        scn = sc.many_allocs(n=5, total=8 * MiB)
        scn.regions[2].has_shadow = False
        scn.regions.insert(1, sc.RegionSpec(id=1, nbytes=0, fill_seed=1, fill_region=99,
                                            dirty_pages=np.zeros(0, np.int64)))
    st, img, bm = _stream(scn, seq=31)
    st2, img2, bm2 = oracle.snapshot(_materialised(scn), scn.page_size, seq=31)
    assert st == st2 and st.code == oracle.OK
    assert np.array_equal(img, img2) and np.array_equal(bm, bm2)
    assert np.array_equal(_bits(bm, scn.total_pages), scn.dirty_global())
    assert st.n_dirty == scn.n_dirty


def test_stream_enospc_and_failing_source():
    scn = sc.many_allocs(n=4, total=4 * MiB)
    st_full, img, _ = _stream(scn)
    st, img2, bm = _stream(scn, image_cap=st_full.image_bytes - 1)
    assert st.code == oracle.ENOSPC and img2.size == 0
    assert st.image_bytes == st_full.image_bytes and st.n_dirty == st_full.n_dirty
    assert np.array_equal(_bits(bm, scn.total_pages), scn.dirty_global())

    calls = []

    @ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64,
                      ctypes.c_void_p, ctypes.c_void_p)
    def failing(user, region, page, cur, shadow):
        calls.append((region, page))
        return -1 if len(calls) == 3 else 0
    regions = [(r.nbytes, r.id, True) for r in scn.regions]
    st, img3, _ = oracle.snapshot_stream(regions, scn.page_size,
                                         ctypes.cast(failing, ctypes.c_void_p).value, 0)
    assert st.code == oracle.EINVAL and img3.size == 0 and len(calls) == 3


def test_stream_argument_errors():
    src = PageSource(sc.many_allocs(n=2, total=2 * MiB))
    st, _, _ = oracle.snapshot_stream([(3 * 4096, 1, True)], 8192, src.fn, src.user)
    assert st.code == oracle.EINVAL
    st, _, _ = oracle.snapshot_stream([(8192, 1, True)], 3000, src.fn, src.user)
    assert st.code == oracle.EINVAL
