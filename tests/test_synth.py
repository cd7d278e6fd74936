"""Synthetic-input generators: the numpy, host-C (and, on a GPU, HIP) byte
generators agree; scenario shapes match the stated workloads; the oracle's
dirty set equals the scenario's chosen page set."""
import numpy as np
import pytest

import oracle
import synth
from synth import scenarios as sc


@pytest.mark.parametrize("off,n", [(0, 64), (3, 100), (8, 8), (4093, 9000), (1 << 33, 40)])
def test_host_fill_matches_numpy(off, n):
    a = synth.fill_host(n, 1234, 7, off)
    j0, j1 = off // 8, (off + n + 7) // 8
    w = synth.splitmix_words(1234, 7, np.arange(j0, j1, dtype=np.uint64))
    b = w.view(np.uint8)[off - 8 * j0: off - 8 * j0 + n]
    assert np.array_equal(a, b)


def test_splitmix_reference_values():
    # SplitMix64 seeded with 0 yields, as its first outputs, mix(G), mix(2G), ...
    # where G is the golden-ratio increment; the published first output of the
    # generator seeded with 0 is 0xE220A8397B1DCDAF.
    assert int(synth.splitmix_words(1, 0, 0)) == 0xE220A8397B1DCDAF
    assert synth.host_lib().synth_word(1, 0, 0) == 0xE220A8397B1DCDAF


@pytest.mark.parametrize("kind,P", [(0, 4096), (0, 65536), (1, 4096), (1, 2 << 20)])
def test_mutation_changes_only_chosen_pages(kind, P):
    n = 6
    cur = synth.fill_host(n * P, 5, 2)
    sh = cur.copy()
    pages = np.array([0, 3, 5], np.int64)
    synth.mutate_host(sh, P, pages, kind, 99, 2)
    for p in range(n):
        d = np.flatnonzero(cur[p * P:(p + 1) * P] != sh[p * P:(p + 1) * P])
        if p in pages:
            assert d.size > 0
            if kind == 0:
                words = np.unique(d // 4)
                assert 1 <= words.size <= 16
            else:
                assert d.max() - d.min() < 256
        else:
            assert d.size == 0


def test_plain_scenario_shape():
    s = sc.plain()
    assert s.total_bytes == 64 << 20 and s.page_size == 4096 and s.total_pages == 16384
    assert s.n_dirty == 819
    assert np.unique(s.regions[0].dirty_pages).size == 819


def test_many_allocs_shape():
    s = sc.many_allocs()
    assert len(s.regions) == 64
    assert s.total_bytes == 16 << 30
    assert all(r.nbytes % (64 << 10) == 0 and r.nbytes > 0 for r in s.regions)
    frac = s.n_dirty / s.total_pages
    assert 0.05 < frac < 0.15, frac
    raw = sc.many_allocs(total=None)
    assert all(4096 <= r.nbytes <= (1 << 30) for r in raw.regions)


def test_managed_shape():
    s = sc.managed()
    assert s.total_pages == 16384 and s.n_dirty == 3277
    assert s.meta["device_pages"].size == 4915


def test_batched_shape():
    reqs = sc.batched(n_requests=256)
    assert len(reqs) == 256
    for r in reqs:
        assert r.page_size in (4096, 65536)
        assert 1 <= len(r.regions) <= 32
        assert (1 << 20) // 2 <= r.total_bytes <= (2 << 30) + r.page_size
    tot = sum(r.total_bytes for r in reqs)
    assert 20e9 < tot < 200e9, tot


def test_oracle_dirty_set_equals_scenario_choice():
    s = sc.many_allocs(seed=77, n=6, page_size=4096, total=6 * 4096 * 64, start_p=0.02,
                       mean_run=4)
    regs = []
    for i, r in enumerate(s.regions):
        cur, sh = sc.materialize_host(s, i)
        regs.append((cur, sh, r.id))
    st, img, bm = oracle.snapshot(regs, s.page_size)
    assert st.code == oracle.OK
    got = np.flatnonzero(np.unpackbits(bm.view(np.uint8), bitorder="little"))
    assert np.array_equal(got, s.dirty_global())


def test_host_page_matches_region():
    s = sc.managed(seed=5, nbytes=8 << 20, page_size=2 << 20, dirty_frac=0.5)
    cur, sh = sc.materialize_host(s, 0)
    P = s.page_size
    for p in range(4):
        assert np.array_equal(sc.host_page(s, 0, p, False), cur[p * P:(p + 1) * P])
        assert np.array_equal(sc.host_page(s, 0, p, True), sh[p * P:(p + 1) * P])
