"""Invariants of the oracle that follow from the definitions and the paper:
restore(S, snap(X, S)) == X (section 3.4, restart copies saved data back);
snap(X, X) is empty; a missing shadow captures every page (a new shadow region
starts all-dirty, section 3.2); after a shadow update a re-snapshot is empty
(Algorithm 1, dirty flags cleared after a flush); n_dirty == popcount(bitmap);
ENOSPC writes nothing; argument errors are EINVAL."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle

P = 4096


def _mk(rng, counts, p_dirty):
    regs = []
    for rid, n in enumerate(counts):
        cur = rng.integers(0, 256, n * P, dtype=np.uint8)
        sh = cur.copy()
        for i in range(n):
            if rng.random() < p_dirty:
                k = int(rng.integers(1, 9))
                pos = rng.integers(0, P, k)
                sh[i * P + pos] ^= rng.integers(1, 256, k).astype(np.uint8)
        regs.append((cur, sh, rid * 11 + 1))
    return regs


counts_st = st.lists(st.integers(0, 9), min_size=0, max_size=5)


@settings(max_examples=40, deadline=None)
@given(counts=counts_st, seed=st.integers(0, 2**31), p=st.floats(0, 1))
def test_restore_of_snapshot_is_identity(counts, seed, p):
    rng = np.random.default_rng(seed)
    regs = _mk(rng, counts, p)
    s, img, bm = oracle.snapshot(regs, P)
    assert s.code == oracle.OK
    assert s.n_dirty == int(sum(bin(int(w)).count("1") for w in bm))
    dst = [(sh.copy(), None, rid) for _, sh, rid in regs]
    r = oracle.restore(dst, img, flags=oracle.VERIFY)
    assert r.code == oracle.OK
    for (d, _, _), (c, _, _) in zip(dst, regs):
        assert np.array_equal(d, c)


@settings(max_examples=25, deadline=None)
@given(counts=counts_st, seed=st.integers(0, 2**31))
def test_identical_shadow_is_empty_and_null_shadow_is_full(counts, seed):
    rng = np.random.default_rng(seed)
    regs = _mk(rng, counts, 0.0)
    s, img, bm = oracle.snapshot(regs, P)
    assert s.code == oracle.OK and s.n_dirty == 0 and not bm.any()
    assert len(img) == oracle.prefix_bytes(len(regs), s.total_pages)
    full = [(c, None, rid) for c, _, rid in regs]
    s2, img2, bm2 = oracle.snapshot(full, P)
    assert s2.n_dirty == s2.total_pages == sum(counts)


@settings(max_examples=25, deadline=None)
@given(counts=counts_st, seed=st.integers(0, 2**31), p=st.floats(0, 1))
def test_update_shadow_then_resnapshot_is_empty(counts, seed, p):
    rng = np.random.default_rng(seed)
    regs = _mk(rng, counts, p)
    s, _, _ = oracle.snapshot(regs, P, flags=oracle.UPDATE_SHADOW)
    assert s.code == oracle.OK
    for c, sh, _ in regs:
        assert np.array_equal(c, sh)
    s2, _, _ = oracle.snapshot(regs, P)
    assert s2.n_dirty == 0


def test_enospc_writes_nothing_and_reports_counts():
    rng = np.random.default_rng(3)
    regs = _mk(rng, (5, 5), 0.5)
    before = [sh.copy() for _, sh, _ in regs]
    s0, img0, bm0 = oracle.snapshot(regs, P)
    D = s0.n_dirty
    assert D >= 2
    s, img, bm = oracle.snapshot(regs, P, flags=oracle.UPDATE_SHADOW, staging_cap=(D - 1) * P)
    assert s.code == oracle.ENOSPC and s.n_dirty == D and img.size == 0
    assert np.array_equal(bm, bm0)
    for (_, sh, _), b in zip(regs, before):
        assert np.array_equal(sh, b)
    s, img, bm = oracle.snapshot(regs, P, image_cap=s0.image_bytes - 1)
    assert s.code == oracle.ENOSPC and s.image_bytes == s0.image_bytes
    s, img, bm = oracle.snapshot(regs, P, staging_cap=D * P, image_cap=s0.image_bytes)
    assert s.code == oracle.OK


def test_invalid_arguments():
    rng = np.random.default_rng(4)
    cur = rng.integers(0, 256, 4 * P, dtype=np.uint8)
    sh = cur.copy()
    good = [(cur, sh, 1)]
    assert oracle.validate(good, P) == oracle.OK
    for bad_p in [0, 2048, 4096 + 1, 3 * 4096, (1 << 30) * 2]:
        assert oracle.validate(good, bad_p) == oracle.EINVAL
    assert oracle.validate([(cur[: 3 * P + 16], None, 1)], P) == oracle.EINVAL  # len % P
    a = cur.ctypes.data
    assert oracle.validate([(a + 8, 0, P, 1)], P) == oracle.EINVAL           # misaligned
    assert oracle.validate([(a, 0, 2 * P, 1), (a + P, 0, P, 2)], P) == oracle.EINVAL
    assert oracle.validate([(a, a + P, 2 * P, 1)], P) == oracle.EINVAL     # cur/shadow overlap
    assert oracle.validate([(a, 0, P, 1), (a + 2 * P, a, P, 2)], P) == oracle.EINVAL
    assert oracle.validate([(0, 0, P, 1)], P) == oracle.EINVAL             # NULL current
    assert oracle.validate([(a, 0, 0, 1), (a, 0, 0, 2)], P) == oracle.OK   # empty never overlaps
    s, _, _ = oracle.snapshot(good, P, image_cap=100)
    assert s.code == oracle.EINVAL                                          # prefix does not fit
