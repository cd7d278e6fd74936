"""Pin the C oracle against the pure-Python brute force on tiny images:
every dirty subset of up to 10 pages, bitmap-word straddles, multi-region
tables, a missing shadow, and the image bytes themselves."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import brute

P = 4096


def _make(counts, seed, dirty, where="random", with_shadow=True):
    """Regions with page counts `counts`; shadow differs exactly on global pages `dirty`."""
    rng = np.random.default_rng(seed)
    curs = [rng.integers(0, 256, n * P, dtype=np.uint8) for n in counts]
    rng = np.random.default_rng(seed + 1_000_003 * (1 + len(dirty)))
    regs = []
    g = 0
    for rid, (n, cur) in enumerate(zip(counts, curs)):
        sh = cur.copy()
        for i in range(n):
            if g + i in dirty:
                off = {"first": 0, "last": P - 1}.get(where, int(rng.integers(0, P)))
                sh[i * P + off] ^= np.uint8(1 + rng.integers(0, 255))
        g += n
        regs.append((cur, sh if with_shadow else None, 1000 + rid))
    return regs


def _compare(regs, seq=7):
    st, img, bitmap = oracle.snapshot(regs, P, seq=seq)
    assert st.code == oracle.OK
    bimg, dirty_g = brute.snapshot([(c.tobytes(), None if s is None else s.tobytes(), rid)
                                    for c, s, rid in regs], P, seq=seq)
    assert img.tobytes() == bimg
    assert st.n_dirty == len(dirty_g)
    got = [g for g in range(st.total_pages) if (int(bitmap[g // 64]) >> (g % 64)) & 1]
    assert got == dirty_g
    return dirty_g


@pytest.mark.parametrize("counts", [(10,), (3, 1, 6), (0, 4, 0, 2, 4)])
def test_every_dirty_subset(counts):
    G = sum(counts)
    assert G <= 10
    regs = _make(counts, 1, set())
    base = {rid: c for c, _, rid in regs}
    n_checked = 0
    for mask in range(1 << G):
        dirty = {g for g in range(G) if (mask >> g) & 1}
        where = ["first", "last", "random"][mask % 3]
        rs = _make(counts, 1, dirty, where)
        for (c, _, rid) in rs:
            assert np.array_equal(c, base[rid])
        got = _compare(rs)
        assert got == sorted(dirty)
        n_checked += 1
    assert n_checked == 1 << G


@pytest.mark.parametrize("counts", [(64,), (63, 2), (1, 64, 65), (130,)])
def test_word_straddles(counts):
    G = sum(counts)
    rng = np.random.default_rng(G)
    for trial in range(3):
        dirty = set(int(x) for x in rng.choice(G, size=int(rng.integers(0, G + 1)),
                                               replace=False))
        dirty |= {0, G - 1} if trial == 2 else set()
        got = _compare(_make(counts, trial, dirty))
        assert got == sorted(dirty)


def test_missing_shadow_means_all_dirty():
    regs = _make((3, 2), 5, set(), with_shadow=False)
    got = _compare(regs)
    assert got == list(range(5))
    _, img, _ = oracle.snapshot(regs, P)
    rc, h = oracle.parse(img)
    assert rc == oracle.OK and h["flags"] == 1


def test_mixed_shadow_flag():
    regs = _make((2, 2), 6, {1})
    regs[1] = (regs[1][0], None, regs[1][2])
    got = _compare(regs)
    assert got == [1, 2, 3]
    _, img, _ = oracle.snapshot(regs, P)
    assert oracle.parse(img)[1]["flags"] == 0


def test_empty_table_and_zero_length_regions():
    for regs in ([], [(np.zeros(0, np.uint8), None, 3)]):
        st, img, bm = oracle.snapshot(regs, P, seq=2)
        assert st.code == oracle.OK and st.total_pages == 0 and st.n_dirty == 0
        bimg, _ = brute.snapshot([(c.tobytes(), None, rid) for c, _, rid in regs], P, seq=2)
        assert img.tobytes() == bimg
        assert len(img) == 4096


def test_restore_brute_matches_oracle():
    rng = np.random.default_rng(9)
    counts = (3, 5, 2)
    for trial in range(4):
        dirty = set(int(x) for x in rng.choice(10, size=int(rng.integers(0, 11)),
                                               replace=False))
        regs = _make(counts, trial, dirty)
        _, img, _ = oracle.snapshot(regs, P)
        # oracle restore into the shadows, brute restore into copies of the shadows
        targets = [(s.copy(), None, rid) for _, s, rid in regs]
        st = oracle.restore(targets, img)
        assert st.code == oracle.OK
        btargets = [(bytearray(s.tobytes()), rid) for _, s, rid in regs]
        brute.restore(btargets, img.tobytes())
        for (t, _, _), (bt, _), (c, _, _) in zip(targets, btargets, regs):
            assert t.tobytes() == bytes(bt) == c.tobytes()
