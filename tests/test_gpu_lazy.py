"""GPU parity of the on-demand restore (crum_lazy_*): images made by the
oracle, regions starting from their old bytes; after every touch the set of
fetched pages equals the oracle's read-fault model and every page holds
either its restored bytes (fetched) or its old bytes (not fetched); after
finish the regions equal the oracle's restore, byte for byte."""
import numpy as np
import pytest

import oracle
from oracle.lazy import LazyModel
from tests.gpu_util import log, to_dev

pytestmark = pytest.mark.gpu

KiB = 1 << 10


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1808_00117_amd as crum
    crum.lib()
    ctx = crum.crum_ctx_create(0)
    status = torch.zeros(64, dtype=torch.uint8, pin_memory=True)
    yield crum, ctx, status
    crum.crum_ctx_destroy(ctx)


def make_case(counts, P, dirty_frac, seed):
    """Host regions (new bytes, old bytes, id) and the oracle's image of the
    new bytes against the old ones."""
    rng = np.random.default_rng(seed)
    regs = []
    for i, n in enumerate(counts):
        new = rng.integers(0, 256, n * P, dtype=np.uint8)
        old = new.copy()
        for p in range(n):
            if rng.random() < dirty_frac:
                old[p * P + int(rng.integers(0, P))] ^= np.uint8(1 + rng.integers(0, 255))
        regs.append((new, old, 900 + 3 * i))
    st, img, bm = oracle.snapshot(regs, P, seq=77)
    assert st.code == oracle.OK
    return regs, img


def image_pages(img, n_regions, total_pages):
    W = (total_pages + 63) // 64
    bm = np.frombuffer(img[64 + 32 * n_regions: 64 + 32 * n_regions + 8 * W].tobytes(),
                       np.uint64)
    return np.flatnonzero(np.unpackbits(bm.view(np.uint8), bitorder="little"))[:total_pages]


class Session:
    """Device targets holding the old bytes, the pinned image, a lazy session."""

    def __init__(self, crum, ctx, status, regs, img, P, flags, small_bytes, shadows=False,
                 image=None):
        import torch
        self.crum, self.P, self.regs = crum, P, regs
        self.targets = [to_dev(old) for _, old, _ in regs]
        self.shadows = [torch.zeros_like(t) for t in self.targets] if shadows else None
        torch.cuda.synchronize()  # the session's stream does not wait for torch's
        table = [(t.data_ptr(), self.shadows[i].data_ptr() if shadows else 0, t.numel(), rid)
                 for i, (t, (_, _, rid)) in enumerate(zip(self.targets, regs))]
        self.img = img if image is None else image
        self.h = torch.from_numpy(self.img.copy()).pin_memory()
        self.staging = torch.empty(max(self.img.size, 16), dtype=torch.uint8, device="cuda")
        self.stream = torch.cuda.Stream()
        self.status = status
        self.lz = crum.Lazy(ctx, table, self.h.data_ptr(), self.img.size, flags, small_bytes,
                            self.staging.data_ptr(), self.staging.numel(), self.stream.cuda_stream,
                            status.data_ptr())
        self.stream.synchronize()

    def st(self):
        return self.crum.read_status(self.status.data_ptr())

    def touch(self, r, off, ln):
        n = self.lz.touch(r, off, ln, self.stream.cuda_stream, self.status.data_ptr())
        self.stream.synchronize()
        return n

    def finish(self):
        self.lz.finish(self.stream.cuda_stream, self.status.data_ptr())
        self.stream.synchronize()

    def host(self, i):
        return self.targets[i].cpu().numpy()


def check_state(s, model, total_pages):
    """Fetched bitmap equals the model's; each page holds new bytes when
    fetched, old bytes otherwise."""
    W = (total_pages + 63) // 64
    got = s.lz.fetched(W)
    want = model.fetched_bitmap(total_pages)
    assert got == want, "fetched pages differ from the read-fault model"
    P = s.P
    g = 0
    for i, (new, old, _) in enumerate(s.regs):
        t = s.host(i)
        for p in range(new.size // P):
            src = new if (g + p) in model.fetched else old
            assert np.array_equal(t[p * P:(p + 1) * P], src[p * P:(p + 1) * P]), (i, p)
        g += new.size // P


@pytest.mark.parametrize("P,flags", [(4 * KiB, 2), (4 * KiB, 0), (64 * KiB, 2), (256 * KiB, 2)])
def test_touch_sequence_matches_model(env, P, flags):
    crum, ctx, status = env
    counts = (30, 3, 90, 1, 40)
    regs, img = make_case(counts, P, 0.35, seed=P + flags)
    G = sum(counts)
    small = 3 * P
    log(f"[lazy] touch sequence P={P} flags={flags}")
    s = Session(crum, ctx, status, regs, img, P, flags, small)
    assert s.st().code == 0 and s.st().n_dirty == len(image_pages(img, len(counts), G))
    model = LazyModel([n * P for n in counts], P, image_pages(img, len(counts), G), small)
    rng = np.random.default_rng(3)
    for t in range(40):
        r = int(rng.integers(0, len(counts)))
        size = counts[r] * P
        off = int(rng.integers(0, size))
        ln = int(rng.integers(1, min(size - off, 6 * P) + 1))
        want = model.touch(r, off, ln)
        got = s.touch(r, off, ln)
        assert got == want, (t, r, off, ln)
        if got:
            assert s.st().code == 0
        check_state(s, model, G)
    st = s.lz.stats()
    assert st["faults"] == sum(model.faults.values())
    assert st["pages_fetched"] == len(model.fetched)
    s.finish()
    assert s.st().code == 0
    model.finish()
    check_state(s, model, G)
    for i, (new, _, _) in enumerate(regs):
        assert np.array_equal(s.host(i), new)
    st = s.lz.stats()
    assert st["pages_fetched"] == st["pages_total"] and st["bytes_fetched"] == st["pages_total"] * P
    s.lz.close()


def test_sequential_sweep_doubles(env):
    """An all-dirty region swept page by page: fetches of 1, 2, 4, ... pages,
    ceil(log2(n + 1)) faults, one copy per fault."""
    crum, ctx, status = env
    P, n = 4 * KiB, 300
    rng = np.random.default_rng(9)
    new = rng.integers(0, 256, n * P, dtype=np.uint8)
    old = new.copy()
    old[::P] ^= 1
    st, img, _ = oracle.snapshot([(new, old, 1)], P)
    assert st.n_dirty == n
    s = Session(crum, ctx, status, [(new, old, 1)], img, P, crum.CRUM_VERIFY, 0)
    got = [s.touch(0, p * P, P) for p in range(n)]
    sizes = [k for k in got if k]
    assert sizes[:-1] == [1 << i for i in range(len(sizes) - 1)]
    assert sum(sizes) == n and len(sizes) == int(np.ceil(np.log2(n + 1)))
    stt = s.lz.stats()
    assert stt["faults"] == len(sizes) and stt["copies"] == len(sizes)
    assert np.array_equal(s.host(0), new)
    s.lz.close()


def test_update_shadow_writes_fetched_pages_only(env):
    crum, ctx, status = env
    P = 16 * KiB
    regs, img = make_case((20, 12), P, 0.5, seed=21)
    s = Session(crum, ctx, status, regs, img, P, crum.CRUM_VERIFY | crum.CRUM_UPDATE_SHADOW, 0,
                shadows=True)
    model = LazyModel([20 * P, 12 * P], P, image_pages(img, 2, 32), 0)
    for r, off, ln in [(0, 3 * P + 5, 10), (1, 0, 2 * P), (0, 11 * P, 3 * P)]:
        assert s.touch(r, off, ln) == model.touch(r, off, ln)
    g = 0
    for i, (new, _, _) in enumerate(regs):
        sh = s.shadows[i].cpu().numpy()
        for p in range(new.size // P):
            want = new[p * P:(p + 1) * P] if g + p in model.fetched else 0
            assert np.all(sh[p * P:(p + 1) * P] == want), (i, p)
        g += new.size // P
    s.lz.close()


@pytest.mark.parametrize("P", [4 * KiB, 64 * KiB])
def test_corrupt_page_stops_the_session(env, P):
    crum, ctx, status = env
    regs, img = make_case((64,), P, 1.0, seed=5)   # every page in the image: slot = page
    bad = img.copy()
    data_off = 4096
    bad[data_off + 20 * P + 9] ^= 0x10             # slot 20
    s = Session(crum, ctx, status, regs, img, P, crum.CRUM_VERIFY, 0, image=bad)
    new, old, _ = regs[0]
    assert s.touch(0, 0, 4 * P) == 4               # pages 0..3: fine
    assert s.st().code == 0
    assert s.touch(0, 18 * P, P) == 2              # window of 2 pages: 18, 19
    assert s.st().code == 0
    n = s.touch(0, 20 * P, P)                      # 4-page window 20..23 holds slot 20
    assert n == 4
    st = s.st()
    assert st.code == crum.CRUM_ECRC and st.first_bad == 20, st
    t = s.host(0)
    assert np.array_equal(t[:4 * P], new[:4 * P])
    assert np.array_equal(t[18 * P:20 * P], new[18 * P:20 * P])
    assert np.array_equal(t[20 * P:24 * P], old[20 * P:24 * P])   # the failed run: not written
    assert s.touch(0, 40 * P, P) == 8              # later fetches write nothing
    assert s.st().code == crum.CRUM_ECRC
    s.finish()
    assert s.st().code == crum.CRUM_ECRC
    assert np.array_equal(s.host(0)[24 * P:], old[24 * P:])
    res = oracle.restore([(old.copy(), None, regs[0][2])], bad, oracle.VERIFY)
    assert res.code == oracle.ECRC and res.first_bad == 20
    s.lz.close()


def test_image_errors(env):
    import torch
    crum, ctx, status = env
    P = 4 * KiB
    regs, img = make_case((10, 6), P, 0.5, seed=61)
    # host-side refusals: nothing is created
    for pos in [0, 9, 13, 17, 25, 33, 49]:
        bad = img.copy()
        bad[pos] ^= 0x04
        with pytest.raises(crum.ImageError):
            Session(crum, ctx, status, regs, img, P, crum.CRUM_VERIFY, 0, image=bad)
    wrong = [(regs[0][0], regs[0][1], 4242), regs[1]]
    with pytest.raises(crum.ImageError) as e:
        Session(crum, ctx, status, wrong, img, P, crum.CRUM_VERIFY, 0)
    assert e.value.code == crum.CRUM_EMISMATCH
    # a bitmap bit flipped: the popcount no longer matches n_dirty (host)
    bad = img.copy()
    bad[64 + 32 * 2] ^= 0x80
    with pytest.raises(crum.ImageError) as e:
        Session(crum, ctx, status, regs, img, P, crum.CRUM_VERIFY, 0, image=bad)
    assert e.value.code == crum.CRUM_EFORMAT
    # meta_crc and crcs_crc are checked on the device: open succeeds, every
    # call reports EFORMAT and nothing is written
    for pos in (57, 61):
        bad = img.copy()
        bad[pos] ^= 0x01
        s = Session(crum, ctx, status, regs, img, P, crum.CRUM_VERIFY, 0, image=bad)
        assert s.st().code == crum.CRUM_EFORMAT
        s.touch(0, 0, 10 * P)
        assert s.st().code == crum.CRUM_EFORMAT
        s.finish()
        assert s.st().code == crum.CRUM_EFORMAT
        for i, (_, old, _) in enumerate(regs):
            assert np.array_equal(s.host(i), old)
        s.lz.close()
    # staging too small
    t = [to_dev(old) for _, old, _ in regs]
    table = [(x.data_ptr(), 0, x.numel(), rid) for x, (_, _, rid) in zip(t, regs)]
    h = torch.from_numpy(img).pin_memory()
    stg = torch.empty(img.size, dtype=torch.uint8, device="cuda")
    with pytest.raises(crum.ImageError) as e:
        crum.Lazy(ctx, table, h.data_ptr(), img.size, 2, 0, stg.data_ptr(), img.size - 1, 0,
                  status.data_ptr())
    assert e.value.code == crum.CRUM_ENOSPC


def test_argument_errors_and_empty_image(env):
    crum, ctx, status = env
    P = 4 * KiB
    regs, img = make_case((8, 4), P, 0.0, seed=7)   # nothing dirty: D = 0
    s = Session(crum, ctx, status, regs, img, P, crum.CRUM_VERIFY, 0)
    assert s.st().code == 0 and s.st().n_dirty == 0
    assert s.touch(0, 0, 8 * P) == 0 and s.touch(1, 5, 1) == 0
    for args in [(2, 0, 1), (0, 0, 0), (0, 8 * P, 1), (1, 1, 4 * P), (0, 2**63, 2**63)]:
        with pytest.raises(ValueError):
            s.lz.touch(*args, s.stream.cuda_stream, s.status.data_ptr())
    s.finish()
    assert s.st().code == 0
    for i, (_, old, _) in enumerate(regs):
        assert np.array_equal(s.host(i), old)
    assert s.lz.stats() == {"pages_total": 0, "pages_fetched": 0, "faults": 0, "copies": 0,
                            "bytes_fetched": 0}
    s.lz.close()


def test_sessions_at_once_on_one_context(env):
    """Two sessions open together on one context (the first uses the
    context's scratch, the second its own), interleaved touches, both end as
    the oracle's restore; a third session afterwards reuses the scratch."""
    crum, ctx, status = env
    P = 4 * KiB
    cases = [make_case((30, 12), P, 0.4, seed=81), make_case((7, 50), P, 0.4, seed=82),
             make_case((64,), P, 0.3, seed=83)]
    a = Session(crum, ctx, status, *cases[0], P, crum.CRUM_VERIFY, 0)
    b = Session(crum, ctx, status, *cases[1], P, crum.CRUM_VERIFY, 0)
    ma = LazyModel([30 * P, 12 * P], P, image_pages(cases[0][1], 2, 42), 0)
    mb = LazyModel([7 * P, 50 * P], P, image_pages(cases[1][1], 2, 57), 0)
    for r, off, ln in [(0, 0, 3 * P), (1, 5 * P, P), (0, 20 * P, 4 * P), (1, 0, 12 * P)]:
        assert a.touch(r, off, ln) == ma.touch(r, off, ln)
        assert b.touch(1 - r, off % (7 * P), P) == mb.touch(1 - r, off % (7 * P), P)
        check_state(a, ma, 42)
        check_state(b, mb, 57)
    for s, m, (regs, _) in ((a, ma, cases[0]), (b, mb, cases[1])):
        s.finish()
        assert s.st().code == 0
        for i, (new, _, _) in enumerate(regs):
            assert np.array_equal(s.host(i), new)
        s.lz.close()
    c = Session(crum, ctx, status, *cases[2], P, crum.CRUM_VERIFY, 0)
    c.finish()
    assert c.st().code == 0 and np.array_equal(c.host(0), cases[2][0][0][0])
    c.lz.close()


def test_empty_region_table(env):
    """An image of no regions: open succeeds, every touch is an argument
    error, finish has nothing to fetch."""
    import torch
    crum, ctx, status = env
    P = 4 * KiB
    st, img, _ = oracle.snapshot([], P)
    assert st.code == oracle.OK and st.total_pages == 0
    h = torch.from_numpy(img.copy()).pin_memory()
    stg = torch.empty(img.size, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    lz = crum.Lazy(ctx, [], h.data_ptr(), img.size, crum.CRUM_VERIFY, 0, stg.data_ptr(),
                   img.size, stream.cuda_stream, status.data_ptr())
    stream.synchronize()
    assert crum.read_status(status.data_ptr()).code == 0
    with pytest.raises(ValueError):
        lz.touch(0, 0, 1, stream.cuda_stream)
    lz.finish(stream.cuda_stream, status.data_ptr())
    stream.synchronize()
    assert crum.read_status(status.data_ptr()).code == 0
    assert lz.fetched(0) == [] and lz.stats()["pages_total"] == 0
    lz.close()


def test_touch_orders_other_streams(env):
    """A page fetched on one stream and touched (no fault) on another: work
    queued after the second touch on the second stream sees the page."""
    import torch
    crum, ctx, status = env
    P = 64 * KiB
    regs, img = make_case((512,), P, 1.0, seed=13)
    s = Session(crum, ctx, status, regs, img, P, crum.CRUM_VERIFY, 0)
    other = torch.cuda.Stream()
    out = torch.empty(regs[0][0].size, dtype=torch.uint8, device="cuda")
    n = s.lz.touch(0, 0, 512 * P, s.stream.cuda_stream, 0)   # one 32 MiB window
    assert n == 512
    assert s.lz.touch(0, 0, 512 * P, other.cuda_stream, 0) == 0
    with torch.cuda.stream(other):
        out.copy_(s.targets[0])
    other.synchronize()
    assert np.array_equal(out.cpu().numpy(), regs[0][0])
    s.lz.close()


def test_property_sessions(env):
    """Drawn sessions (0-5 regions of 0-60 pages, 4-64 KiB pages, dirty
    density, small-region size, with or without verification and shadow
    update, 0-25 touches of drawn ranges): after every touch the fetched
    pages equal the model's, and after finish the regions (and shadows)
    equal the oracle's restore.  Derandomized."""
    from hypothesis import HealthCheck, given, settings
    from hypothesis import strategies as st
    crum, ctx, status = env

    @settings(max_examples=20, deadline=None, derandomize=True,
              suppress_health_check=list(HealthCheck))
    @given(counts=st.lists(st.integers(0, 60), min_size=0, max_size=5),
           pshift=st.sampled_from([12, 14, 16]),
           density=st.sampled_from([0.0, 0.1, 0.5, 1.0]),
           small_pages=st.sampled_from([0, 1, 4, 1000]),
           flags=st.sampled_from([0, 2, 3]),
           seed=st.integers(0, 2**31 - 1),
           touches=st.lists(st.tuples(st.integers(0, 4), st.floats(0, 1), st.floats(0, 1)),
                            max_size=25))
    def run(counts, pshift, density, small_pages, flags, seed, touches):
        P = 1 << pshift
        regs, img = make_case(tuple(counts), P, density, seed)
        G = sum(counts)
        small = small_pages * P
        s = Session(crum, ctx, status, regs, img, P, flags, small, shadows=bool(flags & 1))
        assert s.st().code == 0
        model = LazyModel([n * P for n in counts], P, image_pages(img, len(counts), G), small)
        for r, a, b in touches:
            if not counts or counts[r % len(counts)] == 0:
                continue
            r %= len(counts)
            size = counts[r] * P
            off = min(int(a * size), size - 1)
            ln = max(1, min(int(b * 3 * P), size - off))
            assert s.touch(r, off, ln) == model.touch(r, off, ln)
            assert s.lz.fetched((G + 63) // 64) == model.fetched_bitmap(G)
        s.finish()
        assert s.st().code == 0
        model.finish()
        check_state(s, model, G)
        if flags & 1:
            g = 0
            for i, (new, _, _) in enumerate(regs):
                sh = s.shadows[i].cpu().numpy()
                for p in range(counts[i]):
                    want = new[p * P:(p + 1) * P] if g + p in model.fetched else 0
                    assert np.all(sh[p * P:(p + 1) * P] == want)
                g += counts[i]
        s.lz.close()

    run()
