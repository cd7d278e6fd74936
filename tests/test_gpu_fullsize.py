"""GPU parity at the benchmark workloads' full sizes, in the launch
configuration bench.py times (default context shapes, the chunk-pipelined
order where the capacity allows it).  The regions are tens of GB, so the
oracle takes their bytes one page at a time (``oracle.snapshot_stream`` over
the scenario regenerated on the host by ``synth.lib.PageSource``) and its
whole image is compared with the GPU's byte for byte: header, region table,
bitmap, every packed page, every CRC, both checksums.  Besides:

* the bitmap equals the scenario's chosen dirty set (each chosen page differs
  from its shadow by construction, every other page is equal);
* the oracle's parser accepts the image (magic, layout, popcount, both
  checksums, length);
* the diff-first order gives the same image byte for byte;
* a restore repairs pages overwritten on the device.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from tests.gpu_util import log

pytestmark = pytest.mark.gpu

KiB, MiB, GiB = 1 << 10, 1 << 20, 1 << 30


def page_index(scn):
    """(region index, local page) of every global page, as two arrays."""
    P = scn.page_size
    counts = np.array([r.nbytes // P for r in scn.regions], np.int64)
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    return counts, starts


def check_image(img, scn, n_samples, rng, seq):
    """Layout, bitmap and sampled pages of one image against the scenario."""
    from synth import scenarios as sc
    P = scn.page_size
    rc, hdr = oracle.parse(img)
    assert rc == oracle.OK, rc
    assert hdr["n_dirty"] == scn.n_dirty and hdr["total_pages"] == scn.total_pages
    assert hdr["page_size"] == P and hdr["seq"] == seq
    R = len(scn.regions)
    W = (scn.total_pages + 63) // 64
    bm = np.frombuffer(img[64 + 32 * R: 64 + 32 * R + 8 * W].tobytes(), np.uint64)
    got = np.flatnonzero(np.unpackbits(bm.view(np.uint8), bitorder="little"))
    want = scn.dirty_global()
    assert np.array_equal(got, want), "bitmap differs from the chosen dirty set"
    counts, starts = page_index(scn)
    D, off = scn.n_dirty, hdr["data_off"]
    crcs = np.frombuffer(img[off + D * P: off + D * P + 4 * D].tobytes(), np.uint32)
    for k in rng.choice(D, size=min(n_samples, D), replace=False):
        g = int(want[k])
        ri = int(np.searchsorted(starts, g, side="right") - 1)
        page = sc.host_page(scn, ri, g - int(starts[ri]), shadow=False)
        assert np.array_equal(img[off + k * P: off + (k + 1) * P], page), f"slot {k}"
        assert int(crcs[k]) == oracle.crc32c(page), f"crc of slot {k}"


def oracle_image(scn, seq):
    """The oracle's image of a scenario, region bytes streamed page by page."""
    from synth.lib import PageSource
    src = PageSource(scn)
    st, img, _ = oracle.snapshot_stream(src.regions, scn.page_size, src.fn, src.user, seq=seq)
    assert st.code == oracle.OK and st.n_dirty == scn.n_dirty, st
    return img


def assert_same_image(got, want, what):
    """Byte-for-byte equality; on failure, name the first differing byte's
    part of the image."""
    if got.size == want.size and np.array_equal(got, want):
        return
    n = min(got.size, want.size)
    diff = np.flatnonzero(got[:n] != want[:n])
    first = int(diff[0]) if diff.size else n
    raise AssertionError(f"{what}: images differ (sizes {got.size}/{want.size}, "
                         f"first differing byte {first}, {diff.size} bytes differ)")


@pytest.mark.timeout(900)
def test_many_allocs_16gib():
    """The 16 GiB many-allocations workload (64 regions, 64 KiB pages)."""
    import bench
    import paper_1808_00117_amd as crum
    import paper_1808_00117_amd.hip as H
    import synth
    from synth import scenarios as sc

    scn = sc.many_allocs()
    P, G, D, R = scn.page_size, scn.total_pages, scn.n_dirty, len(scn.regions)
    log(f"[fullsize] many_allocs N={scn.total_bytes} D={D}")
    pairs = bench.materialize_raw(scn, H)
    table = crum.region_table([(c.ptr, s.ptr, r.nbytes, r.id)
                               for (c, s), r in zip(pairs, scn.regions)])
    ib = crum.crum_image_bytes(R, G, D, P)
    cap = crum.crum_image_bytes(R, G, G, P)
    staging = H.DeviceBuffer(cap)
    himg = H.PinnedBuffer(cap)
    status = H.PinnedBuffer(64)
    ctx = crum.crum_ctx_create(0)
    s = H.Stream()
    try:
        images = []
        for c in (cap, ib):  # pipelined (bench's order), then diff-first
            assert crum.crum_snapshot(ctx, table, P, 0, 11, staging.ptr, c, himg.ptr, c,
                                      s.handle, status.ptr) == 0
            s.synchronize()
            st = crum.read_status(status.ptr)
            assert st.code == 0 and st.n_dirty == D and st.image_bytes == ib, st
            images.append(himg.numpy(ib).copy())
        assert np.array_equal(images[0], images[1]), "the two orders disagree"
        rng = np.random.default_rng(16)
        check_image(images[0], scn, 64, rng, seq=11)
        log("[fullsize] many_allocs: oracle image (streamed)")
        want = oracle_image(scn, 11)
        assert_same_image(images[0], want, "pipelined order vs oracle")
        assert_same_image(images[1], want, "diff-first order vs oracle")
        del want
        # overwrite 8 dirty pages on the device, restore, check them and a clean page
        counts, starts = page_index(scn)
        want = scn.dirty_global()
        picks = [int(g) for g in rng.choice(want, size=8, replace=False)]
        for g in picks:
            ri = int(np.searchsorted(starts, g, side="right") - 1)
            synth.fill_dev(pairs[ri][0].ptr + (g - int(starts[ri])) * P, P, 999, 5, 0, 0)
        H.device_synchronize()
        assert crum.crum_restore(ctx, table, himg.ptr, ib, crum.CRUM_VERIFY, staging.ptr, cap,
                                 s.handle, status.ptr) == 0
        s.synchronize()
        assert crum.read_status(status.ptr).code == 0
        buf = np.empty(P, np.uint8)
        for g in picks + [int(np.setdiff1d(np.arange(64), want)[0])]:
            ri = int(np.searchsorted(starts, g, side="right") - 1)
            H.memcpy_dtoh(buf.ctypes.data, pairs[ri][0].ptr + (g - int(starts[ri])) * P, P)
            assert np.array_equal(buf, sc.host_page(scn, ri, g - int(starts[ri]), False)), g
    finally:
        crum.crum_ctx_destroy(ctx)
        for c, sh in pairs:
            c.free()
            sh.free()
        staging.free()
        himg.free()


@pytest.mark.timeout(900)
def test_managed_32gib():
    """The 32 GiB managed workload, 70 % of pages written by host threads and
    30 % prefetched and written by a kernel; then the same workload with the
    host writes tracked (the tracked snapshot's image against the same oracle
    image)."""
    import bench
    import paper_1808_00117_amd as crum
    import paper_1808_00117_amd.hip as H
    import synth
    from synth import scenarios as sc

    scn = sc.managed()
    r = scn.regions[0]
    P, G, D, N = scn.page_size, scn.total_pages, scn.n_dirty, scn.total_bytes
    log(f"[fullsize] managed N={N} D={D}")
    cur = H.ManagedBuffer(N)
    assert cur.device_mapped()
    dev_pages = scn.meta["device_pages"]
    bench.fill_managed_host(cur, scn, 0, np.setdiff1d(np.arange(G), dev_pages))
    bench.fill_managed_device(cur, scn, 0, dev_pages)
    sh = H.DeviceBuffer(N)
    synth.fill_dev(sh.ptr, N, r.fill_seed, r.fill_region, 0, 0)
    pd = np.ascontiguousarray(r.dirty_pages, np.int64)
    d_pages = H.DeviceBuffer(pd.nbytes)
    H.memcpy_htod(d_pages.ptr, pd.ctypes.data, pd.nbytes)
    synth.mutate_dev(sh.ptr, N, P, d_pages.ptr, pd.size, int(pd.max()), r.mut_kind,
                     scn.mut_seed, r.fill_region, 0)
    H.device_synchronize()
    ib = crum.crum_image_bytes(1, G, D, P)
    cap = crum.crum_image_bytes(1, G, G, P)
    staging = H.DeviceBuffer(cap)
    try:
        himg = H.PinnedBuffer(cap)
    except RuntimeError as e:
        # pinned memory is a host-wide resource: where 32 GiB more cannot be
        # pinned beside the 32 GiB managed region, the image gets a pinned
        # buffer of its exact size and the snapshot takes the diff-first
        # order (it cannot reserve the worst case), which checks the same
        # image
        log(f"[fullsize] managed: {e}; pinned image buffer of the image's size")
        himg = H.PinnedBuffer(ib)
    status = H.PinnedBuffer(64)
    ctx = crum.crum_ctx_create(0)
    s = H.Stream()
    try:
        table = crum.region_table([(cur.ptr, sh.ptr, N, r.id)])
        assert crum.crum_snapshot(ctx, table, P, 0, 3, staging.ptr, cap, himg.ptr, himg.nbytes,
                                  s.handle, status.ptr) == 0
        s.synchronize()
        st = crum.read_status(status.ptr)
        assert st.code == 0 and st.n_dirty == D and st.image_bytes == ib, st
        check_image(himg.numpy(ib), scn, 24, np.random.default_rng(32), seq=3)
        log("[fullsize] managed: oracle image (streamed)")
        want = oracle_image(scn, 3)
        assert_same_image(himg.numpy(ib), want, "managed image vs oracle")
        # host write tracking (Algorithm 1): host pages written through a
        # tracker's view and flushed, the snapshot reading only the flushed
        # pages and the device pages; its image must be the oracle's too
        import argparse
        log("[fullsize] managed: tracked snapshot")
        tr = bench.managed_tracked_leg(argparse.Namespace(steps=1, warmup=0), scn, cur, sh,
                                       table, ctx, staging, himg, cap, status, s, want, 0.0)
        assert tr["same_image_as_untracked"] and tr["candidate_pages"] < G, tr
        assert_same_image(himg.numpy(ib), want, "tracked managed image vs oracle")
    finally:
        crum.crum_ctx_destroy(ctx)
        cur.free()
        sh.free()
        staging.free()
        himg.free()


@pytest.mark.timeout(1200)
def test_batched_256_requests():
    """The 256-request batch (71 GB scanned) in one plan launch with the
    package's tuned shapes: every request's status, and every request's image
    against the oracle's, byte for byte."""
    import bench
    import paper_1808_00117_amd as crum
    import paper_1808_00117_amd.hip as H
    from paper_1808_00117_amd import autotune
    from synth import scenarios as sc

    reqs = sc.batched(seed=1004, n_requests=256)
    log(f"[fullsize] batched {len(reqs)} requests")
    pairs = [bench.materialize_raw(r, H) for r in reqs]
    tables = [[(c.ptr, s.ptr if s else 0, g.nbytes, g.id) for (c, s), g in zip(pr, r.regions)]
              for r, pr in zip(reqs, pairs)]
    sizes = [crum.crum_image_bytes(len(r.regions), r.total_pages, r.n_dirty, r.page_size)
             for r in reqs]
    cap = sum((b + 4095) // 4096 * 4096 for b in sizes) + (64 << 20)
    staging = H.DeviceBuffer(cap)
    himg = H.PinnedBuffer(cap)
    status = H.PinnedBuffer(40 * len(reqs))
    ctx = crum.crum_ctx_create(0)
    s = H.Stream()
    try:
        tuned = autotune.load(autotune.class_key("plan", sum(r.total_bytes for r in reqs)))
        if tuned:
            autotune.apply(ctx, tuned)
        plan = crum.Plan(ctx, [(t, r.page_size, 0, 9) for t, r in zip(tables, reqs)],
                         staging.ptr, cap, himg.ptr, cap)
        assert plan.launch(s.handle, status.ptr) == 0
        s.synchronize()
        sts = crum.read_request_statuses(status.ptr, len(reqs))
        for q, (code, _, D, G, b, off) in enumerate(sts):
            assert code == 0 and D == reqs[q].n_dirty and G == reqs[q].total_pages, q
            assert b == sizes[q] and off % 4096 == 0, q
        rng = np.random.default_rng(256)
        for q in rng.choice(len(reqs), size=24, replace=False):
            off, b = sts[q][5], sts[q][4]
            check_image(himg.numpy(off + b)[off:], reqs[q], 4, rng, seq=9)
        plan.destroy()
        log("[fullsize] batched: oracle images (streamed), 256 requests")
        # The requests are independent: the oracle runs on several host
        # threads at once (each call is single-threaded C and releases the
        # GIL); the CRC table is built before the threads start.
        oracle.crc32c(b"")
        with ThreadPoolExecutor(max_workers=8) as pool:
            futs = [pool.submit(oracle_image, reqs[q], 9) for q in range(len(reqs))]
            for q, f in enumerate(futs):
                if q % 32 == 0:
                    log(f"[fullsize] batched: oracle image of request {q}")
                off, b = sts[q][5], sts[q][4]
                assert_same_image(himg.numpy(off + b)[off:], f.result(),
                                  f"request {q} vs oracle")
                futs[q] = None
    finally:
        crum.crum_ctx_destroy(ctx)
        for pr in pairs:
            for c, sh in pr:
                c.free()
                if sh:
                    sh.free()
        staging.free()
        himg.free()


def test_persist_16gib_image(tmp_path):
    """The 16 GiB workload's image, persisted by the writer while the next
    snapshot runs into a second buffer: both files equal their images."""
    import bench
    import paper_1808_00117_amd as crum
    import paper_1808_00117_amd.hip as H
    from synth import scenarios as sc

    scn = sc.many_allocs()
    P, G, D, R = scn.page_size, scn.total_pages, scn.n_dirty, len(scn.regions)
    log("[fullsize] persist")
    pairs = bench.materialize_raw(scn, H)
    table = crum.region_table([(c.ptr, s.ptr, r.nbytes, r.id)
                               for (c, s), r in zip(pairs, scn.regions)])
    ib = crum.crum_image_bytes(R, G, D, P)
    cap = crum.crum_image_bytes(R, G, G, P)
    staging = H.DeviceBuffer(cap)
    # the first image in a buffer for the worst case (the pipelined order),
    # the second in one of its exact size (the diff-first order): less
    # pinned memory, which is a host-wide resource
    bufs = [H.PinnedBuffer(cap), H.PinnedBuffer(ib)]
    status = H.PinnedBuffer(64)
    ctx = crum.crum_ctx_create(0)
    s = H.Stream()
    w = crum.Writer(n_threads=4, chunk_bytes=64 << 20)
    try:
        tickets = []
        for i in range(2):
            assert crum.crum_snapshot(ctx, table, P, 0, 20 + i, staging.ptr, cap, bufs[i].ptr,
                                      bufs[i].nbytes, s.handle, status.ptr) == 0
            s.synchronize()
            assert crum.read_status(status.ptr).code == 0
            tickets.append(w.submit(str(tmp_path / f"ckpt{i}.crum"), bufs[i].ptr, ib))
        for i, t in enumerate(tickets):
            st = w.poll(t)
            assert st["code"] == 0 and st["bytes"] == ib, st
            back = np.fromfile(tmp_path / f"ckpt{i}.crum", np.uint8)
            assert np.array_equal(back, bufs[i].numpy(ib))
            rc, hdr = oracle.parse(back)
            assert rc == oracle.OK and hdr["seq"] == 20 + i and hdr["n_dirty"] == D
    finally:
        w.destroy()
        crum.crum_ctx_destroy(ctx)
        for c, sh in pairs:
            c.free()
            sh.free()
        staging.free()
        for b in bufs:
            b.free()
        for b in bufs:
            b.free()


def test_lazy_restore_16gib():
    """On-demand restore of the 16 GiB many-allocations image into the shadow
    buffers (which hold the old bytes of the dirty pages), swept region by
    region in 8 MiB touches as bench.py does: the fetched pages equal the
    oracle's read-fault model at every 256th touch and at the end, sampled
    pages hold the generator's bytes (restored) or the mutated bytes (not yet
    fetched), and after finish the shadows equal the current buffers (a
    snapshot finds no differing page)."""
    import bench
    import paper_1808_00117_amd as crum
    import paper_1808_00117_amd.hip as H
    from oracle.lazy import LazyModel
    from synth import scenarios as sc

    scn = sc.many_allocs()
    P, G, D, R = scn.page_size, scn.total_pages, scn.n_dirty, len(scn.regions)
    W = (G + 63) // 64
    log(f"[fullsize] lazy restore many_allocs D={D}")
    pairs = bench.materialize_raw(scn, H)
    table = crum.region_table([(c.ptr, s.ptr, r.nbytes, r.id)
                               for (c, s), r in zip(pairs, scn.regions)])
    targets = crum.region_table([(s.ptr, 0, r.nbytes, r.id)
                                 for (c, s), r in zip(pairs, scn.regions)])
    ib = crum.crum_image_bytes(R, G, D, P)
    cap = crum.crum_image_bytes(R, G, G, P)
    staging = H.DeviceBuffer(cap)
    himg = H.PinnedBuffer(cap)
    status = H.PinnedBuffer(64)
    ctx = crum.crum_ctx_create(0)
    s = H.Stream()
    lz = None
    try:
        assert crum.crum_snapshot(ctx, table, P, 0, 12, staging.ptr, cap, himg.ptr, cap,
                                  s.handle, status.ptr) == 0
        s.synchronize()
        assert crum.read_status(status.ptr).n_dirty == D
        small = 2 << 20
        lz = crum.Lazy(ctx, targets, himg.ptr, ib, crum.CRUM_VERIFY, small, staging.ptr, cap,
                       s.handle, status.ptr)
        s.synchronize()
        assert crum.read_status(status.ptr).code == 0
        model = LazyModel([r.nbytes for r in scn.regions], P, scn.dirty_global(), small)
        counts, starts = page_index(scn)
        rng = np.random.default_rng(17)
        want_dirty = scn.dirty_global()
        buf = np.empty(P, np.uint8)
        step, k = 8 << 20, 0
        for ri, r in enumerate(scn.regions):
            for off in range(0, r.nbytes, step):
                ln = min(step, r.nbytes - off)
                assert lz.touch(ri, off, ln, s.handle, 0) == model.touch(ri, off, ln)
                k += 1
                if k % 256 == 1:
                    s.synchronize()
                    assert lz.fetched(W) == model.fetched_bitmap(G), k
                    for g in rng.choice(want_dirty, size=4, replace=False):
                        g = int(g)
                        ri2 = int(np.searchsorted(starts, g, side="right") - 1)
                        H.memcpy_dtoh(buf.ctypes.data,
                                      pairs[ri2][1].ptr + (g - int(starts[ri2])) * P, P)
                        restored = g in model.fetched
                        want = sc.host_page(scn, ri2, g - int(starts[ri2]), not restored)
                        assert np.array_equal(buf, want), (k, g, restored)
        s.synchronize()
        assert lz.fetched(W) == model.fetched_bitmap(G)
        lz.finish(s.handle, status.ptr)
        s.synchronize()
        assert crum.read_status(status.ptr).code == 0
        st = lz.stats()
        assert st["pages_fetched"] == D and st["faults"] == sum(model.faults.values())
        lz.close()
        lz = None
        assert crum.crum_snapshot(ctx, table, P, 0, 13, staging.ptr, cap, 0, 0, s.handle,
                                  status.ptr) == 0
        s.synchronize()
        assert crum.read_status(status.ptr).n_dirty == 0
    finally:
        if lz is not None:
            lz.close()
        crum.crum_ctx_destroy(ctx)
        for c, sh in pairs:
            c.free()
            sh.free()
        staging.free()
        himg.free()
