"""GPU parity for page spaces whose bitmap takes the prefix-sum kernel more
than one pass (more than 4096 bitmap words, i.e. 262 144 pages, in one scan
launch, so the running total carries from pass to pass), compared with the
oracle byte for byte:

* one snapshot of 1.45 GiB of 4 KiB pages (5 920 bitmap words) with sparse
  uniform and clustered dirty pages, in the diff-first order (the whole
  bitmap in one scan), in the chunk-pipelined order with a first chunk of
  5 120 words, and in the direct order (the whole bitmap in one scan, the
  image written into pinned host memory);
* a verified restore of that image into clobbered regions (the restore's
  own scan of the image bitmap, 5 920 words);
* a batched plan whose single group spans 5 600 words of three requests.
"""
import numpy as np
import pytest

import oracle
from synth import scenarios as sc
from synth.lib import PageSource
from tests.gpu_util import log

pytestmark = pytest.mark.gpu

KiB, MiB = 1 << 10, 1 << 20


def _scenario(sizes, seed, P=4 * KiB):
    rng = np.random.Generator(np.random.PCG64(seed))
    regs = []
    for i, nb in enumerate(sizes):
        n = nb // P
        uni = rng.choice(n, size=n // 40, replace=False)          # 2.5 % uniform
        runs = sc.clustered_runs(rng, n, 0.001, 24.0)               # about 2.4 % in runs
        dp = np.union1d(uni, runs).astype(np.int64)
        regs.append(sc.RegionSpec(id=900 + i, nbytes=nb, fill_seed=seed, fill_region=i,
                                  dirty_pages=dp))
    return sc.Scenario("multipass", seed, P, seed + 7919, regs)


def _oracle(scn, seq):
    src = PageSource(scn)
    st, img, _ = oracle.snapshot_stream(src.regions, scn.page_size, src.fn, src.user, seq=seq)
    assert st.code == oracle.OK and st.n_dirty == scn.n_dirty
    return img


def _same(got, want, what):
    if got.size != want.size or not np.array_equal(got, want):
        n = min(got.size, want.size)
        bad = np.flatnonzero(got[:n] != want[:n])
        raise AssertionError(f"{what}: sizes {got.size}/{want.size}, "
                             f"{bad.size} bytes differ, first {bad[:4]}")


@pytest.mark.timeout(600)
def test_multipass_scan_snapshot_orders_and_restore():
    import bench
    import paper_1808_00117_amd as crum
    import paper_1808_00117_amd.hip as H

    scn = _scenario([1280 * MiB, 200 * MiB], seed=4242)
    P, G, D, R = scn.page_size, scn.total_pages, scn.n_dirty, len(scn.regions)
    W = (G + 63) // 64
    assert W > 4096 and 1280 * MiB // P // 64 > 4096
    log(f"[multipass] G={G} W={W} D={D}")
    want = _oracle(scn, 21)
    pairs = bench.materialize_raw(scn, H)
    table = crum.region_table([(c.ptr, s.ptr, r.nbytes, r.id)
                               for (c, s), r in zip(pairs, scn.regions)])
    ib = crum.crum_image_bytes(R, G, D, P)
    cap = crum.crum_image_bytes(R, G, G, P)
    assert ib == want.size
    staging = H.DeviceBuffer(cap)
    himg = H.PinnedBuffer(cap)
    status = H.PinnedBuffer(64)
    s = H.Stream()
    ctxs = []
    try:
        def run(ctx, c, what):
            himg.numpy(ib)[:] = 0
            assert crum.crum_snapshot(ctx, table, P, 0, 21, staging.ptr, c, himg.ptr, c,
                                      s.handle, status.ptr) == 0
            s.synchronize()
            st = crum.read_status(status.ptr)
            assert st.code == 0 and st.n_dirty == D and st.image_bytes == ib, (what, st)
            _same(himg.numpy(ib), want, what)

        first = crum.crum_ctx_create(0)
        ctxs.append(first)
        crum.crum_ctx_set_param(first, crum.CRUM_PARAM_DIRECT_BYTES, 0)
        log("[multipass] diff-first order")
        run(first, ib, "diff-first")
        pipe = crum.crum_ctx_create(0)
        ctxs.append(pipe)
        crum.crum_ctx_set_param(pipe, crum.CRUM_PARAM_DIRECT_BYTES, 0)
        crum.crum_ctx_set_param(pipe, crum.CRUM_PARAM_CHUNK_BYTES, 1280 * MiB)
        log("[multipass] pipelined order, first chunk 5120 words")
        run(pipe, cap, "pipelined")
        direct = crum.crum_ctx_create(0)
        ctxs.append(direct)
        crum.crum_ctx_set_param(direct, crum.CRUM_PARAM_DIRECT_BYTES, 1 << 40)
        log("[multipass] direct order")
        run(direct, cap, "direct")

        # clobber every dirty page of both regions and a few clean ones: a
        # verified restore must put back exactly the image's pages
        import synth
        for (c, _), r in zip(pairs, scn.regions):
            synth.fill_dev(c.ptr, r.nbytes, 31337, r.fill_region, 0, 0)
        H.device_synchronize()
        log("[multipass] verified restore")
        assert crum.crum_restore(first, table, himg.ptr, ib, crum.CRUM_VERIFY, staging.ptr,
                                 cap, s.handle, status.ptr) == 0
        s.synchronize()
        st = crum.read_status(status.ptr)
        assert st.code == 0 and st.n_dirty == D, st
        # the oracle's restore of the same image into host copies of the
        # clobbered regions gives the expected bytes; compare whole regions
        for i, ((c, _), r) in enumerate(zip(pairs, scn.regions)):
            host = synth.fill_host(r.nbytes, 31337, r.fill_region)
            ost = oracle.restore([(host if j == i else np.zeros(g.nbytes, np.uint8), None, g.id)
                                  for j, g in enumerate(scn.regions)], want, oracle.VERIFY)
            assert ost.code == oracle.OK
            got = np.empty(r.nbytes, np.uint8)
            H.memcpy_dtoh(got.ctypes.data, c.ptr, r.nbytes)
            _same(got, host, f"restored region {i}")
    finally:
        for c in ctxs:
            crum.crum_ctx_destroy(c)
        for c, sh in pairs:
            c.free()
            sh.free()
        staging.free()
        himg.free()


@pytest.mark.timeout(600)
def test_multipass_scan_batched_group():
    import bench
    import paper_1808_00117_amd as crum
    import paper_1808_00117_amd.hip as H

    reqs = [_scenario([600 * MiB], seed=51), _scenario([300 * MiB, 200 * MiB], seed=52),
            _scenario([300 * MiB], seed=53)]
    words = sum(sum(r.nbytes // 4096 for r in q.regions) // 64 for q in reqs)
    assert words > 4096
    log(f"[multipass] batched group of {words} words")
    pairs = [bench.materialize_raw(q, H) for q in reqs]
    tables = [[(c.ptr, s.ptr, g.nbytes, g.id) for (c, s), g in zip(pr, q.regions)]
              for q, pr in zip(reqs, pairs)]
    sizes = [crum.crum_image_bytes(len(q.regions), q.total_pages, q.n_dirty, q.page_size)
             for q in reqs]
    cap = sum((b + 4095) // 4096 * 4096 for b in sizes) + (1 << 20)
    staging = H.DeviceBuffer(cap)
    himg = H.PinnedBuffer(cap)
    status = H.PinnedBuffer(40 * len(reqs))
    s = H.Stream()
    ctx = crum.crum_ctx_create(0)
    try:
        crum.crum_ctx_set_param(ctx, crum.CRUM_PARAM_CHUNK_BYTES, 8 << 30)
        crum.crum_ctx_set_param(ctx, crum.CRUM_PARAM_CHUNK_MAX_BYTES, 8 << 30)
        plan = crum.Plan(ctx, [(t, q.page_size, 0, 30 + i) for i, (t, q) in
                               enumerate(zip(tables, reqs))], staging.ptr, cap, himg.ptr, cap)
        assert plan.groups() == [0, len(reqs)], "one group expected"
        assert plan.launch(s.handle, status.ptr) == 0
        s.synchronize()
        sts = crum.read_request_statuses(status.ptr, len(reqs))
        for i, q in enumerate(reqs):
            code, _, D, G, b, off = sts[i]
            assert code == 0 and D == q.n_dirty and b == sizes[i], (i, sts[i])
            _same(himg.numpy(off + b)[off:], _oracle(q, 30 + i), f"request {i}")
        plan.destroy()
    finally:
        crum.crum_ctx_destroy(ctx)
        for pr in pairs:
            for c, sh in pr:
                c.free()
                sh.free()
        staging.free()
        himg.free()
