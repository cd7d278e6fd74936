"""Managed memory: the snapshot of a hipMallocManaged region whose pages were
written partly by host threads and partly by a device kernel after a
prefetch equals the oracle's image of the same bytes, whatever the pages'
residency."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import log

pytestmark = pytest.mark.gpu

KiB, MiB = 1 << 10, 1 << 20


@pytest.mark.parametrize("P,n_pages,device_frac", [(2 * MiB, 24, 0.3), (2 * MiB, 24, 0.0),
                                                    (2 * MiB, 24, 1.0), (64 * KiB, 300, 0.3)])
def test_managed_parity(P, n_pages, device_frac):
    import bench
    import paper_1808_00117_amd as crum
    import paper_1808_00117_amd.hip as H
    import synth
    from synth import scenarios as sc

    log(f"[managed] P={P} pages={n_pages} device_frac={device_frac}")
    scn = sc.managed(seed=77, nbytes=n_pages * P, page_size=P, device_frac=device_frac,
                     dirty_frac=0.25)
    r = scn.regions[0]
    N = scn.total_bytes
    cur = H.ManagedBuffer(N)
    log(f"[managed] attributes {H.pointer_attributes(cur.ptr)}")
    assert cur.device_mapped(), "managed allocation not mapped for the device"
    dev_pages = scn.meta["device_pages"]
    host_pages = np.setdiff1d(np.arange(n_pages), dev_pages)
    bench.fill_managed_host(cur, scn, 0, host_pages, threads=4)
    bench.fill_managed_device(cur, scn, 0, dev_pages)
    sh = H.DeviceBuffer(N)
    synth.fill_dev(sh.ptr, N, r.fill_seed, r.fill_region, 0, 0)
    pd = np.ascontiguousarray(r.dirty_pages, np.int64)
    pages_d = H.DeviceBuffer(pd.nbytes)
    H.memcpy_htod(pages_d.ptr, pd.ctypes.data, pd.nbytes)
    synth.mutate_dev(sh.ptr, N, P, pages_d.ptr, pd.size, int(pd.max()), r.mut_kind,
                     scn.mut_seed, r.fill_region, 0)
    H.device_synchronize()
    host_cur, host_sh = sc.materialize_host(scn, 0)
    st_o, img_o, _ = oracle.snapshot([(host_cur, host_sh, r.id)], P, seq=9)
    assert st_o.n_dirty == pd.size
    cap = crum.crum_image_bytes(1, n_pages, n_pages, P)
    staging = H.DeviceBuffer(cap)
    himg = H.PinnedBuffer(cap)
    status = H.PinnedBuffer(64)
    ctx = crum.crum_ctx_create(0)
    s = H.Stream()
    table = crum.region_table([(cur.ptr, sh.ptr, N, r.id)])
    for c in (cap, st_o.image_bytes):  # pipelined and diff-first orders
        rc = crum.crum_snapshot(ctx, table, P, 0, 9, staging.ptr, c, himg.ptr, c, s.handle,
                                status.ptr)
        assert rc == 0
        s.synchronize()
        st = crum.read_status(status.ptr)
        assert st.code == 0 and st.n_dirty == st_o.n_dirty
        assert np.array_equal(himg.numpy(st.image_bytes), img_o)
    # the host still sees the bytes it and the device wrote
    assert np.array_equal(cur.numpy(0, N), host_cur)
    # the runtime's residency report of every page (recorded, not asserted:
    # on devices without managed-memory support the allocation is host memory
    # and the report carries no location)
    locs = {}
    for p in range(n_pages):
        rc, loc = cur.last_prefetch_location(p * P, P)
        kind = "device" if p in set(int(x) for x in dev_pages) else "host"
        locs.setdefault(kind, {}).setdefault(f"rc{rc}:loc{loc}", 0)
        locs[kind][f"rc{rc}:loc{loc}"] += 1
    log(f"[managed] last prefetch location per page kind: {locs}")
    crum.crum_ctx_destroy(ctx)
