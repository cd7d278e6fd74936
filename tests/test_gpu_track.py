"""GPU parity of the snapshot with a candidate set (host write tracking,
paper section 3.2, Algorithm 1): whenever the candidate set covers every page
that differs from its shadow, the image equals the oracle's (which compares
every page) byte for byte, in the pipelined and diff-first orders; pages
outside the set are not read.  And the whole tracked flow on managed memory:
host pages written through a tracker's view and flushed into a
hipMallocManaged region, device pages written by a kernel, the snapshot given
the flushed pages plus the device pages."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import image_capacity, log, upload

pytestmark = pytest.mark.gpu

KiB = 1 << 10


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1808_00117_amd as crum
    from paper_1808_00117_amd.api import Snapshotter
    s = Snapshotter(0)
    crum.crum_ctx_set_param(s.ctx, crum.CRUM_PARAM_CHUNK_BYTES, 64 * 64 * KiB)
    yield s
    s.close()


def set_bits(words, pages):
    for p in pages:
        words[p >> 6] |= np.uint64(1) << np.uint64(p & 63)


def tracked(s, dev, P, cand, cap, seq=4):
    import torch

    import paper_1808_00117_amd as crum
    from paper_1808_00117_amd.api import regions_of
    staging = torch.empty(cap, dtype=torch.uint8, device="cuda")
    h = torch.empty(cap, dtype=torch.uint8, pin_memory=True)
    rc = crum.crum_snapshot_tracked(s.ctx, regions_of(dev), P, 0, seq, cand, staging.data_ptr(),
                                    cap, h.data_ptr(), cap,
                                    torch.cuda.current_stream().cuda_stream,
                                    s.status_buf.data_ptr())
    assert rc == 0, rc
    torch.cuda.synchronize()
    st = s.status()
    assert st.code == 0, st
    return st, h[: st.image_bytes].numpy().copy()


@pytest.mark.parametrize("seed", range(6))
def test_candidate_supersets_give_the_oracle_image(ctx, seed):
    rng = np.random.default_rng(700 + seed)
    P = [4 * KiB, 16 * KiB, 64 * KiB][seed % 3]
    counts = [int(x) for x in rng.integers(1, 300, int(rng.integers(1, 5)))]
    G = sum(counts)
    dirty = set(int(x) for x in rng.choice(G, size=int(rng.integers(0, G // 3 + 1)),
                                            replace=False))
    host, g = [], 0
    null_region = int(rng.integers(0, len(counts))) if seed % 2 else -1
    for i, n in enumerate(counts):
        cur = rng.integers(0, 256, n * P, dtype=np.uint8)
        sh = cur.copy()
        for k in range(n):
            if g + k in dirty:
                o = int(rng.integers(0, P))
                sh[k * P + o] ^= np.uint8(1 + rng.integers(0, 255))
        host.append((cur, None if i == null_region else sh, 40 + i))
        g += n
    st_o, img_o, _ = oracle.snapshot(host, P, seq=4)
    dev = upload(host)
    W = (G + 63) // 64
    extra = set(int(x) for x in rng.choice(G, size=G // 4, replace=False))
    import paper_1808_00117_amd as crum
    q0 = crum.crum_ctx_get_param(ctx.ctx, crum.CRUM_PARAM_DIFF_GROUP)
    try:
        for group in (1, 2, 4):
            crum.crum_ctx_set_param(ctx.ctx, crum.CRUM_PARAM_DIFF_GROUP, group)
            for name, pages in (("exact", dirty), ("superset", dirty | extra),
                                ("all", range(G))):
                cand = np.zeros(W + int(rng.integers(0, 3)), np.uint64)
                set_bits(cand, pages)
                for cap in (image_capacity(dev, P), st_o.image_bytes):
                    log(f"[track] seed {seed} P={P} G={G} D={st_o.n_dirty} {name} "
                        f"cap={cap} group={group}")
                    st, img = tracked(ctx, dev, P, cand, cap)
                    assert st.n_dirty == st_o.n_dirty
                    assert np.array_equal(img, img_o), (name, cap, group)
    finally:
        crum.crum_ctx_set_param(ctx.ctx, crum.CRUM_PARAM_DIFF_GROUP, q0)


def test_pages_outside_the_set_are_not_read(ctx):
    """A page outside the candidate set is taken as clean even when it
    differs (the caller's guarantee is what makes the image exact): the
    bitmap then holds exactly the candidate pages that differ."""
    P = 4 * KiB
    rng = np.random.default_rng(5)
    cur = rng.integers(0, 256, 200 * P, dtype=np.uint8)
    sh = cur.copy()
    for p in (3, 50, 51, 199):
        sh[p * P + 7] ^= 0x5A
    dev = upload([(cur, sh, 1)])
    cand = np.zeros(4, np.uint64)
    set_bits(cand, [3, 51, 100])
    import paper_1808_00117_amd as crum
    q0 = crum.crum_ctx_get_param(ctx.ctx, crum.CRUM_PARAM_DIFF_GROUP)
    try:
        for group in (1, 2, 4):
            crum.crum_ctx_set_param(ctx.ctx, crum.CRUM_PARAM_DIFF_GROUP, group)
            st, img = tracked(ctx, dev, P, cand, image_capacity(dev, P))
            assert st.n_dirty == 2
            bm = np.frombuffer(img[96:96 + 32].tobytes(), np.uint64)
            bits = np.flatnonzero(np.unpackbits(bm.view(np.uint8), bitorder="little"))
            assert list(bits) == [3, 51], group
    finally:
        crum.crum_ctx_set_param(ctx.ctx, crum.CRUM_PARAM_DIFF_GROUP, q0)


def test_short_candidate_bitmap_is_einval(ctx):
    import torch

    import paper_1808_00117_amd as crum
    from paper_1808_00117_amd.api import regions_of
    P = 4 * KiB
    dev = upload([(np.zeros(130 * P, np.uint8), np.zeros(130 * P, np.uint8), 1)])
    cap = image_capacity(dev, P)
    staging = torch.empty(cap, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    rc = crum.crum_snapshot_tracked(ctx.ctx, regions_of(dev), P, 0, 1, np.zeros(2, np.uint64),
                                    staging.data_ptr(), cap, 0, 0, s, ctx.status_buf.data_ptr())
    assert rc == crum.CRUM_EINVAL


def test_tracked_flow_on_managed_memory(ctx):
    """Algorithm 1 end to end on a 16 MiB hipMallocManaged region of 64 KiB
    pages: host pages written through the view and flushed, device pages
    written by a kernel; after the last snapshot's state is set up, the
    changed host pages are written again through the view; the tracked
    snapshot (flushed pages plus device pages) equals the oracle's image of
    (current bytes, shadow)."""
    import paper_1808_00117_amd as crum
    import paper_1808_00117_amd.hip as H
    import synth

    P, G = 64 * KiB, 256
    N = G * P
    rng = np.random.default_rng(77)
    cur_host = rng.integers(0, 256, N, dtype=np.uint8)
    dev_pages = np.sort(rng.choice(G, size=G * 3 // 10, replace=False))
    host_pages = np.setdiff1d(np.arange(G), dev_pages)
    changed = np.sort(rng.choice(G, size=G // 5, replace=False))
    sh_host = cur_host.copy()
    for p in changed:
        o = int(rng.integers(0, P - 256))
        sh_host[p * P + o: p * P + o + 256] ^= rng.integers(1, 256, 256, dtype=np.uint8)
    st_o, img_o, _ = oracle.snapshot([(cur_host, sh_host, 9)], P, seq=4)
    M = H.ManagedBuffer(N)
    assert M.device_mapped()
    sh = H.DeviceBuffer(N)
    H.memcpy_htod(sh.ptr, sh_host.ctypes.data, N)
    tr = crum.Tracker(N, P)
    try:
        v = tr.view()
        # state at the last snapshot: host pages hold the shadow's bytes
        for p in host_pages:
            v[p * P:(p + 1) * P] = sh_host[p * P:(p + 1) * P]
        tr.flush(M.ptr, 4)
        # device pages: current bytes written on the device
        tmp = H.DeviceBuffer(N)
        H.memcpy_htod(tmp.ptr, cur_host.ctypes.data, N)
        for p in dev_pages:
            synth.copy_dev(M.ptr + int(p) * P, tmp.ptr + int(p) * P, P, 0)
        H.device_synchronize()
        tmp.free()
        tr.pending(clear=True)
        f0 = tr.stats()["faults"]
        changed_host = np.intersect1d(changed, host_pages)
        for p in changed_host:
            v[p * P:(p + 1) * P] = cur_host[p * P:(p + 1) * P]
        assert tr.stats()["faults"] - f0 == changed_host.size
        assert tr.flush(M.ptr, 4) == changed_host.size
        cand = tr.pending(clear=True)
        set_bits(cand, dev_pages)
        assert np.array_equal(M.numpy(0, N), cur_host)
        log(f"[track] managed flow: {changed_host.size} host pages flushed, "
            f"{dev_pages.size} device pages")
        dev = [(M.ptr, sh.ptr, N, 9)]
        import torch
        cap = oracle.prefix_bytes(1, G) + N + 4 * G
        staging = torch.empty(cap, dtype=torch.uint8, device="cuda")
        h = torch.empty(cap, dtype=torch.uint8, pin_memory=True)
        rc = crum.crum_snapshot_tracked(ctx.ctx, dev, P, 0, 4, cand, staging.data_ptr(), cap,
                                        h.data_ptr(), cap,
                                        torch.cuda.current_stream().cuda_stream,
                                        ctx.status_buf.data_ptr())
        assert rc == 0
        torch.cuda.synchronize()
        st = ctx.status()
        assert st.code == 0 and st.n_dirty == st_o.n_dirty, st
        assert np.array_equal(h[: st.image_bytes].numpy(), img_o)
    finally:
        tr.destroy()
        M.free()
        sh.free()
