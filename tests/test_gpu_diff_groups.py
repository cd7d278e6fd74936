"""GPU parity of the diff kernel with 1, 2 and 4 units of 4 KiB per wave at
full size: two regions of 1 GiB and 1 GiB + 12 KiB with 4 KiB pages (the
second ends in a group of three units, done one at a time by groups of two
or four), dirty pages planted at region starts and ends and inside,
snapshotted in the pipelined order (staging for the worst case: chunk
launches of 128 MiB to 1.4 GiB) and in the diff-first order; every image
equals the oracle's."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import image_capacity, log

pytestmark = pytest.mark.gpu

KiB, GiB = 1 << 10, 1 << 30
P = 4 * KiB


def test_diff_groups_full_size():
    import torch

    import paper_1808_00117_amd as crum
    from paper_1808_00117_amd.api import Snapshotter, regions_of
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    sizes = (GiB, GiB + 3 * P)
    g = torch.Generator(device="cuda").manual_seed(1808)
    cur = [torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda", generator=g)
           for n in sizes]
    sh = [c.clone() for c in cur]
    rng = np.random.default_rng(117)
    planted = []
    for i, n in enumerate(sizes):
        G = n // P
        pages = {0, 1, 2, 3, 4, G - 1, G - 2, G - 4} | set(int(x) for x in rng.choice(G, 200))
        for p in sorted(pages):
            o = p * P + int(rng.integers(0, P))
            sh[i][o] ^= 0x5A
            planted.append((i, p))
    torch.cuda.synchronize()
    host = [(c.cpu().numpy(), s.cpu().numpy(), 10 + i) for i, (c, s) in enumerate(zip(cur, sh))]
    st_o, img_o, _ = oracle.snapshot(host, P, seq=9)
    del host
    assert st_o.n_dirty == len(planted)
    dev = [(c, s, 10 + i) for i, (c, s) in enumerate(zip(cur, sh))]
    s = Snapshotter(0)
    try:
        worst = image_capacity(dev, P)
        h = torch.empty(worst, dtype=torch.uint8, pin_memory=True)
        for cap in (worst, st_o.image_bytes):
            staging = torch.empty(cap, dtype=torch.uint8, device="cuda")
            for group in (1, 2, 4):
                log(f"[diff group] cap={cap} group={group}")
                crum.crum_ctx_set_param(s.ctx, crum.CRUM_PARAM_DIFF_GROUP, group)
                rc = crum.crum_snapshot(s.ctx, regions_of(dev), P, 0, 9, staging.data_ptr(),
                                        cap, h.data_ptr(), worst,
                                        torch.cuda.current_stream().cuda_stream,
                                        s.status_buf.data_ptr())
                assert rc == 0, rc
                torch.cuda.synchronize()
                st = s.status()
                assert st.code == 0 and st.n_dirty == st_o.n_dirty, st
                assert st.image_bytes == st_o.image_bytes
                assert np.array_equal(h[: st.image_bytes].numpy(), img_o), (cap, group)
            del staging
    finally:
        s.close()
