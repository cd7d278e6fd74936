"""System-level checks: a full image brings back regions whose device state
was lost, and a co-running application kernel computes the same bits with or
without a snapshot running beside it."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import log, upload

pytestmark = pytest.mark.gpu

KiB = 1 << 10


@pytest.fixture(scope="module")
def snap():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1808_00117_amd as crum
    crum.lib()
    from paper_1808_00117_amd.api import Snapshotter
    s = Snapshotter(0)
    yield s
    s.close()


def test_restore_after_simulated_device_loss(snap):
    """Regions snapshotted without shadows (every page in the image) are
    wiped, as after losing the device's memory; a verified restore of the
    image makes them equal to what was saved, bit for bit."""
    import torch
    P = 16 * KiB
    rng = np.random.default_rng(101)
    host = [(rng.integers(0, 256, n * P, dtype=np.uint8), None, 40 + i)
            for i, n in enumerate((25, 40, 3))]
    st_o, img_o, _ = oracle.snapshot(host, P, seq=8)
    assert st_o.n_dirty == 68
    dev = upload(host)
    staging = torch.empty(img_o.size, dtype=torch.uint8, device="cuda")
    h = torch.empty(img_o.size, dtype=torch.uint8, pin_memory=True)
    rc, st = snap.snapshot(dev, P, staging, h, seq=8)
    assert rc == 0 and st.code == 0 and np.array_equal(h.numpy(), img_o)
    for c, _, _ in dev:
        c.zero_()
    rc, st = snap.restore(dev, h, img_o.size, staging, flags=2)
    assert rc == 0 and st.code == 0
    for (c, _, _), (cur, _, _) in zip(dev, host):
        assert np.array_equal(c.cpu().numpy(), cur)


def test_corunner_output_unchanged_by_a_snapshot(snap):
    """The fp32 SAXPY co-runner gives the same bits alone and with a snapshot
    of 64 MiB running on another stream at the same time."""
    import torch

    import synth
    n = 1 << 22
    rng = np.random.default_rng(6)
    x = torch.from_numpy(rng.random(n, dtype=np.float32)).cuda()
    y0 = torch.from_numpy(rng.random(n, dtype=np.float32)).cuda()
    P = 4 * KiB
    cur = rng.integers(0, 256, 64 << 20, dtype=np.uint8)
    sh = cur.copy()
    sh[:: 37 * P] ^= 1
    dev = upload([(cur, sh, 1)])
    st_o = oracle.snapshot([(cur, sh, 1)], P)[0]
    staging = torch.empty(st_o.image_bytes, dtype=torch.uint8, device="cuda")
    h = torch.empty(st_o.image_bytes, dtype=torch.uint8, pin_memory=True)
    s_app, s_snap = torch.cuda.Stream(), torch.cuda.Stream()

    def saxpy(y):
        synth.saxpy_loop_dev(y.data_ptr(), x.data_ptr(), 1.0001, n, 16, 1024, s_app.cuda_stream)

    torch.cuda.synchronize()
    ya = y0.clone()
    saxpy(ya)
    s_app.synchronize()
    yb = y0.clone()
    torch.cuda.synchronize()
    for _ in range(3):
        saxpy(yb)  # queued on the application stream ...
        rc = snap.snapshot(dev, P, staging, h, stream=s_snap, sync=False)  # ... beside it
        assert rc == 0
    torch.cuda.synchronize()
    st = snap.status()
    assert st.code == 0 and st.n_dirty == st_o.n_dirty
    yc = y0.clone()
    for _ in range(3):
        saxpy(yc)
    s_app.synchronize()
    log("[systems] saxpy alone and beside snapshots")
    assert torch.equal(yb, yc), "SAXPY results differ beside a snapshot"
    assert not torch.equal(ya, y0)
