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

    # each clone runs on torch's current stream, which the application stream
    # does not wait for: synchronise before the SAXPY passes read the copy
    torch.cuda.synchronize()
    ya = y0.clone()
    torch.cuda.synchronize()
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
    torch.cuda.synchronize()
    for _ in range(3):
        saxpy(yc)
    s_app.synchronize()
    log("[systems] saxpy alone and beside snapshots")
    assert torch.equal(yb, yc), "SAXPY results differ beside a snapshot"
    assert not torch.equal(ya, y0)


_CKPT = r"""
import sys
import numpy as np
import torch
import paper_1808_00117_amd as crum
from paper_1808_00117_amd.api import Snapshotter
out = sys.argv[1]
P = 16 << 10
rng = np.random.default_rng(202)
host = [rng.integers(0, 256, n * P, dtype=np.uint8) for n in (25, 40, 3)]
cur = [torch.from_numpy(h).cuda() for h in host]
s = Snapshotter(0)
cap = 4096 * 4 + sum(c.numel() for c in cur) + 4 * 68 + 8
staging = torch.empty(cap, dtype=torch.uint8, device="cuda")
h = torch.empty(cap, dtype=torch.uint8, pin_memory=True)
w = crum.Writer(n_threads=2, chunk_bytes=1 << 20)
# checkpoint 1: full (no shadows: every page in the image)
rc, st = s.snapshot([(c, None, 60 + i) for i, c in enumerate(cur)], P, staging, h, seq=1)
assert rc == 0 and st.code == 0 and st.n_dirty == 68, st
t = w.submit(out + ".1", h.data_ptr(), st.image_bytes)
assert w.poll(t)["code"] == 0
# checkpoint 2: incremental against the state of checkpoint 1
sh = [c.clone() for c in cur]
cur[0][3 * P + 100] ^= 0x5A
cur[1][39 * P] ^= 0x01
cur[1][7 * P:8 * P] = 9
rc, st = s.snapshot([(c, x, 60 + i) for i, (c, x) in enumerate(zip(cur, sh))], P, staging, h,
                    seq=2)
assert rc == 0 and st.code == 0 and st.n_dirty == 3, st
t = w.submit(out + ".2", h.data_ptr(), st.image_bytes)
assert w.poll(t)["code"] == 0
w.destroy()
np.save(out + ".want.npy", np.concatenate([c.cpu().numpy() for c in cur]))
print("checkpointed", flush=True)
"""

_RESTART = r"""
import sys
import numpy as np
import torch
import paper_1808_00117_amd as crum
from paper_1808_00117_amd.api import Snapshotter
out = sys.argv[1]
P = 16 << 10
# the regions re-created by the restarted program: same ids and lengths, new
# addresses, no content
regs = [torch.zeros(n * P, dtype=torch.uint8, device="cuda") for n in (25, 40, 3)]
s = Snapshotter(0)
for k in (1, 2):  # the full image, then the increment on top of it
    img = np.fromfile(out + f".{k}", dtype=np.uint8)
    h = torch.from_numpy(img).pin_memory()
    staging = torch.empty(img.size, dtype=torch.uint8, device="cuda")
    rc, st = s.restore([(r, None, 60 + i) for i, r in enumerate(regs)], h, img.size, staging,
                       flags=crum.CRUM_VERIFY)
    assert rc == 0 and st.code == 0, (k, st)
want = np.load(out + ".want.npy")
got = np.concatenate([r.cpu().numpy() for r in regs])
assert np.array_equal(got, want), "restored state differs"
print("restart ok", flush=True)
"""


def test_restart_in_a_new_process(tmp_path):
    """The paper's restart (section 3.4): a program checkpoints its regions
    (a full image, then an incremental one after changing three pages),
    persists both to files and exits; a new process re-creates regions of the
    same ids and lengths at new addresses and restores the two files in
    order, with verification: its regions equal the first program's last
    state, bit for bit."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, PYTHONPATH=root + os.pathsep + os.environ.get("PYTHONPATH", ""))
    out = str(tmp_path / "ckpt")
    for script, want in ((_CKPT, "checkpointed"), (_RESTART, "restart ok")):
        log(f"[systems] {want.split()[0]} process")
        r = subprocess.run([sys.executable, "-c", script, out], cwd=root, env=env,
                           capture_output=True, text=True, timeout=240)
        assert r.returncode == 0 and want in r.stdout, r.stdout + r.stderr
