"""GPU tests of the serving loop: each request's result (status, dirty count,
image digest) is the same when its client runs alone and when many clients'
requests are interleaved on several slots; restores bring a client's memory
back to its shadow; images are valid for the oracle's parser."""
import ctypes

import numpy as np
import pytest

import oracle
from tests.gpu_util import log

pytestmark = pytest.mark.gpu

KiB, MiB = 1 << 10, 1 << 20
SNAP, REST = 1, 2


class Harness:
    """Client state on the device and the deterministic changes made to it:
    before snapshot `tag` of client c, pages chosen by PCG64(c, tag) get 1-16
    words changed; before a restore, the pages of the client's last snapshot
    are overwritten with other bytes, which the restore must repair."""

    def __init__(self, specs, seed=0):
        import torch
        import synth
        self.torch, self.synth = torch, synth
        self.specs = specs  # list of (n_pages, page_size)
        self.cur, self.sh, self.last_pages = [], [], []
        for c, (n, P) in enumerate(specs):
            cur = torch.empty(n * P, dtype=torch.uint8, device="cuda")
            synth.fill_dev(cur.data_ptr(), n * P, 4242 + seed, c, 0, 0)
            sh = cur.clone()
            self.cur.append(cur)
            self.sh.append(sh)
            self.last_pages.append(None)
        torch.cuda.synchronize()
        self.pages_dev = {}

    def clients(self):
        return [([(c.data_ptr(), s.data_ptr(), c.numel(), 77 + i)], P)
                for i, (c, s, (n, P)) in enumerate(zip(self.cur, self.sh, self.specs))]

    def pages_for(self, client, tag):
        n, P = self.specs[client]
        rng = np.random.Generator(np.random.PCG64(client * 100003 + tag))
        k = max(1, int(n * rng.uniform(0.02, 0.30)))
        return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)

    def precompute(self, schedule):
        """Upload the page lists of every snapshot in the schedule (so the
        prepare hook only launches kernels)."""
        for c, kind, tag in schedule:
            if kind == SNAP:
                pages = self.pages_for(c, tag)
                self.pages_dev[(c, tag)] = (pages, self.torch.from_numpy(pages).to("cuda"))
        self.torch.cuda.synchronize()

    def prepare(self, user, client, kind, tag, stream):
        synth = self.synth
        n, P = self.specs[client]
        if kind == SNAP:
            pages, d = self.pages_dev[(client, tag)]
            self.last_pages[client] = pages
            synth.mutate_dev(self.cur[client].data_ptr(), n * P, P, d.data_ptr(), pages.size,
                             int(pages.max()), 0, 31 + tag, client, stream)
        else:
            for p in self.last_pages[client]:
                synth.fill_dev(self.cur[client].data_ptr() + int(p) * P, P, 999, client, 0,
                               stream)


def run(harness, schedule, n_slots, budget=256 * MiB, policy=0):
    import paper_1808_00117_amd as crum
    clients = harness.clients()
    harness.precompute(schedule)
    srv = crum.Server(clients, n_slots, budget, prepare=harness.prepare)
    srv.set_policy(policy)
    for c, kind, tag in schedule:
        srv.submit(c, kind, tag)
    done = srv.poll(wait_all=True)
    images = {}
    for c in {c for c, _, _ in schedule}:
        li = srv.latest_image(c)
        if li:
            ptr, n = li
            images[c] = np.ctypeslib.as_array((ctypes.c_uint8 * n).from_address(ptr)).copy()
    srv.destroy()
    return {(d["client"], d["tag"]): d for d in done}, images


def schedule_for(clients, n_req=8):
    kinds = [SNAP, SNAP, REST, SNAP, SNAP, REST, SNAP, REST][:n_req]
    sched = []
    for t in range(n_req):
        for c in clients:
            sched.append((c, kinds[t], t))
    return sched


SPECS = [(96, 64 * KiB), (300, 4 * KiB), (40, 64 * KiB), (130, 16 * KiB), (64, 64 * KiB),
         (257, 4 * KiB)]


@pytest.mark.parametrize("policy", [0, 1, 2])
def test_same_alone_and_in_mix(policy):
    import torch
    log(f"[served] 6 clients, 4 slots, mixed vs alone, policy {policy}")
    h = Harness(SPECS)
    mix, mix_images = run(h, schedule_for(range(len(SPECS))), n_slots=4, policy=policy)
    final_mix = [c.cpu().numpy().copy() for c in h.cur]
    for c in range(len(SPECS)):
        hc = Harness(SPECS)  # same initial bytes for every client
        alone, images = run(hc, schedule_for([c]), n_slots=1, policy=(policy + 1) % 3)
        for key, d in alone.items():
            m = mix[key]
            for f in ("code", "n_dirty", "image_bytes", "meta_crc", "crcs_crc"):
                assert d[f] == m[f], (key, f, d[f], m[f])
        assert np.array_equal(hc.cur[c].cpu().numpy(), final_mix[c])
        assert np.array_equal(images[c], mix_images[c])
    for key, d in mix.items():
        assert d["code"] == 0, (key, d)
        assert d["done_s"] >= d["start_s"] >= d["arrival_s"]


def test_restore_repairs_and_images_parse():
    import torch
    h = Harness(SPECS[:3], seed=1)
    sched = [(c, k, t) for t, k in enumerate([SNAP, REST]) for c in range(3)]
    res, images = run(h, sched, n_slots=3)
    for c in range(3):
        assert torch.equal(h.cur[c], h.sh[c]), "restore did not repair the clobbered pages"
        rc, hdr = oracle.parse(images[c])
        assert rc == oracle.OK
        n, P = SPECS[c]
        assert hdr["n_dirty"] == len(h.pages_for(c, 0)) and hdr["page_size"] == P
    for (c, t), d in res.items():
        assert d["code"] == 0
        if t == 0:
            assert d["n_dirty"] == len(h.pages_for(c, 0))


def test_image_matches_oracle():
    """One client's first delta image equals the oracle's snapshot of the
    same (current, shadow) pair regenerated on the host."""
    import torch
    import synth
    h = Harness([(50, 16 * KiB)], seed=2)
    before = h.cur[0].cpu().numpy().copy()
    res, images = run(h, [(0, SNAP, 0)], n_slots=1)
    after = h.cur[0].cpu().numpy()
    st, img, _ = oracle.snapshot([(after.copy(), before, 77)], 16 * KiB, seq=1)
    assert st.code == 0 and np.array_equal(images[0], img)


def test_budget_smaller_than_all_images():
    """A budget that holds only a few images: requests wait for room instead
    of failing, and every result still matches the unconstrained run."""
    h1 = Harness(SPECS, seed=3)
    big, _ = run(h1, schedule_for(range(len(SPECS)), 4), n_slots=4)
    h2 = Harness(SPECS, seed=3)
    small, _ = run(h2, schedule_for(range(len(SPECS)), 4), n_slots=4, budget=20 * MiB)
    for key, d in big.items():
        for f in ("code", "n_dirty", "meta_crc", "crcs_crc"):
            assert small[key][f] == d[f], (key, f)
