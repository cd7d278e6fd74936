"""GPU parity of the batched plan: every request's image, taken in one plan
launch (captured graphs, one per group of requests), must equal the oracle's
image of that request byte for byte, and the plain snapshot's."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import gpu_snapshot, log, upload

pytestmark = pytest.mark.gpu

KiB, MiB = 1 << 10, 1 << 20


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    import paper_1808_00117_amd as crum
    from paper_1808_00117_amd.api import Snapshotter
    s = Snapshotter(0)
    yield s
    s.close()


def make_requests(seed, n, max_regions=5, page_sizes=(4 * KiB, 16 * KiB, 64 * KiB)):
    rng = np.random.default_rng(seed)
    reqs = []
    for q in range(n):
        P = int(rng.choice(page_sizes))
        regs = []
        for i in range(int(rng.integers(0, max_regions + 1))):
            npg = int(rng.integers(0, 40))
            cur = rng.integers(0, 256, npg * P, dtype=np.uint8)
            sh = cur.copy()
            for pg in range(npg):
                if rng.random() < 0.3:
                    sh[pg * P + int(rng.integers(0, P))] ^= np.uint8(1 + rng.integers(0, 255))
            null = rng.random() < 0.1
            regs.append((cur, None if null else sh, 1000 * q + i))
        reqs.append((regs, P, q + 7))
    return reqs


def run_plan(ctx, host_reqs, flags=None, launches=1, staging_bytes=None, small_groups=False,
             dev=None):
    import torch
    import paper_1808_00117_amd as crum
    from paper_1808_00117_amd.api import regions_of
    if dev is None:
        dev = [upload(regs) for regs, _, _ in host_reqs]
    flags = flags or [0] * len(host_reqs)
    worst = sum(oracle.prefix_bytes(len(r), sum(c.size for c, _, _ in r) // P) +
                sum(c.size for c, _, _ in r) + 4 * sum(c.size for c, _, _ in r) // P + 4096 + 8
                for r, P, _ in host_reqs)
    sb = worst if staging_bytes is None else staging_bytes
    staging = torch.empty(max(sb, 16), dtype=torch.uint8, device="cuda")
    himg = torch.empty(max(sb, 16), dtype=torch.uint8, pin_memory=True)
    status = torch.zeros(40 * max(1, len(host_reqs)), dtype=torch.uint8, pin_memory=True)
    if small_groups:
        saved = [crum.crum_ctx_get_param(ctx.ctx, p) for p in
                 (crum.CRUM_PARAM_CHUNK_BYTES, crum.CRUM_PARAM_CHUNK_MAX_BYTES)]
        crum.crum_ctx_set_param(ctx.ctx, crum.CRUM_PARAM_CHUNK_BYTES, 1)
        crum.crum_ctx_set_param(ctx.ctx, crum.CRUM_PARAM_CHUNK_MAX_BYTES, 1)
    reqs = [(regions_of(d), P, f, seq) for d, (_, P, seq), f in zip(dev, host_reqs, flags)]
    plan = crum.Plan(ctx.ctx, reqs, staging.data_ptr(), sb, himg.data_ptr(), sb)
    if small_groups:
        crum.crum_ctx_set_param(ctx.ctx, crum.CRUM_PARAM_CHUNK_BYTES, saved[0])
        crum.crum_ctx_set_param(ctx.ctx, crum.CRUM_PARAM_CHUNK_MAX_BYTES, saved[1])
    results = []
    for _ in range(launches):
        s = torch.cuda.current_stream()
        rc = plan.launch(s.cuda_stream, status.data_ptr())
        assert rc == 0
        torch.cuda.synchronize()
        sts = crum.read_request_statuses(status.data_ptr(), len(host_reqs))
        imgs = []
        for code, _, D, G, ib, off in sts:
            imgs.append(himg[off:off + ib].numpy().copy() if code == 0 else None)
        results.append((sts, imgs))
        x = torch.ones(1 << 20, device="cuda")  # unrelated eager work between replays
        x.mul_(2.0)
        torch.cuda.synchronize()
    groups = plan.groups()
    plan.destroy()
    return dev, results, groups


def test_batched_matches_oracle_and_plain(ctx):
    host = make_requests(1, 24)
    log("[batched] 24 requests, mixed page sizes")
    dev, results, groups = run_plan(ctx, host, launches=3)
    expected = []
    for regs, P, seq in host:
        st_o, img_o, _ = oracle.snapshot(regs, P, seq=seq)
        assert st_o.code == 0
        expected.append(img_o)
    for sts, imgs in results:
        for q, ((code, _, D, G, ib, off), img, exp) in enumerate(zip(sts, imgs, expected)):
            assert code == 0 and off % 4096 == 0, (q, code)
            assert np.array_equal(img, exp), f"request {q} differs from the oracle"
    # the plain path gives the same bytes
    for q in range(0, 24, 5):
        regs, P, seq = host[q]
        rc, st, img, _ = gpu_snapshot(ctx, dev[q], P, seq=seq)
        assert st.code == 0 and np.array_equal(img, expected[q])


def test_batched_many_groups(ctx):
    host = make_requests(2, 40, max_regions=3)
    log("[batched] 40 requests, one group per request")
    dev, results, groups = run_plan(ctx, host, launches=2, small_groups=True)
    # a group closes once it holds any bytes, so empty requests join the next one
    nonempty = sum(1 for regs, _, _ in host if sum(c.size for c, _, _ in regs) > 0)
    assert len(groups) - 1 in (nonempty, nonempty + 1)
    for sts, imgs in results:
        for q, ((code, *_), img) in enumerate(zip(sts, imgs)):
            regs, P, seq = host[q]
            assert code == 0
            assert np.array_equal(img, oracle.snapshot(regs, P, seq=seq)[1]), q


def test_timed_plan_counts_diff_launches_and_keeps_images(ctx):
    """A plan created while the diff class is timed has each group's diff
    kernel record its start and end clock: one timed diff per group that
    scans anything, per launch, and the same images."""
    import paper_1808_00117_amd as crum
    host = make_requests(12, 30, max_regions=3)
    log("[batched] 30 requests, one group per request, diff launches timed")
    crum.crum_ctx_timing_reset(ctx.ctx)
    crum.crum_ctx_set_timing(ctx.ctx, crum.TIMING_DIFF)
    try:
        dev, results, groups = run_plan(ctx, host, launches=3, small_groups=True)
        n, ms = crum.crum_ctx_timing(ctx.ctx, 0)
    finally:
        crum.crum_ctx_set_timing(ctx.ctx, 0)
        crum.crum_ctx_timing_reset(ctx.ctx)
    nonempty = sum(1 for regs, _, _ in host if sum(c.size for c, _, _ in regs) > 0)
    assert n == 3 * nonempty, (n, nonempty, len(groups) - 1)
    assert ms > 0
    for sts, imgs in results:
        for q, ((code, *_), img) in enumerate(zip(sts, imgs)):
            regs, P, seq = host[q]
            assert code == 0
            assert np.array_equal(img, oracle.snapshot(regs, P, seq=seq)[1]), q


def test_batched_update_shadow(ctx):
    import torch
    host = make_requests(3, 10, max_regions=2, page_sizes=(4 * KiB,))
    flags = [1 if q % 2 == 0 else 0 for q in range(10)]
    dev, results, _ = run_plan(ctx, host, flags=flags, launches=2)
    sts1, _ = results[0]
    sts2, _ = results[1]
    for q in range(10):
        exp_d = oracle.snapshot(host[q][0], host[q][1])[0].n_dirty
        assert sts1[q][2] == exp_d
        if flags[q]:
            for c, s, _ in dev[q]:
                if s is not None:
                    assert torch.equal(c, s)
            # the second launch sees only pages of regions without a shadow
            nulls = sum(c.numel() // host[q][1] for c, s, _ in dev[q] if s is None)
            assert sts2[q][2] == nulls
        else:
            assert sts2[q][2] == exp_d


def test_batched_enospc_later_groups(ctx):
    import torch
    host = make_requests(4, 12, max_regions=2, page_sizes=(4 * KiB,))
    flags = [1] * 12
    imgs = [oracle.snapshot(r, P, seq=s)[1] for r, P, s in host]
    # room for roughly the first half of the images only
    cap = sum(((im.size + 4095) // 4096) * 4096 for im in imgs[:6])
    dev = [upload(regs) for regs, _, _ in host]
    before = [[None if s is None else s.clone() for _, s, _ in d] for d in dev]
    dev, results, groups = run_plan(ctx, host, flags=flags, staging_bytes=cap,
                                    small_groups=True, dev=dev)
    sts, got = results[0]
    codes = [st[0] for st in sts]
    first_bad = codes.index(-2)
    assert 1 <= first_bad <= 6 and all(c == -2 for c in codes[first_bad:])
    for q in range(first_bad):
        assert np.array_equal(got[q], imgs[q])
    for q in range(first_bad, 12):
        for (c, s, _), b in zip(dev[q], before[q]):
            if s is not None:
                assert torch.equal(s, b), "shadow changed for a request without room"


def test_empty_plan(ctx):
    dev, results, groups = run_plan(ctx, [], launches=2)
    assert results[0][0] == []


def test_batched_scenario_matches_sequential(ctx):
    """A reduced batched workload (16 requests drawn like the 256-request
    configuration, capped at 64 MiB each): plan images equal the plain
    snapshots' images request by request."""
    import torch
    from synth import scenarios as sc
    from synth.device import materialize
    reqs = sc.batched(seed=1004, n_requests=16, max_total=64 << 20)
    pairs = [materialize(s) for s in reqs]
    torch.cuda.synchronize()
    host = []
    for s, pr in zip(reqs, pairs):
        host.append(([(c, h, r.id) for (c, h), r in zip(pr, s.regions)], s.page_size, 3))
    import paper_1808_00117_amd as crum
    from paper_1808_00117_amd.api import regions_of
    plan_reqs = [(regions_of(regs), P, 0, seq) for regs, P, seq in host]
    worst = sum(crum.crum_image_bytes(len(r), s.total_pages, s.total_pages, s.page_size) + 4096
                for (r, _, _), s in zip(host, reqs))
    staging = torch.empty(worst, dtype=torch.uint8, device="cuda")
    himg = torch.empty(worst, dtype=torch.uint8, pin_memory=True)
    status = torch.zeros(40 * len(host), dtype=torch.uint8, pin_memory=True)
    plan = crum.Plan(ctx.ctx, plan_reqs, staging.data_ptr(), worst, himg.data_ptr(), worst)
    assert plan.launch(torch.cuda.current_stream().cuda_stream, status.data_ptr()) == 0
    torch.cuda.synchronize()
    sts = crum.read_request_statuses(status.data_ptr(), len(host))
    for q, ((regs, P, seq), s) in enumerate(zip(host, reqs)):
        code, _, D, G, ib, off = sts[q]
        assert code == 0 and D == s.n_dirty and G == s.total_pages
        rc, st, img, _ = gpu_snapshot(ctx, regs, P, seq=seq)
        assert st.code == 0 and np.array_equal(himg[off:off + ib].numpy(), img), q
    # one request against the oracle on the host
    q = min(range(len(reqs)), key=lambda i: reqs[i].total_bytes)
    hr = []
    for i, r in enumerate(reqs[q].regions):
        c, h = sc.materialize_host(reqs[q], i)
        hr.append((c, h, r.id))
    code, _, D, G, ib, off = sts[q]
    assert np.array_equal(himg[off:off + ib].numpy(),
                          oracle.snapshot(hr, reqs[q].page_size, seq=3)[1])
    plan.destroy()


def test_autotune_keeps_images(tmp_path):
    """The shape tuner on a small batch: every candidate shape gives the
    same images as the oracle, the best shapes are applied and cached."""
    import time
    import torch
    import paper_1808_00117_amd as crum
    from paper_1808_00117_amd import autotune
    from paper_1808_00117_amd.api import regions_of
    host = make_requests(11, 12, max_regions=3)
    expected = [oracle.snapshot(r, P, seq=s)[1] for r, P, s in host]
    dev = [upload(regs) for regs, _, _ in host]
    ctx = crum.crum_ctx_create(0)
    try:
        cap = sum((e.size + 4095) // 4096 * 4096 for e in expected) + (1 << 20)
        staging = torch.empty(cap, dtype=torch.uint8, device="cuda")
        himg = torch.empty(cap, dtype=torch.uint8, pin_memory=True)
        status = torch.zeros(40 * len(host), dtype=torch.uint8, pin_memory=True)
        reqs = [(regions_of(d), P, 0, s) for d, (_, P, s) in zip(dev, host)]

        def run():
            plan = crum.Plan(ctx, reqs, staging.data_ptr(), cap, himg.data_ptr(), cap)
            t = time.perf_counter()
            assert plan.launch(torch.cuda.current_stream().cuda_stream, status.data_ptr()) == 0
            torch.cuda.synchronize()
            t = time.perf_counter() - t
            for q, (code, _, _, _, b, off) in enumerate(
                    crum.read_request_statuses(status.data_ptr(), len(host))):
                assert code == 0 and np.array_equal(himg[off:off + b].numpy(), expected[q]), q
            plan.destroy()
            return t
        space = {"pack_blocks": [8, 256], "chunk_bytes": [4096, 1 << 20],
                 "crc_variant": [0, 3], "diff_blocks": [16, 1024]}
        best, trials, _ = autotune.search(ctx, run, space, repeats=1)
        assert len(trials) == 1 + sum(len(v) for v in space.values()) - sum(
            1 for k, v in space.items() if trials[0]["params"][k] in v)
        assert autotune.current(ctx) == best
        path = str(tmp_path / "cache.json")
        autotune.save("test", best, trials, path)
        assert autotune.load("test", path) == best
    finally:
        crum.crum_ctx_destroy(ctx)


def test_smallest_first_order(ctx):
    """With CRUM_PARAM_PLAN_ORDER 1 the requests run smallest first: statuses
    stay in the caller's order, every image equals the oracle's, groups
    follow the processing order, and a capacity shortfall hits the largest
    requests (the last in processing order)."""
    import torch
    import paper_1808_00117_amd as crum
    from paper_1808_00117_amd.api import regions_of
    host = make_requests(21, 16, max_regions=3, page_sizes=(4 * KiB,))
    expected = [oracle.snapshot(r, P, seq=s)[1] for r, P, s in host]
    size = [sum(c.size for c, _, _ in r) for r, _, _ in host]
    dev = [upload(regs) for regs, _, _ in host]
    crum.crum_ctx_set_param(ctx.ctx, crum.CRUM_PARAM_PLAN_ORDER, 1)
    saved = [crum.crum_ctx_get_param(ctx.ctx, p) for p in
             (crum.CRUM_PARAM_CHUNK_BYTES, crum.CRUM_PARAM_CHUNK_MAX_BYTES)]
    crum.crum_ctx_set_param(ctx.ctx, crum.CRUM_PARAM_CHUNK_BYTES, 1)
    crum.crum_ctx_set_param(ctx.ctx, crum.CRUM_PARAM_CHUNK_MAX_BYTES, 1)
    try:
        reqs = [(regions_of(d), P, 0, s) for d, (_, P, s) in zip(dev, host)]
        full = sum((e.size + 4095) // 4096 * 4096 for e in expected)
        for cap in (full, full // 2):
            staging = torch.empty(cap, dtype=torch.uint8, device="cuda")
            himg = torch.empty(cap, dtype=torch.uint8, pin_memory=True)
            status = torch.zeros(40 * len(host), dtype=torch.uint8, pin_memory=True)
            plan = crum.Plan(ctx.ctx, reqs, staging.data_ptr(), cap, himg.data_ptr(), cap)
            order = plan.order()
            assert sorted(order) == list(range(len(host)))
            assert [size[q] for q in order] == sorted(size)
            assert plan.launch(torch.cuda.current_stream().cuda_stream, status.data_ptr()) == 0
            torch.cuda.synchronize()
            sts = crum.read_request_statuses(status.data_ptr(), len(host))
            codes = [sts[q][0] for q in order]
            if cap == full:
                assert all(c == 0 for c in codes)
            else:
                k = codes.index(-2)
                assert k >= 1 and all(c == -2 for c in codes[k:])
            for q, (code, _, D, G, b, off) in enumerate(sts):
                if code == 0:
                    assert np.array_equal(himg[off:off + b].numpy(), expected[q]), q
            plan.destroy()
    finally:
        crum.crum_ctx_set_param(ctx.ctx, crum.CRUM_PARAM_PLAN_ORDER, 0)
        crum.crum_ctx_set_param(ctx.ctx, crum.CRUM_PARAM_CHUNK_BYTES, saved[0])
        crum.crum_ctx_set_param(ctx.ctx, crum.CRUM_PARAM_CHUNK_MAX_BYTES, saved[1])


def test_batched_property(ctx):
    """Drawn request sets (0-10 requests of 0-4 regions, page sizes, one or
    many groups, caller's or smallest-first order): every request's image is
    the oracle's, byte for byte, at a 4 KiB-aligned offset.  Derandomized."""
    import paper_1808_00117_amd as crum
    from hypothesis import HealthCheck, given, settings
    from hypothesis import strategies as st

    @settings(max_examples=15, deadline=None, derandomize=True,
              suppress_health_check=list(HealthCheck))
    @given(seed=st.integers(0, 2**31 - 1), n=st.integers(0, 10),
           max_regions=st.integers(0, 4),
           sizes=st.sampled_from([(4 * KiB,), (64 * KiB,), (4 * KiB, 16 * KiB, 64 * KiB)]),
           small_groups=st.booleans(), order=st.sampled_from([0, 1]))
    def run(seed, n, max_regions, sizes, small_groups, order):
        host = make_requests(seed, n, max_regions=max_regions, page_sizes=sizes)
        crum.crum_ctx_set_param(ctx.ctx, crum.CRUM_PARAM_PLAN_ORDER, order)
        try:
            _, results, _ = run_plan(ctx, host, small_groups=small_groups)
        finally:
            crum.crum_ctx_set_param(ctx.ctx, crum.CRUM_PARAM_PLAN_ORDER, 0)
        sts, imgs = results[0]
        for q, ((code, _, D, G, ib, off), img) in enumerate(zip(sts, imgs)):
            regs, P, seq = host[q]
            st_o, img_o, _ = oracle.snapshot(regs, P, seq=seq)
            assert code == 0 and off % 4096 == 0 and (D, G, ib) == \
                (st_o.n_dirty, st_o.total_pages, st_o.image_bytes), q
            assert np.array_equal(img, img_o), f"request {q} differs from the oracle"

    run()


def test_tuning_cache_class_shapes_apply_and_explicit_params_win(tmp_path):
    """A context created with a tuning cache runs a plan of a cached class
    with that class's shapes (here one group per request, visible in the
    plan's group layout), an explicitly set parameter wins over the cache,
    and the images stay the oracle's."""
    import json

    import paper_1808_00117_amd as crum
    from paper_1808_00117_amd import autotune
    from paper_1808_00117_amd.api import Snapshotter
    host = make_requests(41, 6)
    total = sum(c.size for regs, _, _ in host for c, _, _ in regs)
    key = autotune.class_key("plan", total)
    path = tmp_path / "cache.json"
    path.write_text(json.dumps({autotune.device_key(): {
        key: {"params": {"chunk_bytes": 1, "chunk_max_bytes": 1}}}}))
    s = Snapshotter(0)
    crum.crum_ctx_destroy(s.ctx)
    s.ctx = crum.crum_ctx_create(0, str(path))
    try:
        assert crum.crum_ctx_tuned_classes(s.ctx) == 1
        dev, res, groups = run_plan(s, host)
        # groups of one byte: a group closes at every request that scans any
        expect, acc = 0, 0
        for q, (regs, _, _) in enumerate(host):
            acc += sum(c.size for c, _, _ in regs)
            if acc >= 1 or q + 1 == len(host):
                expect, acc = expect + 1, 0
        assert expect > 1 and len(groups) - 1 == expect, groups
        for q, (regs, P, seq) in enumerate(host):
            st_o, img_o, _ = oracle.snapshot(regs, P, seq=seq)
            assert np.array_equal(res[0][1][q], img_o), q
        # the cache's shapes last for the call only
        assert crum.crum_ctx_get_param(s.ctx, crum.CRUM_PARAM_CHUNK_BYTES) == 128 << 20
        # an explicit value wins over the cached class
        crum.crum_ctx_set_param(s.ctx, crum.CRUM_PARAM_CHUNK_BYTES, 1 << 40)
        crum.crum_ctx_set_param(s.ctx, crum.CRUM_PARAM_CHUNK_MAX_BYTES, 1 << 40)
        _, res2, groups2 = run_plan(s, host, dev=dev)
        assert len(groups2) - 1 == 1, groups2
        for q in range(len(host)):
            assert np.array_equal(res2[0][1][q], res[0][1][q]), q
    finally:
        s.close()


def test_batched_shadow_and_capacity_property(ctx):
    """Drawn request sets with drawn shadow-update flags, a drawn staging
    capacity (from too small for anything to room for every image) and the
    caller's or smallest-first order, one request per group: in processing
    order the statuses are OK for a run of groups whose images fit and
    ENOSPC from the first group that does not fit on; every OK image is the
    oracle's; a request that was packed with the flag has its shadows updated,
    every other request's shadows are unchanged.  Derandomized."""
    import torch
    import paper_1808_00117_amd as crum
    from hypothesis import HealthCheck, given, settings
    from hypothesis import strategies as st

    @settings(max_examples=15, deadline=None, derandomize=True,
              suppress_health_check=list(HealthCheck))
    @given(seed=st.integers(0, 2**31 - 1), n=st.integers(1, 10),
           room=st.sampled_from([0.0, 0.3, 0.6, 1.0]), order=st.sampled_from([0, 1]),
           flag_seed=st.integers(0, 2**31 - 1))
    def run(seed, n, room, order, flag_seed):
        host = make_requests(seed, n, max_regions=3, page_sizes=(4 * KiB, 64 * KiB))
        frng = np.random.default_rng(flag_seed)
        flags = [int(frng.integers(0, 2)) for _ in range(n)]
        imgs = [oracle.snapshot(r, P, seq=s)[1] for r, P, s in host]
        aligned = [((im.size + 4095) // 4096) * 4096 for im in imgs]
        scanned = [sum(c.size for c, _, _ in r) for r, _, _ in host]
        proc = sorted(range(n), key=lambda q: scanned[q]) if order else list(range(n))
        cap = max(16, int(room * sum(aligned)))
        dev = [upload(regs) for regs, _, _ in host]
        before = [[None if s is None else s.clone() for _, s, _ in d] for d in dev]
        crum.crum_ctx_set_param(ctx.ctx, crum.CRUM_PARAM_PLAN_ORDER, order)
        try:
            dev, results, groups = run_plan(ctx, host, flags=flags, staging_bytes=cap,
                                            small_groups=True, dev=dev)
        finally:
            crum.crum_ctx_set_param(ctx.ctx, crum.CRUM_PARAM_PLAN_ORDER, 0)
        sts, got = results[0]
        codes = [sts[q][0] for q in proc]
        assert set(codes) <= {0, -2}, codes
        k = codes.index(-2) if -2 in codes else n
        assert all(c == -2 for c in codes[k:]), codes
        used = sum(aligned[q] for q in proc[:k])
        assert used <= cap
        if k < n:  # the group holding the first refused request does not fit
            g = max(i for i in range(len(groups) - 1) if groups[i] <= k)
            assert groups[g] == k, (groups, k)
            need = sum(aligned[proc[i]] for i in range(groups[g], groups[g + 1]))
            assert used + need > cap, (used, need, cap)
        for q in range(n):
            ok = sts[q][0] == 0
            if ok:
                assert np.array_equal(got[q], imgs[q]), q
            for (c, s, _), b in zip(dev[q], before[q]):
                if s is None:
                    continue
                if ok and flags[q]:
                    assert torch.equal(s, c), q
                else:
                    assert torch.equal(s, b), q

    run()
