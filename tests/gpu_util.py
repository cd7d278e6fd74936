"""Helpers for GPU parity tests: upload host regions, run the HIP snapshot
through the C ABI, and return the drained image for comparison with the
oracle."""
from __future__ import annotations

import sys

import numpy as np


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a: np.ndarray):
    import torch
    if a.size == 0:
        return torch.empty(16, dtype=torch.uint8, device="cuda")[:0]
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def upload(host_regions):
    """host_regions: [(cur ndarray, shadow ndarray or None, id)] -> device triples."""
    out = []
    for cur, sh, rid in host_regions:
        out.append((to_dev(cur), None if sh is None else to_dev(sh), rid))
    return out


def image_capacity(regions, page_size: int) -> int:
    import oracle
    G = sum(int(c.numel() if hasattr(c, "numel") else c.size) // page_size
            for c, _, _ in regions)
    return oracle.prefix_bytes(len(regions), G) + G * page_size + ((4 * G + 7) // 8) * 8


def gpu_snapshot(snap, dev_regions, page_size, flags=0, seq=0, staging_bytes=None,
                 image_bytes=None, drain=True):
    """Returns (rc, Status, image ndarray or None, staging tensor)."""
    import torch
    cap = image_capacity(dev_regions, page_size)
    sb = cap if staging_bytes is None else staging_bytes
    staging = torch.empty(max(sb, 16), dtype=torch.uint8, device="cuda")[:sb]
    h = None
    if drain:
        ib = cap if image_bytes is None else image_bytes
        h = torch.empty(max(ib, 16), dtype=torch.uint8, pin_memory=True)[:ib]
    rc, st = snap.snapshot(dev_regions, page_size, staging, h, flags=flags, seq=seq)
    img = None
    if rc == 0 and st.code == 0 and h is not None:
        img = h[: st.image_bytes].numpy().copy()
    return rc, st, img, staging
