"""Materialise scenarios in device memory (torch tensors as plain HBM buffers)."""
from __future__ import annotations

from typing import List, Optional, Tuple

import numpy as np

from .lib import fill_dev, mutate_dev
from .scenarios import Scenario


def materialize(scn: Scenario, device: str = "cuda", stream: int = 0,
                shadows: bool = True) -> List[Tuple["torch.Tensor", Optional["torch.Tensor"]]]:
    """Allocate (current, shadow) uint8 tensors per region and fill them on the
    device: current = generator bytes, shadow = copy with the scenario's page
    mutations applied.  Regions without a shadow get None."""
    import torch

    out = []
    for r in scn.regions:
        cur = torch.empty(max(r.nbytes, 16), dtype=torch.uint8, device=device)[: r.nbytes]
        fill_dev(cur.data_ptr(), r.nbytes, r.fill_seed, r.fill_region, 0, stream)
        sh = None
        if shadows and r.has_shadow:
            sh = torch.empty(max(r.nbytes, 16), dtype=torch.uint8, device=device)[: r.nbytes]
            if r.nbytes:
                sh.copy_(cur)
            if r.dirty_pages.size:
                pages = torch.from_numpy(np.ascontiguousarray(r.dirty_pages, np.int64)).to(device)
                mutate_dev(sh.data_ptr(), r.nbytes, scn.page_size, pages.data_ptr(),
                           int(r.dirty_pages.size), int(r.dirty_pages.max()), r.mut_kind,
                           scn.mut_seed, r.fill_region, stream)
                torch.cuda.current_stream().synchronize()
                del pages
        out.append((cur, sh))
    return out
