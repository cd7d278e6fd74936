"""Build libcrum.so in-tree with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SO = os.path.join(HERE, "libcrum.so")
SOURCES = [os.path.join(HERE, "csrc", f)
           for f in ("crum_kernels.hip", "crum_capi.hip", "crum_plan.hip", "crum_server.hip",
                     "crum_writer.hip", "crum_lazy.hip", "crum_track.hip",
                     "crum_noalloc.hip", "crum_tune.hip")]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
    "-Wno-unused-result",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    cmd = ["hipcc", *FLAGS, "-o", SO + ".tmp", *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("libcrum build failed:\n" + r.stdout + r.stderr)
    os.replace(SO + ".tmp", SO)
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
