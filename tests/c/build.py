"""Build the C99 client of the C ABI (tests/c/abi_roundtrip.c) in-tree with
gcc: only crum.h and the HIP runtime API header, linked against the in-tree
libcrum.so (found at run time through a path relative to the binary)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "abi_roundtrip.c")
BIN = os.path.join(HERE, "abi_roundtrip")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def command(out: str = BIN) -> list:
    return ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
            "-I" + os.path.join(ROCM, "include"), "-I" + os.path.join(ROOT, "include"), SRC,
            "-o", out, "-L" + os.path.join(ROOT, "paper_1808_00117_amd"), "-lcrum",
            "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
            "-Wl,-rpath,$ORIGIN/../../paper_1808_00117_amd", "-Wl,-rpath," + os.path.join(ROCM, "lib")]


def build(verbose: bool = False, out: str = BIN) -> str:
    cmd = command(out)
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("C client build failed:\n" + r.stdout + r.stderr)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
