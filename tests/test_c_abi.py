"""The boundary used from C: a C99 program that includes only crum.h and the
HIP runtime API compiles warning-free and links against libcrum.so (CPU), and
on the GPU takes a snapshot, restores it with verification, runs a plan of two
requests and persists an image with the writer, restores on demand, finds
nothing dirty after a shadow update, snapshots a tracked managed region with
and without allocation, and drives the serving loop (tests/c/abi_roundtrip.c)."""
import os
import subprocess

import pytest

from tests.c import build as cbuild


def test_c_client_compiles_as_c99(tmp_path):
    out = cbuild.build(out=str(tmp_path / "abi_roundtrip"))
    assert os.path.exists(out)


@pytest.mark.gpu
def test_c_client_round_trip():
    assert os.path.exists(cbuild.BIN), "tests/c/abi_roundtrip is built by __graft_entry__.build()"
    r = subprocess.run([cbuild.BIN], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0 and "abi_roundtrip: ok" in r.stdout, r.stdout + r.stderr
