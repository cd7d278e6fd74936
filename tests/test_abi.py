"""The C-ABI library loads on a machine without a GPU and exports every
function that include/crum.h declares; the pure-host size helpers agree with
the oracle's layout."""
import ctypes
import os
import re

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "crum.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void)\s+(crum_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["crum_ctx_create", "crum_ctx_destroy", "crum_snapshot", "crum_restore",
                 "crum_image_prefix_bytes", "crum_image_bytes"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1808_00117_amd as crum
    if not os.path.exists(crum._lib.SO):
        crum.build()
    L = ctypes.CDLL(crum._lib.SO)
    for name in declared_functions():
        assert hasattr(L, name), name


@pytest.mark.parametrize("R,G", [(0, 0), (1, 1), (3, 64), (64, 262144), (4096, 4096)])
def test_prefix_bytes_match_oracle(R, G):
    import paper_1808_00117_amd as crum
    assert crum.crum_image_prefix_bytes(R, G) == oracle.prefix_bytes(R, G)
    for D in [0, 1, G // 2, G]:
        if D <= G:
            exp = oracle.prefix_bytes(R, G) + D * 4096 + ((4 * D + 7) // 8) * 8
            assert crum.crum_image_bytes(R, G, D, 4096) == exp


def test_size_helpers_reject_bad_arguments():
    import paper_1808_00117_amd as crum
    with pytest.raises(ValueError):
        crum.crum_image_bytes(1, 10, 11, 4096)
    with pytest.raises(ValueError):
        crum.crum_image_bytes(1, 10, 1, 1000)


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1808_00117_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in src.replace("oracle-free", ""), f
