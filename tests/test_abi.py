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


def test_null_handles_are_rejected_without_a_gpu():
    """Entry points given no context, session, plan, server or writer return
    CRUM_EINVAL before any HIP call (so this runs on the CPU) and the
    destroy/close calls ignore NULL."""
    import ctypes

    import paper_1808_00117_amd as crum
    lib = crum.lib()
    E = crum.CRUM_EINVAL
    out = ctypes.c_void_p(123)
    st = (ctypes.c_uint8 * 64)()
    assert lib.crum_lazy_open(None, None, 0, None, 0, 0, 0, None, 0, None, st,
                              ctypes.byref(out)) == E
    assert out.value is None  # *out cleared
    assert lib.crum_lazy_open(None, None, 0, None, 0, 0, 0, None, 0, None, None, None) == E
    n = ctypes.c_uint64(7)
    assert lib.crum_lazy_touch(None, 0, 0, 1, None, None, ctypes.byref(n)) == E
    assert n.value == 0
    assert lib.crum_lazy_finish(None, None, st) == E
    info = crum.crum_lazy_info()
    assert lib.crum_lazy_stats(None, ctypes.byref(info)) == E
    assert lib.crum_lazy_fetched(None, None, 0) == E
    lib.crum_lazy_close(None)
    assert lib.crum_snapshot(None, None, 0, 4096, 0, 0, None, 0, None, 0, None, st) == E
    assert lib.crum_restore(None, None, 0, None, 0, 0, None, 0, None, st) == E
    assert lib.crum_ctx_set_param(None, crum.CRUM_PARAM_DIRECT_BYTES, 0) == E
    v = ctypes.c_uint64()
    assert lib.crum_ctx_get_param(None, crum.CRUM_PARAM_DIRECT_BYTES, ctypes.byref(v)) == E
    lib.crum_ctx_destroy(None)
    lib.crum_plan_destroy(None)
    lib.crum_server_destroy(None)
    lib.crum_writer_destroy(None)


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1808_00117_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in src.replace("oracle-free", ""), f
