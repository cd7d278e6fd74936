"""The library's reader of the shape tuner's cache (crum_ctx_create's
tuning_cache, checked on the host through crum_tuning_check): the committed
cache parses, classes are found per device key, unknown classes and fields
are skipped, and malformed or missing files are refused."""
import json
import os

import paper_1808_00117_amd as crum
from paper_1808_00117_amd import autotune

KEY = "cc9.5-256cu|hip70226015"


def test_committed_cache_parses():
    rc, n = crum.crum_tuning_check(autotune.DEFAULT_CACHE, KEY)
    assert rc == crum.CRUM_OK and n >= 1
    keys = json.load(open(autotune.DEFAULT_CACHE))[KEY]
    assert n == sum(1 for k in keys if k.startswith(("snapshot|p", "plan|b")))


def test_classes_per_device_and_skipped_entries(tmp_path):
    cache = {
        KEY: {
            "snapshot|p65536|b34": {"params": {"pack_blocks": 2048, "piece_shift": 14,
                                               "unknown_param": 3, "ratio": 0.5},
                                    "trials": [{"params": {"a": 1}, "seconds": 0.1}],
                                    "default_s": 0.1, "spread_s": 0.001},
            "plan|b36": {"params": {"chunk_bytes": 67108864}},
            "batched": {"params": {"chunk_bytes": 1}},       # not a class key: skipped
            "snapshot|p3000|b10": {"params": {"pack_blocks": 1}},  # bad page size: skipped
        },
        "cc9.4-304cu|hip1": {"plan|b30": {"params": {"diff_blocks": 64}}},
    }
    p = tmp_path / "c.json"
    p.write_text(json.dumps(cache, indent=1))
    assert crum.crum_tuning_check(str(p), KEY) == (crum.CRUM_OK, 2)
    assert crum.crum_tuning_check(str(p), "cc9.4-304cu|hip1") == (crum.CRUM_OK, 1)
    assert crum.crum_tuning_check(str(p), "other") == (crum.CRUM_OK, 0)


def test_malformed_and_missing_files(tmp_path):
    assert crum.crum_tuning_check(str(tmp_path / "none.json"), KEY)[0] == crum.CRUM_EINVAL
    for text in ("", "[]", '{"a": ', '{"' + KEY + '": {"plan|b3": {"params": {"x": 1}}',
                 '{"' + KEY + '": {"plan|b3": {"params": 5}}}'):
        p = tmp_path / "bad.json"
        p.write_text(text)
        assert crum.crum_tuning_check(str(p), KEY)[0] == crum.CRUM_EINVAL, text
    p = tmp_path / "empty.json"
    p.write_text("{}")
    assert crum.crum_tuning_check(str(p), KEY) == (crum.CRUM_OK, 0)


FUZZ = r"""
import os, random, sys
sys.path.insert(0, sys.argv[1])
import paper_1808_00117_amd as crum
KEY, src, tmp = sys.argv[2], open(sys.argv[3], "rb").read(), sys.argv[4]
rng = random.Random(7)
cases = [src[:n] for n in range(0, len(src), max(1, len(src) // 300))]
for _ in range(300):
    b = bytearray(src)
    for _ in range(rng.randint(1, 8)):
        b[rng.randrange(len(b))] = rng.choice(b'{}[]",:-.e0123456789 x\\')
    cases.append(bytes(b))
cases += [b"[" * 100000, b'{"a":' * 50000, b'{"' + KEY.encode() + b'":' + b"[" * 70 + b"]" * 70 + b"}"]
for i, c in enumerate(cases):
    with open(tmp, "wb") as f:
        f.write(c)
    rc, n = crum.crum_tuning_check(tmp, KEY)
    assert rc in (crum.CRUM_OK, crum.CRUM_EINVAL), (i, rc)
print("fuzz ok", len(cases))
"""


def test_reader_survives_truncated_mutated_and_deep_input(tmp_path):
    """Every prefix of the committed cache, random byte mutations of it and
    deeply nested values come back as OK or EINVAL: the reader neither
    crashes nor recurses without bound (run in a child process, so a crash
    fails this test instead of ending the run)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", FUZZ, root, KEY, autotune.DEFAULT_CACHE,
                        str(tmp_path / "f.json")], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "fuzz ok" in r.stdout, r.stdout + r.stderr
