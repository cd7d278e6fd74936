import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session", autouse=True)
def _built_libraries():
    """Build the CPU-side libraries if nothing is built yet (gcc only)."""
    import oracle
    import synth

    if not os.path.exists(oracle.SO):
        oracle.build()
    if not os.path.exists(synth.lib.HOST_SO):
        import subprocess
        subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-o", synth.lib.HOST_SO,
                        os.path.join(ROOT, "synth", "csrc", "synth_host.c")], check=True)
    yield
