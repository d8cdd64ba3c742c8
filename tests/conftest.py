import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running")


@pytest.fixture(scope="session", autouse=True)
def _native_builds():
    """Build the CPU-side native helpers (generators, oracle) if absent."""
    from paper_1805_11938_amd import build as pb
    if not os.path.exists(os.path.join(ROOT, "paper_1805_11938_amd", "synth", "libsynth.so")):
        pb.build_synth()
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        from oracle import build as ob
        ob.build()
    yield
