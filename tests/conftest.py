import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    # ESDG_TEST_HOSTSAN=1: run the GPU tests on the host-sanitized build of the
    # library (the process must preload gcc's ASan runtime)
    if os.environ.get("ESDG_TEST_HOSTSAN") == "1":
        from paper_1804_02221_amd import esdg
        esdg.use_sanitized_build()
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle
