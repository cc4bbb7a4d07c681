import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running")


def _ensure_cpu_libs():
    from paper_2504_19365_amd import build as B
    import oracle
    if not os.path.exists(B.GEN_SO):
        B.build_gen()
    if not os.path.exists(oracle.LIB_PATH):
        oracle.build(force=False)


_ensure_cpu_libs()


@pytest.fixture(scope="session")
def golden_dir():
    return os.path.join(ROOT, "tests", "golden")
