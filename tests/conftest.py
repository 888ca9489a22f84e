import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session", autouse=True)
def _private_tune_cache(tmp_path_factory):
    # the autotuner appends its choices to a file; tests keep theirs apart
    # from the user's cache
    if "BNS_TUNE_CACHE" not in os.environ:
        os.environ["BNS_TUNE_CACHE"] = str(tmp_path_factory.mktemp("tune") / "bns_autotune.txt")
    yield
