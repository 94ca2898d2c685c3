import os
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# the tests' autotuner entries go to a tune-cache file of their own, never to
# the user's (the library reads the variable when it first uses a device)
os.environ["XENG_TUNE_DIR"] = tempfile.mkdtemp(prefix="xeng_tune_tests_")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle
